// Sparse approximate inverse of C_alpha (Sec. 4.3 (sec:csolve), Algorithm alg:mr).
//
// X ~ C_alpha^{-1} from the self-preconditioned global minimal-residual
// iteration with numerical dropping, started from X_0 = diag(C_alpha)^{-1}:
//   R = I - C X,  Z = X R,  drop(Z),  beta = tr(R^T C Z) / ||C Z||_F^2,
//   X <- X + beta Z.
// The C_alpha solve of every A0 solve then becomes one sparse product with X.
//
// Dropping (the paper names a drop tolerance and a per-column fill limit but
// gives neither the rule's details nor values):
//   * Z is symmetrised, z_ij <- (z_ij + z_ji) / 2; X R is symmetric in exact
//     arithmetic when X is, and a symmetric X keeps the preconditioner
//     symmetric for CG;
//   * in column j the diagonal is kept; off-diagonal entries with
//     |z_ij| < tol ||z_:j||_2 are dropped; of the rest the lfil largest in
//     magnitude stay (equal magnitudes: the lower row first);
//   * an entry stays only if it stays in both its column and its row.
// The loop ends early when C Z = 0.
//
// Arithmetic order, so that the result is reproducible bit for bit by any
// implementation of the same rule: each entry of a sparse product
// sum_k a_ik b_kj is accumulated from 0.0 in ascending k; ||z_:j||^2 is
// accumulated down column j; tr(R^T W) and ||W||_F^2 (W = C Z) and ||R||_F^2
// are single running sums over stored entries in row-major order.
//
// X is SPD when ||I - C X||_inf < 1 (largest absolute row sum): I - C X is
// similar to I - C^{1/2} X C^{1/2}, whose spectral radius is at most any
// induced norm of I - C X, so the eigenvalues of C^{1/2} X C^{1/2} lie in
// (0, 2).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ddlr.h"
#include "host_setup.hpp"

namespace ddlr {

namespace {

// Square sparse matrix, rows with ascending columns (symmetric ones double as
// their own column storage).
struct Sp {
    int64_t n = 0;
    std::vector<int64_t> row;  // n + 1
    std::vector<int32_t> col;
    std::vector<double> val;
    explicit Sp(int64_t n_ = 0) : n(n_), row(n_ + 1, 0) {}
    double at(int64_t i, int32_t j) const {
        auto b = col.begin() + row[i], e = col.begin() + row[i + 1];
        auto it = std::lower_bound(b, e, j);
        return (it != e && *it == j) ? val[it - col.begin()] : 0.0;
    }
};

// Row-by-row product a * b with a dense accumulator; every entry sums its
// terms from 0.0 in ascending k (the order of a's row).
Sp product(const Sp& a, const Sp& b) {
    const int64_t n = a.n;
    Sp c(n);
    std::vector<double> acc(n, 0.0);
    std::vector<int64_t> seen(n, -1);
    std::vector<int32_t> cols;
    for (int64_t i = 0; i < n; ++i) {
        cols.clear();
        for (int64_t t = a.row[i]; t < a.row[i + 1]; ++t) {
            const int32_t k = a.col[t];
            const double aik = a.val[t];
            for (int64_t u = b.row[k]; u < b.row[k + 1]; ++u) {
                const int32_t j = b.col[u];
                if (seen[j] != i) {
                    seen[j] = i;
                    acc[j] = 0.0;
                    cols.push_back(j);
                }
                acc[j] += aik * b.val[u];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t j : cols) {
            c.col.push_back(j);
            c.val.push_back(acc[j]);
        }
        c.row[i + 1] = (int64_t)c.col.size();
    }
    return c;
}

// I - w
Sp identity_minus(const Sp& w) {
    Sp r(w.n);
    for (int64_t i = 0; i < w.n; ++i) {
        bool diag = false;
        for (int64_t t = w.row[i]; t < w.row[i + 1]; ++t) {
            const int32_t j = w.col[t];
            if (!diag && j > i) {
                r.col.push_back((int32_t)i);
                r.val.push_back(1.0);
                diag = true;
            }
            if (j == i) {
                r.col.push_back(j);
                r.val.push_back(1.0 - w.val[t]);
                diag = true;
            } else {
                r.col.push_back(j);
                r.val.push_back(-w.val[t]);
            }
        }
        if (!diag) {
            r.col.push_back((int32_t)i);
            r.val.push_back(1.0);
        }
        r.row[i + 1] = (int64_t)r.col.size();
    }
    return r;
}

double frobenius(const Sp& a) {
    double t = 0.0;
    for (double x : a.val) t += x * x;
    return std::sqrt(t);
}

// (z + z^T) / 2 on the union pattern
Sp symmetrised(const Sp& z) {
    const int64_t n = z.n;
    // transpose by counting
    Sp zt(n);
    zt.col.resize(z.col.size());
    zt.val.resize(z.col.size());
    for (int32_t j : z.col) zt.row[j + 1]++;
    for (int64_t i = 0; i < n; ++i) zt.row[i + 1] += zt.row[i];
    std::vector<int64_t> next(zt.row.begin(), zt.row.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = z.row[i]; t < z.row[i + 1]; ++t) {
            const int64_t q = next[z.col[t]]++;
            zt.col[q] = (int32_t)i;
            zt.val[q] = z.val[t];
        }
    Sp s(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = z.row[i], b = zt.row[i];
        const int64_t ae = z.row[i + 1], be = zt.row[i + 1];
        while (a < ae || b < be) {
            const int32_t ja = a < ae ? z.col[a] : INT32_MAX, jb = b < be ? zt.col[b] : INT32_MAX;
            const int32_t j = std::min(ja, jb);
            const double u = ja == j ? z.val[a++] : 0.0;
            const double v = jb == j ? zt.val[b++] : 0.0;
            s.col.push_back(j);
            s.val.push_back(0.5 * (u + v));
        }
        s.row[i + 1] = (int64_t)s.col.size();
    }
    return s;
}

// dual-threshold dropping with a symmetric survivor pattern (z symmetric)
Sp dropped(const Sp& z, double tol, int lfil) {
    const int64_t n = z.n;
    std::vector<char> keep(z.col.size(), 0);
    std::vector<int64_t> cand;
    for (int64_t j = 0; j < n; ++j) {
        double sq = 0.0;
        for (int64_t t = z.row[j]; t < z.row[j + 1]; ++t) sq += z.val[t] * z.val[t];
        const double thr = tol * std::sqrt(sq);
        cand.clear();
        for (int64_t t = z.row[j]; t < z.row[j + 1]; ++t) {
            if (z.col[t] == j) {
                keep[t] = 1;
            } else if (!(std::fabs(z.val[t]) < thr)) {
                cand.push_back(t);
            }
        }
        // larger magnitude first; equal magnitudes by position (= ascending row)
        std::sort(cand.begin(), cand.end(), [&](int64_t x, int64_t y) {
            const double ax = std::fabs(z.val[x]), ay = std::fabs(z.val[y]);
            return ax != ay ? ax > ay : x < y;
        });
        for (size_t q = 0; q < cand.size() && (int64_t)q < lfil; ++q) keep[cand[q]] = 1;
    }
    Sp d(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t t = z.row[i]; t < z.row[i + 1]; ++t) {
            if (!keep[t]) continue;
            const int32_t j = z.col[t];
            auto b = z.col.begin() + z.row[j], e = z.col.begin() + z.row[j + 1];
            auto it = std::lower_bound(b, e, (int32_t)i);
            if (it == e || *it != i || !keep[it - z.col.begin()]) continue;
            d.col.push_back(j);
            d.val.push_back(z.val[t]);
        }
        d.row[i + 1] = (int64_t)d.col.size();
    }
    return d;
}

// x + beta d on the union pattern
Sp plus_scaled(const Sp& x, double beta, const Sp& d) {
    Sp r(x.n);
    for (int64_t i = 0; i < x.n; ++i) {
        int64_t a = x.row[i], b = d.row[i];
        const int64_t ae = x.row[i + 1], be = d.row[i + 1];
        while (a < ae || b < be) {
            const int32_t ja = a < ae ? x.col[a] : INT32_MAX, jb = b < be ? d.col[b] : INT32_MAX;
            if (ja < jb) {
                r.col.push_back(ja);
                r.val.push_back(x.val[a++]);
            } else if (jb < ja) {
                r.col.push_back(jb);
                r.val.push_back(beta * d.val[b++]);
            } else {
                r.col.push_back(ja);
                r.val.push_back(x.val[a++] + beta * d.val[b++]);
            }
        }
        r.row[i + 1] = (int64_t)r.col.size();
    }
    return r;
}

}  // namespace

void build_cinv(HostPlan& P, int nit, double tol, int lfil) {
    const int64_t s = P.s, m = P.m;
    if (nit < 0 || !(tol >= 0.0) || lfil < 0) throw SetupError{DDLR_E_INVALID, "approximate inverse: bad iteration count, tolerance or fill"};
    Sp C(s);
    for (int64_t y = 0; y < s; ++y) {
        for (int64_t t = P.A0.rp[m + y]; t < P.A0.rp[m + y + 1]; ++t) {
            C.col.push_back((int32_t)(P.A0.ci[t] - m));
            C.val.push_back(P.A0.v[t]);
        }
        C.row[y + 1] = (int64_t)C.col.size();
    }
    Sp X(s);
    for (int64_t y = 0; y < s; ++y) {
        const double d = C.at(y, (int32_t)y);
        if (!(d > 0.0)) throw SetupError{DDLR_E_BREAKDOWN, "approximate inverse: C_alpha has a non-positive diagonal entry"};
        X.col.push_back((int32_t)y);
        X.val.push_back(1.0 / d);
        X.row[y + 1] = y + 1;
    }
    P.x_res.clear();
    P.x_iters = 0;
    for (int it = 0;; ++it) {
        const Sp R = identity_minus(product(C, X));
        P.x_res.push_back(frobenius(R));
        P.x_rinf = 0.0;
        for (int64_t i = 0; i < s; ++i) {
            double rowsum = 0.0;
            for (int64_t t = R.row[i]; t < R.row[i + 1]; ++t) rowsum += std::fabs(R.val[t]);
            P.x_rinf = std::max(P.x_rinf, rowsum);
        }
        if (it == nit) break;
        const Sp Z = dropped(symmetrised(product(X, R)), tol, lfil);
        const Sp W = product(C, Z);
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < s; ++i)
            for (int64_t t = W.row[i]; t < W.row[i + 1]; ++t) {
                num += R.at(i, W.col[t]) * W.val[t];
                den += W.val[t] * W.val[t];
            }
        if (!(den > 0.0)) break;
        X = plus_scaled(X, num / den, Z);
        P.x_iters = it + 1;
    }
    P.x_spd = P.x_rinf < 1.0;
    P.X.rp.assign(X.row.begin(), X.row.end());
    P.X.ci = std::move(X.col);
    P.X.v = std::move(X.val);
}

}  // namespace ddlr
