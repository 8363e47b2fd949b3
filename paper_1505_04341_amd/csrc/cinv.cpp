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
// are single running sums over stored entries in row-major order; R keeps an
// entry for every entry of C X and for the diagonal.
//
// This implementation works on coordinate lists: a product expands the
// terms of each output row as (column, k, value) triples, orders them by
// column (stably, so k stays ascending) and sums each run; symmetrisation and
// the two-sided survivor test pair entries by sorting (row, column) keys.
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

// Square sparse matrix in compressed rows, columns ascending in each row.
struct Rows {
    int64_t n = 0;
    std::vector<int64_t> start;  // n + 1
    std::vector<int32_t> col;
    std::vector<double> val;
    explicit Rows(int64_t n_ = 0) : n(n_), start(1, 0) { start.reserve(n_ + 1); }
    void close_row() { start.push_back((int64_t)col.size()); }
    void put(int32_t j, double v) {
        col.push_back(j);
        val.push_back(v);
    }
};

struct Term {
    int32_t j;
    double v;
};

// a * b: row i gathers the terms a_ik b_kj for its k in ascending order,
// orders them by j keeping that order, and sums each run from 0.0.
Rows multiply(const Rows& a, const Rows& b) {
    Rows c(a.n);
    std::vector<Term> terms;
    for (int64_t i = 0; i < a.n; ++i) {
        terms.clear();
        for (int64_t t = a.start[i]; t < a.start[i + 1]; ++t) {
            const int32_t k = a.col[t];
            for (int64_t u = b.start[k]; u < b.start[k + 1]; ++u) terms.push_back({b.col[u], a.val[t] * b.val[u]});
        }
        std::stable_sort(terms.begin(), terms.end(), [](const Term& x, const Term& y) { return x.j < y.j; });
        for (size_t q = 0; q < terms.size();) {
            const int32_t j = terms[q].j;
            double sum = 0.0;
            for (; q < terms.size() && terms[q].j == j; ++q) sum += terms[q].v;
            c.put(j, sum);
        }
        c.close_row();
    }
    return c;
}

// R = I - W on the pattern of W plus the diagonal: 1 - w_ii, -w_ij, or 1
Rows residual(const Rows& w) {
    Rows r(w.n);
    for (int64_t i = 0; i < w.n; ++i) {
        const int32_t d = (int32_t)i;
        int64_t t = w.start[i];
        const int64_t te = w.start[i + 1];
        for (; t < te && w.col[t] < d; ++t) r.put(w.col[t], -w.val[t]);
        if (t < te && w.col[t] == d) r.put(d, 1.0 - w.val[t++]);
        else r.put(d, 1.0);
        for (; t < te; ++t) r.put(w.col[t], -w.val[t]);
        r.close_row();
    }
    return r;
}

struct Coo {
    int32_t i, j;
    double v;
    bool operator<(const Coo& o) const { return i != o.i ? i < o.i : j < o.j; }
};

// (z + z^T) / 2 on the union pattern: every entry listed once as (i, j) and
// once transposed; sorting pairs the two copies of an entry that has both.
Rows symmetrise(const Rows& z) {
    std::vector<Coo> e;
    e.reserve(2 * z.col.size());
    for (int64_t i = 0; i < z.n; ++i)
        for (int64_t t = z.start[i]; t < z.start[i + 1]; ++t) {
            e.push_back({(int32_t)i, z.col[t], z.val[t]});
            e.push_back({z.col[t], (int32_t)i, z.val[t]});
        }
    std::sort(e.begin(), e.end());  // (i, j) and its transposed copy are adjacent
    Rows s(z.n);
    size_t q = 0;
    for (int64_t i = 0; i < z.n; ++i) {
        for (; q < e.size() && e[q].i == i; ++q) {
            if (e[q].i == e[q].j) {  // the diagonal appears twice with one value
                s.put(e[q].j, 0.5 * (e[q].v + e[q].v));
                ++q;
            } else if (q + 1 < e.size() && e[q + 1].i == e[q].i && e[q + 1].j == e[q].j) {
                s.put(e[q].j, 0.5 * (e[q].v + e[q + 1].v));
                ++q;
            } else {
                s.put(e[q].j, 0.5 * (e[q].v + 0.0));
            }
        }
        s.close_row();
    }
    return s;
}

// The dropping rule on symmetric z (column j = row j): each column selects
// its survivors; an entry is kept when both its column and its row selected it.
Rows drop(const Rows& z, double tol, int lfil) {
    std::vector<Coo> picks;  // (column, row) of every selection, listed as (min, max)
    std::vector<int64_t> cand;
    for (int64_t j = 0; j < z.n; ++j) {
        const int64_t a = z.start[j], e = z.start[j + 1];
        double sq = 0.0;
        for (int64_t t = a; t < e; ++t) sq += z.val[t] * z.val[t];
        const double thr = tol * std::sqrt(sq);
        cand.clear();
        for (int64_t t = a; t < e; ++t)
            if (z.col[t] != j && !(std::fabs(z.val[t]) < thr)) cand.push_back(t);
        const size_t keep = std::min<size_t>(cand.size(), (size_t)std::max(lfil, 0));
        // the keep largest magnitudes, equal magnitudes by ascending row
        std::partial_sort(cand.begin(), cand.begin() + keep, cand.end(), [&](int64_t x, int64_t y) {
            const double ax = std::fabs(z.val[x]), ay = std::fabs(z.val[y]);
            return ax != ay ? ax > ay : z.col[x] < z.col[y];
        });
        for (size_t q = 0; q < keep; ++q) {
            const int32_t i = z.col[cand[q]];
            picks.push_back({std::min((int32_t)j, i), std::max((int32_t)j, i), 0.0});
        }
    }
    std::sort(picks.begin(), picks.end());
    // an off-diagonal pair selected from both sides appears twice
    std::vector<Coo> both;
    for (size_t q = 0; q + 1 < picks.size(); ++q)
        if (picks[q].i == picks[q + 1].i && picks[q].j == picks[q + 1].j) {
            both.push_back(picks[q]);
            both.push_back({picks[q].j, picks[q].i, 0.0});
            ++q;
        }
    std::sort(both.begin(), both.end());
    Rows d(z.n);
    size_t q = 0;
    for (int64_t i = 0; i < z.n; ++i) {
        for (int64_t t = z.start[i]; t < z.start[i + 1]; ++t) {
            const int32_t j = z.col[t];
            if (j == i) {
                d.put(j, z.val[t]);
                continue;
            }
            while (q < both.size() && (both[q].i < i || (both[q].i == i && both[q].j < j))) ++q;
            if (q < both.size() && both[q].i == i && both[q].j == j) d.put(j, z.val[t]);
        }
        d.close_row();
    }
    return d;
}

// x + beta d on the union pattern
Rows axpy(const Rows& x, double beta, const Rows& d) {
    Rows r(x.n);
    for (int64_t i = 0; i < x.n; ++i) {
        int64_t a = x.start[i], b = d.start[i];
        const int64_t ae = x.start[i + 1], be = d.start[i + 1];
        while (a < ae && b < be) {
            if (x.col[a] < d.col[b]) {
                r.put(x.col[a], x.val[a]);
                ++a;
            } else if (d.col[b] < x.col[a]) {
                r.put(d.col[b], beta * d.val[b]);
                ++b;
            } else {
                r.put(x.col[a], x.val[a] + beta * d.val[b]);
                ++a, ++b;
            }
        }
        for (; a < ae; ++a) r.put(x.col[a], x.val[a]);
        for (; b < be; ++b) r.put(d.col[b], beta * d.val[b]);
        r.close_row();
    }
    return r;
}

}  // namespace

void build_cinv(HostPlan& P, int nit, double tol, int lfil) {
    const int64_t s = P.s, m = P.m;
    if (nit < 0 || !(tol >= 0.0) || lfil < 0)
        throw SetupError{DDLR_E_INVALID, "approximate inverse: bad iteration count, tolerance or fill"};
    Rows C(s), X(s);
    for (int64_t y = 0; y < s; ++y) {
        double dg = 0.0;
        for (int64_t t = P.A0.rp[m + y]; t < P.A0.rp[m + y + 1]; ++t) {
            const int32_t j = (int32_t)(P.A0.ci[t] - m);
            C.put(j, P.A0.v[t]);
            if (j == y) dg = P.A0.v[t];
        }
        C.close_row();
        if (!(dg > 0.0))
            throw SetupError{DDLR_E_BREAKDOWN, "approximate inverse: C_alpha has a non-positive diagonal entry"};
        X.put((int32_t)y, 1.0 / dg);
        X.close_row();
    }
    P.x_res.clear();
    P.x_iters = 0;
    for (int it = 0;; ++it) {
        const Rows R = residual(multiply(C, X));
        double fro = 0.0;
        for (double v : R.val) fro += v * v;
        P.x_res.push_back(std::sqrt(fro));
        P.x_rinf = 0.0;
        for (int64_t i = 0; i < s; ++i) {
            double rowsum = 0.0;
            for (int64_t t = R.start[i]; t < R.start[i + 1]; ++t) rowsum += std::fabs(R.val[t]);
            P.x_rinf = std::max(P.x_rinf, rowsum);
        }
        if (it == nit) break;
        const Rows Z = drop(symmetrise(multiply(X, R)), tol, lfil);
        const Rows W = multiply(C, Z);
        // tr(R^T W) and ||W||_F^2 over W's entries in row-major order; R_ij by a
        // merge of the two sorted rows
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < s; ++i) {
            int64_t a = R.start[i];
            const int64_t ae = R.start[i + 1];
            for (int64_t t = W.start[i]; t < W.start[i + 1]; ++t) {
                while (a < ae && R.col[a] < W.col[t]) ++a;
                const double rij = (a < ae && R.col[a] == W.col[t]) ? R.val[a] : 0.0;
                num += rij * W.val[t];
                den += W.val[t] * W.val[t];
            }
        }
        if (!(den > 0.0)) break;
        X = axpy(X, num / den, Z);
        P.x_iters = it + 1;
    }
    P.x_spd = P.x_rinf < 1.0;
    P.X.rp.assign(X.start.begin(), X.start.end());
    P.X.ci = std::move(X.col);
    P.X.v = std::move(X.val);
}

}  // namespace ddlr
