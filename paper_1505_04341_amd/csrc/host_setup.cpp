// Host-side construction of the DDLR splitting, local factors and GPU schedule.
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <utility>

#include "ddlr.h"

namespace ddlr {

namespace {

[[noreturn]] void fail(int st, std::string msg) { throw SetupError{st, std::move(msg)}; }

// Stable counting sort of indices 0..cnt-1 by key in [0, nkeys).
std::vector<int32_t> counting_order(const std::vector<int32_t>& key, int32_t nkeys) {
    std::vector<int64_t> start(nkeys + 1, 0);
    for (int32_t k : key) start[k + 1]++;
    for (int32_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
    std::vector<int32_t> out(key.size());
    for (size_t i = 0; i < key.size(); ++i) out[start[key[i]]++] = (int32_t)i;
    return out;
}

}  // namespace

void validate(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, const int32_t* part, int32_t p) {
    if (n < 1 || !rp || !ci || !v || !part) fail(DDLR_E_INVALID, "null array or n < 1");
    if (p < 1 || p > n) fail(DDLR_E_INVALID, "p must be in [1, n]");
    if (rp[0] != 0) fail(DDLR_E_INVALID, "row_ptr[0] must be 0");
    if (rp[n] > INT32_MAX) fail(DDLR_E_INVALID, "nnz(A) must fit in int32");
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) fail(DDLR_E_INVALID, "row_ptr not monotone at row " + std::to_string(i));
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            if (ci[t] < 0 || ci[t] >= n) fail(DDLR_E_INVALID, "column index out of range in row " + std::to_string(i));
            if (t > rp[i] && ci[t] <= ci[t - 1]) fail(DDLR_E_INVALID, "columns not sorted/unique in row " + std::to_string(i));
        }
        if (part[i] < 0 || part[i] >= p) fail(DDLR_E_INVALID, "part[" + std::to_string(i) + "] outside [0,p)");
    }
    // symmetry: the transpose built by counting must equal A entry for entry
    std::vector<int64_t> tp(n + 1, 0);
    for (int64_t t = 0; t < rp[n]; ++t) tp[ci[t] + 1]++;
    for (int64_t j = 0; j < n; ++j) tp[j + 1] += tp[j];
    for (int64_t j = 0; j <= n; ++j)
        if (tp[j] != rp[j]) fail(DDLR_E_NOT_SYMMETRIC, "row and column counts differ at " + std::to_string(j));
    std::vector<int32_t> tc(rp[n]);
    std::vector<double> tv(rp[n]);
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            int64_t q = fill[ci[t]]++;
            tc[q] = (int32_t)i;
            tv[q] = v[t];
        }
    for (int64_t t = 0; t < rp[n]; ++t)
        if (tc[t] != ci[t] || tv[t] != v[t]) fail(DDLR_E_NOT_SYMMETRIC, "A is not symmetric");
}

namespace {

// Step 1: interface flags, internal order, colouring of the interface block.
void order_unknowns(HostPlan& P, const int64_t* rp, const int32_t* ci, const int32_t* part, int corder) {
    const int64_t n = P.n;
    const int32_t p = P.p;
    P.iface.assign(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t)
            if (part[ci[t]] != part[i]) { P.iface[i] = 1; break; }
    // key: interiors of 0..p-1 come first, then interfaces of 0..p-1
    std::vector<int32_t> key(n);
    for (int64_t i = 0; i < n; ++i) key[i] = part[i] + (P.iface[i] ? p : 0);
    P.perm = counting_order(key, 2 * p);
    P.boff.assign(p + 2, 0);
    for (int64_t i = 0; i < n; ++i)
        if (!P.iface[i]) P.boff[part[i] + 1]++;
    for (int32_t b = 0; b < p; ++b) P.boff[b + 1] += P.boff[b];
    P.m = P.boff[p];
    P.s = n - P.m;
    P.boff[p + 1] = n;
    P.iperm.assign(n, 0);
    for (int64_t q = 0; q < n; ++q) P.iperm[P.perm[q]] = (int32_t)q;
    P.colour.assign(P.s, 0);
    P.ncolours = P.s > 0 ? 1 : 0;
    if (corder != 0 || P.s == 0) return;
    // greedy colouring of C's graph, interface positions in ascending order
    std::vector<int64_t> stamp;
    int32_t ncol = 0;
    for (int64_t y = 0; y < P.s; ++y) {
        int32_t u = P.perm[P.m + y];
        for (int64_t t = rp[u]; t < rp[u + 1]; ++t) {
            int32_t w = ci[t];
            if (w == u || !P.iface[w]) continue;
            int64_t yw = P.iperm[w] - P.m;
            if (yw < y) {
                int32_t c = P.colour[yw];
                if ((int32_t)stamp.size() <= c) stamp.resize(c + 1, -1);
                stamp[c] = y;
            }
        }
        int32_t c = 0;
        while (c < (int32_t)stamp.size() && stamp[c] == y) ++c;
        P.colour[y] = c;
        ncol = std::max(ncol, c + 1);
    }
    P.ncolours = ncol;
    std::vector<int32_t> ord = counting_order(P.colour, ncol);
    std::vector<int32_t> nperm(P.s), ncolour(P.s);
    for (int64_t q = 0; q < P.s; ++q) {
        nperm[q] = P.perm[P.m + ord[q]];
        ncolour[q] = P.colour[ord[q]];
    }
    std::copy(nperm.begin(), nperm.end(), P.perm.begin() + P.m);
    P.colour = ncolour;
    for (int64_t q = 0; q < n; ++q) P.iperm[P.perm[q]] = (int32_t)q;
}

// P A P^T by two stable counting passes (columns, then rows).
void permute_matrix(HostPlan& P, const int64_t* rp, const int32_t* ci, const double* v) {
    const int64_t n = P.n, nnz = rp[n];
    std::vector<int32_t> row(nnz), col(nnz);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            row[t] = P.iperm[i];
            col[t] = P.iperm[ci[t]];
        }
    std::vector<int32_t> byc = counting_order(col, (int32_t)n);
    std::vector<int32_t> rkey(nnz);
    for (int64_t q = 0; q < nnz; ++q) rkey[q] = row[byc[q]];
    std::vector<int32_t> byr = counting_order(rkey, (int32_t)n);
    P.A.rp.assign(n + 1, 0);
    P.A.ci.resize(nnz);
    P.A.v.resize(nnz);
    for (int64_t q = 0; q < nnz; ++q) {
        int64_t t = byc[byr[q]];
        P.A.ci[q] = col[t];
        P.A.v[q] = v[t];
        P.A.rp[row[t] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) P.A.rp[i + 1] += P.A.rp[i];
}

// Step 2: A0 = blockdiag(B + alpha^{-2} Ehat Ehat^T, C + alpha^2 I).
void form_a0(HostPlan& P) {
    const int64_t n = P.n, m = P.m;
    const double ia2 = 1.0 / (P.alpha * P.alpha), a2 = P.alpha * P.alpha;
    const HostCsr& A = P.A;
    P.A0.rp.assign(n + 1, 0);
    P.A0.ci.clear();
    P.A0.v.clear();
    std::vector<std::pair<int32_t, double>> prod;
    for (int64_t r = 0; r < n; ++r) {
        prod.clear();
        if (r < m) {
            // products Ehat_{rc} Ehat_{jc} over interface c (ascending), j interior
            for (int64_t t = A.rp[r]; t < A.rp[r + 1]; ++t) {
                int32_t c = A.ci[t];
                if (c < m) continue;
                for (int64_t t2 = A.rp[c]; t2 < A.rp[c + 1]; ++t2) {
                    int32_t j = A.ci[t2];
                    if (j < m) prod.emplace_back(j, ia2 * A.v[t] * A.v[t2]);
                }
            }
            std::stable_sort(prod.begin(), prod.end(),
                             [](const auto& x, const auto& y) { return x.first < y.first; });
            // merge B's row (interior columns) with the combined products
            int64_t t = A.rp[r], te = A.rp[r + 1];
            size_t q = 0;
            while (t < te || q < prod.size()) {
                int32_t cb = (t < te && A.ci[t] < m) ? A.ci[t] : INT32_MAX;
                if (t < te && A.ci[t] >= m) { ++t; continue; }
                int32_t cq = q < prod.size() ? prod[q].first : INT32_MAX;
                int32_t c = std::min(cb, cq);
                if (c == INT32_MAX) break;
                double val = 0.0;
                if (cb == c) { val = A.v[t]; ++t; }
                while (q < prod.size() && prod[q].first == c) { val += prod[q].second; ++q; }
                P.A0.ci.push_back(c);
                P.A0.v.push_back(val);
            }
        } else {
            bool diag_done = false;
            for (int64_t t = A.rp[r]; t < A.rp[r + 1]; ++t) {
                int32_t c = A.ci[t];
                if (c < m) continue;
                if (!diag_done && c > r) {
                    P.A0.ci.push_back((int32_t)r);
                    P.A0.v.push_back(a2);
                    diag_done = true;
                }
                double val = A.v[t];
                if (c == r) { val += a2; diag_done = true; }
                P.A0.ci.push_back(c);
                P.A0.v.push_back(val);
            }
            if (!diag_done) {
                P.A0.ci.push_back((int32_t)r);
                P.A0.v.push_back(a2);
            }
        }
        P.A0.rp[r + 1] = (int64_t)P.A0.ci.size();
    }
}

// Step 3: incomplete LDL^T of each diagonal block of A0 by the IKJ form of the
// zero-fill incomplete LU factorisation on the block's symmetric pattern; for
// a symmetric matrix U = D L^T, so L is the strict lower part and D the
// diagonal of the result.
void factor_blocks(HostPlan& P, int factor, const int32_t* part) {
    const int32_t nfact = P.csolve == 1 ? P.p : P.p + 1;  // blocks factored (C_alpha last)
    const int64_t n = P.n;
    HostCsr W = P.A0;  // working copy, both triangles
    if (P.csolve == 2) {
        // D_alpha = blockdiag(C_i): drop the interface couplings between subdomains
        HostCsr F;
        F.rp.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t t = W.rp[i]; t < W.rp[i + 1]; ++t) {
                const int64_t j = W.ci[t];
                if (i >= P.m && j >= P.m && part[P.perm[i]] != part[P.perm[j]]) continue;
                F.ci.push_back(W.ci[t]);
                F.v.push_back(W.v[t]);
            }
            F.rp[i + 1] = (int64_t)F.ci.size();
        }
        W = std::move(F);
    }
    std::vector<int64_t> diagpos(n, -1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = W.rp[i]; t < W.rp[i + 1]; ++t)
            if (W.ci[t] == i) diagpos[i] = t;
    std::vector<int64_t> where(n, -1);
    for (int32_t b = 0; b < nfact; ++b) {
        const int64_t lo = P.boff[b], hi = P.boff[b + 1];
        for (int64_t i = lo; i < hi; ++i) {
            for (int64_t t = W.rp[i]; t < W.rp[i + 1]; ++t) where[W.ci[t]] = t;
            const double aii = W.v[diagpos[i]];
            for (int64_t t = W.rp[i]; t < W.rp[i + 1]; ++t) {
                const int32_t k = W.ci[t];
                if (k < lo) continue;
                if (k >= i) break;
                W.v[t] /= W.v[diagpos[k]];
                const double lik = W.v[t];
                for (int64_t t2 = diagpos[k] + 1; t2 < W.rp[k + 1]; ++t2) {
                    const int32_t j = W.ci[t2];
                    if (j >= hi) break;
                    const int64_t pos = where[j];
                    if (pos >= 0) W.v[pos] -= lik * W.v[t2];
                }
            }
            for (int64_t t = W.rp[i]; t < W.rp[i + 1]; ++t) where[W.ci[t]] = -1;
            const double d = W.v[diagpos[i]];
            const bool bad = factor == 1 ? (d == 0.0 || std::fabs(d) < 1e-14 * std::fabs(aii)) : !(d > 0.0);
            if (bad)
                fail(DDLR_E_BREAKDOWN, "local factor breakdown: pivot " + std::to_string(d) + " at internal row " +
                                           std::to_string(i) + " (user row " + std::to_string(P.perm[i]) + ")");
        }
    }
    P.L.rp.assign(n + 1, 0);
    P.L.ci.clear();
    P.L.v.clear();
    P.D.assign(n, 1.0);
    for (int32_t b = 0; b <= P.p; ++b) {
        const int64_t lo = P.boff[b];
        for (int64_t i = lo; i < P.boff[b + 1]; ++i) {
            if (b < nfact) {
                for (int64_t t = W.rp[i]; t < diagpos[i]; ++t)
                    if (W.ci[t] >= lo) {
                        P.L.ci.push_back(W.ci[t]);
                        P.L.v.push_back(W.v[t]);
                    }
                P.D[i] = W.v[diagpos[i]];
            }
            P.L.rp[i + 1] = (int64_t)P.L.ci.size();
        }
    }
}

// Level schedule per block and the device order (levels contiguous).
void schedule(HostPlan& P) {
    const int64_t n = P.n;
    P.level.assign(n, 0);
    P.dev2int.assign(n, 0);
    P.int2dev.assign(n, 0);
    P.lvl_ptr.clear();
    P.blk_lvl.assign(P.p + 2, 0);
    P.levels_b_max = 0;
    for (int32_t b = 0; b <= P.p; ++b) {
        const int64_t lo = P.boff[b], hi = P.boff[b + 1];
        int32_t depth = 0;
        for (int64_t i = lo; i < hi; ++i) {
            int32_t lv = 0;
            for (int64_t t = P.L.rp[i]; t < P.L.rp[i + 1]; ++t) lv = std::max(lv, P.level[P.L.ci[t]] + 1);
            P.level[i] = lv;
            depth = std::max(depth, lv + 1);
        }
        std::vector<int32_t> key(hi - lo);
        for (int64_t i = lo; i < hi; ++i) key[i - lo] = P.level[i];
        std::vector<int32_t> ord = counting_order(key, std::max(depth, 1));
        P.blk_lvl[b] = (int32_t)P.lvl_ptr.size();
        int32_t prev = -1;
        for (int64_t q = 0; q < hi - lo; ++q) {
            int64_t i = lo + ord[q];
            P.dev2int[lo + q] = (int32_t)i;
            P.int2dev[i] = (int32_t)(lo + q);
            if (P.level[i] != prev) {
                P.lvl_ptr.push_back((int32_t)(lo + q));
                prev = P.level[i];
            }
        }
        if (b < P.p) P.levels_b_max = std::max(P.levels_b_max, depth);
        else P.levels_c = depth;
    }
    P.blk_lvl[P.p + 1] = (int32_t)P.lvl_ptr.size();
    P.lvl_ptr.push_back((int32_t)n);
}

}  // namespace

void build_plan(HostPlan& P, int64_t n, const int64_t* rp, const int32_t* ci, const double* v, const int32_t* part,
                int32_t p, double alpha, int factor, int corder, int csolve, int cinv_iters, double cinv_tol,
                int cinv_lfil, int cheb_lanczos) {
    if (!(alpha > 0.0) || !std::isfinite(alpha)) fail(DDLR_E_INVALID, "alpha must be positive");
    validate(n, rp, ci, v, part, p);
    P.n = n;
    P.p = p;
    P.alpha = alpha;
    order_unknowns(P, rp, ci, part, corder);
    if (P.s == 0) fail(DDLR_E_INVALID, "partition has no interface unknowns");
    permute_matrix(P, rp, ci, v);
    form_a0(P);
    P.csolve = csolve;
    factor_blocks(P, factor, part);
    if (csolve == 1) build_cinv(P, cinv_iters, cinv_tol, cinv_lfil);
    if (csolve == 2) cheb_bounds(P, cheb_lanczos);
    schedule(P);
}

void build_plan_imported(HostPlan& P, int64_t n, const int64_t* rp, const int32_t* ci, const double* v, int32_t p,
                         double alpha, std::vector<int32_t> perm, std::vector<int64_t> boff,
                         std::vector<int32_t> colour, HostCsr L, std::vector<double> D, int csolve) {
    if (!(alpha > 0.0) || !std::isfinite(alpha)) fail(DDLR_E_INVALID, "alpha must be positive");
    if (p < 1 || p > n) fail(DDLR_E_INVALID, "stored p outside [1, n]");
    if ((int64_t)perm.size() != n || (int64_t)boff.size() != p + 2 || (int64_t)D.size() != n ||
        L.rows() != n)
        fail(DDLR_E_INVALID, "stored setup does not match the matrix order");
    if (boff[0] != 0 || boff[p + 1] != n) fail(DDLR_E_INVALID, "stored block offsets must run from 0 to n");
    for (int32_t b = 0; b <= p; ++b)
        if (boff[b + 1] < boff[b]) fail(DDLR_E_INVALID, "stored block offsets not monotone");
    // the interior row of internal position q belongs to block blk[q]; interface rows to block p
    std::vector<int32_t> blk(n), part(n, 0);
    for (int32_t b = 0; b <= p; ++b)
        for (int64_t q = boff[b]; q < boff[b + 1]; ++q) blk[q] = b;
    std::vector<int32_t> seen(n, 0);
    for (int64_t q = 0; q < n; ++q) {
        const int32_t u = perm[q];
        if (u < 0 || u >= n || seen[u]) fail(DDLR_E_INVALID, "stored ordering is not a permutation");
        seen[u] = 1;
        if (blk[q] < p) part[u] = blk[q];
    }
    validate(n, rp, ci, v, part.data(), p);
    P.n = n;
    P.p = p;
    P.alpha = alpha;
    P.perm = std::move(perm);
    P.boff = std::move(boff);
    P.m = P.boff[p];
    P.s = n - P.m;
    if (P.s == 0) fail(DDLR_E_INVALID, "stored ordering has no interface unknowns");
    P.iperm.assign(n, 0);
    for (int64_t q = 0; q < n; ++q) P.iperm[P.perm[q]] = (int32_t)q;
    P.iface.assign(n, 0);
    for (int64_t u = 0; u < n; ++u) P.iface[u] = P.iperm[u] >= P.m;
    if ((int64_t)colour.size() != P.s) fail(DDLR_E_INVALID, "stored colours must have one entry per interface row");
    P.colour = std::move(colour);
    P.ncolours = 0;
    for (int32_t c : P.colour) {
        if (c < 0) fail(DDLR_E_INVALID, "negative stored colour");
        P.ncolours = std::max(P.ncolours, c + 1);
    }
    permute_matrix(P, rp, ci, v);
    // the splitting needs interior rows coupled only to their own block and the interface
    for (int64_t r = 0; r < P.m; ++r)
        for (int64_t t = P.A.rp[r]; t < P.A.rp[r + 1]; ++t) {
            const int32_t c = P.A.ci[t];
            if (c < P.m && blk[c] != blk[r])
                fail(DDLR_E_INVALID, "stored ordering couples the interiors of blocks " + std::to_string(blk[r]) +
                                         " and " + std::to_string(blk[c]) + " (internal row " + std::to_string(r) +
                                         ")");
        }
    form_a0(P);
    // the factor: strict lower, columns inside the row's block, ascending
    if (L.rp[0] != 0) fail(DDLR_E_INVALID, "stored L row pointer must start at 0");
    for (int64_t r = 0; r < n; ++r) {
        if (L.rp[r + 1] < L.rp[r] || L.rp[r + 1] > (int64_t)L.ci.size())
            fail(DDLR_E_INVALID, "stored L row pointer not monotone");
        const int64_t lo = P.boff[blk[r]];
        for (int64_t t = L.rp[r]; t < L.rp[r + 1]; ++t) {
            const int32_t c = L.ci[t];
            if (c < lo || c >= r || (t > L.rp[r] && c <= L.ci[t - 1]))
                fail(DDLR_E_INVALID, "stored L entry outside the strict lower block pattern in row " +
                                         std::to_string(r));
            if (!std::isfinite(L.v[t])) fail(DDLR_E_INVALID, "stored L value not finite");
        }
        if (!std::isfinite(D[r]) || D[r] == 0.0) fail(DDLR_E_INVALID, "stored pivot zero or not finite");
    }
    if ((int64_t)L.v.size() != L.rp[n] || (int64_t)L.ci.size() != L.rp[n])
        fail(DDLR_E_INVALID, "stored L arrays do not match its row pointer");
    P.L = std::move(L);
    P.D = std::move(D);
    P.csolve = csolve;
    schedule(P);
}

// Implicit symmetric QR with Wilkinson shifts (the implicit QR step of the
// symmetric tridiagonal eigenproblem, Golub & Van Loan, Sec. 8.3), on a dense
// copy with rotations restricted to the band.
void tridiag_eig(int m, const double* a, const double* b, std::vector<double>& ev, std::vector<double>& Z) {
    std::vector<double> T((size_t)m * m, 0.0);
    auto at = [&](int i, int j) -> double& { return T[(size_t)i + (size_t)j * m]; };
    for (int i = 0; i < m; ++i) {
        at(i, i) = a[i];
        if (i + 1 < m) at(i + 1, i) = at(i, i + 1) = b[i];
    }
    Z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Z[(size_t)i + (size_t)i * m] = 1.0;
    const double eps = 2.220446049250313e-16;
    int hi = m - 1, guard = 0;
    while (hi > 0 && guard < 60 * m) {
        if (std::fabs(at(hi, hi - 1)) <= eps * (std::fabs(at(hi - 1, hi - 1)) + std::fabs(at(hi, hi)))) {
            at(hi, hi - 1) = at(hi - 1, hi) = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(at(lo, lo - 1)) > eps * (std::fabs(at(lo - 1, lo - 1)) + std::fabs(at(lo, lo))))
            --lo;
        ++guard;
        const double d = 0.5 * (at(hi - 1, hi - 1) - at(hi, hi));
        const double e = at(hi, hi - 1);
        const double den = d + (d >= 0 ? 1.0 : -1.0) * std::hypot(d, e);
        const double mu = at(hi, hi) - (den != 0.0 ? e * e / den : 0.0);
        double x = at(lo, lo) - mu, z = at(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r > 0 ? x / r : 1.0, s = r > 0 ? z / r : 0.0;
            const int j0 = std::max(lo, k - 1), j1 = std::min(hi, k + 2);
            for (int j = j0; j <= j1; ++j) {  // rows k, k+1
                const double u = at(k, j), w = at(k + 1, j);
                at(k, j) = c * u + s * w;
                at(k + 1, j) = -s * u + c * w;
            }
            for (int i = j0; i <= j1; ++i) {  // columns k, k+1
                const double u = at(i, k), w = at(i, k + 1);
                at(i, k) = c * u + s * w;
                at(i, k + 1) = -s * u + c * w;
            }
            for (int i = 0; i < m; ++i) {
                double& zk = Z[(size_t)i + (size_t)k * m];
                double& zk1 = Z[(size_t)i + (size_t)(k + 1) * m];
                const double u = zk, w = zk1;
                zk = c * u + s * w;
                zk1 = -s * u + c * w;
            }
            if (k + 1 < hi) {
                x = at(k + 1, k);
                z = at(k + 2, k);
            }
        }
    }
    ev.resize(m);
    for (int i = 0; i < m; ++i) ev[i] = at(i, i);
}

}  // namespace ddlr
