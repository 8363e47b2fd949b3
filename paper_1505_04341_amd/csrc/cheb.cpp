// Spectrum estimate for the Chebyshev solver of C_alpha (Sec. 4.3 (sec:csolve)).
//
// The preconditioner of the Chebyshev iteration is the block-Jacobi matrix
// D_alpha = blockdiag(C_i) (C_i: the couplings among subdomain i's interface
// unknowns), kept as the interface block of the incomplete factor,
// D_alpha = L diag(d) L^T.  The interval for the Chebyshev polynomial comes
// from mc Lanczos steps on the pencil (C_alpha, D_alpha) started from the
// vector of ones.  With positive pivots d, G = L diag(d)^{1/2} gives
// D_alpha = G G^T, and the pencil's Lanczos process is the ordinary
// symmetric Lanczos process on K = G^{-1} C_alpha G^{-T} in the Euclidean
// inner product, started from G^{-1} 1 (the basis vectors u_j = G^T v_j of
// the pencil's D_alpha-orthonormal v_j); that is what runs here:
//   w = K u_j - b_{j-1} u_{j-1},  a_j = u_j . w,  w -= a_j u_j,
//   b_j = ||w||,  u_{j+1} = w / b_j,
// stopped early when b_j <= 1e-14 |a_1|.  The extreme eigenvalues of the
// tridiagonal T are widened by their residual bounds b_m |s_m| (s: the Ritz
// vector's last entry), the safeguard that turns the estimates into working
// bounds; a lower end that is not positive becomes half the smallest Ritz
// value.  A pivot of D_alpha that is not positive is refused (the pencil is
// then not definite and the Chebyshev solver has no interval).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ddlr.h"
#include "host_setup.hpp"

namespace ddlr {

void cheb_bounds(HostPlan& P, int mc) {
    const int64_t m = P.m, s = P.s;
    if (mc < 2 || s < 2) throw SetupError{DDLR_E_INVALID, "Chebyshev: at least 2 Lanczos steps and 2 interface unknowns"};
    std::vector<double> sq(s);  // diag(d)^{1/2} of the interface block
    for (int64_t y = 0; y < s; ++y) {
        if (!(P.D[m + y] > 0.0))
            throw SetupError{DDLR_E_BREAKDOWN, "Chebyshev: D_alpha has a pivot that is not positive (interface row " +
                                                   std::to_string(y) + ")"};
        sq[y] = std::sqrt(P.D[m + y]);
    }
    const int64_t* lrp = P.L.rp.data() + m;
    // out = G^{-1} in: forward substitution with L, then the scaling
    auto g_inv = [&](std::vector<double>& t) {
        for (int64_t y = 0; y < s; ++y) {
            double acc = t[y];
            for (int64_t q = lrp[y]; q < lrp[y + 1]; ++q) acc -= P.L.v[q] * t[P.L.ci[q] - m];
            t[y] = acc;
        }
        for (int64_t y = 0; y < s; ++y) t[y] /= sq[y];
    };
    // out = G^{-T} in: the scaling, then backward substitution with L^T
    auto g_inv_t = [&](std::vector<double>& t) {
        for (int64_t y = 0; y < s; ++y) t[y] /= sq[y];
        for (int64_t y = s - 1; y >= 0; --y)
            for (int64_t q = lrp[y]; q < lrp[y + 1]; ++q) t[P.L.ci[q] - m] -= P.L.v[q] * t[y];
    };
    auto c_times = [&](const std::vector<double>& x, std::vector<double>& out) {
        for (int64_t y = 0; y < s; ++y) {
            double acc = 0.0;
            for (int64_t q = P.A0.rp[m + y]; q < P.A0.rp[m + y + 1]; ++q) acc += P.A0.v[q] * x[P.A0.ci[q] - m];
            out[y] = acc;
        }
    };
    auto norm = [&](const std::vector<double>& x) {
        double t = 0.0;
        for (double v : x) t += v * v;
        return std::sqrt(t);
    };
    std::vector<double> u(s, 1.0), uprev(s, 0.0), t(s), w(s), diag, off;
    g_inv(u);
    const double nu = norm(u);
    for (double& v : u) v /= nu;
    double bprev = 0.0;
    for (int j = 0; j < mc; ++j) {
        t = u;
        g_inv_t(t);
        c_times(t, w);
        g_inv(w);
        for (int64_t y = 0; y < s; ++y) w[y] -= bprev * uprev[y];
        double a = 0.0;
        for (int64_t y = 0; y < s; ++y) a += u[y] * w[y];
        for (int64_t y = 0; y < s; ++y) w[y] -= a * u[y];
        diag.push_back(a);
        const double b = norm(w);
        if (!(b > 1e-14 * std::fabs(diag[0]))) {
            off.push_back(0.0);
            break;
        }
        off.push_back(b);
        uprev.swap(u);
        for (int64_t y = 0; y < s; ++y) u[y] = w[y] / b;
        bprev = b;
    }
    const int steps = (int)diag.size();
    std::vector<double> ev, Z;
    tridiag_eig(steps, diag.data(), off.data(), ev, Z);
    const int top = (int)(std::max_element(ev.begin(), ev.end()) - ev.begin());
    const int bot = (int)(std::min_element(ev.begin(), ev.end()) - ev.begin());
    const double blast = off[steps - 1];
    P.ch_rhi = ev[top];
    P.ch_rlo = ev[bot];
    P.ch_hi = ev[top] + blast * std::fabs(Z[(size_t)(steps - 1) + (size_t)top * steps]);
    P.ch_lo = ev[bot] - blast * std::fabs(Z[(size_t)(steps - 1) + (size_t)bot * steps]);
    if (!(P.ch_lo > 0.0)) P.ch_lo = 0.5 * ev[bot];
}

}  // namespace ddlr
