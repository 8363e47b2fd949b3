// Spectrum estimate for the Chebyshev solver of C_alpha (Sec. 4.3 (sec:csolve)).
//
// The preconditioner of the Chebyshev iteration is the block-Jacobi matrix
// D_alpha = blockdiag(C_i) (C_i: the couplings among subdomain i's interface
// unknowns), kept as the interface block of the incomplete factor L, D.  The
// interval for the Chebyshev polynomial comes from mc Lanczos steps on the
// pencil (C_alpha, D_alpha), i.e. on D_alpha^{-1} C_alpha in the D_alpha inner
// product, started from the vector of ones:
//   z = D^{-1} r, b_0 = sqrt(r.z), v = z / b_0, y = r / b_0   (y = D v)
//   w = C v, a_j = v.w, w -= a_j y_j + b_{j-1} y_{j-1},
//   z = D^{-1} w, b_j = sqrt(w.z), v_{j+1} = z / b_j, y_{j+1} = w / b_j.
// The extreme eigenvalues of the tridiagonal T_mc are widened by their
// residual bounds b_mc |s_mc| (s: the Ritz vector's last entry), the
// safeguard that turns the estimates into working bounds; a lower end that is
// not positive becomes half the smallest Ritz value.
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
    // z = D_alpha^{-1} r on interface-local vectors
    auto dsolve = [&](const std::vector<double>& r, std::vector<double>& z) {
        z = r;
        for (int64_t y = 0; y < s; ++y) {
            double acc = z[y];
            for (int64_t t = P.L.rp[m + y]; t < P.L.rp[m + y + 1]; ++t) acc -= P.L.v[t] * z[P.L.ci[t] - m];
            z[y] = acc;
        }
        for (int64_t y = 0; y < s; ++y) z[y] /= P.D[m + y];
        for (int64_t y = s - 1; y >= 0; --y) {
            const double zy = z[y];
            for (int64_t t = P.L.rp[m + y]; t < P.L.rp[m + y + 1]; ++t) z[P.L.ci[t] - m] -= P.L.v[t] * zy;
        }
    };
    auto cmul = [&](const std::vector<double>& x, std::vector<double>& out) {
        for (int64_t y = 0; y < s; ++y) {
            double acc = 0.0;
            for (int64_t t = P.A0.rp[m + y]; t < P.A0.rp[m + y + 1]; ++t) acc += P.A0.v[t] * x[P.A0.ci[t] - m];
            out[y] = acc;
        }
    };
    auto dotp = [&](const std::vector<double>& a, const std::vector<double>& b) {
        double t = 0.0;
        for (int64_t y = 0; y < s; ++y) t += a[y] * b[y];
        return t;
    };
    std::vector<double> r(s, 1.0), z(s), v(s), yv(s), yp(s, 0.0), w(s);
    dsolve(r, z);
    const double b0 = std::sqrt(dotp(r, z));
    for (int64_t y = 0; y < s; ++y) {
        v[y] = z[y] / b0;
        yv[y] = r[y] / b0;
    }
    std::vector<double> al, be;
    double bprev = 0.0;
    for (int j = 0; j < mc; ++j) {
        cmul(v, w);
        const double a = dotp(v, w);
        al.push_back(a);
        for (int64_t y = 0; y < s; ++y) w[y] -= a * yv[y] + bprev * yp[y];
        dsolve(w, z);
        const double wz = dotp(w, z);
        double b = wz > 0.0 ? std::sqrt(wz) : 0.0;
        if (!(b > 1e-14 * std::fabs(al[0]))) {
            be.push_back(0.0);
            break;
        }
        be.push_back(b);
        for (int64_t y = 0; y < s; ++y) {
            yp[y] = yv[y];
            v[y] = z[y] / b;
            yv[y] = w[y] / b;
        }
        bprev = b;
    }
    const int mm = (int)al.size();
    std::vector<double> ev, Z;
    tridiag_eig(mm, al.data(), be.data(), ev, Z);
    int imax = 0, imin = 0;
    for (int i = 1; i < mm; ++i) {
        if (ev[i] > ev[imax]) imax = i;
        if (ev[i] < ev[imin]) imin = i;
    }
    const double bl = be[mm - 1];
    P.ch_rhi = ev[imax];
    P.ch_rlo = ev[imin];
    P.ch_hi = ev[imax] + bl * std::fabs(Z[(size_t)(mm - 1) + (size_t)imax * mm]);
    P.ch_lo = ev[imin] - bl * std::fabs(Z[(size_t)(mm - 1) + (size_t)imin * mm]);
    if (!(P.ch_lo > 0.0)) P.ch_lo = 0.5 * ev[imin];
}

}  // namespace ddlr
