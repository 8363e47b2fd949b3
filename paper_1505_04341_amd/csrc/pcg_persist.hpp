// Persistent PCG: one workgroup runs a whole preconditioned CG solve of one
// (system, right-hand side) lane in a single launch.
//
// The batching form of the path: many independent systems (and right-hand
// sides) go into one launch, one workgroup per lane, with no grid-wide
// synchronisation at all -- each workgroup iterates its own lane until the
// residual test of Sec. 5 holds or maxit is reached, then exits.  Every step of
// an iteration runs inside the workgroup, separated by workgroup barriers:
//   q = A p (CSR rows), alpha, x and r updates, the residual test;
//   z = M^{-1} r with DDLR-1 (eq. Mprec with eq. gkt, two A0 solves) or A0 alone:
//     the A0 solve walks "merged levels": level j of every block of the system
//     (the p subdomain blocks and the interface block are independent, so
//     their level-j rows go together), forward over L then backward over L^T
//     with D^{-1}; the solve vector stays in LDS when the system fits, else in
//     a global buffer of the lane;
//     y = E^T z1, the k coefficients d .* (U_k^T y), w = c0 y + U_k coef,
//     v = r + E w, and the second A0 solve;
//   the CG scalars, and p = z + beta p.
// Reductions are deterministic: a shuffle tree per wave, then the waves'
// partial sums in wave order, every thread forming the same total.  The
// triangular row sums use fnms in CSR order, as the other A0-solve kernels do,
// so the preconditioner's arithmetic is theirs; the Krylov scalars differ from
// the multi-launch form only in the order of the dot-product sums.
#pragma once

#include "kernels.hpp"

namespace ddlr {

struct PSys {
    int64_t r0;      // first device row of the system
    int64_t s0;      // first interface position (rows of U_k, y, w)
    int64_t d0;      // offset of d_1..d_k in the coefficient array
    int32_t n, m;    // rows; interior rows (the interface rows follow)
    int32_t s, k;    // interface rows; rank of the correction (0: A0 alone)
    int32_t l0, l1;  // merged levels l0..l1-1 (row lists in mrow[mlev[j] .. mlev[j+1]])
    int32_t lds;     // 1: the solve vector fits the dynamic LDS
    int32_t pad;
    double c0;       // eq. (gkt): G^{-1} = c0 I + U_k diag(d) U_k^T
};

struct PLane {
    int32_t sys;  // index into the system table
    int32_t col;  // column of the lane in the vectors (offset col * ld)
};

struct PRes {
    int32_t its, status;  // iterations; 0 converged, 1 maxit reached
    double rr, bb;        // ||r||^2 (recursive) and ||b||^2
    double rtrue;         // ||b - A x||^2 after the solve
};

constexpr int kPersistMaxK = 64;  // rank bound of the persistent form

// Sum over the workgroup, the same value in every thread.  `red` holds NT/64
// doubles of LDS; the barriers at entry and exit let consecutive calls reuse it.
template <int NT> __device__ __forceinline__ double wg_sum(double v, double* red) {
    constexpr int NW = NT / 64;
    v = wave_sum(v);  // lane 0 holds the wave's sum
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    __syncthreads();
    return s;
}

// The A0 solve of one lane: forward sweep over the merged levels (unit lower L),
// then backward (z_i = D_i^{-1} y_i - sum_j L_ji z_j).  x: input at global device
// rows; vec: the solve vector, indexed by local row (LDS) or by global row.
template <typename T, int NT, bool kLds, typename TIn>
__device__ void wg_a0_solve(const PSys& S, const int32_t* __restrict__ mlev, const int32_t* __restrict__ mrow,
                            const int32_t* __restrict__ lrp, const int32_t* __restrict__ lci, const T* __restrict__ lv,
                            const int32_t* __restrict__ urp, const int32_t* __restrict__ uci, const T* __restrict__ uv,
                            const T* __restrict__ dinv, const TIn* x, T* vec) {
    const int64_t off = kLds ? S.r0 : 0;
    for (int j = S.l0; j < S.l1; ++j) {
        const int a = mlev[j], e = mlev[j + 1];
        for (int q = a + (int)threadIdx.x; q < e; q += NT) {
            const int i = mrow[q];
            T s = (T)x[i];
            const int t1 = lrp[i + 1];
            for (int t = lrp[i]; t < t1; ++t) s = fnms(s, lv[t], vec[lci[t] - off]);
            vec[i - off] = s;
        }
        __syncthreads();
    }
    for (int j = S.l1 - 1; j >= S.l0; --j) {
        const int a = mlev[j], e = mlev[j + 1];
        for (int q = a + (int)threadIdx.x; q < e; q += NT) {
            const int i = mrow[q];
            T s = vec[i - off] * dinv[i];
            const int t1 = urp[i + 1];
            for (int t = urp[i]; t < t1; ++t) s = fnms(s, uv[t], vec[uci[t] - off]);
            vec[i - off] = s;
        }
        __syncthreads();
    }
}

// z = M^{-1} r for one lane (r, z: double at global device rows; tg: the lane's
// global T buffer of n rows used when the solve vector is not in LDS; y, w: the
// lane's interface vectors).  Ends with a barrier.
template <typename T, int NT, bool kLds>
__device__ void wg_apply(const PSys& S, const int32_t* __restrict__ mlev, const int32_t* __restrict__ mrow,
                         const int32_t* __restrict__ lrp, const int32_t* __restrict__ lci, const T* __restrict__ lv,
                         const int32_t* __restrict__ urp, const int32_t* __restrict__ uci, const T* __restrict__ uv,
                         const T* __restrict__ dinv, const int32_t* __restrict__ erp, const int32_t* __restrict__ eci,
                         const T* __restrict__ ev, const int32_t* __restrict__ etrp, const int32_t* __restrict__ etci,
                         const T* __restrict__ etv, const T* __restrict__ U, int ustride,
                         const double* __restrict__ dcoef, const double* r, double* z, T* tg, T* y, T* w, T* lvec,
                         double* red, double* coef) {
    T* vec = kLds ? lvec : tg;
    const int64_t off = kLds ? S.r0 : 0;
    const int64_t r0 = S.r0, r1 = S.r0 + S.n;
    wg_a0_solve<T, NT, kLds, double>(S, mlev, mrow, lrp, lci, lv, urp, uci, uv, dinv, r, vec);
    if (S.k > 0) {
        const int64_t s0 = S.s0, s1 = S.s0 + S.s;
        // y = E^T z1 over the lane's interface positions (terms in CSR order, one rounding each)
        for (int64_t jg = s0 + threadIdx.x; jg < s1; jg += NT) {
            T acc = T(0);
            const int t1 = etrp[jg + 1];
            for (int t = etrp[jg]; t < t1; ++t) acc = fnms(acc, -etv[t], vec[etci[t] - off]);
            y[jg] = acc;
        }
        __syncthreads();
        // coef_j = d_j sum_i U_ij y_i, 16 columns at a time
        constexpr int NW = NT / 64;
        for (int j0 = 0; j0 < S.k; j0 += 16) {
            double acc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = 0.0;
            for (int64_t ig = s0 + threadIdx.x; ig < s1; ig += NT) {
                const double yi = (double)y[ig];
                const T* Ui = U + ig * ustride + j0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (j0 + u < S.k) acc[u] += (double)Ui[u] * yi;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const double v = wave_sum(acc[u]);
                if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * 16 + u] = v;
            }
            __syncthreads();
            if ((int)threadIdx.x < 16 && j0 + (int)threadIdx.x < S.k) {
                double sum = 0.0;
                for (int wv = 0; wv < NW; ++wv) sum += red[wv * 16 + threadIdx.x];
                coef[j0 + threadIdx.x] = dcoef[S.d0 + j0 + threadIdx.x] * sum;
            }
            __syncthreads();
        }
        // w = c0 y + U_k coef
        for (int64_t ig = s0 + threadIdx.x; ig < s1; ig += NT) {
            double acc = S.c0 * (double)y[ig];
            const T* Ui = U + ig * ustride;
            for (int j = 0; j < S.k; ++j) acc += (double)Ui[j] * coef[j];
            w[ig] = (T)acc;
        }
        __syncthreads();
        // v = r + E w, kept in the lane's global buffer tg (the solve vector may be in LDS)
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
            T acc = (T)r[i];
            const int t1 = erp[i + 1];
            for (int t = erp[i]; t < t1; ++t) acc = fnms(acc, -ev[t], w[eci[t]]);
            tg[i] = acc;
        }
        __syncthreads();
        wg_a0_solve<T, NT, kLds, T>(S, mlev, mrow, lrp, lci, lv, urp, uci, uv, dinv, tg, vec);
    }
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) z[i] = (double)vec[i - off];
    __syncthreads();
}

// One workgroup per lane.  Vectors are double, device order, lane column at
// col * ld: b (right-hand side), x (written), r, p, q, z (work).  T buffers tg
// (n per column, ld), y and w (interface, lds per column).  tol2 = rtol^2.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_pcg_persist(
    const PSys* __restrict__ sys, const PLane* __restrict__ lanes, const int64_t* __restrict__ arp,
    const int32_t* __restrict__ aci, const double* __restrict__ av, const int32_t* __restrict__ mlev,
    const int32_t* __restrict__ mrow, const int32_t* __restrict__ lrp, const int32_t* __restrict__ lci,
    const T* __restrict__ lv, const int32_t* __restrict__ urp, const int32_t* __restrict__ uci,
    const T* __restrict__ uv, const T* __restrict__ dinv, const int32_t* __restrict__ erp,
    const int32_t* __restrict__ eci, const T* __restrict__ ev, const int32_t* __restrict__ etrp,
    const int32_t* __restrict__ etci, const T* __restrict__ etv, const T* __restrict__ U, int ustride,
    const double* __restrict__ dcoef, const double* b, double* x, double* r, double* p, double* q, double* z, T* tg,
    T* yv, T* wv, int64_t ld, int64_t lds_s, double tol2, int maxit, PRes* __restrict__ res) {
    extern __shared__ __attribute__((aligned(16))) unsigned char persist_lds[];
    __shared__ double red[(NT / 64) * 16];
    __shared__ double coef[kPersistMaxK];
    const PLane L = lanes[blockIdx.x];
    const PSys S = sys[L.sys];
    const int64_t c = L.col;
    b += c * ld, x += c * ld, r += c * ld, p += c * ld, q += c * ld, z += c * ld, tg += c * ld;
    yv += c * lds_s, wv += c * lds_s;
    T* lvec = reinterpret_cast<T*>(persist_lds);
    const int64_t r0 = S.r0, r1 = S.r0 + S.n;
    auto apply = [&]() {
        if (S.lds)
            wg_apply<T, NT, true>(S, mlev, mrow, lrp, lci, lv, urp, uci, uv, dinv, erp, eci, ev, etrp, etci, etv, U,
                                  ustride, dcoef, r, z, tg, yv, wv, lvec, red, coef);
        else
            wg_apply<T, NT, false>(S, mlev, mrow, lrp, lci, lv, urp, uci, uv, dinv, erp, eci, ev, etrp, etci, etv, U,
                                   ustride, dcoef, r, z, tg, yv, wv, lvec, red, coef);
    };
    // x0 = 0, r0 = b
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        acc += bi * bi;
    }
    const double bb = wg_sum<NT>(acc, red);
    int its = 0;
    double rr = bb;
    if (bb > 0.0) {
        apply();
        acc = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
            p[i] = z[i];
            acc += r[i] * z[i];
        }
        double rz = wg_sum<NT>(acc, red);  // includes the barrier that publishes p
        for (its = 1; its <= maxit; ++its) {
            acc = 0.0;
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
                double s = 0.0;
                const int64_t t1 = arp[i + 1];
                for (int64_t t = arp[i]; t < t1; ++t) s += av[t] * p[aci[t]];
                q[i] = s;
                acc += p[i] * s;
            }
            const double pq = wg_sum<NT>(acc, red);
            const double alpha = rz / pq;
            acc = 0.0;
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
                x[i] += alpha * p[i];
                const double ri = r[i] - alpha * q[i];
                r[i] = ri;
                acc += ri * ri;
            }
            rr = wg_sum<NT>(acc, red);
            if (rr <= tol2 * bb || its == maxit) break;
            apply();
            acc = 0.0;
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) acc += r[i] * z[i];
            const double rzn = wg_sum<NT>(acc, red);
            const double beta = rzn / rz;
            rz = rzn;
            for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) p[i] = z[i] + beta * p[i];
            __syncthreads();
        }
        if (its > maxit) its = maxit;
    }
    // true residual ||b - A x||
    acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
        double s = 0.0;
        const int64_t t1 = arp[i + 1];
        for (int64_t t = arp[i]; t < t1; ++t) s += av[t] * x[aci[t]];
        const double d = b[i] - s;
        acc += d * d;
    }
    const double rt = wg_sum<NT>(acc, red);
    if (threadIdx.x == 0) {
        PRes o;
        o.its = its;
        o.status = (bb == 0.0 || rr <= tol2 * bb) ? 0 : 1;
        o.rr = rr;
        o.bb = bb;
        o.rtrue = rt;
        res[blockIdx.x] = o;
    }
}

}  // namespace ddlr
