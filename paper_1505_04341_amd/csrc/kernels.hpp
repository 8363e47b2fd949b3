// HIP kernels of the DDLR hot path for gfx950 (CDNA4, wave64).
//
// Vectors are column-major (one column per right-hand side, leading dimension
// ld) in "device order": interior unknowns block by block, then the interface
// block, and inside every block the rows of each level of its triangular
// schedule stored contiguously.  Kernels are templated on the preconditioner's
// arithmetic type T (double for the FP64 path, float for the mixed path); the
// Krylov vectors and reductions are always double.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace ddlr {

constexpr int kMaxRhs = 16;      // right-hand sides per launch for register-blocked kernels
constexpr int kRedBlocks = 1024; // fixed grid of the two-stage reductions (deterministic order)
constexpr int kSell = 64;        // SELL slice height = wavefront size

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of 256 threads; result valid in thread 0. Fixed tree order.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

template <typename T> __device__ __forceinline__ T ld(const T* p) { return *p; }

// --------------------------------------------------------- permutation / casts

// y[d + r*ldy] = x[perm[d] + r*ldx]   (user order -> device order)
template <typename TI, typename TO>
__global__ void k_gather(int64_t n, int nrhs, const int32_t* __restrict__ perm, const TI* __restrict__ x, int64_t ldx,
                         TO* __restrict__ y, int64_t ldy) {
    const int64_t total = n * nrhs;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = g / n, d = g - r * n;
        y[d + r * ldy] = (TO)x[perm[d] + r * ldx];
    }
}

// y[perm[d] + r*ldy] = x[d + r*ldx]   (device order -> user order)
template <typename TI, typename TO>
__global__ void k_scatter(int64_t n, int nrhs, const int32_t* __restrict__ perm, const TI* __restrict__ x, int64_t ldx,
                          TO* __restrict__ y, int64_t ldy) {
    const int64_t total = n * nrhs;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = g / n, d = g - r * n;
        y[perm[d] + r * ldy] = (TO)x[d + r * ldx];
    }
}

template <typename TI, typename TO>
__global__ void k_cast(int64_t n, int nrhs, const TI* __restrict__ x, int64_t ldx, TO* __restrict__ y, int64_t ldy,
                       const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t total = n * nrhs;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = g / n, d = g - r * n;
        y[d + r * ldy] = (TO)x[d + r * ldx];
    }
}

// ------------------------------------------------ A0 solve: narrow blocks
//
// One workgroup per (block, right-hand side).  The block's levels are walked
// forward (unit lower L, y = x - L y) and then backward (z = D^{-1} y - L^T z),
// with a workgroup barrier between levels; rows of one level are independent
// and stored contiguously, so each level is a coalesced sweep.  Workgroup ids
// are laid out so that every right-hand side of a block lands on the same XCD
// (ids are dispatched round-robin over the 8 XCDs) and shares its L2 copy of
// the factor.
struct BlockDesc {
    int32_t lvl0, lvl1;  // levels [lvl0, lvl1) in lvl_ptr
};

template <typename T>
__global__ __launch_bounds__(256) void k_trsv_narrow(
    const BlockDesc* __restrict__ blk, int nblk, int nblk_pad, int nrhs, const int32_t* __restrict__ lvl_ptr,
    const int32_t* __restrict__ lrp, const int32_t* __restrict__ lci, const T* __restrict__ lv,
    const int32_t* __restrict__ urp, const int32_t* __restrict__ uci, const T* __restrict__ uv,
    const T* __restrict__ dinv, const T* x, int64_t ldx, T* z, int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int b = blockIdx.x % nblk_pad, r = blockIdx.x / nblk_pad;
    if (b >= nblk || r >= nrhs) return;
    const BlockDesc d = blk[b];
    const T* xr = x + r * ldx;
    T* zr = z + r * ldz;
    for (int l = d.lvl0; l < d.lvl1; ++l) {
        const int a = lvl_ptr[l], e = lvl_ptr[l + 1];
        for (int i = a + threadIdx.x; i < e; i += blockDim.x) {
            T s = xr[i];
            const int t1 = lrp[i + 1];
            for (int t = lrp[i]; t < t1; ++t) s -= lv[t] * zr[lci[t]];
            zr[i] = s;
        }
        __syncthreads();
    }
    for (int l = d.lvl1 - 1; l >= d.lvl0; --l) {
        const int a = lvl_ptr[l], e = lvl_ptr[l + 1];
        for (int i = a + threadIdx.x; i < e; i += blockDim.x) {
            T s = zr[i] * dinv[i];
            const int t1 = urp[i + 1];
            for (int t = urp[i]; t < t1; ++t) s -= uv[t] * zr[uci[t]];
            zr[i] = s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------ A0 solve: one wide level
//
// For the interface block C_alpha in multicolour order the schedule has a few
// very wide levels; each level is one grid-wide launch over rows x rhs.
// forward:  z_i = x_i - sum L_ij z_j ;  backward: z_i = D_i^{-1} z_i - sum L_ji z_j
template <typename T, bool kBackward>
__global__ __launch_bounds__(256) void k_trsv_level(int a, int e, int nrhs, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                    const T* __restrict__ dinv, const T* x, int64_t ldx, T* z,
                                                    int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int rows = e - a;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= (int64_t)rows * nrhs) return;
    const int r = (int)(g / rows), i = a + (int)(g - (int64_t)r * rows);
    T* zr = z + r * ldz;
    T s = kBackward ? zr[i] * dinv[i] : x[i + r * ldx];
    const int t1 = rp[i + 1];
    for (int t = rp[i]; t < t1; ++t) s -= v[t] * zr[ci[t]];
    zr[i] = s;
}

// ------------------------------------------------------------ SpMV (SELL-64)
//
// y = A x for up to kMaxRhs columns; A is FP64 in SELL-64 (slices of 64 rows,
// entries column-major inside a slice, padding points at the row itself with
// value 0).  Optionally accumulates per-block partial dot products x.y per
// right-hand side into part[block*nrhs + r] (used for p^T A p in CG).
__global__ __launch_bounds__(256) void k_spmv_sell(int64_t n, int nrhs, const int32_t* __restrict__ sptr,
                                                   const int32_t* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                                                   int64_t ldy, double* __restrict__ part,
                                                   const int* __restrict__ done) {
    __shared__ double sh[4 * kMaxRhs];
    if (done && *done) return;
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double acc[kMaxRhs];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r) acc[r] = 0.0;
    if (row < n) {
        const int64_t sl = row >> 6;
        const int lane = (int)(row & 63);
        const int base = sptr[sl], width = (sptr[sl + 1] - base) >> 6;
        for (int j = 0; j < width; ++j) {
            const int q = base + j * kSell + lane;
            const int c = col[q];
            const double a = val[q];
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r)
                if (r < nrhs) acc[r] += a * x[c + r * ldx];
        }
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r)
            if (r < nrhs) y[row + r * ldy] = acc[r];
    }
    if (part) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int r = 0; r < nrhs; ++r) {
            double v = row < n ? acc[r] * x[row + r * ldx] : 0.0;
            v = wave_sum(v);
            if (lane == 0) sh[w * kMaxRhs + r] = v;
        }
        __syncthreads();
        if (threadIdx.x < nrhs) {
            const int r = threadIdx.x;
            part[blockIdx.x * nrhs + r] =
                (sh[0 * kMaxRhs + r] + sh[1 * kMaxRhs + r]) + (sh[2 * kMaxRhs + r] + sh[3 * kMaxRhs + r]);
        }
    }
}

// ------------------------------------------------------- E and E^T products
//
// E (n x s) and E^T (s x n) as CSR in device order (E carries alpha^{-1} Ehat on
// interior rows and -alpha on the interface diagonal, eq. EF).
//   k_csr_mv:  y = M w            (E^T z, or E q for Lanczos)
//   k_csr_add: t = x + M w        (step 4 of the DDLR-1 algorithm fused with x + v)
template <typename T>
__global__ __launch_bounds__(256) void k_csr_mv(int64_t rows, int nrhs, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                const T* __restrict__ w, int64_t ldw, const T* __restrict__ x,
                                                int64_t ldx, T* __restrict__ y, int64_t ldy,
                                                const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t total = rows * nrhs;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = g / rows, i = g - r * rows;
        T s = x ? x[i + r * ldx] : T(0);
        const T* wr = w + r * ldw;
        for (int t = rp[i]; t < rp[i + 1]; ++t) s += v[t] * wr[ci[t]];
        y[i + r * ldy] = s;
    }
}

// ------------------------------------------------------- low-rank correction
//
// DDLR-1 (eq. gkt):  w = c0 y + U_k (d .* (U_k^T y)),   U_k: s x k
// DDLR-2 (eq. Form2a): u = u + U_k (H_k (U_k^T x)),    U_k: n x k
// U_k is row-major (k contiguous per row).  Stage 1 accumulates per-block
// partials of U_k^T y (k x nrhs); stage 2 sums them in fixed order and applies
// d (DDLR-1) or H_k (DDLR-2); stage 3 expands.
template <typename T>
__global__ __launch_bounds__(256) void k_lr_reduce(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                   const T* __restrict__ y, int64_t ldy, double* __restrict__ part,
                                                   const int* __restrict__ done) {
    // part layout: [block][r][j]; lane <-> column j, waves and blocks stride the rows
    __shared__ double sh[4][64];
    if (done && *done) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + lane;
        double acc[kMaxRhs];
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r) acc[r] = 0.0;
        for (int64_t i = blockIdx.x * 4 + w; i < rows; i += (int64_t)gridDim.x * 4) {
            const double u = j < k ? (double)U[i * k + j] : 0.0;
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r)
                if (r < nrhs) acc[r] += u * (double)y[i + r * ldy];
        }
        for (int r = 0; r < nrhs; ++r) {
            sh[w][lane] = acc[r];
            __syncthreads();
            if (w == 0 && j < k)
                part[((int64_t)blockIdx.x * nrhs + r) * k + j] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
            __syncthreads();
        }
    }
}

// coef[r][j] = mode 1: dvec[j] c[r][j] ; mode 2: (H c[r])[j]   (c already reduced)
__global__ void k_lr_coef(int k, int nrhs, const double* __restrict__ c, int mode, const double* __restrict__ dvec,
                          const double* __restrict__ H, double* __restrict__ coef, const int* __restrict__ done) {
    if (done && *done) return;
    for (int q = threadIdx.x; q < nrhs * k; q += blockDim.x) {
        const int r = q / k, j = q - r * k;
        double v;
        if (mode == 1) {
            v = dvec[j] * c[q];
        } else {
            v = 0.0;
            for (int t = 0; t < k; ++t) v += H[j + t * k] * c[r * k + t];
        }
        coef[q] = v;
    }
}

// out[col] = sum over parts of part[b*ncols + col], one workgroup per column, fixed order
__global__ __launch_bounds__(256) void k_reduce_cols(int nparts, int ncols, const double* __restrict__ part,
                                                     double* __restrict__ out, const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    const int col = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) acc += part[(int64_t)b * ncols + col];
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) out[col] = s;
}

// out[i] = beta * in[i] + sum_j U[i][j] coef[r][j]
template <typename T>
__global__ __launch_bounds__(256) void k_lr_expand(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                   const double* __restrict__ coef, double beta, const T* in,
                                                   int64_t ldin, T* out, int64_t ldout, const int* __restrict__ done) {
    __shared__ double cf[kMaxRhs * 128];
    if (done && *done) return;
    for (int q = threadIdx.x; q < nrhs * k; q += blockDim.x) cf[q] = coef[q];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        const T* ui = U + i * k;
        double acc[kMaxRhs];
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r) acc[r] = r < nrhs ? beta * (double)in[i + r * ldin] : 0.0;
        for (int j = 0; j < k; ++j) {
            const double u = (double)ui[j];
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r)
                if (r < nrhs) acc[r] += u * cf[r * k + j];
        }
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r)
            if (r < nrhs) out[i + r * ldout] = (T)acc[r];
    }
}

// --------------------------------------------------------- dots and CG steps

// part[block*nrhs + r] = sum over the block's rows of a_r . b_r
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_dot(int64_t n, int nrhs, const TA* __restrict__ a, int64_t lda,
                                             const TB* __restrict__ b, int64_t ldb, double* __restrict__ part,
                                             const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    for (int r = 0; r < nrhs; ++r) {
        double acc = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            acc += (double)a[i + r * lda] * (double)b[i + r * ldb];
        const double s = block_sum256(acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x * nrhs + r] = s;
    }
}

// Per right-hand-side state of the CG iteration (device resident).
struct CgLane {
    double bb, rz, rr, alpha, beta;
    int32_t active, its;
};

// what: 0 = init (bb, rr from ||b||^2), 1 = first rz, 2 = alpha = rz / p^T q,
//       3 = residual check after the x, r update, 4 = beta from the new rz
// sums[r] holds the reduced dot product of right-hand side r.
__global__ void k_cg_scalar(int what, int nrhs, const double* __restrict__ sums, CgLane* __restrict__ L, double tol2,
                            int maxit, int* __restrict__ done) {
    if (what != 0 && done && *done) return;
    const int r = threadIdx.x;
    if (r < nrhs) {
        const double s = sums[r];
        CgLane& l = L[r];
        switch (what) {
        case 0: l.bb = s; l.rr = s; l.its = 0; l.active = s > 0.0; l.rz = 0; l.alpha = 0; l.beta = 0; break;
        case 1: l.rz = s; break;
        case 2: l.alpha = l.active ? l.rz / s : 0.0; break;
        case 3:
            if (l.active) {
                l.rr = s;
                l.its += 1;
                if (s <= tol2 * l.bb || l.its >= maxit) l.active = 0;
            }
            break;
        case 4:
            if (l.active) {
                l.beta = s / l.rz;
                l.rz = s;
            }
            break;
        }
    }
    if (what == 0 || what == 3) {
        __syncthreads();
        if (threadIdx.x == 0 && done) {
            int any = 0;
            for (int q = 0; q < nrhs; ++q) any |= L[q].active;
            *done = any ? 0 : 1;
        }
    }
}

// x += alpha p ; r -= alpha q ; part = r.r   (active lanes only)
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int nrhs, const CgLane* __restrict__ L,
                                               const double* __restrict__ p, const double* __restrict__ q,
                                               double* __restrict__ x, double* __restrict__ r, int64_t ld,
                                               double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    for (int c = 0; c < nrhs; ++c) {
        const bool act = L[c].active;
        const double a = L[c].alpha;
        double acc = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t o = i + c * ld;
            double ri = r[o];
            if (act) {
                x[o] += a * p[o];
                ri -= a * q[o];
                r[o] = ri;
            }
            acc += ri * ri;
        }
        const double s = block_sum256(acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x * nrhs + c] = s;
    }
}

// p = z + beta p (active lanes); init: p = z
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, int nrhs, const CgLane* __restrict__ L, int init,
                                              const double* __restrict__ z, double* __restrict__ p, int64_t ld,
                                              const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t total = n * nrhs;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = g / n, i = g - c * n;
        if (init) {
            p[i + c * ld] = z[i + c * ld];
        } else if (L[c].active) {
            p[i + c * ld] = z[i + c * ld] + L[c].beta * p[i + c * ld];
        }
    }
}

// ------------------------------------------------------------ Lanczos steps
//
// Q holds the Lanczos vectors as columns (s x (m+1), column-major, ld s).
// coeffs: c_l = q_l . w for l <= j, as per-block partials part[block][l]
__global__ __launch_bounds__(256) void k_multidot(int64_t s, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                  const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sh[4];
    for (int l = 0; l < ncols; ++l) {
        double acc = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s; i += (int64_t)gridDim.x * blockDim.x)
            acc += Q[i + l * ldq] * w[i];
        const double t = block_sum256(acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x * ncols + l] = t;
    }
}

// w -= Q c  (columns 0..ncols-1)
__global__ __launch_bounds__(256) void k_gemv_sub(int64_t s, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                  const double* __restrict__ c, double* __restrict__ w) {
    __shared__ double cs[1024];
    for (int l = threadIdx.x; l < ncols; l += blockDim.x) cs[l] = c[l];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s; i += (int64_t)gridDim.x * blockDim.x) {
        double v = w[i];
        for (int l = 0; l < ncols; ++l) v -= Q[i + l * ldq] * cs[l];
        w[i] = v;
    }
}

// scalars: alpha[j] = sum(part); w -= alpha_j q_j + beta_{j-1} q_{j-1}
__global__ __launch_bounds__(256) void k_lanczos_3term(int64_t s, int j, const double* __restrict__ Q, int64_t ldq,
                                                       const double* __restrict__ alpha,
                                                       const double* __restrict__ beta, double* __restrict__ w) {
    const double a = alpha[j], bprev = j > 0 ? beta[j - 1] : 0.0;
    const double* qj = Q + j * ldq;
    const double* qp = j > 0 ? Q + (j - 1) * ldq : nullptr;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s; i += (int64_t)gridDim.x * blockDim.x) {
        double v = w[i] - a * qj[i];
        if (qp) v -= bprev * qp[i];
        w[i] = v;
    }
}

// dst = reduced sum; beta form: dst = sqrt(sum), inv = dst > 1e-12 max|alpha| ? 1/dst : 0
__global__ void k_lanczos_scalar(const double* __restrict__ sum, double* __restrict__ dst, int sqrt_it,
                                 double* __restrict__ amax, double* __restrict__ inv) {
    if (threadIdx.x == 0) {
        double s = *sum;
        if (sqrt_it) {
            s = sqrt(s);
            *dst = s;
            *inv = (s > 1e-12 * (*amax)) ? 1.0 / s : 0.0;
        } else {
            *dst = s;
            if (fabs(s) > *amax) *amax = fabs(s);
        }
    }
}

// q_{j+1} = w * inv
__global__ __launch_bounds__(256) void k_scale_to(int64_t s, const double* __restrict__ w,
                                                  const double* __restrict__ inv, double* __restrict__ q) {
    const double f = *inv;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s; i += (int64_t)gridDim.x * blockDim.x)
        q[i] = w[i] * f;
}

// Out (rows x k, row-major, type TO) = Q (rows x m, column-major) * Y (m x k, column-major)
template <typename TO>
__global__ __launch_bounds__(256) void k_qy(int64_t rows, int m, int k, const double* __restrict__ Q, int64_t ldq,
                                            const double* __restrict__ Y, TO* __restrict__ out, int out_colmajor,
                                            int64_t ldo) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int l = 0; l < m; ++l) s += Q[i + l * ldq] * Y[l + (int64_t)j * m];
            if (out_colmajor) out[i + j * ldo] = (TO)s;
            else out[i * k + j] = (TO)s;
        }
    }
}

// Gram block: part[block][i*k+j] = sum over the block's rows of A[:,i] . B[:,j]
// (A, B column-major rows x k).  Used once for K = U_k^T (E V_k) of DDLR-2.
__global__ __launch_bounds__(256) void k_gram(int64_t rows, int k, const double* __restrict__ A, int64_t lda,
                                              const double* __restrict__ B, int64_t ldb, double* __restrict__ part) {
    const int pairs = k * k;
    for (int q = threadIdx.x; q < pairs; q += blockDim.x) {
        const int i = q / k, j = q - i * k;
        double acc = 0.0;
        for (int64_t t = blockIdx.x; t < rows; t += gridDim.x) acc += A[t + i * lda] * B[t + j * ldb];
        part[(int64_t)blockIdx.x * pairs + q] = acc;
    }
}

// transpose-convert: out (rows x k row-major, TO) from in (rows x k column-major, double)
template <typename TO>
__global__ void k_to_rowmajor(int64_t rows, int k, const double* __restrict__ in, int64_t ldi, TO* __restrict__ out) {
    const int64_t total = rows * k;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / k;
        const int j = (int)(g - i * k);
        out[g] = (TO)in[i + j * ldi];
    }
}

// out = a - b (flat)
__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - b[i];
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

}  // namespace ddlr
