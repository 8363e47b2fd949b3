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

// s - a b with one rounding.  Every triangular-solve kernel forms its row sums
// with this, so kernels of different shape give bitwise the same results
// whatever the compiler would contract on its own.
__device__ __forceinline__ float fnms(float s, float a, float b) { return __builtin_fmaf(-a, b, s); }
__device__ __forceinline__ double fnms(double s, double a, double b) { return __builtin_fma(-a, b, s); }

// --------------------------------------------------------- permutation / casts

// y[d + r*ldy] = x[perm[d] + r*ldx]   (user order -> device order)
template <typename TI, typename TO>
__global__ void k_gather(int64_t n, int nrhs, const int32_t* __restrict__ perm, const TI* __restrict__ x, int64_t ldx,
                         TO* __restrict__ y, int64_t ldy) {
    const int64_t r = blockIdx.y;  // grid (chunks, nrhs)
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x)
        y[d + r * ldy] = (TO)x[perm[d] + r * ldx];
}

// y[perm[d] + r*ldy] = x[d + r*ldx]   (device order -> user order)
template <typename TI, typename TO>
__global__ void k_scatter(int64_t n, int nrhs, const int32_t* __restrict__ perm, const TI* __restrict__ x, int64_t ldx,
                          TO* __restrict__ y, int64_t ldy) {
    const int64_t r = blockIdx.y;  // grid (chunks, nrhs)
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x)
        y[perm[d] + r * ldy] = (TO)x[d + r * ldx];
}

template <typename TI, typename TO>
__global__ void k_cast(int64_t n, int nrhs, const TI* __restrict__ x, int64_t ldx, TO* __restrict__ y, int64_t ldy,
                       const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t r = blockIdx.y;  // grid (chunks, nrhs)
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x)
        y[d + r * ldy] = (TO)x[d + r * ldx];
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

// Entries per group in the row loops of the plain level kernels: a group's
// column, value and gather loads go out together.
constexpr int kTermGroup = 8;

// s - sum_t v[t] y[c[t]] over t in [t0, t1), the terms applied in order of t,
// the entries in groups of kTermGroup; an index past the row's end repeats
// its last entry and is not applied.
template <typename T, typename TY>
__device__ __forceinline__ T row_terms(T s, int t0, int t1, const int32_t* __restrict__ col,
                                       const T* __restrict__ val, const TY* y) {
    for (int t = t0; t < t1; t += kTermGroup) {
        int c[kTermGroup];
        T v[kTermGroup], g[kTermGroup];
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u) {
            const int q = min(t + u, t1 - 1);
            c[u] = col[q];
            v[u] = val[q];
        }
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u) g[u] = (T)y[c[u]];
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u)
            if (t + u < t1) s = fnms(s, v[u], g[u]);
    }
    return s;
}

template <typename T, typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_trsv_narrow(
    const BlockDesc* __restrict__ blk, int nblk, int nblk_pad, int nrhs, const int32_t* __restrict__ lvl_ptr,
    const int32_t* __restrict__ lrp, const int32_t* __restrict__ lci, const T* __restrict__ lv,
    const int32_t* __restrict__ urp, const int32_t* __restrict__ uci, const T* __restrict__ uv,
    const T* __restrict__ dinv, const TIn* x, int64_t ldx, TOut* z, int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int b = blockIdx.x % nblk_pad, r = blockIdx.x / nblk_pad;
    if (b >= nblk || r >= nrhs) return;
    const BlockDesc d = blk[b];
    const TIn* xr = x + r * ldx;
    TOut* zr = z + r * ldz;
    for (int l = d.lvl0; l < d.lvl1; ++l) {
        const int a = lvl_ptr[l], e = lvl_ptr[l + 1];
        for (int i = a + threadIdx.x; i < e; i += blockDim.x) {
            T s = (T)xr[i];
            s = row_terms<T>(s, lrp[i], lrp[i + 1], lci, lv, zr);
            zr[i] = (TOut)s;
        }
        __syncthreads();
    }
    for (int l = d.lvl1 - 1; l >= d.lvl0; --l) {
        const int a = lvl_ptr[l], e = lvl_ptr[l + 1];
        for (int i = a + threadIdx.x; i < e; i += blockDim.x) {
            T s = (T)zr[i] * dinv[i];
            s = row_terms<T>(s, urp[i], urp[i + 1], uci, uv, zr);
            zr[i] = (TOut)s;
        }
        __syncthreads();
    }
}

// ------------------------------------- A0 solve: narrow blocks, LDS ring
//
// Same schedule as k_trsv_narrow, restructured for latency:
//  * each row's dependencies are stored per level in ELL form (entries
//    column-major, column = row index local to the block; padding has column
//    0 and value 0), so one level's data is one coalesced segment; kernels of
//    width KW <= 4 see every level padded to KW, wider ones see each level
//    padded to its own widest row rounded up to a multiple of 4 (meta.w:
//    forward width in the low 16 bits, backward width in the high 16), so
//    irregular rows do not make every level as wide as the widest row;
//  * the next kD-1 levels' entries, right-hand side values and D^{-1} are
//    loaded into registers ahead of use, so HBM latency overlaps computation
//    and barriers; the steady-state loop has no divergent branches, which
//    lets the compiler wait only for the level being computed;
//  * lanes beyond a level's last row load and recompute that last row (all
//    loads are unconditional) but only the owning lane stores it;
//  * results go to global memory and to a ring of the most recent rmask + 1
//    rows in LDS (a power of two chosen at launch); the host has checked that
//    every dependency of every level lies inside that window (forward:
//    c >= e - ring; backward: c < a + ring), so all gathers hit LDS and levels
//    are separated by LDS-only barriers.
// NT threads with NS rows each per level in registers; rows beyond NS * NT
// finish without prefetch.
struct RingBlock {
    int32_t lvl0, lvl1, row0, pad;
};

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kRingThreads = 512;
constexpr int kRingMaxLevels = 511;

// Registers of one prefetched level: NS row sets of NT rows.  The right-hand-
// side value is kept in its storage type TS and converted when used, so no
// load is waited for early.
template <typename T, int KW, typename TS, int NS> struct LevelRegs {
    int a, e, off, w;
    int c[NS][KW];
    T v[NS][KW];
    TS xv[NS];
    T dv[NS];
};

// Separation of consecutive levels: an LDS-only barrier for several waves; a
// single wave needs none (its LDS operations execute in order), only a
// compiler fence so no access moves across the level boundary.
template <int NT> __device__ __forceinline__ void level_sync() {
    if constexpr (NT > 64) lds_barrier();
    else __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Per-level metadata of one block, staged in LDS at kernel start: local first
// row and the ELL offsets of L and L^T.
template <typename T, int KW, bool kBwd, typename TS, int NT, int NS>
__device__ __forceinline__ void ring_load(LevelRegs<T, KW, TS, NS>& R, int q, int row0, const int4* meta,
                                          const int32_t* __restrict__ ecol, const T* __restrict__ eval,
                                          const T* __restrict__ dinv, const TS* src) {
    const int4 mq = meta[q];  // uniform across the workgroup: keep it in scalar registers
    R.a = __builtin_amdgcn_readfirstlane(mq.x);
    R.e = __builtin_amdgcn_readfirstlane(meta[q + 1].x);
    R.off = __builtin_amdgcn_readfirstlane(kBwd ? mq.z : mq.y);
    R.w = KW > 4 ? __builtin_amdgcn_readfirstlane(kBwd ? (mq.w >> 16) : (mq.w & 0xffff)) : KW;
    const int nr = R.e - R.a;
#pragma unroll
    for (int qq = 0; qq < NS; ++qq) {
        if (qq >= 1 && nr <= qq * NT) break;  // uniform: fewer row sets cover the level
        const int i = min(R.a + (int)threadIdx.x + qq * NT, R.e - 1);
        const int base = R.off + (i - R.a);
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            if (KW > 4 && j % 4 == 0 && j >= R.w) break;  // uniform: the level's width
            R.c[qq][j] = ecol[base + j * nr];
            R.v[qq][j] = eval[base + j * nr];
        }
        R.xv[qq] = src[i];
        if (kBwd) R.dv[qq] = dinv[row0 + i];
    }
}

template <typename T, int KW, bool kBwd, typename TS, typename TD, int NT, int NS>
__device__ __forceinline__ void ring_compute(const LevelRegs<T, KW, TS, NS>& R, int row0, T* ring, int rmask,
                                             const int32_t* __restrict__ ecol, const T* __restrict__ eval,
                                             const T* __restrict__ dinv, const TS* src, TD* dst) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        if (q >= 1 && R.e - R.a <= q * NT) break;
        const int i0 = R.a + (int)threadIdx.x + q * NT;
        const int i = min(i0, R.e - 1);
        T s = kBwd ? (T)R.xv[q] * R.dv[q] : (T)R.xv[q];
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            if (KW > 4 && j % 4 == 0 && j >= R.w) break;
            s = fnms(s, R.v[q][j], ring[R.c[q][j] & rmask]);
        }
        // only the owning lane stores: duplicate global stores of a forward value
        // from other waves are not ordered against the owner's backward store
        if (i0 < R.e) {
            ring[i & rmask] = s;
            dst[i] = (TD)s;
        }
    }
    // rows beyond NS * NT: no prefetch
    const int nr = R.e - R.a;
    for (int i = R.a + NS * NT + (int)threadIdx.x; i < R.e; i += NT) {
        const int base = R.off + (i - R.a);
        T s = kBwd ? (T)src[i] * dinv[row0 + i] : (T)src[i];
        for (int j = 0; j < R.w; ++j) s = fnms(s, eval[base + j * nr], ring[ecol[base + j * nr] & rmask]);
        ring[i & rmask] = s;
        dst[i] = (TD)s;
    }
}

// Prefetch depth (levels in flight) that keeps the register budget under 128
// VGPRs, so two 512-thread workgroups fit on a CU.
template <typename T, int KW> struct RingDepth { static constexpr int value = 2; };
template <> struct RingDepth<float, 2> { static constexpr int value = 4; };
template <> struct RingDepth<float, 3> { static constexpr int value = 4; };
template <> struct RingDepth<float, 4> { static constexpr int value = 3; };
template <> struct RingDepth<double, 2> { static constexpr int value = 3; };
template <> struct RingDepth<double, 3> { static constexpr int value = 3; };

// Row sets per thread: two up to width 16, one at width 32 (registers).
template <int KW> constexpr int ring_sets() { return KW <= 16 ? 2 : 1; }

// One sweep over local levels; kBwd walks them from the last to the first.
template <typename T, int KW, bool kBwd, typename TS, typename TD, int NT, int NS>
__device__ __forceinline__ void ring_sweep(int nlev, int row0, const int4* meta, T* ring, int rmask,
                                           const int32_t* __restrict__ ecol, const T* __restrict__ eval,
                                           const T* __restrict__ dinv, const TS* src, TD* dst) {
    constexpr int kD = RingDepth<T, KW>::value;
    LevelRegs<T, KW, TS, NS> buf[kD];
    auto lev = [&](int q) { return kBwd ? nlev - 1 - q : q; };
    int q0 = 0;
    if (nlev >= 2 * kD - 1) {
        // The steady state sits on its own path behind an unconditional
        // prologue: the compiler's load-counter waits then see every prefetch
        // of the kD - 1 levels ahead on each path into the loop, and wait for
        // the one level being computed, not for all but the newest loads.
#pragma unroll
        for (int u = 0; u < kD - 1; ++u)
            ring_load<T, KW, kBwd, TS, NT, NS>(buf[u], lev(u), row0, meta, ecol, eval, dinv, src);
        // every prefetch in the group is a real level
        for (; q0 + 2 * kD - 1 <= nlev; q0 += kD) {
#pragma unroll
            for (int u = 0; u < kD; ++u) {
                ring_load<T, KW, kBwd, TS, NT, NS>(buf[(u + kD - 1) % kD], lev(q0 + u + kD - 1), row0, meta, ecol,
                                                   eval, dinv, src);
                ring_compute<T, KW, kBwd, TS, TD, NT, NS>(buf[u], row0, ring, rmask, ecol, eval, dinv, src, dst);
                level_sync<NT>();
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < kD - 1; ++u)
            if (u < nlev) ring_load<T, KW, kBwd, TS, NT, NS>(buf[u], lev(u), row0, meta, ecol, eval, dinv, src);
    }
    // tail
    for (; q0 < nlev; q0 += kD) {
#pragma unroll
        for (int u = 0; u < kD; ++u) {
            const int q = q0 + u;
            if (q < nlev) {
                if (q + kD - 1 < nlev)
                    ring_load<T, KW, kBwd, TS, NT, NS>(buf[(u + kD - 1) % kD], lev(q + kD - 1), row0, meta, ecol,
                                                       eval, dinv, src);
                ring_compute<T, KW, kBwd, TS, TD, NT, NS>(buf[u], row0, ring, rmask, ecol, eval, dinv, src, dst);
                level_sync<NT>();
            }
        }
    }
}

// One workgroup of NT threads per (block, column); NT = 512 for wide levels,
// 64 (one wave, no barriers) or 256 for thin ones.  The ring is dynamic LDS of
// rmask + 1 rows (a power of two).
template <typename T, int KW, typename TIn, typename TOut, int NT>
__global__ __launch_bounds__(NT) void k_trsv_ring(
    const RingBlock* __restrict__ blk, int nblk, int nblk_pad, int nrhs, const int32_t* __restrict__ lvl_ptr,
    const int32_t* __restrict__ foff, const int32_t* __restrict__ fcol, const T* __restrict__ fval,
    const int32_t* __restrict__ boff, const int32_t* __restrict__ bcol, const T* __restrict__ bval,
    const int32_t* __restrict__ lwid, int rmask, const T* __restrict__ dinv, const TIn* x, int64_t ldx, TOut* z,
    int64_t ldz, const int* __restrict__ done) {
    constexpr int NS = ring_sets<KW>();
    extern __shared__ __attribute__((aligned(16))) char ring_lds[];
    T* ring = reinterpret_cast<T*>(ring_lds);
    __shared__ int4 meta[kRingMaxLevels + 1];
    if (done && *done) return;
    const int b = blockIdx.x % nblk_pad, r = blockIdx.x / nblk_pad;
    if (b >= nblk || r >= nrhs) return;
    const RingBlock d = blk[b];
    const int nlev = d.lvl1 - d.lvl0;  // <= kRingMaxLevels (checked on the host)
    if (nlev <= 0) return;
    for (int q = threadIdx.x; q <= nlev; q += NT) {
        const int l = d.lvl0 + q;
        meta[q] = q < nlev ? int4{lvl_ptr[l] - d.row0, foff[l], boff[l], lwid[l]} : int4{lvl_ptr[l] - d.row0, 0, 0, 0};
    }
    for (int q = threadIdx.x; q <= rmask; q += NT) ring[q] = T(0);
    __syncthreads();
    const TIn* xr = x + r * ldx + d.row0;
    TOut* zr = z + r * ldz + d.row0;
    // forward sweep: y = x - L y
    ring_sweep<T, KW, false, TIn, TOut, NT, NS>(nlev, d.row0, meta, ring, rmask, fcol, fval, dinv, xr, zr);
    __syncthreads();  // global fence: the backward sweep reads y_i from memory
    // backward sweep: z = D^{-1} y - L^T z
    ring_sweep<T, KW, true, TOut, TOut, NT, NS>(nlev, d.row0, meta, ring, rmask, bcol, bval, dinv, zr, zr);
}

// ----------------------------- A0 solve: narrow blocks, R columns per workgroup
//
// The ring kernel above runs one workgroup per (block, column), so every
// column's workgroup loads the block's level entries of L and L^T again.
// This variant gives a workgroup R columns of one block: the entries are
// loaded once and used R times, and the LDS ring keeps the R values of a row
// side by side, so one vector LDS read gathers a dependency for all R
// columns.  Per column the arithmetic is that of the one-column kernel (same
// operations in the same order), so the results are bitwise the same for any
// R.  The ring holds kRing rows of R values (64 KB); the host checks the
// dependency window against kRing as for the one-column kernel.
//
// The kernel is bound by vector-memory instructions per level, so each row's
// factor data is one packed record read with as few wide loads as possible,
// and the forward result y goes to a private buffer with the R values of a
// row side by side (one store, one load) instead of R column stores and loads.
template <typename T, int R> constexpr int ring_rows_r() { return 65536 / (int)(sizeof(T) * R); }

// Packed record of one row (at most KW <= 4 entries) in 32-bit words: the KW
// values of T; in the backward sweep D_i^{-1} as T; then the KW block-local
// columns modulo 65536 as 16-bit halves (entry j in word kColW + j/2, high
// half for odd j; the ring index only needs the column modulo the ring size, a
// power of two that divides 65536).  A level's records are stored chunk by
// chunk for coalescing: kN4 arrays of four-word chunks, then one array of the
// kRem remaining words (1, 2, or 4 when three remain).  Level offsets are
// multiples of four words.  Padding entries have column 0 and value 0.
template <typename T, int KW, bool kBwd> struct RecLayout {
    static constexpr int kTW = (int)(sizeof(T) / 4);
    static constexpr int kDiag = KW * kTW;
    static constexpr int kColW = kDiag + (kBwd ? kTW : 0);
    static constexpr int kWords = kColW + (KW + 1) / 2;
    static constexpr int kN4 = kWords / 4;
    static constexpr int kRem = kWords % 4 == 3 ? 4 : kWords % 4;
    static constexpr int kPadded = kN4 * 4 + kRem;
};

template <typename T> __device__ __forceinline__ T rec_value(const uint32_t* w, int word) {
    if constexpr (sizeof(T) == 4) return __uint_as_float(w[word]);
    else return __hiloint2double((int)w[word + 1], (int)w[word]);
}

// words of record r (0-based row of the level) of a level with nr rows at word offset off
template <typename T, int KW, bool kBwd>
__device__ __forceinline__ void rec_load(const int32_t* __restrict__ rec, int off, int nr, int r,
                                         uint32_t (&w)[RecLayout<T, KW, kBwd>::kPadded]) {
    using L = RecLayout<T, KW, kBwd>;
    const int4* p4 = reinterpret_cast<const int4*>(rec + off);
#pragma unroll
    for (int c = 0; c < L::kN4; ++c) {
        const int4 t = p4[c * nr + r];
        w[4 * c] = (uint32_t)t.x, w[4 * c + 1] = (uint32_t)t.y, w[4 * c + 2] = (uint32_t)t.z,
                 w[4 * c + 3] = (uint32_t)t.w;
    }
    const int32_t* tail = rec + off + 4 * L::kN4 * nr;
    if constexpr (L::kRem == 1) {
        w[4 * L::kN4] = (uint32_t)tail[r];
    } else if constexpr (L::kRem == 2) {
        const int2 t = reinterpret_cast<const int2*>(tail)[r];
        w[4 * L::kN4] = (uint32_t)t.x, w[4 * L::kN4 + 1] = (uint32_t)t.y;
    } else if constexpr (L::kRem == 4) {
        const int4 t = reinterpret_cast<const int4*>(tail)[r];
        w[4 * L::kN4] = (uint32_t)t.x, w[4 * L::kN4 + 1] = (uint32_t)t.y, w[4 * L::kN4 + 2] = (uint32_t)t.z,
                   w[4 * L::kN4 + 3] = (uint32_t)t.w;
    }
}

// Registers of one prefetched level: up to two row sets (rows a + tid and
// a + tid + kRingThreads), each a packed record and the R right-hand-side
// values in their storage type TS.
template <typename T, int KW, int R, bool kBwd, typename TS> struct LevelRegsR {
    int a, e, off;
    uint32_t w[2][RecLayout<T, KW, kBwd>::kPadded];
    TS xv[2][R];
};

// The right-hand side of row i: interleaved (kIl: R values of T side by side,
// the private forward result) or column-major with leading dimension ld.
template <int R, bool kIl, typename TS>
__device__ __forceinline__ void rhs_load(const TS* src, int64_t ld, int i, TS (&xv)[R]) {
    if constexpr (kIl) {
        using V = TS __attribute__((ext_vector_type(R)));
        const V t = *reinterpret_cast<const V*>(src + (size_t)i * R);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) xv[rr] = t[rr];
    } else {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) xv[rr] = src[i + rr * ld];
    }
}

template <typename T, int KW, int R, bool kBwd, typename TS, bool kSrcIl>
__device__ __forceinline__ void ringr_load(LevelRegsR<T, KW, R, kBwd, TS>& L, int q, const int4* meta,
                                           const int32_t* __restrict__ rec, const TS* src, int64_t lds) {
    const int4 mq = meta[q];
    L.a = __builtin_amdgcn_readfirstlane(mq.x);
    L.e = __builtin_amdgcn_readfirstlane(meta[q + 1].x);
    L.off = __builtin_amdgcn_readfirstlane(kBwd ? mq.z : mq.y);
    const int nr = L.e - L.a;
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
        if (qq == 1 && nr <= kRingThreads) break;  // uniform: one row set covers the level
        const int i = min(L.a + (int)threadIdx.x + qq * kRingThreads, L.e - 1);
        rec_load<T, KW, kBwd>(rec, L.off, nr, i - L.a, L.w[qq]);
        rhs_load<R, kSrcIl>(src, lds, i, L.xv[qq]);
    }
}

// One row: s = x_i (backward: D_i^{-1} x_i), minus its KW entries times the
// gathered ring values, in entry order; the result goes to the ring and to dst.
template <typename T, int KW, int kRing, int R, bool kBwd, typename TS, typename TD, bool kDstIl>
__device__ __forceinline__ void ringr_row(const uint32_t* w, const TS (&xv)[R], int i, bool store, T* ring, TD* dst,
                                          int64_t ldd) {
    using L = RecLayout<T, KW, kBwd>;
    using V = T __attribute__((ext_vector_type(R)));
    V sv;
    if constexpr (kBwd) {
        const T dv = rec_value<T>(w, L::kDiag);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) sv[rr] = (T)xv[rr] * dv;
    } else {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) sv[rr] = (T)xv[rr];
    }
#pragma unroll
    for (int j = 0; j < KW; ++j) {
        const int c = (int)((w[L::kColW + j / 2] >> (16 * (j & 1))) & 0xffffu);
        const T v = rec_value<T>(w, j * L::kTW);
        const V g = *reinterpret_cast<const V*>(ring + (size_t)(c & (kRing - 1)) * R);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) sv[rr] = fnms(sv[rr], v, g[rr]);
    }
    if (store) {
        *reinterpret_cast<V*>(ring + (size_t)(i & (kRing - 1)) * R) = sv;
        if constexpr (kDstIl) {
            *reinterpret_cast<V*>(dst + (size_t)i * R) = sv;
        } else {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) dst[i + rr * ldd] = (TD)sv[rr];
        }
    }
}

template <typename T, int KW, int kRing, int R, bool kBwd, typename TS, bool kSrcIl, typename TD, bool kDstIl>
__device__ __forceinline__ void ringr_compute(const LevelRegsR<T, KW, R, kBwd, TS>& L, T* ring,
                                              const int32_t* __restrict__ rec, const TS* src, int64_t lds, TD* dst,
                                              int64_t ldd) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (q == 1 && L.e - L.a <= kRingThreads) break;
        const int i0 = L.a + (int)threadIdx.x + q * kRingThreads;
        ringr_row<T, KW, kRing, R, kBwd, TS, TD, kDstIl>(L.w[q], L.xv[q], min(i0, L.e - 1), i0 < L.e, ring, dst, ldd);
    }
    // rows beyond 2 * kRingThreads: no prefetch
    const int nr = L.e - L.a;
    for (int i = L.a + 2 * kRingThreads + (int)threadIdx.x; i < L.e; i += kRingThreads) {
        uint32_t w[RecLayout<T, KW, kBwd>::kPadded];
        TS xv[R];
        rec_load<T, KW, kBwd>(rec, L.off, nr, i - L.a, w);
        rhs_load<R, kSrcIl>(src, lds, i, xv);
        ringr_row<T, KW, kRing, R, kBwd, TS, TD, kDstIl>(w, xv, i, true, ring, dst, ldd);
    }
}

// Prefetch depth (levels in flight) of the R-column kernel.  One 512-thread
// workgroup per CU leaves 256 VGPRs per lane; at R = 2 the deeper prefetch
// fits without spills and hides more of the load latency (measured on the
// 128^3 Laplacian: 5 % faster in FP32, 8 % in FP64 than depths 3 / 2), wider
// R keeps the shallower depth its registers allow.
template <typename T, int R> struct RingDepthR { static constexpr int value = R <= 2 ? 5 : 3; };
template <int R> struct RingDepthR<double, R> { static constexpr int value = R <= 2 ? 4 : 2; };

template <typename T, int KW, int kRing, int R, bool kBwd, typename TS, bool kSrcIl, typename TD, bool kDstIl>
__device__ __forceinline__ void ringr_sweep(int nlev, const int4* meta, T* ring, const int32_t* __restrict__ rec,
                                            const TS* src, int64_t lds, TD* dst, int64_t ldd) {
    constexpr int kD = RingDepthR<T, R>::value;
    LevelRegsR<T, KW, R, kBwd, TS> buf[kD];
#define DDLR_RINGR_LOAD(u, q) \
    ringr_load<T, KW, R, kBwd, TS, kSrcIl>(buf[u], kBwd ? nlev - 1 - (q) : (q), meta, rec, src, lds)
#define DDLR_RINGR_COMPUTE(u) \
    ringr_compute<T, KW, kRing, R, kBwd, TS, kSrcIl, TD, kDstIl>(buf[u], ring, rec, src, lds, dst, ldd)
    int q0 = 0;
    if (nlev >= 2 * kD - 1) {  // steady state behind an unconditional prologue, as in ring_sweep
#pragma unroll
        for (int u = 0; u < kD - 1; ++u) DDLR_RINGR_LOAD(u, u);
        for (; q0 + 2 * kD - 1 <= nlev; q0 += kD) {
#pragma unroll
            for (int u = 0; u < kD; ++u) {
                DDLR_RINGR_LOAD((u + kD - 1) % kD, q0 + u + kD - 1);
                DDLR_RINGR_COMPUTE(u);
                lds_barrier();
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < kD - 1; ++u)
            if (u < nlev) DDLR_RINGR_LOAD(u, u);
    }
    for (; q0 < nlev; q0 += kD) {
#pragma unroll
        for (int u = 0; u < kD; ++u) {
            const int q = q0 + u;
            if (q < nlev) {
                if (q + kD - 1 < nlev) DDLR_RINGR_LOAD((u + kD - 1) % kD, q + kD - 1);
                DDLR_RINGR_COMPUTE(u);
                lds_barrier();
            }
        }
    }
#undef DDLR_RINGR_LOAD
#undef DDLR_RINGR_COMPUTE
}

// grid: nblk_pad * ngroups workgroups; workgroup (b, g) solves block b for
// columns g*R .. g*R+R-1 (the host launches only ngroups = nrhs / R).  The
// forward result of the group goes to ry + g * ldry, R values per row.
template <typename T, int KW, int R, typename TIn, typename TOut>
__global__ __launch_bounds__(kRingThreads) void k_trsv_ring_r(
    const RingBlock* __restrict__ blk, int nblk, int nblk_pad, int ngroups, const int32_t* __restrict__ lvl_ptr,
    const int32_t* __restrict__ rfoff, const int32_t* __restrict__ rboff, const int32_t* __restrict__ frec,
    const int32_t* __restrict__ brec, const TIn* x, int64_t ldx, T* ry, int64_t ldry, TOut* z, int64_t ldz,
    const int* __restrict__ done) {
    constexpr int kRing = ring_rows_r<T, R>();
    __shared__ __attribute__((aligned(16))) T ring[kRing * R];
    __shared__ int4 meta[kRingMaxLevels + 1];
    if (done && *done) return;
    const int b = blockIdx.x % nblk_pad, g = blockIdx.x / nblk_pad;
    if (b >= nblk || g >= ngroups) return;
    const RingBlock d = blk[b];
    const int nlev = d.lvl1 - d.lvl0;  // <= kRingMaxLevels (checked on the host)
    if (nlev <= 0) return;
    for (int q = threadIdx.x; q <= nlev; q += kRingThreads) {
        const int l = d.lvl0 + q;
        meta[q] = q < nlev ? int4{lvl_ptr[l] - d.row0, rfoff[l], rboff[l], 0} : int4{lvl_ptr[l] - d.row0, 0, 0, 0};
    }
    for (int q = threadIdx.x; q < kRing * R; q += kRingThreads) ring[q] = T(0);
    __syncthreads();
    const TIn* xr = x + (int64_t)g * R * ldx + d.row0;
    T* yr = ry + (int64_t)g * ldry + (int64_t)d.row0 * R;
    TOut* zr = z + (int64_t)g * R * ldz + d.row0;
    ringr_sweep<T, KW, kRing, R, false, TIn, false, T, true>(nlev, meta, ring, frec, xr, ldx, yr, 0);
    __syncthreads();
    ringr_sweep<T, KW, kRing, R, true, T, true, TOut, false>(nlev, meta, ring, brec, yr, 0, zr, ldz);
}

// ------------------------------------------------ A0 solve: one wide level
//
// For the interface block C_alpha in multicolour order the schedule has a few
// very wide levels; each level is one grid-wide launch over rows x rhs.
// kind 0 forward:   z_i = x_i - sum_j L_ij z_j
// kind 1 backward:  z_i = D_i^{-1} z_i - sum_j L_ji z_j
// kind 2 the last forward level, which has no backward dependencies:
//                   z_i = D_i^{-1} (x_i - sum_j L_ij z_j)
template <typename T, int kKind, typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_trsv_level(int a, int e, int nrhs, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                    const T* __restrict__ dinv, const TIn* x, int64_t ldx, TOut* z,
                                                    int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int r = blockIdx.y;  // grid (row chunks, nrhs)
    const int i = a + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= e) return;
    TOut* zr = z + r * ldz;
    T s = kKind == 1 ? (T)zr[i] * dinv[i] : (T)x[i + r * ldx];
    const int t0 = rp[i], t1 = rp[i + 1];
    // entries in groups of 4 with unconditional loads: an index past the row's
    // end repeats its last entry with weight 0 (s - 0 z leaves s unchanged up
    // to the sign of a zero), so a group's index, value and gather loads go out
    // together; the terms keep their order
    for (int t = t0; t < t1; t += 4) {
        int c[4];
        T w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = min(t + u, t1 - 1);
            c[u] = ci[q];
            w[u] = t + u < t1 ? v[q] : T(0);
        }
        T g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) g[u] = (T)zr[c[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) s = fnms(s, w[u], g[u]);
    }
    if (kKind == 2) s *= dinv[i];
    zr[i] = (TOut)s;
}

// The same level with one thread per row for nrhs <= NR <= kMaxRhs columns
// (NR a power of two): the row's entries are loaded once instead of once per
// column, and column indices past nrhs are clamped to the last column, so all
// loads of a row go out together (no branch per column; the surplus sums are
// not stored).  Per column the arithmetic is k_trsv_level's (same terms, same
// order).
template <typename T, int kKind, typename TIn, typename TOut, int NR>
__global__ __launch_bounds__(256) void k_trsv_level_rows(int a, int e, int nrhs, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                         const T* __restrict__ dinv, const TIn* x, int64_t ldx,
                                                         TOut* z, int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int i = a + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= e) return;
    T s[NR];
    const T di = dinv[i];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int64_t rc = min(r, nrhs - 1);
        s[r] = kKind == 1 ? (T)z[i + rc * ldz] * di : (T)x[i + rc * ldx];
    }
    const int t1 = rp[i + 1];
    for (int t = rp[i]; t < t1; ++t) {
        const int c = ci[t];
        const T vt = v[t];
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] = fnms(s[r], vt, (T)z[c + (int64_t)min(r, nrhs - 1) * ldz]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nrhs) {
            if (kKind == 2) s[r] *= di;
            z[i + (int64_t)r * ldz] = (TOut)s[r];
        }
    }
}

// ------------------------------------------------ A0 solve: interface levels through a private buffer
//
// The interface block's levels as in k_trsv_level_rows, with the values of
// interface row i also kept in a private buffer Y (row i - m holds NR values
// side by side, NR a power of two >= nrhs): a dependency of all columns is one
// vector load instead of one load per column, and each entry is one load of a
// packed (value, column) pair.  The operations and their order per column
// are those of k_trsv_level_rows.
//   kind 0 (forward):             Y_i = x_i - sum_j L_ij Y_j
//   kind 2 (last forward level):  Y_i = z_i = D_i^{-1} (x_i - sum_j L_ij Y_j)
//   kind 1 (backward):            Y_i = z_i = D_i^{-1} Y_i - sum_j L_ji Y_j
// Entry q of the interface rows' CSR: FP32 {column, value bits}, FP64
// {value low word, value high word, column, 0}.
template <typename T> struct IfacePk { using type = int2; };
template <> struct IfacePk<double> { using type = int4; };

__device__ __forceinline__ void pk_unpack(int2 t, int& c, float& v) {
    c = t.x;
    v = __int_as_float(t.y);
}
__device__ __forceinline__ void pk_unpack(int4 t, int& c, double& v) {
    c = t.z;
    v = __hiloint2double(t.y, t.x);
}

// NC columns of one row per thread (NR / NC consecutive threads share a
// row, so a row's vector of Y is read and written by neighbouring lanes).
// The entries go in groups of four with unconditional loads: an index past the
// row's end repeats its last entry with weight 0 (s - 0 g leaves s unchanged up
// to the sign of a zero), so a group's entry and gather loads go out together;
// the terms keep their order.
template <typename T, int kKind, typename TIn, typename TOut, int NR, int NC>
__global__ __launch_bounds__(256) void k_iface_rows(int a, int e, int m, int nrhs, const int32_t* __restrict__ prp,
                                                    const typename IfacePk<T>::type* __restrict__ pk,
                                                    const T* __restrict__ dinv, const TIn* x, int64_t ldx,
                                                    T* __restrict__ Y, TOut* z, int64_t ldz,
                                                    const int* __restrict__ done) {
    using V = T __attribute__((ext_vector_type(NC)));
    constexpr int G = NR / NC;
    if (done && *done) return;
    const int gid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int i = a + gid / G, c0 = (gid % G) * NC;
    if (i >= e) return;
    const int j = i - m;
    V s;
    T di = T(1);
    if constexpr (kKind != 0) di = dinv[i];
    if constexpr (kKind == 1) {
        const V y = *reinterpret_cast<const V*>(Y + (size_t)j * NR + c0);
#pragma unroll
        for (int r = 0; r < NC; ++r) s[r] = y[r] * di;
    } else {
#pragma unroll
        for (int r = 0; r < NC; ++r) s[r] = (T)x[i + (int64_t)min(c0 + r, nrhs - 1) * ldx];
    }
    const int t0 = prp[j], t1 = prp[j + 1];
    for (int t = t0; t < t1; t += 4) {
        int c[4];
        T w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            T v;
            pk_unpack(pk[min(t + u, t1 - 1)], c[u], v);
            w[u] = t + u < t1 ? v : T(0);
        }
        V g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) g[u] = *reinterpret_cast<const V*>(Y + (size_t)(c[u] - m) * NR + c0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < NC; ++r) s[r] = fnms(s[r], w[u], g[u][r]);
    }
    if constexpr (kKind == 2) {
#pragma unroll
        for (int r = 0; r < NC; ++r) s[r] *= di;
    }
    *reinterpret_cast<V*>(Y + (size_t)j * NR + c0) = s;
    if constexpr (kKind != 0) {
#pragma unroll
        for (int r = 0; r < NC; ++r)
            if (c0 + r < nrhs) z[i + (int64_t)(c0 + r) * ldz] = (TOut)s[r];
    }
}

// one thread per (row, column), grid (row chunks, NR): for levels too small
// to fill the chip one row per thread; padding columns repeat column nrhs - 1
template <typename T, int kKind, typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_iface_cols(int a, int e, int m, int nrhs, int NR,
                                                    const int32_t* __restrict__ prp,
                                                    const typename IfacePk<T>::type* __restrict__ pk,
                                                    const T* __restrict__ dinv, const TIn* x, int64_t ldx,
                                                    T* __restrict__ Y, TOut* z, int64_t ldz,
                                                    const int* __restrict__ done) {
    if (done && *done) return;
    const int r = blockIdx.y;
    const int i = a + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= e) return;
    const int j = i - m;
    T s;
    if constexpr (kKind == 1) s = Y[(size_t)j * NR + r] * dinv[i];
    else s = (T)x[i + (int64_t)min(r, nrhs - 1) * ldx];
    // entries in groups of kTermGroup: a group's entry and gather loads go
    // out together (an index past the row's end repeats its last entry and is
    // not applied), then the terms are applied in their order
    const int t1 = prp[j + 1];
    for (int t = prp[j]; t < t1; t += kTermGroup) {
        int c[kTermGroup];
        T v[kTermGroup], g[kTermGroup];
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u) pk_unpack(pk[min(t + u, t1 - 1)], c[u], v[u]);
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u) g[u] = Y[(size_t)(c[u] - m) * NR + r];
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u)
            if (t + u < t1) s = fnms(s, v[u], g[u]);
    }
    if constexpr (kKind == 2) s *= dinv[i];
    Y[(size_t)j * NR + r] = s;
    if (kKind != 0 && r < nrhs) z[i + (int64_t)r * ldz] = (TOut)s;
}

// ------------------------------------------------------------ SpMV (SELL-64)
//
// y = A x for up to kMaxRhs columns; A is FP64 in SELL-64 (slices of 64 rows,
// entries column-major inside a slice, padding points at the row itself with
// value 0).  Optionally accumulates per-chunk partial dot products x.y per
// right-hand side into part[chunk*nrhs + r], chunk = 256-row chunk index
// (used for p^T A p in CG).
// Compact SELL-64 storage: values in FP32 when every value of A is exactly an
// FP32 number (VT = float; the products are then the same doubles), columns
// as 16-bit offsets from the row when every |column - row| <= 32767
// (IT = int16_t).  The arithmetic is that of the FP64 / int32 storage.
template <typename IT> __device__ __forceinline__ int64_t sell_col(IT c, int64_t row) {
    if constexpr (sizeof(IT) == 2) return row + (int64_t)c;
    else return (int64_t)c;
}

// Loads entries j0 .. j0+7 of a lane's row in one slice without branches: an
// entry beyond the slice's width repeats the last one with weight 0, and
// adding 0 * x leaves a sum unchanged (a -0 sum may become +0), so every load
// of the group is issued before the first use.
template <typename VT, typename IT>
__device__ __forceinline__ void sell_group8(const IT* __restrict__ col, const VT* __restrict__ val, int base, int lane,
                                            int j0, int width, IT (&cg)[8], double (&ag)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int q = base + min(j0 + u, width - 1) * kSell + lane;
        cg[u] = col[q];
        const double a = (double)val[q];
        ag[u] = j0 + u < width ? a : 0.0;
    }
}

template <typename VT, typename IT>
__global__ __launch_bounds__(256) void k_spmv_sell(int64_t n, int nrhs, const int32_t* __restrict__ sptr,
                                                   const IT* __restrict__ col, const VT* __restrict__ val,
                                                   const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                                                   int64_t ldy, double* __restrict__ part,
                                                   const int* __restrict__ done) {
    __shared__ double sh[4 * kMaxRhs];
    if (done && *done) return;
    // XCD-aware chunk order: workgroups are dealt round-robin to the 8 XCDs,
    // so give each XCD one contiguous eighth of the rows (grid padded to a
    // multiple of 8); x lines gathered by neighbouring chunks then meet in
    // the same L2 instead of being fetched once per XCD.
    const int64_t per = gridDim.x >> 3;
    const int64_t wg = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int64_t row = wg * blockDim.x + threadIdx.x;
    double acc[kMaxRhs];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r) acc[r] = 0.0;
    if (row < n) {
        const int64_t sl = row >> 6;
        const int lane = (int)(row & 63);
        const int base = sptr[sl], width = (sptr[sl + 1] - base) >> 6;  // uniform: a wave is one slice
        for (int j0 = 0; j0 < width; j0 += 8) {
            IT cg[8];
            double ag[8];
            sell_group8<VT, IT>(col, val, base, lane, j0, width, cg, ag);
            int64_t c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = sell_col<IT>(cg[u], row);
            // per column the group's 8 gathers go out together, then its terms in entry order
#pragma unroll
            for (int r = 0; r < kMaxRhs; ++r) {
                if (r < nrhs) {
                    double xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) xv[u] = x[c[u] + r * ldx];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[r] += ag[u] * xv[u];
                }
            }
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
        if (threadIdx.x < nrhs && wg * blockDim.x < n) {
            const int r = threadIdx.x;
            part[wg * nrhs + r] =
                (sh[0 * kMaxRhs + r] + sh[1 * kMaxRhs + r]) + (sh[2 * kMaxRhs + r] + sh[3 * kMaxRhs + r]);
        }
    }
}

// Same product with x interleaved: x[row * S + r], S a power of two >= nrhs
// (the CG search direction is kept this way).  One gather then brings the
// values of all right-hand sides of a column in one S*8-byte segment, where
// column-major x needs one cache line per right-hand side; with 8 columns of
// 2M rows the column-major lines in flight overflow the L2 and are fetched
// several times.  Per-row sums run over the slice entries in the same order
// as k_spmv_sell, so both give the same y (k_spmv_sell's weight-0 group
// padding can turn a -0 row sum into +0).
// kPk: the entries come as packed (int32 column, FP32 value) pairs from pk
// (one load per entry instead of two; col and val unused).
template <int S, typename VT, typename IT, bool kPk = false>
__global__ __launch_bounds__(256) void k_spmv_sell_il(int64_t n, int nrhs, const int32_t* __restrict__ sptr,
                                                      const IT* __restrict__ col,
                                                      const VT* __restrict__ val, const double* __restrict__ x,
                                                      double* __restrict__ y, int64_t ldy, double* __restrict__ part,
                                                      const int* __restrict__ done,
                                                      const uint64_t* __restrict__ pk = nullptr) {
    __shared__ double sh[4 * S];
    if (done && *done) return;
    const int64_t per = gridDim.x >> 3;
    const int64_t wg = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int64_t row = wg * blockDim.x + threadIdx.x;
    double acc[S];
#pragma unroll
    for (int r = 0; r < S; ++r) acc[r] = 0.0;
    if (row < n) {
        const int64_t sl = row >> 6;
        const int lane = (int)(row & 63);
        const int base = sptr[sl], width = (sptr[sl + 1] - base) >> 6;  // uniform: a wave is one slice
        // entries in groups of 8, each guarded by the slice's width (the
        // compiler still waits for each guarded load; the unguarded grouping
        // of k_spmv_sell was slower here on wide irregular slices)
        for (int j0 = 0; j0 < width; j0 += 8) {
            int64_t cg[8];
            double ag[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j0 + u < width) {
                    const int q = base + (j0 + u) * kSell + lane;
                    // A streams through once: non-temporal loads keep the gathered x lines in L2
                    if constexpr (kPk) {
                        const uint64_t e = __builtin_nontemporal_load(pk + q);
                        cg[u] = (int64_t)(int32_t)(uint32_t)(e & 0xffffffffu);
                        ag[u] = (double)__uint_as_float((uint32_t)(e >> 32));
                    } else {
                        cg[u] = sell_col<IT>(__builtin_nontemporal_load(col + q), row);
                        ag[u] = (double)__builtin_nontemporal_load(val + q);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j0 + u < width) {
                    const double* xc = x + cg[u] * S;
                    double xv[S];
                    if constexpr (S == 1) {
                        xv[0] = xc[0];
                    } else {
#pragma unroll
                        for (int r = 0; r < S; r += 2) {
                            const double2 t = *reinterpret_cast<const double2*>(xc + r);
                            xv[r] = t.x;
                            xv[r + 1] = t.y;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < S; ++r) acc[r] += ag[u] * xv[r];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < S; ++r)
            if (r < nrhs) __builtin_nontemporal_store(acc[r], y + row + r * ldy);
    }
    if (part) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        double xr[S];  // the row's own segment, loaded at once
#pragma unroll
        for (int r = 0; r < S; ++r) xr[r] = 0.0;
        if (row < n) {
            if constexpr (S == 1) {
                xr[0] = x[row];
            } else {
#pragma unroll
                for (int r = 0; r < S; r += 2) {
                    const double2 t = *reinterpret_cast<const double2*>(x + row * S + r);
                    xr[r] = t.x;
                    xr[r + 1] = t.y;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (r < nrhs) {
                double v = acc[r] * xr[r];
                v = wave_sum(v);
                if (lane == 0) sh[w * S + r] = v;
            }
        }
        __syncthreads();
        if (threadIdx.x < nrhs && wg * blockDim.x < n) {
            const int r = threadIdx.x;
            part[wg * nrhs + r] = (sh[0 * S + r] + sh[1 * S + r]) + (sh[2 * S + r] + sh[3 * S + r]);
        }
    }
}

// ------------------------------------------------------- E and E^T products
//
// E (n x s) and E^T (s x n) as CSR in device order (E carries alpha^{-1} Ehat on
// interior rows and -alpha on the interface diagonal, eq. EF).
//   k_csr_mv:  y = M w            (E^T z, or E q for Lanczos)
//   k_csr_add: t = x + M w        (E w added to the apply's input in the same pass)
template <typename T, typename TX = T>
__global__ __launch_bounds__(256) void k_csr_mv(int64_t rows, int nrhs, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                const T* __restrict__ w, int64_t ldw, const TX* __restrict__ x,
                                                int64_t ldx, T* __restrict__ y, int64_t ldy,
                                                const int* __restrict__ done) {
    if (done && *done) return;
    // one thread per row for all columns: the row's entries are read once
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        const int t0 = rp[i], t1 = rp[i + 1];
        for (int r = 0; r < nrhs; ++r) {
            T s = x ? (T)x[i + r * ldx] : T(0);
            const T* wr = w + r * ldw;
            for (int t = t0; t < t1; ++t) s += v[t] * wr[ci[t]];
            y[i + r * ldy] = s;
        }
    }
}

// The same product for nrhs <= NR <= kMaxRhs columns (NR a power of two):
// column indices past nrhs are clamped to the last column, so every load of a
// row is issued before the first use (no branch per column; the surplus
// sums are not stored).  Per column the terms and their order are those of
// k_csr_mv, so both give bitwise the same y.
template <typename T, typename TX, int NR>
__global__ __launch_bounds__(256) void k_csr_mv_n(int64_t rows, int nrhs, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                  const T* __restrict__ w, int64_t ldw, const TX* x, int64_t ldx,
                                                  T* y, int64_t ldy, const int* __restrict__ done) {
    if (done && *done) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        const int t0 = rp[i], t1 = rp[i + 1];
        T s[NR];
        if (x) {  // one uniform branch around all the loads, so they are issued together
#pragma unroll
            for (int r = 0; r < NR; ++r) s[r] = (T)x[i + (int64_t)min(r, nrhs - 1) * ldx];
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) s[r] = T(0);
        }
        for (int t = t0; t < t1; ++t) {
            const int c = ci[t];
            const T vt = v[t];
#pragma unroll
            for (int r = 0; r < NR; ++r) s[r] += vt * w[c + (int64_t)min(r, nrhs - 1) * ldw];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nrhs) y[i + (int64_t)r * ldy] = s[r];
    }
}

// z_C = X x_C: the C_alpha solve by its approximate inverse (Sec. 4.3 (sec:csolve),
// Algorithm alg:mr).  X is stored in SELL-64 over the interface rows: rows
// sorted by entry count (longest first) and cut into slices of 64, entries
// column-major inside a slice so that a wave's loads of one entry position
// are one segment; xrow maps a slice row to its interface row, padding has
// column 0 and value 0.  One thread per row keeps all right-hand sides in
// registers, so each entry is loaded once; the sum runs over the row's
// entries in ascending column order.  x and z point at the first interface
// row (device order, ld = n).
template <typename T, typename TIn, typename TOut>
__global__ __launch_bounds__(256) void k_cinv_sell(int64_t rows, int nrhs, const int32_t* __restrict__ sptr,
                                                   const int32_t* __restrict__ xrow, const int32_t* __restrict__ col,
                                                   const T* __restrict__ val, const TIn* x, int64_t ldx, TOut* z,
                                                   int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= rows) return;
    const int64_t sl = q >> 6;
    const int lane = (int)(q & 63);
    const int base = sptr[sl], width = (sptr[sl + 1] - base) >> 6;
    T acc[kMaxRhs];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r) acc[r] = T(0);
    for (int j = 0; j < width; ++j) {
        const int e = base + j * 64 + lane;
        const int c = col[e];
        const T a = val[e];
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r)
            if (r < nrhs) acc[r] = fnms(acc[r], -a, (T)x[c + r * ldx]);  // acc + a x, one rounding
    }
    const int64_t i = xrow[q];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r)
        if (r < nrhs) z[i + r * ldz] = (TOut)acc[r];
}

// Chebyshev acceleration for the C_alpha solve (Sec. 4.3 (sec:csolve); Saad, Iterative
// Methods for Sparse Linear Systems, Alg. 12.1), on the interface rows:
// pointers at the first interface row, ld = n, grid (row chunks, nrhs).
//   first:  r = x, d = t / theta (t = D^{-1} x), acc = d
//   step:   d = c1 d + c2 t (t = D^{-1} r), acc += d
//   out:    z = acc
template <typename T, typename TIn>
__global__ void k_cheb_first(int64_t rows, const TIn* x, int64_t ldx, const T* t, T* r, T* d, T* acc, int64_t ld,
                             T inv_theta, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t c = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = i + c * ld;
        r[q] = (T)x[i + c * ldx];
        const T v = t[q] * inv_theta;
        d[q] = v;
        acc[q] = v;
    }
}

template <typename T>
__global__ void k_cheb_step(int64_t rows, T c1, T c2, const T* t, T* d, T* acc, int64_t ld,
                            const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t c = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = i + c * ld;
        const T v = c1 * d[q] + c2 * t[q];
        d[q] = v;
        acc[q] += v;
    }
}

template <typename T, typename TOut>
__global__ void k_cheb_out(int64_t rows, const T* acc, int64_t ld, TOut* z, int64_t ldz, const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t c = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
        z[i + c * ldz] = (TOut)acc[i + c * ld];
}

// ------------------------------------------------------- low-rank correction
//
// DDLR-1 (eq. gkt):  w = c0 y + U_k (d .* (U_k^T y)),   U_k: s x k
// DDLR-2 (eq. Form2a): u = u + U_k (H_k (U_k^T x)),    U_k: n x k
// U_k is row-major (k contiguous per row).  Stage 1 accumulates per-block
// partials of U_k^T y (k x nrhs); stage 2 sums them in fixed order and applies
// d (DDLR-1) or H_k (DDLR-2); stage 3 expands.
template <typename T, typename TY = T>
__global__ __launch_bounds__(256) void k_lr_reduce(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                   const TY* __restrict__ y, int64_t ldy, double* __restrict__ part,
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

// Sum of part[b * stride + col] over b = threadIdx.x, threadIdx.x + blockDim.x,
// ... < nparts, in that order; groups of 8 loads are issued before their adds.
__device__ __forceinline__ double strided_sum(const double* __restrict__ part, int nparts, int stride, int col) {
    double acc = 0.0;
    const int step = blockDim.x;
    int b = threadIdx.x;
    for (; b + 7 * step < nparts; b += 8 * step) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u * step) * stride + col];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; b < nparts; b += step) acc += part[(int64_t)b * stride + col];
    return acc;
}

// out[col] = sum over parts of part[b*ncols + col], one workgroup per column, fixed order
__global__ __launch_bounds__(256) void k_reduce_cols(int nparts, int ncols, const double* __restrict__ part,
                                                     double* __restrict__ out, const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    const int col = blockIdx.x;
    const double s = block_sum256(strided_sum(part, nparts, ncols, col), sh);
    if (threadIdx.x == 0) out[col] = s;
}

// out[i] = beta * in[i] + sum_j U[i][j] coef[r][j]
template <typename T, typename TIO = T>
__global__ __launch_bounds__(256) void k_lr_expand(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                   const double* __restrict__ coef, double beta, const TIO* in,
                                                   int64_t ldin, TIO* out, int64_t ldout, const int* __restrict__ done) {
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
            if (r < nrhs) out[i + r * ldout] = (TIO)acc[r];
    }
}

// ------------------------------------------- low-rank correction on MFMA
//
// Tall-skinny products with the matrix cores, 16x16x4 MFMA (FP64 for the FP64
// path, FP32 for the mixed path).  Operand layout of the 16x16x4 MFMA
// (wave64): A (16x4) lane l holds A[l%16][l/16]; B (4x16) lane l holds
// B[l/16][l%16]; C (16x16) lane l, register v holds C[row(l,v)][l%16] with
// row = 4*(l/16)+v for FP32 and row = l/16 + 4*v for FP64 (measured on gfx950).
typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
    typedef mfma_f32x4 type;
    static __device__ __forceinline__ type step(float a, float b, type c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct MfmaAcc<double> {
    typedef mfma_f64x4 type;
    static __device__ __forceinline__ type step(double a, double b, type c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// Reduce: part[block][r][j] = sum over the block's rows of U[row][j] y_r[row].
// C = U^T Y: M = k (tiles of 16), N = nrhs (<= 16), K = rows (steps of 4).
// Each wave owns a contiguous run of rows; k <= 128 -> up to 8 accumulator tiles.
template <typename T, typename TY = T>
__global__ __launch_bounds__(256) void k_lr_reduce_mfma(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                        const TY* __restrict__ y, int64_t ldy,
                                                        double* __restrict__ part, const int* __restrict__ done) {
    typedef typename MfmaAcc<T>::type acc_t;
    __shared__ double stage[4][64];
    if (done && *done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nwaves = gridDim.x * 4;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wv;
    const int64_t per = ((rows + nwaves - 1) / nwaves + 3) & ~(int64_t)3;
    const int64_t r0 = gw * per, r1 = r0 + per < rows ? r0 + per : rows;
    const int ntile = (k + 15) >> 4;
    acc_t acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = acc_t{0, 0, 0, 0};
    const int col = lane & 15, kk = lane >> 4;
    for (int64_t i0 = r0; i0 < r1; i0 += 4) {
        const int64_t i = i0 + kk;
        const bool ok = i < r1;
        const T bval = (ok && col < nrhs) ? (T)y[i + col * ldy] : T(0);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (t < ntile) {
                const int j = t * 16 + col;
                const T aval = (ok && j < k) ? U[i * k + j] : T(0);
                acc[t] = MfmaAcc<T>::step(aval, bval, acc[t]);
            }
    }
    // acc[t] holds C[j = 16t + row(lane, v)][rhs = lane%16]; fold the 4 waves through LDS
    for (int t = 0; t < ntile; ++t) {
        for (int v = 0; v < 4; ++v) {
            stage[wv][lane] = (double)acc[t][v];
            __syncthreads();
            const int j = t * 16 + MfmaAcc<T>::row(lane, v), rr = lane & 15;
            if (wv == 0 && j < k && rr < nrhs)
                part[((int64_t)blockIdx.x * nrhs + rr) * k + j] =
                    (stage[0][lane] + stage[1][lane]) + (stage[2][lane] + stage[3][lane]);
            __syncthreads();
        }
    }
}

// Expand: out[row][r] = beta in[row][r] + sum_j U[row][j] coef[r][j].
// M = 16 rows, N = nrhs (<= 16), K = k (steps of 4); one 16-row tile per wave-step.
template <typename T, typename TIO = T>
__global__ __launch_bounds__(256) void k_lr_expand_mfma(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                        const double* __restrict__ coef, double beta, const TIO* in,
                                                        int64_t ldin, TIO* out, int64_t ldout,
                                                        const int* __restrict__ done) {
    typedef typename MfmaAcc<T>::type acc_t;
    __shared__ T cf[128 * 16];  // cf[j*16 + r]
    if (done && *done) return;
    for (int q = threadIdx.x; q < 128 * 16; q += blockDim.x) {
        const int j = q >> 4, rr = q & 15;
        cf[q] = (j < k && rr < nrhs) ? (T)coef[rr * k + j] : T(0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row_in = lane & 15, kk = lane >> 4;
    const int64_t ntiles = (rows + 15) >> 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t i = tile * 16 + row_in;
        acc_t acc = acc_t{0, 0, 0, 0};
        for (int j0 = 0; j0 < k; j0 += 4) {
            const int j = j0 + kk;
            const T aval = (i < rows && j < k) ? U[i * k + j] : T(0);
            const T bval = cf[j * 16 + (lane & 15)];
            acc = MfmaAcc<T>::step(aval, bval, acc);
        }
        const int rr = lane & 15;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = tile * 16 + MfmaAcc<T>::row(lane, v);
            if (row < rows && rr < nrhs) {
                const double o = beta * (double)in[row + rr * ldin] + (double)acc[v];
                out[row + rr * ldout] = (TIO)o;
            }
        }
    }
}

// ----------------------- low-rank correction, wide operand loads (k % 16 == 0)
//
// The kernels above load one U_k element per lane per MFMA step, so at k =
// 32 a wave walks its rows in a chain of 4-byte loads feeding MFMAs and the
// correction runs at a fraction of HBM bandwidth.  These variants load the
// operands of four MFMA steps with one 16-byte (FP32) or two 16-byte (FP64)
// loads per lane.
//
// Reduction: U_k is also kept in MFMA tile order, Ut: for row tile rt (16
// rows) and column tile jt (16 columns), lane l = (m = l%16, q = l/16) holds
// four consecutive values U[16 rt + 4q + s][16 jt + m], s = 0..3, which are
// its A operands (row j = 16jt + m, K index q) for the four K steps of the
// tile; the y operand of lane (n = l%16, q) at step s is y[16 rt + 4q + s][n].
template <typename T>
__global__ void k_make_ut(int64_t rows, int k, const T* __restrict__ U, T* __restrict__ Ut) {
    const int njt = k >> 4;
    const int64_t nrt = (rows + 15) >> 4;
    const int64_t total = nrt * njt * 256;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(g & 3), l = (int)((g >> 2) & 63);
        const int64_t t = g >> 8;
        const int jt = (int)(t % njt);
        const int64_t rt = t / njt;
        const int64_t row = 16 * rt + 4 * (l >> 4) + s;
        const int j = 16 * jt + (l & 15);
        Ut[g] = row < rows ? U[row * k + j] : T(0);
    }
}

template <typename T> struct Vec4 { typedef T __attribute__((ext_vector_type(4))) type; };

template <typename T, typename TY, int NJT>
__global__ __launch_bounds__(256) void k_lr_reduce_t(int64_t rows, int k, int nrhs, const T* __restrict__ Ut,
                                                     const TY* __restrict__ y, int64_t ldy, double* __restrict__ part,
                                                     const int* __restrict__ done) {
    typedef typename MfmaAcc<T>::type acc_t;
    typedef typename Vec4<T>::type v4;
    __shared__ double stage[4][64];
    if (done && *done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nwaves = gridDim.x * 4;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wv;
    const int64_t nrt = (rows + 15) >> 4;
    const int64_t per = (nrt + nwaves - 1) / nwaves;
    const int64_t t0 = gw * per, t1 = t0 + per < nrt ? t0 + per : nrt;
    // NJT = k / 16 column tiles (a template parameter, so no load sits in a
    // per-tile branch); y is read at clamped indices and zeroed by selection
    acc_t acc[NJT];
#pragma unroll
    for (int t = 0; t < NJT; ++t) acc[t] = acc_t{0, 0, 0, 0};
    const int n = lane & 15, q = lane >> 4;
    const int nc = min(n, nrhs - 1);
    const v4* Ut4 = reinterpret_cast<const v4*>(Ut);
#pragma unroll 2
    for (int64_t rt = t0; rt < t1; ++rt) {
        T b[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int64_t row = 16 * rt + 4 * q + st;
            const T yv = (T)y[(row < rows ? row : rows - 1) + nc * ldy];
            b[st] = (row < rows && n < nrhs) ? yv : T(0);
        }
#pragma unroll
        for (int jt = 0; jt < NJT; ++jt) {
            const v4 a = Ut4[(rt * NJT + jt) * 64 + lane];
#pragma unroll
            for (int st = 0; st < 4; ++st) acc[jt] = MfmaAcc<T>::step(a[st], b[st], acc[jt]);
        }
    }
    // acc[t] holds C[j = 16t + row(lane, v)][rhs = lane%16]; fold the 4 waves through LDS
    for (int t = 0; t < NJT; ++t) {
        for (int v = 0; v < 4; ++v) {
            stage[wv][lane] = (double)acc[t][v];
            __syncthreads();
            const int j = t * 16 + MfmaAcc<T>::row(lane, v), rr = lane & 15;
            if (wv == 0 && rr < nrhs)
                part[((int64_t)blockIdx.x * nrhs + rr) * k + j] =
                    (stage[0][lane] + stage[1][lane]) + (stage[2][lane] + stage[3][lane]);
            __syncthreads();
        }
    }
}

// Expansion: out[row][r] = beta in[row][r] + sum_j U[row][j] coef[r][j] with
// row-major U_k.  Lane (m = l%16 -> row, q = l/16) loads U[row][16c + 4q ..
// 16c + 4q + 3] in one go and uses element s at K step s, whose K index q
// stands for column j = 16c + 4q + s; the coefficient operand follows the
// same j.  M = 16 rows, N = nrhs (<= 16).
template <typename T, typename TIO, int NC>
__global__ __launch_bounds__(256) void k_lr_expand_v(int64_t rows, int k, int nrhs, const T* __restrict__ U,
                                                     const double* __restrict__ coef, double beta, const TIO* in,
                                                     int64_t ldin, TIO* out, int64_t ldout,
                                                     const int* __restrict__ done) {
    typedef typename MfmaAcc<T>::type acc_t;
    typedef typename Vec4<T>::type v4;
    __shared__ T cf[128 * 16];  // cf[j*16 + r]
    if (done && *done) return;
    for (int qq = threadIdx.x; qq < 128 * 16; qq += blockDim.x) {
        const int j = qq >> 4, rr = qq & 15;
        cf[qq] = (j < k && rr < nrhs) ? (T)coef[rr * k + j] : T(0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, q = lane >> 4;
    const int64_t ntiles = (rows + 15) >> 4;
    // NC = k / 16 column chunks (a template parameter, so no load sits in a
    // per-chunk branch); the input is read at clamped indices before the stores
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t i = tile * 16 + m;
        const int64_t ic = i < rows ? i : rows - 1;  // clamped row: loaded, never stored
        acc_t acc = acc_t{0, 0, 0, 0};
        v4 a[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] = *reinterpret_cast<const v4*>(U + ic * k + 16 * c + 4 * q);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int st = 0; st < 4; ++st)
                acc = MfmaAcc<T>::step(a[c][st], cf[(16 * c + 4 * q + st) * 16 + m], acc);
        const int rr = lane & 15, rc = min(rr, nrhs - 1);
        double iv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = tile * 16 + MfmaAcc<T>::row(lane, v);
            iv[v] = (double)in[(row < rows ? row : rows - 1) + rc * ldin];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = tile * 16 + MfmaAcc<T>::row(lane, v);
            if (row < rows && rr < nrhs) {
                const double o = beta * iv[v] + (double)acc[v];
                out[row + rr * ldout] = (TIO)o;
            }
        }
    }
}

// ------------------------------------- low-rank correction, BF16 U_k (gfx950)
//
// U_k stored in bfloat16 (rounded from the FP64 basis), products on the
// 16x16x32 bf16 MFMA with FP32 accumulation.  Operand layout (measured on
// gfx950): lane l, element e holds A[l%16][8(l/16)+e] and B[8(l/16)+e][l%16];
// the FP32 result is laid out as for the 16x16x4 FP32 MFMA.  The vector
// operand (y in the reduction, the coefficients in the expansion) is split
// into a high and a low bf16 part and both are multiplied, so only U_k
// carries bf16 rounding.
typedef __bf16 mfma_bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ mfma_f32x4 mfma_bf16(mfma_bf16x8 a, mfma_bf16x8 b, mfma_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Tiled copy for the reduction: Ut[(rb * ktiles + jt) * 512 + l * 8 + e] =
// U[32 rb + 8 (l/16) + e][16 jt + l%16] (zero outside rows x k).  Row-major
// copy for the expansion: Ur[i * kp + j] (kp = k rounded up to 32).
__global__ void k_make_bf16(int64_t rows, int k, const double* __restrict__ U, int kp, int ktiles,
                            __bf16* __restrict__ Ur, __bf16* __restrict__ Ut) {
    const int64_t nb = (rows + 31) / 32;
    const int64_t tot_t = nb * ktiles * 512, tot_r = rows * kp;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < tot_t + tot_r;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (g < tot_t) {
            const int64_t blk = g / 512;
            const int idx = (int)(g - blk * 512), l = idx / 8, e = idx % 8;
            const int64_t rb = blk / ktiles;
            const int jt = (int)(blk - rb * ktiles);
            const int64_t i = rb * 32 + 8 * (l / 16) + e;
            const int j = jt * 16 + l % 16;
            Ut[g] = (__bf16)((i < rows && j < k) ? U[i * k + j] : 0.0);
        } else {
            const int64_t q = g - tot_t, i = q / kp;
            const int j = (int)(q - i * kp);
            Ur[q] = (__bf16)(j < k ? U[i * k + j] : 0.0);
        }
    }
}

template <typename TY>
__global__ __launch_bounds__(256) void k_lr_reduce_bf16(int64_t rows, int k, int nrhs, const __bf16* __restrict__ Ut,
                                                        const TY* __restrict__ y, int64_t ldy,
                                                        double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double stage[4][64];
    if (done && *done) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ktiles = (k + 15) >> 4;
    const int64_t nb = (rows + 31) / 32;
    const int nwaves = gridDim.x * 4;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wv;
    const int64_t per = (nb + nwaves - 1) / nwaves;
    const int64_t b0 = gw * per, b1 = b0 + per < nb ? b0 + per : nb;
    mfma_f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma_f32x4{0, 0, 0, 0};
    const int n = lane & 15, kg = lane >> 4;
    for (int64_t rb = b0; rb < b1; ++rb) {
        mfma_bf16x8 yh, yl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t i = rb * 32 + 8 * kg + e;
            const float v = (i < rows && n < nrhs) ? (float)y[i + n * ldy] : 0.f;
            const __bf16 hi = (__bf16)v;
            yh[e] = hi;
            yl[e] = (__bf16)(v - (float)hi);
        }
        const __bf16* ub = Ut + (rb * ktiles) * 512 + lane * 8;
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (t < ktiles) {
                const mfma_bf16x8 a = *reinterpret_cast<const mfma_bf16x8*>(ub + t * 512);
                acc[t] = mfma_bf16(a, yh, acc[t]);
                acc[t] = mfma_bf16(a, yl, acc[t]);
            }
    }
    for (int t = 0; t < ktiles; ++t) {
        for (int v = 0; v < 4; ++v) {
            stage[wv][lane] = (double)acc[t][v];
            __syncthreads();
            const int j = t * 16 + 4 * (lane >> 4) + v, rr = lane & 15;
            if (wv == 0 && j < k && rr < nrhs)
                part[((int64_t)blockIdx.x * nrhs + rr) * k + j] =
                    (stage[0][lane] + stage[1][lane]) + (stage[2][lane] + stage[3][lane]);
            __syncthreads();
        }
    }
}

template <typename TIO>
__global__ __launch_bounds__(256) void k_lr_expand_bf16(int64_t rows, int k, int kp, int nrhs,
                                                        const __bf16* __restrict__ Ur,
                                                        const double* __restrict__ coef, double beta, const TIO* in,
                                                        int64_t ldin, TIO* out, int64_t ldout,
                                                        const int* __restrict__ done) {
    __shared__ __bf16 ch[128 * 16], cl[128 * 16];  // coefficient hi / lo parts, [j][r]
    if (done && *done) return;
    for (int q = threadIdx.x; q < kp * 16; q += blockDim.x) {
        const int j = q >> 4, rr = q & 15;
        const float v = (j < k && rr < nrhs) ? (float)coef[rr * k + j] : 0.f;
        const __bf16 hi = (__bf16)v;
        ch[q] = hi;
        cl[q] = (__bf16)(v - (float)hi);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int64_t ntiles = (rows + 15) >> 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t i = tile * 16 + m;
        mfma_f32x4 acc = mfma_f32x4{0, 0, 0, 0};
        for (int k0 = 0; k0 < kp; k0 += 32) {
            mfma_bf16x8 a;
            if (i < rows) a = *reinterpret_cast<const mfma_bf16x8*>(Ur + i * kp + k0 + 8 * kg);
            else
#pragma unroll
                for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.f;
            mfma_bf16x8 bh, bl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                bh[e] = ch[(k0 + 8 * kg + e) * 16 + m];
                bl[e] = cl[(k0 + 8 * kg + e) * 16 + m];
            }
            acc = mfma_bf16(a, bh, acc);
            acc = mfma_bf16(a, bl, acc);
        }
        const int rr = lane & 15;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = tile * 16 + 4 * kg + v;
            if (row < rows && rr < nrhs) {
                const double o = beta * (double)in[row + rr * ldin] + (double)acc[v];
                out[row + rr * ldout] = (TIO)o;
            }
        }
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
// phase: 0 idle, 1 initialising (r = b, x = 0, p = 0 on entry), 2 running,
// 3 finished.  active == (phase == 2).  A lane in phase 1 runs one pass of the
// iteration kernels with alpha = 0 (x and r unchanged) that computes
// bb = ||b||^2, z = M^{-1} r, rz = r.z and p = z, exactly the CG start, so a
// lane's arithmetic does not depend on when it entered or on other lanes.
struct CgLane {
    double bb, rz, rr, alpha, beta, tol2;
    int32_t active, its, phase, maxit;
};

// CG scalar update `what` of one lane from its reduced dot product s
__device__ __forceinline__ void lane_update(int what, CgLane& l, double s) {
    if (what == 2) {
        l.alpha = l.phase == 2 ? l.rz / s : 0.0;
    } else if (what == 3) {
        if (l.phase == 1) {
            l.bb = s;
            l.rr = s;
            if (!(s > 0.0)) { l.phase = 3; l.active = 0; }
        } else if (l.phase == 2) {
            l.rr = s;
            l.its += 1;
            if (s <= l.tol2 * l.bb || l.its >= l.maxit) { l.phase = 3; l.active = 0; }
        }
    } else if (what == 4) {
        if (l.phase == 1) {
            l.rz = s;
            l.beta = 0.0;
            l.phase = 2;
            l.active = 1;
        } else if (l.phase == 2) {
            l.beta = s / l.rz;
            l.rz = s;
        }
    }
}

// Lane-phase CG scalars (one thread per lane, blockDim >= nlanes); sums[r]
// is the reduced dot product of lane r.  what: 2 alpha (p.Ap), 3 residual
// check / initialisation of bb, 4 beta (r.z).  done := no lane initialising
// or running.
__global__ void k_lane_scalar(int what, int nlanes, const double* __restrict__ sums, CgLane* __restrict__ L,
                              int* __restrict__ done) {
    if (done && *done) return;
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < nlanes; r += blockDim.x) {
        CgLane& l = L[r];
        lane_update(what, l, sums[r]);
        if (l.phase == 1 || l.phase == 2) any = 1;  // benign race: every writer stores 1
    }
    __syncthreads();
    if (what == 3 && threadIdx.x == 0 && done) *done = any ? 0 : 1;
}

// k_reduce_cols and k_lane_scalar in one launch: workgroup r sums lane r's
// partials (the order of k_reduce_cols, so the sum is bitwise the same) and
// updates lane r.  The residual check (what == 3) also sets done := no lane
// initialising or running: each workgroup counts itself on a device-scope
// atomic after a release fence, and the one completing the count reads every
// lane (acquire fence), stores done and re-arms the counter.  No workgroup
// waits for another.  256 threads, one workgroup per lane.
__global__ __launch_bounds__(256) void k_reduce_lane(int what, int nparts, int nlanes,
                                                     const double* __restrict__ part, double* __restrict__ sums,
                                                     CgLane* __restrict__ L, int* __restrict__ done,
                                                     unsigned* __restrict__ ctr) {
    __shared__ double sh[4];
    __shared__ int is_last;
    if (*done) return;
    const int col = blockIdx.x;
    const double s = block_sum256(strided_sum(part, nparts, nlanes, col), sh);
    if (threadIdx.x == 0) {
        sums[col] = s;
        lane_update(what, L[col], s);
    }
    if (what != 3) return;
    if (threadIdx.x == 0) {
        __threadfence();
        is_last = atomicAdd(ctr, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last || threadIdx.x != 0) return;
    __threadfence();
    int any = 0;
    for (int r = 0; r < nlanes; ++r) any |= (L[r].phase == 1 || L[r].phase == 2);
    *done = any ? 0 : 1;
    *ctr = 0u;
}

// Admission of lanes: lane r in [0, nlanes) with start[r] != 0 enters phase 1
// with its tolerance and iteration limit; its x and p columns are zeroed.
__global__ void k_lane_admit(int nlanes, const int32_t* __restrict__ start, const double* __restrict__ tol2,
                             const int32_t* __restrict__ maxit, CgLane* __restrict__ L, int* __restrict__ done) {
    const int r = threadIdx.x;
    if (r < nlanes && start[r]) {
        CgLane& l = L[r];
        l.bb = l.rz = l.rr = l.alpha = l.beta = 0.0;
        l.tol2 = tol2[r];
        l.maxit = maxit[r];
        l.its = 0;
        l.phase = 1;
        l.active = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && done) {
        int any = 0;
        for (int q = 0; q < nlanes; ++q) any |= (L[q].phase == 1 || L[q].phase == 2);
        *done = any ? 0 : 1;
    }
}

// x[:, r] = 0 and p[:, r] = 0 for admitted lanes
// x is column-major (ld); p is interleaved with stride S (p[i * S + r]).
__global__ void k_lane_zero(int64_t n, int nlanes, int lgS, const int32_t* __restrict__ start,
                            double* __restrict__ x, double* __restrict__ p, int64_t ld) {
    const int64_t total = n << lgS;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g >> lgS;
        const int r = (int)(g & ((1 << lgS) - 1));
        if (r < nlanes && start[r]) {
            x[i + r * ld] = 0.0;
            p[g] = 0.0;
        }
    }
}

// x += alpha p ; r -= alpha q ; part = r.r   (active lanes only).  x, r, q
// column-major (ld); p interleaved with stride S.  Each thread walks its rows
// once for all lanes; every lane's sum runs over the same rows in the same
// order whatever the number of lanes, so a lane's result does not depend on
// the other lanes.
template <int S>
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int nrhs, const CgLane* __restrict__ L,
                                               const double* __restrict__ p, const double* __restrict__ q,
                                               double* __restrict__ x, double* __restrict__ r, int64_t ld,
                                               double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    bool act[S];
    double a[S], acc[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
        act[c] = c < nrhs && L[c].active;
        a[c] = c < nrhs ? L[c].alpha : 0.0;
        acc[c] = 0.0;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double pv[S];
        if constexpr (S == 1) {
            pv[0] = p[i];
        } else {
#pragma unroll
            for (int c = 0; c < S; c += 2) {
                const double2 t = *reinterpret_cast<const double2*>(p + i * S + c);
                pv[c] = t.x;
                pv[c + 1] = t.y;
            }
        }
#pragma unroll
        for (int c = 0; c < S; ++c) {
            if (c < nrhs) {
                const int64_t o = i + c * ld;
                double ri = r[o];
                if (act[c]) {
                    x[o] += a[c] * pv[c];
                    ri -= a[c] * q[o];
                    r[o] = ri;
                }
                acc[c] += ri * ri;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < S; ++c) {
        if (c < nrhs) {
            const double t = block_sum256(acc[c], sh);
            if (threadIdx.x == 0) part[blockIdx.x * nrhs + c] = t;
        }
    }
}

// The two halves of k_cg_xr for overlapping x with the preconditioner: r -=
// alpha q with the r.r partials on the critical path (it also records the
// step xa[c] = alpha for active lanes, 0 otherwise), and x += xa p on a side
// stream while the preconditioner runs.  Same per-element arithmetic as
// k_cg_xr.
template <int S>
__global__ __launch_bounds__(256) void k_cg_r(int64_t n, int nrhs, const CgLane* __restrict__ L,
                                              const double* __restrict__ q, double* __restrict__ r, int64_t ld,
                                              double* __restrict__ xa, double* __restrict__ part,
                                              const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) {  // nothing running: the forked x update must do nothing
        if (blockIdx.x == 0 && threadIdx.x < nrhs) xa[threadIdx.x] = 0.0;
        return;
    }
    bool act[S];
    double a[S], acc[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
        act[c] = c < nrhs && L[c].active;
        a[c] = c < nrhs ? L[c].alpha : 0.0;
        acc[c] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x < nrhs) xa[threadIdx.x] = L[threadIdx.x].active ? L[threadIdx.x].alpha : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < S; ++c) {
            if (c < nrhs) {
                const int64_t o = i + c * ld;
                double ri = r[o];
                if (act[c]) {
                    ri -= a[c] * q[o];
                    r[o] = ri;
                }
                acc[c] += ri * ri;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < S; ++c) {
        if (c < nrhs) {
            const double t = block_sum256(acc[c], sh);
            if (threadIdx.x == 0) part[blockIdx.x * nrhs + c] = t;
        }
    }
}

// k_cg_x does not read the done flag: it may start after the residual check
// of the same iteration has set it, and must still apply that iteration's
// step.  Its own work list is the xa snapshot (all zero: nothing to do).
template <int S>
__global__ __launch_bounds__(256) void k_cg_x(int64_t n, int nrhs, const double* __restrict__ xa,
                                              const double* __restrict__ p, double* __restrict__ x, int64_t ld) {
    double a[S];
    bool any = false;
#pragma unroll
    for (int c = 0; c < S; ++c) {
        a[c] = c < nrhs ? xa[c] : 0.0;
        any = any || a[c] != 0.0;
    }
    if (!any) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double pv[S];
        if constexpr (S == 1) {
            pv[0] = p[i];
        } else {
#pragma unroll
            for (int c = 0; c < S; c += 2) {
                const double2 t = *reinterpret_cast<const double2*>(p + i * S + c);
                pv[c] = t.x;
                pv[c + 1] = t.y;
            }
        }
#pragma unroll
        for (int c = 0; c < S; ++c)
            if (c < nrhs && a[c] != 0.0) x[i + c * ld] += a[c] * pv[c];
    }
}

// k_cg_x and k_cg_p in one pass: x += xa p with the old p (xa: the step
// k_cg_r recorded, zero for lanes that were not running), then p = z + beta p
// for the active lanes; same per-element arithmetic as the two kernels.  It
// does not read the done flag: the last iteration's x step must still be
// applied after the residual check has set it; with no step and no active
// lane it returns at once.
template <int S>
__global__ __launch_bounds__(256) void k_cg_xp(int64_t n, int nrhs, const CgLane* __restrict__ L,
                                               const double* __restrict__ xa, const double* __restrict__ z,
                                               double* __restrict__ p, double* __restrict__ x, int64_t ld) {
    bool act[S];
    double bt[S], a[S];
    bool any = false;
#pragma unroll
    for (int c = 0; c < S; ++c) {
        act[c] = c < nrhs && L[c].active;
        bt[c] = act[c] ? L[c].beta : 0.0;
        a[c] = c < nrhs ? xa[c] : 0.0;
        any = any || act[c] || a[c] != 0.0;
    }
    if (!any) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double pv[S], zv[S];
        if constexpr (S == 1) {
            pv[0] = p[i];
        } else {
#pragma unroll
            for (int c = 0; c < S; c += 2) {
                const double2 t = *reinterpret_cast<const double2*>(p + i * S + c);
                pv[c] = t.x;
                pv[c + 1] = t.y;
            }
        }
#pragma unroll
        for (int c = 0; c < S; ++c) zv[c] = z[i + (int64_t)min(c, nrhs - 1) * ld];
#pragma unroll
        for (int c = 0; c < S; ++c)
            if (c < nrhs && a[c] != 0.0) x[i + c * ld] += a[c] * pv[c];
#pragma unroll
        for (int c = 0; c < S; ++c)
            if (act[c]) pv[c] = zv[c] + bt[c] * pv[c];
        if constexpr (S == 1) {
            p[i] = pv[0];
        } else {
#pragma unroll
            for (int c = 0; c < S; c += 2)
                *reinterpret_cast<double2*>(p + i * S + c) = double2{pv[c], pv[c + 1]};
        }
    }
}

// p = z + beta p (active lanes); z column-major (ld), p interleaved with
// stride S.  One thread per row: a wave reads and writes 64 whole p segments
// (contiguous) and 64 consecutive rows of each z column; z is read at clamped
// column indices so every load of a row goes out before the first use.  An
// inactive lane's p values are written back unchanged.
template <int S>
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, int nrhs, const CgLane* __restrict__ L,
                                              const double* __restrict__ z, double* __restrict__ p, int64_t ld,
                                              const int* __restrict__ done) {
    if (done && *done) return;
    bool act[S];
    double bt[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
        act[c] = c < nrhs && L[c].active;
        bt[c] = act[c] ? L[c].beta : 0.0;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double pv[S], zv[S];
        if constexpr (S == 1) {
            pv[0] = p[i];
        } else {
#pragma unroll
            for (int c = 0; c < S; c += 2) {
                const double2 t = *reinterpret_cast<const double2*>(p + i * S + c);
                pv[c] = t.x;
                pv[c + 1] = t.y;
            }
        }
#pragma unroll
        for (int c = 0; c < S; ++c) zv[c] = z[i + (int64_t)min(c, nrhs - 1) * ld];
#pragma unroll
        for (int c = 0; c < S; ++c)
            if (act[c]) pv[c] = zv[c] + bt[c] * pv[c];
        if constexpr (S == 1) {
            p[i] = pv[0];
        } else {
#pragma unroll
            for (int c = 0; c < S; c += 2)
                *reinterpret_cast<double2*>(p + i * S + c) = double2{pv[c], pv[c + 1]};
        }
    }
}

// ------------------------------------------------------------ batches
//
// A batch concatenates independent systems: system q owns device rows
// [roff[q], roff[q+1]) and interface positions [soff[q], soff[q+1]).  SpMV,
// the A0 solve and the E / E^T products run over the union unchanged; the
// reductions, the CG scalars and the low-rank correction are per system.
// Grids are (chunks, systems): blockIdx.y selects the system, so every block
// knows its system without a per-row lookup.

// part[chunk * nsys + q] = partial a . b over system q's rows
__global__ __launch_bounds__(256) void k_seg_dot(const int64_t* __restrict__ roff, const double* __restrict__ a,
                                                 const double* __restrict__ b, double* __restrict__ part,
                                                 const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    const int q = blockIdx.y, nsys = gridDim.y;
    const int64_t r0 = roff[q], r1 = roff[q + 1];
    double acc = 0.0;
    for (int64_t i = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < r1; i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    const double t = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nsys + q] = t;
}

// x += alpha_q p ; r -= alpha_q q ; part = r.r   per system
__global__ __launch_bounds__(256) void k_seg_cg_xr(const int64_t* __restrict__ roff, const CgLane* __restrict__ L,
                                                   const double* __restrict__ p, const double* __restrict__ qv,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double sh[4];
    if (done && *done) return;
    const int q = blockIdx.y, nsys = gridDim.y;
    const int64_t r0 = roff[q], r1 = roff[q + 1];
    const bool act = L[q].active;
    const double a = L[q].alpha;
    double acc = 0.0;
    for (int64_t i = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < r1; i += (int64_t)gridDim.x * blockDim.x) {
        double ri = r[i];
        if (act) {
            x[i] += a * p[i];
            ri -= a * qv[i];
            r[i] = ri;
        }
        acc += ri * ri;
    }
    const double t = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nsys + q] = t;
}

// p = z + beta_q p (active systems); init: p = z
__global__ __launch_bounds__(256) void k_seg_cg_p(const int64_t* __restrict__ roff, const CgLane* __restrict__ L,
                                                  int init, const double* __restrict__ z, double* __restrict__ p,
                                                  const int* __restrict__ done) {
    if (done && *done) return;
    const int q = blockIdx.y;
    const int64_t r0 = roff[q], r1 = roff[q + 1];
    const bool act = L[q].active;
    const double be = L[q].beta;
    for (int64_t i = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < r1; i += (int64_t)gridDim.x * blockDim.x) {
        if (init) p[i] = z[i];
        else if (act) p[i] = z[i] + be * p[i];
    }
}

// DDLR-1 coefficients of each system: coef[q][j] = d_q[j] * sum over system
// q's interface positions of U[i][j] y[i].  One workgroup per system; lanes
// own columns, the four waves stride the rows, fixed-order fold.
template <typename T>
__global__ __launch_bounds__(256) void k_seg_lr_coef(const int64_t* __restrict__ soff, int k, const T* __restrict__ U,
                                                     const T* __restrict__ y, const double* __restrict__ dvec,
                                                     double* __restrict__ coef, const int* __restrict__ done) {
    __shared__ double sh[4][64];
    if (done && *done) return;
    const int q = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = soff[q], r1 = soff[q + 1];
    for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + lane;
        double acc = 0.0;
        if (j < k)
            for (int64_t i = r0 + wv; i < r1; i += 4) acc += (double)U[i * k + j] * (double)y[i];
        sh[wv][lane] = acc;
        __syncthreads();
        if (wv == 0 && j < k)
            coef[(int64_t)q * k + j] = dvec[(int64_t)q * k + j] * ((sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]));
        __syncthreads();
    }
}

// w = c0_q y + U coef_q over each system's interface positions
template <typename T>
__global__ __launch_bounds__(256) void k_seg_lr_expand(const int64_t* __restrict__ soff, int k, const T* __restrict__ U,
                                                       const double* __restrict__ coef, const double* __restrict__ c0,
                                                       const T* __restrict__ y, T* __restrict__ w,
                                                       const int* __restrict__ done) {
    __shared__ double cf[128];
    if (done && *done) return;
    const int q = blockIdx.y;
    for (int j = threadIdx.x; j < k; j += blockDim.x) cf[j] = coef[(int64_t)q * k + j];
    __syncthreads();
    const int64_t r0 = soff[q], r1 = soff[q + 1];
    const double cq = c0[q];
    for (int64_t i = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < r1; i += (int64_t)gridDim.x * blockDim.x) {
        double v = cq * (double)y[i];
        for (int j = 0; j < k; ++j) v += (double)U[i * k + j] * cf[j];
        w[i] = (T)v;
    }
}

// CG scalars of many lanes: one thread per lane (blockDim >= nlanes)
__global__ void k_cg_scalar_many(int what, int nlanes, const double* __restrict__ sums, CgLane* __restrict__ L,
                                 double tol2, int maxit, int* __restrict__ done) {
    if (what != 0 && done && *done) return;
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < nlanes; r += blockDim.x) {
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
        if (l.active) any = 1;  // benign race: every writer stores 1
    }
    __syncthreads();
    if ((what == 0 || what == 3) && threadIdx.x == 0 && done) *done = any ? 0 : 1;
}

// ------------------------------------------------------------ GMRES steps
//
// Right-preconditioned restarted GMRES on nrhs independent systems.  Basis
// vectors are stored as V[l][r][i] (l = basis index, r = right-hand side), so
// the l-th vectors of all systems form one column-major n x nrhs block.
struct GmLane {
    double bb, est;
    int32_t its, kc, active, conv, dead, pad;  // kc: steps taken in the current cycle
};

// part[(l * nchunk + chunk) * nrhs + r] = V[l][r] . w[r] over the chunk's rows.
// Grid (nchunk, ceil(ncols / kGmGroup), nrhs): a workgroup takes kGmGroup basis
// vectors of one right-hand side, so w is read once per group instead of once
// per basis vector; per (l, chunk, r) the terms and the reduction tree are
// those of one vector at a time.
constexpr int kGmGroup = 8;
__global__ __launch_bounds__(256) void k_gm_dots(int64_t n, int nrhs, int ncols, const double* __restrict__ V,
                                                 const double* __restrict__ w, double* __restrict__ part,
                                                 const int* __restrict__ done) {
    __shared__ double sh[4][kGmGroup];
    if (done && *done) return;
    const int chunk = blockIdx.x, nchunk = gridDim.x;
    const int l0 = blockIdx.y * kGmGroup, r = blockIdx.z;
    const int ng = min(kGmGroup, ncols - l0);
    double acc[kGmGroup];
#pragma unroll
    for (int g = 0; g < kGmGroup; ++g) acc[g] = 0.0;
    const double* wr = w + (int64_t)r * n;
    for (int64_t i = (int64_t)chunk * blockDim.x + threadIdx.x; i < n; i += (int64_t)nchunk * blockDim.x) {
        // all of the row's loads first (basis indices past the group clamped,
        // their sums unused), then the adds in basis order
        const double wi = wr[i];
        double vv[kGmGroup];
#pragma unroll
        for (int g = 0; g < kGmGroup; ++g) vv[g] = V[((int64_t)(l0 + min(g, ng - 1)) * nrhs + r) * n + i];
#pragma unroll
        for (int g = 0; g < kGmGroup; ++g) acc[g] += vv[g] * wi;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int g = 0; g < kGmGroup; ++g) {
        const double v = wave_sum(acc[g]);
        if (lane == 0) sh[wv][g] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < ng) {
        const int g = threadIdx.x;
        part[((int64_t)(l0 + g) * nchunk + chunk) * nrhs + r] = (sh[0][g] + sh[1][g]) + (sh[2][g] + sh[3][g]);
    }
}

// coef[r][l] = sum over chunks; H column j of lane r accumulates coef (two
// Gram-Schmidt passes add up to the Hessenberg entries).  One wave per (r, l):
// lane c sums chunks c, c + 64, ..., then a fixed shuffle tree; grid
// ceil(nrhs * ncols / 4) workgroups of 256 threads.
__global__ __launch_bounds__(256) void k_gm_coef(int nchunk, int nrhs, int ncols, int m, int j,
                                                 const double* __restrict__ part, double* __restrict__ coef,
                                                 double* __restrict__ H, const GmLane* __restrict__ L,
                                                 const int* __restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= nrhs * ncols) return;  // uniform across the wave
    const int r = q / ncols, l = q - r * ncols;
    double s = 0.0;
    for (int c = lane; c < nchunk; c += 64) s += part[((int64_t)l * nchunk + c) * nrhs + r];
    s = wave_sum(s);
    if (lane == 0) {
        const bool act = L[r].active;
        coef[r * ncols + l] = act ? s : 0.0;
        if (act) H[((int64_t)r * m + j) * (m + 1) + l] += s;
    }
}

// w[r] -= sum_l V[l][r] coef[r][l]
__global__ __launch_bounds__(256) void k_gm_sub(int64_t n, int nrhs, int ncols, const double* __restrict__ V,
                                                const double* __restrict__ coef, double* __restrict__ w,
                                                const int* __restrict__ done) {
    __shared__ double cf[kMaxRhs * 64];
    if (done && *done) return;
    for (int q = threadIdx.x; q < nrhs * ncols; q += blockDim.x) cf[q] = coef[q];
    __syncthreads();
    const int64_t r = blockIdx.y;  // grid (row chunks, nrhs)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = w[r * n + i];
        for (int l = 0; l < ncols; ++l) v -= V[((int64_t)l * nrhs + r) * n + i] * cf[r * ncols + l];
        w[r * n + i] = v;
    }
}

// Step j of every active lane: h_{j+1,j} = ||w||, previous rotations applied
// to column j, a new rotation, the residual estimate |g_{j+1}|, stopping test.
__global__ void k_gm_givens(int j, int nrhs, int m, const double* __restrict__ wn2, double* __restrict__ H,
                            double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                            double* __restrict__ inv, GmLane* __restrict__ L, double tol2, int maxit,
                            int* __restrict__ done) {
    if (done && *done) return;
    const int r = threadIdx.x;
    if (r < nrhs) {
        GmLane& l = L[r];
        inv[r] = 0.0;
        if (l.active) {
            double* h = H + ((int64_t)r * m + j) * (m + 1);
            double* c = cs + (int64_t)r * m;
            double* s = sn + (int64_t)r * m;
            double* gg = g + (int64_t)r * (m + 1);
            const double hn = sqrt(wn2[r]);
            h[j + 1] = hn;
            inv[r] = hn > 0.0 ? 1.0 / hn : 0.0;
            for (int q = 0; q < j; ++q) {
                const double t0 = c[q] * h[q] + s[q] * h[q + 1];
                const double t1 = -s[q] * h[q] + c[q] * h[q + 1];
                h[q] = t0;
                h[q + 1] = t1;
            }
            const double den = sqrt(h[j] * h[j] + h[j + 1] * h[j + 1]);
            c[j] = den > 0.0 ? h[j] / den : 1.0;
            s[j] = den > 0.0 ? h[j + 1] / den : 0.0;
            h[j] = den;
            h[j + 1] = 0.0;
            gg[j + 1] = -s[j] * gg[j];
            gg[j] = c[j] * gg[j];
            l.its += 1;
            l.kc = j + 1;
            l.est = fabs(gg[j + 1]);
            const bool conv = l.est * l.est <= tol2 * l.bb;
            if (conv) l.conv = 1;
            if (conv || l.its >= maxit || j + 1 == m || hn == 0.0) l.active = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && done) {
        int any = 0;
        for (int q = 0; q < nrhs; ++q) any |= L[q].active;
        *done = any ? 0 : 1;
    }
}

// V[j+1][r] = w[r] * inv[r]
__global__ __launch_bounds__(256) void k_gm_scale(int64_t n, int nrhs, const double* __restrict__ w,
                                                  const double* __restrict__ inv, double* __restrict__ Vn) {
    const int64_t r = blockIdx.y;  // grid (row chunks, nrhs)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        Vn[r * n + i] = w[r * n + i] * inv[r];
}

// Cycle start: beta_r = ||r_r||; lanes that converged or ran out of steps are
// retired, the others open a cycle with g = beta e_1 and V[0] = r / beta.
__global__ void k_gm_start(int nrhs, int m, const double* __restrict__ rn2, double* __restrict__ g,
                           double* __restrict__ H, double* __restrict__ inv, GmLane* __restrict__ L, double tol2,
                           int maxit, int first, int* __restrict__ any_active) {
    const int r = threadIdx.x;
    if (r < nrhs) {
        GmLane& l = L[r];
        const double b2 = rn2[r];
        if (first) {
            l.bb = b2;
            l.its = 0;
            l.conv = 0;
            l.dead = 0;
            l.est = sqrt(b2);
        }
        l.kc = 0;
        l.active = 0;
        inv[r] = 0.0;
        if (!l.dead) {
            if (b2 <= tol2 * l.bb) {
                l.conv = 1;
                l.dead = 1;
                l.est = sqrt(b2);
            } else if (l.its >= maxit) {
                l.dead = 1;
            } else {
                l.active = 1;
                const double beta = sqrt(b2);
                inv[r] = 1.0 / beta;
                double* gg = g + (int64_t)r * (m + 1);
                for (int q = 0; q <= m; ++q) gg[q] = 0.0;
                gg[0] = beta;
                double* h = H + (int64_t)r * m * (m + 1);
                for (int q = 0; q < m * (m + 1); ++q) h[q] = 0.0;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int any = 0;
        for (int q = 0; q < nrhs; ++q) any |= L[q].active;
        *any_active = any;
    }
}

// y = H^{-1} g (upper triangular, kc x kc) per lane
__global__ void k_gm_solve(int nrhs, int m, const double* __restrict__ H, const double* __restrict__ g,
                           double* __restrict__ y, const GmLane* __restrict__ L) {
    const int r = threadIdx.x;
    if (r >= nrhs) return;
    const int kc = L[r].kc;
    const double* h = H + (int64_t)r * m * (m + 1);
    const double* gg = g + (int64_t)r * (m + 1);
    double* yy = y + (int64_t)r * m;
    for (int q = 0; q < m; ++q) yy[q] = 0.0;
    for (int i = kc - 1; i >= 0; --i) {
        double v = gg[i];
        for (int q = i + 1; q < kc; ++q) v -= h[(int64_t)q * (m + 1) + i] * yy[q];
        yy[i] = v / h[(int64_t)i * (m + 1) + i];
    }
}

// u[r] = sum_{l < kc_r} V[l][r] y[r][l]
__global__ __launch_bounds__(256) void k_gm_combine(int64_t n, int nrhs, int m, const double* __restrict__ V,
                                                    const double* __restrict__ y, const GmLane* __restrict__ L,
                                                    double* __restrict__ u) {
    const int64_t r = blockIdx.y;  // grid (row chunks, nrhs)
    const int kc = L[r].kc;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int l = 0; l < kc; ++l) v += V[((int64_t)l * nrhs + r) * n + i] * y[r * m + l];
        u[r * n + i] = v;
    }
}

// done := !done (turns the "any lane active" result of k_gm_start into the
// early-exit flag of the step kernels)
__global__ void k_flag_not(int* __restrict__ f) { *f = *f ? 0 : 1; }

// GMRES lane state -> the solve report (rr = est^2, active = converged flag)
__global__ void k_gm_report(int nrhs, const GmLane* __restrict__ G, CgLane* __restrict__ L) {
    const int r = threadIdx.x;
    if (r < nrhs) {
        L[r].bb = G[r].bb;
        L[r].rr = G[r].est * G[r].est;
        L[r].its = G[r].its;
        L[r].active = G[r].conv;
    }
}

// x[r] += z[r] for lanes that took steps in this cycle
__global__ __launch_bounds__(256) void k_gm_xupdate(int64_t n, int nrhs, const GmLane* __restrict__ L,
                                                    const double* __restrict__ z, double* __restrict__ x) {
    const int64_t r = blockIdx.y;  // grid (row chunks, nrhs)
    if (L[r].kc <= 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[r * n + i] += z[r * n + i];
}

// ------------------------------------------------------------ Lanczos steps
//
// Q holds the Lanczos vectors as columns (s x (m+1), column-major, ld s).
// coeffs: c_l = q_l . w for l <= j, as per-block partials part[block][l]
__global__ __launch_bounds__(256) void k_multidot(int64_t s, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                  const double* __restrict__ w, double* __restrict__ part,
                                                  const int* __restrict__ skip) {
    __shared__ double sh[4];
    if (skip && *skip) return;
    for (int l = 0; l < ncols; ++l) {
        double acc = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s; i += (int64_t)gridDim.x * blockDim.x)
            acc += Q[i + l * ldq] * w[i];
        const double t = block_sum256(acc, sh);
        if (threadIdx.x == 0) part[blockIdx.x * ncols + l] = t;
    }
}

// w -= Q c  (columns 0..ncols-1, ncols <= 1024: the coefficients are staged in LDS)
__global__ __launch_bounds__(256) void k_gemv_sub(int64_t s, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                  const double* __restrict__ c, double* __restrict__ w,
                                                  const int* __restrict__ skip) {
    __shared__ double cs[1024];
    if (skip && *skip) return;
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

// Partial reorthogonalisation bookkeeping of Lanczos step j (Simon's omega
// recurrence; the new vector is w with norm *b0 before any reorthogonalisation):
// for i < j
//   om_new_i = (beta_i om_cur_{i+1} + (alpha_i - alpha_j) om_cur_i
//               + beta_{i-1} om_cur_{i-1} - beta_{j-1} om_prev_i + theta) / b0,
// theta = 2 eps ||T||_est carrying the sign of the rest (eps = 2^-52; ||T||_est
// the running max of |alpha_i| + beta_i + beta_{i-1}, kept in *tnorm);
// om_new_j = eps sqrt(s), om_new_{j+1} = 1.  The step is reorthogonalised
// (state[1] = 0) when some |om_new_i|, i <= j, exceeds sqrt(eps) or the
// previous step was (state[0]); its estimates are then reset to eps.
// state[0]: force the next step; state[1]: 1 = skip the reorthogonalisation;
// flags[j]: 1 if step j was reorthogonalised.  One workgroup of 1024 threads,
// j + 2 <= 1024.  A breakdown (b0 <= 1e-12 max|alpha|) skips and leaves the
// estimates alone.
__global__ __launch_bounds__(1024) void k_pro_omega(int j, int64_t s, const double* __restrict__ alpha,
                                                    const double* __restrict__ beta, const double* __restrict__ b0p,
                                                    const double* __restrict__ amax, const double* __restrict__ om_prev,
                                                    const double* __restrict__ om_cur, double* __restrict__ om_new,
                                                    double* __restrict__ tnorm, int* __restrict__ state,
                                                    int* __restrict__ flags) {
    __shared__ double red[16];
    __shared__ int need;
    const double eps = 2.220446049250313e-16;
    const double b0 = *b0p, aj = alpha[j], bprev = j > 0 ? beta[j - 1] : 0.0;
    if (!(b0 > 1e-12 * (*amax))) {
        if (threadIdx.x == 0) {
            state[1] = 1;
            flags[j] = 0;
        }
        return;
    }
    const double tn = fmax(*tnorm, fabs(aj) + b0 + bprev);
    const int i = threadIdx.x;
    double v = 0.0;
    if (i < j) {
        double t = beta[i] * om_cur[i + 1] + (alpha[i] - aj) * om_cur[i];
        if (i > 0) t += beta[i - 1] * om_cur[i - 1];
        t -= bprev * om_prev[i];
        t += (t >= 0.0 ? 1.0 : -1.0) * 2.0 * eps * tn;
        v = t / b0;
        om_new[i] = v;
    }
    double big = fabs(v);
    for (int off = 32; off > 0; off >>= 1) big = fmax(big, __shfl_down(big, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = big;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double psi = eps * sqrt((double)s);
        double m = psi;
        for (int w = 0; w < 16; ++w) m = fmax(m, red[w]);
        const int forced = state[0];
        need = forced || m > sqrt(eps);
        om_new[j] = psi;
        om_new[j + 1] = 1.0;
        *tnorm = tn;
        state[0] = need ? (forced ? 0 : 1) : 0;
        state[1] = need ? 0 : 1;
        flags[j] = need;
    }
    __syncthreads();
    if (need && i <= j) om_new[i] = eps;
}

// dst = reduced sum; beta form: dst = sqrt(sum), inv = dst > 1e-12 max|alpha| ? 1/dst : 0;
// nothing when *skip is set
__global__ void k_lanczos_scalar(const double* __restrict__ sum, double* __restrict__ dst, int sqrt_it,
                                 double* __restrict__ amax, double* __restrict__ inv, const int* __restrict__ skip) {
    if (threadIdx.x == 0 && !(skip && *skip)) {
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

// y -= (*c) x  (a scalar kept on the device)
__global__ __launch_bounds__(256) void k_sub_scaled(int64_t len, const double* __restrict__ c,
                                                    const double* __restrict__ x, double* __restrict__ y) {
    const double f = *c;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        y[i] -= f * x[i];
}

// Bidiagonalisation norms: dst = sqrt(sum); with grow, amax = max(amax, dst);
// inv = dst > 1e-12 amax ? 1 / dst : 0 (a breakdown leaves zero vectors)
__global__ void k_gk_norm(const double* __restrict__ sum, double* __restrict__ dst, int grow,
                          double* __restrict__ amax, double* __restrict__ inv) {
    if (threadIdx.x == 0) {
        const double v = sqrt(*sum);
        *dst = v;
        if (grow && v > *amax) *amax = v;
        *inv = (v > 1e-12 * (*amax)) ? 1.0 / v : 0.0;
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
