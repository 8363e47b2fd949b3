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
//     with D^{-1}, each level's entries in a slot-major ELL copy and the next
//     level's loaded while the current one is computed; the solve vector
//     stays in LDS when the system fits, else in a global buffer of the lane;
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

// One workgroup's share of a system.  A system is solved by G >= 1 workgroups
// (a group).  For the A0 solves the first min(G, p) members own contiguous
// ranges of the system's blocks, rows r0 + o0 .. r0 + o1 - 1, the last of them
// also the interface block (whose rows come last) and the interface step of
// the correction; members beyond own no block.  The vector steps of CG (the
// SpMV, the dot products, the updates) split the rows evenly over all G
// members instead: rows r0 + v0 .. r0 + v1 - 1.  G = 1: the whole system.
struct PSys {
    int64_t r0;      // first device row of the system
    int64_t s0;      // first interface position (rows of U_k, y, w)
    int64_t d0;      // offset of d_1..d_k in the coefficient array
    int32_t n, m;    // rows; interior rows (the interface rows follow)
    int32_t s, k;    // interface rows; rank of the correction (0: A0 alone)
    int32_t l0, l1;  // the member's merged levels l0..l1-1 (metadata meta[j], row lists in mrow)
    int32_t lds;     // 1: the member's solve vector fits the dynamic LDS
    int32_t pad;
    double c0;       // eq. (gkt): G^{-1} = c0 I + U_k diag(d) U_k^T
    int32_t o0, o1;  // the member's block rows (A0 solve), as offsets from r0
    int32_t G, g;    // members of the group; this member's index
    int32_t grp;     // group index (barrier counters and partial sums; -1 when G = 1)
    int32_t ifc;     // 1: the member owns the interface block
    int32_t v0, v1;  // the member's rows of the vector steps, as offsets from r0
};

struct PLane {
    int32_t sys;  // index into the system table
    int32_t col;  // column of the lane in the vectors (offset col * ld)
};

struct PRes {
    int32_t its, status;  // iterations; 0 converged, 1 maxit reached
    double rr, bb;        // ||r||^2 (recursive) and ||b||^2
    double rtrue;         // ||b - A x||^2 after the solve
    int64_t ticks;        // the lane's time in the launch, device wall-clock ticks
};

constexpr int kPersistMaxK = 64;  // rank bound of the persistent form
constexpr int kGroupMax = 32;     // members of a group at most

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

// Per merged level j: meta[j] = {first entry of its rows in mrow, forward width
// | backward width << 16, start of its forward ELL entries, start of its
// backward ones}; meta[j + 1].x ends the row list.  ELL entries of a level with
// nr rows are stored slot-major (entry u of row r at base + u * nr + r); a row
// shorter than the level's width is padded with its own index and weight 0.
// The solve vector is zeroed before the first sweep, so a padded term adds 0
// times a finite value (the row sum keeps its value; its terms keep their
// CSR order).
constexpr int kPersistKW = 4;  // entries per row held in registers one level ahead

template <typename T> struct PLev {
    int nr, fw, i;
    T in;  // forward: input x_i; backward: D_i^{-1}
    int c[kPersistKW];
    T v[kPersistKW];
};

// Loads the first row (threadIdx.x, clamped) of merged level j into registers.
// kBwd selects the backward entries; inq holds the forward input or D^{-1}
// in merged-level order.
template <typename T, bool kBwd>
__device__ __forceinline__ void plev_load(PLev<T>& L, int j, const int4* __restrict__ meta,
                                          const int32_t* __restrict__ mrow, const int32_t* __restrict__ ecol,
                                          const T* __restrict__ eval, const T* inq) {
    const int4 m = meta[j];
    const int a = __builtin_amdgcn_readfirstlane(m.x);
    L.nr = __builtin_amdgcn_readfirstlane(meta[j + 1].x) - a;
    L.fw = __builtin_amdgcn_readfirstlane(kBwd ? (m.y >> 16) : (m.y & 0xffff));
    const int base = __builtin_amdgcn_readfirstlane(kBwd ? m.w : m.z);
    const int r = min((int)threadIdx.x, L.nr - 1);
    L.i = mrow[a + r];
    L.in = inq[a + r];  // input or D^{-1}, stored in merged-level order: no load waits for another
#pragma unroll
    for (int u = 0; u < kPersistKW; ++u) {
        const int q = base + min(u, max(L.fw, 1) - 1) * L.nr + r;  // clamped: every load in bounds
        const int c = ecol[q];
        const T v = eval[q];
        L.c[u] = u < L.fw ? c : L.i;
        L.v[u] = u < L.fw ? v : T(0);
    }
}

// Row sums of merged level j: the prefetched first row of each thread, then
// the rows beyond the first NT (loaded here), entries beyond kPersistKW too.
template <typename T, int NT, bool kBwd>
__device__ __forceinline__ void plev_step(const PLev<T>& L, int j, int64_t off, const int4* __restrict__ meta,
                                          const int32_t* __restrict__ mrow, const int32_t* __restrict__ ecol,
                                          const T* __restrict__ eval, const T* inq, T* vec) {
    const int nr = L.nr;
    if ((int)threadIdx.x < nr) {
        T s = kBwd ? vec[L.i - off] * L.in : L.in;
#pragma unroll
        for (int u = 0; u < kPersistKW; ++u) s = fnms(s, L.v[u], vec[L.c[u] - off]);
        if (L.fw > kPersistKW) {
            const int4 m = meta[j];
            const int base = kBwd ? m.w : m.z;
            for (int u = kPersistKW; u < L.fw; ++u) {
                const int q = base + u * nr + (int)threadIdx.x;
                s = fnms(s, eval[q], vec[ecol[q] - off]);
            }
        }
        vec[L.i - off] = s;
    }
    if (nr > NT) {
        const int4 m = meta[j];
        const int base = kBwd ? m.w : m.z;
        for (int r = NT + (int)threadIdx.x; r < nr; r += NT) {
            const int i = mrow[m.x + r];
            T s = kBwd ? vec[i - off] * inq[m.x + r] : inq[m.x + r];
            for (int u = 0; u < L.fw; ++u) {
                const int q = base + u * nr + r;
                s = fnms(s, eval[q], vec[ecol[q] - off]);
            }
            vec[i - off] = s;
        }
    }
}

// Barrier between two levels.  With the solve vector in LDS only LDS traffic
// must be complete (the next level's global loads stay in flight across it);
// with the solve vector in global memory a full workgroup fence.
template <bool kLds> __device__ __forceinline__ void level_barrier() {
    if constexpr (kLds) lds_barrier();
    else __syncthreads();
}

// Levels in flight: the next kPersistDepth - 1 levels' first rows are loaded
// while the current level is computed, so a global load has that many level
// steps to arrive.
template <typename T> struct PersistDepth { static constexpr int value = sizeof(T) == 4 ? 5 : 4; };

// One sweep over merged levels l0..l1-1 (forward ascending, backward
// descending).  As in the block triangular-solve kernels, the steady state
// runs behind an unconditional prologue (every load of a group is issued on
// the single path into its use, so the compiler's load-counter waits leave
// the newer levels' loads in flight); a conditional tail finishes.
template <typename T, int NT, bool kBwd, bool kLds>
__device__ __forceinline__ void plev_sweep(int l0, int l1, int64_t off, const int4* __restrict__ meta,
                                           const int32_t* __restrict__ mrow, const int32_t* __restrict__ ecol,
                                           const T* __restrict__ eval, const T* inq, T* vec) {
    constexpr int kD = PersistDepth<T>::value;
    const int nl = l1 - l0;
    if (nl <= 0) return;
    auto lev = [&](int q) { return kBwd ? l1 - 1 - q : l0 + q; };
    PLev<T> buf[kD];
    int q0 = 0;
    if (nl >= 2 * kD - 1) {
#pragma unroll
        for (int u = 0; u < kD - 1; ++u) plev_load<T, kBwd>(buf[u], lev(u), meta, mrow, ecol, eval, inq);
        for (; q0 + 2 * kD - 1 <= nl; q0 += kD) {
#pragma unroll
            for (int u = 0; u < kD; ++u) {
                plev_load<T, kBwd>(buf[(u + kD - 1) % kD], lev(q0 + u + kD - 1), meta, mrow, ecol, eval, inq);
                plev_step<T, NT, kBwd>(buf[u], lev(q0 + u), off, meta, mrow, ecol, eval, inq, vec);
                level_barrier<kLds>();
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < kD - 1; ++u)
            if (u < nl) plev_load<T, kBwd>(buf[u], lev(u), meta, mrow, ecol, eval, inq);
    }
    for (; q0 < nl; q0 += kD) {
#pragma unroll
        for (int u = 0; u < kD; ++u) {
            const int q = q0 + u;
            if (q < nl) {
                if (q + kD - 1 < nl)
                    plev_load<T, kBwd>(buf[(u + kD - 1) % kD], lev(q + kD - 1), meta, mrow, ecol, eval, inq);
                plev_step<T, NT, kBwd>(buf[u], lev(q), off, meta, mrow, ecol, eval, inq, vec);
                level_barrier<kLds>();
            }
        }
    }
}

// The A0 solve of one lane: forward sweep over the merged levels (unit lower L),
// then backward (z_i = D_i^{-1} y_i - sum_j L_ji z_j).  xq: the input and dq:
// D^{-1}, both in merged-level order; vec: the solve vector, indexed by local
// row (LDS) or by global row.
template <typename T, int NT, bool kLds>
__device__ __forceinline__ void wg_a0_solve(const PSys& S, const int4* __restrict__ meta, const int32_t* __restrict__ mrow,
                            const int32_t* __restrict__ fcol, const T* __restrict__ fval,
                            const int32_t* __restrict__ bcol, const T* __restrict__ bval, const T* __restrict__ dq,
                            const T* xq, T* vec) {
    const int64_t off = kLds ? S.r0 : 0;
    plev_sweep<T, NT, false, kLds>(S.l0, S.l1, off, meta, mrow, fcol, fval, xq, vec);
    plev_sweep<T, NT, true, kLds>(S.l0, S.l1, off, meta, mrow, bcol, bval, dq, vec);
    if constexpr (kLds) __syncthreads();  // the callers' next phases read and write global memory
}

// z = M^{-1} r for one lane (r, z: double at global device rows; tg: the lane's
// global T buffer of n rows used when the solve vector is not in LDS; y, w: the
// lane's interface vectors).  Ends with a barrier.
template <typename T, int NT, bool kLds>
__device__ __forceinline__ void wg_apply(const PSys& S, const int4* __restrict__ meta, const int32_t* __restrict__ mrow,
                         const int32_t* __restrict__ fcol, const T* __restrict__ fval,
                         const int32_t* __restrict__ bcol, const T* __restrict__ bval, const T* __restrict__ dq,
                         const int32_t* __restrict__ erp, const int32_t* __restrict__ eci,
                         const T* __restrict__ ev, const int32_t* __restrict__ etrp, const int32_t* __restrict__ etci,
                         const T* __restrict__ etv, const T* __restrict__ U, int ustride,
                         const double* __restrict__ dcoef, const double* __restrict__ r, double* __restrict__ z, T* tg,
                         T* tq, T* y, T* w, T* lvec, double* red, double* coef) {
    T* vec = kLds ? lvec : tg;
    const int64_t off = kLds ? S.r0 : 0;
    const int64_t r0 = S.r0, r1 = S.r0 + S.n;
    const int q0 = meta[S.l0].x, q1 = meta[S.l1].x;  // the system's rows in merged-level order
    // the first solve's input in merged-level order
#pragma unroll 4
    for (int q = q0 + (int)threadIdx.x; q < q1; q += NT) tq[q] = (T)r[mrow[q]];
    __syncthreads();
    wg_a0_solve<T, NT, kLds>(S, meta, mrow, fcol, fval, bcol, bval, dq, tq, vec);
    if (S.k > 0) {
        const int64_t s0 = S.s0, s1 = S.s0 + S.s;
        // y = E^T z1 over the lane's interface positions (terms in CSR order, one rounding each)
#pragma unroll 4
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
#pragma unroll 4
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
#pragma unroll 4
        for (int64_t ig = s0 + threadIdx.x; ig < s1; ig += NT) {
            double acc = S.c0 * (double)y[ig];
            const T* Ui = U + ig * ustride;
            for (int j = 0; j < S.k; ++j) acc += (double)Ui[j] * coef[j];
            w[ig] = (T)acc;
        }
        __syncthreads();
        // v = r + E w, the second solve's input, in merged-level order
#pragma unroll 4
        for (int q = q0 + (int)threadIdx.x; q < q1; q += NT) {
            const int i = mrow[q];
            T acc = (T)r[i];
            const int t1 = erp[i + 1];
            for (int t = erp[i]; t < t1; ++t) acc = fnms(acc, -ev[t], w[eci[t]]);
            tq[q] = acc;
        }
        __syncthreads();
        wg_a0_solve<T, NT, kLds>(S, meta, mrow, fcol, fval, bcol, bval, dq, tq, vec);
    }
#pragma unroll 4
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) z[i] = (double)vec[i - off];
    __syncthreads();
}


// ------------------------------------------------ groups of workgroups
//
// A large system is shared by the G workgroups of a group (its blocks are
// independent in the A0 solve, so each member sweeps its own blocks' merged
// levels); dot products, the interface step of the correction and the
// exchange of p and z1 need the group to meet.  A launch holds at most as
// many workgroups as the device keeps resident (the host checks), so every
// member of a group runs at once.
//
// Barrier: every thread waits until its stores are acknowledged by the L2 of
// its XCD; one wave announces the arrival and waits for the group, then
// invalidates the CU's L1 (and non-coherent L2 lines) before the members read
// each other's data.
//   slow form (any placement): that wave first writes the XCD's L2 back to
//     memory; arrival is a device-scope atomic, polled with device-scope loads;
//   fast form (every member on one XCD, checked once at start): the L2 is
//     shared, so no write-back; arrival and polling are L2 atomics.
// A wait gives up after kSpinMax polls (or the launch's smaller limit) and the
// lane reports failure (status 2): no member waits without bound.  Values other members wrote are read
// with lane-dependent addresses (vector loads through the invalidated L1),
// never through the scalar cache.

constexpr unsigned kSpinMax = 1u << 22;

__global__ void k_zero_u32(int64_t n, unsigned* __restrict__ p) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__device__ __forceinline__ int xcc_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return (int)(v & 0xf);
}

// A group member's barrier state, in LDS (thread 0 updates it).
struct GroupLds {
    int flag;         // 1 once a wait of this workgroup gave up
    int fast;         // 1: the fast form (decided once, the same in every member)
    unsigned n_slow;  // arrivals counted by the last barrier of each form
    unsigned n_fast;
    unsigned spin;    // polls before a wait gives up
};

// ctr: the group's 64 counters (slow form at 0, fast form at 32, zero at launch).
__device__ __forceinline__ bool group_barrier(unsigned* ctr, int G, GroupLds* gl) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x < 64) {
        const bool fast = gl->fast != 0;
        if (!fast) asm volatile("buffer_wbl2 sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
        if (threadIdx.x == 0) {
            unsigned* c = fast ? ctr + 32 : ctr;
            const unsigned target = fast ? (gl->n_fast += (unsigned)G) : (gl->n_slow += (unsigned)G);
            if (fast) __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else asm volatile("global_atomic_add %0, %1, off sc1\n\ts_waitcnt vmcnt(0)" ::"v"(c), "v"(1u) : "memory");
            unsigned spins = 0;
            for (;;) {
                unsigned v;
                if (fast) {
                    v = 0u;  // compare-and-swap 0 -> 0: an L2 read of the counter that changes nothing
                    __hip_atomic_compare_exchange_strong(c, &v, 0u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    v = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (v >= target) break;
                __builtin_amdgcn_s_sleep(2);
                if (++spins > gl->spin) {
                    gl->flag = 1;
                    break;
                }
            }
        }
        asm volatile("buffer_inv sc1" ::: "memory");
    }
    __syncthreads();
    return gl->flag == 0;
}

// The G values slots[0..G) (written by the members before a barrier), added
// in member order; the same total in every thread.
__device__ __forceinline__ double group_add(const double* slots, int G) {
    const int ln = (int)(threadIdx.x & 63);
    const double mine = ln < G ? slots[ln] : 0.0;
    double s = 0.0;
    for (int u = 0; u < G; ++u) s += __shfl(mine, u);
    return s;
}

// Sum over the group of every thread's v: the workgroup's sum into slot g,
// a barrier, then the slots in member order (0 if the wait gave up: the
// caller checks gl->flag).
template <int NT>
__device__ __forceinline__ double group_sum(double v, double* red, double* slots, unsigned* ctr, int G, int g,
                                            GroupLds* gl) {
    const double mine = wg_sum<NT>(v, red);
    if (threadIdx.x == 0) slots[g] = mine;
    if (!group_barrier(ctr, G, gl)) return 0.0;
    return group_add(slots, G);
}

// z = M^{-1} r on the member's rows (see wg_apply; here the first solve's
// result z1 is also written to tg for the interface member, which forms y,
// the coefficients and w alone between two barriers).  R0: the member's
// first row (the solve vector's offset in LDS).  Returns false if a wait gave
// up.
template <typename T, int NT, bool kLds>
__device__ __forceinline__ bool member_apply(const PSys& S, int64_t R0, unsigned* ctr, GroupLds* gl,
                                             const int4* __restrict__ meta,
                             const int32_t* __restrict__ mrow, const int32_t* __restrict__ fcol,
                             const T* __restrict__ fval, const int32_t* __restrict__ bcol, const T* __restrict__ bval,
                             const T* __restrict__ dq, const int32_t* __restrict__ erp, const int32_t* __restrict__ eci,
                             const T* __restrict__ ev, const int32_t* __restrict__ etrp,
                             const int32_t* __restrict__ etci, const T* __restrict__ etv, const T* __restrict__ U,
                             int ustride, const double* __restrict__ dcoef, const double* r, double* z, T* tg, T* tq,
                             T* y, T* w, T* lvec, double* red, double* coef) {
    T* vec = kLds ? lvec : tg;
    const int64_t R1 = S.r0 + S.o1;
    const int64_t off = kLds ? R0 : 0;
    const int q0 = meta[S.l0].x, q1 = meta[S.l1].x;
#pragma unroll 4
    for (int q = q0 + (int)threadIdx.x; q < q1; q += NT) tq[q] = (T)r[mrow[q]];
    __syncthreads();
    plev_sweep<T, NT, false, kLds>(S.l0, S.l1, off, meta, mrow, fcol, fval, tq, vec);
    plev_sweep<T, NT, true, kLds>(S.l0, S.l1, off, meta, mrow, bcol, bval, dq, vec);
    if constexpr (kLds) __syncthreads();
    if (S.k > 0) {
        if constexpr (kLds) {
#pragma unroll 4
            for (int64_t i = R0 + threadIdx.x; i < R1; i += NT) tg[i] = vec[i - R0];
        }
        if (!group_barrier(ctr, S.G, gl)) return false;
        if (S.ifc) {
            const int64_t s0 = S.s0, s1 = S.s0 + S.s;
#pragma unroll 4
            for (int64_t jg = s0 + threadIdx.x; jg < s1; jg += NT) {
                T acc = T(0);
                const int t1 = etrp[jg + 1];
                for (int t = etrp[jg]; t < t1; ++t) acc = fnms(acc, -etv[t], tg[etci[t]]);
                y[jg] = acc;
            }
            __syncthreads();
            constexpr int NW = NT / 64;
            for (int j0 = 0; j0 < S.k; j0 += 16) {
                double acc[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) acc[u] = 0.0;
#pragma unroll 4
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
#pragma unroll 4
            for (int64_t ig = s0 + threadIdx.x; ig < s1; ig += NT) {
                double acc = S.c0 * (double)y[ig];
                const T* Ui = U + ig * ustride;
                for (int j = 0; j < S.k; ++j) acc += (double)Ui[j] * coef[j];
                w[ig] = (T)acc;
            }
        }
        if (!group_barrier(ctr, S.G, gl)) return false;
#pragma unroll 4
        for (int q = q0 + (int)threadIdx.x; q < q1; q += NT) {
            const int i = mrow[q];
            T acc = (T)r[i];
            const int t1 = erp[i + 1];
            for (int t = erp[i]; t < t1; ++t) acc = fnms(acc, -ev[t], w[eci[t]]);
            tq[q] = acc;
        }
        __syncthreads();
        plev_sweep<T, NT, false, kLds>(S.l0, S.l1, off, meta, mrow, fcol, fval, tq, vec);
        plev_sweep<T, NT, true, kLds>(S.l0, S.l1, off, meta, mrow, bcol, bval, dq, vec);
        if constexpr (kLds) __syncthreads();
    }
#pragma unroll 4
    for (int64_t i = R0 + threadIdx.x; i < R1; i += NT) z[i] = (double)vec[i - off];
    __syncthreads();
    return true;
}

// A row of A times y: s + sum_t av[t] y[aci[t]] over t in [t0, t1), the
// products added in order of t.  grouped: the entries go in groups of
// kTermGroup whose column, value and gather loads go out together (an index
// past the row's end repeats its last entry and is not added); else one by
// one.  The grouped form pays on large systems, whose gathers miss the caches
// (a batch of 256 systems of 1 k to 65 k rows: 336 ms when the systems from
// 16 k rows take it, 339 ms when all do, 358 ms when none does); on a small
// system the vector stays in cache and the loads of the padding slots cost
// more than the overlap saves (4,096 rows on 512 threads: 134 against 122 us
// per iteration).  Both give the same sums.
__device__ __forceinline__ bool csr_grouped(int64_t n) { return n >= 16384; }

__device__ __forceinline__ double csr_row_dot(double s, int64_t t0, int64_t t1, const int32_t* __restrict__ aci,
                                              const double* __restrict__ av, const double* y, bool grouped) {
    if (!grouped) {
        for (int64_t t = t0; t < t1; ++t) s += av[t] * y[aci[t]];
        return s;
    }
    for (int64_t t = t0; t < t1; t += kTermGroup) {
        int c[kTermGroup];
        double v[kTermGroup], g[kTermGroup];
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u) {
            const int64_t q = t + u < t1 ? t + u : t1 - 1;
            c[u] = aci[q];
            v[u] = av[q];
        }
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u) g[u] = y[c[u]];
#pragma unroll
        for (int u = 0; u < kTermGroup; ++u)
            if (t + u < t1) s += v[u] * g[u];
    }
    return s;
}

// The PCG of k_pcg_persist for one member of a group (S.G > 1): the same
// steps on the member's rows, every scalar summed over the group.
template <typename T, int NT>
__device__ __forceinline__ void member_pcg(const PSys& S, const int64_t* __restrict__ arp, const int32_t* __restrict__ aci,
                           const double* __restrict__ av, const int4* meta, const int32_t* __restrict__ mrow,
                           const int32_t* __restrict__ fcol, const T* __restrict__ fval,
                           const int32_t* __restrict__ bcol, const T* __restrict__ bval, const T* __restrict__ dq,
                           const int32_t* __restrict__ erp, const int32_t* __restrict__ eci, const T* __restrict__ ev,
                           const int32_t* __restrict__ etrp, const int32_t* __restrict__ etci,
                           const T* __restrict__ etv, const T* __restrict__ U, int ustride,
                           const double* __restrict__ dcoef, const double* b, double* x, double* r, double* p,
                           double* q, double* z, T* tg, T* tq, T* yv, T* wv, T* lvec, double* red, double* coef,
                           unsigned* gctr, double* gpart, int* gxcc, int gslow, unsigned gspin, double tol2,
                           int maxit, PRes* res, GroupLds* gl, int64_t t0) {
    const int G = S.G, g = S.g;
    unsigned* ctr = gctr + (size_t)S.grp * 64;
    double* slots = gpart + (size_t)S.grp * 4 * kGroupMax;
    int* xs = gxcc + (size_t)S.grp * kGroupMax;
    const int64_t R0 = S.r0 + S.o0, R1 = S.r0 + S.o1;  // block rows (A0 solve)
    const int64_t V0 = S.r0 + S.v0, V1 = S.r0 + S.v1;  // rows of the vector steps
    const bool grouped = csr_grouped(S.n);
    if (threadIdx.x == 0) {
        gl->flag = 0;
        gl->fast = 0;
        gl->n_slow = 0u;
        gl->n_fast = 0u;
        gl->spin = gspin ? min(gspin, kSpinMax) : kSpinMax;
        xs[g] = xcc_id();
    }
    __syncthreads();
    int its = 0;
    double rr = 0.0, bb = 0.0;
    // placement: the fast barrier only when every member runs on one XCD
    if (group_barrier(ctr, G, gl)) {
        const int ln = (int)(threadIdx.x & 63);
        const int mine = ln < G ? xs[ln] : -1;
        const int x0 = __shfl(mine, 0);
        bool same = true;
        for (int u = 1; u < G; ++u) same = same && __shfl(mine, u) == x0;
        __syncthreads();
        if (threadIdx.x == 0) gl->fast = same && !gslow;
        if (S.lds) {
            for (int i = threadIdx.x; i < S.o1 - S.o0; i += NT) lvec[i] = T(0);
        } else {
#pragma unroll 4
            for (int64_t i = R0 + threadIdx.x; i < R1; i += NT) tg[i] = T(0);
        }
        double acc = 0.0;
#pragma unroll 4
        for (int64_t i = V0 + threadIdx.x; i < V1; i += NT) {
            const double bi = b[i];
            x[i] = 0.0;
            r[i] = bi;
            acc += bi * bi;
        }
        bb = group_sum<NT>(acc, red, slots, ctr, G, g, gl);
        rr = bb;
    }
    double rz = 0.0;
    while (gl->flag == 0 && bb > 0.0) {
        bool ok;
        if (S.lds)
            ok = member_apply<T, NT, true>(S, R0, ctr, gl, meta, mrow, fcol, fval, bcol, bval, dq, erp, eci, ev, etrp,
                                           etci, etv, U, ustride, dcoef, r, z, tg, tq, yv, wv, lvec, red, coef);
        else
            ok = member_apply<T, NT, false>(S, R0, ctr, gl, meta, mrow, fcol, fval, bcol, bval, dq, erp, eci, ev,
                                            etrp, etci, etv, U, ustride, dcoef, r, z, tg, tq, yv, wv, lvec, red, coef);
        if (!ok) break;
        if (!group_barrier(ctr, G, gl)) break;  // z of the block rows, read by the vector steps
        double acc = 0.0;
#pragma unroll 4
        for (int64_t i = V0 + threadIdx.x; i < V1; i += NT) acc += r[i] * z[i];
        const double rzn = group_sum<NT>(acc, red, slots + kGroupMax, ctr, G, g, gl);
        if (gl->flag) break;
        const double beta = its == 0 ? 0.0 : rzn / rz;
        rz = rzn;
#pragma unroll 4
        for (int64_t i = V0 + threadIdx.x; i < V1; i += NT) p[i] = its == 0 ? z[i] : z[i] + beta * p[i];
        if (!group_barrier(ctr, G, gl)) break;  // q = A p reads the other members' p
        ++its;
        acc = 0.0;
#pragma unroll 4
        for (int64_t i = V0 + threadIdx.x; i < V1; i += NT) {
            double s = 0.0;
            const int64_t t1 = arp[i + 1];
            s = csr_row_dot(s, arp[i], t1, aci, av, p, grouped);
            q[i] = s;
            acc += p[i] * s;
        }
        const double pq = group_sum<NT>(acc, red, slots + 2 * kGroupMax, ctr, G, g, gl);
        if (gl->flag) break;
        const double alpha = rz / pq;
        acc = 0.0;
#pragma unroll 4
        for (int64_t i = V0 + threadIdx.x; i < V1; i += NT) {
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            acc += ri * ri;
        }
        rr = group_sum<NT>(acc, red, slots + 3 * kGroupMax, ctr, G, g, gl);
        if (gl->flag) break;
        if (rr <= tol2 * bb || its >= maxit) break;
    }
    // true residual ||b - A x|| (A x reads the other members' x)
    double rt = 0.0;
    if (gl->flag == 0 && group_barrier(ctr, G, gl)) {
        double acc = 0.0;
#pragma unroll 4
        for (int64_t i = V0 + threadIdx.x; i < V1; i += NT) {
            double s = 0.0;
            const int64_t t1 = arp[i + 1];
            s = csr_row_dot(s, arp[i], t1, aci, av, x, grouped);
            const double d = b[i] - s;
            acc += d * d;
        }
        rt = group_sum<NT>(acc, red, slots, ctr, G, g, gl);
    }
    const bool ok = gl->flag == 0;
    if (threadIdx.x == 0) {
        PRes o;
        o.its = its;
        o.status = !ok ? 2 : (bb == 0.0 || rr <= tol2 * bb) ? 0 : 1;
        o.rr = rr;
        o.bb = bb;
        o.rtrue = rt;
        o.ticks = wall_clock64() - t0;
        res[blockIdx.x] = o;
    }
}

// One workgroup per lane.  Vectors are double, device order, lane column at
// col * ld: b (right-hand side), x (written), r, p, q, z (work).  T buffers tg
// (n per column, ld), y and w (interface, lds per column).  tol2 = rtol^2.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_pcg_persist(
    const PSys* __restrict__ sys, const PLane* __restrict__ lanes, const int64_t* __restrict__ arp,
    const int32_t* __restrict__ aci, const double* __restrict__ av, const int4* meta,
    const int32_t* __restrict__ mrow, const int32_t* __restrict__ fcol, const T* __restrict__ fval,
    const int32_t* __restrict__ bcol, const T* __restrict__ bval, const T* __restrict__ dq,
    const int32_t* __restrict__ erp,
    const int32_t* __restrict__ eci, const T* __restrict__ ev, const int32_t* __restrict__ etrp,
    const int32_t* __restrict__ etci, const T* __restrict__ etv, const T* __restrict__ U, int ustride,
    const double* __restrict__ dcoef, const double* __restrict__ b, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ p, double* __restrict__ q, double* __restrict__ z, T* tg, T* tq,
    T* yv, T* wv, int64_t ld, int64_t lds_s, int meta_off, double tol2, int maxit, PRes* __restrict__ res,
    unsigned* gctr, double* gpart, int* gxcc, int gslow, unsigned gspin) {
    extern __shared__ __attribute__((aligned(16))) unsigned char persist_lds[];
    __shared__ double red[(NT / 64) * 16];
    __shared__ double coef[kPersistMaxK];
    __shared__ GroupLds glds;
    const PLane L = lanes[blockIdx.x];
    if (L.sys < 0) return;  // an idle slot of the launch grid
    const int64_t t0 = wall_clock64();
    PSys S = sys[L.sys];
    const int64_t c = L.col;
    b += c * ld, x += c * ld, r += c * ld, p += c * ld, q += c * ld, z += c * ld, tg += c * ld, tq += c * ld;
    yv += c * lds_s, wv += c * lds_s;
    T* lvec = reinterpret_cast<T*>(persist_lds);
    // the lane's level metadata, staged in LDS (read at every level step)
    int4* smeta = reinterpret_cast<int4*>(persist_lds + meta_off);
    for (int j = threadIdx.x; j <= S.l1 - S.l0; j += NT) smeta[j] = meta[S.l0 + j];
    __syncthreads();
    meta = smeta;
    S.l1 -= S.l0;
    S.l0 = 0;
    if (S.G > 1) {
        member_pcg<T, NT>(S, arp, aci, av, meta, mrow, fcol, fval, bcol, bval, dq, erp, eci, ev, etrp, etci, etv, U,
                          ustride, dcoef, b, x, r, p, q, z, tg, tq, yv, wv, lvec, red, coef, gctr, gpart, gxcc, gslow,
                          gspin, tol2, maxit, res, &glds, t0);
        return;
    }
    const int64_t r0 = S.r0, r1 = S.r0 + S.n;
    const bool grouped = csr_grouped(S.n);
    // the solve vector starts at zero (padded ELL terms read it with weight 0)
    if (S.lds) {
        for (int i = threadIdx.x; i < S.n; i += NT) lvec[i] = T(0);
    } else {
#pragma unroll 4
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) tg[i] = T(0);
    }
    // x0 = 0, r0 = b
    double acc = 0.0;
#pragma unroll 4
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        acc += bi * bi;
    }
    const double bb = wg_sum<NT>(acc, red);
    int its = 0;
    double rr = bb;
    // PCG with the preconditioner applied at one place of the loop: each pass
    // forms z = M^{-1} r, then p (z on the first pass, z + beta p after), then
    // one iteration's q = A p, alpha, x, r and the residual test.
    double rz = 0.0;
    while (bb > 0.0) {
        if (S.lds)
            wg_apply<T, NT, true>(S, meta, mrow, fcol, fval, bcol, bval, dq, erp, eci, ev, etrp, etci, etv, U,
                                  ustride, dcoef, r, z, tg, tq, yv, wv, lvec, red, coef);
        else
            wg_apply<T, NT, false>(S, meta, mrow, fcol, fval, bcol, bval, dq, erp, eci, ev, etrp, etci, etv, U,
                                   ustride, dcoef, r, z, tg, tq, yv, wv, lvec, red, coef);
        acc = 0.0;
#pragma unroll 4
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) acc += r[i] * z[i];
        const double rzn = wg_sum<NT>(acc, red);
        const double beta = its == 0 ? 0.0 : rzn / rz;
        rz = rzn;
#pragma unroll 4
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) p[i] = its == 0 ? z[i] : z[i] + beta * p[i];
        __syncthreads();
        ++its;
        acc = 0.0;
#pragma unroll 4
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
            double s = 0.0;
            const int64_t t1 = arp[i + 1];
            s = csr_row_dot(s, arp[i], t1, aci, av, p, grouped);
            q[i] = s;
            acc += p[i] * s;
        }
        const double pq = wg_sum<NT>(acc, red);
        const double alpha = rz / pq;
        acc = 0.0;
#pragma unroll 4
        for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            acc += ri * ri;
        }
        rr = wg_sum<NT>(acc, red);
        if (rr <= tol2 * bb || its >= maxit) break;
    }
    // true residual ||b - A x||
    acc = 0.0;
#pragma unroll 4
    for (int64_t i = r0 + threadIdx.x; i < r1; i += NT) {
        double s = 0.0;
        const int64_t t1 = arp[i + 1];
        s = csr_row_dot(s, arp[i], t1, aci, av, x, grouped);
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
        o.ticks = wall_clock64() - t0;
        res[blockIdx.x] = o;
    }
}

}  // namespace ddlr
