// DDLR preconditioner library: device data, orchestration and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <queue>
#include <thread>
#include <unordered_map>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "ddlr.h"
#include "host_setup.hpp"
#include "kernels.hpp"
#include "pcg_persist.hpp"

using namespace ddlr;

namespace {

thread_local std::string g_err;

// kernel classes timed by ddlr_profile: 0 narrow A0-solve kernel, 1 wide level
// kernels, 2 SpMV with A, 3 low-rank correction kernels
constexpr int kProfClasses = 4;

#define HIPCHK(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw SetupError{e_ == hipErrorOutOfMemory ? DDLR_E_OOM : DDLR_E_DEVICE,                   \
                             std::string(#call) + ": " + hipGetErrorString(e_)};                       \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

// Device-memory budget of a context: every allocation of a handle created in
// the context is counted while it lives; limit 0 means unlimited.
struct Budget {
    std::mutex mu;
    size_t limit = 0, used = 0, peak = 0;
    void take(size_t b) {
        std::lock_guard<std::mutex> lk(mu);
        if (limit && used + b > limit)
            throw SetupError{DDLR_E_BUDGET, "device memory budget exceeded: " + std::to_string(used) + " + " +
                                                std::to_string(b) + " > " + std::to_string(limit) + " bytes"};
        used += b;
        peak = std::max(peak, used);
    }
    void give(size_t b) {
        std::lock_guard<std::mutex> lk(mu);
        used -= std::min(used, b);
    }
};

// Device allocation owned by a handle (counted in its context's budget, if any).
struct DMem {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    Budget* budget = nullptr;
    template <typename T> T* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        const size_t b = count * sizeof(T);
        if (budget) budget->take(b);
        const hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            if (budget) budget->give(b);
            (void)hipGetLastError();
            throw SetupError{e == hipErrorOutOfMemory ? DDLR_E_OOM : DDLR_E_DEVICE,
                             "hipMalloc of " + std::to_string(b) + " bytes: " + hipGetErrorString(e)};
        }
        ptrs.push_back(p);
        bytes += b;
        return static_cast<T*>(p);
    }
    template <typename T> T* upload(const std::vector<T>& h) {
        T* d = alloc<T>(h.size());
        if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }
    void release() {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
        if (budget) budget->give(bytes);
        bytes = 0;
    }
};

// Streams shared by every handle on a device: the interface-level stream, the
// CG stream and the x-update stream.  A process gets few hardware queues (4 by
// default) and the runtime maps further streams onto queues already in use;
// with three streams per handle a second handle's streams would share queues,
// and forked work (the interface levels beside the block solve, the x update)
// would run one after the other.  One set per device keeps them on distinct
// queues.  Calls that put work on them (setup, solves, applies, tuning, the
// server's steps) hold the device's lock, so one thread's graph capture on
// these streams never picks up another thread's work; such calls on one
// device are serialised.
struct DevStreams {
    std::recursive_mutex mu;
    hipStream_t side = nullptr, cg = nullptr, x = nullptr;
};

// The set of device `dev`, created on first use in the order side, cg, x and
// kept until the process ends.
DevStreams& dev_streams(int dev) {
    static std::mutex g;
    static std::map<int, std::unique_ptr<DevStreams>> all;
    DevStreams* D;
    {
        std::lock_guard<std::mutex> lk(g);
        std::unique_ptr<DevStreams>& p = all[dev];
        if (!p) p.reset(new DevStreams());
        D = p.get();
    }
    std::lock_guard<std::recursive_mutex> lk(D->mu);
    if (!D->x) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        HIPCHK(hipSetDevice(dev));
        if (!D->side) HIPCHK(hipStreamCreateWithFlags(&D->side, hipStreamNonBlocking));  // default priority
        if (!D->cg) HIPCHK(hipStreamCreateWithFlags(&D->cg, hipStreamNonBlocking));
        HIPCHK(hipStreamCreateWithFlags(&D->x, hipStreamNonBlocking));
        HIPCHK(hipSetDevice(cur));
    }
    return *D;
}

// Holds the stream lock of a device for its scope.
struct DevLock {
    std::lock_guard<std::recursive_mutex> lk;
    explicit DevLock(int dev) : lk(dev_streams(dev).mu) {}
};

// Scratch memory of ddlr_apply_noalloc: a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol); scratch_ptr() resolves its address per device with
// hipGetSymbolAddress, and kernels take that pointer.
constexpr size_t kScratchBytes = size_t(64) << 20;
}  // namespace
static __device__ __align__(256) char scratch[kScratchBytes];
namespace {

// Device address of `scratch` on device `dev`, which must be current; resolved
// on the first call per device (ddlr_setup makes that call) and kept.
char* scratch_ptr(int dev) {
    static std::mutex mu;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = static_cast<char*>(p);
    return static_cast<char*>(p);
}

// An integer from the environment, else `dflt`.
int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

int grid_for(int64_t work, int block = 256, int cap = 8192) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// 2-D grid (row chunks, right-hand sides) for the column kernels
dim3 grid2(int64_t rows, int nrhs) { return dim3(grid_for(rows, 256, std::max(32, 8192 / std::max(nrhs, 1))), nrhs); }

// Factors of A0 in one precision, device order.
template <typename T> struct DevFactors {
    T *lv = nullptr, *uv = nullptr, *dinv = nullptr;
    T *ev = nullptr, *etv = nullptr;  // E and E^T values
    T *U = nullptr;                   // low-rank basis, row-major (rows x k)
    T *Ut = nullptr;                  // the same in MFMA tile order (k % 16 == 0), for U^T y
    T *xv = nullptr;                  // approximate inverse of C_alpha (values)
    T *cneg = nullptr;                // -C_alpha (values), for the Chebyshev residual update
};

// A Lanczos run kept for continuation: basis Q (s x (cap+1), device
// interface order), alpha / beta on device and host, step scratch.
struct LanczosRun {
    DMem mem;
    double *Q = nullptr, *alpha = nullptr, *beta = nullptr, *sc = nullptr;
    double *w = nullptr, *t1 = nullptr, *t2 = nullptr, *part = nullptr, *csum = nullptr;
    int cap = 0, steps = 0;
    int lvariant = 0;  // operator of the run: DDLR_1 or DDLR_2
    bool broke = false;
    std::vector<double> ha, hb;
    // partial reorthogonalisation (reorth = DDLR_REORTH_PARTIAL): three rows of
    // omega estimates of length cap + 2 (the row of step j is j mod 3), then the
    // running ||T|| estimate; pst = {force next step, skip this step's
    // reorthogonalisation, flag of step 0, 1, ...}
    int reorth = 0;
    double* om = nullptr;
    int* pst = nullptr;
    std::vector<int32_t> hf;  // host copy of the per-step flags
};

struct Workspace {
    int nrhs = 0;
    // Krylov (double, device order)
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    // preconditioner temporaries (type of the preconditioner)
    void *a1 = nullptr, *a2 = nullptr, *ys = nullptr, *ws = nullptr;
    void* ry = nullptr;  // forward results of the R-column ring kernel (ry_cols columns, R values per row)
    int ry_cols = 0;
    void* iy = nullptr;  // interface levels' values, iy_cols (a power of two) per interface row
    int iy_cols = 0;
    double *part = nullptr, *sums = nullptr, *coef = nullptr, *lrsum = nullptr;
    unsigned* ctr = nullptr;  // workgroup counter of k_reduce_lane, zero between launches
    double* xa = nullptr;  // per-lane step of the deferred x update
    CgLane* lanes = nullptr;
    int* done = nullptr;
    int* done_host = nullptr;
    DMem mem;
    // GMRES (allocated on first use, sized for gm_m and nrhs)
    int gm_m = 0, gm_nrhs = 0;
    double *gV = nullptr, *gH = nullptr, *gcs = nullptr, *gsn = nullptr, *gg = nullptr, *gy = nullptr;
    double *gcoef = nullptr, *ginv = nullptr, *gpart = nullptr;
    GmLane* glanes = nullptr;
    DMem gmem;
    // lane admission (device copies of the host request)
    int32_t *adm_start = nullptr, *adm_maxit = nullptr;
    double* adm_tol2 = nullptr;
};

}  // namespace

// Device tables of the persistent PCG form (pcg_persist.hpp) for a handle or
// a batch: systems, merged level lists, A in CSR (device order), lanes and
// results, the lanes' right-hand sides and search directions, and the tuned
// workgroup size.
struct PersistData {
    DMem mem;
    std::vector<PSys> hsys;
    PSys* sys = nullptr;
    int4* meta = nullptr;  // per merged level: rows, widths, ELL starts
    int32_t *mrow = nullptr, *fcol = nullptr, *bcol = nullptr;
    void *fval = nullptr, *bval = nullptr;  // ELL values in the preconditioner's type
    void* dq = nullptr;                      // D^{-1} in merged-level order, same type
    int64_t* arp = nullptr;
    int32_t* aci = nullptr;
    double* av = nullptr;
    PLane* lanes = nullptr;
    PRes* res = nullptr;
    double *b = nullptr, *p = nullptr;  // n x cols each
    int cols = 0;                       // columns b and p hold
    int nlanes = 0;                     // lanes the tables hold
    size_t lds_bytes = 0;               // dynamic LDS of a launch: largest solve vector that fits, then the
    int meta_off = 0;                   // level metadata of the lane, staged at this byte offset
    int nt = 0;                         // threads per workgroup (256, 512, 1024); 0: not tuned
    float nt_us[5] = {0, 0, 0, 0, 0};   // tuning: microseconds per iteration, 64 .. 1024 threads
    // groups: several workgroups on one system (batches only)
    int ngroups = 0;
    unsigned* gctr = nullptr;    // per group 64 counters: the slow barrier's at 0, the fast one's at 32
    double* gpart = nullptr;     // per group 4 x kGroupMax partial sums
    int* gxcc = nullptr;         // per group kGroupMax XCD ids
    int grid = 0;                // lanes of a launch, idle slots included (0: one lane per table entry)
    int gslow = 0;               // 1: group barriers always take the slow form
    unsigned gspin = 0;          // polls before a group wait gives up (0: the kernel's limit)
    std::vector<int> sys_lane;   // per system: the lane of its first member (its result)
    std::vector<int> members;    // per system: workgroups on it
    std::vector<int> entry_sys;  // per table entry: its system
    std::vector<PLane> hlanes;   // the lane table (host copy)
    std::vector<double> sys_us;  // per system: device time of its slowest lane in the last solve
};

// A device and a device-memory budget shared by the handles created in it
// (ddlr_ctx_create).  Freed when the context is destroyed and its last handle
// is gone.
struct ddlr_ctx {
    int device = 0;
    Budget budget;
    std::atomic<int> refs{1};  // the context itself plus every live handle
};

struct ddlr_prec {
    HostPlan plan;
    ddlr_ctx* ctx = nullptr;  // context whose budget counts this handle's memory (NULL: none)
    int device = -1;
    int variant = 0, k = 0, precision = 0, msteps = 0, spd = 0;
    // Proposition (SPD-ness of DDLR-1) assumes A0 SPD: with indefinite local
    // factors the preconditioner is indefinite whatever the Ritz values
    bool pivots_positive = true;
    double theta = 0.0, c0 = 0.0;
    std::vector<double> lam, dvec_h, H_h, ta, tb, ritz;
    int lreorth = DDLR_REORTH_FULL;  // ddlr_reorth of the stored run
    std::vector<int32_t> rflags;     // per step: 1 if the new vector was reorthogonalised
    double setup_ms = 0.0, lanczos_ms = 0.0;
    LanczosRun lrun;     // the setup's Lanczos run (for ddlr_extend_lowrank)
    int theta_mode = 0;  // ddlr_theta of the low-rank build
    DMem mem;
    // device structures (device order)
    int32_t* perm_dev = nullptr;  // device position -> user row
    // SELL-64 of A: values FP64 or (when all exact) FP32, columns int32 or 16-bit row offsets
    int32_t *sell_ptr = nullptr, *sell_col = nullptr;
    int16_t* sell_cold = nullptr;
    double* sell_val = nullptr;
    float* sell_valf = nullptr;
    uint64_t* sell_pk = nullptr;  // (int32 column, FP32 value) pairs when both fit, for the CG's SpMV
    int64_t nslices = 0, sell_nnz = 0;
    int32_t *lrp = nullptr, *lci = nullptr, *urp = nullptr, *uci = nullptr, *lvl_ptr = nullptr;
    int32_t *erp = nullptr, *eci = nullptr, *etrp = nullptr, *etci = nullptr;
    BlockDesc* blk = nullptr;
    int nnarrow = 0, nnarrow_pad = 0;
    // ring variant of the narrow A0-solve kernel (per-level ELL, LDS window)
    RingBlock* rblk = nullptr;
    int32_t *foff = nullptr, *fcol = nullptr, *boff_ = nullptr, *bcol = nullptr, *lwid = nullptr;
    // approximate inverse of C_alpha: SELL-64 slice pointers, slice row -> interface row, columns
    int32_t *xrp = nullptr, *xrow = nullptr, *xci = nullptr;
    int64_t xnnz = 0;
    // Chebyshev solver of C_alpha: C_alpha (CSR, device interface order), steps, scratch
    int32_t *crp = nullptr, *cci = nullptr;
    int cheb_nu = 0;
    DMem chmem;
    void *ch_t = nullptr, *ch_r = nullptr, *ch_d = nullptr, *ch_x = nullptr;  // n x kMaxRhs each, type T
    double *fval64 = nullptr, *bval64 = nullptr;
    float *fval32 = nullptr, *bval32 = nullptr;
    // packed per-row records of the R-column ring kernel (RecLayout), in the
    // handle's precision, with per-level word offsets; null when KW > 4
    int32_t *rfoff = nullptr, *rboff = nullptr, *frec = nullptr, *brec = nullptr;
    int rec_prec = -1;  // DDLR_FP64 (double records) or DDLR_FP32 (float records)
    // interface rows' L and L^T as CSR of packed (value, column) entries
    // (IfacePk) in the handle's precision, for the interface levels through
    // the private buffer; null unless the levels cover exactly the interface
    int32_t *iprp_l = nullptr, *iprp_u = nullptr;
    void *ipk_l = nullptr, *ipk_u = nullptr;
    int ipk_prec = -1;
    int ring_kw = 0;    // 2, 3, 4, 8, 16 or 0 (ring kernel unusable)
    bool ring_ok64 = false, ring_ok32 = false;  // dependency window fits the LDS ring
    int ring_need = 0;                          // rows the ring must hold (dependency window)
    int ring_maxw = 0;                          // widest level of the narrow blocks
    // autotuned launch shape per number of columns: columns per workgroup of
    // the ring kernel (1, 2, 4, 8) and the interface-level overlap; both leave
    // the arithmetic unchanged
    struct Tune {
        int ring_r = 1, ring_nt = 0, overlap = 1;  // ring_nt 0: smallest eligible, -1: plain kernel
        float a0_us[4] = {0, 0, 0, 0};
        float a0_thin_us[2] = {0, 0};  // one column per workgroup of 64 / 256 threads
        float a0_plain_us = 0;         // the plain per-level kernel
        float a0_noov_us = 0;
    };
    std::map<int, Tune> tune;
    int tune_mode = 1;  // 1: tune on first use of a column count, 0: defaults
    // CG runs on a private stream (joined to the caller's by events) so a
    // chunk of iterations can be captured once per column count into a graph
    hipStream_t cg_st = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // x += alpha p runs on its own stream beside the preconditioner
    hipStream_t x_st = nullptr;
    hipEvent_t ev_xf = nullptr, ev_xj = nullptr;
    std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> cg_graphs;  // key: column count * 4 + overlap + 1
    // CG chunk launches: 2 = measured (eager and replayed chunks are timed on
    // the first solves of each column count and the faster is kept), 1 = graphs,
    // 0 = eager (DDLR_CG_GRAPH=1 / 0 force one)
    int graph_mode = 2;
    int level_kernel = 0;  // interface levels: 0 by level size, 1 one thread per row, 2 per (row, column)
    bool cg_xp = true;     // CG: x update in the p-update pass (else on a side stream beside the preconditioner)
    struct CgMode {
        double us[2][3];     // fastest chunk [graph][overlap + 1], overlap -1: not applicable
        int timed[2][3] = {};
        bool captured[3] = {};
        int graph = -1, ov = -2;  // decided form (ov -1: no interface overlap to choose)
        int solves = 0;           // solves run while measuring
        CgMode() {
            for (auto& a : us)
                for (double& v : a) v = 1e30;
        }
    };
    std::map<int, CgMode> cg_mode;
    // persistent PCG (one launch per solve, one workgroup per column): tables,
    // and per column count the measured time per iteration (-1: not measured)
    std::unique_ptr<PersistData> pers;
    std::map<int, double> pers_us;
    int pers_mode = 2;  // 2 measured, 1 forced on, 0 off (DDLR_CG_PERSIST)
    int ov_override = -1;  // >= 0: overlap for the A0 solves being launched (set by the CG driver)
    bool lr_plain = false;                      // low-rank kernels without MFMA (comparison only)
    // the interface block's level kernels run on a side stream, overlapping the
    // B-block kernel (fork/join by events on the caller's stream)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool overlap = true;
    std::vector<std::pair<int, int>> wide;  // rows [a,e) of the wide levels of C (forward order)
    DevFactors<double> f64;
    DevFactors<float> f32;
    int64_t urows = 0;      // rows of U (s for DDLR-1, n for DDLR-2)
    int64_t ndev = 0, sdev = 0;  // device-order rows and interface positions (all systems of a batch)
    // batch of independent systems (batch, any nsys >= 1): per-system row /
    // interface offsets, low-rank scalars; the CG lanes are the systems
    bool batch = false;
    int nsys = 1;
    int64_t *seg_roff = nullptr, *seg_soff = nullptr;
    double *c0s = nullptr, *dvecs = nullptr;
    bool capturing = false;
    __bf16 *ubr = nullptr, *ubt = nullptr;  // BF16 U_k: row-major (k padded to 32) and reduction tiles
    int ukp = 0, uktiles = 0;
    double *dvec = nullptr, *Hk = nullptr;
    Workspace ws;
    DMem lrmem;  // low-rank storage (replaced by set_lowrank)
    // kernel timing (HIP events on the launch stream), per kernel class
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[kProfClasses];
    std::vector<hipEvent_t> prof_pool;
};

namespace {

Budget* budget_of(const ddlr_prec* h) { return h->ctx ? &h->ctx->budget : nullptr; }

// Counts every device allocation of h in ctx's budget from now on.
void attach_ctx(ddlr_prec* h, ddlr_ctx* ctx) {
    if (!ctx) return;
    h->ctx = ctx;
    ctx->refs.fetch_add(1);
    Budget* b = &ctx->budget;
    for (DMem* m : {&h->mem, &h->lrmem, &h->ws.mem, &h->ws.gmem, &h->lrun.mem, &h->chmem}) m->budget = b;
}

void ctx_unref(ddlr_ctx* ctx) {
    if (ctx && ctx->refs.fetch_sub(1) == 1) delete ctx;
}

// ------------------------------------------------------------ device upload

constexpr int kRing64 = 8192, kRing32 = 16384;  // LDS ring rows: 64 KB either way
constexpr int kRingThin = 2048;
constexpr int kMaxLanczos = 1024;  // Lanczos / bidiagonalisation steps (k_gemv_sub stages 1024 coefficients)

// Device-order arrays of one preconditioner (or of several merged), built on
// the host before upload.
struct DevHost {
    int64_t n = 0, s = 0;
    std::vector<int32_t> perm_dev;  // device position -> user row
    std::vector<int64_t> arp;       // A in device order (CSR)
    std::vector<int32_t> aci;
    std::vector<double> av;
    std::vector<int32_t> lrp, lci, urp, uci;  // L (forward) and L^T (backward)
    std::vector<double> lv, uv, dinv;
    std::vector<int32_t> lvl_ptr, lvl_row0;  // level row starts; first row of each level's block
    std::vector<BlockDesc> narrow;           // level ranges of the blocks solved one workgroup each
    std::vector<std::pair<int, int>> wide;   // rows of the interface levels launched one by one
    std::vector<int32_t> erp, eci, etrp, etci;
    std::vector<double> ev, etv;
    std::vector<int32_t> xrp, xci;  // approximate inverse of C_alpha, interface rows in device order
    std::vector<double> xv;
    std::vector<int32_t> crp, cci;  // C_alpha (Chebyshev solver), interface rows in device order, local columns
    std::vector<double> cv;
};

// c_mode: -1 choose (few, wide interface levels -> level launches), 0 interface
// block as one narrow block, 1 interface levels launched one by one
DevHost build_devhost(const HostPlan& P, int c_mode) {
    DevHost D;
    const int64_t n = P.n, m = P.m, s = P.s;
    D.n = n;
    D.s = s;
    D.perm_dev.resize(n);
    for (int64_t d = 0; d < n; ++d) D.perm_dev[d] = P.perm[P.dev2int[d]];
    D.arp.assign(n + 1, 0);
    D.aci.reserve(P.A.nnz());
    D.av.reserve(P.A.nnz());
    for (int64_t d = 0; d < n; ++d) {
        const int64_t i = P.dev2int[d];
        for (int64_t t = P.A.rp[i]; t < P.A.rp[i + 1]; ++t) {
            D.aci.push_back(P.int2dev[P.A.ci[t]]);
            D.av.push_back(P.A.v[t]);
        }
        D.arp[d + 1] = (int64_t)D.aci.size();
    }
    if (P.L.nnz() > INT32_MAX) throw SetupError{DDLR_E_INVALID, "nnz(L) must fit in int32"};
    D.lrp.assign(n + 1, 0);
    D.lci.resize(P.L.nnz());
    D.lv.resize(P.L.nnz());
    for (int64_t d = 0; d < n; ++d) {
        const int64_t i = P.dev2int[d];
        int32_t q = D.lrp[d];
        for (int64_t t = P.L.rp[i]; t < P.L.rp[i + 1]; ++t, ++q) {
            D.lci[q] = P.int2dev[P.L.ci[t]];
            D.lv[q] = P.L.v[t];
        }
        D.lrp[d + 1] = q;
    }
    D.urp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = P.L.rp[i]; t < P.L.rp[i + 1]; ++t) D.urp[P.int2dev[P.L.ci[t]] + 1]++;
    for (int64_t d = 0; d < n; ++d) D.urp[d + 1] += D.urp[d];
    D.uci.resize(P.L.nnz());
    D.uv.resize(P.L.nnz());
    std::vector<int32_t> fill(D.urp.begin(), D.urp.end() - 1);
    for (int64_t i = 0; i < n; ++i)  // ascending internal row j of L_ji -> ascending order in each L^T row
        for (int64_t t = P.L.rp[i]; t < P.L.rp[i + 1]; ++t) {
            const int32_t q = fill[P.int2dev[P.L.ci[t]]]++;
            D.uci[q] = P.int2dev[i];
            D.uv[q] = P.L.v[t];
        }
    D.dinv.resize(n);
    for (int64_t d = 0; d < n; ++d) D.dinv[d] = 1.0 / P.D[P.dev2int[d]];
    D.lvl_ptr = P.lvl_ptr;
    const int nlev = (int)P.lvl_ptr.size() - 1;
    D.lvl_row0.assign(nlev, 0);
    for (int32_t b = 0; b <= P.p; ++b)
        for (int32_t l = P.blk_lvl[b]; l < P.blk_lvl[b + 1]; ++l) D.lvl_row0[l] = (int32_t)P.boff[b];
    // E (n x s) and E^T (s x n)
    const double ia = 1.0 / P.alpha;
    D.erp.assign(n + 1, 0);
    for (int64_t d = 0; d < n; ++d) {
        const int64_t i = P.dev2int[d];
        if (i < m) {
            for (int64_t t = P.A.rp[i]; t < P.A.rp[i + 1]; ++t)
                if (P.A.ci[t] >= m) {
                    D.eci.push_back(P.int2dev[P.A.ci[t]] - (int32_t)m);
                    D.ev.push_back(ia * P.A.v[t]);
                }
        } else {
            D.eci.push_back((int32_t)(d - m));
            D.ev.push_back(-P.alpha);
        }
        D.erp[d + 1] = (int32_t)D.eci.size();
    }
    D.etrp.assign(s + 1, 0);
    D.etci.resize(D.eci.size());
    D.etv.resize(D.eci.size());
    for (size_t t = 0; t < D.eci.size(); ++t) D.etrp[D.eci[t] + 1]++;
    for (int64_t j = 0; j < s; ++j) D.etrp[j + 1] += D.etrp[j];
    std::vector<int32_t> efill(D.etrp.begin(), D.etrp.end() - 1);
    for (int64_t d = 0; d < n; ++d)
        for (int32_t t = D.erp[d]; t < D.erp[d + 1]; ++t) {
            const int32_t q = efill[D.eci[t]]++;
            D.etci[q] = (int32_t)d;
            D.etv[q] = D.ev[t];
        }
    // schedule: B blocks are narrow; the interface block is wide when its
    // levels are few and wide
    const int32_t p = P.p;
    const int32_t c_lv0 = P.blk_lvl[p], c_lv1 = P.blk_lvl[p + 1];
    const int32_t c_levels = c_lv1 - c_lv0;
    bool c_wide = c_levels > 0 && c_levels <= 64 && s / std::max(1, c_levels) >= 2048 && !P.csolve;
    if (const char* env = std::getenv("DDLR_C_WIDE")) {  // "1" forces level launches, "0" one workgroup
        if (env[0] == '1') c_wide = c_levels > 0;
        if (env[0] == '0') c_wide = false;
    }
    if (c_mode == 0) c_wide = false;
    if (c_mode == 1) c_wide = c_levels > 0;
    if (P.csolve == 2) {
        // Chebyshev: D_alpha solves by the interface levels alone; C_alpha for the residual
        c_wide = c_levels > 0;
        D.crp.assign(s + 1, 0);
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t r = 0; r < s; ++r) {
            const int64_t i = P.dev2int[m + r];
            row.clear();
            for (int64_t t = P.A0.rp[i]; t < P.A0.rp[i + 1]; ++t)
                row.emplace_back((int32_t)(P.int2dev[P.A0.ci[t]] - m), P.A0.v[t]);
            std::sort(row.begin(), row.end());
            for (const auto& e : row) {
                D.cci.push_back(e.first);
                D.cv.push_back(-e.second);
            }
            D.crp[r + 1] = (int32_t)D.cci.size();
        }
    }
    for (int32_t b = 0; b < p; ++b)
        if (P.blk_lvl[b + 1] > P.blk_lvl[b]) D.narrow.push_back({P.blk_lvl[b], P.blk_lvl[b + 1]});
    if (P.csolve == 1) {
        // C_alpha by its approximate inverse: X with device-order interface indices
        D.xrp.assign(s + 1, 0);
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t r = 0; r < s; ++r) {
            const int64_t y = P.dev2int[m + r] - m;
            row.clear();
            for (int64_t t = P.X.rp[y]; t < P.X.rp[y + 1]; ++t)
                row.emplace_back((int32_t)(P.int2dev[m + P.X.ci[t]] - m), P.X.v[t]);
            std::sort(row.begin(), row.end());
            for (const auto& e : row) {
                D.xci.push_back(e.first);
                D.xv.push_back(e.second);
            }
            if (D.xci.size() > (size_t)INT32_MAX) throw SetupError{DDLR_E_INVALID, "nnz(X) must fit in int32"};
            D.xrp[r + 1] = (int32_t)D.xci.size();
        }
    } else if (c_wide) {
        for (int32_t l = c_lv0; l < c_lv1; ++l) D.wide.emplace_back(P.lvl_ptr[l], P.lvl_ptr[l + 1]);
    } else if (c_levels > 0) {
        D.narrow.push_back({c_lv0, c_lv1});
    }
    return D;
}

// Concatenates several systems: rows, interface positions and levels are
// offset by the sizes of the systems before.
void merge_devhost(const std::vector<const DevHost*>& parts, DevHost& out) {
    out = DevHost();
    int64_t R = 0, S = 0;
    int32_t Lv = 0;
    out.arp.push_back(0);
    out.lrp.push_back(0);
    out.urp.push_back(0);
    out.erp.push_back(0);
    out.etrp.push_back(0);
    for (const DevHost* P : parts) {
        for (int32_t v : P->perm_dev) out.perm_dev.push_back((int32_t)(v + R));
        for (int64_t d = 0; d < P->n; ++d) {
            for (int64_t t = P->arp[d]; t < P->arp[d + 1]; ++t) {
                out.aci.push_back((int32_t)(P->aci[t] + R));
                out.av.push_back(P->av[t]);
            }
            out.arp.push_back((int64_t)out.aci.size());
            for (int32_t t = P->lrp[d]; t < P->lrp[d + 1]; ++t) {
                out.lci.push_back((int32_t)(P->lci[t] + R));
                out.lv.push_back(P->lv[t]);
            }
            out.lrp.push_back((int32_t)out.lci.size());
            for (int32_t t = P->urp[d]; t < P->urp[d + 1]; ++t) {
                out.uci.push_back((int32_t)(P->uci[t] + R));
                out.uv.push_back(P->uv[t]);
            }
            out.urp.push_back((int32_t)out.uci.size());
            for (int32_t t = P->erp[d]; t < P->erp[d + 1]; ++t) {
                out.eci.push_back((int32_t)(P->eci[t] + S));
                out.ev.push_back(P->ev[t]);
            }
            out.erp.push_back((int32_t)out.eci.size());
            out.dinv.push_back(P->dinv[d]);
        }
        for (int64_t j = 0; j < P->s; ++j) {
            for (int32_t t = P->etrp[j]; t < P->etrp[j + 1]; ++t) {
                out.etci.push_back((int32_t)(P->etci[t] + R));
                out.etv.push_back(P->etv[t]);
            }
            out.etrp.push_back((int32_t)out.etci.size());
        }
        const int nl = (int)P->lvl_ptr.size() - 1;
        for (int l = 0; l < nl; ++l) {
            out.lvl_ptr.push_back((int32_t)(P->lvl_ptr[l] + R));
            out.lvl_row0.push_back((int32_t)(P->lvl_row0[l] + R));
        }
        for (const BlockDesc& b : P->narrow) out.narrow.push_back({b.lvl0 + Lv, b.lvl1 + Lv});
        for (const auto& wv : P->wide) out.wide.emplace_back((int)(wv.first + R), (int)(wv.second + R));
        R += P->n;
        S += P->s;
        Lv += nl;
    }
    out.lvl_ptr.push_back((int32_t)R);
    out.n = R;
    out.s = S;
}

// Packed records (RecLayout) of one sweep's factor for the R-column ring
// kernel: per level, the chunk arrays of its rows one after another, level
// offsets in words (multiples of four).  Values are rounded to T as the
// factor's own T copy is; D^{-1} (backward) likewise.
template <typename T, int KW, bool kBwd>
void pack_records(const DevHost& D, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                  const std::vector<double>& v, std::vector<int32_t>& off, std::vector<int32_t>& rec) {
    using L = RecLayout<T, KW, kBwd>;
    const int nlev = (int)D.lvl_ptr.size() - 1;
    off.assign(nlev, 0);
    rec.clear();
    auto put = [](uint32_t* w, int word, double x) {
        const T t = (T)x;
        std::memcpy(w + word, &t, sizeof(T));
    };
    for (int l = 0; l < nlev; ++l) {
        const int a = D.lvl_ptr[l], e = D.lvl_ptr[l + 1], nr = e - a;
        const size_t o = rec.size();
        off[l] = (int32_t)std::min<size_t>(o, INT32_MAX);
        rec.resize(o + (size_t)L::kPadded * nr, 0);
        for (int i = a; i < e; ++i) {
            uint32_t w[L::kPadded] = {};
            for (int t = rp[i], j = 0; t < rp[i + 1] && j < KW; ++t, ++j) {
                put(w, j * L::kTW, v[t]);
                w[L::kColW + j / 2] |= ((uint32_t)(ci[t] - D.lvl_row0[l]) & 0xffffu) << (16 * (j & 1));
            }
            if (kBwd) put(w, L::kDiag, D.dinv[i]);
            const size_t r = (size_t)(i - a);
            for (int c = 0; c < L::kN4; ++c)
                for (int k = 0; k < 4; ++k) rec[o + ((size_t)c * nr + r) * 4 + k] = (int32_t)w[4 * c + k];
            for (int k = 0; k < L::kRem; ++k)
                rec[o + (size_t)4 * L::kN4 * nr + r * L::kRem + k] = (int32_t)w[4 * L::kN4 + k];
        }
        rec.resize((rec.size() + 3) / 4 * 4, 0);
    }
}

template <int KW>
void pack_all(const DevHost& D, bool f64, std::vector<int32_t>& rfo, std::vector<int32_t>& frec,
              std::vector<int32_t>& rbo, std::vector<int32_t>& brec) {
    if (f64) {
        pack_records<double, KW, false>(D, D.lrp, D.lci, D.lv, rfo, frec);
        pack_records<double, KW, true>(D, D.urp, D.uci, D.uv, rbo, brec);
    } else {
        pack_records<float, KW, false>(D, D.lrp, D.lci, D.lv, rfo, frec);
        pack_records<float, KW, true>(D, D.urp, D.uci, D.uv, rbo, brec);
    }
}

// Per-level ELL copies of L (forward) and L^T (backward) for the ring kernel,
// fixed width KW for every level, block-local column indices, and the check
// that every dependency falls inside the LDS window of the most recent kRing
// rows.
void build_ring(ddlr_prec* h, const DevHost& D) {
    const std::vector<BlockDesc>& bd = D.narrow;
    const std::vector<int32_t>&lrp = D.lrp, &lci = D.lci, &urp = D.urp, &uci = D.uci;
    const int nlev = (int)D.lvl_ptr.size() - 1;
    int kw = 0, need = 0, maxw = 0;
    bool ok64 = true, ok32 = true;
    for (const BlockDesc& b : bd) {
        if (b.lvl1 - b.lvl0 > kRingMaxLevels) ok64 = ok32 = false;
        for (int l = b.lvl0; l < b.lvl1; ++l) {
            const int row0 = D.lvl_row0[l];
            const int a = D.lvl_ptr[l] - row0, e = D.lvl_ptr[l + 1] - row0;
            maxw = std::max(maxw, e - a);
            for (int i = a; i < e; ++i) {
                kw = std::max({kw, lrp[row0 + i + 1] - lrp[row0 + i], urp[row0 + i + 1] - urp[row0 + i]});
                for (int t = lrp[row0 + i]; t < lrp[row0 + i + 1]; ++t) {
                    const int c = lci[t] - row0;
                    ok64 = ok64 && c >= e - kRing64;
                    ok32 = ok32 && c >= e - kRing32;
                    need = std::max(need, e - c);
                }
                for (int t = urp[row0 + i]; t < urp[row0 + i + 1]; ++t) {
                    const int c = uci[t] - row0;
                    ok64 = ok64 && c < a + kRing64;
                    ok32 = ok32 && c < a + kRing32;
                    need = std::max(need, c - a + 1);
                }
            }
        }
    }
    h->ring_kw = kw <= 2 ? 2 : kw <= 3 ? 3 : kw <= 4 ? 4 : kw <= 8 ? 8 : kw <= 16 ? 16 : kw <= 32 ? 32 : 0;
    if (const char* env = std::getenv("DDLR_TRSV_PLAIN"))  // "1": always the plain per-level kernel
        if (env[0] == '1') h->ring_kw = 0;
    h->ring_ok64 = ok64 && h->ring_kw > 0;
    h->ring_ok32 = ok32 && h->ring_kw > 0;
    h->ring_need = need;
    h->ring_maxw = maxw;
    if (!h->ring_ok64 && !h->ring_ok32) return;
    const int KW = h->ring_kw;
    std::vector<int32_t> foff(nlev), boff(nlev), fcol, bcol, lwid(nlev, 0);
    std::vector<double> fval, bval;
    // ELL width of a level: KW for the narrow kernels, else the level's widest
    // row rounded up to a multiple of 4
    auto width = [&](const std::vector<int32_t>& rp, int l) {
        if (KW <= 4) return KW;
        int w = 0;
        for (int i = D.lvl_ptr[l]; i < D.lvl_ptr[l + 1]; ++i) w = std::max(w, rp[i + 1] - rp[i]);
        return std::min(KW, (w + 3) / 4 * 4);
    };
    auto build = [&](const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, const std::vector<double>& v,
                     std::vector<int32_t>& off, std::vector<int32_t>& col, std::vector<double>& val, int shift) {
        for (int l = 0; l < nlev; ++l) {
            const int a = D.lvl_ptr[l], e = D.lvl_ptr[l + 1], nr = e - a;
            const int W = width(rp, l);
            lwid[l] |= W << shift;
            off[l] = (int32_t)col.size();
            col.resize(col.size() + (size_t)W * nr, 0);  // padding: column 0, value 0
            val.resize(val.size() + (size_t)W * nr, 0.0);
            for (int i = a; i < e; ++i) {
                const int t0 = rp[i], t1 = std::min(rp[i + 1], rp[i] + W);
                for (int t = t0, j = 0; t < t1; ++t, ++j) {
                    col[off[l] + (size_t)j * nr + (i - a)] = ci[t] - D.lvl_row0[l];
                    val[off[l] + (size_t)j * nr + (i - a)] = v[t];
                }
            }
        }
    };
    build(lrp, lci, D.lv, foff, fcol, fval, 0);
    build(urp, uci, D.uv, boff, bcol, bval, 16);
    std::vector<RingBlock> rb;
    for (const BlockDesc& b : bd) rb.push_back({b.lvl0, b.lvl1, D.lvl_row0[b.lvl0], 0});
    DMem& M = h->mem;
    h->rblk = M.upload(rb);
    h->foff = M.upload(foff);
    h->fcol = M.upload(fcol);
    h->boff_ = M.upload(boff);
    h->bcol = M.upload(bcol);
    h->lwid = M.upload(lwid);
    h->fval64 = M.upload(fval);
    h->bval64 = M.upload(bval);
    if (h->precision != DDLR_FP64) {
        std::vector<float> f(fval.begin(), fval.end()), g(bval.begin(), bval.end());
        h->fval32 = M.upload(f);
        h->bval32 = M.upload(g);
    }
    if (KW <= 4) {
        std::vector<int32_t> rfo, rbo, frec, brec;
        const bool f64 = h->precision == DDLR_FP64;
        switch (KW) {
        case 2: pack_all<2>(D, f64, rfo, frec, rbo, brec); break;
        case 3: pack_all<3>(D, f64, rfo, frec, rbo, brec); break;
        default: pack_all<4>(D, f64, rfo, frec, rbo, brec); break;
        }
        if (frec.size() <= (size_t)INT32_MAX && brec.size() <= (size_t)INT32_MAX) {
            h->rfoff = M.upload(rfo);
            h->rboff = M.upload(rbo);
            h->frec = M.upload(frec);
            h->brec = M.upload(brec);
            h->rec_prec = f64 ? DDLR_FP64 : DDLR_FP32;
        }
    }
}

// The interface rows' L (forward) and L^T (backward) as CSR of packed
// (value, column) entries for k_iface_rows / k_iface_cols, when the interface
// levels cover the rows m .. n-1 one after another.
template <typename T>
void pack_iface(const DevHost& D, int64_t m, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                const std::vector<double>& v, std::vector<int32_t>& prp, std::vector<typename IfacePk<T>::type>& pk) {
    const int64_t n = D.n;
    prp.assign(n - m + 1, 0);
    pk.clear();
    for (int64_t i = m; i < n; ++i) {
        for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
            const T val = (T)v[t];
            typename IfacePk<T>::type e{};
            if constexpr (sizeof(T) == 4) {
                e.x = ci[t];
                std::memcpy(&e.y, &val, 4);
            } else {
                uint64_t bits;
                std::memcpy(&bits, &val, 8);
                e.x = (int32_t)(uint32_t)(bits & 0xffffffffu);
                e.y = (int32_t)(uint32_t)(bits >> 32);
                e.z = ci[t];
                e.w = 0;
            }
            pk.push_back(e);
        }
        prp[i - m + 1] = (int32_t)pk.size();
    }
}

void build_iface_packs(ddlr_prec* h, const DevHost& D) {
    const int64_t n = D.n, m = D.n - D.s;
    if (D.wide.empty() || D.wide.front().first != m || D.wide.back().second != n) return;
    for (size_t l = 1; l < D.wide.size(); ++l)
        if (D.wide[l].first != D.wide[l - 1].second) return;
    DMem& M = h->mem;
    std::vector<int32_t> pl, pu;
    if (h->precision == DDLR_FP64) {
        std::vector<int4> kl, ku;
        pack_iface<double>(D, m, D.lrp, D.lci, D.lv, pl, kl);
        pack_iface<double>(D, m, D.urp, D.uci, D.uv, pu, ku);
        h->ipk_l = M.upload(kl);
        h->ipk_u = M.upload(ku);
    } else {
        std::vector<int2> kl, ku;
        pack_iface<float>(D, m, D.lrp, D.lci, D.lv, pl, kl);
        pack_iface<float>(D, m, D.urp, D.uci, D.uv, pu, ku);
        h->ipk_l = M.upload(kl);
        h->ipk_u = M.upload(ku);
    }
    h->iprp_l = M.upload(pl);
    h->iprp_u = M.upload(pu);
    h->ipk_prec = h->precision == DDLR_FP64 ? DDLR_FP64 : DDLR_FP32;
}

// Uploads the device-order arrays and builds SELL-64 for A.
void upload_devhost(ddlr_prec* h, const DevHost& D) {
    DMem& M = h->mem;
    const int64_t n = D.n;
    h->ndev = n;
    h->sdev = D.s;
    h->perm_dev = M.upload(D.perm_dev);
    h->nslices = (n + kSell - 1) / kSell;
    std::vector<int32_t> sptr(h->nslices + 1, 0);
    for (int64_t sl = 0; sl < h->nslices; ++sl) {
        int64_t w = 0;
        for (int64_t d = sl * kSell; d < std::min<int64_t>(n, (sl + 1) * kSell); ++d)
            w = std::max<int64_t>(w, D.arp[d + 1] - D.arp[d]);
        if ((int64_t)sptr[sl] + w * kSell > INT32_MAX) throw SetupError{DDLR_E_INVALID, "A too large for SELL-64"};
        sptr[sl + 1] = sptr[sl] + (int32_t)(w * kSell);
    }
    h->sell_nnz = sptr[h->nslices];
    std::vector<int32_t> scol(h->sell_nnz);
    std::vector<double> sval(h->sell_nnz, 0.0);
    for (int64_t sl = 0; sl < h->nslices; ++sl) {
        const int w = (sptr[sl + 1] - sptr[sl]) / kSell;
        for (int lane = 0; lane < kSell; ++lane) {
            const int64_t d = sl * kSell + lane;
            const int64_t cnt = d < n ? D.arp[d + 1] - D.arp[d] : 0;
            for (int j = 0; j < w; ++j) {
                const int64_t q = sptr[sl] + (int64_t)j * kSell + lane;
                if (j < cnt) {
                    scol[q] = D.aci[D.arp[d] + j];
                    sval[q] = D.av[D.arp[d] + j];
                } else {
                    scol[q] = (int32_t)std::min<int64_t>(d, n - 1);
                    sval[q] = 0.0;
                }
            }
        }
    }
    h->sell_ptr = M.upload(sptr);
    bool f32ok = true, i16ok = true;
    for (int64_t sl = 0; sl < h->nslices && (f32ok || i16ok); ++sl)
        for (int64_t q = sptr[sl]; q < sptr[sl + 1]; ++q) {
            const int64_t row = sl * kSell + (q - sptr[sl]) % kSell;
            f32ok = f32ok && (double)(float)sval[q] == sval[q];
            i16ok = i16ok && std::llabs((long long)scol[q] - (long long)row) <= 32767;
        }
    if (const char* env = std::getenv("DDLR_SELL_WIDE"))  // "1": FP64 values and int32 columns always
        if (env[0] == '1') f32ok = i16ok = false;
    if (i16ok) {
        std::vector<int16_t> d(scol.size());
        for (int64_t sl = 0; sl < h->nslices; ++sl)
            for (int64_t q = sptr[sl]; q < sptr[sl + 1]; ++q)
                d[q] = (int16_t)(scol[q] - (sl * kSell + (q - sptr[sl]) % kSell));
        h->sell_cold = M.upload(d);
    } else {
        h->sell_col = M.upload(scol);
    }
    if (f32ok) {
        std::vector<float> f(sval.begin(), sval.end());
        h->sell_valf = M.upload(f);
        if (!i16ok) {  // one 8-byte load per entry in the interleaved SpMV
            std::vector<uint64_t> pk(scol.size());
            for (size_t q = 0; q < pk.size(); ++q) {
                uint32_t bits;
                std::memcpy(&bits, &f[q], 4);
                pk[q] = (uint64_t)(uint32_t)scol[q] | ((uint64_t)bits << 32);
            }
            h->sell_pk = M.upload(pk);
        }
    } else {
        h->sell_val = M.upload(sval);
    }
    h->lrp = M.upload(D.lrp);
    h->lci = M.upload(D.lci);
    h->urp = M.upload(D.urp);
    h->uci = M.upload(D.uci);
    h->f64.lv = M.upload(D.lv);
    h->f64.uv = M.upload(D.uv);
    h->f64.dinv = M.upload(D.dinv);
    h->lvl_ptr = M.upload(D.lvl_ptr);
    h->erp = M.upload(D.erp);
    h->eci = M.upload(D.eci);
    h->etrp = M.upload(D.etrp);
    h->etci = M.upload(D.etci);
    h->f64.ev = M.upload(D.ev);
    h->f64.etv = M.upload(D.etv);
    if (!D.crp.empty()) {
        h->crp = M.upload(D.crp);
        h->cci = M.upload(D.cci);
        h->f64.cneg = M.upload(D.cv);
    }
    std::vector<double> xsell;
    if (!D.xrp.empty()) {
        // SELL-64 of X: rows by entry count (longest first, stable), slices of 64
        const int64_t s = D.s;
        std::vector<int32_t> order(s);
        for (int64_t r = 0; r < s; ++r) order[r] = (int32_t)r;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return D.xrp[a + 1] - D.xrp[a] > D.xrp[b + 1] - D.xrp[b];
        });
        const int64_t ns = (s + 63) / 64;
        std::vector<int32_t> sp(ns + 1, 0), xrow(ns * 64, 0), xcol;
        for (int64_t sl = 0; sl < ns; ++sl) {
            int64_t wmax = 0;
            for (int64_t q = sl * 64; q < std::min<int64_t>(s, (sl + 1) * 64); ++q)
                wmax = std::max<int64_t>(wmax, D.xrp[order[q] + 1] - D.xrp[order[q]]);
            if ((int64_t)sp[sl] + wmax * 64 > INT32_MAX) throw SetupError{DDLR_E_INVALID, "X too large for SELL-64"};
            sp[sl + 1] = sp[sl] + (int32_t)(wmax * 64);
        }
        xcol.assign(sp[ns], 0);
        xsell.assign(sp[ns], 0.0);
        for (int64_t sl = 0; sl < ns; ++sl) {
            const int w = (sp[sl + 1] - sp[sl]) / 64;
            for (int lane = 0; lane < 64; ++lane) {
                const int64_t q = sl * 64 + lane;
                // padding rows of the last slice repeat row 0 with zero entries; their
                // threads are not launched (rows = s)
                const int32_t r = q < s ? order[q] : 0;
                xrow[q] = r;
                const int32_t cnt = q < s ? D.xrp[r + 1] - D.xrp[r] : 0;
                for (int j = 0; j < cnt; ++j) {
                    xcol[sp[sl] + (int64_t)j * 64 + lane] = D.xci[D.xrp[r] + j];
                    xsell[sp[sl] + (int64_t)j * 64 + lane] = D.xv[D.xrp[r] + j];
                }
                (void)w;
            }
        }
        h->xrp = M.upload(sp);
        h->xrow = M.upload(xrow);
        h->xci = M.upload(xcol);
        h->f64.xv = M.upload(xsell);
        h->xnnz = (int64_t)D.xv.size();
    }
    if (h->precision != DDLR_FP64) {
        auto demote = [&](const std::vector<double>& a) {
            std::vector<float> f(a.size());
            for (size_t i = 0; i < a.size(); ++i) f[i] = (float)a[i];
            return M.upload(f);
        };
        h->f32.lv = demote(D.lv);
        h->f32.uv = demote(D.uv);
        h->f32.dinv = demote(D.dinv);
        h->f32.ev = demote(D.ev);
        h->f32.etv = demote(D.etv);
        if (!xsell.empty()) h->f32.xv = demote(xsell);
        if (!D.cv.empty()) h->f32.cneg = demote(D.cv);
    }
    h->wide = D.wide;
    h->nnarrow = (int)D.narrow.size();
    h->nnarrow_pad = (h->nnarrow + 7) / 8 * 8;
    h->blk = M.upload(D.narrow);
    build_ring(h, D);
    build_iface_packs(h, D);
}

void upload_structures(ddlr_prec* h, int c_mode = -1) { upload_devhost(h, build_devhost(h->plan, c_mode)); }

// ------------------------------------------------------------ workspace

constexpr int kLrBlocks = 1024;  // grid of the low-rank reduction
constexpr int kSegChunks = 16;   // blocks per system in the per-system kernels of a batch

template <typename T> T* wsalloc(Workspace& W, size_t count) { return W.mem.alloc<T>(count); }

// stride of the interleaved CG direction p: the power of two >= lanes
int lane_stride(int lanes) {
    int S = 1;
    while (S < lanes) S <<= 1;
    return S;
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

void drop_graphs(ddlr_prec* h);

void ensure_ws(ddlr_prec* h, int nrhs) {
    Workspace& W = h->ws;
    if (W.nrhs >= nrhs) return;
    drop_graphs(h);  // captured kernels hold workspace pointers
    W.mem.release();
    W.gmem.release();
    W.gm_m = W.gm_nrhs = 0;
    if (W.done_host) {
        (void)hipHostFree(W.done_host);
        W.done_host = nullptr;
    }
    const int64_t n = h->ndev, s = h->sdev;
    const size_t tsz = h->precision == DDLR_FP64 ? sizeof(double) : sizeof(float);
    W.x = W.mem.alloc<double>(n * nrhs);
    W.r = W.mem.alloc<double>(n * nrhs);
    W.z = W.mem.alloc<double>(n * nrhs);
    // p is interleaved inside CG (stride lane_stride(nrhs)); zeroed so the
    // padding lanes hold finite values
    W.p = W.mem.alloc<double>(n * lane_stride(nrhs));
    HIPCHK(hipMemset(W.p, 0, sizeof(double) * n * lane_stride(nrhs)));
    W.q = W.mem.alloc<double>(n * nrhs);
    W.a1 = W.mem.alloc<char>(tsz * n * nrhs);
    W.a2 = W.mem.alloc<char>(tsz * n * nrhs);
    W.ry = W.mem.alloc<char>(tsz * n * nrhs);
    W.ry_cols = nrhs;
    W.iy_cols = 1;
    while (W.iy_cols < std::min(nrhs, kMaxRhs)) W.iy_cols <<= 1;
    W.iy = W.mem.alloc<char>(tsz * s * W.iy_cols);
    W.ys = W.mem.alloc<char>(tsz * s * nrhs);
    W.ws = W.mem.alloc<char>(tsz * s * nrhs);
    const int kk = std::max(1, h->k);
    const int64_t parts = std::max({(int64_t)kRedBlocks * nrhs, ((n + 255) / 256) * (int64_t)nrhs,
                                    (int64_t)kLrBlocks * nrhs * kk, (int64_t)kSegChunks * h->nsys});
    W.part = W.mem.alloc<double>(parts);
    W.sums = W.mem.alloc<double>((size_t)std::max(nrhs, h->nsys) * 256);
    W.coef = W.mem.alloc<double>((size_t)std::max(nrhs, h->nsys) * kk);
    W.lrsum = W.mem.alloc<double>((size_t)std::max(nrhs, 1) * kk);
    W.xa = W.mem.alloc<double>(std::max(nrhs, 1));
    W.lanes = W.mem.alloc<CgLane>(std::max(nrhs, h->nsys));
    W.adm_start = W.mem.alloc<int32_t>(std::max(nrhs, 1));
    W.adm_maxit = W.mem.alloc<int32_t>(std::max(nrhs, 1));
    W.adm_tol2 = W.mem.alloc<double>(std::max(nrhs, 1));
    W.done = W.mem.alloc<int>(1);
    W.ctr = W.mem.alloc<unsigned>(1);  // re-armed by k_reduce_lane
    HIPCHK(hipMemset(W.ctr, 0, sizeof(unsigned)));
    HIPCHK(hipHostMalloc((void**)&W.done_host, sizeof(int)));
    W.nrhs = nrhs;
}

// ------------------------------------------------------------ kernel timing

hipEvent_t prof_event(ddlr_prec* h) {
    if (!h->prof_pool.empty()) {
        hipEvent_t e = h->prof_pool.back();
        h->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

struct ProfScope {
    ddlr_prec* h;
    int cls;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    ProfScope(ddlr_prec* h_, int cls_, hipStream_t st_) : h(h_), cls(cls_), st(st_) {
        if (h->prof && !h->capturing) {
            e0 = prof_event(h);
            HIPCHK(hipEventRecord(e0, st));
        }
    }
    ~ProfScope() noexcept(false) {
        if (e0) {
            hipEvent_t e1 = prof_event(h);
            HIPCHK(hipEventRecord(e1, st));
            h->prof_ev[cls].emplace_back(e0, e1);
        }
    }
};

// ------------------------------------------------------------ A0 solve

template <typename T> const DevFactors<T>& factors(const ddlr_prec* h);
template <> const DevFactors<double>& factors<double>(const ddlr_prec* h) { return h->f64; }
template <> const DevFactors<float>& factors<float>(const ddlr_prec* h) { return h->f32; }

template <typename T> bool ring_ready(const ddlr_prec* h);
template <> bool ring_ready<double>(const ddlr_prec* h) { return h->ring_ok64; }
template <> bool ring_ready<float>(const ddlr_prec* h) { return h->ring_ok32 && h->fval32; }
template <typename T> const T* ring_fval(const ddlr_prec* h);
template <> const double* ring_fval<double>(const ddlr_prec* h) { return h->fval64; }
template <> const float* ring_fval<float>(const ddlr_prec* h) { return h->fval32; }
template <typename T> const T* ring_bval(const ddlr_prec* h);
template <> const double* ring_bval<double>(const ddlr_prec* h) { return h->bval64; }
template <> const float* ring_bval<float>(const ddlr_prec* h) { return h->bval32; }
template <typename T> constexpr int ring_rows();
template <> constexpr int ring_rows<double>() { return kRing64; }
template <> constexpr int ring_rows<float>() { return kRing32; }

// Workgroup sizes of the one-column ring kernel: any of 64, 256 and 512 is
// correct (rows beyond a workgroup's row sets are done without prefetch).
// Untuned, 64 or 256 is taken when every level fits their row sets and the
// dependency window is short (small rings leave LDS for more workgroups).
bool ring_nt_ok(const ddlr_prec* h, int nt) { return nt == 64 || nt == 256 || nt == 512; }
int ring_nt_default(const ddlr_prec* h) {
    const int ns = h->ring_kw <= 16 ? 2 : 1;
    for (int nt : {64, 256})
        if (h->ring_maxw <= nt * ns && h->ring_need <= kRingThin) return nt;
    return 512;
}

// ring rows: the dependency window rounded up to a power of two (at least 64)
int ring_rows_for(const ddlr_prec* h) {
    int r = 64;
    while (r < h->ring_need) r <<= 1;
    return r;
}

template <typename T, int KW, typename TIn, typename TOut, int NT>
void launch_ring_nt(ddlr_prec* h, const T* dinv, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                    hipStream_t st, const int* done) {
    const int rows = ring_rows_for(h);  // <= ring_rows<T>(): checked when the ring was enabled
    hipLaunchKernelGGL((k_trsv_ring<T, KW, TIn, TOut, NT>), dim3(h->nnarrow_pad * nrhs), dim3(NT),
                       (size_t)rows * sizeof(T), st, h->rblk, h->nnarrow, h->nnarrow_pad, nrhs, h->lvl_ptr, h->foff,
                       h->fcol, ring_fval<T>(h), h->boff_, h->bcol, ring_bval<T>(h), h->lwid, rows - 1, dinv, x, ldx,
                       z, ldz, done);
    LAUNCHCHK();
}

template <typename T> int ring_nt_for(const ddlr_prec* h, int nrhs);

template <typename T, int KW, typename TIn, typename TOut>
void launch_ring_kw(ddlr_prec* h, const T* dinv, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                    hipStream_t st, const int* done) {
    switch (ring_nt_for<T>(h, nrhs)) {
    case 64: launch_ring_nt<T, KW, TIn, TOut, 64>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    case 256: launch_ring_nt<T, KW, TIn, TOut, 256>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    default: launch_ring_nt<T, KW, TIn, TOut, 512>(h, dinv, nrhs, x, ldx, z, ldz, st, done);
    }
}

template <typename T, typename TIn, typename TOut>
void launch_ring(ddlr_prec* h, const T* dinv, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                 hipStream_t st, const int* done) {
    switch (h->ring_kw) {
    case 2: launch_ring_kw<T, 2, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    case 3: launch_ring_kw<T, 3, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    case 4: launch_ring_kw<T, 4, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    case 8: launch_ring_kw<T, 8, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    case 16: launch_ring_kw<T, 16, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    default: launch_ring_kw<T, 32, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done);
    }
}

// The packed-record kernel for R columns per workgroup: its records in T, the
// workspace's buffer for the forward results of nrhs columns, and a
// dependency window that fits its ring of ring_rows_r<T, R>() rows.
template <typename T> bool rec_ok(const ddlr_prec* h, int R, int nrhs) {
    if (!ring_ready<T>(h) || h->ring_kw > 4 || !h->frec) return false;
    if (h->rec_prec != (sizeof(T) == 8 ? DDLR_FP64 : DDLR_FP32)) return false;
    if (!h->ws.ry || h->ws.ry_cols < nrhs) return false;
    switch (R) {
    case 1: return h->ring_need <= ring_rows_r<T, 1>();
    case 2: return h->ring_need <= ring_rows_r<T, 2>();
    case 4: return h->ring_need <= ring_rows_r<T, 4>();
    case 8: return h->ring_need <= ring_rows_r<T, 8>();
    default: return false;
    }
}

// R columns per workgroup: R > 1 needs the packed-record kernel; one column
// runs it too when it can (512 threads), else the one-column kernel
template <typename T> bool ring_r_ok(const ddlr_prec* h, int R, int nrhs) {
    return R == 1 || rec_ok<T>(h, R, nrhs);
}

template <typename T, int KW, int R, typename TIn, typename TOut>
void launch_ring_rk(ddlr_prec* h, const T* dinv, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                    hipStream_t st, const int* done) {
    (void)dinv;  // D^{-1} is inside the backward records
    const int ng = nrhs / R;
    const int64_t n = h->ndev;
    hipLaunchKernelGGL((k_trsv_ring_r<T, KW, R, TIn, TOut>), dim3(h->nnarrow_pad * ng), dim3(kRingThreads), 0, st,
                       h->rblk, h->nnarrow, h->nnarrow_pad, ng, h->lvl_ptr, h->rfoff, h->rboff, h->frec, h->brec, x,
                       ldx, (T*)h->ws.ry, (int64_t)R * n, z, ldz, done);
    LAUNCHCHK();
}

template <typename T, int R, typename TIn, typename TOut>
void launch_ring_r(ddlr_prec* h, const T* dinv, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                   hipStream_t st, const int* done) {
    switch (h->ring_kw) {
    case 2: launch_ring_rk<T, 2, R, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    case 3: launch_ring_rk<T, 3, R, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done); break;
    default: launch_ring_rk<T, 4, R, TIn, TOut>(h, dinv, nrhs, x, ldx, z, ldz, st, done);
    }
}

// columns per workgroup for an nrhs-column solve: the tuned choice, reduced
// to a power of two that divides nrhs and fits the ring
template <typename T> int ring_r_for(const ddlr_prec* h, int nrhs) {
    int R = 1;
    auto it = h->tune.find(nrhs);
    if (it != h->tune.end()) R = it->second.ring_r;
    if (const char* env = std::getenv("DDLR_RING_R")) R = std::atoi(env);
    while (R > 1 && (nrhs % R != 0 || !ring_r_ok<T>(h, R, nrhs))) R >>= 1;
    return std::max(R, 1);
}

// workgroup size of the one-column ring kernel (tuned, else the smallest eligible)
template <typename T> int ring_nt_for(const ddlr_prec* h, int nrhs) {
    int nt = 0;
    auto it = h->tune.find(nrhs);
    if (it != h->tune.end()) nt = it->second.ring_nt;
    if (const char* env = std::getenv("DDLR_RING_NT")) nt = std::atoi(env);
    if (nt == -1) return -1;  // the plain per-level kernel
    if (nt != 64 && nt != 256 && nt != 512) nt = ring_nt_default(h);
    return ring_nt_ok(h, nt) ? nt : 512;
}

// k_trsv_level_rows for 1..kMaxRhs columns: the power-of-two width that covers nrhs
template <typename T, int kKind, typename TIn, typename TOut>
void launch_level_rows(int a, int e, int nrhs, const int32_t* rp, const int32_t* ci, const T* v, const T* dinv,
                       const TIn* x, int64_t ldx, TOut* z, int64_t ldz, hipStream_t st, const int* done) {
    const dim3 g((e - a + 255) / 256), b(256);
    if (nrhs <= 1)
        hipLaunchKernelGGL((k_trsv_level_rows<T, kKind, TIn, TOut, 1>), g, b, 0, st, a, e, nrhs, rp, ci, v, dinv, x,
                           ldx, z, ldz, done);
    else if (nrhs <= 2)
        hipLaunchKernelGGL((k_trsv_level_rows<T, kKind, TIn, TOut, 2>), g, b, 0, st, a, e, nrhs, rp, ci, v, dinv, x,
                           ldx, z, ldz, done);
    else if (nrhs <= 4)
        hipLaunchKernelGGL((k_trsv_level_rows<T, kKind, TIn, TOut, 4>), g, b, 0, st, a, e, nrhs, rp, ci, v, dinv, x,
                           ldx, z, ldz, done);
    else if (nrhs <= 8)
        hipLaunchKernelGGL((k_trsv_level_rows<T, kKind, TIn, TOut, 8>), g, b, 0, st, a, e, nrhs, rp, ci, v, dinv, x,
                           ldx, z, ldz, done);
    else
        hipLaunchKernelGGL((k_trsv_level_rows<T, kKind, TIn, TOut, kMaxRhs>), g, b, 0, st, a, e, nrhs, rp, ci, v,
                           dinv, x, ldx, z, ldz, done);
}

template <typename T, int kKind, typename TIn, typename TOut>
void launch_iface(ddlr_prec* h, bool rows, int a, int e, int nrhs, int NR, const T* dinv, const TIn* x, int64_t ldx,
                  TOut* z, int64_t ldz, hipStream_t st, const int* done) {
    using PK = typename IfacePk<T>::type;
    const int m = (int)(h->ndev - h->sdev);
    const int32_t* prp = kKind == 1 ? h->iprp_u : h->iprp_l;
    const PK* pk = (const PK*)(kKind == 1 ? h->ipk_u : h->ipk_l);
    T* Y = (T*)h->ws.iy;
    const dim3 b(256);
    if (!rows) {
        hipLaunchKernelGGL((k_iface_cols<T, kKind, TIn, TOut>), dim3((e - a + 255) / 256, NR), b, 0, st, a, e, m, nrhs,
                           NR, prp, pk, dinv, x, ldx, Y, z, ldz, done);
    } else {
        // NC columns per thread: 16-byte vectors of Y (4 FP32 or 2 FP64 values)
        constexpr int NC = sizeof(T) == 4 ? 4 : 2;
        auto grid = [&](int nr) { return dim3((unsigned)(((int64_t)(e - a) * (nr / std::min(nr, NC)) + 255) / 256)); };
        switch (NR) {
        case 1:
            hipLaunchKernelGGL((k_iface_rows<T, kKind, TIn, TOut, 1, 1>), grid(1), b, 0, st, a, e, m, nrhs, prp, pk,
                               dinv, x, ldx, Y, z, ldz, done);
            break;
        case 2:
            hipLaunchKernelGGL((k_iface_rows<T, kKind, TIn, TOut, 2, 2>), grid(2), b, 0, st, a, e, m, nrhs, prp, pk,
                               dinv, x, ldx, Y, z, ldz, done);
            break;
        case 4:
            hipLaunchKernelGGL((k_iface_rows<T, kKind, TIn, TOut, 4, std::min(4, NC)>), grid(4), b, 0, st, a, e, m,
                               nrhs, prp, pk, dinv, x, ldx, Y, z, ldz, done);
            break;
        case 8:
            hipLaunchKernelGGL((k_iface_rows<T, kKind, TIn, TOut, 8, NC>), grid(8), b, 0, st, a, e, m, nrhs, prp, pk,
                               dinv, x, ldx, Y, z, ldz, done);
            break;
        default:
            hipLaunchKernelGGL((k_iface_rows<T, kKind, TIn, TOut, kMaxRhs, NC>), grid(kMaxRhs), b, 0, st, a, e, m,
                               nrhs, prp, pk, dinv, x, ldx, Y, z, ldz, done);
            break;
        }
    }
    LAUNCHCHK();
}

// The interface levels through the private buffer (k_iface_rows / _cols)
template <typename T, typename TIn, typename TOut, typename ByRows>
void iface_levels(ddlr_prec* h, const DevFactors<T>& F, int nrhs, int NR, const TIn* x, int64_t ldx, TOut* z,
                  int64_t ldz, hipStream_t st, const int* done, ByRows&& by_rows) {
    const int nl = (int)h->wide.size();
    for (int l = 0; l < nl; ++l) {
        const int a = h->wide[l].first, e = h->wide[l].second;
        if (l + 1 < nl)
            launch_iface<T, 0, TIn, TOut>(h, by_rows(a, e), a, e, nrhs, NR, F.dinv, x, ldx, z, ldz, st, done);
        else
            launch_iface<T, 2, TIn, TOut>(h, by_rows(a, e), a, e, nrhs, NR, F.dinv, x, ldx, z, ldz, st, done);
    }
    for (int l = nl - 2; l >= 0; --l) {
        const int a = h->wide[l].first, e = h->wide[l].second;
        launch_iface<T, 1, TIn, TOut>(h, by_rows(a, e), a, e, nrhs, NR, F.dinv, x, ldx, z, ldz, st, done);
    }
}

// Interface-block levels (multicolour order): forward levels, the last one
// fused with the diagonal scaling, then backward levels.
template <typename T, typename TIn, typename TOut>
void wide_levels(ddlr_prec* h, const DevFactors<T>& F, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                 hipStream_t st, const int* done) {
    ProfScope ps(h, 1, st);
    const int nl = (int)h->wide.size();
    // levels of at least 256 workgroups of rows take one thread per row for all
    // columns (entries loaded once); smaller ones one thread per (row, column)
    auto by_rows = [&](int a, int e) {
        if (nrhs > kMaxRhs || h->level_kernel == 2) return false;
        return h->level_kernel == 1 || e - a >= 256 * 256;
    };
    int NR = 1;
    while (NR < nrhs) NR <<= 1;
    if (nrhs <= kMaxRhs && h->level_kernel != 2 && h->ipk_l && h->ipk_prec == (sizeof(T) == 8 ? DDLR_FP64 : DDLR_FP32) &&
        h->ws.iy && h->ws.iy_cols >= NR) {
        iface_levels<T, TIn, TOut>(h, F, nrhs, NR, x, ldx, z, ldz, st, done, by_rows);
        return;
    }
    for (int l = 0; l < nl; ++l) {
        const int a = h->wide[l].first, e = h->wide[l].second;
        const bool last = l + 1 == nl;
        if (by_rows(a, e)) {
            if (!last)
                launch_level_rows<T, 0, TIn, TOut>(a, e, nrhs, h->lrp, h->lci, F.lv, F.dinv, x, ldx, z, ldz, st, done);
            else
                launch_level_rows<T, 2, TIn, TOut>(a, e, nrhs, h->lrp, h->lci, F.lv, F.dinv, x, ldx, z, ldz, st, done);
        } else {
            const dim3 g((e - a + 255) / 256, nrhs);
            if (!last)
                hipLaunchKernelGGL((k_trsv_level<T, 0, TIn, TOut>), g, dim3(256), 0, st, a, e, nrhs, h->lrp, h->lci,
                                   F.lv, F.dinv, x, ldx, z, ldz, done);
            else
                hipLaunchKernelGGL((k_trsv_level<T, 2, TIn, TOut>), g, dim3(256), 0, st, a, e, nrhs, h->lrp, h->lci,
                                   F.lv, F.dinv, x, ldx, z, ldz, done);
        }
        LAUNCHCHK();
    }
    for (int l = nl - 2; l >= 0; --l) {
        const int a = h->wide[l].first, e = h->wide[l].second;
        if (by_rows(a, e))
            launch_level_rows<T, 1, TIn, TOut>(a, e, nrhs, h->urp, h->uci, F.uv, F.dinv, x, ldx, z, ldz, st, done);
        else
            hipLaunchKernelGGL((k_trsv_level<T, 1, TIn, TOut>), dim3((e - a + 255) / 256, nrhs), dim3(256), 0, st, a, e,
                               nrhs, h->urp, h->uci, F.uv, F.dinv, x, ldx, z, ldz, done);
        LAUNCHCHK();
    }
}

// E / E^T / C products for 1..kMaxRhs columns: the power-of-two kernel that
// covers nrhs, else the generic one
template <typename T, typename TX>
void csr_mv(int64_t rows, int nrhs, const int32_t* rp, const int32_t* ci, const T* v, const T* w, int64_t ldw,
            const TX* x, int64_t ldx, T* y, int64_t ldy, hipStream_t st, const int* done) {
    const dim3 g(grid_for(rows)), b(256);
    if (nrhs <= 1)
        hipLaunchKernelGGL((k_csr_mv_n<T, TX, 1>), g, b, 0, st, rows, nrhs, rp, ci, v, w, ldw, x, ldx, y, ldy, done);
    else if (nrhs <= 2)
        hipLaunchKernelGGL((k_csr_mv_n<T, TX, 2>), g, b, 0, st, rows, nrhs, rp, ci, v, w, ldw, x, ldx, y, ldy, done);
    else if (nrhs <= 4)
        hipLaunchKernelGGL((k_csr_mv_n<T, TX, 4>), g, b, 0, st, rows, nrhs, rp, ci, v, w, ldw, x, ldx, y, ldy, done);
    else if (nrhs <= 8)
        hipLaunchKernelGGL((k_csr_mv_n<T, TX, 8>), g, b, 0, st, rows, nrhs, rp, ci, v, w, ldw, x, ldx, y, ldy, done);
    else if (nrhs <= kMaxRhs)
        hipLaunchKernelGGL((k_csr_mv_n<T, TX, kMaxRhs>), g, b, 0, st, rows, nrhs, rp, ci, v, w, ldw, x, ldx, y, ldy,
                           done);
    else
        hipLaunchKernelGGL((k_csr_mv<T, TX>), g, b, 0, st, rows, nrhs, rp, ci, v, w, ldw, x, ldx, y, ldy, done);
    LAUNCHCHK();
}

// z = A0^{-1} x, device order (x may equal z when TIn == TOut)
// the interface block is solved apart from the B blocks (level launches or X)
bool has_cpart(const ddlr_prec* h) { return !h->wide.empty() || h->xrp != nullptr; }

// z_C = nu steps of Chebyshev acceleration for C_alpha z = x with the
// block-Jacobi D_alpha (its solves: the interface levels), on the safeguarded
// interval from setup; groups of kMaxRhs columns through the scratch.
template <typename T, typename TIn, typename TOut>
void cheb_dev(ddlr_prec* h, const DevFactors<T>& F, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
              hipStream_t st, const int* done) {
    // (the D_alpha level solves are timed by wide_levels under class 1)
    const int64_t n = h->ndev, s = h->sdev, m = n - s;
    const HostPlan& P = h->plan;
    const double th = 0.5 * (P.ch_hi + P.ch_lo), de = 0.5 * (P.ch_hi - P.ch_lo), sg = th / de;
    T* t = static_cast<T*>(h->ch_t);
    T* r = static_cast<T*>(h->ch_r);
    T* d = static_cast<T*>(h->ch_d);
    T* acc = static_cast<T*>(h->ch_x);
    for (int c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
        const int nr = std::min(kMaxRhs, nrhs - c0);
        const TIn* xc = x + c0 * ldx;
        TOut* zc = z + c0 * ldz;
        const dim3 g = grid2(s, nr);
        wide_levels<T, TIn, T>(h, F, nr, xc, ldx, t, n, st, done);  // t = D^{-1} x
        hipLaunchKernelGGL((k_cheb_first<T, TIn>), g, dim3(256), 0, st, s, xc + m, ldx, t + m, r + m, d + m, acc + m, n,
                           (T)(1.0 / th), done);
        LAUNCHCHK();
        double rho = 1.0 / sg;
        for (int k = 1; k < h->cheb_nu; ++k) {
            csr_mv<T, T>(s, nr, h->crp, h->cci, F.cneg, d + m, n, r + m, n, r + m, n, st, done);  // r -= C d
            const double rn = 1.0 / (2.0 * sg - rho);
            wide_levels<T, T, T>(h, F, nr, r, n, t, n, st, done);  // t = D^{-1} r
            hipLaunchKernelGGL((k_cheb_step<T>), g, dim3(256), 0, st, s, (T)(rn * rho), (T)(2.0 * rn / de), t + m,
                               d + m, acc + m, n, done);
            LAUNCHCHK();
            rho = rn;
        }
        hipLaunchKernelGGL((k_cheb_out<T, TOut>), g, dim3(256), 0, st, s, acc + m, n, zc + m, ldz, done);
        LAUNCHCHK();
    }
}

template <typename T, typename TIn, typename TOut>
void a0_solve_dev(ddlr_prec* h, const DevFactors<T>& F, int nrhs, const TIn* x, int64_t ldx, TOut* z, int64_t ldz,
                  hipStream_t st, const int* done) {
    bool ov = h->overlap;
    if (auto it = h->tune.find(nrhs); it != h->tune.end()) ov = ov && it->second.overlap;
    if (h->ov_override >= 0) ov = h->overlap && h->ov_override;
    const bool fork = has_cpart(h) && h->nnarrow > 0 && ov && h->side;
    hipStream_t cst = st;
    if (fork) {
        HIPCHK(hipEventRecord(h->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
        cst = h->side;
    }
    if (h->cheb_nu > 0) cheb_dev<T, TIn, TOut>(h, F, nrhs, x, ldx, z, ldz, cst, done);
    else if (!h->wide.empty()) wide_levels<T, TIn, TOut>(h, F, nrhs, x, ldx, z, ldz, cst, done);
    if (h->xrp) {  // z_C = X x_C
        ProfScope ps(h, 1, cst);
        const int64_t m = h->ndev - h->sdev;
        for (int c0 = 0; c0 < nrhs; c0 += kMaxRhs) {  // the kernel keeps up to kMaxRhs columns in registers
            hipLaunchKernelGGL((k_cinv_sell<T, TIn, TOut>), dim3((h->sdev + 255) / 256), dim3(256), 0, cst, h->sdev,
                               std::min(kMaxRhs, nrhs - c0), h->xrp, h->xrow, h->xci, F.xv, x + m + c0 * ldx, ldx,
                               z + m + c0 * ldz, ldz, done);
            LAUNCHCHK();
        }
    }
    if (h->nnarrow > 0) {
        ProfScope ps(h, 0, st);
        if (ring_ready<T>(h) && ring_nt_for<T>(h, nrhs) > 0) {
            switch (ring_r_for<T>(h, nrhs)) {
            case 2: launch_ring_r<T, 2, TIn, TOut>(h, F.dinv, nrhs, x, ldx, z, ldz, st, done); break;
            case 4: launch_ring_r<T, 4, TIn, TOut>(h, F.dinv, nrhs, x, ldx, z, ldz, st, done); break;
            case 8: launch_ring_r<T, 8, TIn, TOut>(h, F.dinv, nrhs, x, ldx, z, ldz, st, done); break;
            default:
                if (ring_nt_for<T>(h, nrhs) == 512 && rec_ok<T>(h, 1, nrhs))
                    launch_ring_r<T, 1, TIn, TOut>(h, F.dinv, nrhs, x, ldx, z, ldz, st, done);
                else
                    launch_ring<T, TIn, TOut>(h, F.dinv, nrhs, x, ldx, z, ldz, st, done);
            }
        } else {
            hipLaunchKernelGGL((k_trsv_narrow<T, TIn, TOut>), dim3(h->nnarrow_pad * nrhs), dim3(256), 0, st, h->blk,
                               h->nnarrow, h->nnarrow_pad, nrhs, h->lvl_ptr, h->lrp, h->lci, F.lv, h->urp, h->uci,
                               F.uv, F.dinv, x, ldx, z, ldz, done);
            LAUNCHCHK();
        }
    }
    if (fork) {
        HIPCHK(hipEventRecord(h->ev_join, h->side));
        HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
    }
}

// ------------------------------------------------------------ low-rank part

// Calls f(std::integral_constant<int, t>) for t = ntiles in 1..8 (16-column
// tiles of U_k), so the low-rank kernels get the tile count at compile time.
template <typename F> void with_tiles(int ntiles, F&& f) {
    switch (ntiles) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    default: f(std::integral_constant<int, 8>{});
    }
}

// coef = d .* (U^T y) (mode 1) or H (U^T y) (mode 2)
template <typename T, typename TY>
void lr_coef(ddlr_prec* h, const T* U, int64_t rows, int nrhs, const TY* y, int64_t ldy, int mode, hipStream_t st,
             const int* done) {
    Workspace& W = h->ws;
    const int k = h->k;
    ProfScope ps(h, 3, st);
    if (h->ubt && std::is_same<T, float>::value)
        hipLaunchKernelGGL((k_lr_reduce_bf16<TY>), dim3(kLrBlocks), dim3(256), 0, st, rows, k, nrhs, h->ubt, y, ldy,
                           W.part, done);
    else if (h->lr_plain)
        hipLaunchKernelGGL((k_lr_reduce<T, TY>), dim3(kLrBlocks), dim3(256), 0, st, rows, k, nrhs, U, y, ldy, W.part,
                           done);
    else if (factors<T>(h).Ut && factors<T>(h).U == U)
        with_tiles(k >> 4, [&](auto nt) {
            hipLaunchKernelGGL((k_lr_reduce_t<T, TY, decltype(nt)::value>), dim3(kLrBlocks), dim3(256), 0, st, rows,
                               k, nrhs, factors<T>(h).Ut, y, ldy, W.part, done);
        });
    else
        hipLaunchKernelGGL((k_lr_reduce_mfma<T, TY>), dim3(kLrBlocks), dim3(256), 0, st, rows, k, nrhs, U, y, ldy,
                           W.part, done);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_cols, dim3(nrhs * k), dim3(256), 0, st, kLrBlocks, nrhs * k, W.part, W.lrsum, done);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_lr_coef, dim3(1), dim3(256), 0, st, k, nrhs, W.lrsum, mode, h->dvec, h->Hk, W.coef, done);
    LAUNCHCHK();
}

// out = beta in + U coef
template <typename T, typename TIO>
void lr_expand(ddlr_prec* h, const T* U, int64_t rows, int nrhs, double beta, const TIO* in, int64_t ldin, TIO* out,
               int64_t ldout, hipStream_t st, const int* done) {
    ProfScope ps(h, 3, st);
    if (h->ubr && std::is_same<T, float>::value) {
        const int64_t tiles = (rows + 15) / 16;
        hipLaunchKernelGGL((k_lr_expand_bf16<TIO>), dim3(grid_for(tiles, 4)), dim3(256), 0, st, rows, h->k, h->ukp,
                           nrhs, h->ubr, h->ws.coef, beta, in, ldin, out, ldout, done);
    } else if (h->lr_plain) {
        hipLaunchKernelGGL((k_lr_expand<T, TIO>), dim3(grid_for(rows)), dim3(256), 0, st, rows, h->k, nrhs, U,
                           h->ws.coef, beta, in, ldin, out, ldout, done);
    } else if (h->k >= 16 && h->k % 16 == 0 && h->k <= 128) {
        const int64_t tiles = (rows + 15) / 16;
        with_tiles(h->k >> 4, [&](auto nt) {
            hipLaunchKernelGGL((k_lr_expand_v<T, TIO, decltype(nt)::value>), dim3(grid_for(tiles, 4)), dim3(256), 0,
                               st, rows, h->k, nrhs, U, h->ws.coef, beta, in, ldin, out, ldout, done);
        });
    } else {
        const int64_t tiles = (rows + 15) / 16;
        hipLaunchKernelGGL((k_lr_expand_mfma<T, TIO>), dim3(grid_for(tiles, 4)), dim3(256), 0, st, rows, h->k, nrhs,
                           U, h->ws.coef, beta, in, ldin, out, ldout, done);
    }
    LAUNCHCHK();
}

// ------------------------------------------------------------ preconditioner

// out = M^{-1} in (device order); I/O in double, preconditioner arithmetic in T.
// Precision changes happen inside the kernels that read the input and write
// the output (no separate cast passes).  DDLR-1 (eq. Mprec with eq. gkt,
// organised as Algorithm alg:prec1 so that only two A0 solves run):
//   a0_solve_dev (double in, T out)        block + interface triangular solves
//   csr_mv over E^T                         interface gather into ys
//   lr_coef / lr_expand (MFMA)              ws = c0 ys + U_k (d .* (U_k^T ys))
//   csr_mv over E, input added in the pass  a2 = in + E ws (one fused pass)
//   a0_solve_dev (T in, double out)         the second pair of sweeps
template <typename T>
void apply_dev_T(ddlr_prec* h, int nrhs, const double* in, int64_t ldin, double* out, int64_t ldout, hipStream_t st,
                 const int* done) {
    const DevFactors<T>& F = factors<T>(h);
    Workspace& W = h->ws;
    const int64_t n = h->ndev, s = h->sdev;
    if (h->variant == DDLR_1) {
        T* a1 = (T*)W.a1;
        T* a2 = (T*)W.a2;
        T* ys = (T*)W.ys;
        T* wsv = (T*)W.ws;
        a0_solve_dev<T, double, T>(h, F, nrhs, in, ldin, a1, n, st, done);
        csr_mv<T, T>(s, nrhs, h->etrp, h->etci, F.etv, a1, n, (const T*)nullptr, 0, ys, s, st, done);
        if (h->batch) {  // per system of a batch (one column)
            ProfScope ps(h, 3, st);
            hipLaunchKernelGGL(k_seg_lr_coef<T>, dim3(h->nsys), dim3(256), 0, st, h->seg_soff, h->k, F.U, ys, h->dvecs,
                               W.coef, done);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_seg_lr_expand<T>, dim3(kSegChunks, h->nsys), dim3(256), 0, st, h->seg_soff, h->k, F.U,
                               W.coef, h->c0s, ys, wsv, done);
            LAUNCHCHK();
        } else {
            lr_coef<T, T>(h, F.U, s, nrhs, ys, s, 1, st, done);
            lr_expand<T, T>(h, F.U, s, nrhs, h->c0, ys, s, wsv, s, st, done);
        }
        csr_mv<T, double>(n, nrhs, h->erp, h->eci, F.ev, wsv, s, in, ldin, a2, n, st, done);
        a0_solve_dev<T, T, double>(h, F, nrhs, a2, n, out, ldout, st, done);
    } else if (h->variant == DDLR_2) {
        a0_solve_dev<T, double, double>(h, F, nrhs, in, ldin, out, ldout, st, done);
        lr_coef<T, double>(h, F.U, n, nrhs, in, ldin, 2, st, done);
        lr_expand<T, double>(h, F.U, n, nrhs, 1.0, out, ldout, out, ldout, st, done);
    } else {
        a0_solve_dev<T, double, double>(h, F, nrhs, in, ldin, out, ldout, st, done);
    }
}

// out = M^{-1} in for double device-order columns
void apply_dev(ddlr_prec* h, int nrhs, const double* in, int64_t ldin, double* out, int64_t ldout, hipStream_t st,
               const int* done) {
    if (h->precision == DDLR_FP64) apply_dev_T<double>(h, nrhs, in, ldin, out, ldout, st, done);
    else apply_dev_T<float>(h, nrhs, in, ldin, out, ldout, st, done);
}

// Calls f(col, val) with the SELL arrays in their stored types.
template <typename F> void with_sell(const ddlr_prec* h, F&& f) {
    if (h->sell_cold) {
        if (h->sell_valf) f(h->sell_cold, h->sell_valf);
        else f(h->sell_cold, h->sell_val);
    } else {
        if (h->sell_valf) f(h->sell_col, h->sell_valf);
        else f(h->sell_col, h->sell_val);
    }
}

void spmv_dev(ddlr_prec* h, int nrhs, const double* x, int64_t ldx, double* y, int64_t ldy, double* part,
              hipStream_t st, const int* done) {
    const int64_t n = h->ndev;
    ProfScope ps(h, 2, st);
    const int64_t chunks = (n + 255) / 256;
    with_sell(h, [&](auto col, auto val) {
        using IT = std::remove_const_t<std::remove_pointer_t<decltype(col)>>;
        using VT = std::remove_const_t<std::remove_pointer_t<decltype(val)>>;
        hipLaunchKernelGGL((k_spmv_sell<VT, IT>), dim3((chunks + 7) / 8 * 8), dim3(256), 0, st, n, nrhs, h->sell_ptr,
                           col, val, x, ldx, y, ldy, part, done);
    });
    LAUNCHCHK();
}

// y = A x with x interleaved (x[i * S + r], S = lane_stride(nrhs))
// S: the interleave stride of x (0: lane_stride(nrhs))
void spmv_il_dev(ddlr_prec* h, int nrhs, const double* x, double* y, int64_t ldy, double* part, hipStream_t st,
                 const int* done, int S = 0) {
    const int64_t n = h->ndev;
    ProfScope ps(h, 2, st);
    const int64_t chunks = (n + 255) / 256;
    const dim3 grid((chunks + 7) / 8 * 8), blk(256);
    if (!S) S = lane_stride(nrhs);
    if (h->sell_pk) {
        const int32_t* nc = nullptr;
        const float* nv = nullptr;
        switch (S) {
#define DDLR_SPMV_PK(SS)                                                                                             \
    case SS:                                                                                                         \
        hipLaunchKernelGGL((k_spmv_sell_il<SS, float, int32_t, true>), grid, blk, 0, st, n, nrhs, h->sell_ptr, nc, nv, \
                           x, y, ldy, part, done, h->sell_pk);                                                       \
        break;
            DDLR_SPMV_PK(1)
            DDLR_SPMV_PK(2)
            DDLR_SPMV_PK(4)
            DDLR_SPMV_PK(8)
            DDLR_SPMV_PK(16)
#undef DDLR_SPMV_PK
        default: throw SetupError{DDLR_E_INVALID, "CG runs at most 16 lanes per launch"};
        }
        LAUNCHCHK();
        return;
    }
    with_sell(h, [&](auto col, auto val) {
        using IT = std::remove_const_t<std::remove_pointer_t<decltype(col)>>;
        using VT = std::remove_const_t<std::remove_pointer_t<decltype(val)>>;
        switch (S) {
        case 1:
            hipLaunchKernelGGL((k_spmv_sell_il<1, VT, IT>), grid, blk, 0, st, n, nrhs, h->sell_ptr, col, val, x, y, ldy,
                               part, done, nullptr);
            break;
        case 2:
            hipLaunchKernelGGL((k_spmv_sell_il<2, VT, IT>), grid, blk, 0, st, n, nrhs, h->sell_ptr, col, val, x, y, ldy,
                               part, done, nullptr);
            break;
        case 4:
            hipLaunchKernelGGL((k_spmv_sell_il<4, VT, IT>), grid, blk, 0, st, n, nrhs, h->sell_ptr, col, val, x, y, ldy,
                               part, done, nullptr);
            break;
        case 8:
            hipLaunchKernelGGL((k_spmv_sell_il<8, VT, IT>), grid, blk, 0, st, n, nrhs, h->sell_ptr, col, val, x, y, ldy,
                               part, done, nullptr);
            break;
        default:
            hipLaunchKernelGGL((k_spmv_sell_il<16, VT, IT>), grid, blk, 0, st, n, nrhs, h->sell_ptr, col, val, x, y,
                               ldy, part, done, nullptr);
            break;
        }
    });
    LAUNCHCHK();
}

// x += alpha p ; r -= alpha q per lane (p interleaved)
void cg_xr_dev(ddlr_prec* h, int nr, int S, hipStream_t st) {
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    const dim3 grid(kRedBlocks), blk(256);
    switch (S) {
        case 1:
            hipLaunchKernelGGL(k_cg_xr<1>, grid, blk, 0, st, n, nr, W.lanes, W.p, W.q, W.x, W.r, n, W.part, W.done);
            break;
        case 2:
            hipLaunchKernelGGL(k_cg_xr<2>, grid, blk, 0, st, n, nr, W.lanes, W.p, W.q, W.x, W.r, n, W.part, W.done);
            break;
        case 4:
            hipLaunchKernelGGL(k_cg_xr<4>, grid, blk, 0, st, n, nr, W.lanes, W.p, W.q, W.x, W.r, n, W.part, W.done);
            break;
        case 8:
            hipLaunchKernelGGL(k_cg_xr<8>, grid, blk, 0, st, n, nr, W.lanes, W.p, W.q, W.x, W.r, n, W.part, W.done);
            break;
        default:
            hipLaunchKernelGGL(k_cg_xr<16>, grid, blk, 0, st, n, nr, W.lanes, W.p, W.q, W.x, W.r, n, W.part, W.done);
            break;
    }
    LAUNCHCHK();
}

// Streams of the lane-phase CG: the CG stream (private to the library, so
// graph capture never touches a caller's stream) and the x-update stream,
// taken from the device's shared set (created outside any graph capture).
void ensure_cg_streams(ddlr_prec* h) {
    if (h->x_st) return;
    DevStreams& D = dev_streams(h->device);
    h->cg_st = D.cg;
    h->x_st = D.x;
    HIPCHK(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_xf, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_xj, hipEventDisableTiming));
}

template <int S> void cg_split_launch(ddlr_prec* h, int nr, hipStream_t st) {
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    hipLaunchKernelGGL(k_cg_r<S>, dim3(kRedBlocks), dim3(256), 0, st, n, nr, W.lanes, W.q, W.r, n, W.xa, W.part,
                       W.done);
    LAUNCHCHK();
    HIPCHK(hipEventRecord(h->ev_xf, st));
    HIPCHK(hipStreamWaitEvent(h->x_st, h->ev_xf, 0));
    hipLaunchKernelGGL(k_cg_x<S>, dim3(grid_for(n)), dim3(256), 0, h->x_st, n, nr, W.xa, W.p, W.x, n);
    LAUNCHCHK();
    HIPCHK(hipEventRecord(h->ev_xj, h->x_st));
}

// r -= alpha q (with r.r partials and the step record xa) on st
void cg_r_dev(ddlr_prec* h, int nr, int S, hipStream_t st) {
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    const dim3 g(kRedBlocks), b(256);
    switch (S) {
    case 1: hipLaunchKernelGGL(k_cg_r<1>, g, b, 0, st, n, nr, W.lanes, W.q, W.r, n, W.xa, W.part, W.done); break;
    case 2: hipLaunchKernelGGL(k_cg_r<2>, g, b, 0, st, n, nr, W.lanes, W.q, W.r, n, W.xa, W.part, W.done); break;
    case 4: hipLaunchKernelGGL(k_cg_r<4>, g, b, 0, st, n, nr, W.lanes, W.q, W.r, n, W.xa, W.part, W.done); break;
    case 8: hipLaunchKernelGGL(k_cg_r<8>, g, b, 0, st, n, nr, W.lanes, W.q, W.r, n, W.xa, W.part, W.done); break;
    default: hipLaunchKernelGGL(k_cg_r<16>, g, b, 0, st, n, nr, W.lanes, W.q, W.r, n, W.xa, W.part, W.done); break;
    }
    LAUNCHCHK();
}

// r -= alpha q (with r.r partials) on st; x += alpha p forked to the x stream
// (joined by cg_join before p changes)
void cg_split_dev(ddlr_prec* h, int nr, int S, hipStream_t st) {
    switch (S) {
    case 1: cg_split_launch<1>(h, nr, st); break;
    case 2: cg_split_launch<2>(h, nr, st); break;
    case 4: cg_split_launch<4>(h, nr, st); break;
    case 8: cg_split_launch<8>(h, nr, st); break;
    default: cg_split_launch<16>(h, nr, st); break;
    }
}

// sums[r] = a_r . b_r
void dot_dev(ddlr_prec* h, int nrhs, const double* a, const double* b, int64_t ld, hipStream_t st, const int* done) {
    Workspace& W = h->ws;
    hipLaunchKernelGGL((k_dot<double, double>), dim3(kRedBlocks), dim3(256), 0, st, h->ndev, nrhs, a, ld, b, ld,
                       W.part, done);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_cols, dim3(nrhs), dim3(256), 0, st, kRedBlocks, nrhs, W.part, W.sums, done);
    LAUNCHCHK();
}

// Tile-ordered copies of U_k for the wide-load reduction (k a multiple of 16)
void make_tiled_basis(ddlr_prec* h) {
    h->f64.Ut = nullptr;
    h->f32.Ut = nullptr;
    if (h->k < 16 || h->k % 16 != 0 || h->k > 128) return;
    const int64_t rows = h->urows;
    const int64_t total = (rows + 15) / 16 * 16 * h->k;
    if (h->f64.U) {
        h->f64.Ut = h->lrmem.alloc<double>((size_t)total);
        hipLaunchKernelGGL(k_make_ut<double>, dim3(grid_for(total)), dim3(256), 0, nullptr, rows, h->k, h->f64.U,
                           h->f64.Ut);
        LAUNCHCHK();
    }
    if (h->f32.U) {
        h->f32.Ut = h->lrmem.alloc<float>((size_t)total);
        hipLaunchKernelGGL(k_make_ut<float>, dim3(grid_for(total)), dim3(256), 0, nullptr, rows, h->k, h->f32.U,
                           h->f32.Ut);
        LAUNCHCHK();
    }
}

// BF16 copies of U_k for the DDLR_FP32_UK_BF16 configuration
void make_bf16_basis(ddlr_prec* h) {
    if (h->precision != DDLR_FP32_UK_BF16 || !h->f64.U || h->k < 1) return;
    const int64_t rows = h->urows;
    const int k = h->k;
    h->ukp = (k + 31) / 32 * 32;
    h->uktiles = (k + 15) / 16;
    const int64_t nb = (rows + 31) / 32;
    h->ubt = h->lrmem.alloc<__bf16>((size_t)nb * h->uktiles * 512);
    h->ubr = h->lrmem.alloc<__bf16>((size_t)rows * h->ukp);
    hipLaunchKernelGGL(k_make_bf16, dim3(grid_for(nb * h->uktiles * 512 + rows * h->ukp)), dim3(256), 0, nullptr, rows,
                       k, h->f64.U, h->ukp, h->uktiles, h->ubr, h->ubt);
    LAUNCHCHK();
}

// ------------------------------------------------------------ Lanczos build

// Lanczos run on E^T A0^{-1} E (DDLR-1) or E^T A0^{-2} E (DDLR-2), Sec. 4.4 (sec:Lan),
// kept on the device so it can be continued (improving a given
// preconditioner by more steps and a larger k).
void lanczos_reserve(ddlr_prec* h, int cap) {
    LanczosRun& R = h->lrun;
    if (cap <= R.cap) return;
    const int64_t n = h->plan.n, s = h->plan.s;
    DMem nm;
    nm.budget = budget_of(h);
    double* Q = nm.alloc<double>((size_t)s * (cap + 1));
    double* al = nm.alloc<double>(cap);
    double* be = nm.alloc<double>(cap);
    double* sc = nm.alloc<double>(4);
    if (R.Q) {
        HIPCHK(hipMemcpy(Q, R.Q, sizeof(double) * (size_t)s * (R.steps + 1), hipMemcpyDeviceToDevice));
        if (R.steps > 0) {
            HIPCHK(hipMemcpy(al, R.alpha, sizeof(double) * R.steps, hipMemcpyDeviceToDevice));
            HIPCHK(hipMemcpy(be, R.beta, sizeof(double) * R.steps, hipMemcpyDeviceToDevice));
        }
        HIPCHK(hipMemcpy(sc, R.sc, sizeof(double) * 4, hipMemcpyDeviceToDevice));
    } else {
        HIPCHK(hipMemset(sc, 0, sizeof(double) * 4));
    }
    R.w = nm.alloc<double>(s);
    R.t1 = nm.alloc<double>(n);
    R.t2 = nm.alloc<double>(n);
    R.part = nm.alloc<double>((size_t)kRedBlocks * (cap + 1));
    R.csum = nm.alloc<double>(cap + 1);
    const size_t orow = (size_t)cap + 2;
    double* om = nm.alloc<double>(3 * orow + 1);
    int* pst = nm.alloc<int>((size_t)cap + 2);
    HIPCHK(hipMemset(om, 0, sizeof(double) * (3 * orow + 1)));
    HIPCHK(hipMemset(pst, 0, sizeof(int) * ((size_t)cap + 2)));
    if (R.om) {
        const size_t oold = (size_t)R.cap + 2;
        for (int r = 0; r < 3; ++r)
            HIPCHK(hipMemcpy(om + r * orow, R.om + r * oold, sizeof(double) * oold, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(om + 3 * orow, R.om + 3 * oold, sizeof(double), hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(pst, R.pst, sizeof(int) * ((size_t)R.steps + 2), hipMemcpyDeviceToDevice));
    }
    HIPCHK(hipDeviceSynchronize());
    R.mem.release();
    R.mem = std::move(nm);
    R.Q = Q;
    R.alpha = al;
    R.beta = be;
    R.sc = sc;
    R.om = om;
    R.pst = pst;
    R.cap = cap;
}

void lanczos_start(ddlr_prec* h, const double* v0_user, uint64_t seed) {
    HostPlan& P = h->plan;
    const int64_t n = P.n, s = P.s, mI = P.m;
    // start vector in device interface order
    std::vector<double> q0(s);
    std::vector<int32_t> pd(n);
    for (int64_t d = 0; d < n; ++d) pd[d] = P.perm[P.dev2int[d]];
    if (v0_user) {
        for (int64_t j = 0; j < s; ++j) q0[j] = v0_user[pd[mI + j]];
    } else {
        // SplitMix64 (Steele, Lea & Flood 2014) keyed by seed and user row
        for (int64_t j = 0; j < s; ++j) {
            uint64_t z = seed * 0x9E3779B97F4A7C15ULL + (uint64_t)(pd[mI + j] + 1) * 0xBF58476D1CE4E5B9ULL;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
            z ^= z >> 31;
            q0[j] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
        }
    }
    double nq = 0.0;
    for (double v : q0) nq += v * v;
    nq = std::sqrt(nq);
    if (!(nq > 0.0)) throw SetupError{DDLR_E_INVALID, "Lanczos start vector is zero on the interface"};
    for (double& v : q0) v /= nq;
    LanczosRun& R = h->lrun;
    R.steps = 0;
    R.broke = false;
    R.lvariant = h->variant;
    R.ha.clear();
    R.hb.clear();
    R.hf.clear();
    lanczos_reserve(h, 1);
    HIPCHK(hipMemcpy(R.Q, q0.data(), s * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(R.sc, 0, sizeof(double) * 4));
    // omega estimates: q_0^T q_0 = 1 in the row of step 0, ||T|| estimate 0,
    // no forced step
    const size_t orow = (size_t)R.cap + 2;
    HIPCHK(hipMemset(R.om, 0, sizeof(double) * (3 * orow + 1)));
    HIPCHK(hipMemset(R.pst, 0, sizeof(int) * orow));
    const double one = 1.0;
    HIPCHK(hipMemcpy(R.om, &one, sizeof(double), hipMemcpyHostToDevice));
}

// Sum of the k largest eigenvalues of the leading j x j block of T
// (the sigma of eq. converge).
double ritz_top_sum(const std::vector<double>& ta, const std::vector<double>& tb, int j, int k) {
    std::vector<double> ev, Z;
    tridiag_eig(j, ta.data(), tb.data(), ev, Z);
    std::sort(ev.begin(), ev.end(), [](double a, double b) { return a > b; });
    double sum = 0.0;
    for (int c = 0; c < k && c < j; ++c) sum += ev[c];
    return sum;
}

// Copies alpha / beta of the run to the host and cuts it at the first
// breakdown (beta_j <= 1e-12 max_{i<=j} |alpha_i|, that step included).
void lanczos_sync(ddlr_prec* h, int done_steps) {
    LanczosRun& R = h->lrun;
    R.ha.resize(done_steps);
    R.hb.resize(done_steps);
    R.hf.assign(done_steps, 0);
    HIPCHK(hipMemcpy(R.ha.data(), R.alpha, done_steps * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(R.hb.data(), R.beta, done_steps * sizeof(double), hipMemcpyDeviceToHost));
    if (R.reorth == DDLR_REORTH_PARTIAL && done_steps > 0)
        HIPCHK(hipMemcpy(R.hf.data(), R.pst + 2, done_steps * sizeof(int), hipMemcpyDeviceToHost));
    double am = 0.0;
    R.steps = done_steps;
    for (int j = 0; j < done_steps; ++j) {
        am = std::max(am, std::fabs(R.ha[j]));
        if (R.hb[j] <= 1e-12 * am) {
            R.steps = j + 1;
            R.broke = true;
            break;
        }
    }
    R.ha.resize(R.steps);
    R.hb.resize(R.steps);
    R.hf.resize(R.steps);
}

// Continues the run up to m_max steps.  With check > 0 it stops at the first
// step m that is a multiple of check (m >= k+1) where the sums of the k
// largest Ritz values of T_{m-1} and T_m satisfy eq. (converge) with eps.
void lanczos_advance(ddlr_prec* h, int m_max, int check, double eps, int k) {
    LanczosRun& R = h->lrun;
    const int64_t n = h->plan.n, s = h->plan.s;
    m_max = (int)std::min<int64_t>(m_max, s);
    if (R.broke || R.steps >= m_max) return;
    lanczos_reserve(h, m_max);
    hipStream_t st = nullptr;
    double* Q = R.Q;
    double* w = R.w;
    double* t1 = R.t1;
    double* t2 = R.t2;
    double* alpha = R.alpha;
    double* beta = R.beta;
    double* part = R.part;
    double* csum = R.csum;
    double* amax = R.sc;
    double* inv = R.sc + 1;
    double* sum1 = R.sc + 2;
    const int gs = grid_for(s, 256, kRedBlocks);
    for (int j = R.steps; j < m_max; ++j) {
        double* qj = Q + (size_t)j * s;
        // w = Op q_j : E, A0^{-1} (twice for DDLR-2), E^T
        hipLaunchKernelGGL(k_csr_mv<double>, dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->erp, h->eci, h->f64.ev, qj,
                           s, (const double*)nullptr, 0, t1, n, nullptr);
        LAUNCHCHK();
        a0_solve_dev<double, double, double>(h, h->f64, 1, t1, n, t2, n, st, nullptr);
        const double* src = t2;
        if (R.lvariant == DDLR_2) {
            a0_solve_dev<double, double, double>(h, h->f64, 1, t2, n, t1, n, st, nullptr);
            src = t1;
        }
        hipLaunchKernelGGL(k_csr_mv<double>, dim3(grid_for(s)), dim3(256), 0, st, s, 1, h->etrp, h->etci, h->f64.etv,
                           src, n, (const double*)nullptr, 0, w, s, nullptr);
        LAUNCHCHK();
        // alpha_j = q_j . w
        hipLaunchKernelGGL((k_dot<double, double>), dim3(gs), dim3(256), 0, st, s, 1, qj, s, w, s, part, nullptr);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, st, gs, 1, part, sum1, nullptr);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_lanczos_scalar, dim3(1), dim3(64), 0, st, sum1, alpha + j, 0, amax, inv,
                           (const int*)nullptr);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_lanczos_3term, dim3(gs), dim3(256), 0, st, s, j, Q, s, alpha, beta, w);
        LAUNCHCHK();
        // Full reorthogonalisation: classical Gram-Schmidt twice at every step.
        // Partial: ||w|| first, Simon's omega recurrence decides on the device
        // whether this step is reorthogonalised (skip = 0); the skipped
        // kernels return at once and beta_j keeps the norm already taken.
        const int* skip = nullptr;
        if (R.reorth == DDLR_REORTH_PARTIAL) {
            hipLaunchKernelGGL((k_dot<double, double>), dim3(gs), dim3(256), 0, st, s, 1, w, s, w, s, part, nullptr);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, st, gs, 1, part, sum1, nullptr);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_lanczos_scalar, dim3(1), dim3(64), 0, st, sum1, beta + j, 1, amax, inv,
                               (const int*)nullptr);
            LAUNCHCHK();
            const size_t orow = (size_t)R.cap + 2;
            double* om_cur = R.om + (size_t)(j % 3) * orow;
            double* om_prev = R.om + (size_t)((j + 2) % 3) * orow;
            double* om_new = R.om + (size_t)((j + 1) % 3) * orow;
            hipLaunchKernelGGL(k_pro_omega, dim3(1), dim3(1024), 0, st, j, s, alpha, beta, beta + j, amax, om_prev,
                               om_cur, om_new, R.om + 3 * orow, R.pst, R.pst + 2);
            LAUNCHCHK();
            skip = R.pst + 1;
        }
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_multidot, dim3(gs), dim3(256), 0, st, s, j + 1, Q, s, w, part, skip);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_reduce_cols, dim3(j + 1), dim3(256), 0, st, gs, j + 1, part, csum, skip);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_gemv_sub, dim3(gs), dim3(256), 0, st, s, j + 1, Q, s, csum, w, skip);
            LAUNCHCHK();
        }
        // beta_j = ||w||, q_{j+1} = w / beta_j
        hipLaunchKernelGGL((k_dot<double, double>), dim3(gs), dim3(256), 0, st, s, 1, w, s, w, s, part, skip);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, st, gs, 1, part, sum1, skip);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_lanczos_scalar, dim3(1), dim3(64), 0, st, sum1, beta + j, 1, amax, inv, skip);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_scale_to, dim3(gs), dim3(256), 0, st, s, w, inv, Q + (size_t)(j + 1) * s);
        LAUNCHCHK();
        const int m = j + 1;
        if (check > 0 && m % check == 0 && m >= k + 1) {
            lanczos_sync(h, m);
            if (R.broke) return;
            const double sp = ritz_top_sum(R.ha, R.hb, m - 1, k), sm = ritz_top_sum(R.ha, R.hb, m, k);
            if (std::fabs((sm - sp) / sp) < eps) return;
        }
    }
    lanczos_sync(h, m_max);
}

// Reduced-precision copies and the MFMA/BF16 layouts of U_k
void lowrank_copies(ddlr_prec* h, int k) {
    hipStream_t st = nullptr;
    if (h->precision != DDLR_FP64) {
        h->f32.U = h->lrmem.alloc<float>((size_t)h->urows * k);
        hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(h->urows * k)), dim3(256), 0, st, h->urows * k, 1,
                           h->f64.U, (int64_t)0, h->f32.U, (int64_t)0, nullptr);
        LAUNCHCHK();
    }
    make_bf16_basis(h);
    make_tiled_basis(h);
}

// DDLR-2 from U_k (column-major n x k, device order) and EV = E V_k:
// K = U_k^T E V_k, H_k = (I - sym(K))^{-1} by Cholesky (not SPD: error), U_k
// stored row-major.
void ddlr2_finish(ddlr_prec* h, int k, const double* Ucm, const double* EV, DMem& tmp) {
    const int64_t n = h->plan.n;
    hipStream_t st = nullptr;
    h->urows = n;
    const int gblk = 512;
    double* gp = tmp.alloc<double>((size_t)gblk * k * k);
    hipLaunchKernelGGL(k_gram, dim3(gblk), dim3(256), 0, st, n, k, Ucm, n, EV, n, gp);
    LAUNCHCHK();
    std::vector<double> gh((size_t)gblk * k * k);
    HIPCHK(hipMemcpy(gh.data(), gp, gh.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> K((size_t)k * k, 0.0);
    for (int b = 0; b < gblk; ++b)
        for (int q = 0; q < k * k; ++q) K[q] += gh[(size_t)b * k * k + q];
    // I - (K + K^T)/2, Cholesky (lower, column-major), then its inverse
    std::vector<double> Mx((size_t)k * k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i)
            Mx[i + j * k] = (i == j ? 1.0 : 0.0) - 0.5 * (K[i * k + j] + K[j * k + i]);
    for (int j = 0; j < k; ++j) {
        double d = Mx[j + j * k];
        for (int t = 0; t < j; ++t) d -= Mx[j + t * k] * Mx[j + t * k];
        if (!(d > 0.0)) {
            tmp.release();
            throw SetupError{DDLR_E_NOT_SPD, "I - U_k^T E V_k is not SPD (DDLR-2 preconditioner not SPD)"};
        }
        d = std::sqrt(d);
        Mx[j + j * k] = d;
        for (int i = j + 1; i < k; ++i) {
            double v = Mx[i + j * k];
            for (int t = 0; t < j; ++t) v -= Mx[i + t * k] * Mx[j + t * k];
            Mx[i + j * k] = v / d;
        }
    }
    h->H_h.assign((size_t)k * k, 0.0);
    for (int c = 0; c < k; ++c) {
        std::vector<double> e(k, 0.0);
        e[c] = 1.0;
        for (int i = 0; i < k; ++i) {
            double v = e[i];
            for (int t = 0; t < i; ++t) v -= Mx[i + t * k] * e[t];
            e[i] = v / Mx[i + i * k];
        }
        for (int i = k - 1; i >= 0; --i) {
            double v = e[i];
            for (int t = i + 1; t < k; ++t) v -= Mx[t + i * k] * e[t];
            e[i] = v / Mx[i + i * k];
        }
        for (int i = 0; i < k; ++i) h->H_h[i + (size_t)c * k] = e[i];
    }
    h->spd = h->pivots_positive;
    h->f64.U = h->lrmem.alloc<double>((size_t)n * k);
    hipLaunchKernelGGL(k_to_rowmajor<double>, dim3(grid_for(n * k)), dim3(256), 0, st, n, k, Ucm, n, h->f64.U);
    LAUNCHCHK();
    h->Hk = h->lrmem.upload(h->H_h);
    h->theta = 0.0;
    h->c0 = 0.0;
}

// U_k and G_k^{-1} (DDLR-1) or H_k (DDLR-2) of rank k from the run's Ritz pairs.
void lanczos_finish(ddlr_prec* h, int k, int theta_mode) {
    HostPlan& P = h->plan;
    const int64_t n = P.n, s = P.s;
    LanczosRun& R = h->lrun;
    hipStream_t st = nullptr;
    const int meff = R.steps;
    const double* Q = R.Q;
    h->ta = R.ha;
    h->tb = R.hb;
    h->lreorth = R.reorth;
    if (R.reorth == DDLR_REORTH_PARTIAL) h->rflags = R.hf;
    else h->rflags.assign(meff, 1);
    h->msteps = meff;
    h->theta_mode = theta_mode;
    drop_graphs(h);  // captured kernels hold the low-rank pointers
    DMem tmp;
    tmp.budget = budget_of(h);
    if (meff < k + 1)
        throw SetupError{DDLR_E_LANCZOS, "Lanczos broke down after " + std::to_string(meff) + " steps (k+1 = " +
                                             std::to_string(k + 1) + " needed)"};
    // Ritz pairs of T_m, descending (stable by index), largest-|.| entry of each vector positive
    std::vector<double> ev, Z;
    tridiag_eig(meff, h->ta.data(), h->tb.data(), ev, Z);
    std::vector<int> idx(meff);
    for (int i = 0; i < meff; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ev[a] > ev[b]; });
    h->ritz.resize(meff);
    std::vector<double> Y((size_t)meff * k);
    for (int c = 0; c < meff; ++c) h->ritz[c] = ev[idx[c]];
    for (int c = 0; c < k; ++c) {
        const double* z = Z.data() + (size_t)idx[c] * meff;
        int big = 0;
        for (int r = 1; r < meff; ++r)
            if (std::fabs(z[r]) > std::fabs(z[big])) big = r;
        const double sg = z[big] < 0 ? -1.0 : 1.0;
        for (int r = 0; r < meff; ++r) Y[r + (size_t)c * meff] = sg * z[r];
    }
    double* Yd = tmp.alloc<double>(Y.size());
    HIPCHK(hipMemcpy(Yd, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice));
    h->lrmem.release();
    h->k = k;
    if (h->variant == DDLR_1) {
        h->urows = s;
        h->f64.U = h->lrmem.alloc<double>((size_t)s * k);
        hipLaunchKernelGGL(k_qy<double>, dim3(grid_for(s)), dim3(256), 0, st, s, meff, k, Q, s, Yd, h->f64.U, 0,
                           (int64_t)0);
        LAUNCHCHK();
        h->lam.assign(h->ritz.begin(), h->ritz.begin() + k);
        h->theta = theta_mode == DDLR_THETA_ZERO ? 0.0 : h->ritz[k];
        if (!(h->theta < 1.0)) {
            tmp.release();
            throw SetupError{DDLR_E_NOT_SPD, "theta = lambda_{k+1} >= 1: G_{k,theta} is singular or indefinite"};
        }
        h->c0 = 1.0 / (1.0 - h->theta);
        h->dvec_h.resize(k);
        for (int j = 0; j < k; ++j) {
            if (h->lam[j] == 1.0) {
                tmp.release();
                throw SetupError{DDLR_E_NOT_SPD, "Ritz value equal to 1"};
            }
            h->dvec_h[j] = 1.0 / (1.0 - h->lam[j]) - h->c0;
        }
        h->spd = h->lam[0] < 1.0 && h->pivots_positive;
        h->dvec = h->lrmem.upload(h->dvec_h);
    } else {
        // V_k = Q_m Y_k, U_k = A0^{-1} E V_k, K = U_k^T E V_k, H_k = (I - sym(K))^{-1}
        h->urows = n;
        double* V = tmp.alloc<double>((size_t)s * k);
        hipLaunchKernelGGL(k_qy<double>, dim3(grid_for(s)), dim3(256), 0, st, s, meff, k, Q, s, Yd, V, 1, s);
        LAUNCHCHK();
        double* EV = tmp.alloc<double>((size_t)n * k);
        double* Ucm = tmp.alloc<double>((size_t)n * k);
        hipLaunchKernelGGL(k_csr_mv<double>, dim3(grid_for(n)), dim3(256), 0, st, n, k, h->erp, h->eci, h->f64.ev,
                           V, s, (const double*)nullptr, 0, EV, n, nullptr);
        LAUNCHCHK();
        a0_solve_dev<double, double, double>(h, h->f64, k, EV, n, Ucm, n, st, nullptr);
        ddlr2_finish(h, k, Ucm, EV, tmp);
    }
    lowrank_copies(h, k);
    HIPCHK(hipDeviceSynchronize());
    tmp.release();
}

// DDLR-2 with U_k and V_k from m steps of the Lanczos (Golub-Kahan)
// bidiagonalisation of B = A0^{-1} E, the alternative build of Sec. 4.4 (sec:Lan)
// (Golub & Van Loan, Sec. 10.4).  From the unit interface vector q_1:
//   p_j = (B q_j - beta_{j-1} p_{j-1}) / alpha_j,   B q = A0^{-1} (E q)
//   q_{j+1} = (B^T p_j - alpha_j q_j) / beta_j,     B^T p = E^T (A0^{-1} p)
// with full reorthogonalisation (classical Gram-Schmidt twice) of p_j against
// p_1..p_{j-1} (n-vectors) and of q_{j+1} against q_1..q_j, so that
// B Q_m = P_m B_m with B_m upper bidiagonal.  Right singular vectors Z of B_m
// = eigenvectors of the tridiagonal B_m^T B_m (implicit QR on the host,
// descending, largest-|.| entry positive); V_k = Q_m Z_k, U_k = P_m (B_m Z_k)
// = B V_k, then H_k as in the Lanczos build.  Two A0 solves per step and none
// afterwards.  The run is cut at the first alpha_j or beta_j <= 1e-12 times
// the largest alpha (breakdown); it is not kept for ddlr_extend_lowrank.
void gk_build(ddlr_prec* h, int k, int m, const double* v0_user, uint64_t seed) {
    HostPlan& P = h->plan;
    const int64_t n = P.n, s = P.s;
    m = (int)std::min<int64_t>(m, s);
    h->lrun.reorth = DDLR_REORTH_FULL;
    lanczos_start(h, v0_user, seed);  // q_1 in R.Q (device interface order)
    LanczosRun& R = h->lrun;
    hipStream_t st = nullptr;
    DMem tmp;
    tmp.budget = budget_of(h);
    double* Qb = tmp.alloc<double>((size_t)s * (m + 1));
    double* Pb = tmp.alloc<double>((size_t)n * m);
    double* al = tmp.alloc<double>(m);
    double* be = tmp.alloc<double>(m);
    double* sc = tmp.alloc<double>(3);  // amax, inv, sum
    double* t = tmp.alloc<double>(n);
    double* w = tmp.alloc<double>(s);
    double* part = tmp.alloc<double>((size_t)kRedBlocks * (m + 1));
    double* csum = tmp.alloc<double>(m + 1);
    HIPCHK(hipMemcpy(Qb, R.Q, sizeof(double) * s, hipMemcpyDeviceToDevice));
    HIPCHK(hipMemset(sc, 0, sizeof(double) * 3));
    R.steps = 0;  // the bidiagonalisation replaces the Lanczos run
    R.lvariant = 0;
    double *amax = sc, *inv = sc + 1, *sum1 = sc + 2;
    const int gn = grid_for(n, 256, kRedBlocks), gs = grid_for(s, 256, kRedBlocks);
    // CGS2 of v (len) against the first ncols columns of V (ld = len)
    auto reorth = [&](int64_t len, int g, int ncols, const double* V, double* v) {
        if (ncols == 0) return;
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_multidot, dim3(g), dim3(256), 0, st, len, ncols, V, len, v, part, (const int*)nullptr);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_reduce_cols, dim3(ncols), dim3(256), 0, st, g, ncols, part, csum, nullptr);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_gemv_sub, dim3(g), dim3(256), 0, st, len, ncols, V, len, csum, v, (const int*)nullptr);
            LAUNCHCHK();
        }
    };
    auto norm = [&](int64_t len, int g, double* v, double* dst, int grow) {
        hipLaunchKernelGGL((k_dot<double, double>), dim3(g), dim3(256), 0, st, len, 1, v, len, v, len, part, nullptr);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, st, g, 1, part, sum1, nullptr);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_gk_norm, dim3(1), dim3(64), 0, st, sum1, dst, grow, amax, inv);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_scale_to, dim3(g), dim3(256), 0, st, len, v, inv, v);
        LAUNCHCHK();
    };
    for (int j = 0; j < m; ++j) {
        const double* qj = Qb + (size_t)j * s;
        double* pj = Pb + (size_t)j * n;
        hipLaunchKernelGGL(k_csr_mv<double>, dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->erp, h->eci, h->f64.ev, qj,
                           s, (const double*)nullptr, 0, t, n, nullptr);
        LAUNCHCHK();
        a0_solve_dev<double, double, double>(h, h->f64, 1, t, n, pj, n, st, nullptr);  // B q_j
        if (j > 0) {
            hipLaunchKernelGGL(k_sub_scaled, dim3(gn), dim3(256), 0, st, n, be + j - 1, Pb + (size_t)(j - 1) * n, pj);
            LAUNCHCHK();
        }
        reorth(n, gn, j, Pb, pj);
        norm(n, gn, pj, al + j, 1);  // alpha_j, p_j
        a0_solve_dev<double, double, double>(h, h->f64, 1, pj, n, t, n, st, nullptr);
        hipLaunchKernelGGL(k_csr_mv<double>, dim3(grid_for(s)), dim3(256), 0, st, s, 1, h->etrp, h->etci, h->f64.etv,
                           t, n, (const double*)nullptr, 0, w, s, nullptr);  // B^T p_j
        LAUNCHCHK();
        hipLaunchKernelGGL(k_sub_scaled, dim3(gs), dim3(256), 0, st, s, al + j, qj, w);
        LAUNCHCHK();
        reorth(s, gs, j + 1, Qb, w);
        norm(s, gs, w, be + j, 0);  // beta_j
        HIPCHK(hipMemcpyAsync(Qb + (size_t)(j + 1) * s, w, sizeof(double) * s, hipMemcpyDeviceToDevice, st));
    }
    std::vector<double> ha(m), hb(m);
    HIPCHK(hipMemcpy(ha.data(), al, m * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hb.data(), be, m * sizeof(double), hipMemcpyDeviceToHost));
    int meff = m;
    double am = 0.0;
    for (int j = 0; j < m; ++j) {
        am = std::max(am, ha[j]);
        if (!(ha[j] > 1e-12 * am)) {
            meff = j;
            break;
        }
        if (!(hb[j] > 1e-12 * am)) {
            meff = j + 1;
            break;
        }
    }
    ha.resize(meff);
    hb.resize(meff);
    drop_graphs(h);
    if (meff < k + 1) {
        tmp.release();
        throw SetupError{DDLR_E_LANCZOS, "bidiagonalisation broke down after " + std::to_string(meff) +
                                             " steps (k+1 = " + std::to_string(k + 1) + " needed)"};
    }
    // B_m^T B_m: diagonal alpha_j^2 + beta_{j-1}^2, off-diagonal alpha_j beta_j
    std::vector<double> td(meff), to(meff > 1 ? meff - 1 : 1, 0.0);
    for (int j = 0; j < meff; ++j) td[j] = ha[j] * ha[j] + (j > 0 ? hb[j - 1] * hb[j - 1] : 0.0);
    for (int j = 0; j + 1 < meff; ++j) to[j] = ha[j] * hb[j];
    std::vector<double> ev, Z;
    tridiag_eig(meff, td.data(), to.data(), ev, Z);
    std::vector<int> idx(meff);
    for (int i = 0; i < meff; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ev[a] > ev[b]; });
    std::vector<double> Zk((size_t)meff * k), Wk((size_t)meff * k);
    for (int c = 0; c < k; ++c) {
        const double* z = Z.data() + (size_t)idx[c] * meff;
        int big = 0;
        for (int r = 1; r < meff; ++r)
            if (std::fabs(z[r]) > std::fabs(z[big])) big = r;
        const double sg = z[big] < 0 ? -1.0 : 1.0;
        for (int r = 0; r < meff; ++r) Zk[r + (size_t)c * meff] = sg * z[r];
        for (int r = 0; r < meff; ++r)  // W = B_m Z_k
            Wk[r + (size_t)c * meff] = ha[r] * Zk[r + (size_t)c * meff] +
                                       (r + 1 < meff ? hb[r] * sg * z[r + 1] : 0.0);
    }
    h->ta = ha;
    h->tb = hb;
    h->lreorth = DDLR_REORTH_FULL;
    h->rflags.assign(meff, 1);
    h->msteps = meff;
    h->ritz.resize(meff);
    for (int c = 0; c < meff; ++c) h->ritz[c] = ev[idx[c]];
    double* Zd = tmp.upload(Zk);
    double* Wd = tmp.upload(Wk);
    h->lrmem.release();
    h->k = k;
    double* V = tmp.alloc<double>((size_t)s * k);
    hipLaunchKernelGGL(k_qy<double>, dim3(grid_for(s)), dim3(256), 0, st, s, meff, k, Qb, s, Zd, V, 1, s);
    LAUNCHCHK();
    double* Ucm = tmp.alloc<double>((size_t)n * k);
    hipLaunchKernelGGL(k_qy<double>, dim3(grid_for(n)), dim3(256), 0, st, n, meff, k, Pb, n, Wd, Ucm, 1, n);
    LAUNCHCHK();
    double* EV = tmp.alloc<double>((size_t)n * k);
    hipLaunchKernelGGL(k_csr_mv<double>, dim3(grid_for(n)), dim3(256), 0, st, n, k, h->erp, h->eci, h->f64.ev, V, s,
                       (const double*)nullptr, 0, EV, n, nullptr);
    LAUNCHCHK();
    ddlr2_finish(h, k, Ucm, EV, tmp);
    lowrank_copies(h, k);
    HIPCHK(hipDeviceSynchronize());
    tmp.release();
}

void lanczos_build(ddlr_prec* h, int k, int m_max, const double* v0_user, uint64_t seed, int theta_mode, int check,
                   double eps) {
    lanczos_start(h, v0_user, seed);
    lanczos_advance(h, m_max, check, eps, k);
    lanczos_finish(h, k, theta_mode);
}

void drop_graphs(ddlr_prec* h) {
    for (auto& g : h->cg_graphs) {
        if (g.second.second) (void)hipGraphExecDestroy(g.second.second);
        if (g.second.first) (void)hipGraphDestroy(g.second.first);
    }
    h->cg_graphs.clear();
    h->cg_mode.clear();  // launch shapes changed: measure again
    if (h->pers) {       // the persistent form's tables hold the rank and c0
        h->pers->mem.release();
        h->pers.reset();
    }
    h->pers_us.clear();
}

// The streams belong to the device's shared set; only the events are the handle's.
void release_streams(ddlr_prec* h) {
    drop_graphs(h);
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->ev_out) (void)hipEventDestroy(h->ev_out);
    h->cg_st = nullptr;
    h->ev_in = h->ev_out = nullptr;
    if (h->ev_xf) (void)hipEventDestroy(h->ev_xf);
    if (h->ev_xj) (void)hipEventDestroy(h->ev_xj);
    h->x_st = nullptr;
    h->ev_xf = h->ev_xj = nullptr;
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    h->side = nullptr;
    h->ev_fork = h->ev_join = nullptr;
}

// Device part of a build once the host plan exists: scratch address, device
// structures, Chebyshev vectors, launch options and streams.  The device is
// current and its lock held.
void device_init(ddlr_prec* h, int cheb_iters, int no_autotune) {
    (void)scratch_ptr(h->device);  // ddlr_apply_noalloc's array on this device
    upload_structures(h);
    if (h->plan.csolve == 2) {  // Chebyshev scratch, kMaxRhs columns
        h->cheb_nu = cheb_iters;
        const size_t tsz = h->precision == DDLR_FP64 ? sizeof(double) : sizeof(float);
        const size_t bytes = tsz * (size_t)h->plan.n * kMaxRhs;
        h->ch_t = h->chmem.alloc<char>(bytes);
        h->ch_r = h->chmem.alloc<char>(bytes);
        h->ch_d = h->chmem.alloc<char>(bytes);
        h->ch_x = h->chmem.alloc<char>(bytes);
    }
    if (const char* env = std::getenv("DDLR_NO_OVERLAP")) h->overlap = env[0] != '1';
    h->tune_mode = no_autotune ? 0 : 1;
    if (const char* env = std::getenv("DDLR_CG_GRAPH")) h->graph_mode = env[0] == '0' ? 0 : env[0] == '1' ? 1 : 2;
    if (const char* env = std::getenv("DDLR_CG_PERSIST")) h->pers_mode = env[0] == '0' ? 0 : env[0] == '1' ? 1 : 2;
    if (const char* env = std::getenv("DDLR_CG_XP")) h->cg_xp = env[0] != '0';
    if (const char* env = std::getenv("DDLR_LEVEL_KERNEL"))  // "rows" / "cols" force one form
        h->level_kernel = env[0] == 'r' ? 1 : env[0] == 'c' ? 2 : 0;
    if (has_cpart(h)) {
        h->side = dev_streams(h->device).side;
        HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    ensure_cg_streams(h);
}

// Frees what a handle that failed to build holds and leaves its context.
void discard_handle(ddlr_prec* h) {
    if (h->device >= 0) (void)hipDeviceSynchronize();
    release_streams(h);
    h->ws.mem.release();
    h->ws.gmem.release();
    h->lrmem.release();
    h->lrun.mem.release();
    h->chmem.release();
    h->mem.release();
    ctx_unref(h->ctx);
    h->ctx = nullptr;
}

ddlr_status fail_status(const SetupError& e) {
    g_err = e.msg;
    return (ddlr_status)e.status;
}

bool dev_ok(const ddlr_prec* h) {
    if (!h) {
        g_err = "null handle";
        return false;
    }
    if (h->device < 0) {
        g_err = "host-only handle (device = -1) cannot run device work";
        return false;
    }
    return true;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

int32_t ddlr_version(void) { return 100; }

void ddlr_options_default(ddlr_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->alpha = 1.0;
    o->lanczos_steps = 0;
    o->theta = DDLR_THETA_LAMBDA_K1;
    o->factor = DDLR_FACTOR_IC0;
    o->corder = DDLR_CORDER_MULTICOLOR;
    o->precision = DDLR_FP64;
    o->device = 0;
    o->seed = 0;
    o->lanczos_start = nullptr;
    o->csolve = DDLR_CSOLVE_FACTOR;
    o->cinv_iters = 3;
    o->cinv_tol = 0.01;
    o->cinv_lfil = 20;
    o->cheb_iters = 5;
    o->cheb_lanczos = 10;
}

void ddlr_solve_options_default(ddlr_solve_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = 0;
    o->restart = 40;
    o->maxit = 500;
    o->rtol = 1e-6;
}

ddlr_status ddlr_setup(ddlr_ctx* ctx, const ddlr_csr* A, const int32_t* part, int32_t p, int32_t k, int32_t variant,
                       const ddlr_options* opt_in, ddlr_prec** out) {
    if (out) *out = nullptr;
    if (!A || !part || !out) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    ddlr_options opt;
    if (opt_in) opt = *opt_in;
    else ddlr_options_default(&opt);
    if (ctx) opt.device = ctx->device;
    std::unique_ptr<ddlr_prec> h(new ddlr_prec());
    attach_ctx(h.get(), ctx);
    auto t0 = std::chrono::steady_clock::now();
    try {
        if (variant < 0 || variant > 2) throw SetupError{DDLR_E_INVALID, "variant must be 0, 1 or 2"};
        if (opt.precision < 0 || opt.precision > 2) throw SetupError{DDLR_E_INVALID, "bad precision"};
        if (opt.factor < 0 || opt.factor > 1 || opt.corder < 0 || opt.corder > 1)
            throw SetupError{DDLR_E_INVALID, "bad factor/corder option"};
        h->precision = opt.precision;
        h->variant = variant;
        if (const char* env = std::getenv("DDLR_LR_PLAIN")) h->lr_plain = env[0] == '1';
        if (opt.csolve != DDLR_CSOLVE_FACTOR && opt.csolve != DDLR_CSOLVE_MR && opt.csolve != DDLR_CSOLVE_CHEB)
            throw SetupError{DDLR_E_INVALID, "csolve must be DDLR_CSOLVE_FACTOR, DDLR_CSOLVE_MR or DDLR_CSOLVE_CHEB"};
        if (opt.csolve == DDLR_CSOLVE_CHEB && (opt.cheb_iters < 1 || opt.cheb_iters > 64 || opt.cheb_lanczos < 2 ||
                                               opt.cheb_lanczos > 200))
            throw SetupError{DDLR_E_INVALID, "Chebyshev: 1 <= cheb_iters <= 64 and 2 <= cheb_lanczos <= 200"};
        if (opt.lanczos_reorth != DDLR_REORTH_FULL && opt.lanczos_reorth != DDLR_REORTH_PARTIAL)
            throw SetupError{DDLR_E_INVALID, "lanczos_reorth must be DDLR_REORTH_FULL or DDLR_REORTH_PARTIAL"};
        if (opt.lanczos_reorth == DDLR_REORTH_PARTIAL && opt.lowrank_build == DDLR_BUILD_BIDIAG)
            throw SetupError{DDLR_E_INVALID, "partial reorthogonalisation is for the Lanczos build"};
        build_plan(h->plan, A->n, A->row_ptr, A->col_idx, A->val, part, p, opt.alpha, opt.factor, opt.corder,
                   opt.csolve == DDLR_CSOLVE_MR ? 1 : opt.csolve == DDLR_CSOLVE_CHEB ? 2 : 0, opt.cinv_iters,
                   opt.cinv_tol, opt.cinv_lfil, opt.cheb_lanczos);
        for (double d : h->plan.D) h->pivots_positive = h->pivots_positive && d > 0.0;
        // with the approximate inverse, A0 is SPD when the B factors are and X is;
        // with Chebyshev, when D_alpha's pivots are positive and so is the
        // estimated spectrum of D_alpha^{-1} C_alpha (the polynomial is then
        // positive on the safeguarded interval)
        if (h->plan.csolve == 1) h->pivots_positive = h->pivots_positive && h->plan.x_spd;
        if (h->plan.csolve == 2) h->pivots_positive = h->pivots_positive && h->plan.ch_rlo > 0.0;
        h->spd = variant == 0 ? (int)h->pivots_positive : 0;
        const int64_t s = h->plan.s;
        if (variant != 0) {
            if (k < 1 || (int64_t)k + 1 > s || k > 128)
                throw SetupError{DDLR_E_INVALID, "k must satisfy 1 <= k, k+1 <= s and k <= 128"};
        }
        h->device = opt.device;
        if (h->plan.csolve == 2) h->cheb_nu = opt.cheb_iters;
        if (opt.device >= 0) {
            HIPCHK(hipSetDevice(opt.device));
            DevLock dl(opt.device);
            device_init(h.get(), opt.cheb_iters, opt.no_autotune);
            if (variant != 0) {
                // fixed m steps (default 2k), or the paper's control: at most
                // lanczos_max steps (default 5k), stopped by eq. (converge)
                // tested every lanczos_check steps with lanczos_tol (default 1e-4)
                const bool ctl = opt.lanczos_check > 0;
                int m = ctl ? (opt.lanczos_max > 0 ? opt.lanczos_max : 5 * k)
                            : (opt.lanczos_steps > 0 ? opt.lanczos_steps : 2 * k);
                // reorthogonalisation coefficients of one step are staged in LDS (k_gemv_sub: 1024)
                if (m < k + 1 || m > kMaxLanczos)
                    throw SetupError{DDLR_E_INVALID, "Lanczos step limit must be in [k+1, 1024]"};
                if (ctl && !(opt.lanczos_tol >= 0.0))
                    throw SetupError{DDLR_E_INVALID, "lanczos_tol must be >= 0"};
                const double eps = ctl ? (opt.lanczos_tol > 0.0 ? opt.lanczos_tol : 1e-4) : 0.0;
                auto l0 = std::chrono::steady_clock::now();
                if (opt.lowrank_build != DDLR_BUILD_LANCZOS && opt.lowrank_build != DDLR_BUILD_BIDIAG)
                    throw SetupError{DDLR_E_INVALID, "lowrank_build must be DDLR_BUILD_LANCZOS or DDLR_BUILD_BIDIAG"};
                if (opt.lowrank_build == DDLR_BUILD_BIDIAG) {
                    if (variant != DDLR_2 || ctl)
                        throw SetupError{DDLR_E_INVALID, "the bidiagonalisation build is for DDLR-2 with fixed steps"};
                    gk_build(h.get(), k, m, opt.lanczos_start, opt.seed);
                } else {
                    h->lrun.reorth = opt.lanczos_reorth;
                    lanczos_build(h.get(), k, m, opt.lanczos_start, opt.seed, opt.theta, ctl ? opt.lanczos_check : 0,
                                  eps);
                }
                h->lanczos_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - l0).count();
            }
            HIPCHK(hipDeviceSynchronize());
        } else if (variant != 0) {
            h->k = 0;
        }
    } catch (const SetupError& e) {
        discard_handle(h.get());
        return fail_status(e);
    } catch (const std::bad_alloc&) {
        discard_handle(h.get());
        g_err = "host out of memory";
        return DDLR_E_OOM;
    }
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
    return DDLR_OK;
}

}  // extern "C"

static ddlr_status check_vec(const ddlr_prec* h, int32_t nrhs, const void* x, int64_t ldx, const void* y,
                             int64_t ldy) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    if (nrhs < 0 || (nrhs > 0 && (!x || !y)) || ldx < h->ndev || ldy < h->ndev) {
        g_err = "bad nrhs, pointer or leading dimension";
        return DDLR_E_INVALID;
    }
    return DDLR_OK;
}

// ------------------------------------------------------------ autotuner
//
// On the first A0 solve with a given number of columns, times the block
// triangular solve with 1, 2, 4 and 8 columns per workgroup (those that divide
// the column count and whose LDS ring holds the dependency window), then the
// interface-level overlap on and off with the best shape, and keeps the
// fastest.  The candidates differ in launch shape only, not in arithmetic, so
// the choice never changes a result.  Scratch: workspace buffers q and a1.
template <typename T>
void autotune_T(ddlr_prec* h, const DevFactors<T>& F, int nrhs, hipStream_t st) {
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    const bool prof = h->prof;
    h->prof = false;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n * nrhs)), dim3(256), 0, st, n * nrhs, 0.0, W.q);
    LAUNCHCHK();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_a0 = [&]() -> float {
        a0_solve_dev<T, double, T>(h, F, nrhs, W.q, n, (T*)W.a1, n, st, nullptr);
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(e0, st));
            a0_solve_dev<T, double, T>(h, F, nrhs, W.q, n, (T*)W.a1, n, st, nullptr);
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return 1e3f * best;
    };
    ddlr_prec::Tune& tn = h->tune[nrhs];
    tn = ddlr_prec::Tune();
    const int Rs[4] = {1, 2, 4, 8};
    float best = 1e30f;
    int bestR = 1, bestNT = 512;
    tn.ring_nt = 512;
    for (int q = 0; q < 4; ++q) {
        const int R = Rs[q];
        if (nrhs % R != 0 || !ring_r_ok<T>(h, R, nrhs) || (R > 1 && h->nnarrow == 0)) continue;
        tn.ring_r = R;
        tn.a0_us[q] = time_a0();
        if (tn.a0_us[q] < best) {
            best = tn.a0_us[q];
            bestR = R;
        }
    }
    // thin workgroups (one column each) for narrow levels
    if (ring_ready<T>(h) && h->nnarrow > 0) {
        const int nts[2] = {64, 256};
        for (int q = 0; q < 2; ++q) {
            if (!ring_nt_ok(h, nts[q])) continue;
            tn.ring_r = 1;
            tn.ring_nt = nts[q];
            tn.a0_thin_us[q] = time_a0();
            if (tn.a0_thin_us[q] < best) {
                best = tn.a0_thin_us[q];
                bestR = 1;
                bestNT = nts[q];
            }
        }
    }
    // the plain per-level kernel (padding to a wide ELL can cost more than it saves)
    if (ring_ready<T>(h) && h->nnarrow > 0) {
        tn.ring_r = 1;
        tn.ring_nt = -1;
        tn.a0_plain_us = time_a0();
        if (tn.a0_plain_us < best) {
            best = tn.a0_plain_us;
            bestR = 1;
            bestNT = -1;
        }
    }
    tn.ring_r = bestR;
    tn.ring_nt = bestR > 1 ? 512 : bestNT;
    tn.overlap = 1;
    if (h->overlap && h->side && has_cpart(h) && h->nnarrow > 0) {
        tn.overlap = 0;
        tn.a0_noov_us = time_a0();
        tn.overlap = tn.a0_noov_us < best ? 0 : 1;
    }
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    h->prof = prof;
}

void autotune(ddlr_prec* h, int nrhs, hipStream_t st, bool force) {
    if (h->capturing || h->batch) return;
    if (!force && (h->tune_mode == 0 || h->tune.count(nrhs))) return;
    ensure_ws(h, nrhs);
    drop_graphs(h);  // captured launches embed the shape
    if (h->precision == DDLR_FP64) autotune_T<double>(h, h->f64, nrhs, st);
    else autotune_T<float>(h, h->f32, nrhs, st);
}

// Applies op to columns in chunks of kMaxRhs: gather -> op (device order) -> scatter
template <typename Op>
static ddlr_status run_chunked(ddlr_prec* h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                               void* stream, Op op) {
    try {
        HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        hipStream_t st = (hipStream_t)stream;
        const int64_t n = h->ndev;
        for (int32_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
            const int nr = std::min<int>(kMaxRhs, nrhs - c0);
            ensure_ws(h, nr);
            autotune(h, nr, st, false);
            Workspace& W = h->ws;
            hipLaunchKernelGGL((k_gather<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr,
                               h->perm_dev, x + c0 * ldx, ldx, W.r, n);
            LAUNCHCHK();
            op(nr, W.r, W.z, st);
            hipLaunchKernelGGL((k_scatter<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr,
                               h->perm_dev, W.z, n, y + c0 * ldy, ldy);
            LAUNCHCHK();
        }
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

extern "C" {

ddlr_status ddlr_apply(ddlr_prec* h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                       void* stream) {
    ddlr_status st = check_vec(h, nrhs, x, ldx, y, ldy);
    if (st != DDLR_OK) return st;
    return run_chunked(h, nrhs, x, ldx, y, ldy, stream, [&](int nr, double* in, double* out, hipStream_t s) {
        apply_dev(h, nr, in, h->ndev, out, h->ndev, s, nullptr);
    });
}

ddlr_status ddlr_a0_solve(ddlr_prec* h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                          void* stream) {
    ddlr_status st = check_vec(h, nrhs, x, ldx, y, ldy);
    if (st != DDLR_OK) return st;
    const int v = h->variant;
    h->variant = 0;
    ddlr_status r = run_chunked(h, nrhs, x, ldx, y, ldy, stream, [&](int nr, double* in, double* out, hipStream_t s) {
        apply_dev(h, nr, in, h->ndev, out, h->ndev, s, nullptr);
    });
    h->variant = v;
    return r;
}

ddlr_status ddlr_spmv(ddlr_prec* h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                      void* stream) {
    ddlr_status st = check_vec(h, nrhs, x, ldx, y, ldy);
    if (st != DDLR_OK) return st;
    return run_chunked(h, nrhs, x, ldx, y, ldy, stream, [&](int nr, double* in, double* out, hipStream_t s) {
        spmv_dev(h, nr, in, h->ndev, out, h->ndev, nullptr, s, nullptr);
    });
}

}  // extern "C"

// ------------------------------------------------------------ apply without allocation

namespace {

// Bytes one column of ddlr_apply_noalloc takes in the scratch array, each
// buffer rounded up to 256 bytes: the gathered input and the output (double),
// the two A0-solve results a1, a2 and the interface vectors ys, ws (type of the
// preconditioner), the low-rank reduction partials (kLrBlocks x k doubles) with
// the k sums and coefficients, and the Chebyshev solver's four vectors.
size_t noalloc_bytes(const ddlr_prec* h, int nr) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t tsz = h->precision == DDLR_FP64 ? sizeof(double) : sizeof(float);
    const size_t n = (size_t)h->ndev, s = (size_t)h->sdev, k = (size_t)std::max(1, h->k), c = (size_t)nr;
    size_t b = 2 * up(8 * n * c) + 2 * up(tsz * n * c) + 2 * up(tsz * s * c) + up(8 * kLrBlocks * k * c) +
               2 * up(8 * k * c);
    if (h->cheb_nu > 0) b += 4 * up(tsz * n * c);
    return b;
}

// Points the apply's temporaries at the scratch array for one chunk of nr
// columns and restores the handle's own buffers when it goes out of scope.
// Profiling is off meanwhile (its events would be created on demand).
struct ScratchView {
    ddlr_prec* h;
    void *a1, *a2, *ys, *ws, *ct, *cr, *cd, *cx;
    double *part, *lrsum, *coef;
    int ry_cols, iy_cols;
    bool prof;
    double *in = nullptr, *out = nullptr;
    ScratchView(ddlr_prec* h_, char* base, int nr) : h(h_) {
        Workspace& W = h->ws;
        a1 = W.a1, a2 = W.a2, ys = W.ys, ws = W.ws, part = W.part, lrsum = W.lrsum, coef = W.coef;
        ry_cols = W.ry_cols, iy_cols = W.iy_cols;
        W.ry_cols = 0;  // no buffer for the R-column ring kernel: one column per workgroup
        W.iy_cols = 0;  // nor for the interface levels: the column-major kernels
        ct = h->ch_t, cr = h->ch_r, cd = h->ch_d, cx = h->ch_x;
        prof = h->prof;
        auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t tsz = h->precision == DDLR_FP64 ? sizeof(double) : sizeof(float);
        const size_t n = (size_t)h->ndev, s = (size_t)h->sdev, k = (size_t)std::max(1, h->k), c = (size_t)nr;
        char* p = base;
        auto take = [&](size_t b) {
            char* q = p;
            p += up(b);
            return q;
        };
        in = (double*)take(8 * n * c);
        out = (double*)take(8 * n * c);
        W.a1 = take(tsz * n * c);
        W.a2 = take(tsz * n * c);
        W.ys = take(tsz * s * c);
        W.ws = take(tsz * s * c);
        W.part = (double*)take(8 * kLrBlocks * k * c);
        W.lrsum = (double*)take(8 * k * c);
        W.coef = (double*)take(8 * k * c);
        if (h->cheb_nu > 0) {
            h->ch_t = take(tsz * n * c);
            h->ch_r = take(tsz * n * c);
            h->ch_d = take(tsz * n * c);
            h->ch_x = take(tsz * n * c);
        }
        h->prof = false;
    }
    ~ScratchView() {
        Workspace& W = h->ws;
        W.a1 = a1, W.a2 = a2, W.ys = ys, W.ws = ws, W.part = part, W.lrsum = lrsum, W.coef = coef;
        W.ry_cols = ry_cols, W.iy_cols = iy_cols;
        h->ch_t = ct, h->ch_r = cr, h->ch_d = cd, h->ch_x = cx;
        h->prof = prof;
    }
};

}  // namespace

extern "C" {

ddlr_status ddlr_apply_noalloc(ddlr_prec* h, int32_t nrhs, const double* x, int64_t ldx, double* y, int64_t ldy,
                               void* stream) {
    ddlr_status st = check_vec(h, nrhs, x, ldx, y, ldy);
    if (st != DDLR_OK) return st;
    if (nrhs == 0) return DDLR_OK;
    try {
        int cur = -1;
        HIPCHK(hipGetDevice(&cur));
        if (cur != h->device) HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        char* base = scratch_ptr(h->device);
        size_t cap = kScratchBytes;
        if (const char* env = std::getenv("DDLR_NOALLOC_CAP")) {  // may only lower the usable size
            const long long c = std::atoll(env);
            if (c >= 0 && (size_t)c < cap) cap = (size_t)c;
        }
        int nr = std::min<int>(kMaxRhs, nrhs);
        while (nr > 0 && noalloc_bytes(h, nr) > cap) --nr;
        if (nr == 0) {
            g_err = "ddlr_apply_noalloc: one column needs " + std::to_string(noalloc_bytes(h, 1)) +
                    " bytes of scratch; the library's scratch array holds " + std::to_string(cap);
            return DDLR_E_INVALID;
        }
        hipStream_t sm = (hipStream_t)stream;
        const int64_t n = h->ndev;
        for (int32_t c0 = 0; c0 < nrhs; c0 += nr) {
            const int w = std::min<int>(nr, nrhs - c0);
            ScratchView v(h, base, w);
            hipLaunchKernelGGL((k_gather<double, double>), grid2(n, w), dim3(256), 0, sm, n, w, h->perm_dev,
                               x + c0 * ldx, ldx, v.in, n);
            LAUNCHCHK();
            apply_dev(h, w, v.in, n, v.out, n, sm, nullptr);
            hipLaunchKernelGGL((k_scatter<double, double>), grid2(n, w), dim3(256), 0, sm, n, w, h->perm_dev, v.out,
                               n, y + c0 * ldy, ldy);
            LAUNCHCHK();
        }
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

}  // extern "C"

constexpr int kGmChunks = 1024;  // row chunks of the Gram-Schmidt dot products (per group of basis vectors)

static void ensure_gmres(ddlr_prec* h, int nr, int m) {
    Workspace& W = h->ws;
    if (W.gm_m >= m && W.gm_nrhs >= nr) return;
    W.gmem.release();
    const int64_t n = h->ndev;
    W.gV = W.gmem.alloc<double>((size_t)(m + 1) * nr * n);
    W.gH = W.gmem.alloc<double>((size_t)nr * m * (m + 1));
    W.gcs = W.gmem.alloc<double>((size_t)nr * m);
    W.gsn = W.gmem.alloc<double>((size_t)nr * m);
    W.gg = W.gmem.alloc<double>((size_t)nr * (m + 1));
    W.gy = W.gmem.alloc<double>((size_t)nr * m);
    W.gcoef = W.gmem.alloc<double>((size_t)nr * (m + 1));
    W.ginv = W.gmem.alloc<double>(nr);
    W.gpart = W.gmem.alloc<double>((size_t)kGmChunks * (m + 1) * nr);
    W.glanes = W.gmem.alloc<GmLane>(nr);
    W.gm_m = m;
    W.gm_nrhs = nr;
}

// Right-preconditioned GMRES(m) on nr columns already gathered into W.r (b);
// result in W.x.  Arnoldi by classical Gram-Schmidt applied twice.
static void gmres_dev(ddlr_prec* h, int nr, const ddlr_solve_options& o, hipStream_t st) {
    const int m = o.restart;
    ensure_gmres(h, nr, m);
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    const double tol2 = o.rtol * o.rtol;
    // W.p keeps b; W.x = 0
    HIPCHK(hipMemcpyAsync(W.p, W.r, sizeof(double) * n * nr, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n * nr)), dim3(256), 0, st, n * nr, 0.0, W.x);
    LAUNCHCHK();
    for (int cycle = 0;; ++cycle) {
        // r = b - A x, beta = ||r||
        spmv_dev(h, nr, W.x, n, W.q, n, nullptr, st, nullptr);
        hipLaunchKernelGGL(k_sub, dim3(grid_for(n * nr)), dim3(256), 0, st, n * nr, W.p, W.q, W.r);
        LAUNCHCHK();
        dot_dev(h, nr, W.r, W.r, n, st, nullptr);
        hipLaunchKernelGGL(k_gm_start, dim3(1), dim3(64), 0, st, nr, m, W.sums, W.gg, W.gH, W.ginv, W.glanes, tol2,
                           o.maxit, cycle == 0 ? 1 : 0, W.done);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(W.done_host, W.done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!*W.done_host) break;  // no lane opened a cycle
        // done := 0 while any lane is active (k_gm_start wrote "any active" into it)
        hipLaunchKernelGGL(k_gm_scale, grid2(n, nr), dim3(256), 0, st, n, nr, W.r, W.ginv, W.gV);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_flag_not, dim3(1), dim3(1), 0, st, W.done);
        LAUNCHCHK();
        for (int j = 0; j < m; ++j) {
            double* Vj = W.gV + (size_t)j * nr * n;
            apply_dev(h, nr, Vj, n, W.z, n, st, W.done);               // z = M^{-1} v_j
            spmv_dev(h, nr, W.z, n, W.q, n, nullptr, st, W.done);      // w = A z
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_gm_dots, dim3(kGmChunks, (j + kGmGroup) / kGmGroup, nr), dim3(256), 0, st, n, nr,
                                   j + 1, W.gV, W.q, W.gpart, W.done);
                LAUNCHCHK();
                hipLaunchKernelGGL(k_gm_coef, dim3((nr * (j + 1) + 3) / 4), dim3(256), 0, st, kGmChunks, nr, j + 1, m,
                                   j, W.gpart, W.gcoef, W.gH, W.glanes, W.done);
                LAUNCHCHK();
                hipLaunchKernelGGL(k_gm_sub, grid2(n, nr), dim3(256), 0, st, n, nr, j + 1, W.gV, W.gcoef,
                                   W.q, W.done);
                LAUNCHCHK();
            }
            dot_dev(h, nr, W.q, W.q, n, st, W.done);
            hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(64), 0, st, j, nr, m, W.sums, W.gH, W.gcs, W.gsn, W.gg,
                               W.ginv, W.glanes, tol2, o.maxit, W.done);
            LAUNCHCHK();
            if (j + 1 < m) {
                hipLaunchKernelGGL(k_gm_scale, grid2(n, nr), dim3(256), 0, st, n, nr, W.q, W.ginv,
                                   W.gV + (size_t)(j + 1) * nr * n);
                LAUNCHCHK();
            }
            if ((j + 1) % 8 == 0 || j + 1 == m) {
                HIPCHK(hipMemcpyAsync(W.done_host, W.done, sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                if (*W.done_host) break;
            }
        }
        // x += M^{-1} V y
        hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, st, nr, m, W.gH, W.gg, W.gy, W.glanes);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_gm_combine, grid2(n, nr), dim3(256), 0, st, n, nr, m, W.gV, W.gy, W.glanes,
                           W.r);
        LAUNCHCHK();
        apply_dev(h, nr, W.r, n, W.z, n, st, nullptr);
        hipLaunchKernelGGL(k_gm_xupdate, grid2(n, nr), dim3(256), 0, st, n, nr, W.glanes, W.z, W.x);
        LAUNCHCHK();
    }
    // lanes -> CG lane records used by the reporting code
    hipLaunchKernelGGL(k_gm_report, dim3(1), dim3(64), 0, st, nr, W.glanes, W.lanes);
    LAUNCHCHK();
}

extern "C" {

}  // extern "C"

// One CG iteration of every lane (lane phases, see CgLane), nr columns of the
// handle's workspace.  Kernels exit early once W.done is set.
// S: the interleave stride of p, at least lane_stride(nr) (0: that stride);
// a lane's arithmetic does not depend on it or on the other lanes.
static void lane_iteration(ddlr_prec* h, int nr, hipStream_t st, int S = 0) {
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    if (!S) S = lane_stride(nr);
    const int npart_spmv = (int)((n + 255) / 256);
    // each dot product: partials, then one launch reducing them and updating the lanes
    spmv_il_dev(h, nr, W.p, W.q, n, W.part, st, W.done, S);
    hipLaunchKernelGGL(k_reduce_lane, dim3(nr), dim3(256), 0, st, 2, npart_spmv, nr, W.part, W.sums, W.lanes, W.done,
                       W.ctr);
    LAUNCHCHK();
    // x += alpha p: with the p update (k_cg_xp), on the x stream beside the
    // preconditioner, or with the r update
    const bool xp = h->cg_xp;
    const bool split = !xp && h->x_st != nullptr;
    if (xp) cg_r_dev(h, nr, S, st);
    else if (split) cg_split_dev(h, nr, S, st);
    else cg_xr_dev(h, nr, S, st);
    hipLaunchKernelGGL(k_reduce_lane, dim3(nr), dim3(256), 0, st, 3, kRedBlocks, nr, W.part, W.sums, W.lanes, W.done,
                       W.ctr);
    LAUNCHCHK();
    apply_dev(h, nr, W.r, n, W.z, n, st, W.done);
    hipLaunchKernelGGL((k_dot<double, double>), dim3(kRedBlocks), dim3(256), 0, st, n, nr, W.r, n, W.z, n, W.part,
                       W.done);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_lane, dim3(nr), dim3(256), 0, st, 4, kRedBlocks, nr, W.part, W.sums, W.lanes, W.done,
                       W.ctr);
    LAUNCHCHK();
    if (split) HIPCHK(hipStreamWaitEvent(st, h->ev_xj, 0));  // x used the old p
    const dim3 gp(grid_for(n)), bp(256);
    if (xp) {
        switch (S) {
        case 1: hipLaunchKernelGGL(k_cg_xp<1>, gp, bp, 0, st, n, nr, W.lanes, W.xa, W.z, W.p, W.x, n); break;
        case 2: hipLaunchKernelGGL(k_cg_xp<2>, gp, bp, 0, st, n, nr, W.lanes, W.xa, W.z, W.p, W.x, n); break;
        case 4: hipLaunchKernelGGL(k_cg_xp<4>, gp, bp, 0, st, n, nr, W.lanes, W.xa, W.z, W.p, W.x, n); break;
        case 8: hipLaunchKernelGGL(k_cg_xp<8>, gp, bp, 0, st, n, nr, W.lanes, W.xa, W.z, W.p, W.x, n); break;
        case 16: hipLaunchKernelGGL(k_cg_xp<16>, gp, bp, 0, st, n, nr, W.lanes, W.xa, W.z, W.p, W.x, n); break;
        default: throw SetupError{DDLR_E_INVALID, "CG runs at most 16 lanes per launch"};
        }
        LAUNCHCHK();
        return;
    }
    switch (S) {
    case 1: hipLaunchKernelGGL(k_cg_p<1>, gp, bp, 0, st, n, nr, W.lanes, W.z, W.p, n, W.done); break;
    case 2: hipLaunchKernelGGL(k_cg_p<2>, gp, bp, 0, st, n, nr, W.lanes, W.z, W.p, n, W.done); break;
    case 4: hipLaunchKernelGGL(k_cg_p<4>, gp, bp, 0, st, n, nr, W.lanes, W.z, W.p, n, W.done); break;
    case 8: hipLaunchKernelGGL(k_cg_p<8>, gp, bp, 0, st, n, nr, W.lanes, W.z, W.p, n, W.done); break;
    case 16: hipLaunchKernelGGL(k_cg_p<16>, gp, bp, 0, st, n, nr, W.lanes, W.z, W.p, n, W.done); break;
    default: throw SetupError{DDLR_E_INVALID, "CG runs at most 16 lanes per launch"};
    }
    LAUNCHCHK();
}

// Admits lanes flagged in the host array start[0..nr) (tolerance rtol^2,
// limit maxit); their b must already be in W.r.
static void lane_admit(ddlr_prec* h, int nr, const std::vector<int32_t>& start, const std::vector<double>& tol2,
                       const std::vector<int32_t>& maxit, hipStream_t st) {
    Workspace& W = h->ws;
    HIPCHK(hipMemcpyAsync(W.adm_start, start.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(W.adm_tol2, tol2.data(), nr * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(W.adm_maxit, maxit.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_lane_zero, dim3(grid_for(h->ndev * lane_stride(nr))), dim3(256), 0, st, h->ndev, nr,
                       ilog2(lane_stride(nr)), W.adm_start, W.x, W.p, h->ndev);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_lane_admit, dim3(1), dim3(64), 0, st, nr, W.adm_start, W.adm_tol2, W.adm_maxit, W.lanes,
                       W.done);
    LAUNCHCHK();
}

// PCG on nr columns already gathered into W.r (b); result in W.x.
constexpr int kCgChunk = 8;

// kCgChunk lane iterations on st: eager launches, or replayed from a graph
// captured on first use for this column count (eager if capture fails)
static void cg_chunk(ddlr_prec* h, int nr, hipStream_t st, bool graph) {
    if (!graph) {
        for (int c = 0; c < kCgChunk; ++c) lane_iteration(h, nr, st);
        return;
    }
    const int key = nr * 4 + h->ov_override + 1;  // the overlap choice is baked into the capture
    auto it = h->cg_graphs.find(key);
    if (it == h->cg_graphs.end()) {
        h->capturing = true;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        bool ok = true;
        try {
            for (int c = 0; c < kCgChunk; ++c) lane_iteration(h, nr, st);
        } catch (const SetupError&) {
            ok = false;
        }
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        h->capturing = false;
        hipGraphExec_t ge = nullptr;
        if (ok && ec == hipSuccess && g && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess) {
            it = h->cg_graphs.emplace(key, std::make_pair(g, ge)).first;
        } else {
            (void)hipGetLastError();
            if (g) (void)hipGraphDestroy(g);
            h->graph_mode = 0;  // fall back to eager launches for this handle
            for (int c = 0; c < kCgChunk; ++c) lane_iteration(h, nr, st);
            return;
        }
    }
    HIPCHK(hipGraphLaunch(it->second.second, st));
}

constexpr int kCgSamples = 3;        // timed chunks per launch-form candidate
constexpr int kCgMeasureSolves = 6;  // after this many solves, chunks where lanes finished count too

static void pcg_dev(ddlr_prec* h, int nr, const ddlr_solve_options& o, hipStream_t ust) {
    ensure_cg_streams(h);
    hipStream_t st = h->cg_st;
    HIPCHK(hipEventRecord(h->ev_in, ust));
    HIPCHK(hipStreamWaitEvent(st, h->ev_in, 0));
    std::vector<int32_t> start(nr, 1), maxit(nr, o.maxit);
    std::vector<double> tol2(nr, o.rtol * o.rtol);
    lane_admit(h, nr, start, tol2, maxit, st);
    // Launch form of the chunks, measured on the first solves of a column
    // count: chunk boundaries are synchronous anyway, so whole chunks are timed
    // on the host.  Candidates: replayed graph or eager launches (unless
    // DDLR_CG_GRAPH forces one), each with the interface levels beside or in
    // line with the block solve when both are possible (inside an iteration the
    // overlapped levels compete with other forked work, and a replayed graph
    // may run forked branches one after the other, so neither the A0-only
    // timing nor eager timing decides it).  Each candidate gets kCgSamples
    // timed chunks (a graph's capture chunk is not timed); the fastest is kept.
    // A chunk is a sample only when every lane ran through all of it: lanes
    // that finish leave later chunks of a solve cheaper, and the candidates
    // are sampled at different points of the solves.
    ddlr_prec::CgMode& m = h->cg_mode[nr];
    if (m.graph < 0) ++m.solves;
    std::vector<CgLane> lh(nr);
    int run_prev = -1;  // lanes running at the end of the previous chunk of this solve
    const bool can_ov = has_cpart(h) && h->nnarrow > 0 && h->overlap && h->side;
    const int gfirst = h->graph_mode == 0 ? 0 : 1, glast = h->graph_mode == 1 ? 1 : 0;
    const int ofirst = can_ov ? 1 : -1, olast = can_ov ? 0 : -1;
    for (int it = 0; it <= o.maxit; it += kCgChunk) {
        int g = gfirst, ov = ofirst;
        bool timed = false;
        if (h->prof) {
            g = 0;  // per-launch events need eager launches; keep the measured overlap
            ov = m.ov >= -1 ? m.ov : ofirst;
        } else if (m.graph >= 0) {
            g = m.graph;
            ov = m.ov;
        } else {
            // first candidate (graph form descending, overlap descending) with fewer than two samples
            bool found = false;
            for (int gg = gfirst; gg >= glast && !found; --gg)
                for (int oo = ofirst; oo >= olast && !found; --oo)
                    if (m.timed[gg][oo + 1] < kCgSamples) {
                        g = gg;
                        ov = oo;
                        found = true;
                    }
            timed = !(g == 1 && !m.captured[ov + 1]);
        }
        h->ov_override = ov;
        const auto t0 = std::chrono::steady_clock::now();
        cg_chunk(h, nr, st, g == 1 && h->graph_mode != 0);
        HIPCHK(hipMemcpyAsync(h->ws.done_host, h->ws.done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        h->ov_override = -1;
        const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
        const bool done = *h->ws.done_host != 0;
        if (!h->prof && m.graph < 0) {
            HIPCHK(hipMemcpyAsync(lh.data(), h->ws.lanes, sizeof(CgLane) * nr, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            int run = 0;
            for (const CgLane& l : lh) run += l.phase == 2;
            const bool full = (run_prev == nr && run == nr) || m.solves > kCgMeasureSolves;
            run_prev = run;
            if (g == 1) m.captured[ov + 1] = true;
            if (timed && !done && full) {  // a chunk that ran all its iterations on every lane
                m.us[g][ov + 1] = std::min(m.us[g][ov + 1], us);
                ++m.timed[g][ov + 1];
            }
            bool all = true;
            double best = 1e30;
            for (int gg = gfirst; gg >= glast; --gg)
                for (int oo = ofirst; oo >= olast; --oo) {
                    all = all && m.timed[gg][oo + 1] >= kCgSamples;
                    if (m.us[gg][oo + 1] < best) {
                        best = m.us[gg][oo + 1];
                        m.graph = gg;  // provisional; kept only when all are measured
                        m.ov = oo;
                    }
                }
            // the plain form (replayed if allowed, interface solve in line) stays
            // unless another is faster by more than the noise of a minimum over
            // kCgSamples chunks
            if (m.us[gfirst][olast + 1] <= best / 0.99) {
                m.graph = gfirst;
                m.ov = olast;
            }
            if (!all) {
                m.graph = -1;
                m.ov = -2;
            }
        }
        if (done) break;
    }
    HIPCHK(hipEventRecord(h->ev_out, st));
    HIPCHK(hipStreamWaitEvent(ust, h->ev_out, 0));
}

namespace {

// ------------------------------------------------------------ persistent PCG

constexpr int64_t kPersistMaxRows = 262144;  // rows of a system the one-workgroup form is tried on

// Merged levels of one system (plan P, rows offset by r0 in the concatenated
// device order): level j lists the device rows of level j of every block,
// blocks in order, with slot-major ELL copies of their rows of L (forward) and
// of L^T (backward), entries in the CSR order of the other A0-solve kernels
// (L: ascending internal column; L^T: ascending internal row), short rows
// padded with their own index and weight 0.  Appends to the batch-wide lists.
struct MergedLevels {
    std::vector<int4> meta;
    std::vector<int32_t> mrow, fcol, bcol;
    std::vector<double> fval, bval, dq;
};

// L^T of a plan by device rows (each row's entries in ascending internal row order)
struct PlanTranspose {
    std::vector<int32_t> tcnt, tcol;
    std::vector<double> tval;
};

void plan_transpose(const HostPlan& P, PlanTranspose& X) {
    const int64_t n = P.n;
    X.tcnt.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = P.L.rp[i]; t < P.L.rp[i + 1]; ++t) X.tcnt[P.int2dev[P.L.ci[t]] + 1]++;
    for (int64_t d = 0; d < n; ++d) X.tcnt[d + 1] += X.tcnt[d];
    X.tcol.assign(X.tcnt[n], 0);
    X.tval.assign(X.tcnt[n], 0.0);
    std::vector<int32_t> fill(X.tcnt.begin(), X.tcnt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = P.L.rp[i]; t < P.L.rp[i + 1]; ++t) {
            const int32_t q = fill[P.int2dev[P.L.ci[t]]]++;
            X.tcol[q] = P.int2dev[i];
            X.tval[q] = P.L.v[t];
        }
}

// Merged levels of blocks b0..b1-1 of a plan (block P.p is the interface block).
void persist_levels(const HostPlan& P, const PlanTranspose& X, int64_t r0, int32_t b0, int32_t b1, MergedLevels& M,
                    int32_t& l0, int32_t& l1) {
    const std::vector<int32_t>& tcnt = X.tcnt;
    const std::vector<int32_t>& tcol = X.tcol;
    const std::vector<double>& tval = X.tval;
    int depth = 0;
    for (int32_t b = b0; b < b1; ++b) depth = std::max(depth, P.blk_lvl[b + 1] - P.blk_lvl[b]);
    l0 = (int32_t)M.meta.size();
    std::vector<int32_t> rows;
    for (int j = 0; j < depth; ++j) {
        rows.clear();
        for (int32_t b = b0; b < b1; ++b) {
            const int32_t l = P.blk_lvl[b] + j;
            if (l >= P.blk_lvl[b + 1]) continue;
            for (int32_t d = P.lvl_ptr[l]; d < P.lvl_ptr[l + 1]; ++d) rows.push_back(d);
        }
        const int nr = (int)rows.size();
        int fw = 0, bw = 0;
        for (int32_t d : rows) {
            const int64_t i = P.dev2int[d];
            fw = std::max(fw, (int)(P.L.rp[i + 1] - P.L.rp[i]));
            bw = std::max(bw, tcnt[d + 1] - tcnt[d]);
        }
        if (fw > 0xffff || bw > 0x7fff) throw SetupError{DDLR_E_INVALID, "a factor row is too long for the persistent form"};
        M.meta.push_back(int4{(int)M.mrow.size(), fw | (bw << 16), (int)M.fcol.size(), (int)M.bcol.size()});
        for (int32_t d : rows) {
            M.mrow.push_back((int32_t)(r0 + d));
            M.dq.push_back(1.0 / P.D[P.dev2int[d]]);
        }
        for (int u = 0; u < fw; ++u)
            for (int32_t d : rows) {
                const int64_t i = P.dev2int[d];
                const int64_t t = P.L.rp[i] + u;
                const bool has = t < P.L.rp[i + 1];
                M.fcol.push_back((int32_t)(r0 + (has ? P.int2dev[P.L.ci[t]] : d)));
                M.fval.push_back(has ? P.L.v[t] : 0.0);
            }
        for (int u = 0; u < bw; ++u)
            for (int32_t d : rows) {
                const int32_t t = tcnt[d] + u;
                const bool has = t < tcnt[d + 1];
                M.bcol.push_back((int32_t)(r0 + (has ? tcol[t] : d)));
                M.bval.push_back(has ? tval[t] : 0.0);
            }
        (void)nr;
    }
    l1 = (int32_t)M.meta.size();
}

// A of one plan in device order as CSR, rows and columns offset by r0.
void persist_csr(const HostPlan& P, int64_t r0, std::vector<int64_t>& arp, std::vector<int32_t>& aci,
                 std::vector<double>& av) {
    for (int64_t d = 0; d < P.n; ++d) {
        const int64_t i = P.dev2int[d];
        for (int64_t t = P.A.rp[i]; t < P.A.rp[i + 1]; ++t) {
            aci.push_back((int32_t)(r0 + P.int2dev[P.A.ci[t]]));
            av.push_back(P.A.v[t]);
        }
        arp.push_back((int64_t)aci.size());
    }
}

// Largest dynamic LDS a persistent launch may take on device `dev`.
size_t persist_lds_budget(int dev) {
    if (const char* env = std::getenv("DDLR_PERSIST_NO_LDS"))  // "1": every solve vector in global memory
        if (env[0] == '1') return 0;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
        (void)hipGetLastError();
        v = 65536;
    }
    const size_t cap = std::min<size_t>((size_t)v, 160 * 1024);
    return cap > 8192 ? cap - 8192 : 0;  // the static reduction arrays and a margin
}

// First block of each of G members of a plan (G + 1 entries, the last P.p + 1):
// contiguous ranges of the subdomain blocks balanced by rows, at least one per
// member; the last member also takes the interface block (its rows count).
std::vector<int32_t> member_blocks(const HostPlan& P, int G) {
    std::vector<int32_t> cut(G + 1, 0);
    cut[G] = P.p + 1;
    const double target = (double)P.n / G;
    for (int g = 1; g < G; ++g) {
        int32_t b = cut[g - 1] + 1;
        while (b < P.p - (G - g) && (double)P.boff[b] < g * target) ++b;
        cut[g] = b;
    }
    return cut;
}

// Tables for the systems of `plans` (one per system; offsets r0 / s0 / d0, c0
// per system, rank k), tsz = bytes of the preconditioner's type.  groups: the
// workgroups per system (empty: one each); lds_cap: largest dynamic LDS of a
// launch (0: the device's).
void persist_build(PersistData& PD, const std::vector<const HostPlan*>& plans, const std::vector<int64_t>& roff,
                   const std::vector<int64_t>& soff, const std::vector<int>& ks, const std::vector<double>& c0s,
                   int kstride, size_t tsz, int dev, const std::vector<int>& groups = {}, size_t lds_cap = 0) {
    MergedLevels M;
    std::vector<int64_t> arp(1, 0);
    std::vector<int32_t> aci;
    std::vector<double> av;
    size_t budget = persist_lds_budget(dev);
    if (lds_cap) budget = std::min(budget, lds_cap);
    PD.hsys.clear();
    PD.lds_bytes = 0;
    // the level metadata of the deepest system takes (levels + 1) x 16 bytes of LDS
    int maxlev = 0;
    for (const HostPlan* P : plans) {
        int depth = 0;
        for (int32_t b = 0; b <= P->p; ++b) depth = std::max(depth, P->blk_lvl[b + 1] - P->blk_lvl[b]);
        maxlev = std::max(maxlev, depth);
    }
    const size_t meta_bytes = 16 * (size_t)(maxlev + 1);
    if (meta_bytes + 16 > persist_lds_budget(dev) + 8192 - 4096)
        throw SetupError{DDLR_E_INVALID, "too many levels for the persistent form"};
    budget = budget > meta_bytes ? budget - meta_bytes : 0;
    PD.ngroups = 0;
    PD.members.assign(plans.size(), 1);
    PD.entry_sys.clear();
    PlanTranspose X;
    for (size_t q = 0; q < plans.size(); ++q) {
        const HostPlan& P = *plans[q];
        const int G = groups.empty() || P.p < 1 ? 1 : std::max(1, std::min(groups[q], kGroupMax));
        const int Gb = std::min(G, (int)P.p);  // members that own blocks
        PD.members[q] = G;
        const std::vector<int32_t> cut = member_blocks(P, Gb);
        plan_transpose(P, X);
        const int grp = G > 1 ? PD.ngroups++ : -1;
        for (int g = 0; g < G; ++g) {
            PSys S{};
            S.r0 = roff[q];
            S.s0 = soff[q];
            S.d0 = (int64_t)q * kstride;
            S.n = (int32_t)P.n;
            S.m = (int32_t)P.m;
            S.s = (int32_t)P.s;
            S.k = ks[q];
            S.c0 = c0s[q];
            const int32_t b0 = g < Gb ? cut[g] : P.p + 1, b1 = g < Gb ? cut[g + 1] : P.p + 1;
            S.o0 = (int32_t)P.boff[b0];
            S.o1 = (int32_t)P.boff[b1];
            S.G = G;
            S.g = g;
            S.grp = grp;
            S.ifc = g == Gb - 1;
            S.v0 = (int32_t)(P.n * g / G);
            S.v1 = (int32_t)(P.n * (g + 1) / G);
            persist_levels(P, X, roff[q], b0, b1, M, S.l0, S.l1);
            const size_t need = (size_t)(S.o1 - S.o0) * tsz;
            S.lds = need <= budget;
            if (S.lds) PD.lds_bytes = std::max(PD.lds_bytes, need);
            PD.hsys.push_back(S);
            PD.entry_sys.push_back((int)q);
        }
        persist_csr(P, roff[q], arp, aci, av);
    }
    PD.meta_off = (int)((PD.lds_bytes + 15) & ~(size_t)15);
    PD.lds_bytes = PD.meta_off + meta_bytes;
    M.meta.push_back(int4{(int)M.mrow.size(), 0, (int)M.fcol.size(), (int)M.bcol.size()});
    // clamped prefetch loads of a level without entries read up to 1024 entries past its start
    for (int u = 0; u < 1024; ++u) {
        M.fcol.push_back(0);
        M.fval.push_back(0.0);
        M.bcol.push_back(0);
        M.bval.push_back(0.0);
    }
    PD.sys = PD.mem.upload(PD.hsys);
    PD.meta = PD.mem.upload(M.meta);
    PD.mrow = PD.mem.upload(M.mrow);
    PD.fcol = PD.mem.upload(M.fcol);
    PD.bcol = PD.mem.upload(M.bcol);
    if (tsz == sizeof(double)) {
        PD.fval = PD.mem.upload(M.fval);
        PD.bval = PD.mem.upload(M.bval);
        PD.dq = PD.mem.upload(M.dq);
    } else {
        PD.fval = PD.mem.upload(std::vector<float>(M.fval.begin(), M.fval.end()));
        PD.bval = PD.mem.upload(std::vector<float>(M.bval.begin(), M.bval.end()));
        PD.dq = PD.mem.upload(std::vector<float>(M.dq.begin(), M.dq.end()));
    }
    PD.arp = PD.mem.upload(arp);
    PD.aci = PD.mem.upload(aci);
    PD.av = PD.mem.upload(av);
    if (PD.ngroups > 0) {
        PD.gctr = PD.mem.alloc<unsigned>((size_t)PD.ngroups * 64);
        PD.gpart = PD.mem.alloc<double>((size_t)PD.ngroups * 4 * kGroupMax);
        PD.gxcc = PD.mem.alloc<int>((size_t)PD.ngroups * kGroupMax);
    }
}

void persist_lanes(PersistData& PD, const std::vector<PLane>& lanes, int cols, int64_t n);

// Lane table of a batch whose systems have PD.members workgroups each (table
// entries in system order).  Ungrouped: lane q is system q.  Grouped: lanes
// are dealt to the XCDs (lane l runs on XCD l mod nxcd, the dispatch order of
// the device), every group on one XCD so that its barriers take the fast form,
// the groups first, largest first, each on the XCD with the fewest lanes;
// idle lanes fill the grid to a multiple of nxcd.
void persist_batch_lanes(PersistData& PD, int64_t n, int nxcd) {
    const int ns = (int)PD.members.size();
    std::vector<int> first(ns + 1, 0);
    for (int q = 0; q < ns; ++q) first[q + 1] = first[q] + PD.members[q];
    PD.sys_lane.assign(ns, 0);
    std::vector<PLane> lanes;
    if (PD.ngroups == 0) {
        for (int q = 0; q < ns; ++q) {
            lanes.push_back(PLane{first[q], 0});
            PD.sys_lane[q] = q;
        }
        PD.grid = ns;
    } else {
        std::vector<int> ord(ns);
        for (int q = 0; q < ns; ++q) ord[q] = q;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return PD.members[a] > PD.members[b]; });
        std::vector<std::vector<int>> slot(nxcd);  // table entries per XCD, in slot order
        for (int q : ord) {
            int x = 0;
            for (int y = 1; y < nxcd; ++y)
                if (slot[y].size() < slot[x].size()) x = y;
            for (int g = 0; g < PD.members[q]; ++g) slot[x].push_back(first[q] + g);
        }
        size_t depth = 0;
        for (const auto& v : slot) depth = std::max(depth, v.size());
        lanes.assign(depth * nxcd, PLane{-1, 0});
        for (int x = 0; x < nxcd; ++x)
            for (size_t t = 0; t < slot[x].size(); ++t) lanes[t * nxcd + x] = PLane{slot[x][t], 0};
        for (size_t l = 0; l < lanes.size(); ++l)
            if (lanes[l].sys >= 0 && PD.hsys[lanes[l].sys].g == 0) {
                int q = 0;
                while (first[q + 1] <= lanes[l].sys) ++q;
                PD.sys_lane[q] = (int)l;
            }
        PD.grid = (int)lanes.size();
    }
    persist_lanes(PD, lanes, 1, n);
}

// Lane table and per-lane results / vectors for `nl` lanes (columns `cols`).
void persist_lanes(PersistData& PD, const std::vector<PLane>& lanes, int cols, int64_t n) {
    if ((int)lanes.size() > PD.nlanes) {
        PD.lanes = PD.mem.alloc<PLane>(lanes.size());
        PD.res = PD.mem.alloc<PRes>(lanes.size());
        PD.nlanes = (int)lanes.size();
    }
    HIPCHK(hipMemcpy(PD.lanes, lanes.data(), lanes.size() * sizeof(PLane), hipMemcpyHostToDevice));
    PD.hlanes = lanes;
    if (cols > PD.cols) {
        PD.b = PD.mem.alloc<double>((size_t)n * cols);
        PD.p = PD.mem.alloc<double>((size_t)n * cols);
        PD.cols = cols;
    }
}

// Workgroups of k_pcg_persist<T, NT> with PD's dynamic LDS the device keeps
// resident at once (the dynamic-LDS attribute must be set first).
template <typename T, int NT> int persist_resident_nt(const ddlr_prec* h, const PersistData& PD) {
    int occ = 0, cus = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_pcg_persist<T, NT>, NT, PD.lds_bytes));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    return occ * cus;
}

template <typename T, int NT>
void persist_launch_nt(ddlr_prec* h, PersistData& PD, int nl, double tol2, int maxit, hipStream_t st) {
    const DevFactors<T>& F = factors<T>(h);
    Workspace& W = h->ws;
    const bool multi = h->batch;  // per-system coefficients of a batch (also of one system)
    const T* U = F.U;
    const int ustride = std::max(1, h->k);
    const double* dco = multi ? h->dvecs : h->dvec;
    if (PD.ngroups > 0) {
        // every member of a group must be resident together: the grid may not
        // exceed what the device holds at once
        if (nl > persist_resident_nt<T, NT>(h, PD))
            throw SetupError{DDLR_E_INVALID, "grouped persistent launch larger than the resident workgroups"};
        const int64_t nc = (int64_t)PD.ngroups * 64;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, nc, PD.gctr);
        LAUNCHCHK();
    }
    auto kern = k_pcg_persist<T, NT>;
    hipLaunchKernelGGL(kern, dim3(nl), dim3(NT), PD.lds_bytes, st, PD.sys, PD.lanes, PD.arp, PD.aci, PD.av, PD.meta,
                       PD.mrow, PD.fcol, (const T*)PD.fval, PD.bcol, (const T*)PD.bval, (const T*)PD.dq, h->erp,
                       h->eci, F.ev, h->etrp,
                       h->etci, F.etv, U, ustride, dco, PD.b, W.x, W.r, PD.p, W.q, W.z, (T*)W.a1, (T*)W.a2, (T*)W.ys,
                       (T*)W.ws, h->ndev, h->sdev, PD.meta_off, tol2, maxit, PD.res, PD.gctr, PD.gpart, PD.gxcc,
                       PD.gslow, PD.gspin);
    LAUNCHCHK();
}

// Allows the kernel of `nt` threads the dynamic LDS of PD (above 64 KB it must be
// raised first; done once per device, kernel and size, outside any capture).
template <typename T, int NT> void persist_lds_attr_nt(int dev, size_t bytes) {
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, bool> done;
    if (bytes <= 65536) return;
    std::lock_guard<std::mutex> lk(mu);
    bool& d = done[std::make_pair(dev, bytes)];
    if (d) return;
    HIPCHK(hipFuncSetAttribute((const void*)k_pcg_persist<T, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes));
    d = true;
}

void persist_lds_attr(const ddlr_prec* h, const PersistData& PD, int nt) {
    const bool f64 = h->precision == DDLR_FP64;
    switch (nt) {
    case 64:
        f64 ? persist_lds_attr_nt<double, 64>(h->device, PD.lds_bytes) : persist_lds_attr_nt<float, 64>(h->device, PD.lds_bytes);
        break;
    case 128:
        f64 ? persist_lds_attr_nt<double, 128>(h->device, PD.lds_bytes) : persist_lds_attr_nt<float, 128>(h->device, PD.lds_bytes);
        break;
    case 256:
        f64 ? persist_lds_attr_nt<double, 256>(h->device, PD.lds_bytes) : persist_lds_attr_nt<float, 256>(h->device, PD.lds_bytes);
        break;
    case 512:
        f64 ? persist_lds_attr_nt<double, 512>(h->device, PD.lds_bytes) : persist_lds_attr_nt<float, 512>(h->device, PD.lds_bytes);
        break;
    default:
        f64 ? persist_lds_attr_nt<double, 1024>(h->device, PD.lds_bytes)
            : persist_lds_attr_nt<float, 1024>(h->device, PD.lds_bytes);
    }
}

template <typename T> void persist_launch_T(ddlr_prec* h, PersistData& PD, int nl, double tol2, int maxit,
                                            hipStream_t st, int nt) {
    switch (nt) {
    case 64: persist_launch_nt<T, 64>(h, PD, nl, tol2, maxit, st); break;
    case 128: persist_launch_nt<T, 128>(h, PD, nl, tol2, maxit, st); break;
    case 256: persist_launch_nt<T, 256>(h, PD, nl, tol2, maxit, st); break;
    case 512: persist_launch_nt<T, 512>(h, PD, nl, tol2, maxit, st); break;
    default: persist_launch_nt<T, 1024>(h, PD, nl, tol2, maxit, st);
    }
}

// persist_resident_nt for the preconditioner's type and nt threads
int persist_resident(ddlr_prec* h, const PersistData& PD, int nt) {
    persist_lds_attr(h, PD, nt);
    const bool f64 = h->precision == DDLR_FP64;
    switch (nt) {
    case 64: return f64 ? persist_resident_nt<double, 64>(h, PD) : persist_resident_nt<float, 64>(h, PD);
    case 128: return f64 ? persist_resident_nt<double, 128>(h, PD) : persist_resident_nt<float, 128>(h, PD);
    case 256: return f64 ? persist_resident_nt<double, 256>(h, PD) : persist_resident_nt<float, 256>(h, PD);
    case 512: return f64 ? persist_resident_nt<double, 512>(h, PD) : persist_resident_nt<float, 512>(h, PD);
    default: return f64 ? persist_resident_nt<double, 1024>(h, PD) : persist_resident_nt<float, 1024>(h, PD);
    }
}

void persist_launch(ddlr_prec* h, PersistData& PD, int nl, double tol2, int maxit, hipStream_t st, int nt) {
    if (!h->capturing) persist_lds_attr(h, PD, nt);
    if (h->precision == DDLR_FP64) persist_launch_T<double>(h, PD, nl, tol2, maxit, st, nt);
    else persist_launch_T<float>(h, PD, nl, tol2, maxit, st, nt);
}

// Tunes the workgroup size of a persistent launch over nl lanes whose b is in
// PD.b: each candidate runs min(maxit, 12) iterations, timed with events on
// st; the fastest per iteration is kept.  The trial results are overwritten by
// the real solve.
void persist_tune(ddlr_prec* h, PersistData& PD, int nl, double tol2, int maxit, hipStream_t st) {
    if (const char* env = std::getenv("DDLR_PERSIST_NT")) {
        const int v = std::atoi(env);
        if (v == 64 || v == 128 || v == 256 || v == 512 || v == 1024) {
            PD.nt = v;
            return;
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int trial = std::min(maxit, 12);
    const int cand[5] = {64, 128, 256, 512, 1024};
    float best = 1e30f;
    std::vector<PRes> r(nl);
    for (int c = 0; c < 5; ++c) {
        PD.nt_us[c] = 0.f;
        if (PD.ngroups > 0 && nl > persist_resident(h, PD, cand[c])) continue;  // groups would not be resident
        HIPCHK(hipEventRecord(e0, st));
        persist_launch(h, PD, nl, tol2, trial, st, cand[c]);
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        HIPCHK(hipMemcpy(r.data(), PD.res, nl * sizeof(PRes), hipMemcpyDeviceToHost));
        int its = 1;
        if (PD.sys_lane.empty())
            for (const PRes& x : r) its = std::max(its, x.its);
        else
            for (int l : PD.sys_lane) its = std::max(its, r[l].its);
        PD.nt_us[c] = 1e3f * ms / (float)its;
        if (PD.nt_us[c] < best) {
            best = PD.nt_us[c];
            PD.nt = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (PD.nt == 0) throw SetupError{DDLR_E_INVALID, "no workgroup size keeps the grouped launch resident"};
}

// Workgroups per system of a persistent batch.  The batch takes as long as its
// slowest system, so the system with the largest estimated solve time gets
// more members while that lowers its estimate and the lanes fit `slots`.
// Estimate (256-thread workgroups): iterations ~ sqrt(n) (these stencils'
// condition numbers grow with the grid side); per iteration four sweeps over
// the deepest block member's merged levels (0.25 us a level with its solve
// vector in LDS, 2.5 us in global memory) and 5 ns per row of its blocks,
// 12 ns per row of the vector steps (n / G rows), and seven group barriers of
// 3 us when G > 1.  Systems start at the fewest members whose solve vectors
// fit LDS.  Only the ratios matter; of the forms tried on the 256-system
// batch this one measured fastest.
//
// scale (optional, per system): measured time over the estimate at the
// grouping measured, so that the estimates of other groupings follow the
// measurement (the first solve's regrouping).
double group_est(const HostPlan& P, int g, size_t tsz, size_t lds_cap) {
    const int gb = std::max(1, std::min(g, (int)P.p));
    const std::vector<int32_t> cut = member_blocks(P, gb);
    double worst = 0.0;
    for (int u = 0; u < gb; ++u) {
        const int64_t rows = P.boff[cut[u + 1]] - P.boff[cut[u]];
        int depth = 0;
        for (int32_t b = cut[u]; b < cut[u + 1]; ++b) depth = std::max(depth, P.blk_lvl[b + 1] - P.blk_lvl[b]);
        const double lev = (size_t)rows * tsz <= lds_cap ? 0.25 : 2.5;
        worst = std::max(worst, 4.0 * depth * lev + 0.005 * (double)rows);
    }
    worst += 0.012 * (double)P.n / g;
    if (g > 1) worst += 7 * 3.0;
    return std::sqrt((double)P.n) * worst;
}

std::vector<int> choose_groups(const std::vector<const HostPlan*>& plans, size_t tsz, size_t lds_cap, int slots,
                               const std::vector<double>* scale = nullptr) {
    const int ns = (int)plans.size();
    std::vector<int> G(ns, 1);
    auto est = [&](int q, int g) { return group_est(*plans[q], g, tsz, lds_cap) * (scale ? (*scale)[q] : 1.0); };
    int total = ns;
    if (total >= slots) return G;
    // the fewest members that bring every member's solve vector into LDS
    for (int q = 0; q < ns; ++q) {
        const HostPlan& P = *plans[q];
        const int gmax = std::min((int)P.p, kGroupMax);
        for (int g = 1; g <= gmax && P.p >= 1; ++g) {
            const std::vector<int32_t> cut = member_blocks(P, g);
            int64_t big = 0;
            for (int u = 0; u < g; ++u) big = std::max(big, P.boff[cut[u + 1]] - P.boff[cut[u]]);
            if ((size_t)big * tsz <= lds_cap || g == gmax) {
                if ((size_t)big * tsz <= lds_cap && est(q, g) < est(q, G[q])) {
                    total += g - G[q];
                    G[q] = g;
                }
                break;
            }
        }
    }
    if (total > slots) return std::vector<int>(ns, 1);
    std::priority_queue<std::pair<double, int>> pq;
    for (int q = 0; q < ns; ++q) pq.push({est(q, G[q]), q});
    while (!pq.empty() && total < slots) {
        const auto [e, q] = pq.top();
        pq.pop();
        const int gmax = plans[q]->p < 1 ? 1 : std::min(kGroupMax, G[q] + (slots - total));
        int best = 0;
        double eb = e;
        for (int g = G[q] + 1; g <= std::min(gmax, G[q] + 4); ++g) {
            const double e2 = est(q, g);
            if (e2 < 0.98 * eb) {
                eb = e2;
                best = g;
                break;  // the smallest step that helps
            }
        }
        if (!best) break;  // the slowest system cannot be made faster
        total += best - G[q];
        G[q] = best;
        pq.push({eb, q});
    }
    return G;
}

// Whether a handle may solve with the persistent form: CG, DDLR-1 or A0 only,
// C_alpha factored, FP64 or FP32, rank at most kPersistMaxK.
bool persist_eligible(const ddlr_prec* h) {
    return (h->variant == DDLR_1 || h->variant == DDLR_VARIANT_A0) && h->plan.csolve == 0 &&
           h->precision != DDLR_FP32_UK_BF16 && h->k <= kPersistMaxK && !h->batch;
}

// Tables of a single-system handle, built on first use.
PersistData& persist_single(ddlr_prec* h) {
    if (!h->pers) {
        std::unique_ptr<PersistData> PD(new PersistData());
        PD->mem.budget = budget_of(h);
        persist_build(*PD, {&h->plan}, {0}, {0}, {h->variant == DDLR_1 ? h->k : 0}, {h->c0}, 0,
                      h->precision == DDLR_FP64 ? sizeof(double) : sizeof(float), h->device);
        h->pers = std::move(PD);
    }
    return *h->pers;
}

// Whether ddlr_solve runs an nr-column CG with the persistent form: forced by
// DDLR_CG_PERSIST, else measured -- the first eligible solve of a column count
// runs persistent (its time per iteration is kept), the following ones run the
// chunked forms until their measurement is done, then the faster per
// iteration is used.
bool persist_choose(ddlr_prec* h, int nr) {
    if (h->pers_mode == 0 || !persist_eligible(h) || h->ndev > kPersistMaxRows || h->capturing) return false;
    if (h->pers_mode == 1) return true;
    auto it = h->pers_us.find(nr);
    if (it == h->pers_us.end()) return true;
    const ddlr_prec::CgMode& m = h->cg_mode[nr];
    if (m.graph < 0) return false;
    const double chunk = m.us[m.graph][m.ov + 1];
    return it->second < chunk / 8.0;
}

// One persistent launch solving nr columns (b, x user order); fills info,
// returns DDLR_E_NO_CONVERGENCE if a column hit maxit.
ddlr_status persist_solve(ddlr_prec* h, int nr, const double* b, int64_t ldb, double* x, int64_t ldx,
                          const ddlr_solve_options& o, hipStream_t st, ddlr_solve_info* info) {
    PersistData& PD = persist_single(h);
    const int64_t n = h->ndev;
    std::vector<PLane> lanes(nr);
    for (int c = 0; c < nr; ++c) lanes[c] = PLane{0, c};
    persist_lanes(PD, lanes, nr, n);
    hipLaunchKernelGGL((k_gather<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr, h->perm_dev, b, ldb, PD.b,
                       n);
    LAUNCHCHK();
    const double tol2 = o.rtol * o.rtol;
    if (PD.nt == 0) persist_tune(h, PD, nr, tol2, o.maxit, st);
    const bool measure = h->pers_mode == 2 && !h->pers_us.count(nr);
    const auto t0 = std::chrono::steady_clock::now();
    persist_launch(h, PD, nr, tol2, o.maxit, st, PD.nt);
    hipLaunchKernelGGL((k_scatter<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr, h->perm_dev, h->ws.x, n, x,
                       ldx);
    LAUNCHCHK();
    std::vector<PRes> r(nr);
    HIPCHK(hipMemcpyAsync(r.data(), PD.res, nr * sizeof(PRes), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int its = 1;
    ddlr_status out = DDLR_OK;
    for (int c = 0; c < nr; ++c) {
        ddlr_solve_info& inf = info[c];
        inf.iters = r[c].its;
        inf.status = r[c].status == 0 ? DDLR_OK : DDLR_E_NO_CONVERGENCE;
        inf.relres = r[c].bb > 0 ? std::sqrt(r[c].rr / r[c].bb) : 0.0;
        inf.relres_true = r[c].bb > 0 ? std::sqrt(r[c].rtrue / r[c].bb) : 0.0;
        if (r[c].status) out = DDLR_E_NO_CONVERGENCE;
        its = std::max(its, r[c].its);
    }
    if (measure)
        h->pers_us[nr] = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() / its;
    return out;
}


}  // namespace

extern "C" {

ddlr_status ddlr_solve(ddlr_prec* h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                       const ddlr_solve_options* opt_in, ddlr_solve_info* info, void* stream) {
    ddlr_status st0 = check_vec(h, nrhs, b, ldb, x, ldx);
    if (st0 != DDLR_OK) return st0;
    ddlr_solve_options o;
    if (opt_in) o = *opt_in;
    else ddlr_solve_options_default(&o);
    if (!info || o.maxit < 1 || !(o.rtol > 0.0) || (o.method != 0 && o.method != 1)) {
        g_err = "bad solve options";
        return DDLR_E_INVALID;
    }
    if (o.method == 1 && (o.restart < 1 || o.restart > 60)) {
        g_err = "GMRES restart must be in [1, 60]";
        return DDLR_E_INVALID;
    }
    if (o.method == 0 && !h->spd) {
        g_err = "preconditioner is not certified SPD (negative local pivot or largest Ritz value >= 1): use GMRES";
        return DDLR_E_NOT_SPD;
    }
    ddlr_status result = DDLR_OK;
    try {
        HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        hipStream_t st = (hipStream_t)stream;
        const int64_t n = h->ndev;
        for (int32_t c0 = 0; c0 < nrhs; c0 += kMaxRhs) {
            const int nr = std::min<int>(kMaxRhs, nrhs - c0);
            ensure_ws(h, nr);
            autotune(h, nr, st, false);
            Workspace& W = h->ws;
            if (o.method == 0 && persist_choose(h, nr)) {
                const ddlr_status ps = persist_solve(h, nr, b + c0 * ldb, ldb, x + c0 * ldx, ldx, o, st, info + c0);
                if (ps != DDLR_OK) result = ps;
                continue;
            }
            hipLaunchKernelGGL((k_gather<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr,
                               h->perm_dev, b + c0 * ldb, ldb, W.r, n);
            LAUNCHCHK();
            if (o.method == 0) pcg_dev(h, nr, o, st);
            else gmres_dev(h, nr, o, st);
            hipLaunchKernelGGL((k_scatter<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr,
                               h->perm_dev, W.x, n, x + c0 * ldx, ldx);
            LAUNCHCHK();
            // true residual: q = b - A x (device order), recursive residual from the lanes
            hipLaunchKernelGGL((k_gather<double, double>), grid2(n, nr), dim3(256), 0, st, n, nr,
                               h->perm_dev, b + c0 * ldb, ldb, W.r, n);
            LAUNCHCHK();
            spmv_dev(h, nr, W.x, n, W.q, n, nullptr, st, nullptr);
            hipLaunchKernelGGL(k_sub, dim3(grid_for(n * nr)), dim3(256), 0, st, n * nr, W.r, W.q, W.z);
            LAUNCHCHK();
            std::vector<CgLane> lanes(nr);
            std::vector<double> rr(nr);
            HIPCHK(hipMemcpyAsync(lanes.data(), W.lanes, nr * sizeof(CgLane), hipMemcpyDeviceToHost, st));
            dot_dev(h, nr, W.z, W.z, n, st, nullptr);
            HIPCHK(hipMemcpyAsync(rr.data(), W.sums, nr * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int c = 0; c < nr; ++c) {
                ddlr_solve_info& inf = info[c0 + c];
                const double bb = lanes[c].bb;
                inf.iters = lanes[c].its;
                const bool conv = bb == 0.0 || lanes[c].rr <= o.rtol * o.rtol * bb || (o.method == 1 && lanes[c].active);
                inf.status = conv ? DDLR_OK : DDLR_E_NO_CONVERGENCE;
                inf.relres = bb > 0 ? std::sqrt(lanes[c].rr / bb) : 0.0;
                inf.relres_true = bb > 0 ? std::sqrt(rr[c] / bb) : 0.0;
                if (!conv) result = DDLR_E_NO_CONVERGENCE;
            }
        }
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    if (result != DDLR_OK) g_err = "some right-hand sides did not converge";
    return result;
}

ddlr_status ddlr_query(const ddlr_prec* h, ddlr_info* info) {
    if (!h || !info) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::memset(info, 0, sizeof(*info));
    const HostPlan& P = h->plan;
    info->n = P.n;
    info->m = P.m;
    info->s = P.s;
    info->nnz_a = P.A.nnz();
    info->nnz_l = P.L.nnz();
    info->nnz_e = P.A.nnz() - P.A0.nnz() + P.s;  // unused rough figure, recomputed below
    int64_t ne = 0;
    for (int64_t i = 0; i < P.m; ++i)
        for (int64_t t = P.A.rp[i]; t < P.A.rp[i + 1]; ++t) ne += P.A.ci[t] >= P.m;
    info->nnz_e = ne + P.s;
    info->p = P.p;
    info->k = h->k;
    info->variant = h->variant;
    info->lanczos_steps = h->msteps;
    info->ncolours = P.ncolours;
    info->levels_b_max = P.levels_b_max;
    info->levels_c = P.levels_c;
    info->spd = h->spd;
    info->precision = h->precision;
    info->on_device = h->device >= 0;
    info->theta = h->theta;
    info->c0 = h->c0;
    // stored entries: L (strict lower) + D + E + U_k (+ H_k)
    const double stored = (double)P.L.nnz() + (double)P.n + (double)info->nnz_e + (double)h->urows * h->k +
                          (h->variant == DDLR_2 ? (double)h->k * h->k : 0.0);
    info->fill_ratio = stored / (double)P.A.nnz();
    info->setup_ms = h->setup_ms;
    info->lanczos_ms = h->lanczos_ms;
    info->lanczos_reorth = h->lreorth;
    info->lanczos_reorth_steps = 0;
    for (int32_t f : h->rflags) info->lanczos_reorth_steps += f;
    info->csolve = P.csolve == 1 ? DDLR_CSOLVE_MR : P.csolve == 2 ? DDLR_CSOLVE_CHEB : DDLR_CSOLVE_FACTOR;
    info->cheb_lo = P.ch_lo;
    info->cheb_hi = P.ch_hi;
    info->cheb_ritz_lo = P.ch_rlo;
    info->cheb_ritz_hi = P.ch_rhi;
    info->cinv_iters = P.x_iters;
    info->nnz_cinv = P.csolve == 1 ? P.X.nnz() : 0;
    info->cinv_res = P.csolve == 1 ? P.x_res.back() : 0.0;
    info->cinv_res_inf = P.csolve == 1 ? P.x_rinf : 0.0;
    if (P.csolve == 1) info->fill_ratio += (double)P.X.nnz() / (double)P.A.nnz();
    return DDLR_OK;
}

ddlr_status ddlr_get_cinv(const ddlr_prec* h, int64_t* row_ptr, int32_t* col, double* val, double* res) {
    if (!h || !row_ptr || !col || !val) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    const HostPlan& P = h->plan;
    if (P.csolve != 1) {
        g_err = "the preconditioner does not solve C_alpha by the approximate inverse";
        return DDLR_E_INVALID;
    }
    std::copy(P.X.rp.begin(), P.X.rp.end(), row_ptr);
    std::copy(P.X.ci.begin(), P.X.ci.end(), col);
    std::copy(P.X.v.begin(), P.X.v.end(), val);
    if (res) std::copy(P.x_res.begin(), P.x_res.end(), res);
    return DDLR_OK;
}

ddlr_status ddlr_get_ordering(const ddlr_prec* h, int32_t* perm, int32_t* iface, int32_t* colour) {
    if (!h) {
        g_err = "null handle";
        return DDLR_E_INVALID;
    }
    const HostPlan& P = h->plan;
    if (perm) std::copy(P.perm.begin(), P.perm.end(), perm);
    if (iface) std::copy(P.iface.begin(), P.iface.end(), iface);
    if (colour) std::copy(P.colour.begin(), P.colour.end(), colour);
    return DDLR_OK;
}

ddlr_status ddlr_get_factor(const ddlr_prec* h, int64_t* row_ptr, int32_t* col, double* val, double* D) {
    if (!h) {
        g_err = "null handle";
        return DDLR_E_INVALID;
    }
    const HostPlan& P = h->plan;
    if (row_ptr) std::copy(P.L.rp.begin(), P.L.rp.end(), row_ptr);
    if (col) std::copy(P.L.ci.begin(), P.L.ci.end(), col);
    if (val) std::copy(P.L.v.begin(), P.L.v.end(), val);
    if (D) std::copy(P.D.begin(), P.D.end(), D);
    return DDLR_OK;
}

ddlr_status ddlr_partition_graph(const ddlr_csr* A, int32_t p, int32_t* part) {
    if (!A || !part || !A->row_ptr || !A->col_idx || A->n < 1 || p < 1) {
        g_err = "null argument, n < 1 or p < 1";
        return DDLR_E_INVALID;
    }
    try {
        partition_graph(A->n, A->row_ptr, A->col_idx, p, part);
    } catch (const SetupError& e) {
        return fail_status(e);
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return DDLR_E_OOM;
    }
    return DDLR_OK;
}

ddlr_status ddlr_partition_box(int32_t nx, int32_t ny, int32_t nz, int32_t px, int32_t py, int32_t pz,
                               int32_t* part) {
    if (!part || nx < 1 || ny < 1 || nz < 1 || px < 1 || py < 1 || pz < 1 || px > nx || py > ny || pz > nz) {
        g_err = "ddlr_partition_box: need 1 <= p_d <= n_d on every axis and a non-null output";
        return DDLR_E_INVALID;
    }
    // first index of each part along an axis: the first (N mod P) parts hold one point more
    auto cuts = [](int32_t N, int32_t P) {
        std::vector<int32_t> lab(N);
        const int32_t base = N / P, extra = N % P;
        int32_t i = 0;
        for (int32_t q = 0; q < P; ++q)
            for (int32_t c = 0; c < base + (q < extra ? 1 : 0); ++c) lab[i++] = q;
        return lab;
    };
    const std::vector<int32_t> lx = cuts(nx, px), ly = cuts(ny, py), lz = cuts(nz, pz);
    int64_t u = 0;
    for (int32_t z = 0; z < nz; ++z)
        for (int32_t y = 0; y < ny; ++y)
            for (int32_t x = 0; x < nx; ++x) part[u++] = lx[x] + px * (ly[y] + py * lz[z]);
    return DDLR_OK;
}

ddlr_status ddlr_get_levels(const ddlr_prec* h, int32_t* level) {
    if (!h || !level) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::copy(h->plan.level.begin(), h->plan.level.end(), level);
    return DDLR_OK;
}

ddlr_status ddlr_get_lanczos(const ddlr_prec* h, double* alpha, double* beta, double* ritz) {
    if (!h) {
        g_err = "null handle";
        return DDLR_E_INVALID;
    }
    if (alpha) std::copy(h->ta.begin(), h->ta.end(), alpha);
    if (beta) std::copy(h->tb.begin(), h->tb.end(), beta);
    if (ritz) std::copy(h->ritz.begin(), h->ritz.end(), ritz);
    return DDLR_OK;
}

ddlr_status ddlr_get_lanczos_reorth(const ddlr_prec* h, int32_t* flags) {
    if (!h || !flags) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    if (h->ta.empty()) {
        g_err = "no Lanczos run";
        return DDLR_E_INVALID;
    }
    std::copy(h->rflags.begin(), h->rflags.end(), flags);
    return DDLR_OK;
}

ddlr_status ddlr_get_lowrank(const ddlr_prec* h, double* U, double* aux) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    if (h->variant == 0 || h->k == 0) {
        g_err = "no low-rank part";
        return DDLR_E_INVALID;
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        const HostPlan& P = h->plan;
        const int k = h->k;
        std::vector<double> Ur((size_t)h->urows * k);
        HIPCHK(hipMemcpy(Ur.data(), h->f64.U, Ur.size() * sizeof(double), hipMemcpyDeviceToHost));
        if (U) {
            std::fill(U, U + (size_t)P.n * k, 0.0);
            const int64_t off = h->variant == DDLR_1 ? P.m : 0;
            for (int64_t i = 0; i < h->urows; ++i) {
                const int32_t user = P.perm[P.dev2int[off + i]];
                for (int j = 0; j < k; ++j) U[user + (size_t)j * P.n] = Ur[(size_t)i * k + j];
            }
        }
        if (aux) {
            if (h->variant == DDLR_1) {
                std::copy(h->lam.begin(), h->lam.end(), aux);
                aux[k] = h->theta;
            } else {
                std::copy(h->H_h.begin(), h->H_h.end(), aux);
            }
        }
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

ddlr_status ddlr_set_lowrank(ddlr_prec* h, int32_t variant, int32_t k, const double* U, const double* aux) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    if ((variant != 1 && variant != 2) || k < 1 || k > 128 || !U || !aux) {
        g_err = "bad set_lowrank arguments";
        return DDLR_E_INVALID;
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        HIPCHK(hipDeviceSynchronize());
        const HostPlan& P = h->plan;
        const int64_t rows = variant == 1 ? P.s : P.n, off = variant == 1 ? P.m : 0;
        std::vector<double> Ur((size_t)rows * k);
        for (int64_t i = 0; i < rows; ++i) {
            const int32_t user = P.perm[P.dev2int[off + i]];
            for (int j = 0; j < k; ++j) Ur[(size_t)i * k + j] = U[user + (size_t)j * P.n];
        }
        drop_graphs(h);  // captured kernels hold the low-rank pointers
        h->lrun.mem.release();  // imported data: no Lanczos run to continue
        h->lrun = LanczosRun();
        h->lrmem.release();
        h->dvec = nullptr;
        h->Hk = nullptr;
        h->f64.U = nullptr;
        h->f32.U = nullptr;
        h->variant = variant;
        h->k = k;
        h->urows = rows;
        h->f64.U = h->lrmem.upload(Ur);
        if (h->precision != DDLR_FP64) {
            std::vector<float> f(Ur.size());
            for (size_t i = 0; i < f.size(); ++i) f[i] = (float)Ur[i];
            h->f32.U = h->lrmem.upload(f);
        }
        h->ubr = h->ubt = nullptr;
        make_bf16_basis(h);
        make_tiled_basis(h);
        if (variant == 1) {
            h->lam.assign(aux, aux + k);
            h->theta = aux[k];
            h->c0 = 1.0 / (1.0 - h->theta);
            h->dvec_h.resize(k);
            for (int j = 0; j < k; ++j) h->dvec_h[j] = 1.0 / (1.0 - h->lam[j]) - h->c0;
            h->spd = h->theta < 1.0 && h->lam[0] < 1.0 && h->pivots_positive;
            h->dvec = h->lrmem.upload(h->dvec_h);
        } else {
            h->H_h.assign(aux, aux + (size_t)k * k);
            h->Hk = h->lrmem.upload(h->H_h);
            h->spd = h->pivots_positive;
            h->theta = 0.0;
            h->c0 = 0.0;
        }
        h->ws.nrhs = 0;  // coefficient buffers depend on k
        h->ws.mem.release();
        h->ws.gmem.release();
        h->ws.gm_m = h->ws.gm_nrhs = 0;
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

}  // extern "C"

// ------------------------------------------------------------ setup files

namespace {

// One array of a setup file: name (at most 15 characters), element type
// (1 int32, 2 int64, 3 float64) and the elements.
struct SetupRec {
    int32_t type = 0;
    int64_t count = 0;
    std::vector<char> data;
};
constexpr char kSetupMagic[8] = {'D', 'D', 'L', 'R', 'S', 'E', 'T', '1'};

size_t rec_elem(int32_t type) { return type == 1 ? 4 : 8; }

template <typename T> int32_t rec_type();
template <> int32_t rec_type<int32_t>() { return 1; }
template <> int32_t rec_type<int64_t>() { return 2; }
template <> int32_t rec_type<double>() { return 3; }

template <typename T> void rec_put(std::map<std::string, SetupRec>& R, const char* name, const T* p, size_t count) {
    SetupRec& r = R[name];
    r.type = rec_type<T>();
    r.count = (int64_t)count;
    r.data.resize(count * sizeof(T));
    if (count) std::memcpy(r.data.data(), p, count * sizeof(T));
}

template <typename T> std::vector<T> rec_get(const std::map<std::string, SetupRec>& R, const char* name,
                                            int64_t want = -1) {
    auto it = R.find(name);
    if (it == R.end()) throw SetupError{DDLR_E_INVALID, std::string("setup file lacks the array ") + name};
    const SetupRec& r = it->second;
    if (r.type != rec_type<T>() || (want >= 0 && r.count != want))
        throw SetupError{DDLR_E_INVALID, std::string("setup file array ") + name + " has the wrong type or length"};
    std::vector<T> out((size_t)r.count);
    if (r.count) std::memcpy(out.data(), r.data.data(), (size_t)r.count * sizeof(T));
    return out;
}

void write_setup_file(const char* path, const std::map<std::string, SetupRec>& R) {
    FILE* f = std::fopen(path, "wb");
    if (!f) throw SetupError{DDLR_E_INVALID, std::string("cannot open ") + path + " for writing"};
    bool ok = std::fwrite(kSetupMagic, 1, 8, f) == 8;
    const int32_t head[2] = {1, (int32_t)R.size()};
    ok = ok && std::fwrite(head, sizeof(head), 1, f) == 1;
    for (const auto& kv : R) {
        char name[16] = {0};
        std::strncpy(name, kv.first.c_str(), 15);
        const int32_t tr[2] = {kv.second.type, 0};
        ok = ok && std::fwrite(name, 1, 16, f) == 16 && std::fwrite(tr, sizeof(tr), 1, f) == 1 &&
             std::fwrite(&kv.second.count, sizeof(int64_t), 1, f) == 1;
        if (!kv.second.data.empty())
            ok = ok && std::fwrite(kv.second.data.data(), 1, kv.second.data.size(), f) == kv.second.data.size();
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw SetupError{DDLR_E_INVALID, std::string("write error on ") + path};
}

std::map<std::string, SetupRec> read_setup_file(const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) throw SetupError{DDLR_E_INVALID, std::string("cannot open ") + path};
    std::map<std::string, SetupRec> R;
    auto bad = [&](const char* what) {
        std::fclose(f);
        return SetupError{DDLR_E_INVALID, std::string(path) + ": " + what};
    };
    char magic[8];
    int32_t head[2];
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, kSetupMagic, 8) != 0) throw bad("not a DDLR setup file");
    if (std::fread(head, sizeof(head), 1, f) != 1 || head[0] != 1 || head[1] < 0) throw bad("unsupported version");
    std::fseek(f, 0, SEEK_END);
    const long fsize = std::ftell(f);
    std::fseek(f, 16, SEEK_SET);
    for (int32_t q = 0; q < head[1]; ++q) {
        char name[17] = {0};
        int32_t tr[2];
        int64_t count = 0;
        if (std::fread(name, 1, 16, f) != 16 || std::fread(tr, sizeof(tr), 1, f) != 1 ||
            std::fread(&count, sizeof(count), 1, f) != 1)
            throw bad("truncated record header");
        if (tr[0] < 1 || tr[0] > 3 || count < 0) throw bad("bad record type or count");
        const size_t bytes = (size_t)count * rec_elem(tr[0]);
        if ((long)bytes > fsize - std::ftell(f)) throw bad("record longer than the file");
        SetupRec& r = R[name];
        r.type = tr[0];
        r.count = count;
        r.data.resize(bytes);
        if (bytes && std::fread(r.data.data(), 1, bytes, f) != bytes) throw bad("truncated record");
    }
    std::fclose(f);
    return R;
}

}  // namespace

extern "C" {

ddlr_status ddlr_ctx_create(int32_t device, size_t hbm_budget_bytes, ddlr_ctx** out) {
    if (!out) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    *out = nullptr;
    if (device < -1) {
        g_err = "device must be a HIP device ordinal or -1 (host only)";
        return DDLR_E_INVALID;
    }
    if (device >= 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
            (void)hipGetLastError();
            g_err = "no HIP device " + std::to_string(device);
            return DDLR_E_DEVICE;
        }
    }
    ddlr_ctx* c = new ddlr_ctx();
    c->device = device;
    c->budget.limit = hbm_budget_bytes;
    *out = c;
    return DDLR_OK;
}

ddlr_status ddlr_ctx_usage(const ddlr_ctx* ctx, size_t* used, size_t* peak, size_t* budget) {
    if (!ctx) {
        g_err = "null context";
        return DDLR_E_INVALID;
    }
    ddlr_ctx* c = const_cast<ddlr_ctx*>(ctx);
    std::lock_guard<std::mutex> lk(c->budget.mu);
    if (used) *used = c->budget.used;
    if (peak) *peak = c->budget.peak;
    if (budget) *budget = c->budget.limit;
    return DDLR_OK;
}

void ddlr_ctx_destroy(ddlr_ctx* ctx) { ctx_unref(ctx); }

ddlr_status ddlr_export_setup(const ddlr_prec* h, const char* path) {
    if (!h || !path) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    try {
        const HostPlan& P = h->plan;
        std::map<std::string, SetupRec> R;
        const int64_t np[2] = {P.n, P.p};
        rec_put(R, "n_p", np, 2);
        const double alpha = P.alpha;
        rec_put(R, "alpha", &alpha, 1);
        const int32_t flags[3] = {P.csolve, h->precision, h->cheb_nu};
        rec_put(R, "csolve_prec_nu", flags, 3);
        rec_put(R, "perm", P.perm.data(), P.perm.size());
        rec_put(R, "boff", P.boff.data(), P.boff.size());
        rec_put(R, "colour", P.colour.data(), P.colour.size());
        rec_put(R, "L.rowptr", P.L.rp.data(), P.L.rp.size());
        rec_put(R, "L.col", P.L.ci.data(), P.L.ci.size());
        rec_put(R, "L.val", P.L.v.data(), P.L.v.size());
        rec_put(R, "D", P.D.data(), P.D.size());
        rec_put(R, "level", P.level.data(), P.level.size());
        if (P.csolve == 1) {
            rec_put(R, "X.rowptr", P.X.rp.data(), P.X.rp.size());
            rec_put(R, "X.col", P.X.ci.data(), P.X.ci.size());
            rec_put(R, "X.val", P.X.v.data(), P.X.v.size());
            const double xi[2] = {P.x_rinf, P.x_spd ? 1.0 : 0.0};
            rec_put(R, "X.cert", xi, 2);
            rec_put(R, "X.res", P.x_res.data(), P.x_res.size());
        }
        if (P.csolve == 2) {
            const double ch[4] = {P.ch_lo, P.ch_hi, P.ch_rlo, P.ch_rhi};
            rec_put(R, "cheb", ch, 4);
        }
        if (h->device >= 0 && h->variant != 0 && h->k > 0) {
            const int k = h->k;
            std::vector<double> U((size_t)P.n * k), aux(h->variant == DDLR_1 ? (size_t)k + 1 : (size_t)k * k);
            ddlr_status st = ddlr_get_lowrank(h, U.data(), aux.data());
            if (st != DDLR_OK) return st;
            const int32_t vk[2] = {h->variant, k};
            rec_put(R, "lowrank", vk, 2);
            rec_put(R, "U", U.data(), U.size());
            rec_put(R, "aux", aux.data(), aux.size());
        }
        write_setup_file(path, R);
    } catch (const SetupError& e) {
        return fail_status(e);
    } catch (const std::bad_alloc&) {
        g_err = "host out of memory";
        return DDLR_E_OOM;
    }
    return DDLR_OK;
}

ddlr_status ddlr_import_setup(ddlr_ctx* ctx, const ddlr_csr* A, const char* path, ddlr_prec** out) {
    if (out) *out = nullptr;
    if (!A || !path || !out || !A->row_ptr || !A->col_idx || !A->val) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::unique_ptr<ddlr_prec> h(new ddlr_prec());
    attach_ctx(h.get(), ctx);
    auto t0 = std::chrono::steady_clock::now();
    try {
        const auto R = read_setup_file(path);
        const std::vector<int64_t> np = rec_get<int64_t>(R, "n_p", 2);
        if (np[0] != A->n) throw SetupError{DDLR_E_INVALID, "setup file is for another matrix order"};
        const int64_t n = np[0];
        const int32_t p = (int32_t)np[1];
        const double alpha = rec_get<double>(R, "alpha", 1)[0];
        const std::vector<int32_t> flags = rec_get<int32_t>(R, "csolve_prec_nu", 3);
        const int csolve = flags[0];
        if (csolve < 0 || csolve > 2 || flags[1] < 0 || flags[1] > 2 || (csolve == 2 && (flags[2] < 1 || flags[2] > 64)))
            throw SetupError{DDLR_E_INVALID, "setup file has a bad C_alpha solver, precision or step count"};
        h->precision = flags[1];
        HostCsr L;
        L.rp = rec_get<int64_t>(R, "L.rowptr", n + 1);
        L.ci = rec_get<int32_t>(R, "L.col");
        L.v = rec_get<double>(R, "L.val");
        build_plan_imported(h->plan, n, A->row_ptr, A->col_idx, A->val, p, alpha, rec_get<int32_t>(R, "perm", n),
                            rec_get<int64_t>(R, "boff", (int64_t)p + 2), rec_get<int32_t>(R, "colour"), std::move(L),
                            rec_get<double>(R, "D", n), csolve);
        HostPlan& P = h->plan;
        if (csolve == 1)
            for (int64_t r = P.m; r < n; ++r)
                if (P.L.rp[r + 1] != P.L.rp[r] || P.D[r] != 1.0)
                    throw SetupError{DDLR_E_INVALID,
                                     "with the approximate inverse of C_alpha the interface rows of L must be empty "
                                     "and D must be 1 there"};
        if (R.count("level") && rec_get<int32_t>(R, "level", n) != P.level)
            throw SetupError{DDLR_E_INVALID, "stored levels differ from the schedule of the stored factor"};
        if (csolve == 1) {
            P.X.rp = rec_get<int64_t>(R, "X.rowptr", P.s + 1);
            P.X.ci = rec_get<int32_t>(R, "X.col", P.X.rp.back());
            P.X.v = rec_get<double>(R, "X.val", P.X.rp.back());
            for (int64_t y = 0; y < P.s; ++y)
                for (int64_t t = P.X.rp[y]; t < P.X.rp[y + 1]; ++t)
                    if (P.X.ci[t] < 0 || P.X.ci[t] >= P.s || P.X.rp[y + 1] < P.X.rp[y])
                        throw SetupError{DDLR_E_INVALID, "stored X has a column outside the interface"};
            const std::vector<double> xc = rec_get<double>(R, "X.cert", 2);
            P.x_rinf = xc[0];
            P.x_spd = xc[1] != 0.0;
            P.x_res = rec_get<double>(R, "X.res");
            if (P.x_res.empty()) throw SetupError{DDLR_E_INVALID, "stored X has no residual history"};
            P.x_iters = (int)P.x_res.size() - 1;
        }
        if (csolve == 2) {
            const std::vector<double> ch = rec_get<double>(R, "cheb", 4);
            P.ch_lo = ch[0], P.ch_hi = ch[1], P.ch_rlo = ch[2], P.ch_rhi = ch[3];
            if (!(P.ch_hi > P.ch_lo)) throw SetupError{DDLR_E_INVALID, "stored Chebyshev interval is empty"};
        }
        for (double d : P.D) h->pivots_positive = h->pivots_positive && d > 0.0;
        if (csolve == 1) h->pivots_positive = h->pivots_positive && P.x_spd;
        if (csolve == 2) h->pivots_positive = h->pivots_positive && P.ch_rlo > 0.0;
        h->variant = 0;
        h->spd = (int)h->pivots_positive;
        if (csolve == 2) h->cheb_nu = flags[2];
        h->device = ctx ? ctx->device : 0;
        if (h->device >= 0) {
            HIPCHK(hipSetDevice(h->device));
            {
                DevLock dl(h->device);
                device_init(h.get(), flags[2], 0);
                HIPCHK(hipDeviceSynchronize());
            }
            if (R.count("lowrank")) {
                const std::vector<int32_t> vk = rec_get<int32_t>(R, "lowrank", 2);
                const int variant = vk[0], k = vk[1];
                if ((variant != 1 && variant != 2) || k < 1 || k > 128)
                    throw SetupError{DDLR_E_INVALID, "setup file has a bad low-rank variant or rank"};
                const std::vector<double> U = rec_get<double>(R, "U", n * (int64_t)k);
                const std::vector<double> aux =
                    rec_get<double>(R, "aux", variant == 1 ? (int64_t)k + 1 : (int64_t)k * k);
                const ddlr_status st = ddlr_set_lowrank(h.get(), variant, k, U.data(), aux.data());
                if (st != DDLR_OK) throw SetupError{st, g_err};
            }
        }
    } catch (const SetupError& e) {
        discard_handle(h.get());
        return fail_status(e);
    } catch (const std::bad_alloc&) {
        discard_handle(h.get());
        g_err = "host out of memory";
        return DDLR_E_OOM;
    }
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
    return DDLR_OK;
}

static void prof_reset(ddlr_prec* h) {
    for (int c = 0; c < kProfClasses; ++c) {
        for (auto& pr : h->prof_ev[c]) {
            h->prof_pool.push_back(pr.first);
            h->prof_pool.push_back(pr.second);
        }
        h->prof_ev[c].clear();
    }
}

ddlr_status ddlr_profile(ddlr_prec* h, int32_t on) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    try {
        HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        HIPCHK(hipDeviceSynchronize());
        prof_reset(h);
        h->prof = on != 0;
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

ddlr_status ddlr_profile_read(ddlr_prec* h, int32_t which, double min_us, double* total_ms, int64_t* launches) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    if (which < 0 || which >= kProfClasses || !total_ms || !launches) {
        g_err = "bad profile query";
        return DDLR_E_INVALID;
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipDeviceSynchronize());
        double t = 0.0;
        int64_t cnt = 0;
        for (auto& pr : h->prof_ev[which]) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
            if (1e3 * ms < min_us) continue;
            t += ms;
            ++cnt;
        }
        *total_ms = t;
        *launches = cnt;
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

ddlr_status ddlr_extend_lowrank(ddlr_prec* h, int32_t k, int32_t more_steps, int32_t check, double tol) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    if (h->lrun.steps == 0 || h->lrun.lvariant == 0 || h->batch) {
        g_err = "no Lanczos run to continue (variant 0, imported low-rank data, or a batch)";
        return DDLR_E_INVALID;
    }
    if (k < 1 || k > 128 || more_steps < 0 || check < 0 || !(tol >= 0.0) ||
        (int64_t)h->lrun.steps + more_steps > kMaxLanczos) {
        g_err = "bad extend arguments (1 <= k <= 128, more_steps >= 0, total steps <= 1024, check >= 0, tol >= 0)";
        return DDLR_E_INVALID;
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        HIPCHK(hipDeviceSynchronize());
        h->variant = h->lrun.lvariant;
        const int m = (int)std::min<int64_t>((int64_t)h->lrun.steps + more_steps, h->plan.s);
        lanczos_advance(h, m, check, check > 0 ? (tol > 0.0 ? tol : 1e-4) : 0.0, k);
        lanczos_finish(h, k, h->theta_mode);
        HIPCHK(hipDeviceSynchronize());
    } catch (const SetupError& e) {
        // the previous low-rank part may be gone: fall back to the A0 part alone
        h->variant = 0;
        h->k = 0;
        h->f64.U = nullptr;
        h->f32.U = nullptr;
        h->f64.Ut = nullptr;
        h->f32.Ut = nullptr;
        h->ubr = h->ubt = nullptr;
        h->spd = (int)h->pivots_positive;
        return fail_status(e);
    }
    return DDLR_OK;
}

ddlr_status ddlr_tune(ddlr_prec* h, int32_t nrhs, int32_t retune, ddlr_tuning* out, void* stream) {
    if (!dev_ok(h)) return h ? DDLR_E_DEVICE : DDLR_E_INVALID;
    if (nrhs < 1 || nrhs > kMaxRhs || !out) {
        g_err = "nrhs must be in [1, 16] and out non-null";
        return DDLR_E_INVALID;
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        DevLock dl(h->device);
        hipStream_t st = (hipStream_t)stream;
        autotune(h, nrhs, st, retune != 0 || !h->tune.count(nrhs));
        HIPCHK(hipStreamSynchronize(st));
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    std::memset(out, 0, sizeof(*out));
    out->nrhs = nrhs;
    out->cg_graph = -1;
    out->cg_overlap = -1;
    if (auto mi = h->cg_mode.find(nrhs); mi != h->cg_mode.end()) {
        const ddlr_prec::CgMode& m = mi->second;
        out->cg_graph = m.graph;
        out->cg_overlap = m.ov >= 0 ? m.ov : -1;
        const int o = m.ov == -1 ? 0 : 2;  // "beside", or the only form when nothing overlaps
        auto val = [](double v) { return v < 1e29 ? (float)v : 0.0f; };
        out->cg_eager_us = val(m.us[0][o]);
        out->cg_graph_us = val(m.us[1][o]);
        out->cg_eager_in_line_us = val(m.us[0][1]);
        out->cg_graph_in_line_us = val(m.us[1][1]);
    }
    out->cg_persist = h->pers_mode == 0 || !persist_eligible(h) || h->ndev > kPersistMaxRows ? 0 : -1;
    if (auto pi = h->pers_us.find(nrhs); pi != h->pers_us.end()) {
        out->cg_persist_us = (float)pi->second;
        if (auto mi = h->cg_mode.find(nrhs); mi != h->cg_mode.end() && mi->second.graph >= 0)
            out->cg_persist = pi->second < mi->second.us[mi->second.graph][mi->second.ov + 1] / 8.0 ? 1 : 0;
    }
    if (h->pers_mode == 1 && out->cg_persist != 0) out->cg_persist = 1;
    if (h->pers) {
        out->persist_threads = h->pers->nt;
        for (int c = 0; c < 5; ++c) out->persist_nt_us[c] = h->pers->nt_us[c];
    }
    auto it = h->tune.find(nrhs);
    if (it == h->tune.end()) {  // batches: fixed shape
        out->ring_cols = 1;
        out->ring_threads = ring_nt_default(h);
        out->overlap = h->overlap ? 1 : 0;
        return DDLR_OK;
    }
    out->ring_cols = it->second.ring_r;
    out->ring_threads = it->second.ring_r > 1 ? 512 : (h->precision == DDLR_FP64 ? ring_nt_for<double>(h, nrhs)
                                                                                   : ring_nt_for<float>(h, nrhs));
    if (!(h->precision == DDLR_FP64 ? ring_ready<double>(h) : ring_ready<float>(h))) out->ring_threads = -1;
    out->a0_plain_us = it->second.a0_plain_us;
    out->overlap = it->second.overlap;
    for (int q = 0; q < 4; ++q) out->a0_us[q] = it->second.a0_us[q];
    for (int q = 0; q < 2; ++q) out->a0_thin_us[q] = it->second.a0_thin_us[q];
    out->a0_no_overlap_us = it->second.a0_noov_us;
    return DDLR_OK;
}

void ddlr_destroy(ddlr_prec* h) {
    if (!h) return;
    if (h->device >= 0) {
        (void)hipSetDevice(h->device);
        DevLock dl(h->device);
        (void)hipDeviceSynchronize();
        prof_reset(h);
        for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
        release_streams(h);
    }
    h->ws.mem.release();
    h->ws.gmem.release();
    if (h->ws.done_host) (void)hipHostFree(h->ws.done_host);
    h->lrmem.release();
    h->lrun.mem.release();
    h->chmem.release();
    h->mem.release();
    ctx_unref(h->ctx);
    delete h;
}

const char* ddlr_status_string(int32_t s) {
    switch (s) {
    case DDLR_OK: return "ok";
    case DDLR_E_INVALID: return "invalid argument";
    case DDLR_E_NOT_SYMMETRIC: return "matrix not symmetric";
    case DDLR_E_BREAKDOWN: return "local factorisation breakdown";
    case DDLR_E_NOT_SPD: return "preconditioner not SPD";
    case DDLR_E_NO_CONVERGENCE: return "no convergence";
    case DDLR_E_LANCZOS: return "Lanczos breakdown";
    case DDLR_E_OOM: return "out of device memory";
    case DDLR_E_BUDGET: return "HBM budget exceeded";
    case DDLR_E_DEVICE: return "device error";
    default: return "unknown status";
    }
}

const char* ddlr_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ================================================================ batches

struct ddlr_batch {
    ddlr_prec* h = nullptr;  // merged preconditioner, one CG lane per system
    int nsys = 0;
    std::vector<int64_t> roff, soff;
    std::vector<int32_t> spd;
    hipStream_t own = nullptr;  // internal stream (captured into the iteration graph)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_chunk = 0, graph_maxit = -1;
    double graph_tol2 = -1.0;
    // persistent form: one workgroup per system, the launch captured into a graph
    std::unique_ptr<PersistData> pers;
    hipGraph_t pgraph = nullptr;
    hipGraphExec_t pgexec = nullptr;
    int pg_maxit = -1, pg_nt = 0;
    double pg_tol2 = -1.0;
    // measured regrouping (groups chosen by the library): what a rebuild of the
    // persistent tables needs, kept until the first persistent solve has run
    int regroup = 0;  // regrouping passes left
    std::vector<HostPlan> plans;
    std::vector<int> ks;
    std::vector<double> c0v;
    size_t tsz = 0, cap = 0;
    int nxcd = 1, slots = 0;
};

namespace {

constexpr int kBatchChunk = 8;  // CG iterations per graph launch

void batch_release(ddlr_batch* B) {
    if (B->pgexec) (void)hipGraphExecDestroy(B->pgexec);
    if (B->pgraph) (void)hipGraphDestroy(B->pgraph);
    if (B->pers) B->pers->mem.release();
    B->pers.reset();
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->own) (void)hipStreamDestroy(B->own);
    if (B->ev_in) (void)hipEventDestroy(B->ev_in);
    if (B->ev_out) (void)hipEventDestroy(B->ev_out);
    if (B->h) ddlr_destroy(B->h);
    B->h = nullptr;
}

void seg_dot(ddlr_prec* h, const double* a, const double* b, hipStream_t st, const int* done) {
    Workspace& W = h->ws;
    hipLaunchKernelGGL(k_seg_dot, dim3(kSegChunks, h->nsys), dim3(256), 0, st, h->seg_roff, a, b, W.part, done);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_cols, dim3(h->nsys), dim3(256), 0, st, kSegChunks, h->nsys, W.part, W.sums, done);
    LAUNCHCHK();
}

void seg_scalar(ddlr_prec* h, int what, double tol2, int maxit, hipStream_t st) {
    Workspace& W = h->ws;
    hipLaunchKernelGGL(k_cg_scalar_many, dim3(1), dim3(256), 0, st, what, h->nsys, W.sums, W.lanes, tol2, maxit,
                       W.done);
    LAUNCHCHK();
}

// one CG iteration of every system (device-side early exit through W.done)
void batch_iteration(ddlr_prec* h, double tol2, int maxit, hipStream_t st) {
    Workspace& W = h->ws;
    const int64_t n = h->ndev;
    spmv_dev(h, 1, W.p, n, W.q, n, nullptr, st, W.done);
    seg_dot(h, W.p, W.q, st, W.done);
    seg_scalar(h, 2, tol2, maxit, st);
    hipLaunchKernelGGL(k_seg_cg_xr, dim3(kSegChunks, h->nsys), dim3(256), 0, st, h->seg_roff, W.lanes, W.p, W.q, W.x,
                       W.r, W.part, W.done);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_cols, dim3(h->nsys), dim3(256), 0, st, kSegChunks, h->nsys, W.part, W.sums, W.done);
    LAUNCHCHK();
    seg_scalar(h, 3, tol2, maxit, st);
    apply_dev(h, 1, W.r, n, W.z, n, st, W.done);
    seg_dot(h, W.r, W.z, st, W.done);
    seg_scalar(h, 4, tol2, maxit, st);
    hipLaunchKernelGGL(k_seg_cg_p, dim3(kSegChunks, h->nsys), dim3(256), 0, st, h->seg_roff, W.lanes, 0, W.z, W.p,
                       W.done);
    LAUNCHCHK();
}

}  // namespace

extern "C" {

ddlr_status ddlr_batch_create(int32_t nsys, ddlr_prec* const* members, ddlr_batch** out) {
    if (out) *out = nullptr;
    if (!out || !members || nsys < 1 || nsys > 1024) {
        g_err = "bad batch arguments (1 <= nsys <= 1024)";
        return DDLR_E_INVALID;
    }
    const ddlr_prec* m0 = members[0];
    for (int q = 0; q < nsys; ++q) {
        const ddlr_prec* m = members[q];
        if (!m || m->device < 0 || m->nsys != 1 || m->device != m0->device || m->precision != m0->precision ||
            m->variant != m0->variant || m->variant == DDLR_2 || m->precision == DDLR_FP32_UK_BF16 ||
            m->plan.csolve) {
            g_err = "batch members must be single-system device handles with the same device, precision and "
                    "variant (DDLR-1 or A0 only; FP64 or FP32; C_alpha factored)";
            return DDLR_E_INVALID;
        }
    }
    std::unique_ptr<ddlr_batch> B(new ddlr_batch());
    B->nsys = nsys;
    try {
        HIPCHK(hipSetDevice(m0->device));
        ddlr_prec* h = new ddlr_prec();
        B->h = h;
        h->device = m0->device;
        h->precision = m0->precision;
        h->variant = m0->variant;
        h->nsys = nsys;
        h->batch = true;
        h->overlap = false;
        h->tune_mode = 0;
        // device structures of every member, interface blocks as single blocks
        std::vector<DevHost> parts(nsys);
        std::vector<const DevHost*> pp(nsys);
        B->roff.assign(nsys + 1, 0);
        B->soff.assign(nsys + 1, 0);
        for (int q = 0; q < nsys; ++q) {
            parts[q] = build_devhost(members[q]->plan, 0);
            pp[q] = &parts[q];
            B->roff[q + 1] = B->roff[q] + parts[q].n;
            B->soff[q + 1] = B->soff[q] + parts[q].s;
            B->spd.push_back(members[q]->spd);
        }
        DevHost D;
        merge_devhost(pp, D);
        parts.clear();
        upload_devhost(h, D);
        h->seg_roff = h->mem.upload(B->roff);
        h->seg_soff = h->mem.upload(B->soff);
        int kmax = 0;
        for (int q = 0; q < nsys; ++q) kmax = std::max(kmax, members[q]->k);
        h->k = h->variant == DDLR_1 ? kmax : 0;
        h->spd = 1;
        for (int q = 0; q < nsys; ++q) h->spd = h->spd && members[q]->spd;
        if (h->variant == DDLR_1) {
            // U of every system (interface rows in device order), padded to kmax columns
            const int64_t s = B->soff[nsys];
            std::vector<double> U((size_t)s * kmax, 0.0), dv((size_t)nsys * kmax, 0.0), c0(nsys);
            for (int q = 0; q < nsys; ++q) {
                const ddlr_prec* m = members[q];
                std::vector<double> Uq((size_t)m->urows * m->k);
                HIPCHK(hipMemcpy(Uq.data(), m->f64.U, Uq.size() * sizeof(double), hipMemcpyDeviceToHost));
                for (int64_t i = 0; i < m->urows; ++i)
                    for (int j = 0; j < m->k; ++j) U[(size_t)(B->soff[q] + i) * kmax + j] = Uq[(size_t)i * m->k + j];
                for (int j = 0; j < m->k; ++j) dv[(size_t)q * kmax + j] = m->dvec_h[j];
                c0[q] = m->c0;
            }
            h->urows = s;
            h->f64.U = h->lrmem.upload(U);
            if (h->precision != DDLR_FP64) {
                std::vector<float> f(U.begin(), U.end());
                h->f32.U = h->lrmem.upload(f);
            }
            h->dvecs = h->lrmem.upload(dv);
            h->c0s = h->lrmem.upload(c0);
        }
        // persistent form (rank at most kPersistMaxK), unless DDLR_BATCH_PERSIST=0
        const char* pe = std::getenv("DDLR_BATCH_PERSIST");
        if (h->k <= kPersistMaxK && !(pe && pe[0] == '0')) {
            std::vector<const HostPlan*> plans(nsys);
            std::vector<int> ks(nsys);
            std::vector<double> c0v(nsys);
            for (int q = 0; q < nsys; ++q) {
                plans[q] = &members[q]->plan;
                ks[q] = h->variant == DDLR_1 ? members[q]->k : 0;
                c0v[q] = members[q]->c0;
            }
            // large systems get several workgroups (groups) when the lanes fit
            // the device at two 512-thread workgroups per CU: the dynamic LDS is
            // then capped at 76 KB; DDLR_BATCH_GROUP=0 keeps one workgroup per
            // system, =N asks for N per system
            const size_t tsz = h->precision == DDLR_FP64 ? sizeof(double) : sizeof(float);
            const size_t cap2 = (size_t)env_int("DDLR_GROUP_LDS_KB", 76) * 1024;
            const int per_cu = env_int("DDLR_GROUP_PER_CU", 2);
            int cus = 0, nxcd = 1;
            HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
            hipDeviceProp_t prop;
            HIPCHK(hipGetDeviceProperties(&prop, h->device));
            if (std::strstr(prop.gcnArchName, "gfx950") || std::strstr(prop.gcnArchName, "gfx942")) nxcd = 8;
            std::vector<int> groups;
            const char* ge = std::getenv("DDLR_BATCH_GROUP");
            if (ge && std::atoi(ge) > 0) groups.assign(nsys, std::atoi(ge));
            else if (!(ge && ge[0] == '0')) groups = choose_groups(plans, tsz, cap2, per_cu * cus);
            bool grouped = false;
            for (int g : groups) grouped = grouped || g > 1;
            B->pers.reset(new PersistData());
            if (grouped) {
                persist_build(*B->pers, plans, B->roff, B->soff, ks, c0v, std::max(1, h->k), tsz, h->device, groups,
                              cap2);
                persist_batch_lanes(*B->pers, h->ndev, nxcd);
                PersistData& PD = *B->pers;
                if (PD.grid > std::max(persist_resident(h, PD, 256), persist_resident(h, PD, 512))) {
                    PD.mem.release();  // does not fit: one workgroup per system
                    B->pers.reset(new PersistData());
                    grouped = false;
                }
            }
            if (!grouped) {
                persist_build(*B->pers, plans, B->roff, B->soff, ks, c0v, std::max(1, h->k), tsz, h->device);
                persist_batch_lanes(*B->pers, h->ndev, nxcd);
            }
            if (const char* gs = std::getenv("DDLR_GROUP_SLOW")) B->pers->gslow = gs[0] == '1';
            // a smaller limit on the group waits (the failure path can be forced)
            if (const char* sp = std::getenv("DDLR_GROUP_SPIN")) B->pers->gspin = (unsigned)std::strtoul(sp, nullptr, 10);
            // groups the library chose are chosen again from the first solve's
            // measured times (DDLR_BATCH_REGROUP=0: not)
            const char* rg = std::getenv("DDLR_BATCH_REGROUP");
            if (grouped && !ge && !(rg && rg[0] == '0')) {
                B->regroup = env_int("DDLR_BATCH_REGROUP", 2);
                B->plans.reserve(nsys);
                for (int q = 0; q < nsys; ++q) B->plans.push_back(members[q]->plan);
                B->ks = ks;
                B->c0v = c0v;
                B->tsz = tsz;
                B->cap = cap2;
                B->nxcd = nxcd;
                B->slots = per_cu * cus;
            }
        }
        HIPCHK(hipStreamCreateWithFlags(&B->own, hipStreamNonBlocking));  // default priority
        HIPCHK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
        ensure_ws(h, 1);
        HIPCHK(hipDeviceSynchronize());
    } catch (const SetupError& e) {
        batch_release(B.get());
        return fail_status(e);
    } catch (const std::bad_alloc&) {
        batch_release(B.get());
        g_err = "host out of memory";
        return DDLR_E_OOM;
    }
    *out = B.release();
    return DDLR_OK;
}

ddlr_status ddlr_batch_offsets(const ddlr_batch* B, int64_t* offsets) {
    if (!B || !offsets) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::copy(B->roff.begin(), B->roff.end(), offsets);
    return DDLR_OK;
}

ddlr_status ddlr_batch_tuning(const ddlr_batch* B, int32_t* persistent, int32_t* threads, float* us_per_iter) {
    if (!B || !persistent || !threads || !us_per_iter) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    *persistent = B->pers ? 1 : 0;
    *threads = B->pers ? B->pers->nt : 0;
    for (int c = 0; c < 5; ++c) us_per_iter[c] = B->pers ? B->pers->nt_us[c] : 0.f;
    return DDLR_OK;
}

ddlr_status ddlr_batch_times(const ddlr_batch* B, double* us) {
    if (!B || !us) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    for (int q = 0; q < B->nsys; ++q)
        us[q] = B->pers && (int)B->pers->sys_us.size() == B->nsys ? B->pers->sys_us[q] : 0.0;
    return DDLR_OK;
}

ddlr_status ddlr_batch_members(const ddlr_batch* B, int32_t* members) {
    if (!B || !members) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    for (int q = 0; q < B->nsys; ++q) members[q] = B->pers ? B->pers->members[q] : 0;
    return DDLR_OK;
}

ddlr_status ddlr_batch_apply(ddlr_batch* B, const double* x, double* y, void* stream) {
    if (!B || !x || !y) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    ddlr_prec* h = B->h;
    return run_chunked(h, 1, x, h->ndev, y, h->ndev, stream, [&](int nr, double* in, double* out, hipStream_t s) {
        apply_dev(h, nr, in, h->ndev, out, h->ndev, s, nullptr);
    });
}

// After the first persistent solve of a batch whose groups the library chose:
// the measured per-system times calibrate the estimate (per system, its time
// over the estimate at the groups it ran with), the groups are chosen again,
// and when that lowers the slowest calibrated time by a tenth the tables are
// rebuilt (the next solve tunes and captures anew).  Up to two passes (after
// the first solves with at least 20 iterations; a pass that changes nothing
// ends them); the kept plans are released afterwards.
static void batch_regroup(ddlr_batch* B) {
    --B->regroup;
    bool rebuilt = false;
    PersistData& PD = *B->pers;
    ddlr_prec* h = B->h;
    const int ns = B->nsys;
    std::vector<const HostPlan*> plans(ns);
    for (int q = 0; q < ns; ++q) plans[q] = &B->plans[q];
    std::vector<double> scale(ns, 1.0);
    double tmax = 0.0;
    bool timed = (int)PD.sys_us.size() == ns;
    for (int q = 0; q < ns && timed; ++q) {
        const double e = group_est(*plans[q], PD.members[q], B->tsz, B->cap);
        timed = PD.sys_us[q] > 0.0 && e > 0.0;
        if (timed) scale[q] = PD.sys_us[q] / e;
        tmax = std::max(tmax, PD.sys_us[q]);
    }
    if (timed) {
        const std::vector<int> G = choose_groups(plans, B->tsz, B->cap, B->slots, &scale);
        double pmax = 0.0;
        for (int q = 0; q < ns; ++q) pmax = std::max(pmax, group_est(*plans[q], G[q], B->tsz, B->cap) * scale[q]);
        if (G != PD.members && pmax < 0.9 * tmax) {
            std::unique_ptr<PersistData> N(new PersistData());
            bool fits = false;
            try {  // a regrouping that cannot be built leaves the batch as it was
                persist_build(*N, plans, B->roff, B->soff, B->ks, B->c0v, std::max(1, h->k), B->tsz, h->device, G,
                              B->cap);
                persist_batch_lanes(*N, h->ndev, B->nxcd);
                fits = N->grid <= std::max(persist_resident(h, *N, 256), persist_resident(h, *N, 512));
            } catch (const SetupError&) {
                (void)hipGetLastError();
            }
            if (fits) {
                N->gslow = PD.gslow;
                N->gspin = PD.gspin;
                N->sys_us = PD.sys_us;  // the times measured, until the next solve
                if (B->pgexec) (void)hipGraphExecDestroy(B->pgexec);
                if (B->pgraph) (void)hipGraphDestroy(B->pgraph);
                B->pgexec = nullptr;
                B->pgraph = nullptr;
                PD.mem.release();  // device memory is freed explicitly (DMem has no destructor)
                B->pers = std::move(N);
                rebuilt = true;
            } else {
                N->mem.release();
            }
        }
    }
    if (!rebuilt) B->regroup = 0;
    if (B->regroup <= 0) std::vector<HostPlan>().swap(B->plans);
}

ddlr_status ddlr_batch_solve(ddlr_batch* B, const double* b, double* x, const ddlr_solve_options* opt_in,
                             ddlr_solve_info* info, void* stream) {
    if (!B || !b || !x || !info) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    ddlr_solve_options o;
    if (opt_in) o = *opt_in;
    else ddlr_solve_options_default(&o);
    if (o.method != 0 || o.maxit < 1 || !(o.rtol > 0.0)) {
        g_err = "batch solves use CG (method 0) with maxit >= 1 and rtol > 0";
        return DDLR_E_INVALID;
    }
    ddlr_prec* h = B->h;
    if (!h->spd) {
        g_err = "a member preconditioner is not certified SPD";
        return DDLR_E_NOT_SPD;
    }
    const double tol2 = o.rtol * o.rtol;
    ddlr_status result = DDLR_OK;
    if (B->pers) {
        try {
            HIPCHK(hipSetDevice(h->device));
            hipStream_t ust = (hipStream_t)stream, st = B->own;
            HIPCHK(hipEventRecord(B->ev_in, ust));
            HIPCHK(hipStreamWaitEvent(st, B->ev_in, 0));
            PersistData& PD = *B->pers;
            const int64_t n = h->ndev;
            const int ns = B->nsys;
            hipLaunchKernelGGL((k_gather<double, double>), dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->perm_dev, b,
                               n, PD.b, n);
            LAUNCHCHK();
            if (PD.nt == 0) persist_tune(h, PD, PD.grid, tol2, o.maxit, st);
            if (!B->pgexec || B->pg_tol2 != tol2 || B->pg_maxit != o.maxit || B->pg_nt != PD.nt) {
                if (B->pgexec) (void)hipGraphExecDestroy(B->pgexec);
                if (B->pgraph) (void)hipGraphDestroy(B->pgraph);
                B->pgexec = nullptr;
                B->pgraph = nullptr;
                persist_lds_attr(h, PD, PD.nt);
                h->capturing = true;
                HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                persist_launch(h, PD, PD.grid, tol2, o.maxit, st, PD.nt);
                hipGraph_t g = nullptr;
                const hipError_t ec = hipStreamEndCapture(st, &g);
                h->capturing = false;
                HIPCHK(ec);
                B->pgraph = g;
                HIPCHK(hipGraphInstantiate(&B->pgexec, B->pgraph, nullptr, nullptr, 0));
                B->pg_tol2 = tol2;
                B->pg_maxit = o.maxit;
                B->pg_nt = PD.nt;
            }
            HIPCHK(hipGraphLaunch(B->pgexec, st));
            hipLaunchKernelGGL((k_scatter<double, double>), dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->perm_dev,
                               h->ws.x, n, x, n);
            LAUNCHCHK();
            std::vector<PRes> rl(PD.grid);
            HIPCHK(hipMemcpyAsync(rl.data(), PD.res, PD.grid * sizeof(PRes), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipEventRecord(B->ev_out, st));
            HIPCHK(hipStreamWaitEvent(ust, B->ev_out, 0));
            bool gave_up = false;
            int khz = 0;  // the wall clock the lanes' ticks count
            if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess || khz <= 0) {
                (void)hipGetLastError();
                khz = 100000;
            }
            PD.sys_us.assign(ns, 0.0);
            for (int l = 0; l < PD.grid; ++l)
                if (PD.hlanes[l].sys >= 0) {
                    double& u = PD.sys_us[PD.entry_sys[PD.hlanes[l].sys]];
                    u = std::max(u, 1e3 * (double)rl[l].ticks / khz);
                }
            for (int q = 0; q < ns; ++q) {
                const PRes& r = rl[PD.sys_lane[q]];
                ddlr_solve_info& inf = info[q];
                inf.iters = r.its;
                inf.status = r.status == 0 ? DDLR_OK : DDLR_E_NO_CONVERGENCE;
                inf.relres = r.bb > 0 ? std::sqrt(r.rr / r.bb) : 0.0;
                inf.relres_true = r.bb > 0 ? std::sqrt(r.rtrue / r.bb) : 0.0;
                if (r.status) result = DDLR_E_NO_CONVERGENCE;
                if (r.status == 2) gave_up = true;
            }
            if (gave_up) {
                g_err = "a group barrier of the persistent batch gave up waiting";
                return DDLR_E_DEVICE;
            }
            int itmax = 0;
            for (int q = 0; q < ns; ++q) itmax = std::max(itmax, info[q].iters);
            if (B->regroup > 0 && itmax >= 20) {
                try {  // optional: any failure keeps the batch as it is
                    batch_regroup(B);
                } catch (...) {
                    (void)hipGetLastError();
                    B->regroup = 0;
                    std::vector<HostPlan>().swap(B->plans);
                }
            }
        } catch (const SetupError& e) {
            h->capturing = false;
            return fail_status(e);
        }
        if (result != DDLR_OK) g_err = "some systems did not converge";
        return result;
    }
    try {
        HIPCHK(hipSetDevice(h->device));
        hipStream_t ust = (hipStream_t)stream, st = B->own;
        HIPCHK(hipEventRecord(B->ev_in, ust));
        HIPCHK(hipStreamWaitEvent(st, B->ev_in, 0));
        Workspace& W = h->ws;
        const int64_t n = h->ndev;
        hipLaunchKernelGGL((k_gather<double, double>), dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->perm_dev, b, n,
                           W.r, n);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, n, 0.0, W.x);
        LAUNCHCHK();
        seg_dot(h, W.r, W.r, st, nullptr);
        seg_scalar(h, 0, tol2, o.maxit, st);
        apply_dev(h, 1, W.r, n, W.z, n, st, W.done);
        seg_dot(h, W.r, W.z, st, W.done);
        seg_scalar(h, 1, tol2, o.maxit, st);
        hipLaunchKernelGGL(k_seg_cg_p, dim3(kSegChunks, h->nsys), dim3(256), 0, st, h->seg_roff, W.lanes, 1, W.z, W.p,
                           W.done);
        LAUNCHCHK();
        // kBatchChunk iterations captured once into a graph, replayed until every system is done
        if (!B->gexec || B->graph_tol2 != tol2 || B->graph_maxit != o.maxit) {
            if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
            if (B->graph) (void)hipGraphDestroy(B->graph);
            B->gexec = nullptr;
            B->graph = nullptr;
            h->capturing = true;
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int c = 0; c < kBatchChunk; ++c) batch_iteration(h, tol2, o.maxit, st);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &g);
            h->capturing = false;
            HIPCHK(ec);
            B->graph = g;
            HIPCHK(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
            B->graph_tol2 = tol2;
            B->graph_maxit = o.maxit;
        }
        for (int it = 0; it < o.maxit; it += kBatchChunk) {
            HIPCHK(hipGraphLaunch(B->gexec, st));
            HIPCHK(hipMemcpyAsync(W.done_host, W.done, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (*W.done_host) break;
        }
        hipLaunchKernelGGL((k_scatter<double, double>), dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->perm_dev, W.x, n,
                           x, n);
        LAUNCHCHK();
        // true residual per system
        hipLaunchKernelGGL((k_gather<double, double>), dim3(grid_for(n)), dim3(256), 0, st, n, 1, h->perm_dev, b, n,
                           W.r, n);
        LAUNCHCHK();
        spmv_dev(h, 1, W.x, n, W.q, n, nullptr, st, nullptr);
        hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(256), 0, st, n, W.r, W.q, W.z);
        LAUNCHCHK();
        seg_dot(h, W.z, W.z, st, nullptr);
        const int ns = h->nsys;
        std::vector<CgLane> lanes(ns);
        std::vector<double> rr(ns);
        HIPCHK(hipMemcpyAsync(lanes.data(), W.lanes, ns * sizeof(CgLane), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(rr.data(), W.sums, ns * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipEventRecord(B->ev_out, st));
        HIPCHK(hipStreamWaitEvent(ust, B->ev_out, 0));
        for (int q = 0; q < ns; ++q) {
            ddlr_solve_info& inf = info[q];
            const double bb = lanes[q].bb;
            inf.iters = lanes[q].its;
            const bool conv = bb == 0.0 || lanes[q].rr <= tol2 * bb;
            inf.status = conv ? DDLR_OK : DDLR_E_NO_CONVERGENCE;
            inf.relres = bb > 0 ? std::sqrt(lanes[q].rr / bb) : 0.0;
            inf.relres_true = bb > 0 ? std::sqrt(rr[q] / bb) : 0.0;
            if (!conv) result = DDLR_E_NO_CONVERGENCE;
        }
    } catch (const SetupError& e) {
        h->capturing = false;
        return fail_status(e);
    }
    if (result != DDLR_OK) g_err = "some systems did not converge";
    return result;
}

void ddlr_batch_destroy(ddlr_batch* B) {
    if (!B) return;
    if (B->h && B->h->device >= 0) {
        (void)hipSetDevice(B->h->device);
        (void)hipDeviceSynchronize();
    }
    batch_release(B);
    delete B;
}

}  // extern "C"

// ================================================================ serving

struct SrvRequest {
    uint64_t ticket = 0;
    int mid = 0, nrhs = 0;
    const double* b = nullptr;
    double* x = nullptr;
    double tol2 = 0.0;
    int maxit = 0;
    int next_col = 0, done_cols = 0;
    std::vector<ddlr_solve_info> info;
    double t_submit = 0.0, t_done = 0.0;
    bool done = false;
};

struct SrvMatrix {
    ddlr_prec* h = nullptr;
    hipStream_t st = nullptr;
    double* stage = nullptr;  // user-order staging, n x slots
    double* bdev = nullptr;   // each slot's right-hand side in device order (n x slots), for the true residual
    double* tq = nullptr;     // n: b - A x of a retiring slot
    double* rpart = nullptr;  // kRedBlocks partials of its squared norm
    double* rtrue = nullptr;  // slots: ||b - A x||^2 per retired slot
    std::vector<double> rtrue_h;
    DMem mem;
    size_t bytes = 0;
    std::vector<SrvRequest*> slot_req;
    std::vector<int> slot_col;
    std::vector<CgLane> lanes_h;
};

struct ddlr_server {
    int device = 0, slots = 16, tick = 4;
    size_t budget = 0, used = 0;
    std::vector<std::unique_ptr<SrvMatrix>> mats;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::thread worker;
    bool stop = false;
    std::deque<SrvRequest*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<SrvRequest>> reqs;
    uint64_t next_ticket = 1;
    std::vector<double> lat_ms;
    int64_t solves_done = 0, submitted = 0, requests_done = 0;
    double t_first = -1.0, t_last = 0.0;
    int worker_status = DDLR_OK;
    std::string worker_err;
};

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One pass of the engine: admit queued columns into free slots, run `tick`
// iterations on every matrix that has lanes, retire finished lanes.  A matrix
// iterates only the slots up to its highest occupied one (p keeps the stride
// of all slots, so running lanes are not moved); its launch shapes for that
// width are tuned on first use.  The device lock is held per matrix while its
// work is enqueued, not across the whole pass, so other calls on the device
// interleave.  A retiring lane's true residual ||b - A x|| is computed before
// its x leaves the device.
bool server_step(ddlr_server* S) {
    struct Adm {
        int slot;
        SrvRequest* r;
        int col;
    };
    std::vector<std::vector<Adm>> adm(S->mats.size());
    std::vector<int> width(S->mats.size(), 0);
    bool any = false;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = S->queue.begin(); it != S->queue.end();) {
            SrvRequest* r = *it;
            SrvMatrix& M = *S->mats[r->mid];
            for (int sl = 0; sl < S->slots && r->next_col < r->nrhs; ++sl)
                if (!M.slot_req[sl]) {
                    M.slot_req[sl] = r;
                    M.slot_col[sl] = r->next_col;
                    adm[r->mid].push_back({sl, r, r->next_col});
                    r->next_col++;
                }
            if (r->next_col == r->nrhs) it = S->queue.erase(it);
            else ++it;
        }
        for (size_t mi = 0; mi < S->mats.size(); ++mi)
            for (int sl = 0; sl < S->slots; ++sl)
                if (S->mats[mi]->slot_req[sl]) width[mi] = sl + 1;
        for (int wdt : width) any = any || wdt > 0;
    }
    if (!any) return false;
    const int ns = S->slots, stride = lane_stride(ns);
    for (size_t mi = 0; mi < S->mats.size(); ++mi) {
        SrvMatrix& M = *S->mats[mi];
        ddlr_prec* h = M.h;
        const int64_t n = h->ndev;
        if (adm[mi].empty() && width[mi] == 0) continue;
        DevLock dl(S->device);
        if (!adm[mi].empty()) {
            std::vector<int32_t> start(ns, 0), maxit(ns, 0);
            std::vector<double> tol2(ns, 0.0);
            for (const Adm& a : adm[mi]) {
                HIPCHK(hipMemcpyAsync(M.stage + (size_t)a.slot * n, a.r->b + (size_t)a.col * n, n * sizeof(double),
                                      hipMemcpyHostToDevice, M.st));
                hipLaunchKernelGGL((k_gather<double, double>), dim3(grid_for(n)), dim3(256), 0, M.st, n, 1, h->perm_dev,
                                   M.stage + (size_t)a.slot * n, n, h->ws.r + (size_t)a.slot * n, n);
                LAUNCHCHK();
                hipLaunchKernelGGL((k_gather<double, double>), dim3(grid_for(n)), dim3(256), 0, M.st, n, 1, h->perm_dev,
                                   M.stage + (size_t)a.slot * n, n, M.bdev + (size_t)a.slot * n, n);
                LAUNCHCHK();
                start[a.slot] = 1;
                tol2[a.slot] = a.r->tol2;
                maxit[a.slot] = a.r->maxit;
            }
            lane_admit(h, ns, start, tol2, maxit, M.st);
        }
        if (width[mi] == 0) continue;
        autotune(h, width[mi], M.st, false);
        for (int c = 0; c < S->tick; ++c) lane_iteration(h, width[mi], M.st, stride);
        HIPCHK(hipMemcpyAsync(M.lanes_h.data(), h->ws.lanes, ns * sizeof(CgLane), hipMemcpyDeviceToHost, M.st));
    }
    for (auto& Mp : S->mats) HIPCHK(hipStreamSynchronize(Mp->st));
    // retire finished lanes
    for (size_t mi = 0; mi < S->mats.size(); ++mi) {
        SrvMatrix& M = *S->mats[mi];
        ddlr_prec* h = M.h;
        const int64_t n = h->ndev;
        std::vector<int> fin;
        for (int sl = 0; sl < width[mi]; ++sl)
            if (M.slot_req[sl] && M.lanes_h[sl].phase == 3) fin.push_back(sl);
        if (fin.empty()) continue;
        {
            DevLock dl(S->device);
            for (int sl : fin) {
                const double* xs = h->ws.x + (size_t)sl * n;
                spmv_dev(h, 1, xs, n, M.tq, n, nullptr, M.st, nullptr);
                hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(256), 0, M.st, n, M.bdev + (size_t)sl * n, M.tq,
                                   M.tq);
                LAUNCHCHK();
                hipLaunchKernelGGL((k_dot<double, double>), dim3(kRedBlocks), dim3(256), 0, M.st, n, 1, M.tq, n, M.tq,
                                   n, M.rpart, nullptr);
                LAUNCHCHK();
                hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, M.st, kRedBlocks, 1, M.rpart, M.rtrue + sl,
                                   nullptr);
                LAUNCHCHK();
                hipLaunchKernelGGL((k_scatter<double, double>), dim3(grid_for(n)), dim3(256), 0, M.st, n, 1,
                                   h->perm_dev, xs, n, M.stage + (size_t)sl * n, n);
                LAUNCHCHK();
                SrvRequest* r = M.slot_req[sl];
                HIPCHK(hipMemcpyAsync(r->x + (size_t)M.slot_col[sl] * n, M.stage + (size_t)sl * n, n * sizeof(double),
                                      hipMemcpyDeviceToHost, M.st));
            }
            HIPCHK(hipMemcpyAsync(M.rtrue_h.data(), M.rtrue, ns * sizeof(double), hipMemcpyDeviceToHost, M.st));
        }
        HIPCHK(hipStreamSynchronize(M.st));
        const double t = now_s();
        std::lock_guard<std::mutex> lk(S->mu);
        for (int sl : fin) {
            SrvRequest* r = M.slot_req[sl];
            const CgLane& l = M.lanes_h[sl];
            ddlr_solve_info& inf = r->info[M.slot_col[sl]];
            const bool conv = l.bb == 0.0 || l.rr <= l.tol2 * l.bb;
            inf.iters = l.its;
            inf.status = conv ? DDLR_OK : DDLR_E_NO_CONVERGENCE;
            inf.relres = l.bb > 0 ? std::sqrt(l.rr / l.bb) : 0.0;
            inf.relres_true = l.bb > 0 ? std::sqrt(M.rtrue_h[sl] / l.bb) : 0.0;
            r->done_cols++;
            S->solves_done++;
            M.slot_req[sl] = nullptr;
            if (r->done_cols == r->nrhs) {
                r->done = true;
                r->t_done = t;
                S->lat_ms.push_back(1e3 * (t - r->t_submit));
                S->requests_done++;
                S->t_last = t;
            }
        }
        S->cv_done.notify_all();
    }
    return true;
}

void server_loop(ddlr_server* S) {
    try {
        HIPCHK(hipSetDevice(S->device));
        while (true) {
            {
                std::unique_lock<std::mutex> lk(S->mu);
                if (S->stop) break;
            }
            if (!server_step(S)) {
                std::unique_lock<std::mutex> lk(S->mu);
                if (S->stop) break;
                S->cv.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    } catch (const SetupError& e) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->worker_status = e.status;
        S->worker_err = e.msg;
        S->cv_done.notify_all();
    }
}

size_t prec_bytes(const ddlr_prec* h) {
    return h->mem.bytes + h->lrmem.bytes + h->ws.mem.bytes + h->ws.gmem.bytes + h->lrun.mem.bytes + h->chmem.bytes;
}

}  // namespace

extern "C" {

ddlr_status ddlr_server_create(int32_t device, size_t hbm_budget_bytes, int32_t slots_per_matrix, ddlr_server** out) {
    if (out) *out = nullptr;
    if (!out || device < 0 || slots_per_matrix < 1 || slots_per_matrix > kMaxRhs) {
        g_err = "bad server arguments (1 <= slots_per_matrix <= 16)";
        return DDLR_E_INVALID;
    }
    std::unique_ptr<ddlr_server> S(new ddlr_server());
    S->device = device;
    S->budget = hbm_budget_bytes;
    S->slots = slots_per_matrix;
    try {
        HIPCHK(hipSetDevice(device));
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    ddlr_server* raw = S.get();
    S->worker = std::thread(server_loop, raw);
    *out = S.release();
    return DDLR_OK;
}

ddlr_status ddlr_server_add(ddlr_server* S, ddlr_prec* h, int32_t* matrix_id) {
    if (!S || !h || !matrix_id || h->device != S->device || h->nsys != 1) {
        g_err = "bad server_add arguments (single-system handle on the server's device)";
        return DDLR_E_INVALID;
    }
    std::unique_ptr<SrvMatrix> M(new SrvMatrix());
    M->h = h;
    try {
        HIPCHK(hipSetDevice(S->device));
        DevLock dl(S->device);
        std::lock_guard<std::mutex> lk(S->mu);
        const size_t before = prec_bytes(h);
        // staging, device-order right-hand sides, the residual vector and its partials and sums
        const size_t stage = ((size_t)h->ndev * (2 * S->slots + 1) + kRedBlocks + S->slots) * sizeof(double);
        // workspace for the slots, then the budget check on everything resident
        ensure_ws(h, S->slots);
        ensure_cg_streams(h);
        const size_t need = prec_bytes(h) + stage;
        if (S->budget > 0 && S->used + need > S->budget) {
            (void)before;
            g_err = "HBM budget exceeded: " + std::to_string((S->used + need) >> 20) + " MiB > " +
                    std::to_string(S->budget >> 20) + " MiB";
            return DDLR_E_BUDGET;
        }
        M->stage = M->mem.alloc<double>((size_t)h->ndev * S->slots);
        M->bdev = M->mem.alloc<double>((size_t)h->ndev * S->slots);
        M->tq = M->mem.alloc<double>((size_t)h->ndev);
        M->rpart = M->mem.alloc<double>(kRedBlocks);
        M->rtrue = M->mem.alloc<double>(S->slots);
        M->rtrue_h.assign(S->slots, 0.0);
        HIPCHK(hipStreamCreateWithFlags(&M->st, hipStreamNonBlocking));  // default priority
        M->bytes = need;
        M->slot_req.assign(S->slots, nullptr);
        M->slot_col.assign(S->slots, 0);
        M->lanes_h.resize(S->slots);
        // no lane is active until admitted
        std::vector<int32_t> none(S->slots, 0), mx(S->slots, 0);
        std::vector<double> tz(S->slots, 0.0);
        HIPCHK(hipMemset(h->ws.lanes, 0, S->slots * sizeof(CgLane)));
        HIPCHK(hipDeviceSynchronize());
        S->used += need;
        *matrix_id = (int32_t)S->mats.size();
        S->mats.push_back(std::move(M));
    } catch (const SetupError& e) {
        return fail_status(e);
    }
    return DDLR_OK;
}

ddlr_status ddlr_server_submit(ddlr_server* S, int32_t matrix_id, int32_t nrhs, const double* b_host, double* x_host,
                               const ddlr_solve_options* opt_in, uint64_t* ticket) {
    if (!S || !b_host || !x_host || !ticket || nrhs < 1) {
        g_err = "bad submit arguments";
        return DDLR_E_INVALID;
    }
    ddlr_solve_options o;
    if (opt_in) o = *opt_in;
    else ddlr_solve_options_default(&o);
    if (o.method != 0 || o.maxit < 1 || !(o.rtol > 0.0)) {
        g_err = "the server runs CG (method 0) with maxit >= 1 and rtol > 0";
        return DDLR_E_INVALID;
    }
    std::unique_ptr<SrvRequest> r(new SrvRequest());
    r->nrhs = nrhs;
    r->b = b_host;
    r->x = x_host;
    r->tol2 = o.rtol * o.rtol;
    r->maxit = o.maxit;
    r->info.assign(nrhs, ddlr_solve_info{0, 0, 0.0, 0.0});
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->worker_status != DDLR_OK) {
            g_err = S->worker_err;
            return (ddlr_status)S->worker_status;
        }
        if (matrix_id < 0 || matrix_id >= (int32_t)S->mats.size()) {
            g_err = "unknown matrix id";
            return DDLR_E_INVALID;
        }
        if (!S->mats[matrix_id]->h->spd) {
            g_err = "preconditioner is not certified SPD";
            return DDLR_E_NOT_SPD;
        }
        r->mid = matrix_id;
        r->ticket = S->next_ticket++;
        r->t_submit = now_s();
        if (S->t_first < 0) S->t_first = r->t_submit;
        S->submitted++;
        *ticket = r->ticket;
        S->queue.push_back(r.get());
        S->reqs[r->ticket] = std::move(r);
    }
    S->cv.notify_all();
    return DDLR_OK;
}

ddlr_status ddlr_server_poll(ddlr_server* S, uint64_t ticket, int32_t* done, ddlr_solve_info* info) {
    if (!S || !done) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->worker_status != DDLR_OK) {
        g_err = S->worker_err;
        return (ddlr_status)S->worker_status;
    }
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        g_err = "unknown ticket";
        return DDLR_E_INVALID;
    }
    *done = it->second->done ? 1 : 0;
    if (it->second->done && info) std::copy(it->second->info.begin(), it->second->info.end(), info);
    return DDLR_OK;
}

ddlr_status ddlr_server_wait(ddlr_server* S, uint64_t ticket, ddlr_solve_info* info) {
    if (!S) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        g_err = "unknown ticket";
        return DDLR_E_INVALID;
    }
    SrvRequest* r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->done || S->worker_status != DDLR_OK; });
    if (S->worker_status != DDLR_OK) {
        g_err = S->worker_err;
        return (ddlr_status)S->worker_status;
    }
    if (info) std::copy(r->info.begin(), r->info.end(), info);
    for (const ddlr_solve_info& i : r->info)
        if (i.status != DDLR_OK) return DDLR_E_NO_CONVERGENCE;
    return DDLR_OK;
}

ddlr_status ddlr_server_stats(ddlr_server* S, ddlr_server_counters* st) {
    if (!S || !st) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(st, 0, sizeof(*st));
    std::vector<double> l = S->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const double pos = q * (l.size() - 1);
        const size_t lo = (size_t)pos;
        const size_t hi = std::min(lo + 1, l.size() - 1);
        return l[lo] + (pos - lo) * (l[hi] - l[lo]);
    };
    st->requests_submitted = S->submitted;
    st->requests_done = S->requests_done;
    st->solves_done = S->solves_done;
    st->queued = (int64_t)S->queue.size();
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    const double span = S->t_last - S->t_first;
    st->solves_per_s = (span > 0 && S->solves_done > 0) ? S->solves_done / span : 0.0;
    st->hbm_used = S->used;
    st->hbm_budget = S->budget;
    st->matrices = (int32_t)S->mats.size();
    return DDLR_OK;
}

ddlr_status ddlr_server_reset_stats(ddlr_server* S) {
    if (!S) {
        g_err = "null argument";
        return DDLR_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->lat_ms.clear();
    S->solves_done = S->submitted = S->requests_done = 0;
    S->t_first = -1.0;
    S->t_last = 0.0;
    return DDLR_OK;
}

void ddlr_server_destroy(ddlr_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->device);
    (void)hipDeviceSynchronize();
    for (auto& M : S->mats) {
        if (M->st) (void)hipStreamDestroy(M->st);
        M->mem.release();
    }
    delete S;
}

}  // extern "C"
