// Host-side construction of the DDLR splitting and local factors.
//
// Steps 1-3 of the build (Sec. 4.1): classification and reordering (Sec. 2.1,
// eq. Bmat), the splitting A = A0 - E E^T (Sec. 3.1), incomplete LDL^T of every
// diagonal block of A0 (Sec. 5), plus what the GPU needs to run those factors:
// a level schedule per block and the "device order" that stores every level of
// every block contiguously.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ddlr {

struct SetupError {
    int status;
    std::string msg;
};

struct HostCsr {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    int64_t rows() const { return rp.empty() ? 0 : (int64_t)rp.size() - 1; }
    int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

struct HostPlan {
    int64_t n = 0, m = 0, s = 0;
    int32_t p = 0;
    double alpha = 1.0;
    int32_t ncolours = 0;
    // ordering (internal = factor order)
    std::vector<int32_t> iface;   // user row -> 0/1
    std::vector<int32_t> perm;    // internal -> user
    std::vector<int32_t> iperm;   // user -> internal
    std::vector<int32_t> colour;  // interface position -> colour
    std::vector<int64_t> boff;    // p+2 block offsets (internal order)
    // internal-order matrices
    HostCsr A;    // P A P^T
    HostCsr A0;   // blockdiag(B_alpha, C_alpha)
    HostCsr L;    // strict lower incomplete factor, internal order
    std::vector<double> D;
    // level schedule (internal order) and device order
    std::vector<int32_t> level;   // internal row -> level inside its block
    std::vector<int32_t> dev2int; // device position -> internal row
    std::vector<int32_t> int2dev; // internal row -> device position
    std::vector<int32_t> lvl_ptr; // device-order row offsets of all levels, all blocks, concatenated
    std::vector<int32_t> blk_lvl; // p+2: levels of block b are lvl_ptr[blk_lvl[b] .. blk_lvl[b+1]]
    int32_t levels_b_max = 0, levels_c = 0;
    // C_alpha solved by its approximate inverse (csolve = 1; cinv.cpp): the
    // interface rows of L are then empty and D is 1 there
    int csolve = 0;
    HostCsr X;                  // s x s, symmetric, interface positions (internal order)
    std::vector<double> x_res;  // ||I - C_alpha X_j||_F, j = 0..x_iters
    int x_iters = 0;
    double x_rinf = 0.0;        // ||I - C_alpha X||_inf of the final X
    bool x_spd = false;         // x_rinf < 1
    // C_alpha by preconditioned Chebyshev (csolve = 2; cheb.cpp): the interface
    // block of L, D factors D_alpha = blockdiag(C_i); safeguarded interval
    // [ch_lo, ch_hi] and extreme Ritz values of D_alpha^{-1} C_alpha
    double ch_lo = 0.0, ch_hi = 0.0, ch_rlo = 0.0, ch_rhi = 0.0;
};

// Validates A (sorted columns, symmetric values) and part.
void validate(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, const int32_t* part, int32_t p);

// Steps 1-3.  factor: 0 = IC(0) (pivots must be > 0), 1 = ILDL(0) (|pivot| >=
// 1e-14 |a_ii|).  corder: 0 = greedy multicolour interface order, 1 = natural.
// csolve: 0 = C_alpha factored like the B blocks; 1 = C_alpha by the
// approximate inverse of Algorithm alg:mr (cinv_iters steps, drop tolerance
// cinv_tol, at most cinv_lfil kept off-diagonal entries per column); 2 =
// preconditioned Chebyshev with D_alpha = blockdiag(C_i), its spectrum from
// cheb_lanczos Lanczos steps on (C_alpha, D_alpha).
void build_plan(HostPlan& P, int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                const int32_t* part, int32_t p, double alpha, int factor, int corder, int csolve = 0,
                int cinv_iters = 3, double cinv_tol = 0.01, int cinv_lfil = 20, int cheb_lanczos = 10);

// Steps 1-3 from stored data (ddlr_import_setup): the ordering (perm,
// block offsets, interface colours) and the local factors (strict lower L and
// D in internal order) are taken as given and checked against A (perm a
// permutation, interiors of different blocks uncoupled, L strictly lower
// inside its row's block with sorted columns, pivots finite and nonzero);
// P A P^T and A0 are formed and the level schedule recomputed from L as in
// build_plan.  The caller sets X or the Chebyshev interval for csolve 1 / 2.
void build_plan_imported(HostPlan& P, int64_t n, const int64_t* rp, const int32_t* ci, const double* v, int32_t p,
                         double alpha, std::vector<int32_t> perm, std::vector<int64_t> boff,
                         std::vector<int32_t> colour, HostCsr L, std::vector<double> D, int csolve);

// Spectrum interval of D_alpha^{-1} C_alpha for the Chebyshev solver (cheb.cpp).
void cheb_bounds(HostPlan& P, int mc);

// X ~ C_alpha^{-1} by Algorithm alg:mr into P.X, P.x_res, P.x_iters, P.x_spd.
void build_cinv(HostPlan& P, int nit, double tol, int lfil);

// Eigen-decomposition of a symmetric tridiagonal matrix (diag a[0..m-1],
// off-diagonal b[0..m-2]) by implicit QR steps with Wilkinson shifts.
// Returns eigenvalues (unsorted) in ev and eigenvectors column-major in Z.
void tridiag_eig(int m, const double* a, const double* b, std::vector<double>& ev, std::vector<double>& Z);

// Recursive bisection of the adjacency graph of a symmetric pattern into p
// parts (partition.cpp).
void partition_graph(int64_t n, const int64_t* rp, const int32_t* ci, int32_t p, int32_t* part);

}  // namespace ddlr
