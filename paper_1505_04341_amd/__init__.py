"""MI355X-native DDLR preconditioner (Li & Saad, domain-decomposition low-rank).

Thin ctypes binding over the C ABI in include/ddlr.h (libddlr.so, HIP for
gfx950).  Functions carry the C names; they only marshal arguments: every step
of setup, apply and solve runs in the library.  Device vectors are torch
tensors on the GPU, float64, shaped (n,) or (nrhs, n) and contiguous (row r of
the tensor is right-hand side r, i.e. column-major with ld = n).  There is no
CPU fallback: if the library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddlr.so")

OK, E_INVALID, E_NOT_SYMMETRIC, E_BREAKDOWN, E_NOT_SPD, E_NO_CONVERGENCE, E_LANCZOS, E_OOM, E_BUDGET, E_DEVICE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
VARIANT_A0, DDLR_1, DDLR_2 = 0, 1, 2
THETA_LAMBDA_K1, THETA_ZERO = 0, 1
FACTOR_IC0, FACTOR_ILDL0 = 0, 1
CORDER_MULTICOLOR, CORDER_NATURAL = 0, 1
FP64, FP32, FP32_UK_BF16 = 0, 1, 2
CSOLVE_FACTOR, CSOLVE_MR, CSOLVE_CHEB = 0, 1, 2
BUILD_LANCZOS, BUILD_BIDIAG = 0, 1
REORTH_FULL, REORTH_PARTIAL = 0, 1


class ddlr_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class ddlr_options(C.Structure):
    _fields_ = [("alpha", C.c_double), ("lanczos_steps", C.c_int32), ("theta", C.c_int32),
                ("factor", C.c_int32), ("corder", C.c_int32), ("precision", C.c_int32), ("device", C.c_int32),
                ("no_autotune", C.c_int32), ("lanczos_check", C.c_int32), ("lanczos_max", C.c_int32),
                ("lanczos_tol", C.c_double), ("seed", C.c_uint64), ("lanczos_start", C.c_void_p),
                ("csolve", C.c_int32), ("cinv_iters", C.c_int32), ("cinv_tol", C.c_double), ("cinv_lfil", C.c_int32),
                ("lowrank_build", C.c_int32), ("cheb_iters", C.c_int32), ("cheb_lanczos", C.c_int32),
                ("lanczos_reorth", C.c_int32)]


class ddlr_tuning(C.Structure):
    _fields_ = [("nrhs", C.c_int32), ("ring_cols", C.c_int32), ("overlap", C.c_int32), ("ring_threads", C.c_int32),
                ("a0_us", C.c_float * 4), ("a0_no_overlap_us", C.c_float), ("a0_thin_us", C.c_float * 2),
                ("a0_plain_us", C.c_float), ("cg_graph", C.c_int32), ("cg_eager_us", C.c_float),
                ("cg_graph_us", C.c_float), ("cg_overlap", C.c_int32), ("cg_eager_in_line_us", C.c_float),
                ("cg_graph_in_line_us", C.c_float), ("cg_persist", C.c_int32), ("cg_persist_us", C.c_float),
                ("persist_threads", C.c_int32), ("persist_nt_us", C.c_float * 5)]

    def as_dict(self):
        return dict(nrhs=self.nrhs, ring_cols=self.ring_cols, overlap=self.overlap, ring_threads=self.ring_threads,
                    a0_us=list(self.a0_us), a0_no_overlap_us=self.a0_no_overlap_us, a0_thin_us=list(self.a0_thin_us),
                    a0_plain_us=self.a0_plain_us, cg_graph=self.cg_graph, cg_eager_us=self.cg_eager_us,
                    cg_graph_us=self.cg_graph_us, cg_overlap=self.cg_overlap,
                    cg_eager_in_line_us=self.cg_eager_in_line_us, cg_graph_in_line_us=self.cg_graph_in_line_us,
                    cg_persist=self.cg_persist, cg_persist_us=self.cg_persist_us,
                    persist_threads=self.persist_threads, persist_nt_us=list(self.persist_nt_us))


class ddlr_solve_options(C.Structure):
    _fields_ = [("method", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32), ("reserved", C.c_int32),
                ("rtol", C.c_double)]


class ddlr_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double), ("relres_true", C.c_double)]


class ddlr_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("s", C.c_int64), ("nnz_a", C.c_int64), ("nnz_l", C.c_int64),
                ("nnz_e", C.c_int64), ("p", C.c_int32), ("k", C.c_int32), ("variant", C.c_int32),
                ("lanczos_steps", C.c_int32), ("ncolours", C.c_int32), ("levels_b_max", C.c_int32),
                ("levels_c", C.c_int32), ("spd", C.c_int32), ("precision", C.c_int32), ("on_device", C.c_int32),
                ("theta", C.c_double), ("c0", C.c_double), ("fill_ratio", C.c_double), ("setup_ms", C.c_double),
                ("lanczos_ms", C.c_double), ("csolve", C.c_int32), ("cinv_iters", C.c_int32),
                ("nnz_cinv", C.c_int64), ("cinv_res", C.c_double), ("cinv_res_inf", C.c_double),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double), ("cheb_ritz_lo", C.c_double),
                ("cheb_ritz_hi", C.c_double), ("lanczos_reorth", C.c_int32), ("lanczos_reorth_steps", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ddlr_server_counters(C.Structure):
    _fields_ = [("requests_submitted", C.c_int64), ("requests_done", C.c_int64), ("solves_done", C.c_int64),
                ("queued", C.c_int64), ("solves_per_s", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("hbm_used", C.c_size_t), ("hbm_budget", C.c_size_t), ("matrices", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class DDLRError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libddlr.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"DDLR HIP library not built: {path} is missing (run paper_1505_04341_amd/build.py)")
    lib = C.CDLL(path)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "ddlr_version": (I32, []),
        "ddlr_options_default": (None, [P]),
        "ddlr_solve_options_default": (None, [P]),
        "ddlr_setup": (I32, [P, P, P, I32, I32, I32, P, P]),
        "ddlr_ctx_create": (I32, [I32, C.c_size_t, P]),
        "ddlr_ctx_usage": (I32, [P, P, P, P]),
        "ddlr_ctx_destroy": (None, [P]),
        "ddlr_export_setup": (I32, [P, C.c_char_p]),
        "ddlr_import_setup": (I32, [P, P, C.c_char_p, P]),
        "ddlr_apply": (I32, [P, I32, P, I64, P, I64, P]),
        "ddlr_apply_noalloc": (I32, [P, I32, P, I64, P, I64, P]),
        "ddlr_a0_solve": (I32, [P, I32, P, I64, P, I64, P]),
        "ddlr_spmv": (I32, [P, I32, P, I64, P, I64, P]),
        "ddlr_solve": (I32, [P, I32, P, I64, P, I64, P, P, P]),
        "ddlr_query": (I32, [P, P]),
        "ddlr_get_ordering": (I32, [P, P, P, P]),
        "ddlr_get_factor": (I32, [P, P, P, P, P]),
        "ddlr_get_cinv": (I32, [P, P, P, P, P]),
        "ddlr_get_levels": (I32, [P, P]),
        "ddlr_get_lanczos": (I32, [P, P, P, P]),
        "ddlr_get_lanczos_reorth": (I32, [P, P]),
        "ddlr_get_lowrank": (I32, [P, P, P]),
        "ddlr_set_lowrank": (I32, [P, I32, I32, P, P]),
        "ddlr_profile": (I32, [P, I32]),
        "ddlr_profile_read": (I32, [P, I32, C.c_double, P, P]),
        "ddlr_batch_create": (I32, [I32, P, P]),
        "ddlr_batch_offsets": (I32, [P, P]),
        "ddlr_batch_apply": (I32, [P, P, P, P]),
        "ddlr_batch_tuning": (I32, [P, P, P, P]),
        "ddlr_batch_members": (I32, [P, P]),
        "ddlr_batch_times": (I32, [P, P]),
        "ddlr_batch_solve": (I32, [P, P, P, P, P, P]),
        "ddlr_batch_destroy": (None, [P]),
        "ddlr_server_create": (I32, [I32, C.c_size_t, I32, P]),
        "ddlr_server_add": (I32, [P, P, P]),
        "ddlr_server_submit": (I32, [P, I32, I32, P, P, P, P]),
        "ddlr_server_poll": (I32, [P, C.c_uint64, P, P]),
        "ddlr_server_wait": (I32, [P, C.c_uint64, P]),
        "ddlr_server_stats": (I32, [P, P]),
        "ddlr_server_reset_stats": (I32, [P]),
        "ddlr_server_destroy": (None, [P]),
        "ddlr_tune": (I32, [P, I32, I32, P, P]),
        "ddlr_extend_lowrank": (I32, [P, I32, I32, I32, C.c_double]),
        "ddlr_partition_graph": (I32, [P, I32, P]),
        "ddlr_partition_box": (I32, [I32, I32, I32, I32, I32, I32, P]),
        "ddlr_destroy": (None, [P]),
        "ddlr_status_string": (C.c_char_p, [I32]),
        "ddlr_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int, where: str):
    if st != OK:
        lib = load_library()
        raise DDLRError(st, where, lib.ddlr_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_cols(t, n: int):
    """(ptr, nrhs, ld) of a contiguous float64 GPU tensor shaped (n,) or (nrhs, n)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if t.dim() == 1:
        if t.shape[0] != n:
            raise ValueError("length mismatch")
        return C.c_void_p(t.data_ptr()), 1, n
    if t.dim() != 2 or t.shape[1] != n:
        raise ValueError("expected shape (nrhs, n)")
    return C.c_void_p(t.data_ptr()), t.shape[0], n


class Ctx:
    """Handle of a context (ddlr_ctx*): device and device-memory budget."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ddlr_ctx_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h


def ddlr_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> Ctx:
    h = C.c_void_p()
    _check(load_library().ddlr_ctx_create(int(device), int(hbm_budget_bytes), C.byref(h)), "ddlr_ctx_create")
    return Ctx(h.value)


def ddlr_ctx_usage(ctx: Ctx) -> dict:
    used, peak, budget = C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(load_library().ddlr_ctx_usage(ctx.handle, C.byref(used), C.byref(peak), C.byref(budget)),
           "ddlr_ctx_usage")
    return dict(used=used.value, peak=peak.value, budget=budget.value)


class Prec:
    """Handle of a built preconditioner (ddlr_prec*); keeps its context alive."""

    def __init__(self, handle: int, n: int, keep=(), ctx=None):
        self._h = C.c_void_p(handle)
        self.n = n
        self._keep = keep
        self._ctx = ctx

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ddlr_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h


def ddlr_setup(A, part, p: int, k: int, variant: int = DDLR_1, *, alpha: float = 1.0, lanczos_steps: int = 0,
               theta: int = THETA_LAMBDA_K1, factor: int = FACTOR_IC0, corder: int = CORDER_MULTICOLOR,
               precision: int = FP64, device: int = 0, seed: int = 0, lanczos_start=None,
               autotune: bool = True, lanczos_check: int = 0, lanczos_max: int = 0, lanczos_tol: float = 0.0,
               csolve: int = CSOLVE_FACTOR, cinv_iters: int = 3, cinv_tol: float = 0.01, cinv_lfil: int = 20,
               lowrank_build: int = BUILD_LANCZOS, cheb_iters: int = 5, cheb_lanczos: int = 10,
               lanczos_reorth: int = REORTH_FULL, ctx: "Ctx | None" = None) -> Prec:
    """Builds the preconditioner. A: object with n, rowptr (int64), col (int32), val (float64).
    ctx: a context (its device replaces `device`) or None."""
    lib = load_library()
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    pa = np.ascontiguousarray(part, dtype=np.int32)
    csr = ddlr_csr(int(A.n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    opt = ddlr_options()
    lib.ddlr_options_default(C.byref(opt))
    opt.alpha, opt.lanczos_steps, opt.theta = float(alpha), int(lanczos_steps), int(theta)
    opt.factor, opt.corder, opt.precision, opt.device, opt.seed = int(factor), int(corder), int(precision), int(
        device), int(seed)
    opt.no_autotune = 0 if autotune else 1
    opt.lanczos_check, opt.lanczos_max, opt.lanczos_tol = int(lanczos_check), int(lanczos_max), float(lanczos_tol)
    opt.csolve, opt.cinv_iters, opt.cinv_tol, opt.cinv_lfil = int(csolve), int(cinv_iters), float(cinv_tol), int(
        cinv_lfil)
    opt.lowrank_build = int(lowrank_build)
    opt.cheb_iters, opt.cheb_lanczos = int(cheb_iters), int(cheb_lanczos)
    opt.lanczos_reorth = int(lanczos_reorth)
    v0 = None
    if lanczos_start is not None:
        v0 = np.ascontiguousarray(lanczos_start, dtype=np.float64)
        opt.lanczos_start = v0.ctypes.data
    h = C.c_void_p()
    st = lib.ddlr_setup(ctx.handle if ctx is not None else None, C.byref(csr), _ptr(pa), int(p), int(k),
                        int(variant), C.byref(opt), C.byref(h))
    _check(st, "ddlr_setup")
    return Prec(h.value, int(A.n), ctx=ctx)


def ddlr_export_setup(prec: Prec, path: str) -> None:
    _check(load_library().ddlr_export_setup(prec.handle, os.fsencode(path)), "ddlr_export_setup")


def ddlr_import_setup(A, path: str, ctx: "Ctx | None" = None) -> Prec:
    """Rebuilds a preconditioner for A from a file of ddlr_export_setup's layout."""
    lib = load_library()
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    csr = ddlr_csr(int(A.n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    h = C.c_void_p()
    _check(lib.ddlr_import_setup(ctx.handle if ctx is not None else None, C.byref(csr), os.fsencode(path),
                                 C.byref(h)), "ddlr_import_setup")
    return Prec(h.value, int(A.n), ctx=ctx)


def _vec_op(name: str, prec: Prec, x, y, stream):
    lib = load_library()
    xp, nx, ldx = _dev_cols(x, prec.n)
    yp, ny, ldy = _dev_cols(y, prec.n)
    if nx != ny:
        raise ValueError("x and y must have the same number of columns")
    _check(getattr(lib, name)(prec.handle, nx, xp, ldx, yp, ldy, _stream(stream)), name)
    return y


def ddlr_apply(prec: Prec, x, y, stream=None):
    """y = M^{-1} x (device tensors, user order)."""
    return _vec_op("ddlr_apply", prec, x, y, stream)


def ddlr_apply_noalloc(prec: Prec, x, y, stream=None):
    """y = M^{-1} x with every temporary in the library's static scratch array."""
    return _vec_op("ddlr_apply_noalloc", prec, x, y, stream)


def ddlr_a0_solve(prec: Prec, x, y, stream=None):
    """y = A0^{-1} x with the local factors."""
    return _vec_op("ddlr_a0_solve", prec, x, y, stream)


def ddlr_spmv(prec: Prec, x, y, stream=None):
    """y = A x."""
    return _vec_op("ddlr_spmv", prec, x, y, stream)


def ddlr_solve(prec: Prec, b, x, *, method: int = 0, restart: int = 40, maxit: int = 500, rtol: float = 1e-6,
               stream=None, raise_on_noconv: bool = False):
    """Solves A x = b (PCG or GMRES); returns (status, list of per-rhs info dicts)."""
    lib = load_library()
    bp, nb, ldb = _dev_cols(b, prec.n)
    xp, nxc, ldx = _dev_cols(x, prec.n)
    if nb != nxc:
        raise ValueError("b and x must have the same number of columns")
    opt = ddlr_solve_options()
    lib.ddlr_solve_options_default(C.byref(opt))
    opt.method, opt.restart, opt.maxit, opt.rtol = int(method), int(restart), int(maxit), float(rtol)
    infos = (ddlr_solve_info * nb)()
    st = lib.ddlr_solve(prec.handle, nb, bp, ldb, xp, ldx, C.byref(opt), infos, _stream(stream))
    if st not in (OK, E_NO_CONVERGENCE) or (raise_on_noconv and st != OK):
        _check(st, "ddlr_solve")
    return st, [dict(iters=i.iters, status=i.status, relres=i.relres, relres_true=i.relres_true) for i in infos]


def ddlr_query(prec: Prec) -> dict:
    lib = load_library()
    info = ddlr_info()
    _check(lib.ddlr_query(prec.handle, C.byref(info)), "ddlr_query")
    return info.as_dict()


def ddlr_get_ordering(prec: Prec):
    """(perm, iface, colour) as numpy arrays (see ddlr.h)."""
    lib = load_library()
    q = ddlr_query(prec)
    perm = np.zeros(q["n"], np.int32)
    iface = np.zeros(q["n"], np.int32)
    colour = np.zeros(max(q["s"], 1), np.int32)
    _check(lib.ddlr_get_ordering(prec.handle, _ptr(perm), _ptr(iface), _ptr(colour)), "ddlr_get_ordering")
    return perm, iface, colour[: q["s"]]


def ddlr_get_factor(prec: Prec):
    """(L as scipy CSR in internal order, D)."""
    import scipy.sparse as sp
    lib = load_library()
    q = ddlr_query(prec)
    n, nnz = q["n"], q["nnz_l"]
    rp = np.zeros(n + 1, np.int64)
    ci = np.zeros(max(nnz, 1), np.int32)
    v = np.zeros(max(nnz, 1))
    D = np.zeros(n)
    _check(lib.ddlr_get_factor(prec.handle, _ptr(rp), _ptr(ci), _ptr(v), _ptr(D)), "ddlr_get_factor")
    return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(n, n)), D


def ddlr_get_cinv(prec: Prec):
    """(X as scipy CSR s x s in interface positions of the internal order,
    residual norms ||I - C_alpha X_j||_F for j = 0..cinv_iters)."""
    import scipy.sparse as sp
    lib = load_library()
    q = ddlr_query(prec)
    s, nnz = q["s"], q["nnz_cinv"]
    rp = np.zeros(s + 1, np.int64)
    ci = np.zeros(max(nnz, 1), np.int32)
    v = np.zeros(max(nnz, 1))
    res = np.zeros(q["cinv_iters"] + 1)
    _check(lib.ddlr_get_cinv(prec.handle, _ptr(rp), _ptr(ci), _ptr(v), _ptr(res)), "ddlr_get_cinv")
    return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(s, s)), res


def ddlr_partition_box(dims, parts) -> np.ndarray:
    """Box partition of a lexicographic 2-D or 3-D grid (x fastest)."""
    d = list(dims) + [1] * (3 - len(dims))
    q = list(parts) + [1] * (3 - len(parts))
    part = np.zeros(int(np.prod(d)), np.int32)
    _check(load_library().ddlr_partition_box(*[int(v) for v in d], *[int(v) for v in q], _ptr(part)),
           "ddlr_partition_box")
    return part


def ddlr_get_levels(prec: Prec):
    lib = load_library()
    lev = np.zeros(prec.n, np.int32)
    _check(lib.ddlr_get_levels(prec.handle, _ptr(lev)), "ddlr_get_levels")
    return lev


def ddlr_get_lanczos(prec: Prec):
    lib = load_library()
    m = ddlr_query(prec)["lanczos_steps"]
    a, b, r = np.zeros(max(m, 1)), np.zeros(max(m, 1)), np.zeros(max(m, 1))
    _check(lib.ddlr_get_lanczos(prec.handle, _ptr(a), _ptr(b), _ptr(r)), "ddlr_get_lanczos")
    return a[:m], b[:m], r[:m]


def ddlr_get_lanczos_reorth(prec: Prec):
    """Per-step flags of the stored Lanczos run: 1 where the new vector was reorthogonalised."""
    m = ddlr_query(prec)["lanczos_steps"]
    f = np.zeros(max(m, 1), np.int32)
    _check(load_library().ddlr_get_lanczos_reorth(prec.handle, _ptr(f)), "ddlr_get_lanczos_reorth")
    return f[:m]


def ddlr_get_lowrank(prec: Prec):
    """DDLR-1: (U n x k, lambda, theta); DDLR-2: (U, H_k)."""
    lib = load_library()
    q = ddlr_query(prec)
    n, k = q["n"], q["k"]
    U = np.zeros((n, k), order="F")
    aux = np.zeros(k + 1 if q["variant"] == 1 else k * k)
    _check(lib.ddlr_get_lowrank(prec.handle, _ptr(U), _ptr(aux)), "ddlr_get_lowrank")
    if q["variant"] == 1:
        return U, aux[:k].copy(), float(aux[k])
    return U, aux.reshape(k, k, order="F").copy()


def ddlr_set_lowrank(prec: Prec, variant: int, U, lam_or_H, theta: float = 0.0):
    lib = load_library()
    U = np.asfortranarray(U, dtype=np.float64)
    k = U.shape[1]
    if variant == 1:
        aux = np.concatenate([np.asarray(lam_or_H, np.float64), [float(theta)]])
    else:
        aux = np.asfortranarray(lam_or_H, dtype=np.float64).reshape(-1, order="F")
    _check(lib.ddlr_set_lowrank(prec.handle, int(variant), int(k), _ptr(U), _ptr(aux)), "ddlr_set_lowrank")


class Batch:
    """Handle of a batch of independent systems (ddlr_batch*)."""

    def __init__(self, handle: int, offsets: np.ndarray):
        self._h = C.c_void_p(handle)
        self.offsets = offsets
        self.n = int(offsets[-1])
        self.nsys = len(offsets) - 1

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ddlr_batch_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h


def ddlr_batch_create(members) -> Batch:
    """Merges built preconditioners of independent systems into one batch."""
    lib = load_library()
    arr = (C.c_void_p * len(members))(*[m.handle.value for m in members])
    h = C.c_void_p()
    _check(lib.ddlr_batch_create(len(members), arr, C.byref(h)), "ddlr_batch_create")
    off = np.zeros(len(members) + 1, np.int64)
    _check(lib.ddlr_batch_offsets(h, _ptr(off)), "ddlr_batch_offsets")
    return Batch(h.value, off)


def ddlr_batch_apply(batch: Batch, x, y, stream=None):
    xp, _, _ = _dev_cols(x, batch.n)
    yp, _, _ = _dev_cols(y, batch.n)
    _check(load_library().ddlr_batch_apply(batch.handle, xp, yp, _stream(stream)), "ddlr_batch_apply")
    return y


def ddlr_batch_tuning(batch: Batch) -> dict:
    """The batch's solve form and the tuned workgroup size of its persistent launch."""
    pers, nt = C.c_int32(), C.c_int32()
    us = (C.c_float * 5)()
    _check(load_library().ddlr_batch_tuning(batch.handle, C.byref(pers), C.byref(nt), us), "ddlr_batch_tuning")
    return dict(persistent=pers.value, threads=nt.value, us_per_iter=list(us))


def ddlr_batch_members(batch: Batch) -> list:
    """Workgroups that solve each system in the persistent form (0: chunked form)."""
    arr = (C.c_int32 * batch.nsys)()
    _check(load_library().ddlr_batch_members(batch.handle, arr), "ddlr_batch_members")
    return list(arr)


def ddlr_batch_times(batch: Batch) -> list:
    """Device time (microseconds) of each system in the last persistent batch solve."""
    arr = (C.c_double * batch.nsys)()
    _check(load_library().ddlr_batch_times(batch.handle, arr), "ddlr_batch_times")
    return list(arr)


def ddlr_batch_solve(batch: Batch, b, x, *, maxit: int = 500, rtol: float = 1e-6, stream=None):
    """PCG on every system; returns (status, list of per-system info dicts)."""
    lib = load_library()
    bp, _, _ = _dev_cols(b, batch.n)
    xp, _, _ = _dev_cols(x, batch.n)
    opt = ddlr_solve_options()
    lib.ddlr_solve_options_default(C.byref(opt))
    opt.maxit, opt.rtol = int(maxit), float(rtol)
    infos = (ddlr_solve_info * batch.nsys)()
    st = lib.ddlr_batch_solve(batch.handle, bp, xp, C.byref(opt), infos, _stream(stream))
    if st not in (OK, E_NO_CONVERGENCE):
        _check(st, "ddlr_batch_solve")
    return st, [dict(iters=i.iters, status=i.status, relres=i.relres, relres_true=i.relres_true) for i in infos]


class Server:
    """Handle of a serving engine (ddlr_server*).  Keeps the host arrays of
    pending requests alive until they complete."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)
        self._pending = {}
        self._members = []

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ddlr_server_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h


def ddlr_server_create(device: int = 0, hbm_budget_bytes: int = 0, slots_per_matrix: int = 16) -> Server:
    h = C.c_void_p()
    _check(load_library().ddlr_server_create(int(device), int(hbm_budget_bytes), int(slots_per_matrix), C.byref(h)),
           "ddlr_server_create")
    return Server(h.value)


def ddlr_server_add(server: Server, prec: Prec) -> int:
    mid = C.c_int32()
    _check(load_library().ddlr_server_add(server.handle, prec.handle, C.byref(mid)), "ddlr_server_add")
    server._members.append(prec)  # the server uses the handle from now on
    return mid.value


def ddlr_server_submit(server: Server, matrix_id: int, b: np.ndarray, *, rtol: float = 1e-6, maxit: int = 500):
    """b: host (n,) or (n, nrhs); returns (ticket, x) where x is filled when the request is done."""
    lib = load_library()
    b2 = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1))
    x = np.zeros_like(b2, order="F")
    opt = ddlr_solve_options()
    lib.ddlr_solve_options_default(C.byref(opt))
    opt.rtol, opt.maxit = float(rtol), int(maxit)
    t = C.c_uint64()
    _check(lib.ddlr_server_submit(server.handle, int(matrix_id), b2.shape[1], _ptr(b2), _ptr(x), C.byref(opt),
                                  C.byref(t)), "ddlr_server_submit")
    server._pending[t.value] = (b2, x)
    return t.value, x


def ddlr_server_poll(server: Server, ticket: int):
    b2, x = server._pending[ticket]
    infos = (ddlr_solve_info * b2.shape[1])()
    done = C.c_int32()
    _check(load_library().ddlr_server_poll(server.handle, C.c_uint64(ticket), C.byref(done), infos), "ddlr_server_poll")
    if not done.value:
        return False, None
    return True, [dict(iters=i.iters, status=i.status, relres=i.relres) for i in infos]


def ddlr_server_wait(server: Server, ticket: int):
    b2, x = server._pending[ticket]
    infos = (ddlr_solve_info * b2.shape[1])()
    st = load_library().ddlr_server_wait(server.handle, C.c_uint64(ticket), infos)
    if st not in (OK, E_NO_CONVERGENCE):
        _check(st, "ddlr_server_wait")
    return st, [dict(iters=i.iters, status=i.status, relres=i.relres, relres_true=i.relres_true) for i in infos]


def ddlr_server_stats(server: Server) -> dict:
    c = ddlr_server_counters()
    _check(load_library().ddlr_server_stats(server.handle, C.byref(c)), "ddlr_server_stats")
    return c.as_dict()


def ddlr_partition_graph(A, p: int) -> np.ndarray:
    """Recursive-bisection partition of the adjacency graph of A into p parts (host)."""
    lib = load_library()
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    csr = ddlr_csr(int(A.n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    part = np.zeros(int(A.n), np.int32)
    _check(lib.ddlr_partition_graph(C.byref(csr), int(p), _ptr(part)), "ddlr_partition_graph")
    return part


def ddlr_extend_lowrank(prec: Prec, k: int, more_steps: int, check: int = 0, tol: float = 0.0) -> None:
    """Continues the setup's Lanczos run and rebuilds the low-rank part with rank k."""
    _check(load_library().ddlr_extend_lowrank(prec.handle, int(k), int(more_steps), int(check), float(tol)),
           "ddlr_extend_lowrank")


def ddlr_tune(prec: Prec, nrhs: int, retune: bool = False, stream=None) -> dict:
    """Runs (or reports) the launch-shape autotuner for nrhs columns."""
    t = ddlr_tuning()
    _check(load_library().ddlr_tune(prec.handle, int(nrhs), 1 if retune else 0, C.byref(t), _stream(stream)),
           "ddlr_tune")
    return t.as_dict()


def ddlr_server_reset_stats(server: Server) -> None:
    _check(load_library().ddlr_server_reset_stats(server.handle), "ddlr_server_reset_stats")


PROF_TRSV_BLOCKS, PROF_TRSV_LEVELS, PROF_SPMV, PROF_LOWRANK = 0, 1, 2, 3


def ddlr_profile(prec: Prec, on: bool = True):
    _check(load_library().ddlr_profile(prec.handle, 1 if on else 0), "ddlr_profile")


def ddlr_profile_read(prec: Prec, which: int, min_us: float = 0.0):
    """(total milliseconds, launches) of a kernel class since profiling was
    enabled, counting launches of at least min_us microseconds."""
    t = C.c_double()
    cnt = C.c_int64()
    _check(load_library().ddlr_profile_read(prec.handle, int(which), float(min_us), C.byref(t), C.byref(cnt)),
           "ddlr_profile_read")
    return t.value, cnt.value


def ddlr_version() -> int:
    return int(load_library().ddlr_version())


EXPORTED = ["ddlr_version", "ddlr_options_default", "ddlr_solve_options_default", "ddlr_setup", "ddlr_apply",
            "ddlr_apply_noalloc", "ddlr_ctx_create", "ddlr_ctx_usage", "ddlr_ctx_destroy", "ddlr_export_setup",
            "ddlr_import_setup", "ddlr_partition_box", "ddlr_batch_tuning", "ddlr_batch_members", "ddlr_batch_times",
            "ddlr_a0_solve", "ddlr_spmv", "ddlr_solve", "ddlr_query", "ddlr_get_ordering", "ddlr_get_factor",
            "ddlr_get_cinv",
            "ddlr_get_levels", "ddlr_get_lanczos", "ddlr_get_lanczos_reorth", "ddlr_get_lowrank", "ddlr_set_lowrank", "ddlr_profile",
            "ddlr_profile_read", "ddlr_batch_create", "ddlr_batch_offsets", "ddlr_batch_apply",
            "ddlr_batch_solve", "ddlr_batch_destroy", "ddlr_server_create", "ddlr_server_add", "ddlr_server_submit",
            "ddlr_server_poll", "ddlr_server_wait", "ddlr_server_stats", "ddlr_server_reset_stats", "ddlr_server_destroy", "ddlr_extend_lowrank", "ddlr_partition_graph", "ddlr_tune", "ddlr_destroy",
            "ddlr_status_string", "ddlr_last_error"]
