"""CPU FP64 oracle of the DDLR preconditioner -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ddlr_oracle.c (plain C, FP64). Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
HIP library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddlr_oracle.c")
_LIB = os.path.join(_HERE, "libddlr_oracle.so")

OK, E_INVALID, E_NOT_SYMMETRIC, E_BREAKDOWN, E_NOT_SPD, E_NO_CONVERGENCE, E_LANCZOS = 0, -1, -2, -3, -4, -5, -6
FACTOR_IC, FACTOR_ILDL, FACTOR_EXACT = 0, 1, 2
CORDER_MULTICOLOR, CORDER_NATURAL = 0, 1


def build(force: bool = True, out: str = _LIB, native: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O3, OpenMP).  native=True adds
    -march=native: only for a build made and run on the same machine (the
    CPU-baseline timing builds its own copy that way).  sanitize=True builds
    with AddressSanitizer and UndefinedBehaviorSanitizer (-O1 -g, stop at the
    first report); a process loading it needs libasan preloaded."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        flags = ["-O3"] + (["-march=native"] if native else [])
        if sanitize:
            flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all"]
        subprocess.check_call(["gcc", *flags, "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None
_lib_path = _LIB


def use_native_build(directory: str) -> str:
    """Builds an -O3 -march=native copy of the oracle in `directory` and makes
    it the one this process loads (call before the first Oracle)."""
    global _lib_path
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _lib_path = build(True, os.path.join(directory, "libddlr_oracle_native.so"), native=True)
    return _lib_path


def use_library(path: str) -> str:
    """Makes the oracle library at `path` (a build() output) the one this
    process loads (call before the first Oracle)."""
    global _lib_path
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _lib_path = path
    return _lib_path


def _load():
    global _lib
    if _lib is None:
        if _lib_path == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        lib = C.CDLL(_lib_path)
        P = C.c_void_p
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [C.c_int64, P, P, P, P, C.c_int32, C.c_double, C.c_int, C.c_int,
                                   C.POINTER(C.c_int)]
        lib.orc_free.argtypes = [P]
        lib.orc_size.restype = C.c_int64
        lib.orc_size.argtypes = [P, C.c_int]
        lib.orc_ordering.argtypes = [P, P, P, P, P]
        lib.orc_csr.argtypes = [P, C.c_int, P, P, P]
        lib.orc_diag.argtypes = [P, P]
        lib.orc_a0_solve.argtypes = [P, C.c_int, P, P]
        lib.orc_lowrank.restype = C.c_int
        lib.orc_lowrank.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, P]
        lib.orc_lowrank_ctl.restype = C.c_int
        lib.orc_lowrank_ctl.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, P]
        lib.orc_lowrank_gk.restype = C.c_int
        lib.orc_lowrank_gk.argtypes = [P, C.c_int, C.c_int, P]
        lib.orc_extend.restype = C.c_int
        lib.orc_extend.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int]
        lib.orc_lanczos_record.argtypes = [P, P, P, P]
        lib.orc_lanczos_basis.argtypes = [P, P]
        lib.orc_get_lowrank.argtypes = [P, P, P]
        lib.orc_set_lowrank.argtypes = [P, C.c_int, C.c_int, P, P]
        lib.orc_apply.argtypes = [P, C.c_int, P, P]
        lib.orc_pcg.restype = C.c_int
        lib.orc_pcg.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int, P, P]
        lib.orc_gmres.restype = C.c_int
        lib.orc_gmres.argtypes = [P, C.c_int, P, P, C.c_int, C.c_double, C.c_int, P, P]
        lib.orc_matvec.argtypes = [P, P, P]
        lib.orc_use_cinv.restype = C.c_int
        lib.orc_use_cinv.argtypes = [P, C.c_int, C.c_double, C.c_int]
        lib.orc_cinv.argtypes = [P, P, P, P, P]
        lib.orc_use_cheb.restype = C.c_int
        lib.orc_use_cheb.argtypes = [P, C.c_int, C.c_int]
        lib.orc_cheb.argtypes = [P, P]
        lib.orc_set_reorth.restype = C.c_int
        lib.orc_set_reorth.argtypes = [P, C.c_int]
        lib.orc_reorth_steps.restype = C.c_int
        lib.orc_reorth_steps.argtypes = [P, P]
        lib.orc_threads.restype = C.c_int
        lib.orc_threads.argtypes = []
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Sets the OpenMP thread count of the oracle's parallel loops."""
    _load().orc_set_threads(int(n))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"oracle status {status} {msg}")
        self.status = status


class Oracle:
    """One DDLR preconditioner built by the oracle.

    A: workloads.CSR (user order); part: int32[n]; p subdomains.
    factor: FACTOR_IC / FACTOR_ILDL / FACTOR_EXACT; corder: colour or natural
    order of the interface block.
    """

    def __init__(self, A, part, p, alpha=1.0, corder=CORDER_MULTICOLOR, factor=FACTOR_IC):
        lib = _load()
        self.n = int(A.n)
        self._keep = (np.ascontiguousarray(A.rowptr, dtype=np.int64),
                      np.ascontiguousarray(A.col, dtype=np.int32),
                      np.ascontiguousarray(A.val, dtype=np.float64),
                      np.ascontiguousarray(part, dtype=np.int32))
        st = C.c_int(0)
        self._h = lib.orc_create(self.n, *[_p(a) for a in self._keep], int(p), float(alpha), int(corder),
                                 int(factor), C.byref(st))
        self.p = int(p)
        self.status = st.value
        if st.value != OK:
            row = lib.orc_size(self._h, 8)
            lib.orc_free(self._h)
            self._h = None
            raise OracleError(st.value, f"(breakdown row {row})" if st.value == E_BREAKDOWN else "")
        self.m = int(lib.orc_size(self._h, 1))
        self.s = int(lib.orc_size(self._h, 2))
        self.ncolours = int(lib.orc_size(self._h, 6))
        self.variant = 0
        self.k = 0

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_free(self._h)
            self._h = None

    # ---- setup data
    def ordering(self):
        """(perm, iface, colour, boff): perm[internal] = user row; iface[user];
        colour[interface position]; block offsets (p+2)."""
        perm = np.zeros(self.n, np.int32)
        iface = np.zeros(self.n, np.int32)
        colour = np.zeros(max(self.s, 1), np.int32)
        boff = np.zeros(self.p + 2, np.int64)
        _lib.orc_ordering(self._h, _p(perm), _p(iface), _p(colour), _p(boff))
        return perm, iface, colour[: self.s], boff

    def csr(self, which: str):
        """Internal-order sparse matrix: 'PAP', 'A0', 'E' (n x s) or 'L' (strict lower)."""
        import scipy.sparse as sp
        code = {"PAP": 0, "A0": 1, "E": 2, "L": 3}[which]
        nnz = {0: int(self._keep[0][-1]), 1: int(_lib.orc_size(self._h, 4)), 2: int(_lib.orc_size(self._h, 5)),
               3: int(_lib.orc_size(self._h, 3))}[code]
        rp = np.zeros(self.n + 1, np.int64)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1), np.float64)
        _lib.orc_csr(self._h, code, _p(rp), _p(ci), _p(v))
        ncol = self.s if which == "E" else self.n
        return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(self.n, ncol))

    def diag(self):
        D = np.zeros(self.n)
        _lib.orc_diag(self._h, _p(D))
        return D

    def use_cinv(self, nit=3, tol=0.01, lfil=20):
        """Solve C_alpha with the MR approximate inverse (Algorithm alg:mr,
        X_0 = diag(C_alpha)^{-1}, nit steps, dual-threshold dropping tol /
        lfil). Call before lowrank."""
        st = _lib.orc_use_cinv(self._h, int(nit), float(tol), int(lfil))
        if st != OK:
            raise OracleError(st, "cinv")
        return self

    def use_cheb(self, nu=5, mc=10):
        """Solve C_alpha with nu preconditioned Chebyshev steps, block-Jacobi
        D_alpha = blockdiag(C_i) by incomplete LDL^T, spectrum from mc Lanczos
        steps on (C_alpha, D_alpha) with residual safeguards. Call before lowrank."""
        st = _lib.orc_use_cheb(self._h, int(nu), int(mc))
        if st != OK:
            raise OracleError(st, "cheb")
        return self

    def cheb(self):
        """(lo, hi) safeguarded interval and (smallest, largest) Ritz value."""
        out = np.zeros(4)
        _lib.orc_cheb(self._h, _p(out))
        return tuple(out)

    def cinv(self):
        """(X: scipy CSR s x s in interface order, residual norms
        ||I - C_alpha X_j||_F for j = 0..steps, SPD certificate
        ||I - C_alpha X||_inf < 1).  .cinv_rinf holds ||I - C_alpha X||_inf."""
        import scipy.sparse as sp
        nnz = int(_lib.orc_size(self._h, 11))
        steps = int(_lib.orc_size(self._h, 12))
        rp = np.zeros(self.s + 1, np.int64)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1))
        res = np.zeros(steps + 2)
        _lib.orc_cinv(self._h, _p(rp), _p(ci), _p(v), _p(res))
        X = sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(self.s, self.s))
        self.cinv_rinf = float(res[-1])
        return X, res[:-1], bool(_lib.orc_size(self._h, 13))

    # ---- operators (user order, columns of an (n, nrhs) array)
    @staticmethod
    def _cols(x):
        x = np.asarray(x, dtype=np.float64)
        one = x.ndim == 1
        x2 = np.asfortranarray(x.reshape(x.shape[0], -1))
        return x2, one

    def a0_solve(self, x):
        x2, one = self._cols(x)
        z = np.zeros_like(x2, order="F")
        _lib.orc_a0_solve(self._h, x2.shape[1], _p(x2), _p(z))
        return z[:, 0] if one else z

    def set_reorth(self, mode):
        """Reorthogonalisation of the following Lanczos runs: 0 full (CGS2 every
        step), 1 partial (Simon's omega recurrence), 2 none (tests only)."""
        if _lib.orc_set_reorth(self._h, int(mode)) != 0:
            raise OracleError(E_INVALID, "reorth mode")
        return self

    def reorth_steps(self):
        """Per-step flags (1: the new vector was reorthogonalised) of the stored run."""
        msteps = int(_lib.orc_size(self._h, 7))
        f = np.zeros(max(msteps, 1), np.int32)
        _lib.orc_reorth_steps(self._h, _p(f))
        return f[:msteps]

    def lowrank(self, variant, k, m, v0, theta_zero=False, check=0, eps=1e-4):
        """Lanczos of m steps (check = 0) or of at most m steps stopped by the
        convergence test every `check` steps with tolerance eps, then the
        low-rank build with rank k."""
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        st = _lib.orc_lowrank_ctl(self._h, int(variant), int(k), int(m), int(check), float(eps),
                                  1 if theta_zero else 0, _p(v0))
        if st != OK:
            raise OracleError(st, "lowrank")
        self.variant, self.k = int(variant), int(k)
        self.spd = bool(_lib.orc_size(self._h, 10))
        return self

    def lowrank_gk(self, k, m, v0):
        """DDLR-2 with U_k, V_k from m steps of the bidiagonalisation of
        A0^{-1} E (Sec. 4.4 (sec:Lan) alternative)."""
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        st = _lib.orc_lowrank_gk(self._h, int(k), int(m), _p(v0))
        if st != OK:
            raise OracleError(st, "lowrank_gk")
        self.variant, self.k = 2, int(k)
        self.spd = bool(_lib.orc_size(self._h, 10))
        return self

    def extend(self, k, more, check=0, eps=1e-4, theta_zero=False):
        """Continue the stored Lanczos run by `more` steps (or until the
        convergence test holds) and rebuild with rank k."""
        st = _lib.orc_extend(self._h, int(k), int(more), int(check), float(eps), 1 if theta_zero else 0)
        if st != OK:
            raise OracleError(st, "extend")
        self.k = int(k)
        self.spd = bool(_lib.orc_size(self._h, 10))
        return self

    @property
    def msteps(self):
        return int(_lib.orc_size(self._h, 7))

    def lanczos_record(self):
        msteps = int(_lib.orc_size(self._h, 7))
        ta, tb, rz = np.zeros(msteps), np.zeros(msteps), np.zeros(msteps)
        _lib.orc_lanczos_record(self._h, _p(ta), _p(tb), _p(rz))
        return ta, tb, rz

    def lanczos_basis(self):
        msteps = int(_lib.orc_size(self._h, 7))
        Q = np.zeros((self.s, msteps), order="F")
        _lib.orc_lanczos_basis(self._h, _p(Q))
        return Q

    def get_lowrank(self):
        """DDLR-1: (U n x k user order, lambda[k], theta). DDLR-2: (U, H_k)."""
        k = self.k
        U = np.zeros((self.n, k), order="F")
        aux = np.zeros(k * k if self.variant == 2 else k + 1)
        _lib.orc_get_lowrank(self._h, _p(U), _p(aux))
        if self.variant == 1:
            return U, aux[:k].copy(), float(aux[k])
        return U, aux.reshape(k, k, order="F").copy()

    def set_lowrank(self, variant, U, lam_or_H, theta=0.0):
        U = np.asfortranarray(U, dtype=np.float64)
        k = U.shape[1]
        if variant == 1:
            aux = np.concatenate([np.asarray(lam_or_H, np.float64), [float(theta)]])
        else:
            aux = np.asfortranarray(lam_or_H, dtype=np.float64).reshape(-1, order="F")
        _lib.orc_set_lowrank(self._h, int(variant), int(k), _p(U), _p(aux))
        self.variant, self.k = int(variant), int(k)
        return self

    def matvec(self, x):
        """y = A x in user order, row sums in ascending column order."""
        x2, one = self._cols(x)
        y = np.zeros_like(x2, order="F")
        for j in range(x2.shape[1]):
            xj = np.ascontiguousarray(x2[:, j])
            yj = np.zeros(self.n)
            _lib.orc_matvec(self._h, _p(xj), _p(yj))
            y[:, j] = yj
        return y[:, 0] if one else y

    def apply(self, x):
        x2, one = self._cols(x)
        y = np.zeros_like(x2, order="F")
        _lib.orc_apply(self._h, x2.shape[1], _p(x2), _p(y))
        return y[:, 0] if one else y

    def pcg(self, b, rtol=1e-6, maxit=500):
        b2, one = self._cols(b)
        x = np.zeros_like(b2, order="F")
        its = np.zeros(b2.shape[1], np.int32)
        rel = np.zeros(2 * b2.shape[1])
        st = _lib.orc_pcg(self._h, b2.shape[1], _p(b2), _p(x), float(rtol), int(maxit), _p(its), _p(rel))
        info = dict(status=st, its=its, relres=rel[0::2], relres_true=rel[1::2])
        return (x[:, 0] if one else x), info

    def gmres(self, b, restart=40, rtol=1e-6, maxit=500):
        b2, one = self._cols(b)
        x = np.zeros_like(b2, order="F")
        its = np.zeros(b2.shape[1], np.int32)
        rel = np.zeros(2 * b2.shape[1])
        st = _lib.orc_gmres(self._h, b2.shape[1], _p(b2), _p(x), int(restart), float(rtol), int(maxit),
                            _p(its), _p(rel))
        info = dict(status=st, its=its, relres=rel[0::2], relres_true=rel[1::2])
        return (x[:, 0] if one else x), info
