"""Seeded synthetic inputs for the DDLR preconditioner.

This module produces the *inputs* of the method only: symmetric sparse matrices
in CSR form (the model problems of the numerical-experiments section: the
5-point / 7-point finite-difference Laplacians of the model PDE, optionally
shifted to become indefinite, plus random-coefficient diffusion and 27-point
stand-ins for the general sparse SPD class), geometric box partitions standing
in for the external graph partitioner of the background section, right-hand
sides b = A x* with seeded x*, and Lanczos start vectors.

It holds none of the preconditioner's arithmetic (no splitting, factorization,
Lanczos, low-rank correction or Krylov step). Both the CPU oracle and the HIP
library take what it returns as plain arrays.

Random numbers come from a counter-based generator: value i of stream `stream`
under seed `seed` is a pure function of (seed, stream, i), built on the
SplitMix64 finaliser of Steele, Lea and Flood ("Fast splittable pseudorandom
number generators", OOPSLA 2014), so any element can be regenerated alone.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "uniform", "uniform_pm1", "laplacian_2d", "laplacian_3d",
    "tpfa_2d", "random27_3d", "box_partition", "shift_with_negatives",
    "rhs_from_solution", "lanczos_start", "config",
]

_M64 = (1 << 64) - 1
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (variant 13 of Stafford's mixers)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


def _stream_key(seed: int, stream: str) -> np.uint64:
    h = 1469598103934665603  # FNV-1a 64 over the stream name
    for ch in stream.encode():
        h = ((h ^ ch) * 1099511628211) & _M64
    return _mix64(np.uint64((seed * 0x9E3779B97F4A7C15 + h) & _M64))


def uniform(seed: int, stream: str, idx) -> np.ndarray:
    """Counter-based uniform [0,1) doubles: u(seed, stream, i), top 53 bits."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = _stream_key(seed, stream)
    with np.errstate(over="ignore"):
        z = _mix64(key + (idx + np.uint64(1)) * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm1(seed: int, stream: str, n: int) -> np.ndarray:
    """n values uniform in [-1, 1)."""
    return 2.0 * uniform(seed, stream, np.arange(n, dtype=np.uint64)) - 1.0


@dataclass
class CSR:
    """Symmetric sparse matrix, full storage, 0-based, sorted columns."""
    n: int
    rowptr: np.ndarray  # int64, n+1
    col: np.ndarray     # int32, nnz
    val: np.ndarray     # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.col] = self.val
        return d

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.to_scipy() @ x


def _from_triplets(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n, rowptr, cols.astype(np.int32), vals.astype(np.float64))


def _grid_stencil(dims, offsets, offdiag_fn, diag_fn) -> CSR:
    """Assemble a stencil matrix on a lexicographic grid (x fastest).

    offsets: list of integer offset tuples (excluding the zero offset), closed
    under negation. offdiag_fn(idx_a, idx_b, k) returns the value of the coupling
    a_{ab} for the pair (a, a+offset_k); diag_fn(sum_abs_offdiag, n_missing)
    returns the diagonal.
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    coords = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]  # coords[d][i]
    strides = np.cumprod((1,) + dims[:-1])
    idx = np.arange(n, dtype=np.int64)
    rows_l, cols_l, vals_l = [], [], []
    absum = np.zeros(n)
    missing = np.zeros(n, dtype=np.int64)
    for k, off in enumerate(offsets):
        ok = np.ones(n, dtype=bool)
        for d, o in enumerate(off):
            c = coords[d] + o
            ok &= (c >= 0) & (c < dims[d])
        nb = idx + int(np.dot(off, strides))
        a = idx[ok]
        b = nb[ok]
        v = offdiag_fn(a, b, k)
        rows_l.append(a)
        cols_l.append(b)
        vals_l.append(v)
        np.add.at(absum, a, np.abs(v))
        missing += ~ok
    diag = diag_fn(absum, missing)
    rows_l.append(idx)
    cols_l.append(idx)
    vals_l.append(diag)
    return _from_triplets(n, np.concatenate(rows_l), np.concatenate(cols_l), np.concatenate(vals_l))


def laplacian_2d(nx: int, ny: int) -> CSR:
    """5-point centred-difference Laplacian, Dirichlet, unscaled (4 / -1)."""
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    return _grid_stencil((nx, ny), offs, lambda a, b, k: -np.ones(a.size),
                         lambda s, m: np.full(s.size, 4.0))


def laplacian_3d(nx: int, ny: int, nz: int, shift: float = 0.0) -> CSR:
    """7-point centred-difference Laplacian, Dirichlet, unscaled (6 / -1), minus shift*I."""
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return _grid_stencil((nx, ny, nz), offs, lambda a, b, k: -np.ones(a.size),
                         lambda s, m: np.full(s.size, 6.0 - shift))


def shift_with_negatives(nx: int, ny: int, nz: int, count: int = 20) -> float:
    """Shift sigma for which the 7-point Laplacian minus sigma*I has exactly
    `count` negative eigenvalues: the midpoint of its count-th and (count+1)-th
    smallest eigenvalues, from the closed form sum_d 4 sin^2(j_d pi / (2(N_d+1)))."""
    lim = count + 2
    ev = []
    for jx, jy, jz in itertools.product(range(1, min(nx, lim) + 1), range(1, min(ny, lim) + 1),
                                        range(1, min(nz, lim) + 1)):
        ev.append(4 * math.sin(jx * math.pi / (2 * (nx + 1))) ** 2
                  + 4 * math.sin(jy * math.pi / (2 * (ny + 1))) ** 2
                  + 4 * math.sin(jz * math.pi / (2 * (nz + 1))) ** 2)
    ev.sort()
    return 0.5 * (ev[count - 1] + ev[count])


def tpfa_2d(nx: int, ny: int, seed: int) -> CSR:
    """Cell-centred two-point-flux diffusion on an nx-by-ny grid.

    Cell coefficients kappa = 10^U(-2,2); interior faces carry the harmonic mean
    2 k_a k_b / (k_a + k_b); Dirichlet boundary faces carry 2 kappa (half-cell
    distance). a_ij = -T_ij, a_ii = sum of the cell's face transmissibilities.
    """
    n = nx * ny
    kap = 10.0 ** (4.0 * uniform(seed, "kappa", np.arange(n, dtype=np.uint64)) - 2.0)
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]

    def off(a, b, k):
        return -2.0 * kap[a] * kap[b] / (kap[a] + kap[b])

    def diag(s, m):
        return s + 2.0 * kap * m
    return _grid_stencil((nx, ny), offs, off, diag)


def random27_3d(nx: int, ny: int, nz: int, seed: int) -> CSR:
    """27-point random-coefficient SPD M-matrix: a_ij = -U[0,1) per unordered pair,
    a_ii = sum_j |a_ij| + 0.5 per stencil neighbour slot that falls off the grid."""
    offs = [o for o in itertools.product((-1, 0, 1), repeat=3) if o != (0, 0, 0)]

    def off(a, b, k):
        lo = np.minimum(a, b).astype(np.uint64)
        hi = np.maximum(a, b).astype(np.uint64)
        n = np.uint64(nx * ny * nz)
        return -uniform(seed, "pair27", lo * n + hi)

    def diag(s, m):
        return s + 0.5 * m
    return _grid_stencil((nx, ny, nz), offs, off, diag)


def _split(N: int, P: int) -> np.ndarray:
    """Part index of each of N points when an axis is cut into P parts, the first
    N mod P parts one point larger."""
    base, rem = divmod(N, P)
    sizes = [base + (1 if i < rem else 0) for i in range(P)]
    return np.repeat(np.arange(P), sizes)


def box_partition(dims, parts) -> np.ndarray:
    """Geometric box partition of a lexicographic grid (x fastest).

    Subdomain id = bx + px*(by + py*bz). Returns int32 part[n]."""
    dims = tuple(int(d) for d in dims)
    parts = tuple(int(q) for q in parts)
    labels = [_split(N, P) for N, P in zip(dims, parts)]
    if len(dims) == 2:
        bx, by = np.meshgrid(labels[0], labels[1], indexing="xy")
        part = bx + parts[0] * by
    else:
        bz3, by3, bx3 = np.meshgrid(labels[2], labels[1], labels[0], indexing="ij")
        part = bx3 + parts[0] * (by3 + parts[1] * bz3)
    return np.ascontiguousarray(part.reshape(-1).astype(np.int32))


def rhs_from_solution(A: CSR, seed: int, nrhs: int = 1):
    """x* uniform[-1,1) (stream 'xstar', one seed per right-hand side), b = A x*.

    Returns (b, xstar) as (n, nrhs) Fortran-ordered arrays."""
    xs = np.empty((A.n, nrhs), order="F")
    for r in range(nrhs):
        xs[:, r] = uniform_pm1(seed + r, "xstar", A.n)
    b = np.asfortranarray(A.to_scipy() @ xs)
    return b, xs


def lanczos_start(n: int, seed: int = 0) -> np.ndarray:
    """Length-n vector in user row order, uniform[-1,1) (stream 'lanczos'); its
    entries at interface rows form the Lanczos start vector."""
    return uniform_pm1(seed, "lanczos", n)


def config(name: str) -> dict:
    """The model-problem configurations used by tests and the benchmark.

    c1: 5-point 64x64, 2x2 boxes, DDLR-1 k=8, 16 Lanczos steps.
    c2: 7-point 128^3, 4x4x4 boxes, k=32, 64 Lanczos steps, 8 right-hand sides.
    c3: 7-point 100^3 shifted to have 20 negative eigenvalues, 4x4x8 boxes,
        k=64, 128 Lanczos steps, GMRES(40).
    small2d / small3d: reduced versions used by parity tests.
    """
    if name == "c1":
        A = laplacian_2d(64, 64)
        return dict(A=A, part=box_partition((64, 64), (2, 2)), p=4, k=8, m=16, nrhs=1,
                    dims=(64, 64), variant=1, method="cg")
    if name == "c2":
        A = laplacian_3d(128, 128, 128)
        return dict(A=A, part=box_partition((128,) * 3, (4, 4, 4)), p=64, k=32, m=64, nrhs=8,
                    dims=(128,) * 3, variant=1, method="cg")
    if name == "c3":
        sig = shift_with_negatives(100, 100, 100, 20)
        A = laplacian_3d(100, 100, 100, shift=sig)
        return dict(A=A, part=box_partition((100,) * 3, (4, 4, 8)), p=128, k=64, m=128, nrhs=1,
                    dims=(100,) * 3, variant=1, method="gmres", sigma=sig)
    if name == "small2d":
        A = laplacian_2d(40, 36)
        return dict(A=A, part=box_partition((40, 36), (3, 2)), p=6, k=6, m=14, nrhs=3,
                    dims=(40, 36), variant=1, method="cg")
    if name == "small3d":
        A = laplacian_3d(18, 17, 16)
        return dict(A=A, part=box_partition((18, 17, 16), (2, 3, 2)), p=12, k=10, m=24, nrhs=4,
                    dims=(18, 17, 16), variant=1, method="cg")
    raise KeyError(name)


def _draw_int(seed: int, stream: str, idx: int, lo: int, hi: int) -> int:
    """Integer uniform on {lo..hi} from the counter-based generator."""
    u = float(uniform(seed, stream, np.array([idx], dtype=np.uint64))[0])
    return lo + min(int(u * (hi - lo + 1)), hi - lo)


def batch_systems(count: int = 256, seed: int = 0, side_lo: int = 32, side_hi: int = 256) -> list:
    """Batch of independent SPD 2-D diffusion systems (cell-centred two-point
    flux, per-cell log-uniform coefficients).  System i: grid sides Nx, Ny
    uniform on {side_lo..side_hi}, box split px x py with px, py uniform on
    {2,3,4}, coefficients from seed + i, rank 16 from 32 Lanczos steps."""
    out = []
    for i in range(count):
        nx = _draw_int(seed, "batch_nx", i, side_lo, side_hi)
        ny = _draw_int(seed, "batch_ny", i, side_lo, side_hi)
        px = _draw_int(seed, "batch_px", i, 2, 4)
        py = _draw_int(seed, "batch_py", i, 2, 4)
        A = tpfa_2d(nx, ny, seed + i)
        out.append(dict(A=A, part=box_partition((nx, ny), (px, py)), p=px * py, k=16, m=32, dims=(nx, ny),
                        seed=seed + i))
    return out


def rgg_laplacian(n: int, degree: float, seed: int) -> tuple:
    """Random geometric graph Laplacian, an unstructured SPD M-matrix: n points
    uniform in the unit cube (counter-based, stream "rgg"), numbered along a
    Morton curve, joined when closer than r with n (4/3) pi r^3 = degree;
    a_ij = -w_ij with w_ij uniform in [0.5, 1.5) per pair (stream "rggw"),
    a_ii = sum_j w_ij + 0.01.  Returns (CSR, points)."""
    from scipy.spatial import cKDTree
    idx = np.arange(3 * n, dtype=np.uint64)
    P = uniform(seed, "rgg", idx).reshape(n, 3)
    # Morton order (10 bits per axis) for a locality-preserving numbering
    q = np.minimum((P * 1024).astype(np.uint64), np.uint64(1023))
    code = np.zeros(n, dtype=np.uint64)
    for b in range(10):
        for d in range(3):
            code |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    P = P[np.argsort(code, kind="stable")]
    r = (3.0 * degree / (4.0 * np.pi * n)) ** (1.0 / 3.0)
    pairs = cKDTree(P).query_pairs(r, output_type="ndarray").astype(np.int64)
    lo, hi = np.minimum(pairs[:, 0], pairs[:, 1]), np.maximum(pairs[:, 0], pairs[:, 1])
    wgt = 0.5 + uniform(seed, "rggw", (lo * n + hi).astype(np.uint64))
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    dsum = np.bincount(lo, wgt, n) + np.bincount(hi, wgt, n)
    vals = np.concatenate([-wgt, -wgt, dsum + 0.01])
    return _from_triplets(n, rows, cols, vals), P


# resident matrices of the serving stream: grid side, box split, rank
SERVING_MATRICES = ((37, (2, 2, 4), 32), (46, (2, 2, 4), 32), (55, (2, 4, 4), 40), (64, (2, 4, 4), 40),
                    (73, (4, 4, 4), 48), (82, (4, 4, 4), 48), (91, (4, 4, 8), 64), (100, (4, 4, 8), 64))


def serving_matrix(j: int, seed: int = 0) -> dict:
    """Matrix j of the serving stream: 27-point random-coefficient SPD
    M-matrix on an N^3 grid, N^3 from 50,653 to 10^6, 16..128 box
    subdomains, rank 32..64 from 2k Lanczos steps."""
    N, parts, k = SERVING_MATRICES[j]
    A = random27_3d(N, N, N, seed + j)
    p = parts[0] * parts[1] * parts[2]
    return dict(A=A, part=box_partition((N, N, N), parts), p=p, k=k, m=2 * k, dims=(N, N, N), seed=seed + j)
