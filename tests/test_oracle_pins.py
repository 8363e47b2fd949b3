"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each checks a property the
method must have (an identity, a theorem, a defining property, a brute-force
definition on a tiny input, a closed form), chosen so that a dropped term, a
wrong sign, a wrong index or a transposed operand in the oracle breaks one.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as w
from oracle import (CORDER_NATURAL, E_BREAKDOWN, E_INVALID, E_NO_CONVERGENCE, E_NOT_SYMMETRIC, FACTOR_EXACT,
                    FACTOR_ILDL, Oracle, OracleError)

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ helpers

def geometric_interface(part, dims, diagonal=False):
    """Interface flags from the grid geometry: a point is an interface point iff
    one of its stencil neighbours lies in another box (edge separator, Sec. 2.1)."""
    g = part.reshape(dims[::-1])
    flag = np.zeros(g.shape, dtype=bool)
    nd = g.ndim
    if diagonal:
        offs = [o for o in np.ndindex(*(3,) * nd) if o != (1,) * nd]
        offs = [tuple(x - 1 for x in o) for o in offs]
    else:
        offs = []
        for d in range(nd):
            for s in (-1, 1):
                o = [0] * nd
                o[d] = s
                offs.append(tuple(o))
    for o in offs:
        src = tuple(slice(max(0, -x), g.shape[d] - max(0, x)) for d, x in enumerate(o))
        dst = tuple(slice(max(0, x), g.shape[d] - max(0, -x)) for d, x in enumerate(o))
        flag[src] |= g[src] != g[dst]
    return flag.reshape(-1)


def user_A0_E(o):
    """A0 and E as dense arrays in internal order."""
    return o.csr("A0").toarray(), o.csr("E").toarray()


def dense_H(o, power=1):
    A0, E = user_A0_E(o)
    X = np.linalg.solve(A0, E)
    if power == 2:
        X = np.linalg.solve(A0, X)
    return E.T @ X


def ldl_dense(o):
    L = o.csr("L").toarray() + np.eye(o.n)
    return L @ np.diag(o.diag()) @ L.T


def tiny_irregular(seed=3):
    """Random-coefficient diffusion on 12x10 with an uneven 2x2 split: no
    symmetry, so the spectra below are simple."""
    A = w.tpfa_2d(12, 10, seed)
    part = w.box_partition((12, 10), (2, 2))
    return A, part, 4


# ------------------------------------------------------ inputs (generators)

def test_laplacian_closed_form_spectrum():
    A = w.laplacian_3d(5, 4, 3)
    ev = np.sort(np.linalg.eigvalsh(A.to_dense()))
    ref = np.sort([4 * np.sin(i * np.pi / 12) ** 2 + 4 * np.sin(j * np.pi / 10) ** 2 + 4 * np.sin(k * np.pi / 8) ** 2
                   for i in range(1, 6) for j in range(1, 5) for k in range(1, 4)])
    assert np.allclose(ev, ref, atol=1e-12)


def test_shift_gives_twenty_negative_eigenvalues():
    sig = w.shift_with_negatives(10, 10, 10, 20)
    ev = np.linalg.eigvalsh(w.laplacian_3d(10, 10, 10, shift=sig).to_dense())
    assert (ev < 0).sum() == 20


def test_generated_matrices_symmetric_and_spd():
    for A in (w.tpfa_2d(9, 7, 1), w.random27_3d(5, 4, 3, 2), w.laplacian_2d(6, 5)):
        d = A.to_dense()
        assert np.array_equal(d, d.T)
        assert np.linalg.eigvalsh(d).min() > 0


# --------------------------------------------------- ordering (Sec. 2.1-2.2)

@pytest.mark.parametrize("dims,parts,stencil", [((13, 11), (3, 2), "5"), ((7, 6, 5), (2, 2, 2), "7"),
                                               ((6, 5, 4), (2, 2, 1), "27")])
def test_classification_and_natural_order_bruteforce(dims, parts, stencil):
    if stencil == "5":
        A = w.laplacian_2d(*dims)
    elif stencil == "7":
        A = w.laplacian_3d(*dims)
    else:
        A = w.random27_3d(*dims, seed=4)
    part = w.box_partition(dims, parts)
    p = int(np.prod(parts))
    o = Oracle(A, part, p, corder=CORDER_NATURAL)
    perm, iface, colour, boff = o.ordering()
    geo = geometric_interface(part, dims, diagonal=(stencil == "27"))
    assert np.array_equal(iface.astype(bool), geo)
    expect = [np.flatnonzero((part == b) & ~geo) for b in range(p)]
    expect += [np.flatnonzero((part == b) & geo) for b in range(p)]
    assert np.array_equal(perm, np.concatenate(expect))
    assert boff[p] == (~geo).sum() and boff[p + 1] == A.n
    assert np.array_equal(np.diff(boff[: p + 1]), [len(e) for e in expect[:p]])


def test_greedy_colouring_bruteforce():
    A = w.random27_3d(6, 5, 4, seed=5)
    dims, parts = (6, 5, 4), (2, 2, 1)
    part = w.box_partition(dims, parts)
    o_nat = Oracle(A, part, 4, corder=CORDER_NATURAL)
    o = Oracle(A, part, 4)
    perm_nat, _, _, _ = o_nat.ordering()
    perm, _, colour, _ = o.ordering()
    m = o.m
    nat = list(perm_nat[m:])
    Ad = A.to_dense()
    # greedy in natural interface order: smallest colour unused by coloured neighbours
    col = {}
    for u in nat:
        used = {col[v] for v in nat if v in col and v != u and Ad[u, v] != 0}
        c = 0
        while c in used:
            c += 1
        col[u] = c
    expect = sorted(nat, key=lambda u: (col[u], nat.index(u)))
    assert list(perm[m:]) == expect
    assert list(colour) == [col[u] for u in expect]
    assert o.ncolours == max(col.values()) + 1


def test_structure_counts_c1():
    c = w.config("c1")
    o = Oracle(c["A"], c["part"], c["p"])
    assert (o.m, o.s, o.ncolours) == (3844, 252, 2)
    L = o.csr("L")
    perm, _, _, boff = o.ordering()
    nnzB = L[: o.m].nnz
    assert (nnzB, L.nnz - nnzB) == (7440, 376)


@pytest.mark.slow
def test_structure_counts_c2():
    c = w.config("c2")
    o = Oracle(c["A"], c["part"], c["p"])
    assert (o.n, o.s, o.ncolours) == (2097152, 281304, 2)
    L = o.csr("L")
    nnzB = L[: o.m].nnz
    assert (nnzB, L.nnz - nnzB) == (5268936, 705456)


# ------------------------------------------------------ splitting (Sec. 3.1)

@pytest.mark.parametrize("alpha", [1.0, 2.0, 0.5])
@pytest.mark.parametrize("kind", ["lap2", "lap3", "r27"])
def test_splitting_identity(alpha, kind):
    if kind == "lap2":
        A, part, p = w.laplacian_2d(11, 9), w.box_partition((11, 9), (2, 2)), 4
    elif kind == "lap3":
        A, part, p = w.laplacian_3d(6, 5, 4), w.box_partition((6, 5, 4), (2, 1, 2)), 4
    else:
        A, part, p = w.random27_3d(6, 5, 4, 7), w.box_partition((6, 5, 4), (2, 2, 1)), 4
    o = Oracle(A, part, p, alpha=alpha)
    perm, _, _, boff = o.ordering()
    PAP = o.csr("PAP").toarray()
    assert np.array_equal(PAP, A.to_dense()[np.ix_(perm, perm)])
    A0, E = user_A0_E(o)
    diff = np.abs(A0 - E @ E.T - PAP).max()  # eq. (split): A = A0 - E E^T
    assert diff <= (0.0 if kind != "r27" else 1e-15 * np.abs(A0).max())
    # E = [alpha^{-1} Ehat ; -alpha I]  (eq. EF)
    assert np.array_equal(E[o.m:], -alpha * np.eye(o.s))
    # A0 is block diagonal over the p interior blocks and the interface block
    # (Proposition: Ehat Ehat^T has no inter-domain blocks)
    mask = np.zeros_like(A0, dtype=bool)
    for b in range(p + 1):
        mask[boff[b]:boff[b + 1], boff[b]:boff[b + 1]] = True
    assert not np.any(A0[~mask])


# ----------------------------------------------- local factorisation (Sec. 5)

@pytest.mark.parametrize("kind", ["lap3", "r27", "tpfa"])
def test_incomplete_ldl_defining_property(kind):
    """IC(0)/LDL(0): (L D L^T)_ij = a_ij on the pattern of A0, L has A0's strict
    lower pattern (the zero-fill incomplete factorisation, Saad's ILU(0))."""
    if kind == "lap3":
        A, part, p = w.laplacian_3d(7, 6, 5), w.box_partition((7, 6, 5), (2, 2, 2)), 8
    elif kind == "r27":
        A, part, p = w.random27_3d(6, 5, 4, 8), w.box_partition((6, 5, 4), (2, 2, 1)), 4
    else:
        A, part, p = tiny_irregular()
    o = Oracle(A, part, p, alpha=2.0 if kind == "r27" else 1.0)
    A0 = o.csr("A0").toarray()
    L = o.csr("L").toarray()
    assert np.array_equal(L != 0, np.tril(A0 != 0, -1)) or np.all((L != 0) <= np.tril(A0 != 0, -1))
    assert o.csr("L").nnz == np.count_nonzero(np.tril(A0 != 0, -1))
    LDL = ldl_dense(o)
    pat = A0 != 0
    assert np.abs(LDL - A0)[pat].max() <= 1e-12 * np.abs(A0).max()
    assert np.all(o.diag() > 0)


def test_ic0_exact_on_chains():
    """On a 1-D chain IC(0) has no fill to drop, so it is the exact LDL^T."""
    n = 40
    d = np.full(n, 2.5)
    rows = np.r_[np.arange(n), np.arange(n - 1), np.arange(1, n)]
    cols = np.r_[np.arange(n), np.arange(1, n), np.arange(n - 1)]
    vals = np.r_[d, -np.ones(n - 1), -np.ones(n - 1)]
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    M.sort_indices()
    A = w.CSR(n, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)
    part = np.repeat(np.arange(4), 10).astype(np.int32)
    o = Oracle(A, part, 4, corder=CORDER_NATURAL)
    A0, _ = user_A0_E(o)
    x = np.random.default_rng(0).standard_normal(n)
    perm, *_ = o.ordering()
    z = o.a0_solve(x)
    zi = np.linalg.solve(A0, x[perm])
    assert np.allclose(z[perm], zi, rtol=1e-13, atol=1e-13)


def test_a0_solve_matches_factors_and_exact():
    A, part, p = w.random27_3d(5, 5, 4, 9), w.box_partition((5, 5, 4), (2, 2, 1)), 4
    x = np.random.default_rng(1).standard_normal((A.n, 2))
    o = Oracle(A, part, p, alpha=2.0)
    perm, *_ = o.ordering()
    z = o.a0_solve(x)
    ref = np.linalg.solve(ldl_dense(o), x[perm])
    assert np.allclose(z[perm], ref, rtol=1e-12, atol=1e-12)
    oe = Oracle(A, part, p, alpha=2.0, factor=FACTOR_EXACT)
    A0, _ = user_A0_E(oe)
    ze = oe.a0_solve(x)
    assert np.allclose(ze[perm], np.linalg.solve(A0, x[perm]), rtol=1e-11, atol=1e-12)


def test_breakdown_and_input_errors():
    A = w.laplacian_2d(6, 6)
    part = w.box_partition((6, 6), (2, 2))
    # make one interior pivot negative: a_ii = -3 for an interior point of box 0
    d = A.to_dense()
    d[7, 7] = -3.0
    M = sp.csr_matrix(d)
    M.sort_indices()
    B = w.CSR(36, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)
    with pytest.raises(OracleError) as e:
        Oracle(B, part, 4)
    assert e.value.status == E_BREAKDOWN
    ob = Oracle(B, part, 4, factor=FACTOR_ILDL)  # nonzero pivots: accepted
    ob.lowrank(1, 2, 6, w.lanczos_start(36, 0))
    assert np.any(ob.diag() < 0) and not ob.spd  # indefinite local factor: never certified SPD
    d2 = A.to_dense()
    d2[0, 1] = -2.0
    M2 = sp.csr_matrix(d2)
    M2.sort_indices()
    with pytest.raises(OracleError) as e:
        Oracle(w.CSR(36, M2.indptr.astype(np.int64), M2.indices.astype(np.int32), M2.data), part, 4)
    assert e.value.status == E_NOT_SYMMETRIC
    bad = part.copy()
    bad[3] = 9
    with pytest.raises(OracleError) as e:
        Oracle(A, bad, 4)
    assert e.value.status == E_INVALID


# ---------------------------------------------------------- Lanczos (Sec. 4.4 (sec:Lan))

@pytest.mark.parametrize("variant", [1, 2])
def test_lanczos_relations(variant):
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p)
    m = 12
    o.lowrank(variant, 4, m, w.lanczos_start(A.n, 2))
    ta, tb, rz = o.lanczos_record()
    Q = o.lanczos_basis()
    H = dense_H(o_ic_dense(o), power=variant)
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 1e-12
    T = np.diag(ta) + np.diag(tb[:-1], 1) + np.diag(tb[:-1], -1)
    R = H @ Q - Q @ T
    scale = np.abs(H).max()
    assert np.abs(R[:, :-1]).max() <= 1e-11 * scale
    assert abs(np.linalg.norm(R[:, -1]) - tb[-1]) <= 1e-11 * scale
    assert np.allclose(np.sort(rz), np.linalg.eigvalsh(T), atol=1e-13)
    assert np.all(np.diff(rz) <= 0)


def o_ic_dense(o):
    """A stand-in with the oracle's incomplete factors as 'A0' (dense)."""
    class _V:
        pass
    v = _V()
    LDL = ldl_dense(o)
    E = o.csr("E").toarray()
    v.csr = lambda which: sp.csr_matrix(LDL) if which == "A0" else sp.csr_matrix(E)
    return v


def test_full_lanczos_recovers_spectrum():
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    H = dense_H(o)
    o.lowrank(1, 5, o.s, w.lanczos_start(A.n, 3))
    _, _, rz = o.lanczos_record()
    ev = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert len(rz) == o.s
    assert np.allclose(rz, ev, atol=1e-9)
    # Lemma (eigenvalues of H): 0 <= lambda < 1 for SPD A
    assert ev.min() > -1e-12 and ev.max() < 1


# ------------------------------------------------------------- DDLR-1 (Sec. 3.2)

def _eigh_desc(H):
    lam, U = np.linalg.eigh(H)
    return lam[::-1], U[:, ::-1]


def _user_rows(o, Uint):
    perm, *_ = o.ordering()
    U = np.zeros((o.n, Uint.shape[1]))
    U[perm[o.m:]] = Uint
    return U


def _dense_minv(o):
    perm, *_ = o.ordering()
    Mi = o.apply(np.eye(o.n))
    return Mi


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_ddlr1_smw_full_rank_is_exact_inverse(theta):
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    lam, U = _eigh_desc(dense_H(o))
    o.set_lowrank(1, _user_rows(o, U), lam, theta)
    Minv = _dense_minv(o)
    Ainv = np.linalg.inv(A.to_dense())
    assert np.abs(Minv - Ainv).max() <= 1e-10 * np.abs(Ainv).max()


def test_ddlr1_gkt_equals_modified_spectrum_form():
    """eq. (gkt) equals (I - U Lambda~ U^T)^{-1} with the full U and Lambda~
    holding lambda_1..lambda_k then theta (Proposition on G_{k,theta})."""
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    A0, E = user_A0_E(o)
    H = dense_H(o)
    lam, U = _eigh_desc(H)
    k, theta = 3, lam[3]
    o.set_lowrank(1, _user_rows(o, U[:, :k]), lam[:k], theta)
    lt = np.r_[lam[:k], np.full(o.s - k, theta)]
    Ginv = np.linalg.inv(np.eye(o.s) - U @ np.diag(lt) @ U.T)
    X = np.linalg.solve(A0, E)
    Mint = np.linalg.inv(A0) + X @ Ginv @ X.T
    perm, *_ = o.ordering()
    Minv = _dense_minv(o)
    assert np.abs(Minv[np.ix_(perm, perm)] - Mint).max() <= 1e-11 * np.abs(Mint).max()


def test_ddlr1_symmetric_with_incomplete_factors():
    c = w.config("small2d")
    o = Oracle(c["A"], c["part"], c["p"])
    o.lowrank(1, c["k"], c["m"], w.lanczos_start(c["A"].n, 0))
    Mi = _dense_minv(o)
    assert np.linalg.norm(Mi - Mi.T) <= 1e-12 * np.linalg.norm(Mi)


def test_ddlr1_spectral_theorem():
    """Theorem (DDLR-1 eigenvalues): 1 <= eta <= 1 + ||A^{1/2} A0^{-1} E||^2/(1-theta),
    with the norm at most 1/4; with theta = 0: m+k unit eigenvalues, the rest in (0,1)."""
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    k = 5
    o.lowrank(1, k, o.s, w.lanczos_start(A.n, 4))
    _, _, theta = o.get_lowrank()
    A0, E = user_A0_E(o)
    perm, *_ = o.ordering()
    PAP = A.to_dense()[np.ix_(perm, perm)]
    X = sl.sqrtm(PAP).real @ np.linalg.solve(A0, E)
    nrm = np.linalg.norm(X, 2) ** 2
    assert nrm <= 0.25 + 1e-12
    ev = np.linalg.eigvals(A.to_dense() @ _dense_minv(o)).real
    assert ev.min() >= 1 - 1e-9
    assert ev.max() <= 1 + nrm / (1 - theta) + 1e-9
    o.lowrank(1, k, o.s, w.lanczos_start(A.n, 4), theta_zero=True)
    ev0 = np.linalg.eigvals(A.to_dense() @ _dense_minv(o)).real
    ones = np.abs(ev0 - 1) <= 1e-8
    assert ones.sum() == o.m + k
    assert np.all((ev0[~ones] > 0) & (ev0[~ones] < 1))


def test_worked_example_relations():
    """Sec. 3.2 worked example (30x30 Laplacian, 4 subdomains, k = 5). The
    paper's partition is not recoverable (119 vs 116 interface points), so the
    printed theta / eigenvalues are parity unpinned; the relations are pinned."""
    g = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    A = w.laplacian_2d(30, 30)
    part = w.box_partition((30, 30), (2, 2))
    for row in g["rows"]:
        paper_bound = 1 + row["norm2"] / (1 - row["theta"])
        assert abs(paper_bound - row["bound"]) <= 5e-4 * row["bound"]   # the paper's own numbers agree
        assert row["max_eig"] <= row["bound"]
        o = Oracle(A, part, 4, alpha=row["alpha"], factor=FACTOR_EXACT)
        assert o.s == 116
        o.lowrank(1, 5, o.s, w.lanczos_start(A.n, 0))
        _, lam, theta = o.get_lowrank()
        A0, E = user_A0_E(o)
        perm, *_ = o.ordering()
        X = sl.sqrtm(A.to_dense()[np.ix_(perm, perm)]).real @ np.linalg.solve(A0, E)
        nrm = np.linalg.norm(X, 2) ** 2
        assert 0.2499 <= nrm <= 0.25 + 1e-12  # "close to 1/4 for Laplacian matrices"
        ev = np.linalg.eigvals(A.to_dense() @ _dense_minv(o)).real
        assert 0.8 < theta < 1.0
        assert 1 - 1e-9 <= ev.min() and ev.max() <= 1 + nrm / (1 - theta) + 1e-9


# ------------------------------------------------------------- DDLR-2 (Sec. 3.3)

def _ddlr2_from_svd(o, k):
    A0, E = user_A0_E(o)
    X = np.linalg.solve(A0, E)
    _, sv, Vt = np.linalg.svd(X, full_matrices=False)
    V = Vt.T[:, :k]
    Uk = X @ V
    Hk = np.linalg.inv(np.eye(k) - Uk.T @ E @ V)
    return Uk, Hk, sv


def test_ddlr2_full_rank_is_exact_inverse():
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    Uk, Hk, _ = _ddlr2_from_svd(o, o.s)
    perm, *_ = o.ordering()
    U = np.zeros((o.n, o.s))
    U[perm] = Uk
    o.set_lowrank(2, U, Hk)
    Ainv = np.linalg.inv(A.to_dense())
    assert np.abs(_dense_minv(o) - Ainv).max() <= 1e-10 * np.abs(Ainv).max()


def test_ddlr2_build_and_spectral_theorem():
    """Theorem (DDLR-2 eigenvalues): 0 < eta <= 1 with n-s+k unit eigenvalues;
    the built U_k H_k U_k^T equals the one from the SVD of A0^{-1}E (eq. LR,
    Lemma on H_k), which is invariant to the signs of the singular vectors."""
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    k = 4
    o.lowrank(2, k, o.s, w.lanczos_start(A.n, 5))
    U, Hk = o.get_lowrank()
    Uk_ref, Hk_ref, sv = _ddlr2_from_svd(o, k)
    assert sv[k - 1] - sv[k] > 1e-6
    perm, *_ = o.ordering()
    C_or = (U @ Hk @ U.T)[np.ix_(perm, perm)]
    C_ref = Uk_ref @ Hk_ref @ Uk_ref.T
    assert np.abs(C_or - C_ref).max() <= 1e-9 * np.abs(C_ref).max()
    assert np.allclose(Hk, Hk.T, atol=1e-12)
    ev = np.linalg.eigvals(A.to_dense() @ _dense_minv(o)).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-9
    assert (np.abs(ev - 1) <= 1e-8).sum() == o.n - o.s + k


# ------------------------------------------------------------ Krylov (Sec. 5)

def test_pcg_one_step_with_exact_preconditioner():
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    lam, U = _eigh_desc(dense_H(o))
    o.set_lowrank(1, _user_rows(o, U), lam, 0.0)
    b, _ = w.rhs_from_solution(A, 0, 1)
    x, info = o.pcg(b)
    assert info["its"][0] == 1 and info["relres_true"][0] <= 1e-12


def test_pcg_c1_end_to_end():
    c = w.config("c1")
    A = c["A"]
    o = Oracle(A, c["part"], c["p"])
    o.lowrank(1, c["k"], c["m"], w.lanczos_start(A.n, 0))
    assert o.spd
    b, xs = w.rhs_from_solution(A, 0, 1)
    x, info = o.pcg(b)
    assert info["status"] == 0
    assert info["relres"][0] <= 1e-6 and info["relres_true"][0] <= 1.01e-6
    ref = spla.spsolve(A.to_scipy().tocsc(), b[:, 0])
    assert np.linalg.norm(x[:, 0] - ref) <= 1e-3 * np.linalg.norm(ref)
    # trend of the tables: DDLR-1 needs fewer iterations than DDLR-2 at equal k
    o2 = Oracle(A, c["part"], c["p"])
    o2.lowrank(2, c["k"], c["m"], w.lanczos_start(A.n, 0))
    _, info2 = o2.pcg(b)
    assert info["its"][0] < info2["its"][0]
    # maximum iterations reached -> no-convergence status, x still written
    x1, info1 = o.pcg(b, maxit=1)
    assert info1["status"] == E_NO_CONVERGENCE and info1["its"][0] == 1 and np.any(x1 != 0)


def test_gmres_indefinite():
    sig = 0.1
    A = w.laplacian_2d(24, 20)
    d = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    d[rows == A.col] -= sig
    A = w.CSR(A.n, A.rowptr, A.col, d)
    assert (np.linalg.eigvalsh(A.to_dense()) < 0).sum() > 0
    part = w.box_partition((24, 20), (2, 2))
    o = Oracle(A, part, 4, factor=FACTOR_ILDL)
    o.lowrank(1, 10, 30, w.lanczos_start(A.n, 1))
    assert o.spd  # sigma = 0.1 keeps every local pivot positive here
    ob = Oracle(A.__class__(A.n, A.rowptr, A.col, np.where(rows == A.col, A.val - 0.6, A.val)), part, 4,
                factor=FACTOR_ILDL)
    ob.lowrank(1, 10, 30, w.lanczos_start(A.n, 1))
    assert ob.lanczos_record()[2][0] >= 1 and not ob.spd  # Sec. 5: largest eigenvalue >= 1 -> not SPD
    b, _ = w.rhs_from_solution(A, 0, 2)
    x, info = o.gmres(b, restart=40)
    assert info["status"] == 0
    ref = spla.spsolve(A.to_scipy().tocsc(), b)
    assert np.all(info["relres_true"] <= 2e-6)
    assert np.linalg.norm(x - ref) <= 1e-4 * np.linalg.norm(ref)
    # exact preconditioner: one step
    oe = Oracle(A, part, 4, factor=FACTOR_EXACT)
    lam, U = _eigh_desc(dense_H(oe))
    oe.set_lowrank(1, _user_rows(oe, U), lam, 0.0)
    _, info_e = oe.gmres(b[:, 0])
    assert info_e["its"][0] == 1


# ------------------------------------------- Lanczos control and rank extension
def _sigma(ta, tb, j, k):
    """Sum of the k largest eigenvalues of the leading j x j block of T (LAPACK)."""
    T = np.diag(ta[:j]) + np.diag(tb[: j - 1], 1) + np.diag(tb[: j - 1], -1)
    return float(np.sort(np.linalg.eigvalsh(T))[::-1][:k].sum())


@pytest.mark.parametrize("variant", [1, 2])
def test_lanczos_convergence_rule(variant):
    """Sec. 5 / eq. (converge): checked every 10 steps, the run stops at the
    first multiple m of 10 (m >= k+1) with |sigma_m - sigma_{m-1}| <
    eps |sigma_{m-1}|, sigma_j = sum of the k largest Ritz values of T_j.
    The stopping step is re-derived from the recorded T with LAPACK."""
    cfg = w.config("small3d")
    k, eps, mmax = 10, 1e-4, 5 * 10
    o = Oracle(cfg["A"], cfg["part"], cfg["p"])
    o.lowrank(variant, k, mmax, w.lanczos_start(cfg["A"].n, 0), check=10, eps=eps)
    ta, tb, _ = o.lanczos_record()
    m = o.msteps
    assert m % 10 == 0 or m == mmax
    for j in range(10, m + 1, 10):
        if j < k + 1:
            continue
        sp, sm = _sigma(ta, tb, j - 1, k), _sigma(ta, tb, j, k)
        hit = abs((sm - sp) / sp) < eps
        assert hit == (j == m) or (j == m == mmax), (j, m)
    # eps extremes: a huge tolerance stops at the first check past k; zero runs to the cap
    o.lowrank(variant, k, mmax, w.lanczos_start(cfg["A"].n, 0), check=10, eps=10.0)
    assert o.msteps == 20
    o.lowrank(variant, k, mmax, w.lanczos_start(cfg["A"].n, 0), check=10, eps=0.0)
    assert o.msteps == mmax


@pytest.mark.parametrize("variant", [1, 2])
def test_extend_equals_direct_run(variant):
    """Improving a given preconditioner: continuing the stored Lanczos run and
    rebuilding with a larger k gives exactly the preconditioner built from a
    single run of the combined length (the steps are the same operations)."""
    cfg = w.config("small3d")
    v0 = w.lanczos_start(cfg["A"].n, 0)
    a = Oracle(cfg["A"], cfg["part"], cfg["p"]).lowrank(variant, 6, 16, v0)
    a.extend(10, 12)
    b = Oracle(cfg["A"], cfg["part"], cfg["p"]).lowrank(variant, 10, 28, v0)
    assert a.msteps == b.msteps == 28
    for x, y in zip(a.lanczos_record(), b.lanczos_record()):
        assert np.array_equal(x, y)
    for x, y in zip(a.get_lowrank(), b.get_lowrank()):
        assert np.array_equal(np.asarray(x), np.asarray(y))


# ------------------------------------------------------------ graph partitioner
def _path(n):
    rows = np.concatenate([np.arange(n - 1), np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(1, n), np.arange(n - 1), np.arange(n)])
    return w._from_triplets(n, rows, cols, np.ones(len(rows)))


def _expected_sizes(n, p):
    """Part sizes of the recursive bisection depend only on (n, p)."""
    if p == 1:
        return [n]
    q1 = p // 2
    t = (n * q1 * 2 + p) // (2 * p)
    return _expected_sizes(t, q1) + _expected_sizes(n - t, p - q1)


def test_partition_path_graph_by_hand():
    from oracle.partition import partition_graph
    # path 0-1-...-8: BFS from the end vertex 0 visits 0..8 in order; 3 parts of 3
    assert partition_graph(_path(9), 3).tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2]
    # path numbered from the middle: the pseudo-peripheral search moves to an end
    n = 7
    perm = np.array([3, 2, 4, 1, 5, 0, 6])  # vertex i sits at position perm[i] on the line
    pos = np.empty(n, int)
    pos[perm] = np.arange(n)
    rows, cols = [], []
    for a in range(n - 1):
        u, v = pos[a], pos[a + 1]
        rows += [u, v]
        cols += [v, u]
    A = w._from_triplets(n, np.array(rows + list(range(n))), np.array(cols + list(range(n))), np.ones(len(rows) + n))
    part = partition_graph(A, 2)
    # halves are contiguous along the line: positions 0..3 in one part (t = 4), 4..6 in the other
    assert len(set(part[pos[:4]])) == 1 and len(set(part[pos[4:]])) == 1 and part[pos[0]] != part[pos[6]]


def test_partition_sizes_and_components():
    from oracle.partition import partition_graph
    A, _ = w.rgg_laplacian(3000, 8, 2)
    for p in (2, 5, 8, 13):
        part = partition_graph(A, p)
        assert sorted(np.bincount(part, minlength=p).tolist()) == sorted(_expected_sizes(A.n, p))
    # two disconnected paths: the component of vertex 0 comes first in the BFS order
    B = w._from_triplets(8, np.array([0, 1, 1, 2, 4, 5, 5, 6, 6, 7] + list(range(8))),
                         np.array([1, 0, 2, 1, 5, 4, 6, 5, 7, 6] + list(range(8))), np.ones(18))
    assert partition_graph(B, 2).tolist() == [0, 0, 0, 0, 1, 1, 1, 1]


# ------------------------------------- C_alpha approximate inverse (Sec. 4.3 (sec:csolve))

def _c_alpha(o):
    """C_alpha = A0[m:, m:] (dense), interface order."""
    return o.csr("A0").toarray()[o.m:, o.m:]


def _ring_matrix():
    """Six unknowns, two parts: interior 0 and 5, interface 1, 2 (part 0) and
    3, 4 (part 1).  The interface unknowns form the cycle 1-2-4-3-1 with -1
    couplings and a_ii = 3, so C_alpha (alpha = 1) has diagonal 4."""
    edges = [(0, 1), (0, 2), (1, 2), (2, 4), (4, 3), (3, 1), (5, 3), (5, 4)]
    n = 6
    rows = [i for i in range(n)] + [a for a, b in edges] + [b for a, b in edges]
    cols = [i for i in range(n)] + [b for a, b in edges] + [a for a, b in edges]
    vals = [3.0] * n + [-1.0] * (2 * len(edges))
    A = w._from_triplets(n, np.array(rows), np.array(cols), np.array(vals))
    part = np.array([0, 0, 0, 1, 1, 1], np.int32)
    return A, part


def test_cinv_one_step_by_hand():
    """Worked by hand from Algorithm alg:mr with the stated dropping rule.
    X_0 = I/4, R_0 = I - C/4 (0.25 on the cycle edges), Z_0 = X_0 R_0 (1/16 on
    the edges), ||z_j|| = sqrt(2)/16.  tol = 0.5 keeps both neighbours of each
    column; lfil = 1 keeps the lower row on the tie: columns keep rows
    (1, 0, 0, 1) for interface positions (0..3) = unknowns (1, 2, 3, 4);
    only the pair {0, 1} survives in both its columns.  Then
    tr(R_0^T C Z) = 1/8, ||C Z||_F^2 = 9/64, beta = 8/9, and
    X_1 = I/4 + (1/18)(e_0 e_1^T + e_1 e_0^T)."""
    A, part = _ring_matrix()
    o = Oracle(A, part, 2, corder=CORDER_NATURAL)
    C = _c_alpha(o)
    assert np.allclose(np.diag(C), 4.0)
    o.use_cinv(nit=1, tol=0.5, lfil=1)
    X, res, spd = o.cinv()
    Xe = np.eye(4) / 4
    Xe[0, 1] = Xe[1, 0] = 1.0 / 18.0
    assert np.abs(X.toarray() - Xe).max() < 1e-16
    assert abs(res[0] - np.sqrt(0.5)) < 1e-15
    assert abs(res[1] - np.linalg.norm(np.eye(4) - C @ Xe)) < 1e-14
    assert spd
    # a tolerance above 1/16 / (sqrt(2)/16) drops every off-diagonal entry: Z = 0, X stays X_0
    o2 = Oracle(A, part, 2, corder=CORDER_NATURAL).use_cinv(nit=3, tol=0.8, lfil=4)
    X2, res2, _ = o2.cinv()
    assert np.array_equal(X2.toarray(), np.eye(4) / 4) and len(res2) == 1


def test_cinv_without_dropping_converges_to_inverse():
    """No dropping: the self-preconditioned MR iterates converge to C_alpha^{-1}
    (checked against LAPACK's inverse) with a non-increasing residual."""
    cfg = w.config("c1")
    o = Oracle(cfg["A"], cfg["part"], cfg["p"]).use_cinv(nit=8, tol=0.0, lfil=10 ** 6)
    X, res, spd = o.cinv()
    Ci = np.linalg.inv(_c_alpha(o))
    assert np.linalg.norm(X.toarray() - Ci) / np.linalg.norm(Ci) < 1e-12
    assert np.all(np.diff(res) <= 1e-15 * res[0]) and res[-1] < 1e-12 and spd
    assert abs(res[0] - np.linalg.norm(np.eye(o.s) - _c_alpha(o) / np.diag(_c_alpha(o))[None, :])) < 1e-12


@pytest.mark.parametrize("nit,tol,lfil", [(3, 0.01, 20), (4, 0.05, 6)])
def test_cinv_dropping_properties(nit, tol, lfil):
    """With dropping: X exactly symmetric; each step adds a symmetric pattern
    with at most lfil off-diagonal entries per column; the residual
    ||I - C X_j||_F never increases (beta is the minimiser over the step)."""
    cfg = w.config("c1")
    C = None
    prev = None
    for j in range(nit + 1):
        o = Oracle(cfg["A"], cfg["part"], cfg["p"]).use_cinv(nit=j, tol=tol, lfil=lfil)
        X, res, spd = o.cinv()
        if C is None:
            C = _c_alpha(o)
        Xd = X.toarray()
        assert np.array_equal(Xd, Xd.T)
        assert abs(res[-1] - np.linalg.norm(np.eye(o.s) - C @ Xd)) < 1e-12 * max(1.0, res[-1])
        if prev is not None:
            D = Xd - prev
            pat = D != 0
            np.fill_diagonal(pat, False)
            assert np.array_equal(pat, pat.T)
            assert pat.sum(axis=0).max() <= lfil
            assert res[-1] <= res[-2] * (1 + 1e-14)
        prev = Xd


def test_cinv_step_is_minimal_residual():
    """beta minimises ||R - beta C Z||_F: the new residual is orthogonal (in
    the trace inner product) to C (X_{j+1} - X_j).  X_j is the j-step result
    (the iteration is deterministic, so shorter runs are prefixes)."""
    cfg = w.config("c1")
    o1 = Oracle(cfg["A"], cfg["part"], cfg["p"]).use_cinv(nit=1, tol=0.01, lfil=12)
    o2 = Oracle(cfg["A"], cfg["part"], cfg["p"]).use_cinv(nit=2, tol=0.01, lfil=12)
    C = _c_alpha(o1)
    X1, X2 = o1.cinv()[0].toarray(), o2.cinv()[0].toarray()
    R2 = np.eye(o1.s) - C @ X2
    CD = C @ (X2 - X1)
    assert abs(np.sum(R2 * CD)) < 1e-12 * np.linalg.norm(R2) * np.linalg.norm(CD)


def test_cinv_preconditioner_end_to_end():
    """DDLR-1 with the approximate inverse for C_alpha: certified SPD, CG on C1
    converges to the direct solution."""
    cfg = w.config("c1")
    A = cfg["A"]
    o = Oracle(A, cfg["part"], cfg["p"]).use_cinv(nit=3, tol=0.01, lfil=20)
    o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(A.n, 0))
    assert o.spd
    b, xs = w.rhs_from_solution(A, 0, 2)
    x, info = o.pcg(b)
    assert info["status"] == 0 and np.all(info["relres_true"] <= 1.01e-6)
    xd = spla.spsolve(A.to_scipy().tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-3 * np.linalg.norm(xd)
    # the factor path on the same problem, for scale: both preconditioners work
    of = Oracle(A, cfg["part"], cfg["p"])
    of.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(A.n, 0))
    _, infof = of.pcg(b)
    assert infof["status"] == 0 and abs(int(info["its"][0]) - int(infof["its"][0])) <= 20


@pytest.mark.parametrize("name", ["c1", "small3d"])
def test_cinv_spd_certificate(name):
    """||I - C X||_inf bounds the spectral radius of I - C X (LAPACK
    eigenvalues), and when it is below 1, X is SPD."""
    cfg = w.config(name)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"]).use_cinv(nit=3, tol=0.01, lfil=20)
    X, res, spd = o.cinv()
    C = _c_alpha(o)
    R = np.eye(o.s) - C @ X.toarray()
    assert abs(o.cinv_rinf - np.abs(R).sum(axis=1).max()) <= 1e-12
    assert np.abs(np.linalg.eigvals(R)).max() <= o.cinv_rinf + 1e-12
    assert spd == (o.cinv_rinf < 1.0) and spd
    assert np.linalg.eigvalsh(X.toarray()).min() > 0.0


# ------------------ DDLR-2 by bidiagonalisation of A0^{-1} E (Sec. 4.4 (sec:Lan) alternative)

def test_gk_full_run_gives_singular_values():
    """A full bidiagonalisation (m = s) recovers the singular values of
    A0^{-1} E (LAPACK SVD of the dense operator); sigma^2 are recorded."""
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    k = 4
    o.lowrank_gk(k, o.s, w.lanczos_start(A.n, 5))
    _, _, sv = _ddlr2_from_svd(o, k)
    ta, tb, rz = o.lanczos_record()
    assert len(rz) == o.s
    assert np.abs(np.sqrt(np.maximum(rz, 0)) - sv[: len(rz)]).max() <= 1e-10 * sv[0]


def test_gk_build_matches_svd_and_spectral_theorem():
    """The bidiagonalisation build gives the U_k H_k U_k^T of the SVD of
    A0^{-1} E (as the Lanczos build does) and the DDLR-2 theorem holds:
    0 < eta <= 1 with n-s+k unit eigenvalues."""
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p, factor=FACTOR_EXACT)
    k = 4
    o.lowrank_gk(k, o.s, w.lanczos_start(A.n, 5))
    U, Hk = o.get_lowrank()
    Uk_ref, Hk_ref, sv = _ddlr2_from_svd(o, k)
    perm, *_ = o.ordering()
    C_or = (U @ Hk @ U.T)[np.ix_(perm, perm)]
    C_ref = Uk_ref @ Hk_ref @ Uk_ref.T
    assert np.abs(C_or - C_ref).max() <= 1e-9 * np.abs(C_ref).max()
    ev = np.linalg.eigvals(A.to_dense() @ _dense_minv(o)).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-9
    assert (np.abs(ev - 1) <= 1e-8).sum() == o.n - o.s + k


def test_gk_short_run_close_to_lanczos_route():
    """With incomplete factors and m = 2k steps both builds approximate the
    same dominant singular subspace: the two preconditioners agree closely,
    and CG converges with either."""
    cfg = w.config("c1")
    A = cfg["A"]
    v0 = w.lanczos_start(A.n, 0)
    og = Oracle(A, cfg["part"], cfg["p"]).lowrank_gk(cfg["k"], cfg["m"], v0)
    ol = Oracle(A, cfg["part"], cfg["p"]).lowrank(2, cfg["k"], cfg["m"], v0)
    rg, rl = og.lanczos_record()[2], ol.lanczos_record()[2]
    # sigma^2 of the bidiagonal and the Ritz values of E^T A0^{-2} E: both Krylov
    # approximations of the same largest eigenvalues
    assert np.abs(rg[:3] - rl[:3]).max() <= 1e-6 * rl[0]
    b, _ = w.rhs_from_solution(A, 0, 2)
    xg, ig = og.pcg(b)
    xl, il = ol.pcg(b)
    assert ig["status"] == 0 and il["status"] == 0 and og.spd
    assert np.all(np.abs(ig["its"] - il["its"]) <= 2)


# ---------------------- C_alpha by preconditioned Chebyshev (Sec. 4.3 (sec:csolve), Table 3)

def _cheb_setup(name, nu=5, mc=10):
    cfg = w.config(name)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"]).use_cheb(nu, mc)
    m = o.m
    C = o.csr("A0").toarray()[m:, m:]
    L = o.csr("L").toarray()[m:, m:]
    Dg = o.diag()[m:]
    M = (np.eye(o.s) + L) @ np.diag(Dg) @ (np.eye(o.s) + L).T
    return cfg, o, C, M


def test_cheb_block_jacobi_factor():
    """D_alpha keeps only couplings inside one subdomain's interface, and its
    LDL^T reproduces C_alpha on that pattern (incomplete-factor property)."""
    cfg, o, C, M = _cheb_setup("c1")
    perm, *_ = o.ordering()
    part = np.asarray(cfg["part"])[perm[o.m:]]
    L = o.csr("L").toarray()[o.m:, o.m:]
    nz = np.nonzero(L)
    assert np.all(part[nz[0]] == part[nz[1]])
    pat = (C != 0) & (part[:, None] == part[None, :])
    assert np.abs((M - C)[pat]).max() <= 1e-12 * np.abs(C).max()


@pytest.mark.parametrize("nu", [1, 3, 5])
def test_cheb_matches_chebyshev_polynomial(nu):
    """The solve is nu steps of Chebyshev acceleration on [lo, hi]: the error
    operator I - X C (X = the solve) has eigenvalues
    T_nu((theta - lambda)/delta) / T_nu(theta/delta) at the eigenvalues lambda
    of D_alpha^{-1} C_alpha (closed form of the scaled Chebyshev residual
    polynomial; eigenvalues from LAPACK)."""
    cfg, o, C, M = _cheb_setup("c1", nu=nu)
    lo, hi, rlo, rhi = o.cheb()
    s, m, n = o.s, o.m, o.n
    perm, *_ = o.ordering()
    E = np.zeros((n, s))
    E[perm[m:], np.arange(s)] = 1.0  # unit vectors on the interface, user order
    Z = o.a0_solve(E)
    X = Z[perm[m:], :]
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(M, C)).real)
    th, de = (hi + lo) / 2, (hi - lo) / 2
    T = np.polynomial.chebyshev.Chebyshev.basis(nu)
    want = np.sort(T((th - lam) / de) / T(th / de))
    got = np.sort(np.linalg.eigvals(np.eye(s) - X @ C).real)
    assert np.abs(got - want).max() <= 1e-10
    # the safeguarded interval covers the spectrum here, and X is SPD
    assert lo <= lam[0] and hi >= lam[-1] and rlo >= lam[0] - 1e-12 and rhi <= lam[-1] + 1e-12
    assert np.abs(X - X.T).max() <= 1e-12 * np.abs(X).max()
    assert np.linalg.eigvalsh((X + X.T) / 2).min() > 0


def test_cheb_preconditioner_end_to_end():
    cfg = w.config("c1")
    A = cfg["A"]
    o = Oracle(A, cfg["part"], cfg["p"]).use_cheb(5, 10)
    o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(A.n, 0))
    assert o.spd
    b, _ = w.rhs_from_solution(A, 0, 2)
    x, info = o.pcg(b)
    assert info["status"] == 0 and np.all(info["relres_true"] <= 1.01e-6)
    xd = spla.spsolve(A.to_scipy().tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-3 * np.linalg.norm(xd)


# ------------------------------------- partial reorthogonalisation (Sec. 4.4)

def _pro_case():
    """Random-coefficient diffusion on 48x40 in 4x3 boxes (s = 408): a run of
    120 steps converges Ritz values and, without reorthogonalisation, loses
    orthogonality of the Lanczos vectors by many orders of magnitude."""
    dims = (48, 40)
    return w.tpfa_2d(*dims, 5), w.box_partition(dims, (4, 3)), 12


def _pro_run(mode, m=120):
    A, part, p = _pro_case()
    o = Oracle(A, part, p).set_reorth(mode)
    o.lowrank(1, 8, m, w.lanczos_start(A.n, 0))
    return o


def test_partial_reorth_semi_orthogonality_and_projection():
    """Simon's theorem behind partial reorthogonalisation: with |q_i^T q_j| kept
    below sqrt(eps), Q^T H Q equals T_m to rounding level, so the Ritz values
    are eigenvalues of the exactly projected operator.  The same run without
    reorthogonalisation shows both fail (so the pin has teeth), and a Ritz
    value whose residual bound beta_m |s_mi| is small lies within that bound
    of an eigenvalue of H computed by LAPACK."""
    m = 120
    out = {}
    for mode in (1, 2):
        o = _pro_run(mode, m)
        ta, tb, rz = o.lanczos_record()
        Q = o.lanczos_basis()
        H = dense_H(o_ic_dense(o))
        T = np.diag(ta) + np.diag(tb[:-1], 1) + np.diag(tb[:-1], -1)
        th, S = np.linalg.eigh(T)
        orth = np.abs(Q.T @ Q - np.eye(m)).max()
        proj = np.abs(np.linalg.eigvalsh(Q.T @ H @ Q) - th).max()
        out[mode] = (orth, proj)
        if mode == 1:
            ev = np.linalg.eigvalsh(H)
            bound = np.abs(tb[-1] * S[-1, :])
            conv = bound <= 1e-8
            assert conv.sum() >= 3
            for t, b in zip(th[conv], bound[conv]):
                assert np.abs(ev - t).min() <= b + 1e-12
    assert out[1][0] <= 1e-7 and out[1][1] <= 1e-11
    assert out[2][0] >= 1e-2 and out[2][1] >= 1e-4


def test_partial_reorth_schedule():
    """Reorthogonalisation happens at few steps, never in the first ones (the
    estimates start at rounding level), and each triggered step is followed by
    a reorthogonalised step (Simon: the next vector is orthogonalised too)."""
    m = 120
    f = _pro_run(1, m).reorth_steps()
    assert len(f) == m
    steps = np.nonzero(f)[0]
    assert 0 < len(steps) <= m // 8
    assert steps[0] >= 10
    runs = np.split(steps, np.nonzero(np.diff(steps) != 1)[0] + 1)
    assert all(len(r) >= 2 or r[-1] == m - 1 for r in runs)
    assert not _pro_run(0, m).reorth_steps().any()


def test_partial_reorth_same_preconditioner_as_full():
    """The preconditioner built from a partially reorthogonalised run equals the
    one from full reorthogonalisation: Ritz values to 1e-12 (relative), the
    action of M^{-1} to sqrt(eps) (relative: the basis is orthonormal to that
    order, and so are the Ritz vectors built from it), in DDLR-1 and DDLR-2."""
    x = np.random.default_rng(4).standard_normal((1920, 4))
    for variant in (1, 2):
        ys, rzs = [], []
        for mode in (0, 1):
            A, part, p = _pro_case()
            o = Oracle(A, part, p).set_reorth(mode)
            o.lowrank(variant, 8, 120, w.lanczos_start(A.n, 0))
            rzs.append(o.lanczos_record()[2])
            ys.append(o.apply(x))
        assert np.abs(rzs[0] - rzs[1]).max() <= 1e-12 * abs(rzs[0][0])
        assert np.abs(ys[0] - ys[1]).max() <= np.sqrt(2.0 ** -52) * np.abs(ys[0]).max()


def test_partial_reorth_mode_checked():
    A, part, p = tiny_irregular()
    o = Oracle(A, part, p)
    with pytest.raises(OracleError):
        o.set_reorth(3)
