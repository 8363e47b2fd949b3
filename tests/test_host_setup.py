"""CPU tests of the HIP library's host side: the C ABI loads and exports every
declared symbol, and the host setup (ordering, colouring, splitting, local
factors, level schedule) matches the oracle.  No device work is done here
(setup with device = -1)."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_1505_04341_amd as D
import workloads as w
from oracle import Oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ddlr.h")).read()
    declared = sorted(set(re.findall(r"\b(ddlr_[a-z0-9_]+)\s*\(", hdr)))
    lib = D.load_library()
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared) == set(D.EXPORTED)


def _cases():
    yield "c1", w.config("c1"), {}
    yield "small2d", w.config("small2d"), {}
    yield "small3d", w.config("small3d"), {}
    A = w.random27_3d(9, 8, 7, 3)
    yield "r27", dict(A=A, part=w.box_partition((9, 8, 7), (2, 2, 2)), p=8, k=6), dict(alpha=2.0)
    A = w.tpfa_2d(31, 27, 5)
    yield "tpfa", dict(A=A, part=w.box_partition((31, 27), (3, 3)), p=9, k=6), {}
    yield "c1-natural", w.config("c1"), dict(corder=D.CORDER_NATURAL)


@pytest.mark.parametrize("name,cfg,kw", list(_cases()), ids=[c[0] for c in _cases()])
def test_host_setup_matches_oracle(name, cfg, kw):
    A = cfg["A"]
    h = D.ddlr_setup(A, cfg["part"], cfg["p"], cfg["k"], D.DDLR_1, device=-1, **kw)
    o = Oracle(A, cfg["part"], cfg["p"], alpha=kw.get("alpha", 1.0), corder=kw.get("corder", 0))
    perm, iface, colour = D.ddlr_get_ordering(h)
    operm, oiface, ocolour, _ = o.ordering()
    assert np.array_equal(perm, operm)
    assert np.array_equal(iface, oiface)
    assert np.array_equal(colour, ocolour)
    q = D.ddlr_query(h)
    assert (q["m"], q["s"], q["ncolours"]) == (o.m, o.s, o.ncolours)
    L, Dg = D.ddlr_get_factor(h)
    Lo = o.csr("L")
    assert np.array_equal(L.indptr, Lo.indptr) and np.array_equal(L.indices, Lo.indices)
    assert np.abs(L.data - Lo.data).max(initial=0) <= 1e-12 * max(1.0, np.abs(Lo.data).max(initial=0))
    assert np.abs(Dg - o.diag()).max() <= 1e-12 * np.abs(o.diag()).max()


@pytest.mark.parametrize("name,cfg,kw", list(_cases()), ids=[c[0] for c in _cases()])
def test_level_schedule_valid(name, cfg, kw):
    """Every row's level is 1 + the largest level of the rows it depends on
    (0 if none), so rows of one level are independent."""
    h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], D.DDLR_1, device=-1, **kw)
    L, _ = D.ddlr_get_factor(h)
    lev = D.ddlr_get_levels(h)
    Lc = L.tocsr()
    for i in range(L.shape[0]):
        cols = Lc.indices[Lc.indptr[i]:Lc.indptr[i + 1]]
        expect = 0 if cols.size == 0 else lev[cols].max() + 1
        assert lev[i] == expect


def test_level_depth_closed_form():
    """Lexicographic box: level of (x,y) is x+y inside the interior block, so the
    depth of a B-block is (nx-1)+(ny-1) of its interior box (C1: 31+31 - 1 = 61)."""
    c = w.config("c1")
    h = D.ddlr_setup(c["A"], c["part"], c["p"], c["k"], D.DDLR_1, device=-1)
    q = D.ddlr_query(h)
    assert q["levels_b_max"] == 61 and q["levels_c"] == q["ncolours"] == 2


def test_setup_errors_are_reported():
    A = w.laplacian_2d(6, 6)
    part = w.box_partition((6, 6), (2, 2))
    bad = part.copy()
    bad[0] = 7
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_setup(A, bad, 4, 2, D.DDLR_1, device=-1)
    assert e.value.status == D.E_INVALID
    d = A.to_dense()
    d[0, 1] = -3.0
    M = sp.csr_matrix(d)
    M.sort_indices()
    B = w.CSR(36, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_setup(B, part, 4, 2, D.DDLR_1, device=-1)
    assert e.value.status == D.E_NOT_SYMMETRIC
    d = A.to_dense()
    d[7, 7] = -3.0
    M = sp.csr_matrix(d)
    M.sort_indices()
    B = w.CSR(36, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_setup(B, part, 4, 2, D.DDLR_1, device=-1)
    assert e.value.status == D.E_BREAKDOWN
    assert "row" in str(e.value)
    D.ddlr_setup(B, part, 4, 2, D.DDLR_1, device=-1, factor=D.FACTOR_ILDL0)
    with pytest.raises(D.DDLRError) as e:  # k + 1 > s
        D.ddlr_setup(A, part, 4, 400, D.DDLR_1, device=-1)
    assert e.value.status == D.E_INVALID
    with pytest.raises(D.DDLRError) as e:  # a single subdomain has no interface
        D.ddlr_setup(A, np.zeros(36, np.int32), 1, 2, D.DDLR_1, device=-1)
    assert e.value.status == D.E_INVALID


def test_host_only_handle_refuses_device_work():
    c = w.config("c1")
    h = D.ddlr_setup(c["A"], c["part"], c["p"], c["k"], D.DDLR_1, device=-1)
    lib = D.load_library()
    st = lib.ddlr_apply(h.handle, 1, None, c["A"].n, None, c["A"].n, None)
    assert st == D.E_DEVICE


@pytest.mark.parametrize("p", [2, 7, 16])
def test_partitioner_matches_reference(p):
    """Library recursive bisection == the reference definition, bit-exact."""
    from oracle.partition import partition_graph
    A, _ = w.rgg_laplacian(6000, 9, 3)
    assert np.array_equal(D.ddlr_partition_graph(A, p), partition_graph(A, p))
    G = w.laplacian_2d(23, 17)
    assert np.array_equal(D.ddlr_partition_graph(G, p), partition_graph(G, p))


def test_partitioner_errors():
    G = w.laplacian_2d(3, 2)
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_partition_graph(G, 7)  # more parts than vertices
    assert e.value.status == D.E_INVALID


@pytest.mark.parametrize("name,cfg,kw", list(_cases()), ids=[c[0] for c in _cases()])
@pytest.mark.parametrize("nit,tol,lfil", [(3, 0.01, 20), (2, 0.0, 6), (4, 0.1, 4)])
def test_cinv_matches_oracle_bitwise(name, cfg, kw, nit, tol, lfil):
    """The library's approximate inverse of C_alpha (host build, Algorithm
    alg:mr) equals the oracle's bit for bit: both follow the stated arithmetic
    order, so every drop decision agrees."""
    A = cfg["A"]
    h = D.ddlr_setup(A, cfg["part"], cfg["p"], cfg["k"], D.DDLR_1, device=-1, csolve=D.CSOLVE_MR,
                     cinv_iters=nit, cinv_tol=tol, cinv_lfil=lfil, **kw)
    o = Oracle(A, cfg["part"], cfg["p"], alpha=kw.get("alpha", 1.0), corder=kw.get("corder", 0))
    o.use_cinv(nit, tol, lfil)
    X, res = D.ddlr_get_cinv(h)
    Xo, reso, spdo = o.cinv()
    assert np.array_equal(X.indptr, Xo.indptr) and np.array_equal(X.indices, Xo.indices)
    assert np.array_equal(X.data, Xo.data)
    assert np.array_equal(res, reso)
    q = D.ddlr_query(h)
    assert q["csolve"] == D.CSOLVE_MR and q["nnz_cinv"] == Xo.nnz and q["cinv_res"] == reso[-1]
    assert q["cinv_res_inf"] == o.cinv_rinf
    # interface rows of L are empty, D is 1 there
    L, Dg = D.ddlr_get_factor(h)
    assert L.indptr[-1] == L.indptr[q["m"]] and np.all(Dg[q["m"]:] == 1.0)


def test_cinv_option_errors():
    c = w.config("c1")
    with pytest.raises(D.DDLRError):
        D.ddlr_setup(c["A"], c["part"], c["p"], c["k"], D.DDLR_1, device=-1, csolve=7)
    with pytest.raises(D.DDLRError):
        D.ddlr_setup(c["A"], c["part"], c["p"], c["k"], D.DDLR_1, device=-1, csolve=D.CSOLVE_MR, cinv_iters=-1)
    h = D.ddlr_setup(c["A"], c["part"], c["p"], c["k"], D.DDLR_1, device=-1)
    with pytest.raises(D.DDLRError):
        D.ddlr_get_cinv(h)


def test_reorth_option_errors():
    """lanczos_reorth takes DDLR_REORTH_FULL or _PARTIAL, and partial
    reorthogonalisation belongs to the Lanczos build, not the
    bidiagonalisation; a handle without a Lanczos run has no flags."""
    c = w.config("c1")
    args = (c["A"], c["part"], c["p"], c["k"])
    for kw in (dict(lanczos_reorth=2), dict(lanczos_reorth=-1),
               dict(lanczos_reorth=D.REORTH_PARTIAL, lowrank_build=D.BUILD_BIDIAG)):
        with pytest.raises(D.DDLRError) as e:
            D.ddlr_setup(*args, D.DDLR_2, device=-1, **kw)
        assert e.value.status == D.E_INVALID
    h = D.ddlr_setup(*args, D.DDLR_1, device=-1, lanczos_reorth=D.REORTH_PARTIAL)
    assert D.ddlr_query(h)["lanczos_reorth_steps"] == 0
    with pytest.raises(D.DDLRError):
        D.ddlr_get_lanczos_reorth(h)


@pytest.mark.parametrize("name,cfg,kw", list(_cases()), ids=[c[0] for c in _cases()])
def test_cheb_factor_and_interval_match_oracle(name, cfg, kw):
    """Chebyshev C_alpha solver: the block-Jacobi factor of D_alpha (interface
    rows of L, D) equals the oracle's; the spectrum interval from the pencil
    Lanczos agrees to rounding (the two use different tridiagonal eigensolvers)."""
    A = cfg["A"]
    h = D.ddlr_setup(A, cfg["part"], cfg["p"], cfg["k"], D.DDLR_1, device=-1, csolve=D.CSOLVE_CHEB, **kw)
    o = Oracle(A, cfg["part"], cfg["p"], alpha=kw.get("alpha", 1.0), corder=kw.get("corder", 0))
    o.use_cheb(5, 10)
    L, Dg = D.ddlr_get_factor(h)
    Lo = o.csr("L")
    assert np.array_equal(L.indptr, Lo.indptr) and np.array_equal(L.indices, Lo.indices)
    assert np.abs(L.data - Lo.data).max(initial=0) <= 1e-12 * max(1.0, np.abs(Lo.data).max(initial=0))
    assert np.abs(Dg - o.diag()).max() <= 1e-12 * np.abs(o.diag()).max()
    q = D.ddlr_query(h)
    lo, hi, rlo, rhi = o.cheb()
    assert q["csolve"] == D.CSOLVE_CHEB
    for a, b in ((q["cheb_lo"], lo), (q["cheb_hi"], hi), (q["cheb_ritz_lo"], rlo), (q["cheb_ritz_hi"], rhi)):
        assert abs(a - b) <= 1e-10 * abs(b)
    assert 0 < q["cheb_lo"] <= q["cheb_ritz_lo"] <= q["cheb_ritz_hi"] <= q["cheb_hi"]


def test_cheb_refuses_indefinite_block_jacobi():
    """The Chebyshev solver needs D_alpha SPD: ILDL(0) of a matrix shifted to
    negative diagonals gives negative pivots, and the setup is refused."""
    A = w.laplacian_3d(8, 8, 8, shift=7.0)
    part = w.box_partition((8, 8, 8), (2, 2, 1))
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_setup(A, part, 4, 4, D.DDLR_1, device=-1, factor=D.FACTOR_ILDL0, csolve=D.CSOLVE_CHEB)
    assert e.value.status == D.E_BREAKDOWN and "pivot" in str(e.value)


@pytest.mark.parametrize("dims,parts", [((64, 64), (2, 2)), ((37, 29), (3, 2)), ((25, 25, 25), (4, 4, 8)),
                                        ((100, 100, 100), (4, 4, 8)), ((7, 5, 3), (7, 1, 3))])
def test_partition_box_matches_generator(dims, parts):
    """The library's box split equals the workload generator's (an independent
    statement of the same rule), and every box has the sizes the rule gives."""
    got = D.ddlr_partition_box(dims, parts)
    assert np.array_equal(got, w.box_partition(dims, parts))
    counts = np.bincount(got, minlength=int(np.prod(parts)))
    d3, p3 = list(dims) + [1] * (3 - len(dims)), list(parts) + [1] * (3 - len(parts))
    sx, sy, sz = [[N // P + (1 if i < N % P else 0) for i in range(P)] for N, P in zip(d3, p3)]
    expect = np.zeros_like(counts)
    for bz in range(p3[2]):
        for by in range(p3[1]):
            for bx in range(p3[0]):
                expect[bx + p3[0] * (by + p3[1] * bz)] = sx[bx] * sy[by] * sz[bz]
    assert np.array_equal(counts, expect)
    with pytest.raises(D.DDLRError):
        D.ddlr_partition_box((4, 4), (5, 1))
