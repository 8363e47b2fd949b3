"""Setup files and contexts on the CPU (host-only handles, device = -1).

- The library's export holds the ordering the oracle computes (bit for bit)
  and its factors (pattern bit for bit, values to 1e-12: the two factor
  codes sum in different orders), in the layout include/ddlr.h documents
  (read back by an independent reader, tests/setup_file.py).
- Import rebuilds the same plan: ordering, factor, levels equal; exporting the
  import gives the same file byte for byte.
- Files that fail the documented checks are refused with DDLR_E_INVALID.
"""
import numpy as np
import pytest

import paper_1505_04341_amd as D
import setup_file as SF
import workloads as w
from oracle import Oracle

CASES = {
    "c1": lambda: w.config("c1"),
    "small3d": lambda: w.config("small3d"),
    "tpfa": lambda: dict(A=w.tpfa_2d(37, 29, 11), part=w.box_partition((37, 29), (3, 2)), p=6, k=6),
}


def close(a, b, tol=1e-12):
    assert np.abs(a - b).max() <= tol * np.abs(b).max()


def host_ctx():
    return D.ddlr_ctx_create(-1, 0)


def setup(cfg, **kw):
    return D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], D.DDLR_1, ctx=host_ctx(), **kw)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("csolve", [D.CSOLVE_FACTOR, D.CSOLVE_MR, D.CSOLVE_CHEB])
def test_export_matches_oracle_and_round_trips(name, csolve, tmp_path):
    cfg = CASES[name]()
    h = setup(cfg, csolve=csolve)
    f1 = str(tmp_path / "a.ddlr")
    D.ddlr_export_setup(h, f1)
    rec = SF.read(f1)
    n, p = cfg["A"].n, cfg["p"]
    assert list(rec["n_p"]) == [n, p] and rec["alpha"][0] == 1.0
    assert list(rec["csolve_prec_nu"][:2]) == [csolve, 0]
    o = Oracle(cfg["A"], cfg["part"], p)
    if csolve == D.CSOLVE_MR:
        o.use_cinv()
    if csolve == D.CSOLVE_CHEB:
        o.use_cheb()
    perm, iface, colour, boff = o.ordering()
    assert np.array_equal(rec["perm"], perm) and np.array_equal(rec["boff"], boff)
    assert np.array_equal(rec["colour"], colour)
    m = int(boff[p])
    L = o.csr("L")
    Dg = o.diag()
    if csolve == D.CSOLVE_MR:  # no factor of the interface block
        assert np.all(np.diff(rec["L.rowptr"][m:]) == 0) and np.all(rec["D"][m:] == 1.0)
        assert np.array_equal(rec["L.rowptr"][:m + 1], L.indptr[:m + 1])
        nb = int(L.indptr[m])
        assert np.array_equal(rec["L.col"], L.indices[:nb])
        close(rec["L.val"], L.data[:nb])
        close(rec["D"][:m], Dg[:m])
        X, _, _ = o.cinv()
        assert np.array_equal(rec["X.rowptr"], X.indptr) and np.array_equal(rec["X.col"], X.indices)
        assert np.array_equal(rec["X.val"], X.data)
    else:
        assert np.array_equal(rec["L.rowptr"], L.indptr) and np.array_equal(rec["L.col"], L.indices)
        close(rec["L.val"], L.data)
        close(rec["D"], Dg)
    if csolve == D.CSOLVE_CHEB:
        close(rec["cheb"], np.array(o.cheb()), 1e-10)  # different tridiagonal eigensolvers
    # levels: lev(i) = 0 for an empty row of L, else 1 + max over its columns
    lev = np.zeros(n, np.int64)
    for i in range(n):
        cols = rec["L.col"][rec["L.rowptr"][i]:rec["L.rowptr"][i + 1]]
        lev[i] = 1 + lev[cols].max() if len(cols) else 0
    assert np.array_equal(rec["level"], lev)
    # import into another host-only context: the same plan, the same file
    h2 = D.ddlr_import_setup(cfg["A"], f1, ctx=host_ctx())
    for a, b in zip(D.ddlr_get_ordering(h), D.ddlr_get_ordering(h2)):
        assert np.array_equal(a, b)
    (L1, D1), (L2, D2) = D.ddlr_get_factor(h), D.ddlr_get_factor(h2)
    assert np.array_equal(L1.indptr, L2.indptr) and np.array_equal(L1.indices, L2.indices)
    assert np.array_equal(L1.data, L2.data) and np.array_equal(D1, D2)
    assert np.array_equal(D.ddlr_get_levels(h), D.ddlr_get_levels(h2))
    f2 = str(tmp_path / "b.ddlr")
    D.ddlr_export_setup(h2, f2)
    assert open(f1, "rb").read() == open(f2, "rb").read()


def refused(A, path):
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_import_setup(A, path, ctx=host_ctx())
    assert e.value.status == D.E_INVALID
    return str(e.value)


def test_import_refuses_bad_files(tmp_path):
    cfg = w.config("c1")
    A = cfg["A"]
    good = str(tmp_path / "good.ddlr")
    D.ddlr_export_setup(setup(cfg), good)
    rec = SF.read(good)
    path = str(tmp_path / "bad.ddlr")

    def variant(**changes):
        r = {k: v.copy() for k, v in rec.items()}
        for k, v in changes.items():
            if v is None:
                r.pop(k)
            else:
                r[k] = v
        SF.write(path, r)
        return refused(A, path)

    refused(A, str(tmp_path / "missing.ddlr"))
    open(path, "wb").write(b"not a setup file")
    refused(A, path)
    open(path, "wb").write(open(good, "rb").read()[:-9])  # truncated
    refused(A, path)
    # another matrix order
    B = w.laplacian_2d(10, 10)
    refused(B, good)
    # not a permutation
    perm = rec["perm"].copy()
    perm[1] = perm[0]
    variant(perm=perm)
    # interiors of two blocks swapped: rows coupled across blocks
    perm = rec["perm"].copy()
    b1 = int(rec["boff"][1])
    perm[0], perm[b1] = perm[b1], perm[0]
    assert "couples" in variant(perm=perm, level=None)
    # an L entry on the diagonal
    col = rec["L.col"].copy()
    r = int(np.argmax(np.diff(rec["L.rowptr"]) > 0))
    col[rec["L.rowptr"][r]] = r
    variant(**{"L.col": col, "level": None})
    # a zero pivot
    Dz = rec["D"].copy()
    Dz[3] = 0.0
    variant(D=Dz)
    # levels that do not belong to the factor
    lv = rec["level"].copy()
    lv[5] += 1
    variant(level=lv)
    # a missing array
    variant(D=None)


def test_ddlr_setup_rejects_device_in_host_context():
    """A host-only context gives host-only handles, which refuse device work."""
    cfg = w.config("c1")
    h = setup(cfg)
    assert D.ddlr_query(h)["on_device"] == 0
    assert D.ddlr_ctx_usage(h._ctx)["used"] == 0
