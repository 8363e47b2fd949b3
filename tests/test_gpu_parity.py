"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances (FP64 path): A0 solve and SpMV 1e-12 relative, preconditioner
application with imported low-rank data 1e-10 relative, CG iterate after a
fixed number of steps 1e-10, own end-to-end setup: Ritz values 1e-8 and
iteration counts within one of the oracle.  Mixed path: true residual
<= 1e-6 and at most 10% (+1) more iterations than FP64.
"""
import os
import sys

import numpy as np
import pytest

import paper_1505_04341_amd as D
import workloads as w
from oracle import FACTOR_ILDL, Oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def to_dev(x):
    """(n, nrhs) numpy -> (nrhs, n) contiguous cuda float64."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)


def to_host(t):
    a = t.cpu().numpy()
    return a if a.ndim == 1 else a.T


from parity import assert_close, assert_converged_close, rel  # noqa: E402


def setup_pair(cfg, variant=1, wide=None, env=None, **kw):
    """Builds the GPU preconditioner (kernel choices forced through env) and the oracle."""
    env = dict(env or {})
    if wide is not None:
        env["DDLR_C_WIDE"] = "1" if wide else "0"
    os.environ.update(env)
    try:
        h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], variant, lanczos_steps=cfg.get("m", 0),
                         lanczos_start=w.lanczos_start(cfg["A"].n, 0), **kw)
    finally:
        for key in env:
            os.environ.pop(key, None)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"], alpha=kw.get("alpha", 1.0), corder=kw.get("corder", 0),
               factor=FACTOR_ILDL if kw.get("factor", 0) == 1 else 0)
    return h, o


def irregular():
    A = w.tpfa_2d(37, 29, 11)
    return dict(A=A, part=w.box_partition((37, 29), (3, 2)), p=6, k=6, m=20)


def big3d():
    """Blocks of about 10,000 rows: larger than the FP64 LDS ring (8,192 rows),
    so the ring wraps within a block."""
    A = w.laplacian_3d(48, 48, 40)
    return dict(A=A, part=w.box_partition((48, 48, 40), (2, 2, 2)), p=8, k=8, m=20)


CASES = {"c1": lambda: w.config("c1"), "small2d": lambda: w.config("small2d"),
         "small3d": lambda: w.config("small3d"), "irregular": irregular, "big3d": big3d}


@pytest.mark.parametrize("name", ["c1", "small3d", "irregular", "big3d"])
@pytest.mark.parametrize("wide", [False, "auto", "rows", "cols"])
@pytest.mark.parametrize("kernel", ["ring", "plain"])
def test_a0_solve_and_spmv(name, wide, kernel):
    """wide: the interface block as one narrow block, or its colour levels
    launched one by one: through the private buffer with the form chosen by
    level size (auto) or one thread per row (rows), or the column-major
    kernel with one thread per (row, column) (cols)."""
    cfg = CASES[name]()
    say("a0_solve", name, "wide", wide, kernel)
    env = {"DDLR_TRSV_PLAIN": "1" if kernel == "plain" else "0"}
    if wide in ("rows", "cols"):
        env["DDLR_LEVEL_KERNEL"] = wide
    h, o = setup_pair(cfg, variant=D.VARIANT_A0, wide=bool(wide), env=env)
    n = cfg["A"].n
    rng = np.random.default_rng(7)
    for nrhs in (1, 3, 17):  # 17: two launches of up to 16 columns, ragged tail
        x = rng.standard_normal((n, nrhs))
        y = torch.empty((nrhs, n), dtype=torch.float64, device=DEV)
        D.ddlr_a0_solve(h, to_dev(x), y)
        got = to_host(y)
        ref = o.a0_solve(x)
        assert_close(got, ref, 1e-12)
        D.ddlr_spmv(h, to_dev(x), y)
        assert_close(to_host(y), o.matvec(x), 1e-14)


@pytest.mark.parametrize("name", ["small3d", "irregular"])
@pytest.mark.parametrize("prec", [0, 1])
def test_columns_independent_of_batch_width(name, prec):
    """A column's A0 solve is bitwise the same whether it is solved alone or
    with 1..16 others (interface levels and E products come in column widths
    1, 2, 4, 8 and 16 with clamped surplus columns), and its full DDLR-1
    apply agrees to rounding; both match the oracle."""
    cfg = CASES[name]()
    say("column widths", name, prec)
    h, o = setup_pair(cfg, variant=1, wide=True, precision=[D.FP64, D.FP32][prec])
    n = cfg["A"].n
    x = np.random.default_rng(17).standard_normal((n, 16))
    alone_a0, alone_ap = [], []
    for j in range(16):
        y = torch.empty((1, n), dtype=torch.float64, device=DEV)
        D.ddlr_a0_solve(h, to_dev(x[:, j:j + 1]), y)
        alone_a0.append(y.cpu())
        D.ddlr_apply(h, to_dev(x[:, j:j + 1]), y)
        alone_ap.append(y.cpu())
    tol = 1e-13 if prec == 0 else 1e-6
    for w in (2, 3, 5, 8, 11, 16):
        y = torch.empty((w, n), dtype=torch.float64, device=DEV)
        D.ddlr_a0_solve(h, to_dev(x[:, :w]), y)
        got = y.cpu()
        for j in range(w):
            assert torch.equal(got[j:j + 1], alone_a0[j]), (w, j)
        D.ddlr_apply(h, to_dev(x[:, :w]), y)
        got = y.cpu().numpy()
        for j in range(w):
            assert_close(got[j], alone_ap[j].numpy()[0], tol)
    ref = o.a0_solve(x[:, :3])
    assert_close(torch.cat(alone_a0[:3]).numpy().T, ref, (1e-12 if prec == 0 else 1e-5))


@pytest.mark.parametrize("name", ["c1", "small2d", "irregular"])
@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("lr", ["mfma", "plain"])
def test_apply_with_imported_lowrank(name, variant, lr):
    cfg = CASES[name]()
    say("apply imported", name, variant, lr)
    h, o = setup_pair(cfg, variant=variant, env={"DDLR_LR_PLAIN": "1" if lr == "plain" else "0"})
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    lr = o.get_lowrank()
    if variant == 1:
        D.ddlr_set_lowrank(h, 1, lr[0], lr[1], lr[2])
    else:
        D.ddlr_set_lowrank(h, 2, lr[0], lr[1])
    n = cfg["A"].n
    x = np.random.default_rng(3).standard_normal((n, 5))
    y = torch.empty((5, n), dtype=torch.float64, device=DEV)
    D.ddlr_apply(h, to_dev(x), y)
    ref = o.apply(x)
    assert_close(to_host(y), ref, 1e-10)
    # round trip of the low-rank data through the ABI
    back = D.ddlr_get_lowrank(h)
    assert np.array_equal(back[0], lr[0])


@pytest.mark.parametrize("name", ["c1", "irregular", "small3d"])
@pytest.mark.parametrize("variant", [1, 2])
def test_own_lanczos_matches_oracle(name, variant):
    cfg = CASES[name]()
    say("lanczos", name, variant)
    h, o = setup_pair(cfg, variant=variant)
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    ga, gb, gr = D.ddlr_get_lanczos(h)
    oa, ob, orz = o.lanczos_record()
    assert len(ga) == len(oa)
    k = cfg["k"]
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * max(1.0, abs(orz[0]))
    assert np.abs(ga[:4] - oa[:4]).max() <= 1e-10 * np.abs(oa).max()
    q = D.ddlr_query(h)
    if variant == 1:
        assert abs(q["theta"] - orz[k]) <= 1e-8


def test_interface_and_cg_forms_bitwise():
    """Launch forms that leave the arithmetic unchanged give bitwise the same
    results: the interface levels through the private buffer (one thread per
    row, or per (row, column)) or column-major (per (row, column)), and the CG
    x update with the p update or on a side stream beside the preconditioner.
    Checked on the apply and on 30 CG iterations of 8 columns."""
    cfg = big3d()
    n = cfg["A"].n
    say("interface / CG forms")
    forms = [{}, {"DDLR_LEVEL_KERNEL": "rows"}, {"DDLR_LEVEL_KERNEL": "cols"}, {"DDLR_CG_XP": "0"}]
    x = to_dev(np.random.default_rng(21).standard_normal((n, 8)))
    b = to_dev(w.rhs_from_solution(cfg["A"], 0, 8)[0])
    outs = []
    for env in forms:
        h, _ = setup_pair(cfg, variant=1, wide=True, env=dict(env, DDLR_CG_PERSIST="0"), precision=D.FP32)
        y = torch.empty_like(x)
        D.ddlr_apply(h, x, y)
        xt = torch.zeros_like(b)
        D.ddlr_solve(h, b, xt, maxit=30)
        outs.append((y.cpu().numpy(), xt.cpu().numpy()))
    for y, xs in outs[1:]:
        assert np.array_equal(y, outs[0][0]) and np.array_equal(xs, outs[0][1])


@pytest.mark.parametrize("name", ["c1", "small3d", "irregular"])
def test_pcg_fixed_steps_matches_oracle(name):
    """Same preconditioner (imported), same number of CG steps: same iterate."""
    cfg = CASES[name]()
    say("pcg fixed", name)
    h, o = setup_pair(cfg, variant=1)
    o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    U, lam, th = o.get_lowrank()
    D.ddlr_set_lowrank(h, 1, U, lam, th)
    b, _ = w.rhs_from_solution(cfg["A"], 0, 3)
    x = torch.zeros((3, cfg["A"].n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x, maxit=6)
    assert st == D.E_NO_CONVERGENCE and all(i["iters"] == 6 for i in info)
    xo, infoo = o.pcg(b, maxit=6)
    assert_close(to_host(x), xo, 1e-10)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    xo, infoo = o.pcg(b)
    assert st == D.OK
    # the iterates agree to rounding, so the step that crosses 1e-6 may differ by one
    assert all(abs(i["iters"] - int(io)) <= 1 for i, io in zip(info, infoo["its"]))
    assert_converged_close(to_host(x), xo, 1e-5)


@pytest.mark.parametrize("name", ["c1", "small3d"])
@pytest.mark.parametrize("variant", [1, 2])
def test_pcg_end_to_end_own_setup(name, variant):
    cfg = CASES[name]()
    say("pcg e2e", name, variant)
    h, o = setup_pair(cfg, variant=variant)
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    nrhs = cfg.get("nrhs", 1)
    b, xs = w.rhs_from_solution(cfg["A"], 0, nrhs)
    x = torch.zeros((nrhs, cfg["A"].n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    assert st == D.OK
    xo, infoo = o.pcg(b)
    for i, io in zip(info, infoo["its"]):
        assert abs(i["iters"] - io) <= 1
        assert i["relres_true"] <= 1e-6
    assert_converged_close(to_host(x), xo, 1e-5)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("lr", ["mfma", "plain"])
def test_fp32_apply_matches_oracle(variant, lr):
    """FP32 preconditioner (factors, E, U_k in single precision): same operator
    as the FP64 oracle up to single-precision rounding."""
    cfg = irregular()
    say("fp32 apply", variant, lr)
    h, o = setup_pair(cfg, variant=variant, precision=D.FP32, env={"DDLR_LR_PLAIN": "1" if lr == "plain" else "0"})
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    lr_ = o.get_lowrank()
    D.ddlr_set_lowrank(h, variant, *lr_)
    n = cfg["A"].n
    for nrhs in (1, 5, 16):
        x = np.random.default_rng(nrhs).standard_normal((n, nrhs))
        y = torch.empty((nrhs, n), dtype=torch.float64, device=DEV)
        D.ddlr_apply(h, to_dev(x), y)
        assert_close(to_host(y), o.apply(x), 1e-4)


@pytest.mark.parametrize("variant", [1, 2])
def test_bf16_basis_apply_matches_oracle(variant):
    """FP32 preconditioner with U_k in bfloat16 on the bf16 MFMA: the operator
    matches the FP64 oracle up to bf16 rounding of U_k (2^-9 relative)."""
    cfg = irregular()
    say("bf16 apply", variant)
    h, o = setup_pair(cfg, variant=variant, precision=D.FP32_UK_BF16)
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    D.ddlr_set_lowrank(h, variant, *o.get_lowrank())
    n = cfg["A"].n
    for nrhs in (1, 7, 16):
        x = np.random.default_rng(nrhs).standard_normal((n, nrhs))
        y = torch.empty((nrhs, n), dtype=torch.float64, device=DEV)
        D.ddlr_apply(h, to_dev(x), y)
        assert_close(to_host(y), o.apply(x), 5e-3)


@pytest.mark.parametrize("prec", [D.FP32, D.FP32_UK_BF16])
def test_mixed_precision_solve(prec):
    cfg = w.config("small3d")
    say("mixed", prec)
    h64, _ = setup_pair(cfg, variant=1)
    h32 = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], 1, lanczos_steps=cfg["m"],
                       lanczos_start=w.lanczos_start(cfg["A"].n, 0), precision=prec)
    b, xs = w.rhs_from_solution(cfg["A"], 0, 4)
    x64 = torch.zeros((4, cfg["A"].n), dtype=torch.float64, device=DEV)
    x32 = torch.zeros_like(x64)
    _, i64 = D.ddlr_solve(h64, to_dev(b), x64)
    st, i32 = D.ddlr_solve(h32, to_dev(b), x32)
    assert st == D.OK
    for a, c in zip(i64, i32):
        assert c["relres_true"] <= 1e-6
        assert c["iters"] <= int(1.1 * a["iters"]) + 1
    # state the error against the FP64 result
    err = rel(to_host(x32), to_host(x64))
    say("mixed vs fp64 relative difference", err)
    assert err <= 1e-4


def test_solve_edge_cases():
    cfg = w.config("c1")
    say("edge cases")
    h, o = setup_pair(cfg, variant=1)
    n = cfg["A"].n
    b = np.zeros((n, 2))
    b[:, 1] = w.rhs_from_solution(cfg["A"], 1, 1)[0][:, 0]
    x = torch.full((2, n), 5.0, dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    assert st == D.OK
    assert info[0]["iters"] == 0 and float(x[0].abs().max()) == 0.0
    assert info[1]["iters"] > 0
    st, info = D.ddlr_solve(h, to_dev(b), x, maxit=1)
    assert st == D.E_NO_CONVERGENCE and info[1]["iters"] == 1 and info[1]["status"] == D.E_NO_CONVERGENCE
    # zero columns is a no-op
    lib = D.load_library()
    assert lib.ddlr_apply(h.handle, 0, None, n, None, n, None) == D.OK
    # leading dimension too small
    t = torch.zeros(n, dtype=torch.float64, device=DEV)
    assert lib.ddlr_apply(h.handle, 1, t.data_ptr(), n - 1, t.data_ptr(), n, None) == D.E_INVALID


def test_cg_refused_for_indefinite_preconditioner():
    A = w.laplacian_2d(24, 20)
    d = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    d[rows == A.col] -= 0.7  # largest Ritz value of E^T A0^{-1} E above 1
    A = w.CSR(A.n, A.rowptr, A.col, d)
    part = w.box_partition((24, 20), (2, 2))
    say("indefinite")
    h = D.ddlr_setup(A, part, 4, 10, 1, lanczos_steps=30, factor=D.FACTOR_ILDL0,
                     lanczos_start=w.lanczos_start(A.n, 1))
    q = D.ddlr_query(h)
    assert q["spd"] == 0
    b = to_dev(w.rhs_from_solution(A, 0, 1)[0])
    x = torch.zeros_like(b)
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_solve(h, b, x)
    assert e.value.status == D.E_NOT_SPD


@pytest.mark.parametrize("overlap", ["0", "1"])
def test_interface_levels_on_side_stream(overlap):
    """The interface block's level kernels on a side stream (fork/join by
    events) or on the caller's stream give the same result."""
    cfg = big3d()
    say("side stream", overlap)
    h, o = setup_pair(cfg, variant=1, wide=True, env={"DDLR_NO_OVERLAP": "1" if overlap == "0" else "0"},
                      precision=D.FP32)
    n = cfg["A"].n
    x = np.random.default_rng(11).standard_normal((n, 8))
    y = torch.empty((8, n), dtype=torch.float64, device=DEV)
    for _ in range(3):
        D.ddlr_a0_solve(h, to_dev(x), y)
    assert_close(to_host(y), o.a0_solve(x), 1e-5)


def shifted2d(sig, nx=24, ny=20):
    A = w.laplacian_2d(nx, ny)
    d = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    d[rows == A.col] -= sig
    return w.CSR(A.n, A.rowptr, A.col, d), w.box_partition((nx, ny), (2, 2))


@pytest.mark.parametrize("restart", [40, 7])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_gmres_matches_oracle(restart, variant):
    """Right-preconditioned GMRES(restart) on an indefinite shifted Laplacian:
    iterate and iteration count as in the oracle's GMRES."""
    A, part = shifted2d(0.3)
    say("gmres", restart, variant)
    h = D.ddlr_setup(A, part, 4, 10, variant, lanczos_steps=30, factor=D.FACTOR_ILDL0,
                     lanczos_start=w.lanczos_start(A.n, 1))
    o = Oracle(A, part, 4, factor=FACTOR_ILDL)
    if variant:
        o.lowrank(variant, 10, 30, w.lanczos_start(A.n, 1))
        lr = o.get_lowrank()
        D.ddlr_set_lowrank(h, variant, *lr)  # same preconditioner on both sides
    b, _ = w.rhs_from_solution(A, 0, 3)
    x = torch.zeros((3, A.n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x, method=1, restart=restart)
    xo, io = o.gmres(b, restart=restart)
    # short restarts with the A0 part alone may stagnate on this indefinite
    # problem: the statuses must agree either way
    assert st == io["status"]
    for i, it in zip(info, io["its"]):
        # rounding differences accumulate over many short restart cycles
        assert abs(i["iters"] - int(it)) <= max(1, int(0.03 * int(it)))
        if st == D.OK:
            assert i["relres"] <= 1e-6 and i["relres_true"] <= 2e-6
    if st == D.OK:
        assert_converged_close(to_host(x), xo, 1e-5)
    # a fixed number of steps gives the same iterate
    st, info = D.ddlr_solve(h, to_dev(b), x, method=1, restart=restart, maxit=restart + 3)
    xo, io = o.gmres(b, restart=restart, maxit=restart + 3)
    assert st == D.E_NO_CONVERGENCE and all(i["iters"] == restart + 3 for i in info)
    assert_close(to_host(x), xo, 1e-9)


def batch_members(count, prec, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        nx, ny = int(rng.integers(12, 40)), int(rng.integers(12, 40))
        px, py = int(rng.integers(2, 4)), int(rng.integers(1, 4))
        A = w.tpfa_2d(nx, ny, 100 + q)
        part = w.box_partition((nx, ny), (px, py))
        out.append((A, part, px * py))
    return out


@pytest.mark.parametrize("prec", [D.FP64, D.FP32])
def test_batch_matches_single_and_oracle(prec):
    """Each system's result in the batch equals its solve alone (same operator,
    different reduction grouping: within 1e-9) and the oracle's; the captured
    iteration graph gives identical results on every replay, with other eager
    work between replays."""
    mem = batch_members(11, prec)
    say("batch", prec)
    k, m = 4, 10
    hs = [D.ddlr_setup(A, part, p, k, 1, lanczos_steps=m, lanczos_start=w.lanczos_start(A.n, 3), precision=prec)
          for A, part, p in mem]
    B = D.ddlr_batch_create(hs)
    bs = [w.rhs_from_solution(A, q, 1)[0][:, 0] for q, (A, _, _) in enumerate(mem)]
    bt = torch.from_numpy(np.concatenate(bs)).to(DEV)
    xs = []
    for rep in range(3):
        x = torch.zeros_like(bt)
        st, info = D.ddlr_batch_solve(B, bt, x)
        assert st == D.OK
        xs.append(x.cpu().numpy())
        # eager work between replays: a single-system solve on another handle
        b0 = torch.from_numpy(bs[0]).to(DEV)
        D.ddlr_solve(hs[0], b0, torch.zeros_like(b0))
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    off = B.offsets
    for q, ((A, part, p), h) in enumerate(zip(mem, hs)):
        b = torch.from_numpy(bs[q]).to(DEV)
        xq = torch.zeros_like(b)
        st1, i1 = D.ddlr_solve(h, b, xq)
        xb = xs[0][off[q]:off[q + 1]]
        # FP32: the batch's per-system correction accumulates in FP64, the single
        # path's FP32 MFMA in FP32 (operators equal to ~1e-7)
        slack = 1 if prec == D.FP64 else max(1, int(0.1 * i1[0]["iters"]))
        assert abs(info[q]["iters"] - i1[0]["iters"]) <= slack
        assert info[q]["relres_true"] <= 1e-6
        # two CG runs stopped at 1e-6 residual differ by up to ~cond * 1e-6 in x;
        # these random-coefficient systems (contrast 1e4) are ill-conditioned
        assert_converged_close(xb, xq.cpu().numpy(), 1e-4)
        o = Oracle(A, part, p)
        o.lowrank(1, k, m, w.lanczos_start(A.n, 3))
        xo, io = o.pcg(bs[q])
        if prec == D.FP64:
            assert abs(info[q]["iters"] - int(io["its"][0])) <= 1
        else:  # mixed-precision bar against the FP64 oracle
            assert info[q]["iters"] <= int(1.1 * int(io["its"][0])) + 1
        assert_converged_close(xb, xo, 1e-4)
    # the batch's preconditioner application equals each member's
    y = torch.empty_like(bt)
    D.ddlr_batch_apply(B, bt, y)
    for q, h in enumerate(hs):
        b = torch.from_numpy(bs[q]).to(DEV)
        yq = torch.empty_like(b)
        D.ddlr_apply(h, b, yq)
        assert_close(y.cpu().numpy()[off[q]:off[q + 1]], yq.cpu().numpy(), (1e-12 if prec == D.FP64 else 1e-6))


def test_serving_same_alone_and_in_mix():
    """Continuous batching: a right-hand side solved alone, by the server with
    an otherwise empty queue, and by the server inside a stream of requests on
    three matrices (requests arriving while others run, more columns than
    lanes, the iterated lane width changing with occupancy) gives bitwise the
    same x, and the server reports each column's true residual (<= 1e-6)."""
    import time
    cfgs = [w.config("c1"), w.config("small3d"), irregular()]
    hs, refs, bsets = [], [], []
    for q, cfg in enumerate(cfgs):
        say("serving setup", q)
        # the reference solves take the served form's lane-phase CG (the persistent form sums its dot
        # products in another order)
        os.environ["DDLR_CG_PERSIST"] = "0"
        try:
            h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], 1, lanczos_steps=cfg["m"],
                             lanczos_start=w.lanczos_start(cfg["A"].n, 0), precision=D.FP32)
        finally:
            os.environ.pop("DDLR_CG_PERSIST")
        b, _ = w.rhs_from_solution(cfg["A"], 10 * q, 6)
        bt = torch.from_numpy(np.ascontiguousarray(b.T)).to(DEV)
        xt = torch.zeros_like(bt)
        st, info = D.ddlr_solve(h, bt, xt)
        assert st == D.OK
        hs.append(h)
        refs.append(xt.cpu().numpy().T)
        bsets.append(b)
    srv = D.ddlr_server_create(0, 0, 4)
    mids = [D.ddlr_server_add(srv, h) for h in hs]
    # alone
    t, x = D.ddlr_server_submit(srv, mids[1], bsets[1][:, 2])
    st, info = D.ddlr_server_wait(srv, t)
    assert st == D.OK and np.array_equal(x[:, 0], refs[1][:, 2])
    assert 0 < info[0]["relres_true"] <= 1e-6
    # in a mix: random matrices, 1..6 columns, staggered arrivals
    rng = np.random.default_rng(5)
    jobs = []
    for j in range(24):
        q = int(rng.integers(0, 3))
        cols = sorted(rng.choice(6, size=int(rng.integers(1, 7)), replace=False))
        t, x = D.ddlr_server_submit(srv, mids[q], bsets[q][:, cols])
        jobs.append((t, x, q, cols))
        time.sleep(float(rng.exponential(0.002)))
    for t, x, q, cols in jobs:
        st, info = D.ddlr_server_wait(srv, t)
        assert st == D.OK
        assert all(i["relres"] <= 1e-6 and 0 < i["relres_true"] <= 1e-6 for i in info)
        assert np.array_equal(x, refs[q][:, cols]), (q, cols)
    stats = D.ddlr_server_stats(srv)
    assert stats["requests_done"] == 25 and stats["queued"] == 0
    assert stats["p99_ms"] >= stats["p50_ms"] > 0 and stats["solves_per_s"] > 0
    say("serving stats", stats)
    del srv


def test_serving_budget_admission():
    cfg = w.config("small3d")
    h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], 1, lanczos_steps=cfg["m"],
                     lanczos_start=w.lanczos_start(cfg["A"].n, 0))
    srv = D.ddlr_server_create(0, 1 << 20, 4)  # 1 MiB cannot hold the matrix
    with pytest.raises(D.DDLRError) as e:
        D.ddlr_server_add(srv, h)
    assert e.value.status == D.E_BUDGET
    del srv


@pytest.mark.parametrize("prec", [0, 1])
def test_autotuner_shapes_bitwise(prec):
    """Every launch shape the autotuner may pick (1, 2, 4, 8 columns per
    workgroup of the block triangular solve; interface overlap on/off) gives
    bitwise the same A0 solve, and ddlr_tune reports an eligible choice."""
    import os
    cfg = w.config("small3d")
    A = cfg["A"]
    h = D.ddlr_setup(A, cfg["part"], cfg["p"], cfg["k"], 0, precision=[D.FP64, D.FP32][prec], autotune=False)
    x = torch.randn(8, A.n, dtype=torch.float64, device=DEV)
    outs = []
    for R in ("1", "2", "4", "8"):
        os.environ["DDLR_RING_R"] = R
        y = torch.empty_like(x)
        D.ddlr_a0_solve(h, x, y)
        torch.cuda.synchronize()
        outs.append(y.cpu())
    os.environ.pop("DDLR_RING_R")
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    t = D.ddlr_tune(h, 8, retune=True)
    say("tune", t)
    assert t["ring_cols"] in (1, 2, 4, 8) and t["a0_us"][0] > 0
    y = torch.empty_like(x)
    D.ddlr_a0_solve(h, x, y)
    torch.cuda.synchronize()
    assert torch.equal(y.cpu(), outs[0])


def wide_k():
    """A 3-D case with k a multiple of 16 (the wide-load low-rank kernels) and
    interface rows not a multiple of 16 (ragged last tile)."""
    A = w.laplacian_3d(22, 19, 17)
    return dict(A=A, part=w.box_partition((22, 19, 17), (3, 2, 2)), p=12, k=32, m=48)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("k", [16, 32])
def test_apply_wide_lowrank_kernels(variant, prec, k):
    """k % 16 == 0 selects the low-rank kernels with 16-byte operand loads
    (tile-ordered U_k for U_k^T y, permuted K for U_k c): the apply matches the
    oracle (FP64 to 1e-10, FP32 to single-precision rounding) and the
    one-element-per-lane MFMA kernels up to rounding order."""
    cfg = wide_k()
    cfg["k"], cfg["m"] = k, 2 * k + 8
    say("wide lowrank", variant, prec, k)
    p_ = D.FP64 if prec == "fp64" else D.FP32
    h, o = setup_pair(cfg, variant=variant, precision=p_)
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    lr_ = o.get_lowrank()
    D.ddlr_set_lowrank(h, variant, *lr_)
    n = cfg["A"].n
    tol = 1e-10 if prec == "fp64" else 1e-4
    for nrhs in (1, 6, 16):
        x = np.random.default_rng(nrhs).standard_normal((n, nrhs))
        y = torch.empty((nrhs, n), dtype=torch.float64, device=DEV)
        D.ddlr_apply(h, to_dev(x), y)
        assert_close(to_host(y), o.apply(x), tol, f"nrhs {nrhs}")


@pytest.mark.parametrize("variant", [1, 2])
def test_lanczos_control_matches_oracle(variant):
    """The paper's Lanczos control (eq. converge every 10 steps, eps 1e-4,
    at most 5k steps): same stopping step and Ritz values as the oracle."""
    cfg = w.config("small3d")
    k = cfg["k"]
    say("lanczos control", variant)
    h, o = setup_pair(cfg, variant=variant, lanczos_check=10, lanczos_tol=1e-4)
    o.lowrank(variant, k, 5 * k, w.lanczos_start(cfg["A"].n, 0), check=10, eps=1e-4)
    q = D.ddlr_query(h)
    assert q["lanczos_steps"] == o.msteps
    ga, gb, gr = D.ddlr_get_lanczos(h)
    oa, ob, orz = o.lanczos_record()
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * max(1.0, abs(orz[0]))
    n = cfg["A"].n
    x = np.random.default_rng(4).standard_normal((n, 3))
    y = torch.empty((3, n), dtype=torch.float64, device=DEV)
    D.ddlr_set_lowrank(h, variant, *o.get_lowrank())
    D.ddlr_apply(h, to_dev(x), y)
    assert_close(to_host(y), o.apply(x), 1e-10)


@pytest.mark.parametrize("variant", [1, 2])
def test_extend_lowrank(variant):
    """Improving a given preconditioner: setup with (k=6, m=16), then
    continuing by 12 steps to k=10 gives bitwise the preconditioner of a
    single (k=10, m=28) setup, and matches the oracle's extended build."""
    cfg = w.config("small3d")
    v0 = w.lanczos_start(cfg["A"].n, 0)
    say("extend", variant)
    h1 = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], 6, variant, lanczos_steps=16, lanczos_start=v0)
    D.ddlr_extend_lowrank(h1, 10, 12)
    h2 = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], 10, variant, lanczos_steps=28, lanczos_start=v0)
    assert D.ddlr_query(h1)["lanczos_steps"] == D.ddlr_query(h2)["lanczos_steps"] == 28
    for a, b in zip(D.ddlr_get_lanczos(h1), D.ddlr_get_lanczos(h2)):
        assert np.array_equal(a, b)
    n = cfg["A"].n
    x = np.random.default_rng(6).standard_normal((n, 4))
    y1 = torch.empty((4, n), dtype=torch.float64, device=DEV)
    y2 = torch.empty_like(y1)
    D.ddlr_apply(h1, to_dev(x), y1)
    D.ddlr_apply(h2, to_dev(x), y2)
    assert torch.equal(y1, y2)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"]).lowrank(variant, 6, 16, v0)
    o.extend(10, 12)
    # same operator as the oracle up to the eigensolver's rounding of T_m
    assert_close(to_host(y1), o.apply(x), 1e-8)
    # errors: no run to continue after imported low-rank data
    D.ddlr_set_lowrank(h2, variant, *o.get_lowrank())
    with pytest.raises(D.DDLRError):
        D.ddlr_extend_lowrank(h2, 12, 4)


def test_unstructured_rgg_end_to_end():
    """General sparse SPD matrix (random geometric graph Laplacian) with the
    library's graph partitioner: the partition equals the reference
    definition, the A0 solve matches the oracle to 1e-12 and PCG takes the
    oracle's iteration count (+-1) to the same solution."""
    from oracle.partition import partition_graph
    A, _ = w.rgg_laplacian(30000, 10, 5)
    p = 16
    part = D.ddlr_partition_graph(A, p)
    part_o = partition_graph(A, p)
    assert np.array_equal(part, part_o)
    cfg = dict(A=A, part=part, p=p, k=16, m=32)
    say("rgg", A.n, len(A.col))
    h, _ = setup_pair(cfg, variant=1)
    o = Oracle(A, part_o, p)  # the oracle takes the partition its own rule produced
    n = A.n
    x = np.random.default_rng(9).standard_normal((n, 3))
    y = torch.empty((3, n), dtype=torch.float64, device=DEV)
    D.ddlr_a0_solve(h, to_dev(x), y)
    assert_close(to_host(y), o.a0_solve(x), 1e-12)
    o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(n, 0))
    b, xs = w.rhs_from_solution(A, 3, 2)
    xt = torch.zeros((2, n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), xt)
    xo, io = o.pcg(b)
    assert st == D.OK
    for i, its in zip(info, io["its"]):
        assert abs(i["iters"] - int(its)) <= 1 and i["relres_true"] <= 1e-6
    assert_converged_close(to_host(xt), xo, 1e-5)


@pytest.mark.parametrize("case", ["small3d", "rgg", "tpfa"])
@pytest.mark.parametrize("prec", [0, 1])
def test_ring_workgroup_sizes_bitwise(case, prec):
    """The one-column block triangular solve with 64 (single wave, no
    barriers), 256 and 512 threads per workgroup, and the plain per-level
    kernel, give bitwise the same A0 solve (where eligible) and match the
    oracle; covers ELL width 32 (unstructured rows) and narrow 2-D levels."""
    import os
    if case == "small3d":
        cfg = w.config("small3d")
    elif case == "rgg":
        A, _ = w.rgg_laplacian(12000, 12, 8)
        cfg = dict(A=A, part=D.ddlr_partition_graph(A, 8), p=8, k=8, m=16)
    else:
        A = w.tpfa_2d(90, 70, 3)
        cfg = dict(A=A, part=w.box_partition((90, 70), (3, 2)), p=6, k=8, m=16)
    A = cfg["A"]
    h, o = setup_pair(cfg, variant=0, precision=[D.FP64, D.FP32][prec], autotune=False)
    x = np.random.default_rng(2).standard_normal((A.n, 3))
    outs = {}
    for nt in ("64", "256", "512", "-1"):
        os.environ["DDLR_RING_NT"] = nt
        y = torch.empty((3, A.n), dtype=torch.float64, device=DEV)
        D.ddlr_a0_solve(h, to_dev(x), y)
        torch.cuda.synchronize()
        outs[nt] = y.cpu()
    os.environ.pop("DDLR_RING_NT")
    for nt in ("64", "256", "-1"):  # -1: the plain per-level kernel
        assert torch.equal(outs[nt], outs["512"]), nt
    ref = o.a0_solve(x)
    assert_close(outs["512"].numpy().T, ref, (1e-12 if prec == 0 else 1e-5))
    t = D.ddlr_tune(h, 1, retune=True)
    say("tune", case, prec, t)
    assert t["ring_threads"] in (-1, 64, 256, 512)


# ------------------------------ C_alpha by its approximate inverse (Sec. 4.3 (sec:csolve))

def setup_pair_mr(cfg, variant=1, nit=3, tol=0.01, lfil=20, env=None, **kw):
    """GPU preconditioner and oracle, both solving C_alpha with the MR approximate inverse."""
    env = dict(env or {})
    os.environ.update(env)
    try:
        h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], variant, lanczos_steps=cfg.get("m", 0),
                         lanczos_start=w.lanczos_start(cfg["A"].n, 0), csolve=D.CSOLVE_MR, cinv_iters=nit,
                         cinv_tol=tol, cinv_lfil=lfil, **kw)
    finally:
        for key in env:
            os.environ.pop(key, None)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"], alpha=kw.get("alpha", 1.0), corder=kw.get("corder", 0))
    o.use_cinv(nit, tol, lfil)
    return h, o


@pytest.mark.parametrize("name", ["c1", "small3d", "irregular", "big3d"])
@pytest.mark.parametrize("overlap", ["0", "1"])
def test_cinv_a0_solve(name, overlap):
    cfg = CASES[name]()
    say("cinv a0_solve", name, "overlap", overlap)
    h, o = setup_pair_mr(cfg, variant=D.VARIANT_A0, env={"DDLR_NO_OVERLAP": "1" if overlap == "0" else "0"})
    q = D.ddlr_query(h)
    X, res, spd = o.cinv()
    assert q["csolve"] == D.CSOLVE_MR and q["nnz_cinv"] == X.nnz and q["cinv_res"] == res[-1]
    n = cfg["A"].n
    rng = np.random.default_rng(11)
    for nrhs in (1, 3, 17):
        x = rng.standard_normal((n, nrhs))
        y = torch.empty((nrhs, n), dtype=torch.float64, device=DEV)
        D.ddlr_a0_solve(h, to_dev(x), y)
        ref = o.a0_solve(x)
        assert_close(to_host(y), ref, 1e-12)


@pytest.mark.parametrize("name", ["c1", "irregular", "small3d"])
@pytest.mark.parametrize("variant", [1, 2])
def test_cinv_lanczos_and_apply(name, variant):
    """Own Lanczos on the operator with X: Ritz values as the oracle's; the
    application with the oracle's low-rank data imported."""
    cfg = CASES[name]()
    say("cinv lanczos/apply", name, variant)
    h, o = setup_pair_mr(cfg, variant=variant)
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    gr = D.ddlr_get_lanczos(h)[2]
    orz = o.lanczos_record()[2]
    k = cfg["k"]
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * max(1.0, abs(orz[0]))
    assert bool(D.ddlr_query(h)["spd"]) == bool(o.spd)
    if variant == 1:
        U, lam, th = o.get_lowrank()
        D.ddlr_set_lowrank(h, 1, U, lam, th)
    else:
        U, H = o.get_lowrank()
        D.ddlr_set_lowrank(h, 2, U, H)
    x = np.random.default_rng(3).standard_normal((cfg["A"].n, 4))
    y = torch.empty((4, cfg["A"].n), dtype=torch.float64, device=DEV)
    D.ddlr_apply(h, to_dev(x), y)
    assert_close(to_host(y), o.apply(x), 1e-10)


@pytest.mark.parametrize("name", ["c1", "small3d"])
@pytest.mark.parametrize("prec", [D.FP64, D.FP32])
def test_cinv_pcg_end_to_end(name, prec):
    cfg = CASES[name]()
    say("cinv pcg", name, prec)
    h, o = setup_pair_mr(cfg, variant=1, precision=prec)
    o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    assert D.ddlr_query(h)["spd"] and o.spd
    b, xs = w.rhs_from_solution(cfg["A"], 0, 3)
    x = torch.zeros((3, cfg["A"].n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    assert st == D.OK
    xo, infoo = o.pcg(b)
    for i, io in zip(info, infoo["its"]):
        assert i["relres_true"] <= 1e-6
        if prec == D.FP64:
            assert abs(i["iters"] - int(io)) <= 1
        else:
            assert i["iters"] <= int(1.1 * io) + 1
    assert_converged_close(to_host(x), xo, 1e-5)


def test_cinv_ddlr2_rank_above_register_block():
    """DDLR-2 builds U_k = A0^{-1} E V_k with k columns at once; k = 20 takes
    the X product in two column groups."""
    cfg = dict(w.config("small3d"), k=20, m=48)
    say("cinv ddlr2 k=20")
    h, o = setup_pair_mr(cfg, variant=2)
    o.lowrank(2, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    x = np.random.default_rng(5).standard_normal((cfg["A"].n, 2))
    y = torch.empty((2, cfg["A"].n), dtype=torch.float64, device=DEV)
    D.ddlr_apply(h, to_dev(x), y)
    assert_close(to_host(y), o.apply(x), 1e-8)


# ------------------- DDLR-2 by bidiagonalisation of A0^{-1} E (Sec. 4.4 (sec:Lan) alternative)

@pytest.mark.parametrize("name", ["c1", "irregular", "small3d"])
def test_bidiag_build_matches_oracle(name):
    cfg = CASES[name]()
    say("bidiag build", name)
    h, o = setup_pair(cfg, variant=2, lowrank_build=D.BUILD_BIDIAG)
    o.lowrank_gk(cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    ga, gb, gr = D.ddlr_get_lanczos(h)
    oa, ob, orz = o.lanczos_record()
    assert len(gr) == len(orz)
    k = cfg["k"]
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * orz[0]
    assert np.abs(ga[:4] - oa[:4]).max() <= 1e-10 * np.abs(oa).max()
    x = np.random.default_rng(9).standard_normal((cfg["A"].n, 2))
    y = torch.empty((2, cfg["A"].n), dtype=torch.float64, device=DEV)
    D.ddlr_apply(h, to_dev(x), y)
    assert_close(to_host(y), o.apply(x), 1e-6)
    # the same preconditioner (imported) gives the oracle's application to 1e-10
    U, H = o.get_lowrank()
    D.ddlr_set_lowrank(h, 2, U, H)
    D.ddlr_apply(h, to_dev(x), y)
    assert_close(to_host(y), o.apply(x), 1e-10)


def test_bidiag_solve_and_limits():
    cfg = w.config("small3d")
    say("bidiag solve")
    h, o = setup_pair(cfg, variant=2, lowrank_build=D.BUILD_BIDIAG)
    o.lowrank_gk(cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    assert D.ddlr_query(h)["spd"] and o.spd
    b, _ = w.rhs_from_solution(cfg["A"], 0, 2)
    x = torch.zeros((2, cfg["A"].n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    xo, infoo = o.pcg(b)
    assert st == D.OK
    for i, io in zip(info, infoo["its"]):
        assert abs(i["iters"] - int(io)) <= 1 and i["relres_true"] <= 1e-6
    # the run is not kept: no continuation
    with pytest.raises(D.DDLRError):
        D.ddlr_extend_lowrank(h, cfg["k"], 4)
    # DDLR-1, or the convergence control, with the bidiagonalisation: refused
    with pytest.raises(D.DDLRError):
        D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], 1, lowrank_build=D.BUILD_BIDIAG)
    with pytest.raises(D.DDLRError):
        D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], 2, lowrank_build=D.BUILD_BIDIAG, lanczos_check=4)
    # step limit
    with pytest.raises(D.DDLRError):
        D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], 2, lanczos_steps=1100)


@pytest.mark.parametrize("name", ["c1", "irregular", "big3d"])
def test_spmv_compact_storage_bitwise(name):
    """SELL with FP32 values (when all are exact) and 16-bit column offsets
    gives bitwise the results of FP64 / int32 storage: the SpMV, and CG
    (interleaved SpMV) after a few steps.  c1/big3d: Laplacians (compact
    values); irregular: random coefficients (FP64 values, 16-bit columns)."""
    cfg = CASES[name]()
    say("spmv compact", name)
    # both handles take the chunked CG form: the persistent form, which a small system may
    # choose by timing, sums its dot products in an order set by its tuned workgroup size
    h1, o = setup_pair(cfg, variant=D.VARIANT_A0, env={"DDLR_CG_PERSIST": "0"})
    h2, _ = setup_pair(cfg, variant=D.VARIANT_A0, env={"DDLR_SELL_WIDE": "1", "DDLR_CG_PERSIST": "0"})
    n = cfg["A"].n
    x = np.random.default_rng(2).standard_normal((n, 3))
    y1 = torch.empty((3, n), dtype=torch.float64, device=DEV)
    y2 = torch.empty_like(y1)
    D.ddlr_spmv(h1, to_dev(x), y1)
    D.ddlr_spmv(h2, to_dev(x), y2)
    assert torch.equal(y1, y2)
    assert_close(to_host(y1), o.matvec(x), 1e-14)
    b, _ = w.rhs_from_solution(cfg["A"], 0, 3)
    x1 = torch.zeros((3, n), dtype=torch.float64, device=DEV)
    x2 = torch.zeros_like(x1)
    D.ddlr_solve(h1, to_dev(b), x1, maxit=5)
    D.ddlr_solve(h2, to_dev(b), x2, maxit=5)
    assert torch.equal(x1, x2)


# ------------------------ C_alpha by preconditioned Chebyshev (Sec. 4.3 (sec:csolve), Table 3)

def setup_pair_cheb(cfg, variant=1, nu=5, mc=10, env=None, **kw):
    env = dict(env or {})
    os.environ.update(env)
    try:
        h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], variant, lanczos_steps=cfg.get("m", 0),
                         lanczos_start=w.lanczos_start(cfg["A"].n, 0), csolve=D.CSOLVE_CHEB, cheb_iters=nu,
                         cheb_lanczos=mc, **kw)
    finally:
        for key in env:
            os.environ.pop(key, None)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"], alpha=kw.get("alpha", 1.0), corder=kw.get("corder", 0))
    o.use_cheb(nu, mc)
    return h, o


@pytest.mark.parametrize("name", ["c1", "small3d", "irregular", "big3d"])
@pytest.mark.parametrize("overlap", ["0", "1"])
def test_cheb_a0_solve(name, overlap):
    cfg = CASES[name]()
    say("cheb a0_solve", name, "overlap", overlap)
    h, o = setup_pair_cheb(cfg, variant=D.VARIANT_A0, env={"DDLR_NO_OVERLAP": "1" if overlap == "0" else "0"})
    n = cfg["A"].n
    rng = np.random.default_rng(13)
    for nrhs in (1, 3, 17):  # 17: two column groups of the scratch
        x = rng.standard_normal((n, nrhs))
        y = torch.empty((nrhs, n), dtype=torch.float64, device=DEV)
        D.ddlr_a0_solve(h, to_dev(x), y)
        ref = o.a0_solve(x)
        assert_close(to_host(y), ref, 1e-11)


@pytest.mark.parametrize("name", ["c1", "small3d"])
@pytest.mark.parametrize("variant", [1, 2])
def test_cheb_lanczos_apply_and_solve(name, variant):
    cfg = CASES[name]()
    say("cheb lanczos/apply/solve", name, variant)
    h, o = setup_pair_cheb(cfg, variant=variant)
    o.lowrank(variant, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    gr, orz = D.ddlr_get_lanczos(h)[2], o.lanczos_record()[2]
    k = cfg["k"]
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * max(1.0, abs(orz[0]))
    assert bool(D.ddlr_query(h)["spd"]) == bool(o.spd) and o.spd
    b, _ = w.rhs_from_solution(cfg["A"], 0, 2)
    x = torch.zeros((2, cfg["A"].n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    xo, infoo = o.pcg(b)
    assert st == D.OK
    for i, io in zip(info, infoo["its"]):
        assert abs(i["iters"] - int(io)) <= 1 and i["relres_true"] <= 1e-6
    if variant == 1:
        U, lam, th = o.get_lowrank()
        D.ddlr_set_lowrank(h, 1, U, lam, th)
    else:
        U, H = o.get_lowrank()
        D.ddlr_set_lowrank(h, 2, U, H)
    xx = np.random.default_rng(4).standard_normal((cfg["A"].n, 3))
    y = torch.empty((3, cfg["A"].n), dtype=torch.float64, device=DEV)
    D.ddlr_apply(h, to_dev(xx), y)
    assert_close(to_host(y), o.apply(xx), 1e-10)


def test_cheb_mixed_precision_solve():
    cfg = CASES["small3d"]()
    say("cheb mixed")
    h, o = setup_pair_cheb(cfg, variant=1, precision=D.FP32)
    o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
    b, _ = w.rhs_from_solution(cfg["A"], 0, 3)
    x = torch.zeros((3, cfg["A"].n), dtype=torch.float64, device=DEV)
    st, info = D.ddlr_solve(h, to_dev(b), x)
    _, infoo = o.pcg(b)
    assert st == D.OK
    for i, io in zip(info, infoo["its"]):
        assert i["relres_true"] <= 1e-6 and i["iters"] <= int(1.1 * io) + 1
