"""GPU parity at the launch shapes of the full-size 3-D runs, element by element.

The 128^3 7-point workload (64 subdomains of 32^3) solves 8 right-hand sides
at once, which selects launch shapes that the small parity cases never reach:
  - the block triangular solve with R = 2 columns per workgroup, whose LDS
    ring (8,192 rows in FP32, 4,096 in FP64 at R = 2) wraps inside a
    32,768-row block, and whose levels (up to about 770 rows) need the second
    row set of a 512-thread workgroup;
  - CG's SpMV on the interleaved search direction with S = 8;
  - the low-rank kernels with k = 32 (two 16-column tiles).
The cases below use blocks of exactly that shape (64^3 grid, 2x2x2 boxes) and
blocks of 40^3 (80^3 grid), whose levels exceed 1,024 rows and so also run the
rows beyond the two prefetched row sets.  Every column count per workgroup
(R = 1, 2, 4, 8, each reduced by the library to what the ring can hold) and
both CG launch forms (replayed graphs and eager launches) are forced, in FP64
and with the FP32 preconditioner.

Comparisons (tests/parity.py: relative 2-norm and per-column elementwise):
  - A0 solve and SpMV against the oracle: FP64 1e-12 (SpMV 1e-14), FP32 1e-5;
    bitwise equal across R (the shapes differ in launch geometry only);
  - the preconditioner with the oracle's low-rank data imported: FP64 1e-10,
    FP32 1e-4;
  - the CG iterate after 6 steps (same preconditioner, same start): FP64
    1e-10, FP32 1e-4 (single-precision preconditioner, six steps); bitwise
    equal across R and across the two launch forms.
"""
import os
import sys

import numpy as np
import pytest

import paper_1505_04341_amd as D
import workloads as w
from oracle import Oracle
from parity import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NRHS = 8
RS = ("1", "2", "4", "8")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float64).T)).to(DEV)


def to_host(t):
    return t.cpu().numpy().T


def case(name):
    if name == "blocks32":  # the 128^3 run's block shape: 32^3 boxes
        N, P, k, m = 64, 2, 32, 64
    else:  # "blocks40": levels above 1,024 rows
        N, P, k, m = 80, 2, 16, 32
    A = w.laplacian_3d(N, N, N)
    return dict(A=A, part=w.box_partition((N, N, N), (P, P, P)), p=P ** 3, k=k, m=m)


_ORACLES = {}


def oracle_for(name, cfg):
    """One oracle per case (its setup and Lanczos are the slow part on the CPU)."""
    if name not in _ORACLES:
        o = Oracle(cfg["A"], cfg["part"], cfg["p"])
        o.lowrank(1, cfg["k"], cfg["m"], w.lanczos_start(cfg["A"].n, 0))
        _ORACLES[name] = (o, o.get_lowrank())
    return _ORACLES[name]


def setup(cfg, prec, env=None):
    env = dict(env or {})
    os.environ.update(env)
    try:
        # the Lanczos run is short: the oracle's low-rank data is imported
        h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], 4, D.DDLR_1, lanczos_steps=8,
                         lanczos_start=w.lanczos_start(cfg["A"].n, 0), precision=prec, autotune=False)
    finally:
        for key in env:
            os.environ.pop(key, None)
    return h


def with_r(R, fn):
    os.environ["DDLR_RING_R"] = R
    try:
        return fn()
    finally:
        os.environ.pop("DDLR_RING_R", None)


@pytest.mark.parametrize("name", ["blocks32", "blocks40"])
@pytest.mark.parametrize("prec", [D.FP64, D.FP32])
def test_headline_a0_solve_spmv_apply(name, prec):
    cfg = case(name)
    n = cfg["A"].n
    say("headline a0/spmv/apply", name, "prec", prec)
    o, lr = oracle_for(name, cfg)
    h = setup(cfg, prec)
    D.ddlr_set_lowrank(h, 1, *lr)
    x = np.random.default_rng(21).standard_normal((n, NRHS))
    xd = to_dev(x)
    a0_ref, ap_ref = o.a0_solve(x), o.apply(x)
    tol_a0, tol_ap = (1e-12, 1e-10) if prec == D.FP64 else (1e-5, 1e-4)
    a0s, aps = [], []
    for R in RS:
        say("  R", R)
        y = torch.empty((NRHS, n), dtype=torch.float64, device=DEV)
        with_r(R, lambda: D.ddlr_a0_solve(h, xd, y))
        a0s.append(y.cpu())
        assert_close(to_host(y), a0_ref, tol_a0, f"A0 solve R={R}")
        with_r(R, lambda: D.ddlr_apply(h, xd, y))
        aps.append(y.cpu())
        assert_close(to_host(y), ap_ref, tol_ap, f"apply R={R}")
    for R, a, b in zip(RS[1:], a0s[1:], aps[1:]):
        assert torch.equal(a, a0s[0]), f"A0 solve differs between R=1 and R={R}"
        assert torch.equal(b, aps[0]), f"apply differs between R=1 and R={R}"
    y = torch.empty((NRHS, n), dtype=torch.float64, device=DEV)
    D.ddlr_spmv(h, xd, y)
    assert_close(to_host(y), o.matvec(x), 1e-14, "SpMV")


@pytest.mark.parametrize("name", ["blocks32", "blocks40"])
@pytest.mark.parametrize("prec", [D.FP64, D.FP32])
def test_headline_pcg_six_steps(name, prec):
    """Each (R, launch form) on its own handle, so that a captured chunk graph
    holds the forced shape."""
    cfg = case(name)
    n = cfg["A"].n
    o, lr = oracle_for(name, cfg)
    b, _ = w.rhs_from_solution(cfg["A"], 0, NRHS)
    xo, io = o.pcg(b, maxit=6)
    tol = 1e-10 if prec == D.FP64 else 1e-4
    first = None
    for graph in ("1", "0"):
        for R in (RS if name == "blocks32" else ("1", "2")):
            say("headline pcg", name, "prec", prec, "graph", graph, "R", R)
            h = setup(cfg, prec, env={"DDLR_CG_GRAPH": graph})
            D.ddlr_set_lowrank(h, 1, *lr)
            x = torch.zeros((NRHS, n), dtype=torch.float64, device=DEV)
            st, info = with_r(R, lambda: D.ddlr_solve(h, to_dev(b), x, maxit=6))
            assert st == D.E_NO_CONVERGENCE and all(i["iters"] == 6 for i in info)
            got = x.cpu()
            assert_close(got.numpy().T, xo, tol, f"CG iterate graph={graph} R={R}")
            if first is None:
                first = got
            else:
                assert torch.equal(got, first), f"CG iterate differs at graph={graph} R={R}"
            del h
