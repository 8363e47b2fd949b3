"""Partial reorthogonalisation of the Lanczos run on the GPU (Sec. 4.4,
Simon's omega recurrence), through the C ABI, against the oracle's.

- The device run and the oracle's reorthogonalise at the same steps (each
  oracle step within one of a device step, counts within two: both take the
  decision in FP64 from alpha and beta that agree to rounding), give the same
  Ritz values (1e-8 relative, the bar of the full-reorthogonalisation tests)
  and the same preconditioner (1e-8 relative: the two sides' tridiagonal
  eigensolvers differ).
- On the device, partial and full reorthogonalisation give Ritz values equal
  to 1e-12 (relative) and preconditioners equal to sqrt(eps); CG takes the
  same iteration count (+-1).
- Continuing a partially reorthogonalised run (ddlr_extend_lowrank) carries
  the omega estimates: bitwise the run of a single setup.
"""
import sys

import numpy as np
import pytest

import paper_1505_04341_amd as D
import workloads as w
from oracle import Oracle
from parity import assert_close, assert_converged_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SQRT_EPS = np.sqrt(2.0 ** -52)


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float64).T)).to(DEV)


def to_host(t):
    return t.cpu().numpy().T


def tpfa_case():
    """Random-coefficient diffusion on 48x40 in 4x3 boxes (s = 408): a run of
    120 steps loses orthogonality without reorthogonalisation."""
    dims = (48, 40)
    return dict(A=w.tpfa_2d(*dims, 5), part=w.box_partition(dims, (4, 3)), p=12, k=8, m=120)


def with_m(name, m):
    cfg = w.config(name)
    cfg["m"] = m
    return cfg


CASES = {"tpfa": tpfa_case, "c1": lambda: with_m("c1", 80), "small3d": lambda: with_m("small3d", 120)}


def setup(cfg, variant, reorth, **kw):
    return D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], variant, lanczos_steps=cfg["m"],
                        lanczos_start=w.lanczos_start(cfg["A"].n, 0), lanczos_reorth=reorth, **kw)


def assert_same_schedule(dev, orc):
    a, b = np.nonzero(dev)[0], np.nonzero(orc)[0]
    assert abs(len(a) - len(b)) <= 2, (a, b)
    for j in b:
        assert len(a) and np.abs(a - j).min() <= 1, (a, b)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("variant", [1, 2])
def test_partial_reorth_matches_oracle(name, variant):
    cfg = CASES[name]()
    A, n, k = cfg["A"], cfg["A"].n, cfg["k"]
    say("partial reorth vs oracle", name, variant)
    h = setup(cfg, variant, D.REORTH_PARTIAL)
    o = Oracle(A, cfg["part"], cfg["p"]).set_reorth(1)
    o.lowrank(variant, k, cfg["m"], w.lanczos_start(n, 0))
    flags = D.ddlr_get_lanczos_reorth(h)
    oflags = o.reorth_steps()
    assert len(flags) == len(oflags) == cfg["m"]
    assert_same_schedule(flags, oflags)
    q = D.ddlr_query(h)
    assert q["lanczos_reorth"] == D.REORTH_PARTIAL and q["lanczos_reorth_steps"] == int(flags.sum())
    assert 0 < flags.sum() <= cfg["m"] // 4
    gr, orz = D.ddlr_get_lanczos(h)[2], o.lanczos_record()[2]
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * max(1.0, abs(orz[0]))
    x = np.random.default_rng(11).standard_normal((n, 4))
    y = torch.empty((4, n), dtype=torch.float64, device=DEV)
    D.ddlr_apply(h, to_dev(x), y)
    assert_close(to_host(y), o.apply(x), 1e-8, "apply")


@pytest.mark.parametrize("variant", [1, 2])
def test_partial_equals_full_on_device(variant):
    cfg = tpfa_case()
    A, n, k = cfg["A"], cfg["A"].n, cfg["k"]
    say("partial vs full", variant)
    hp = setup(cfg, variant, D.REORTH_PARTIAL)
    hf = setup(cfg, variant, D.REORTH_FULL)
    qf = D.ddlr_query(hf)
    assert qf["lanczos_reorth"] == D.REORTH_FULL and qf["lanczos_reorth_steps"] == cfg["m"]
    assert D.ddlr_get_lanczos_reorth(hf).all()
    rp, rf = D.ddlr_get_lanczos(hp)[2], D.ddlr_get_lanczos(hf)[2]
    assert np.abs(rp - rf).max() <= 1e-12 * abs(rf[0])
    x = to_dev(np.random.default_rng(12).standard_normal((n, 4)))
    yp, yf = torch.empty_like(x), torch.empty_like(x)
    D.ddlr_apply(hp, x, yp)
    D.ddlr_apply(hf, x, yf)
    assert_close(to_host(yp), to_host(yf), SQRT_EPS, "apply")
    if variant == 1:
        b = to_dev(w.rhs_from_solution(A, 0, 3)[0])
        xp, xf = torch.zeros_like(b), torch.zeros_like(b)
        sp, ip = D.ddlr_solve(hp, b, xp)
        sf, if_ = D.ddlr_solve(hf, b, xf)
        assert sp == sf == D.OK
        assert all(abs(a["iters"] - c["iters"]) <= 1 for a, c in zip(ip, if_))
        assert_converged_close(to_host(xp), to_host(xf), 1e-5)


@pytest.mark.parametrize("variant", [1, 2])
def test_partial_reorth_extend_carries_estimates(variant):
    """Setup with 50 steps, continued by 70 (across a growth of the run's
    buffers): the flags, alpha, beta, Ritz values and the preconditioner are
    bitwise those of one 120-step setup."""
    cfg = tpfa_case()
    n = cfg["A"].n
    say("partial reorth extend", variant)
    h1 = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], 6, variant, lanczos_steps=50,
                      lanczos_start=w.lanczos_start(n, 0), lanczos_reorth=D.REORTH_PARTIAL)
    D.ddlr_extend_lowrank(h1, cfg["k"], 70)
    h2 = setup(cfg, variant, D.REORTH_PARTIAL)
    assert np.array_equal(D.ddlr_get_lanczos_reorth(h1), D.ddlr_get_lanczos_reorth(h2))
    for a, b in zip(D.ddlr_get_lanczos(h1), D.ddlr_get_lanczos(h2)):
        assert np.array_equal(a, b)
    x = to_dev(np.random.default_rng(13).standard_normal((n, 3)))
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    D.ddlr_apply(h1, x, y1)
    D.ddlr_apply(h2, x, y2)
    assert torch.equal(y1, y2)


def test_partial_reorth_with_lanczos_control():
    """The paper's stopping control (eq. converge every 10 steps) on a
    partially reorthogonalised run stops where the oracle's does."""
    cfg = w.config("small3d")
    A, n, k = cfg["A"], cfg["A"].n, cfg["k"]
    say("partial reorth control")
    h = D.ddlr_setup(A, cfg["part"], cfg["p"], k, 1, lanczos_check=10, lanczos_start=w.lanczos_start(n, 0),
                     lanczos_reorth=D.REORTH_PARTIAL)
    o = Oracle(A, cfg["part"], cfg["p"]).set_reorth(1)
    o.lowrank(1, k, 5 * k, w.lanczos_start(n, 0), check=10, eps=1e-4)
    assert D.ddlr_query(h)["lanczos_steps"] == o.msteps
    gr, orz = D.ddlr_get_lanczos(h)[2], o.lanczos_record()[2]
    assert np.abs(gr[: k + 1] - orz[: k + 1]).max() <= 1e-8 * max(1.0, abs(orz[0]))
