"""ddlr_apply_noalloc (every temporary in the library's static scratch array)
against ddlr_apply on the same handle, through the C ABI.

Two calls in a row, the second with a smaller input (so that the second call
runs on scratch that still holds the first call's larger contents), then a
call with more columns than one chunk, and the refusal of a size the scratch
cannot hold.  Bar: the FP64 path agrees with ddlr_apply to 1e-12 and with the
oracle to 1e-10; the FP32 preconditioner agrees with ddlr_apply to 1e-6 and
with the oracle to 1e-4.
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


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def build(name, prec):
    cfg = w.config(name)
    v0 = w.lanczos_start(cfg["A"].n, 0)
    h = D.ddlr_setup(cfg["A"], cfg["part"], cfg["p"], cfg["k"], D.DDLR_1, lanczos_steps=cfg["m"],
                     lanczos_start=v0, precision=prec)
    o = Oracle(cfg["A"], cfg["part"], cfg["p"]).lowrank(1, cfg["k"], cfg["m"], v0)
    D.ddlr_set_lowrank(h, 1, *o.get_lowrank())  # same preconditioner on both sides
    return cfg, h, o


def noalloc(h, xt, yt):
    """Raw C-ABI call: (nrhs, n) contiguous device tensors, ld = n."""
    lib = D.load_library()
    nrhs, n = xt.shape
    st = lib.ddlr_apply_noalloc(h.handle, nrhs, xt.data_ptr(), n, yt.data_ptr(), n,
                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return st


def check(name, prec, nrhs, seed):
    cfg, h, o = build(name, prec)
    n = cfg["A"].n
    say("noalloc", name, "prec", prec, "nrhs", nrhs)
    x = np.random.default_rng(seed).standard_normal((nrhs, n))
    xt = torch.from_numpy(x).to(DEV)
    y_na = torch.full((nrhs, n), np.nan, dtype=torch.float64, device=DEV)
    assert noalloc(h, xt, y_na) == D.OK, D.load_library().ddlr_last_error()
    y_ref = torch.empty_like(y_na)
    D.ddlr_apply(h, xt, y_ref)
    torch.cuda.synchronize()
    tol_lib, tol_orc = (1e-12, 1e-10) if prec == D.FP64 else (1e-6, 1e-4)
    assert_close(y_na.cpu().numpy().T, y_ref.cpu().numpy().T, tol_lib, "noalloc vs ddlr_apply")
    assert_close(y_na.cpu().numpy().T, o.apply(x.T), tol_orc, "noalloc vs oracle")
    return h


def test_noalloc_matches_apply_two_calls_second_smaller():
    check("small3d", D.FP64, 5, 1)   # larger input first
    check("c1", D.FP32, 3, 2)        # then a smaller one, other precision


def test_noalloc_chunks_and_refusal():
    h = check("c1", D.FP64, 19, 3)   # 16 + 3 columns
    n = h.n
    xt = torch.ones((1, n), dtype=torch.float64, device=DEV)
    yt = torch.zeros((1, n), dtype=torch.float64, device=DEV)
    os.environ["DDLR_NOALLOC_CAP"] = "4096"  # lowers the usable scratch below one column
    try:
        st = noalloc(h, xt, yt)
    finally:
        os.environ.pop("DDLR_NOALLOC_CAP")
    assert st == D.E_INVALID
    assert b"scratch" in D.load_library().ddlr_last_error()
    assert float(yt.abs().max()) == 0.0  # nothing written
