"""Runs the oracle's code paths on small inputs; tests/test_sanitizers.py
executes it with an AddressSanitizer / UndefinedBehaviorSanitizer build of
the oracle (argv[1]).  Prints "ok" at the end."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.join(ROOT, "tests")]

import numpy as np  # noqa: E402

import oracle  # noqa: E402

oracle.use_library(sys.argv[1])
import workloads as w  # noqa: E402
from oracle import Oracle, OracleError  # noqa: E402

oracle.set_threads(2)
cfg = w.config("c1")
A, n = cfg["A"], cfg["A"].n
v0 = w.lanczos_start(n, 0)
b, _ = w.rhs_from_solution(A, 0, 2)
x = np.random.default_rng(0).standard_normal((n, 3))
for factor in (0, 1):
    o = Oracle(A, cfg["part"], cfg["p"], factor=factor)
    o.ordering(), o.csr("L"), o.csr("A0"), o.csr("E"), o.diag(), o.a0_solve(x)
    for variant in (1, 2):
        for reorth in (0, 1, 2):
            o.set_reorth(reorth).lowrank(variant, cfg["k"], cfg["m"], v0)
            o.reorth_steps(), o.lanczos_record(), o.lanczos_basis(), o.apply(x)
        o.set_reorth(1).lowrank(variant, 4, 10, v0)
        o.extend(cfg["k"], 12)
        o.apply(x)
    o.set_reorth(0).lowrank(1, cfg["k"], 80, v0, check=10, eps=1e-4)
    o.pcg(b, maxit=50), o.gmres(b, restart=10, maxit=30), o.matvec(x)
    U, lam, th = o.get_lowrank()
    o.set_lowrank(1, U, lam, th)
    o.lowrank_gk(cfg["k"], cfg["m"], v0)
    o.apply(x)
o = Oracle(A, cfg["part"], cfg["p"]).use_cinv()
o.cinv(), o.a0_solve(x)
o = Oracle(A, cfg["part"], cfg["p"]).use_cheb()
o.cheb(), o.a0_solve(x)
# an indefinite shift (20 negative eigenvalues): IC(0) breaks down (a reported
# error), ILDL(0) and GMRES run
sig = w.shift_with_negatives(12, 12, 10, 20)
As = w.laplacian_3d(12, 12, 10, shift=sig)
part = w.box_partition((12, 12, 10), (2, 2, 1))
try:
    Oracle(As, part, 4)
except OracleError:
    pass
o = Oracle(As, part, 4, factor=oracle.FACTOR_ILDL).lowrank(1, 6, 12, w.lanczos_start(As.n, 1))
o.gmres(w.rhs_from_solution(As, 1, 1)[0], restart=20, maxit=60)
print("ok")
