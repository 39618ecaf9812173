"""GPU parity of the per-wavefront kernel of the plain passes (one axis forward or
inverse: complex, real-to-complex, complex-to-real, DCT / DST) against the FP64 oracle:
each plain pass of a power-of-two FFT length is put into launch mode 3 (16 values per
lane) and 4 (8 values per lane) through fm_plan_set_tiling, one pass at a time, on grids
whose tile counts leave a ragged last tile; strided and contiguous lines, node fix-ups,
several components."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, TOL64, check_conventions, gpu_solve, oracle_solve, rel_linf

pytestmark = pytest.mark.gpu

CASES = [
    # (n, h, bc, layout, kind): every plain kind, lengths 32 ... 128
    ([16, 32, 12], [0.1, 0.07, 0.12], [[3, 3]] * 3, F.CELL, F.POISSON),              # R2C, C2C, C2R
    ([64, 32, 14], [1 / 64, 1 / 32, 0.1], [[2, 2], [0, 1], [3, 3]], F.NODE, F.POISSON),  # R2R, R2C (cfg-like)
    ([32, 64, 10], [0.05, 0.05, 0.1], [[2, 2], [2, 2], [3, 3]], F.NODE, F.POISSON),    # periodic fix-ups
    ([16, 8, 12], [0.1, 0.1, 0.1], [[0, 3], [3, 1], [3, 3]], F.CELL, F.POISSON),       # semi-unbounded R2R
    ([32, 16, 12], [0.1, 0.1, 0.1], [[1, 1], [0, 0], [2, 2]], F.NODE, F.POISSON),      # DST-I / DCT-I
    ([16, 32, 12], [0.1, 0.07, 0.12], [[3, 3]] * 3, F.CELL, F.BIOT_SAVART),           # three components
    # first axis not x: strided first-axis lines
    ([16, 32, 12], [0.1, 0.07, 0.12], [[3, 3], [1, 1], [3, 3]], F.CELL, F.POISSON),    # DST along y
    ([24, 16, 8], [0.1, 0.1, 0.1], [[3, 3], [3, 3], [0, 3]], F.CELL, F.POISSON),       # semi-unbounded z
    ([24, 32, 8], [0.1, 0.1, 0.1], [[3, 3], [2, 2], [3, 3]], F.NODE, F.POISSON),       # R2C / C2R along y
    ([16, 32, 12], [0.1, 0.07, 0.12], [[3, 3], [2, 2], [2, 2]], F.CELL, F.BIOT_SAVART),  # 3 comps, y first
]


def _pow2_lines():
    return [1 << k for k in range(10)]


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_plain_passes_in_the_per_wavefront_kernel(case, prec, tol):
    n, h, bc, layout, kind = CASES[case]
    ncomp = 3 if kind else 1
    f = W.random_field(((3,) if kind else ()) + O.user_shape(n, layout), 60 + case)
    ref = oracle_solve(f, n, h, bc, layout, 0, kind)
    plan = F.Plan(n, h, bc, layout, F.CHAT2, prec, kind, ncomp)
    base = plan.tiling()
    err = rel_linf(gpu_solve(plan, f), ref)
    assert err < tol, ("default", err)
    ran = 0
    for p in (0, 1, 3, 4):
        for mode in (3, 4):
            for lines in _pow2_lines():
                b, q = list(base["lines_per_tile"]), list(base["persistent"])
                b[p], q[p] = lines, mode
                try:
                    t = plan.set_tiling(b, q)
                except F.FluxmiError:
                    continue
                u = gpu_solve(plan, f)
                check_conventions(u, bc, layout)
                err = rel_linf(u, ref)
                print(f"case {case} prec {prec} pass {p + 1} mode {mode} lines {lines} "
                      f"tiles {t['tiles'][p]} rel_linf={err:.2e}")
                assert err < tol, (case, p, mode, lines, err)
                ran += 1
                break
    plan.close()
    assert ran >= 4, ran


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
def test_long_lines(prec, tol):
    """FFT lengths 512 and 1024 along the first axis (unbounded, 256 and 512 cells) and
    a contiguous-line second pass."""
    for n in ([256, 6, 5], [512, 5, 4]):
        h = [1.0 / n[0], 0.1, 0.1]
        bc = [[3, 3]] * 3
        f = W.random_field(O.user_shape(n, F.CELL), 71)
        ref = oracle_solve(f, n, h, bc, F.CELL)
        plan = F.Plan(n, h, bc, F.CELL, F.CHAT2, prec)
        base = plan.tiling()
        ran = 0
        for mode in (3, 4):
            for lines in _pow2_lines():
                b, q = list(base["lines_per_tile"]), list(base["persistent"])
                b[0], q[0] = lines, mode
                b[4], q[4] = lines, mode
                try:
                    plan.set_tiling(b, q)
                except F.FluxmiError:
                    continue
                err = rel_linf(gpu_solve(plan, f), ref)
                assert err < tol, (n, mode, lines, err)
                ran += 1
                break
        plan.close()
        assert ran >= 1, n
