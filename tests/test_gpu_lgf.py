"""GPU parity of the lattice Green's function LGF2 (Sec. IV) against the FP64 oracle:
fully and semi-unbounded domains (the lattice kernel sampled on the device), spectral
domains (the inverse second-difference symbol), Poisson and Biot-Savart, both layouts and
precisions; the printed LGF2 error of the unbounded validation reproduced on the GPU; and
at 96^3 the property that holds at any size: the 7-point Laplacian of the solution is the
right-hand side."""
import json
import os

import numpy as np
import pytest

import analytic as A
import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, TOL64, check_conventions, gpu_solve, oracle_solve, rel_linf

pytestmark = pytest.mark.gpu

DOMAINS = [
    [[3, 3]] * 3,
    [[0, 3], [3, 1], [3, 3]],
    [[2, 2], [2, 2], [2, 2]],
    [[2, 2], [0, 1], [1, 1]],
]


def _case(n, h, bc, layout, prec, seed, kind=0):
    f = W.random_field(((3,) if kind else ()) + O.user_shape(n, layout), seed)
    ref = oracle_solve(f, n, h, bc, layout, F.LGF2, kind)
    plan = F.Plan(n, h, bc, layout, F.LGF2, prec, kind, 3 if kind else 1)
    u = gpu_solve(plan, f)
    plan.close()
    check_conventions(u, bc, layout)
    return rel_linf(u, ref)


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
def test_poisson_every_domain(prec, tol):
    for layout in (F.CELL, F.NODE):
        for i, bc in enumerate(DOMAINS):
            err = _case([12, 10, 14], [0.1, 0.12, 0.09], bc, layout, prec, 50 + i)
            print(f"LGF2 prec={prec} layout={layout} bc={bc} rel_linf={err:.2e}")
            assert err < tol, (bc, layout, prec, err)


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
def test_biot_savart(prec, tol):
    for layout in (F.CELL, F.NODE):
        for bc in ([[3, 3]] * 3, [[2, 2]] * 3):
            err = _case([12, 10, 16], [0.1, 0.12, 0.09], bc, layout, prec, 9, kind=F.BIOT_SAVART)
            assert err < tol, (bc, layout, prec, err)


def test_printed_unbounded_error_on_the_gpu():
    """The FP64 GPU solve of the fully unbounded validation at N = 32 and 64 gives the
    E_inf the paper prints for LGF2."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_lgf2_errors.json")) as fh:
        g = json.load(fh)["unbounded"]
    for N in (32, 64):
        f, phi, bc = A.app_b_unbounded(N)
        plan = F.Plan([N] * 3, [1.0 / N] * 3, bc, F.NODE, F.LGF2, F.F64)
        err = np.abs(gpu_solve(plan, f) - phi).max()
        plan.close()
        assert err == pytest.approx(g["E_inf"][str(N)], rel=1e-9), (N, err)


def test_discrete_laplacian_of_the_solution_at_96():
    """Fully unbounded cell 96^3, FP64: the 7-point Laplacian of u equals f at every
    interior point (LGF2 inverts the discrete operator on the unbounded lattice)."""
    n, h = [96, 96, 96], [1.0 / 96] * 3
    f = W.gaussian_blob(96)[0]
    plan = F.Plan(n, h, [[3, 3]] * 3, F.CELL, F.LGF2, F.F64)
    u = gpu_solve(plan, f)
    plan.close()
    c = u[1:-1, 1:-1, 1:-1]
    lap = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1] +
           u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2] - 6 * c) / h[0] ** 2
    err = np.abs(lap - f[1:-1, 1:-1, 1:-1]).max() / np.abs(f).max()
    print(f"LGF2 96^3 discrete Laplacian residual {err:.2e}")
    assert err < 1e-10
