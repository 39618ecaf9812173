"""Autotuned plans (fm_plan_tune): the tuned tiling is valid, results stay within the
parity tolerance of the oracle, and batches of tuned plans equal their single solves."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, TOL64, gpu_solve, oracle_solve, rel_linf

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
def test_tuned_mixed_node_128x128x256(prec, tol):
    n, h = [128, 128, 256], [1 / 128] * 3
    bc = [[2, 2], [0, 1], [3, 3]]
    coords = [np.arange(n[a] + 1) * h[a] for a in range(3)]
    f = W.gaussian_bumps(coords, [1.0, 1.0, 2.0])
    ref = oracle_solve(f, n, h, bc, O.NODE)
    plan = F.Plan(n, h, bc, F.NODE, F.CHAT2, prec)
    before = plan.tiling()
    after = plan.tune()
    print(f"prec={prec} tiling before {before} after {after}")
    for i in range(5):
        assert 1 <= after["lines_per_tile"][i] <= 64
    err = rel_linf(gpu_solve(plan, f), ref)
    assert err < tol, err
    plan.close()


def test_tuned_small_plans_batch_equals_single():
    import torch
    cases = [([12, 10, 9], [[3, 3], [2, 2], [0, 1]], F.CELL),
             ([10, 12, 14], [[3, 3], [3, 3], [3, 3]], F.NODE)]
    h = [0.11, 0.07, 0.13]
    plans, rhs = [], []
    for i, (n, bc, layout) in enumerate(cases):
        p = F.Plan(n, h, bc, layout, F.CHAT2, F.F64)
        p.tune()
        f = W.random_field(p.shape, 90 + i)
        assert rel_linf(gpu_solve(p, f), oracle_solve(f, n, h, bc, layout)) < TOL64
        plans.append(p)
        rhs.append(torch.from_numpy(f).cuda())
    singles = [p.solve(r) for p, r in zip(plans, rhs)]
    outs = [torch.empty_like(r) for r in rhs]
    ws = torch.empty(F.batched_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    F.solve_batched(plans, rhs, outs, ws)
    torch.cuda.synchronize()
    for s, o in zip(singles, outs):
        assert torch.equal(s, o)
    for p in plans:
        p.close()
