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


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    """FLUXMI_TUNE_CACHE: the first tune times and appends one line; a new plan of the same
    problem applies that line without timing and gets the same tiling and the same
    result; an entry that does not validate for the plan is ignored (the plan is tuned)."""
    import torch
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("FLUXMI_TUNE_CACHE", str(path))
    n, h, bc = [64, 48, 40], [0.02, 0.03, 0.025], [[2, 2], [0, 1], [3, 3]]
    f = W.random_field(O.user_shape(n, O.NODE), 77)
    a = F.Plan(n, h, bc, F.NODE, F.CHAT2, F.F32)
    ta = a.tune()
    assert not a.tuned_from_cache()
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and " B" in lines[0] and " M" in lines[0]
    b = F.Plan(n, h, bc, F.NODE, F.CHAT2, F.F32)
    tb = b.tune()
    assert b.tuned_from_cache() and tb == ta
    ua, ub = gpu_solve(a, f), gpu_solve(b, f)
    assert np.array_equal(ua, ub)
    # a different problem has its own entry
    c = F.Plan(n, h, bc, F.NODE, F.CHAT2, F.F64)
    c.tune()
    assert not c.tuned_from_cache() and len(path.read_text().splitlines()) == 2
    # a corrupted tiling for this key is not applied
    key = lines[0].split(" B")[0]
    path.write_text(key + " B1000,1,1,1,1 M0,0,0,0,0\n")
    d = F.Plan(n, h, bc, F.NODE, F.CHAT2, F.F32)
    d.tune()
    assert not d.tuned_from_cache()
    for p in (a, b, c, d):
        p.close()
    torch.cuda.synchronize()
