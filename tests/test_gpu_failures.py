"""Failure paths of plan creation, forced from the host: with FLUXMI_FAIL_ALLOC=k the
k-th device allocation of plan creation reports out-of-memory.  Every k up to the last
allocation must fail cleanly with FM_E_NOMEM (nothing leaked, nothing left queued), and
plans created afterwards must solve correctly."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, gpu_solve, oracle_solve, rel_linf

pytestmark = pytest.mark.gpu

FM_E_NOMEM = -5

CONFIGS = [
    # (n, h, bc, layout, green, kind): the allocations of each generation path
    ([24, 20, 16], [0.05, 0.06, 0.07], [[2, 2], [0, 1], [3, 3]], F.NODE, F.CHAT2, F.POISSON),
    ([16, 16, 16], [0.05] * 3, [[3, 3]] * 3, F.CELL, F.LGF2, F.POISSON),
    ([16, 12, 16], [0.05] * 3, [[3, 3], [2, 2], [3, 3]], F.CELL, F.CHAT2, F.BIOT_SAVART),
]


@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_every_allocation_failure_of_plan_creation(cfg, monkeypatch):
    import torch
    n, h, bc, layout, green, kind = CONFIGS[cfg]
    ncomp = 3 if kind else 1
    f = W.random_field(((3,) if kind else ()) + O.user_shape(n, layout), 90 + cfg)
    # warm-up: the runtime's own first-use allocations (code objects, scratch) happen here
    warm = F.Plan(n, h, bc, layout, green, F.F32, kind, ncomp)
    gpu_solve(warm, f)
    warm.close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    for k in range(1, 64):
        monkeypatch.setenv("FLUXMI_FAIL_ALLOC", str(k))
        try:
            plan = F.Plan(n, h, bc, layout, green, F.F32, kind)
        except F.FluxmiError as e:
            assert e.status == FM_E_NOMEM, (k, e.status)
            failures += 1
            continue
        plan.close()
        break
    else:
        pytest.fail("plan creation never succeeded")
    monkeypatch.delenv("FLUXMI_FAIL_ALLOC")
    assert failures >= 5, failures
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (16 << 20), (free0, free1)  # no device memory kept by failed plans
    plan = F.Plan(n, h, bc, layout, green, F.F32, kind, ncomp)
    err = rel_linf(gpu_solve(plan, f), oracle_solve(f, n, h, bc, layout, green, kind))
    plan.close()
    assert err < TOL32, err
