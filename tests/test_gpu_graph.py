"""Batches bound to fixed buffers (fm_batch_prepare / fm_batch_run), captured in a HIP
graph and replayed: every replay must reproduce the eager result of the same inputs."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, TOL64, oracle_solve, rel_linf

pytestmark = pytest.mark.gpu

# small grids whose transform lengths use the runtime-length kernels
CASES = [
    ([12, 10, 9], [[3, 3], [2, 2], [0, 1]], F.CELL),
    ([10, 12, 14], [[3, 3], [3, 3], [3, 3]], F.NODE),
    ([9, 10, 12], [[1, 0], [3, 0], [2, 2]], F.CELL),
    ([14, 9, 10], [[0, 3], [1, 1], [3, 3]], F.NODE),
]
H = [0.11, 0.07, 0.13]


def _setup(prec):
    import torch
    plans, rhs, outs, f64 = [], [], [], []
    for i, (n, bc, layout) in enumerate(CASES):
        p = F.Plan(n, H, bc, layout, F.CHAT2, prec)
        f = W.random_field(p.shape, 70 + i)
        plans.append(p)
        f64.append(f)
        rhs.append(torch.from_numpy(f).to("cuda", p.dtype))
        outs.append(torch.empty(p.shape, dtype=p.dtype, device="cuda"))
    ws = torch.empty(F.batched_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    return plans, rhs, outs, f64, ws


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
def test_batch_graph_replays_match_eager(prec, tol):
    import torch
    plans, rhs, outs, f64, ws = _setup(prec)
    batch = F.Batch(plans, rhs, outs, ws)
    batch.run()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    for (n, bc, layout), f, u in zip(CASES, f64, eager):
        assert rel_linf(u.double().cpu().numpy(), oracle_solve(f, n, H, bc, layout)) < tol
    # eager single solves agree bitwise with the batch
    for p, r, u in zip(plans, rhs, eager):
        assert torch.equal(p.solve(r), u)
    torch.cuda.synchronize()

    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            batch.run()
    torch.cuda.synchronize()
    for rep in range(4):
        sign = -1.0 if rep % 2 == 0 else 1.0
        # the program's own eager work between replays: new inputs, cleared outputs
        for r, f in zip(rhs, f64):
            r.copy_(torch.from_numpy(sign * f).to(r.dtype))
        for o in outs:
            o.fill_(7.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, u in zip(outs, eager):
            # the solve is linear and its arithmetic is odd in the input: exact sign flip
            assert torch.equal(o, sign * u), rep
    batch.close()
    for p in plans:
        p.close()


def test_single_solve_graph_replays_match_eager():
    import torch
    n, bc, layout = [12, 10, 14], [[3, 3], [2, 2], [3, 3]], F.CELL
    p = F.Plan(n, H, bc, layout, F.CHAT2, F.F64)
    f = W.random_field(p.shape, 5)
    x = torch.from_numpy(f).cuda()
    out = torch.empty_like(x)
    ws = torch.empty(p.workspace_bytes, dtype=torch.uint8, device="cuda")
    p.solve(x, out, ws)
    torch.cuda.synchronize()
    eager = out.clone()
    assert rel_linf(eager.cpu().numpy(), oracle_solve(f, n, H, bc, layout)) < TOL64
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            p.solve(x, out, ws)
    for rep in range(3):
        out.zero_()
        x.mul_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager * (-1.0 if rep % 2 == 0 else 1.0)), rep
    p.close()
