"""Serving loop (fm_server_*): requests of mixed grids, boundary conditions and layouts
run concurrently on several streams within an HBM budget; every result equals the same
request solved alone, and the small ones match the oracle."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, oracle_solve, rel_linf

pytestmark = pytest.mark.gpu


def _shape(req):
    return tuple(v + (1 if req["layout"] == 1 else 0) for v in reversed(req["n"]))


def test_served_results_equal_alone_and_oracle():
    import torch
    reqs = W.serving_stream(count=24, qps=1e4, seed=31, edges=(32, 48, 64))
    rhs, outs = [], []
    for r in reqs:
        f = W.request_rhs(r)
        assert f.shape == _shape(r)
        rhs.append(torch.from_numpy(f).to("cuda", torch.float32))
        outs.append(torch.full(f.shape, float("nan"), dtype=torch.float32, device="cuda"))
    # cold pass: every plan is created (generated on the server's stream, each solve
    # ordered after its plan); a generous plan budget keeps them all for the warm pass
    server = F.Server(workspace_budget_bytes=96 << 20, plan_budget_bytes=1 << 30, slots=6)
    tickets = [server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o) for r, x, o in zip(reqs, rhs, outs)]
    finished = list(server.progress())
    server.wait_all()
    finished += server.progress()
    assert sorted(finished) == sorted(tickets)
    cold = [o.clone() for o in outs]
    # warm pass: plans cached, requests admitted while others run
    for o in outs:
        o.fill_(float("nan"))
    torch.cuda.synchronize()
    tickets = [server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o) for r, x, o in zip(reqs, rhs, outs)]
    finished = list(server.progress())
    server.wait_all()
    finished += server.progress()
    st = server.stats()
    print("serving stats", st)
    assert sorted(finished) == sorted(tickets)
    assert st["submitted"] == st["finished"] == 2 * len(reqs)
    assert st["plan_hits"] >= len(reqs) and st["plan_hits"] + st["plan_misses"] == 2 * len(reqs)
    assert st["peak_inflight"] > 1            # requests overlapped on the device
    assert st["peak_workspace_bytes"] <= 96 << 20
    for c, o in zip(cold, outs):
        assert torch.equal(c, o)
    server.close()
    torch.cuda.synchronize()
    for i, (r, x, o) in enumerate(zip(reqs, rhs, outs)):
        p = F.Plan(r["n"], r["h"], r["bc"], r["layout"], F.CHAT2, F.F32)
        alone = p.solve(x)
        torch.cuda.synchronize()
        assert torch.equal(alone, o), (i, r)
        p.close()
    # against the FP64 oracle (the smallest requests)
    small = sorted(range(len(reqs)), key=lambda i: np.prod(reqs[i]["n"]))[:4]
    for i in small:
        r = reqs[i]
        ref = oracle_solve(W.request_rhs(r), r["n"], r["h"], r["bc"], r["layout"])
        assert rel_linf(outs[i].double().cpu().numpy(), ref) < TOL32, (i, r)


def test_server_rejects_a_request_larger_than_its_budget():
    import torch
    server = F.Server(workspace_budget_bytes=1 << 20, plan_budget_bytes=1 << 30, slots=2)
    x = torch.zeros((65, 65, 65), dtype=torch.float32, device="cuda")
    with pytest.raises(F.FluxmiError) as e:
        server.submit([64, 64, 64], [0.1] * 3, [[3, 3]] * 3, F.NODE, x, torch.empty_like(x))
    assert e.value.status == -5
    server.close()


def test_server_evicts_plans_beyond_its_budget():
    import torch
    reqs = W.serving_stream(count=8, qps=1e4, seed=32, edges=(32, 48))
    server = F.Server(workspace_budget_bytes=64 << 20, plan_budget_bytes=1, slots=4)
    outs = []
    for r in reqs:
        x = torch.from_numpy(W.request_rhs(r)).to("cuda", torch.float32)
        o = torch.empty_like(x)
        server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o)
        outs.append((r, x, o))
    server.wait_all()
    st = server.stats()
    assert st["finished"] == len(reqs)
    assert st["plan_evictions"] >= len(reqs) - 2 and st["cached_plans"] <= 2
    for r, x, o in outs:
        p = F.Plan(r["n"], r["h"], r["bc"], r["layout"], F.CHAT2, F.F32)
        assert torch.equal(p.solve(x), o)
        p.close()
    server.close()


def test_serving_distribution_sample_matches_oracle():
    """Requests drawn from the full serving distribution (edges 32 ... 192, every class,
    both layouts), FP32 through the server, against the FP64 oracle."""
    import torch
    reqs = W.serving_stream(count=10, qps=1e4, seed=33)
    server = F.Server(workspace_budget_bytes=2 << 30, plan_budget_bytes=1 << 30, slots=4)
    work = []
    for r in reqs:
        x = W.request_rhs_device(r, torch.float32)
        o = torch.empty_like(x)
        server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o)
        work.append((r, o))
    server.wait_all()
    server.close()
    for r, o in work:
        ref = oracle_solve(W.request_rhs(r), r["n"], r["h"], r["bc"], r["layout"])
        err = rel_linf(o.double().cpu().numpy(), ref)
        print("request", r["n"], r["bc"], r["layout"], f"rel_linf={err:.2e}")
        assert err < TOL32, (r, err)


def test_requests_wait_for_their_producer_stream():
    """Warm-plan requests submitted right after an asynchronous fill of their right-hand
    sides on another stream, with no host synchronisation: each solve must see the filled
    input (its submission recorded the producer stream)."""
    import torch
    reqs = W.serving_stream(count=12, qps=1e4, seed=34, edges=(32, 48))
    server = F.Server(workspace_budget_bytes=64 << 20, plan_budget_bytes=1 << 30, slots=4)
    fields = [torch.from_numpy(W.request_rhs(r)).to("cuda", torch.float32) for r in reqs]
    rhs = [torch.zeros_like(f) for f in fields]
    outs = [torch.empty_like(f) for f in fields]
    for r, x, o in zip(reqs, rhs, outs):  # plans cached
        server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o)
    server.wait_all()
    server.progress()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    a = torch.randn(2048, 2048, device="cuda")
    with torch.cuda.stream(side):
        for r, x, f, o in zip(reqs, rhs, fields, outs):
            for _ in range(4):
                a = a @ a / 64.0  # keeps the stream busy before the fill
            x.copy_(f)
            server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o, stream=side)
    server.wait_all()
    server.progress()
    torch.cuda.synchronize()
    for r, f, o in zip(reqs, fields, outs):
        p = F.Plan(r["n"], r["h"], r["bc"], r["layout"], F.CHAT2, F.F32)
        assert torch.equal(p.solve(f), o), r
        p.close()
    server.close()


def test_a_failed_request_is_reported_finished_with_its_error(monkeypatch):
    """The error path of a request, forced from the host: the admission of one ticket is
    made to fail before anything is enqueued; that ticket finishes with FM_E_HIP, the
    others run, and wait_all returns."""
    import torch
    monkeypatch.setenv("FLUXMI_SERVER_FAIL_TICKET", "3")
    reqs = W.serving_stream(count=6, qps=1e4, seed=35, edges=(32,))
    server = F.Server(workspace_budget_bytes=64 << 20, plan_budget_bytes=1 << 30, slots=2)
    work, tickets = [], []
    for r in reqs:
        x = torch.from_numpy(W.request_rhs(r)).to("cuda", torch.float32)
        o = torch.full_like(x, float("nan"))
        tickets.append(server.submit(r["n"], r["h"], r["bc"], r["layout"], x, o))
        work.append((r, x, o))
    done = server.progress()
    server.wait_all()
    done += server.progress()
    assert sorted(done) == sorted(tickets)
    assert server.failed == {3: -6}
    st = server.stats()
    assert st["finished"] == len(reqs) and st["failed"] == 1
    for t, (r, x, o) in zip(tickets, work):
        if t == 3:
            assert torch.isnan(o).all()
            continue
        p = F.Plan(r["n"], r["h"], r["bc"], r["layout"], F.CHAT2, F.F32)
        assert torch.equal(p.solve(x), o)
        p.close()
    server.close()
