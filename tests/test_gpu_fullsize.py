"""Parity at the benchmark sizes, in the configuration bench.py times (tuned plans).

* unbounded cell 512^3, scalar Poisson: sampled outputs against the oracle's direct
  convolution sum, point by point;
* Biot-Savart vortex ring, cell 256^3: the whole field against the FP64 oracle;
* Biot-Savart vortex tubes, cell 512^3: FP32 against FP64 on the GPU (a consistency
  property; the oracle's full field at 1024^3 padded is out of reach here)."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import workloads as W

from gpu_common import TOL32, TOL64, rel_linf

pytestmark = pytest.mark.gpu


def _solve(n, h, bc, layout, kind, f64, prec):
    import torch
    ncomp = 3 if kind == 1 else 1
    plan = F.Plan(n, h, bc, layout, F.CHAT2, prec, kind, ncomp)
    plan.tune()  # the tiling bench.py times
    x = torch.from_numpy(f64).to("cuda", plan.dtype).reshape(plan.shape).contiguous()
    u = plan.solve(x)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    plan.close()
    del x, u
    torch.cuda.empty_cache()
    return out


def test_unbounded_cell_512_sampled_direct_sums():
    n, h, bc = [512] * 3, [2 / 512] * 3, [[3, 3]] * 3
    f = W.gaussian_blob(512, sigma=0.1)[0]
    rng = np.random.default_rng(512)
    pts = [(256, 256, 256), (255, 256, 257), (0, 0, 0), (511, 511, 511), (0, 511, 255), (300, 200, 256)]
    pts += [tuple(int(v) for v in rng.integers(0, 512, size=3)) for _ in range(10)]
    ref = O.direct_points(f, n, h, bc, 0, pts)
    scale = np.abs(ref).max()
    for prec, tol in ((F.F64, TOL64), (F.F32, TOL32)):
        u = _solve(n, h, bc, 0, 0, f, prec)
        got = np.array([u[z, y, x] for (x, y, z) in pts])
        err = float(np.abs(got - ref).max() / scale)
        print(f"512^3 scalar prec={prec} sampled rel err {err:.2e}")
        assert err < tol, err


def test_biot_savart_ring_256_full_field():
    n, h, bc = [256] * 3, [2 / 256] * 3, [[3, 3]] * 3
    f = W.vortex_ring(256)[0]
    ref = O.solve(f, n, h, bc, 0, 0, 1)
    for prec, tol in ((F.F64, TOL64), (F.F32, TOL32)):
        u = _solve(n, h, bc, 0, 1, f, prec)
        err = rel_linf(u, ref)
        print(f"ring 256^3 prec={prec} rel_linf {err:.2e}")
        assert err < tol, err


def test_biot_savart_tubes_512_fp32_matches_fp64():
    n, h, bc = [512] * 3, [2 / 512] * 3, [[3, 3]] * 3
    f = W.vortex_tubes(512)[0]
    u64 = _solve(n, h, bc, 0, 1, f, F.F64)
    u32 = _solve(n, h, bc, 0, 1, f, F.F32)
    err = rel_linf(u32, u64)
    print(f"tubes 512^3 FP32 vs FP64 rel_linf {err:.2e}")
    assert err < TOL32, err
    assert np.all(np.isfinite(u64))
