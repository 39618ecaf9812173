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


_TUNED_512 = {}


def _tuned_512_tiling(prec):
    """The tiling fm_plan_tune picks for the Biot-Savart 512^3 plan (the one bench.py
    times), per precision."""
    if prec not in _TUNED_512:
        import torch
        plan = F.Plan([512] * 3, [2 / 512] * 3, [[3, 3]] * 3, F.CELL, F.CHAT2, prec, F.BIOT_SAVART, 3)
        _TUNED_512[prec] = plan.tune()
        plan.close()
        torch.cuda.empty_cache()
    return _TUNED_512[prec]


@pytest.mark.parametrize("prec,tol", [(F.F32, TOL32), (F.F64, TOL64)])
@pytest.mark.parametrize("long_axis", [0, 1, 2])
def test_biot_savart_1024_lines_against_oracle(long_axis, prec, tol):
    """The kernels of the 512^3 Biot-Savart solve, against the oracle: one axis of 512
    cells (FFT length 1024, as every axis at 512^3) and two short ones.  The passes along
    the long axis run in the launch mode the tuner picks at 512^3, with as many lines per
    tile as the short axes allow; along z this is the fused curl pass, along x the first
    and last passes, along y the second and fourth."""
    n = [6, 6, 6]
    n[long_axis] = 512
    h = [2 / 512] * 3
    bc = [[3, 3]] * 3
    tuned = _tuned_512_tiling(prec)
    passes = {0: (0, 4), 1: (1, 3), 2: (2,)}[long_axis]
    plan = F.Plan(n, h, bc, F.CELL, F.CHAT2, prec, F.BIOT_SAVART, 3)
    t = plan.tiling()
    for i in passes:
        want_mode = tuned["persistent"][i]
        for b in range(tuned["lines_per_tile"][i], 0, -1):
            lines = list(t["lines_per_tile"])
            modes = list(t["persistent"])
            lines[i], modes[i] = b, want_mode
            try:
                t = plan.set_tiling(lines, modes)
                break
            except F.FluxmiError:
                continue
        assert t["persistent"][i] == want_mode, (i, t, tuned)
    rng = np.random.default_rng(1024 + long_axis)
    f = rng.standard_normal((3,) + O.user_shape(n, O.CELL))
    import torch
    x = torch.from_numpy(f).to("cuda", plan.dtype)
    u = plan.solve(x)
    torch.cuda.synchronize()
    ref = O.solve(f, n, h, bc, O.CELL, 0, 1)
    err = rel_linf(u.double().cpu().numpy(), ref)
    print(f"Biot-Savart n={n} prec={prec} tiling={t} rel_linf={err:.2e}")
    plan.close()
    assert err < tol, err
