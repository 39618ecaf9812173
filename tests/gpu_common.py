"""Helpers shared by the GPU tests: run the HIP path through the C ABI binding and the
FP64 oracle on the same seeded inputs, and measure relative L-infinity differences."""
import numpy as np

import oracle as O

TOL64 = 1e-12   # FP64 path vs FP64 oracle, relative L-inf
TOL32 = 1e-5    # FP32 path vs FP64 oracle, relative L-inf


def torch_mod():
    import torch
    return torch


def gpu_solve(plan, f64, out_dtype=None):
    torch = torch_mod()
    rhs = torch.from_numpy(np.ascontiguousarray(f64)).to(device="cuda", dtype=plan.dtype)
    rhs = rhs.reshape(plan.shape).contiguous()
    out = plan.solve(rhs)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def rel_linf(a, ref):
    s = np.abs(ref).max()
    return float(np.abs(a - ref).max() / (s if s > 0 else 1.0))


def oracle_solve(f, n, h, bc, layout, green=0, kind=0):
    return O.solve(f, n, h, bc, layout, green, kind)


def check_conventions(u, bc, layout):
    """Exact output conventions of node-centred data: nodes on odd faces are 0 and the
    periodic duplicate f_N equals f_0, along every axis (u is [..., z, y, x])."""
    if layout != 1:
        return
    for a in range(3):
        ax = u.ndim - 1 - a
        v = np.moveaxis(u, ax, -1)
        left, right = bc[a]
        if left == 2:
            assert np.array_equal(v[..., -1], v[..., 0]), f"periodic duplicate, axis {a}"
        if left == 1:
            assert np.all(v[..., 0] == 0.0), f"odd left face, axis {a}"
        if right == 1:
            assert np.all(v[..., -1] == 0.0), f"odd right face, axis {a}"
