"""Seeded synthetic right-hand sides shaped like the paper's test cases.

Input generators only: nothing here belongs to the solver's arithmetic, and both the
GPU path and the FP64 oracle take their inputs from these functions.  All fields are
generated in FP64 with ``numpy.random.default_rng(seed)``.

* ``gaussian_blob``  — f = exp(-r^2 / (2 sigma^2)) on a cell-centred cube (free-space
  potential known in closed form).
* ``gaussian_bumps`` — sum of 8 Gaussian bumps with sigma ~ U[0.05, 0.15], amplitudes
  ~ N(0, 1), centres uniform in the interior box [0.15, L - 0.15] per axis.
* ``vortex_ring``    — Gaussian-core vortex ring in the z = 0 plane with a seeded axial
  perturbation of the centreline (vorticity, 3 components).
* ``vortex_tubes``   — several seeded closed Gaussian-core rings with random centres,
  normals, radii, cores and circulations (vorticity, 3 components).
* ``serving_stream`` — a seeded stream of mixed-size, mixed-BC Poisson requests with
  Poisson-process arrival times.
"""
from __future__ import annotations

import numpy as np

DEFAULT_SEED = 2211


def cell_axis(N, lo, hi):
    h = (hi - lo) / N
    return lo + (np.arange(N) + 0.5) * h, h


def node_axis(N, lo, hi):
    h = (hi - lo) / N
    return lo + np.arange(N + 1) * h, h


def gaussian_blob(N=32, lo=-1.0, hi=1.0, sigma=0.1):
    """Cell-centred N^3 grid on [lo, hi]^3; returns (f[z, y, x], h)."""
    x, h = cell_axis(N, lo, hi)
    r2 = x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2
    return np.exp(-r2 / (2 * sigma ** 2)), h


def _bump_profiles(coords, L, seed, count):
    """The seeded bumps as (amplitude, gz, gy, gx) 1-D profiles."""
    rng = np.random.default_rng(seed)
    x, y, z = coords
    for _ in range(count):
        sigma = rng.uniform(0.05, 0.15)
        amp = rng.normal()
        c = [rng.uniform(0.15, La - 0.15) for La in L]
        gx = np.exp(-((x - c[0]) ** 2) / (2 * sigma ** 2))
        gy = np.exp(-((y - c[1]) ** 2) / (2 * sigma ** 2))
        gz = np.exp(-((z - c[2]) ** 2) / (2 * sigma ** 2))
        yield amp, gz, gy, gx


def gaussian_bumps(coords, L, seed=DEFAULT_SEED, count=8):
    """coords = (x, y, z) 1-D point arrays, L = (Lx, Ly, Lz); returns f[z, y, x]."""
    x, y, z = coords
    f = np.zeros((len(z), len(y), len(x)))
    for amp, gz, gy, gx in _bump_profiles(coords, L, seed, count):
        f += amp * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return f


def gaussian_bumps_device(coords, L, seed=DEFAULT_SEED, count=8, dtype=None):
    """gaussian_bumps evaluated with torch on the current GPU (same draws, FP64, then cast
    to dtype): for workloads too large to generate on the host."""
    import torch
    x, y, z = coords
    f = torch.zeros((len(z), len(y), len(x)), dtype=torch.float64, device="cuda")
    for amp, gz, gy, gx in _bump_profiles(coords, L, seed, count):
        tz, ty, tx = (torch.from_numpy(v).cuda() for v in (gz, gy, gx))
        f += amp * tz[:, None, None] * ty[None, :, None] * tx[None, None, :]
    return f if dtype is None else f.to(dtype)


def _ring_vorticity(out, x, centre, normal, R, a, gamma, zpert=None, cutoff=6.0):
    """Add the vorticity of one Gaussian-core ring (core profile gamma/(pi a^2)
    exp(-d^2/a^2) along the unit tangent) to out[3, z, y, x], on the box around it."""
    h = x[1] - x[0]
    reach = R + cutoff * a + (0.0 if zpert is None else np.abs(zpert[1]).sum() * R)
    lo = [np.searchsorted(x, centre[i] - reach) for i in range(3)]
    hi = [np.searchsorted(x, centre[i] + reach) for i in range(3)]
    sx, sy, sz = (slice(lo[i], hi[i]) for i in range(3))
    X = x[sx][None, None, :] - centre[0]
    Y = x[sy][None, :, None] - centre[1]
    Z = x[sz][:, None, None] - centre[2]
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    # orthonormal frame (e1, e2, n)
    helper = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    pa = X * e1[0] + Y * e1[1] + Z * e1[2]
    pb = X * e2[0] + Y * e2[1] + Z * e2[2]
    pn = X * n[0] + Y * n[1] + Z * n[2]
    theta = np.arctan2(pb, pa)
    rho = np.sqrt(pa ** 2 + pb ** 2)
    zc = np.zeros_like(theta)
    dzc = np.zeros_like(theta)
    if zpert is not None:
        amps, phases = zpert
        for m, (am, ph) in enumerate(zip(amps, phases), start=1):
            zc = zc + R * am * np.cos(m * theta + ph)
            dzc = dzc - R * am * m * np.sin(m * theta + ph)
    d2 = (rho - R) ** 2 + (pn - zc) ** 2
    w = gamma / (np.pi * a * a) * np.exp(-d2 / (a * a))
    w[d2 > (cutoff * a) ** 2] = 0.0
    # tangent of the centreline c(theta) = R (cos, sin) in (e1, e2) + zc n
    ta = -R * np.sin(theta)
    tb = R * np.cos(theta)
    tn = dzc
    tnorm = np.sqrt(ta ** 2 + tb ** 2 + tn ** 2)
    ta, tb, tn = ta / tnorm, tb / tnorm, tn / tnorm
    for comp in range(3):
        t = ta * e1[comp] + tb * e2[comp] + tn * n[comp]
        out[comp, sz, sy, sx] += w * t
    del h


def vortex_ring(N=256, lo=-1.0, hi=1.0, R=0.5, a=0.05, gamma=1.0, eps=1e-3, seed=DEFAULT_SEED):
    """Cell-centred N^3 grid on [lo, hi]^3: ring in the z = 0 plane, centreline
    z(theta) = eps R sum_{m=1}^{8} alpha_m cos(m theta + beta_m), alpha_m ~ N(0,1)/sqrt(8),
    beta_m ~ U[0, 2 pi).  Returns (omega[3, z, y, x], h)."""
    rng = np.random.default_rng(seed)
    alpha = rng.normal(size=8) / np.sqrt(8.0) * eps
    beta = rng.uniform(0.0, 2 * np.pi, size=8)
    x, h = cell_axis(N, lo, hi)
    out = np.zeros((3, N, N, N))
    _ring_vorticity(out, x, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), R, a, gamma, zpert=(alpha, beta))
    return out, h


def vortex_tubes(N=512, lo=-1.0, hi=1.0, count=16, seed=DEFAULT_SEED):
    """Cell-centred N^3 grid on [lo, hi]^3 with `count` closed rings: centres
    U[-0.45, 0.45]^3, normals uniform on the sphere, radii U[0.15, 0.35], cores
    U[0.02, 0.04], circulations N(0, 1); rings whose support leaves [-0.9, 0.9]^3 are
    redrawn.  Returns (omega[3, z, y, x], h)."""
    rng = np.random.default_rng(seed)
    x, h = cell_axis(N, lo, hi)
    out = np.zeros((3, N, N, N))
    placed = 0
    while placed < count:
        c = rng.uniform(-0.45, 0.45, size=3)
        nrm = rng.normal(size=3)
        R = rng.uniform(0.15, 0.35)
        a = rng.uniform(0.02, 0.04)
        g = rng.normal()
        if np.any(np.abs(c) + R + 6 * a > 0.9):
            continue
        _ring_vorticity(out, x, c, nrm, R, a, g)
        placed += 1
    return out, h


SERVING_EDGES = (32, 48, 64, 96, 128, 192)


def draw_axis_bc(rng):
    """Both faces uniform over {unbounded, periodic, even, odd}; a pair that mixes
    periodic with non-periodic is redrawn (periodic only pairs with periodic)."""
    while True:
        left, right = rng.choice([3, 2, 0, 1], size=2)
        if (left == 2) == (right == 2):
            return [int(left), int(right)]


def serving_stream(count=2000, qps=1000.0, seed=DEFAULT_SEED, h=1.0 / 64, edges=None):
    """List of request dicts: n (x, y, z), h, bc, layout, arrival time (s), seed.
    Grid edges are drawn from `edges` (default: the serving edges 32 ... 192)."""
    rng = np.random.default_rng(seed)
    edges = SERVING_EDGES if edges is None else edges
    t = 0.0
    reqs = []
    for i in range(count):
        t += rng.exponential(1.0 / qps)
        n = [int(rng.choice(edges)) for _ in range(3)]
        bc = [draw_axis_bc(rng) for _ in range(3)]
        layout = int(rng.integers(0, 2))
        reqs.append({"id": i, "n": n, "h": [h, h, h], "bc": bc, "layout": layout, "t": t,
                     "seed": seed + i})
    return reqs


def _request_grid(req):
    n, h, layout = req["n"], req["h"], req["layout"]
    coords = []
    for a in range(3):
        if layout == 1:
            coords.append(np.arange(n[a] + 1) * h[a])
        else:
            coords.append((np.arange(n[a]) + 0.5) * h[a])
    return coords, [n[a] * h[a] for a in range(3)]


def request_rhs(req):
    """The seeded Gaussian-bump right-hand side of one serving request, f[z, y, x]."""
    coords, L = _request_grid(req)
    return gaussian_bumps(coords, L, seed=req["seed"])


def request_rhs_device(req, dtype=None):
    """request_rhs generated on the current GPU."""
    coords, L = _request_grid(req)
    return gaussian_bumps_device(coords, L, seed=req["seed"], dtype=dtype)


def random_field(shape, seed):
    """Standard-normal field (parity tests over arbitrary boundary classes)."""
    return np.random.default_rng(seed).standard_normal(shape)
