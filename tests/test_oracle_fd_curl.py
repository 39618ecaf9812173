"""Pins of the oracle's finite-difference Biot-Savart solve (Sec. V: the derivative of
the spectral curl replaced by the symbol of a central difference of order 2, 4 or 6).

The same result is formed independently: the curl is taken on the grid by explicit
central-difference stencils (the textbook coefficients, applied with periodic wrap), and
each component of that curl is handed to the oracle's Poisson solve.  Both must agree to
roundoff on periodic grids, and on unbounded grids whenever the field vanishes within the
stencil radius of the boundary (the stencil then stays inside the data and the domain
doubling sees the same field).  On a Gaussian column the error still converges at the
kernel's second order for every stencil.
"""
import numpy as np
import pytest

import analytic as A
import oracle as O

# f'(x) ~ sum_j c_j (f(x + j h) - f(x - j h)) / h
STENCILS = {2: [0.5], 4: [2 / 3, -1 / 12], 6: [0.75, -0.15, 1 / 60]}
KIND = {2: 2, 4: 3, 6: 4}


def d_dx(f, axis_pos, h, order):
    """Central difference along physical axis axis_pos (0 = x, the last array axis)."""
    ax = f.ndim - 1 - axis_pos
    out = np.zeros_like(f)
    for j, c in enumerate(STENCILS[order], start=1):
        out += c * (np.roll(f, -j, axis=ax) - np.roll(f, j, axis=ax)) / h
    return out


def stencil_curl(f, h, order):
    fx, fy, fz = f
    return np.stack([d_dx(fz, 1, h[1], order) - d_dx(fy, 2, h[2], order),
                     d_dx(fx, 2, h[2], order) - d_dx(fz, 0, h[0], order),
                     d_dx(fy, 0, h[0], order) - d_dx(fx, 1, h[1], order)])


def _poisson3(g, n, h, bc, layout):
    return np.stack([O.solve(g[c], n, h, bc, layout) for c in range(3)])


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_periodic_equals_stencil_curl_then_poisson(order, layout):
    n, h = [8, 7, 6], [0.11, 0.13, 0.09]
    bc = [[2, 2]] * 3
    f = np.random.default_rng(order + 10 * layout).standard_normal((3,) + O.user_shape(n, layout))
    if layout == O.NODE:  # the duplicate nodes repeat the first ones (the periodic field)
        f[..., -1] = f[..., 0]
        f[..., -1, :] = f[..., 0, :]
        f[:, -1] = f[:, 0]
    core = f[:, :n[2], :n[1], :n[0]]
    ref = _poisson3(stencil_curl(core, h, order), n, h, bc, O.CELL)
    for mode in (O.FAST, O.NAIVE):
        u = O.solve(f, n, h, bc, layout, 0, KIND[order], mode)[:, :n[2], :n[1], :n[0]]
        assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max(), (order, layout, mode)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_unbounded_compact_field_equals_stencil_curl_then_poisson(order):
    n, h = [14, 12, 16], [0.1, 0.12, 0.08]
    for bc in ([[3, 3]] * 3, [[2, 2], [3, 3], [3, 3]], [[3, 3], [2, 2], [2, 2]]):
        rng = np.random.default_rng(order)
        f = rng.standard_normal((3,) + O.user_shape(n, O.CELL))
        r = 3  # zero within the stencil radius of every unbounded face
        for a in range(3):
            if bc[a][0] == 3:
                ax = 3 - a
                idx = [slice(None)] * 4
                idx[ax] = slice(0, r)
                f[tuple(idx)] = 0
                idx[ax] = slice(-r, None)
                f[tuple(idx)] = 0
        ref = _poisson3(stencil_curl(f, h, order), n, h, bc, O.CELL)
        u = O.solve(f, n, h, bc, O.CELL, 0, KIND[order])
        assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max(), (order, bc)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_gaussian_column_second_order(order):
    sigma, errs = 0.1, []
    for N in (32, 64):
        x, h = A.cell_coords(N, -1.0, 1.0)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        g = np.exp(-r ** 2 / (2 * sigma ** 2))
        f = np.stack([np.zeros_like(g), np.zeros_like(g), g])
        ref = A.gaussian_column_velocity(X, Y, Z, sigma)
        u = O.solve(f, [N] * 3, [h] * 3, [[3, 3]] * 3, O.CELL, 1, KIND[order])
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    assert 1.6 < np.log2(errs[0] / errs[1]) < 2.6, errs
