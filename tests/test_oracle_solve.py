"""Pins for the oracle's solve (CPU only).

* Table I / Sec. II-B / Sec. II-C class table as the oracle builds it.
* All 10^3 per-axis class combinations x 2 layouts: fast (own FFT) == naive (defining
  sums) == direct (real-space convolution with explicit images) on tiny grids.
* The CHAT2 errors printed in Sec. IV (App. B fields) to 12 significant digits.
* Closed-form free-space solutions for Gaussian sources with 3, 2 and 1 convolution
  directions and for the Biot-Savart velocity of a Gaussian column: second order.
* Invariants: linearity, output symmetry, real and even Green's spectrum, axis
  permutation, zero mean without a convolution direction.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy import integrate, special

import analytic as A
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_chat2_errors.json")
PAIRS = [(2, 2), (0, 0), (1, 1), (0, 1), (1, 0), (3, 3), (0, 3), (1, 3), (3, 0), (3, 1)]
CLASS_OF_PAIR = ["P", "EE", "OO", "EO", "OE", "UU", "EU", "OU", "UE", "UO"]


# ---------------------------------------------------------------------------------
def test_class_table_matches_table_I():
    N, h = 8, 0.1
    # Table I: forward transform of each symmetric class per layout
    node = {"EE": O.REDFT00, "OO": O.RODFT00, "OE": O.RODFT01, "EO": O.REDFT01}
    cell = {"EE": O.REDFT10, "OO": O.RODFT10, "OE": O.RODFT11, "EO": O.REDFT11}
    for (bl, br), name in zip(PAIRS, CLASS_OF_PAIR):
        for layout, table in ((O.NODE, node), (O.CELL, cell)):
            d = O.axis_info(N, h, layout, bl, br)
            assert d["cls_name"] == name
            assert d["nuser"] == N + (1 if layout == O.NODE else 0)
            if name in table:
                assert d["fwd"] == table[name]
                assert d["nlog"] == 2 * N
            if name == "P":
                assert (d["nspec"], d["nlog"], d["dft"]) == (N, N, 1)
            if name == "UU":
                assert (d["nspec"], d["nlog"], d["dft"], d["unb"]) == (2 * N, 2 * N, 1, 1)
            if name in ("EU", "OU", "UE", "UO"):
                assert d["nlog"] == 4 * N and d["unb"] == 1
                assert d["rev"] == (name in ("UE", "UO"))
    # node spectral sizes: DCT-I N+1 outputs, DST-I N-1 (Sec. II-B)
    assert O.axis_info(N, h, O.NODE, 0, 0)["nspec"] == N + 1
    assert O.axis_info(N, h, O.NODE, 1, 1)["nspec"] == N - 1
    # periodic on one face only is not a valid pair
    for other in (0, 1, 3):
        with pytest.raises(ValueError):
            O.axis_info(N, h, O.NODE, 2, other)
        with pytest.raises(ValueError):
            O.axis_info(N, h, O.CELL, other, 2)


# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_all_class_combinations_three_ways(layout):
    n, h = [3, 4, 5], [0.3, 0.25, 0.2]
    rng = np.random.default_rng(11 + layout)
    shp = O.user_shape(n, layout)
    worst_fast, worst_direct = 0.0, 0.0
    for combo in itertools.product(PAIRS, repeat=3):
        f = rng.standard_normal(shp)
        a = O.solve(f, n, h, combo, layout, 0, 0, O.FAST)
        b = O.solve(f, n, h, combo, layout, 0, 0, O.NAIVE)
        c = O.solve(f, n, h, combo, layout, 0, 0, O.DIRECT)
        s = np.abs(b).max()
        worst_fast = max(worst_fast, np.abs(a - b).max() / s)
        worst_direct = max(worst_direct, np.abs(c - b).max() / s)
    assert worst_fast < 1e-13
    assert worst_direct < 1e-12


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
@pytest.mark.parametrize("green", [0, 1])
def test_direct_sum_bigger_grid(layout, green):
    """Fully unbounded and one mixed case at a size where wrap-around would show."""
    n, h = [6, 7, 5], [0.11, 0.13, 0.09]
    rng = np.random.default_rng(3)
    shp = O.user_shape(n, layout)
    for bc in ([[3, 3]] * 3, [[3, 0], [2, 2], [1, 3]], [[3, 3], [0, 1], [3, 3]]):
        f = rng.standard_normal(shp)
        a = O.solve(f, n, h, bc, layout, green, 0, O.FAST)
        c = O.solve(f, n, h, bc, layout, green, 0, O.DIRECT)
        assert np.abs(a - c).max() / np.abs(c).max() < 1e-12


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_biot_savart_fast_vs_naive(layout):
    n, h = [4, 6, 5], [0.2, 0.15, 0.1]
    rng = np.random.default_rng(7)
    shp = (3,) + O.user_shape(n, layout)
    for combo in itertools.product([(2, 2), (3, 3)], repeat=3):
        f = rng.standard_normal(shp)
        a = O.solve(f, n, h, combo, layout, 0, 1, O.FAST)
        b = O.solve(f, n, h, combo, layout, 0, 1, O.NAIVE)
        assert np.abs(a - b).max() / np.abs(b).max() < 1e-13
    with pytest.raises(ValueError):  # curl only on periodic / fully unbounded axes
        O.solve(f, n, h, [[0, 0], [3, 3], [3, 3]], layout, 0, 1)


# ---------------------------------------------------------------------------------
def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.mark.parametrize("case,maker", [("unbounded", A.app_b_unbounded), ("semi", A.app_b_semi)])
@pytest.mark.parametrize("N", [32, 64])
def test_paper_chat2_errors(case, maker, N):
    g = _golden()[case]
    f, phi, bc = maker(N)
    assert bc == g["bc"]
    u = O.solve(f, [N] * 3, [1.0 / N] * 3, bc, O.NODE, 0, 0)
    err = np.abs(u - phi).max()
    assert err == pytest.approx(g["E_inf"][str(N)], rel=1e-11)


@pytest.mark.slow
@pytest.mark.parametrize("case,maker", [("unbounded", A.app_b_unbounded), ("semi", A.app_b_semi)])
def test_paper_chat2_errors_128(case, maker):
    g = _golden()[case]
    f, phi, bc = maker(128)
    u = O.solve(f, [128] * 3, [1.0 / 128] * 3, bc, O.NODE, 0, 0)
    assert np.abs(u - phi).max() == pytest.approx(g["E_inf"]["128"], rel=1e-10)


@pytest.mark.parametrize("N", [32, 64])
def test_paper_spectral_case_exact(N):
    g = _golden()["spectral"]
    f, phi, bc = A.app_b_spectral(N)
    u = O.solve(f, [N] * 3, [1.0 / N] * 3, bc, O.NODE, 0, 0)
    # the paper reports roundoff-level errors (<= ~2.2e-15) at every resolution
    assert np.abs(u - phi).max() < 2 * g["E_inf_max"]


def test_sphere_mean_self_term_gives_different_errors():
    """Green 1 (sphere mean without the extra cell volume) does not reproduce the
    printed CHAT2 values: the printed values pin green 0."""
    g = _golden()["unbounded"]
    f, phi, bc = A.app_b_unbounded(32)
    u = O.solve(f, [32] * 3, [1.0 / 32] * 3, bc, O.NODE, 1, 0)
    assert abs(np.abs(u - phi).max() - g["E_inf"]["32"]) > 1e-3


# ---------------------------------------------------------------------------------
def _gauss_case(N, sigma=0.1):
    x, h = A.cell_coords(N, -1.0, 1.0)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    return X, Y, Z, r, h


@pytest.mark.parametrize("green,expect", [(0, (7.86e-2, 2.14e-2)), (1, (1.05e-2, 3.08e-3))])
def test_gaussian_source_3d_second_order(green, expect):
    errs = []
    for N in (32, 64):
        X, Y, Z, r, h = _gauss_case(N)
        f = np.exp(-r ** 2 / (2 * 0.1 ** 2))
        ref = A.gaussian_potential_3d(r, 0.1)
        u = O.solve(f, [N] * 3, [h] * 3, [[3, 3]] * 3, O.CELL, green, 0)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    assert errs[0] == pytest.approx(expect[0], rel=0.01)
    assert errs[1] == pytest.approx(expect[1], rel=0.01)
    assert 1.7 < np.log2(errs[0] / errs[1]) < 2.3


def test_biot_savart_gaussian_column_second_order():
    sigma = 0.1
    errs = []
    for N in (32, 64):
        X, Y, Z, r, h = _gauss_case(N, sigma)
        g = np.exp(-r ** 2 / (2 * sigma ** 2))
        f = np.stack([np.zeros_like(g), np.zeros_like(g), g])
        ref = A.gaussian_column_velocity(X, Y, Z, sigma)
        u = O.solve(f, [N] * 3, [h] * 3, [[3, 3]] * 3, O.CELL, 1, 1)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    order = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-2
    assert 1.7 < order < 2.4


def test_one_convolution_direction_closed_form():
    """x, y periodic; z unbounded: f = (1 + cos(2 pi x / Lx)) exp(-z^2/(2 s^2))."""
    sigma, Lx = 0.1, 1.0
    errs = []
    for N in (32, 64):
        hx = Lx / N
        x = np.arange(N) * hx
        z, hz = A.cell_coords(N, -1.0, 1.0)
        k = 2 * np.pi / Lx
        gz = np.exp(-z ** 2 / (2 * sigma ** 2))
        f = np.broadcast_to(gz[:, None, None] * (1 + np.cos(k * x))[None, None, :], (N, 8, N)).copy()
        ref_z0 = A.gaussian_1unb(z, 0.0, sigma)
        ref_zk = A.gaussian_1unb(z, k, sigma)
        ref = ref_z0[:, None, None] + ref_zk[:, None, None] * np.cos(k * x)[None, None, :]
        ref = np.broadcast_to(ref, f.shape)
        u = O.solve(f, [N, 8, N], [hx, 0.125, hz], [[2, 2], [2, 2], [3, 3]], O.CELL, 0, 0)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    assert errs[1] < 2e-3
    assert 1.8 < np.log2(errs[0] / errs[1]) < 2.3


def test_two_convolution_directions_closed_form():
    """x, y unbounded; z periodic: f = (1 + cos(2 pi z / Lz)) exp(-rho^2/(2 s^2))."""
    sigma, Lz = 0.1, 1.0
    k = 2 * np.pi / Lz
    table = np.linspace(0.0, 1.6, 321)
    Uk_tab = A.gaussian_2unb_k(table, k, sigma)
    errs = []
    for N in (32, 64):
        x, h = A.cell_coords(N, -0.8, 0.8)
        hz = Lz / 8
        zz = np.arange(8) * hz
        Yg, Xg = np.meshgrid(x, x, indexing="ij")
        rho = np.sqrt(Xg ** 2 + Yg ** 2)
        g = np.exp(-rho ** 2 / (2 * sigma ** 2))
        f = g[None, :, :] * (1 + np.cos(k * zz))[:, None, None]
        U0 = A.gaussian_2unb_k0(rho, sigma)
        Uk = np.interp(rho, table, Uk_tab)
        ref = U0[None] + Uk[None] * np.cos(k * zz)[:, None, None]
        u = O.solve(f, [N, N, 8], [h, h, hz], [[3, 3], [3, 3], [2, 2]], O.CELL, 0, 0)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    assert errs[1] < 2e-3
    assert 1.6 < np.log2(errs[0] / errs[1]) < 2.6


# ---------------------------------------------------------------------------------
def test_self_terms():
    h = 0.05
    vol3 = h ** 3
    r_eq3 = (3 * vol3 / (4 * np.pi)) ** (1 / 3)
    sphere = -3 / (8 * np.pi * r_eq3)
    # sphere mean of -1/(4 pi r) over the equal-volume ball, by quadrature
    mean, _ = integrate.quad(lambda r: -1 / (4 * np.pi * r) * 4 * np.pi * r * r, 0, r_eq3)
    assert sphere == pytest.approx(mean / (4 / 3 * np.pi * r_eq3 ** 3), rel=1e-12)
    assert O.green_value(3, 1, vol3, 0.0, 0.0) == pytest.approx(sphere, rel=1e-14)
    assert O.green_value(3, 0, vol3, 0.0, 0.0) == pytest.approx(sphere * vol3, rel=1e-14)
    assert O.green_value(3, 0, vol3, 0.7, 0.0) == pytest.approx(-1 / (4 * np.pi * 0.7), rel=1e-15)
    # d_u = 2, k = 0: mean of ln(rho)/(2 pi) over the square cell of side h
    tri = lambda t: ((0.5 * h / np.cos(t)) ** 2 / 2 * np.log(0.5 * h / np.cos(t)) - (0.5 * h / np.cos(t)) ** 2 / 4)
    sq, _ = integrate.quad(tri, 0, np.pi / 4, epsabs=1e-15)
    sq = 8 * sq / h ** 2 / (2 * np.pi)
    assert O.green_value(2, 0, h * h, 0.0, 0.0) == pytest.approx(sq, rel=1e-12)
    # d_u = 2, k > 0: mean of -K0(k rho)/(2 pi) over the disc of area h^2
    k = 7.0
    R = h / np.sqrt(np.pi)
    disc, _ = integrate.quad(lambda r: -special.k0(k * r) / (2 * np.pi) * 2 * np.pi * r, 0, R, epsabs=1e-16)
    assert O.green_value(2, 0, h * h, 0.0, k) == pytest.approx(disc / (np.pi * R * R), rel=1e-10)
    assert O.green_value(2, 0, h * h, 0.3, k) == pytest.approx(-special.k0(k * 0.3) / (2 * np.pi), rel=1e-13)
    assert O.green_value(1, 0, h, 0.3, k) == pytest.approx(-np.exp(-k * 0.3) / (2 * k), rel=1e-14)
    assert O.green_value(1, 0, h, 0.3, 0.0) == pytest.approx(0.15, rel=1e-15)
    assert O.green_value(0, 0, 1.0, 0.0, 2.0) == pytest.approx(-0.25, rel=1e-15)
    assert O.green_value(0, 0, 1.0, 0.0, 0.0) == 0.0


# ---------------------------------------------------------------------------------
def _mirror_check(u, axis_pos, cls, node):
    """Return max violation of the class's parity at the faces, for axis of u at
    position axis_pos (0 = last array axis, x)."""
    ax = u.ndim - 1 - axis_pos
    v = np.moveaxis(u, ax, -1)
    viol = 0.0
    if node:
        if cls[0] == "O":
            viol = max(viol, np.abs(v[..., 0]).max())
        if cls[1] == "O":
            viol = max(viol, np.abs(v[..., -1]).max())
    return viol


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_invariants(layout):
    n, h = [6, 5, 4], [0.2, 0.3, 0.25]
    rng = np.random.default_rng(99)
    shp = O.user_shape(n, layout)
    for combo in ([[1, 1], [0, 1], [1, 0]], [[1, 3], [3, 1], [2, 2]], [[3, 3], [1, 1], [0, 3]]):
        f, g = rng.standard_normal(shp), rng.standard_normal(shp)
        a, b = 1.7, -0.3
        uf = O.solve(f, n, h, combo, layout)
        ug = O.solve(g, n, h, combo, layout)
        ufg = O.solve(a * f + b * g, n, h, combo, layout)
        assert np.abs(ufg - (a * uf + b * ug)).max() < 1e-12 * np.abs(ufg).max()
        for axp, pair in enumerate(combo):
            cls = "".join("EOPU"[p] for p in pair)
            assert _mirror_check(uf, axp, cls, layout == O.NODE) == 0.0
    # zero mean without a convolution direction (mean of f discarded)
    combo = [[2, 2], [0, 0], [2, 2]]
    f = rng.standard_normal(O.user_shape(n, O.CELL))
    u = O.solve(f, n, h, combo, O.CELL)
    assert abs(u.mean()) < 1e-14 * np.abs(u).max()
    # node periodic duplicate equals the first point
    u = O.solve(rng.standard_normal(O.user_shape(n, O.NODE)), n, h, [[2, 2], [3, 3], [3, 3]], O.NODE)
    assert np.array_equal(u[..., -1], u[..., 0])


def test_green_spectrum_real_and_even():
    n, h = [6, 5, 4], [0.2, 0.3, 0.25]
    G = O.green_spectrum(n, h, [[3, 3], [3, 3], [3, 3]], O.CELL)
    assert np.abs(G.imag).max() == 0.0
    for ax, N in zip((2, 1, 0), n):
        k = np.arange(2 * N)
        flipped = np.take(G, (-k) % (2 * N), axis=ax)
        assert np.abs(flipped - G).max() < 1e-15 * np.abs(G).max()


def test_axis_permutation_equivariance():
    n, h = [6, 5, 4], [0.2, 0.3, 0.25]
    bc = [[3, 3], [0, 3], [1, 1]]
    rng = np.random.default_rng(5)
    f = rng.standard_normal(O.user_shape(n, O.NODE))
    u = O.solve(f, n, h, bc, O.NODE)
    # swap x and z: array axes (z, y, x) -> (x, y, z)
    n2, h2, bc2 = [n[2], n[1], n[0]], [h[2], h[1], h[0]], [bc[2], bc[1], bc[0]]
    u2 = O.solve(np.ascontiguousarray(np.transpose(f, (2, 1, 0))), n2, h2, bc2, O.NODE)
    assert np.abs(np.transpose(u2, (2, 1, 0)) - u).max() < 1e-14 * np.abs(u).max()


@pytest.mark.parametrize("layout", [0, 1])
def test_direct_points_equal_the_full_solves(layout):
    """Sampled direct sums (used at sizes where the full oracle is too slow) agree with the
    full direct and FFT forms on every combination of unbounded and semi-unbounded axes."""
    rng = np.random.default_rng(50 + layout)
    U = [(3, 3), (0, 3), (1, 3), (3, 0), (3, 1)]
    for trial in range(12):
        bc = [list(U[rng.integers(len(U))]) for _ in range(3)]
        n = [int(v) for v in rng.choice([3, 4, 5, 6, 7], size=3)]
        h = [float(v) for v in rng.uniform(0.05, 0.2, size=3)]
        shp = O.user_shape(n, layout)
        f = rng.standard_normal(shp)
        full = O.solve(f, n, h, bc, layout, mode=O.DIRECT)
        fast = O.solve(f, n, h, bc, layout)
        pts = [(int(rng.integers(shp[2])), int(rng.integers(shp[1])), int(rng.integers(shp[0]))) for _ in range(6)]
        pts += [(0, 0, 0), (shp[2] - 1, shp[1] - 1, shp[0] - 1)]
        got = O.direct_points(f, n, h, bc, layout, pts)
        scale = np.abs(full).max()
        for (ix, iy, iz), v in zip(pts, got):
            assert abs(v - full[iz, iy, ix]) <= 1e-13 * scale, (bc, n, (ix, iy, iz))
            assert abs(v - fast[iz, iy, ix]) <= 1e-12 * scale, (bc, n, (ix, iy, iz))
