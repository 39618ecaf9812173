"""Pins of the oracle's lattice Green's function LGF2 (Sec. IV names it, citing Martinsson
& Rodin; it is the Green's function of the second-order discrete Laplacian): the E_inf
values the paper prints for LGF2 in the three validation cases of Sec. IV at N = 32 and
64; Watson's closed form of its origin value; the discrete Laplacian of the table; the
far field; the three oracle forms against each other; the spectral form against the
second-difference operator on a periodic grid."""
import json
import os

import numpy as np
import pytest
from scipy import special

import analytic as A
import oracle as O
from oracle.lgf import lgf_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_lgf2_errors.json")
MAKER = {"unbounded": A.app_b_unbounded, "semi": A.app_b_semi, "spectral": A.app_b_spectral}


def _cases():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    return [(case, int(N), v, g[case]["bc"]) for case in MAKER for N, v in g[case]["E_inf"].items()]


@pytest.mark.parametrize("case,N,value,bc", _cases())
def test_paper_lgf2_errors(case, N, value, bc):
    f, phi, bc2 = MAKER[case](N)
    assert bc2 == bc
    u = O.solve(f, [N] * 3, [1.0 / N] * 3, bc, O.NODE, O.LGF2, 0)
    err = np.abs(u - phi).max()
    assert err == pytest.approx(value, rel=1e-9), (case, N, err)


def _laplacian(G, h, i, j, k):
    """Second-difference Laplacian of the even table G[z][y][x] at offset (i, j, k)."""
    def g(a, b, c):
        return G[abs(c), abs(b), abs(a)]
    return ((g(i + 1, j, k) - 2 * g(i, j, k) + g(i - 1, j, k)) / h[0] ** 2 +
            (g(i, j + 1, k) - 2 * g(i, j, k) + g(i, j - 1, k)) / h[1] ** 2 +
            (g(i, j, k + 1) - 2 * g(i, j, k) + g(i, j, k - 1)) / h[2] ** 2)


def test_origin_value_is_watsons_integral():
    """G(0) = -W / (6 h) with Watson's simple-cubic integral
    W = sqrt(6) / (32 pi^3) Gamma(1/24) Gamma(5/24) Gamma(7/24) Gamma(11/24)."""
    W = np.sqrt(6) / (32 * np.pi ** 3) * special.gamma(1 / 24) * special.gamma(5 / 24) * \
        special.gamma(7 / 24) * special.gamma(11 / 24)
    for h in (1.0, 0.05):
        G = lgf_table([3, 3, 3], [h] * 3)
        assert G[0, 0, 0] == pytest.approx(-W / (6 * h), rel=1e-13)


@pytest.mark.parametrize("h", [[1.0, 1.0, 1.0], [0.1, 0.07, 0.13]])
def test_table_is_the_inverse_of_the_discrete_laplacian(h):
    G = lgf_table([9, 8, 7], h)
    vol = np.prod(h)
    assert _laplacian(G, h, 0, 0, 0) * vol == pytest.approx(1.0, abs=1e-12)
    scale = abs(G[0, 0, 0]) / min(h) ** 2
    for p in [(1, 0, 0), (0, 2, 1), (3, 3, 3), (7, 6, 5), (5, 1, 2)]:
        assert abs(_laplacian(G, h, *p)) < 1e-12 * scale, p


def test_far_field_is_the_point_source():
    """G(n) -> -1/(4 pi |n| h) with a relative correction of order |n|^-2."""
    G = lgf_table([201, 2, 2], [1.0] * 3)[0, 0, :]
    for n in (20, 50, 100, 200):
        rel = G[n] * 4 * np.pi * n + 1
        assert abs(rel) < 0.3 / n ** 2 and rel < 0, (n, rel)


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_three_forms_agree(layout):
    rng = np.random.default_rng(5)
    for bc in ([[3, 3]] * 3, [[3, 0], [3, 3], [1, 3]], [[2, 2], [0, 1], [1, 1]]):
        n, h = [5, 4, 6], [0.1, 0.12, 0.09]
        f = rng.standard_normal(O.user_shape(n, layout))
        fast = O.solve(f, n, h, bc, layout, O.LGF2, 0, O.FAST)
        naive = O.solve(f, n, h, bc, layout, O.LGF2, 0, O.NAIVE)
        direct = O.solve(f, n, h, bc, layout, O.LGF2, 0, O.DIRECT)
        s = np.abs(direct).max()
        assert np.abs(fast - direct).max() < 1e-12 * s, bc
        assert np.abs(naive - direct).max() < 1e-12 * s, bc


def test_spectral_form_inverts_the_second_difference_laplacian():
    """All-periodic node grid: the 7-point Laplacian (written here) of the LGF2 solution
    returns the zero-mean part of the right-hand side exactly."""
    n, h = [12, 10, 8], [0.1, 0.13, 0.07]
    rng = np.random.default_rng(8)
    f = rng.standard_normal(O.user_shape(n, O.NODE))
    f[-1, :, :] = f[0, :, :]
    f[:, -1, :] = f[:, 0, :]
    f[:, :, -1] = f[:, :, 0]
    u = O.solve(f, n, h, [[2, 2]] * 3, O.NODE, O.LGF2, 0)[:-1, :-1, :-1]
    lap = sum((np.roll(u, 1, ax) - 2 * u + np.roll(u, -1, ax)) / h[2 - ax] ** 2 for ax in range(3))
    g = f[:-1, :-1, :-1]
    assert np.abs(lap - (g - g.mean())).max() < 1e-10 * np.abs(g).max()


def test_mixed_directions_are_refused():
    with pytest.raises(ValueError):
        O.solve(np.zeros((9, 9, 9)), [8] * 3, [0.1] * 3, [[3, 3], [3, 3], [2, 2]], O.NODE, O.LGF2, 0)
