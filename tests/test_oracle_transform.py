"""Pins of the oracle's plain 3-D transforms (the forward and backward operations of a
plan without the spectral multiplication), against numpy / scipy, CPU only.

* all periodic: the 3-D DFT (numpy.fft.fftn), in both layouts (the node-centred
  duplicate point is not used and is written back as the first point);
* fully unbounded: the DFT of the field zero-padded to twice its cells (Sec. II-C);
* cell even-even / odd-odd axes: scipy's type-2 DCT / DST (FFTW's unnormalised REDFT10 /
  RODFT10), node even-even: type-1 DCT;
* backward(forward(f)) = prod(n_log) f, with the odd-face nodes zero.
"""
import numpy as np
import pytest
from scipy import fft as sfft

import oracle as O


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_periodic_is_the_3d_dft(layout):
    n, h = [6, 5, 8], [0.1, 0.2, 0.3]
    f = _rng(1).standard_normal(O.user_shape(n, layout))
    F = O.forward(f, n, h, [[2, 2]] * 3, layout)
    core = f[:n[2], :n[1], :n[0]]
    assert np.abs(F - np.fft.fftn(core)).max() < 1e-12 * np.abs(F).max()
    u = O.backward(F, n, h, [[2, 2]] * 3, layout)
    ref = core * np.prod(n)
    assert np.abs(u[:n[2], :n[1], :n[0]] - ref).max() < 1e-12 * np.abs(ref).max()
    if layout == O.NODE:
        assert np.array_equal(u[..., -1], u[..., 0])


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_unbounded_is_the_dft_of_the_padded_field(layout):
    n, h = [5, 4, 6], [0.1, 0.2, 0.3]
    f = _rng(2).standard_normal(O.user_shape(n, layout))
    F = O.forward(f, n, h, [[3, 3]] * 3, layout)
    pad = np.zeros((2 * n[2], 2 * n[1], 2 * n[0]))
    pad[:f.shape[0], :f.shape[1], :f.shape[2]] = f
    assert np.abs(F - np.fft.fftn(pad)).max() < 1e-12 * np.abs(F).max()
    u = O.backward(F, n, h, [[3, 3]] * 3, layout)
    assert np.abs(u - 8 * np.prod(n) * f).max() < 1e-11 * np.abs(f).max() * np.prod(n)


def test_symmetric_axes_are_scipys_dct_and_dst():
    n, h = [6, 5, 7], [0.1, 0.2, 0.3]
    f = _rng(3).standard_normal(O.user_shape(n, O.CELL))
    # x even-even (DCT-II), y odd-odd (DST-II), z periodic
    F = O.forward(f, n, h, [[0, 0], [1, 1], [2, 2]], O.CELL)
    ref = np.fft.fft(sfft.dst(sfft.dct(f, type=2, axis=2), type=2, axis=1), axis=0)
    assert np.abs(F - ref).max() < 1e-12 * np.abs(ref).max()
    # node even-even along every axis: type-1 DCT of the N + 1 points
    g = _rng(4).standard_normal(O.user_shape(n, O.NODE))
    G = O.forward(g, n, h, [[0, 0]] * 3, O.NODE)
    ref = sfft.dctn(g, type=1)
    assert np.abs(G - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_round_trip_every_class(layout):
    pairs = [(2, 2), (0, 0), (1, 1), (0, 1), (1, 0), (3, 3), (0, 3), (1, 3), (3, 0), (3, 1)]
    n, h = [5, 6, 4], [0.1, 0.2, 0.3]
    rng = _rng(5 + layout)
    for trial in range(30):
        bc = [list(pairs[rng.integers(10)]) for _ in range(3)]
        f = rng.standard_normal(O.user_shape(n, layout))
        u = O.backward(O.forward(f, n, h, bc, layout), n, h, bc, layout)
        nlog = np.prod([O.axis_info(n[a], h[a], layout, *bc[a])["nlog"] for a in range(3)])
        # the points a plan does not use (odd-face nodes, the periodic duplicate) come back
        # as 0 or as the first point; compare where the field is used
        mask = np.ones_like(f, dtype=bool)
        for a in range(3):
            ax = 2 - a
            idx = [slice(None)] * 3
            if layout == O.NODE and bc[a][0] == 1:
                idx[ax] = 0; mask[tuple(idx)] = False
            if layout == O.NODE and (bc[a][1] == 1 or bc[a][0] == 2):
                idx[ax] = -1; mask[tuple(idx)] = False
        assert np.abs((u - nlog * f)[mask]).max() < 1e-11 * nlog * np.abs(f).max(), bc
