"""Pins for the oracle's 1-D transforms (CPU only).

The oracle's own FFT and its symmetric-extension real-to-real routes are checked
against (a) their defining sums, (b) independent library routines (numpy.fft,
scipy.fft.dct/dst, which implement the same FFTW-style definitions), (c) the node-centred
formulas of Sec. II-B written in the paper's own index form, and (d) round trips.
"""
import numpy as np
import pytest
import scipy.fft as sf

import oracle as O

LENGTHS = list(range(1, 41)) + [48, 49, 60, 64, 81, 96, 97, 125, 127, 128, 192, 210, 243, 256, 343, 385]


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_definition_and_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.fft.fft(x)
    scale = np.abs(x).sum()
    assert np.abs(O.fft(x) - ref).max() / scale < 1e-14
    assert np.abs(O.dft_naive(x) - ref).max() / scale < 1e-14
    assert np.abs(O.fft(x, +1) - n * np.fft.ifft(x)).max() / scale < 1e-14
    # forward then backward = n * identity
    assert np.abs(O.fft(O.fft(x), +1) / n - x).max() < 1e-13


SCIPY = {
    O.REDFT00: ("dct", 1), O.REDFT10: ("dct", 2), O.REDFT01: ("dct", 3), O.REDFT11: ("dct", 4),
    O.RODFT00: ("dst", 1), O.RODFT10: ("dst", 2), O.RODFT01: ("dst", 3), O.RODFT11: ("dst", 4),
}
# inverse kind and its normalisation, as functions of n
INVERSE = {
    O.REDFT00: (O.REDFT00, lambda n: 2 * (n - 1)), O.RODFT00: (O.RODFT00, lambda n: 2 * (n + 1)),
    O.REDFT10: (O.REDFT01, lambda n: 2 * n), O.REDFT01: (O.REDFT10, lambda n: 2 * n),
    O.RODFT10: (O.RODFT01, lambda n: 2 * n), O.RODFT01: (O.RODFT10, lambda n: 2 * n),
    O.REDFT11: (O.REDFT11, lambda n: 2 * n), O.RODFT11: (O.RODFT11, lambda n: 2 * n),
}


@pytest.mark.parametrize("kind", list(SCIPY))
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 17, 31, 33, 64, 65, 97, 128, 129, 192, 193])
def test_r2r_definition_fft_route_and_scipy(kind, n):
    rng = np.random.default_rng(1000 * kind + n)
    x = rng.standard_normal(n)
    fn, typ = SCIPY[kind]
    ref = getattr(sf, fn)(x, type=typ)
    scale = np.abs(ref).max()
    assert np.abs(O.r2r(kind, x, naive=True) - ref).max() / scale < 1e-13
    assert np.abs(O.r2r(kind, x) - ref).max() / scale < 1e-13
    inv, norm = INVERSE[kind]
    back = O.r2r(inv, O.r2r(kind, x)) / norm(n)
    assert np.abs(back - x).max() < 1e-12


# Sec. II-B node-centred definitions, written with the paper's indices f_0..f_N.
def paper_dct1(f):
    N = f.size - 1
    k = np.arange(N + 1)
    j = np.arange(1, N)
    return f[0] + (-1.0) ** k * f[N] + 2 * (f[1:N, None] * np.cos(2 * np.pi / (2 * N) * j[:, None] * k)).sum(0)


def paper_dst1(f):
    N = f.size - 1
    k = np.arange(1, N)
    j = np.arange(1, N)
    return 2 * (f[1:N, None] * np.sin(2 * np.pi / (2 * N) * j[:, None] * k)).sum(0)


def paper_dst3(f):
    N = f.size - 1
    k = np.arange(N)
    j = np.arange(1, N)
    return (-1.0) ** k * f[N] + 2 * (f[1:N, None] * np.sin(2 * np.pi / (2 * N) * j[:, None] * (k + 0.5))).sum(0)


def paper_dct3(f):
    N = f.size - 1
    k = np.arange(N)
    j = np.arange(1, N)
    return f[0] + 2 * (f[1:N, None] * np.cos(2 * np.pi / (2 * N) * j[:, None] * (k + 0.5))).sum(0)


@pytest.mark.parametrize("N", [2, 3, 4, 8, 11, 32])
def test_node_transforms_match_paper_definitions(N):
    """Table I node column: even-even DCT-I, odd-odd DST-I, odd-even DST-III,
    even-odd DCT-III, fed with the points the paper says are used."""
    rng = np.random.default_rng(N)
    f = rng.standard_normal(N + 1)
    assert np.allclose(O.r2r(O.REDFT00, f), paper_dct1(f), rtol=0, atol=1e-12)
    if N >= 2:
        assert np.allclose(O.r2r(O.RODFT00, f[1:N]), paper_dst1(f), rtol=0, atol=1e-12)
    assert np.allclose(O.r2r(O.RODFT01, f[1:N + 1]), paper_dst3(f), rtol=0, atol=1e-12)
    assert np.allclose(O.r2r(O.REDFT01, f[0:N]), paper_dct3(f), rtol=0, atol=1e-12)


def test_periodic_dft_matches_paper_definition():
    """Sec. II-B periodic DFT: f_k = sum_j f(x_j) exp(-i w_k x_j), w_k = 2 pi k / L."""
    N, L = 12, 3.0
    rng = np.random.default_rng(5)
    f = rng.standard_normal(N)
    x = np.arange(N) * L / N
    w = 2 * np.pi * np.arange(N) / L
    ref = (f[:, None] * np.exp(-1j * w[None, :] * x[:, None])).sum(0)
    assert np.abs(O.fft(f.astype(complex)) - ref).max() < 1e-12
