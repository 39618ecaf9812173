"""Pins of the oracle's spectral axes and of its spectral curl (CPU only).

Each spectral class of Table I (periodic, and the four symmetric pairs of Sec. II-B, in
both layouts) has continuous eigenfunctions b with b'' = -w^2 b that satisfy the class's
face conditions: cosines and sines whose wavenumber is fixed by the faces alone
(written out below from the conditions, not taken from the oracle).  Sampled on the
class's grid, a product of such functions is an exact eigenvector of the discrete
solve, so the oracle must return u = -f / |w|^2 to roundoff in all three of its forms
(own FFT, defining sums, direct).  A wrong wavenumber, index shift or half-sample shift
on any axis breaks this by O(1).

The spectral curl (Sec. V) on periodic axes is pinned the same way: a field
f = Re(A exp(i k.x)) has u = Re(-(i k x A) exp(i k.x)) / |k|^2.  The Nyquist mode of an
even-length axis enters with the phase whose continuous derivative vanishes on the grid
(cosine on nodes, sine on cell centres), where setting its derivative to zero (the
reading for the Nyquist mode) is the exact answer.

The printed App. B values at N = 256 need about 8 GB and two minutes of the oracle; that
test runs when FLUXMI_SLOW=1 is set.
"""
import json
import os

import numpy as np
import pytest

import analytic as A
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_chat2_errors.json")

# (left, right) face codes: 0 even, 1 odd, 2 periodic
SPECTRAL = {"P": (2, 2), "EE": (0, 0), "OO": (1, 1), "EO": (0, 1), "OE": (1, 0)}


def grid(N, h, layout):
    """User point positions on [0, L]: cell centres or nodes (Sec. II-A)."""
    if layout == O.CELL:
        return (np.arange(N) + 0.5) * h
    return np.arange(N + 1) * h


def eigenmodes(cls, N, L, layout):
    """The class's continuous eigenfunctions that the grid resolves, as (function, w).

    Even face at x = 0: cosine (phase 0); odd face at x = 0: sine.  The right face fixes
    the wavenumber: even-even and odd-odd need w L = m pi, mixed faces
    w L = (m + 1/2) pi; periodic needs w L = 2 pi m (cosine and sine)."""
    pi = np.pi
    out = []
    if cls == "P":
        for m in range(0, N // 2 + 1):
            w = 2 * pi * m / L
            out.append((lambda x, w=w: np.cos(w * x), w))
            if 0 < m and 2 * m < N:
                out.append((lambda x, w=w: np.sin(w * x), w))
            if 2 * m == N and layout == O.CELL:  # the Nyquist sine is the one a cell grid sees
                out.append((lambda x, w=w: np.sin(w * x), w))
        return out
    if cls == "EE":
        ms = range(0, N + (1 if layout == O.NODE else 0))
        return [(lambda x, w=m * pi / L: np.cos(w * x), m * pi / L) for m in ms]
    if cls == "OO":
        ms = range(1, N + (0 if layout == O.NODE else 1))
        return [(lambda x, w=m * pi / L: np.sin(w * x), m * pi / L) for m in ms]
    half = [(m + 0.5) * pi / L for m in range(N)]
    if cls == "EO":
        return [(lambda x, w=w: np.cos(w * x), w) for w in half]
    return [(lambda x, w=w: np.sin(w * x), w) for w in half]  # OE


def _eigen_case(rng, classes, n, h, layout, nterms):
    """f = sum of random products of eigenfunctions; the exact u = sum -f_t / |w_t|^2."""
    xs = [grid(n[a], h[a], layout) for a in range(3)]
    modes = [eigenmodes(classes[a], n[a], n[a] * h[a], layout) for a in range(3)]
    f = 0.0
    u = 0.0
    for _ in range(nterms):
        pick = [modes[a][rng.integers(len(modes[a]))] for a in range(3)]
        amp = rng.standard_normal()
        fx, fy, fz = (pick[a][0](xs[a]) for a in range(3))
        term = amp * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
        w2 = sum(pick[a][1] ** 2 for a in range(3))
        f = f + term
        if w2 > 0:  # the zero mode has no solution; its mean is discarded
            u = u - term / w2
    f = np.broadcast_to(f, O.user_shape(n, layout)).copy()
    u = np.broadcast_to(u, f.shape).copy()
    return f, u


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
@pytest.mark.parametrize("cls", list(SPECTRAL))
def test_spectral_class_eigenfunctions(cls, layout):
    """Every eigenfunction of a class, one at a time, along each axis position; the
    other two axes carry random spectral classes and modes."""
    rng = np.random.default_rng(hash((cls, layout)) % (1 << 31))
    names = list(SPECTRAL)
    for axis in range(3):
        n = [6, 7, 5]
        n[axis] = 8 if cls == "P" else 7
        h = [0.13, 0.1, 0.17]
        classes = [names[rng.integers(len(names))] for _ in range(3)]
        classes[axis] = cls
        bc = [list(SPECTRAL[c]) for c in classes]
        L = n[axis] * h[axis]
        xs = [grid(n[a], h[a], layout) for a in range(3)]
        for fn, w in eigenmodes(cls, n[axis], L, layout):
            others = []
            for a in range(3):
                if a == axis:
                    others.append((fn, w))
                else:
                    m = eigenmodes(classes[a], n[a], n[a] * h[a], layout)
                    others.append(m[rng.integers(len(m))])
            g = [others[a][0](xs[a]) for a in range(3)]
            f = g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
            w2 = sum(o[1] ** 2 for o in others)
            exact = -f / w2 if w2 > 0 else np.zeros_like(f)
            if np.abs(f).max() < 1e-12:
                continue  # a mode the grid does not see
            for mode in (O.FAST, O.NAIVE, O.DIRECT):
                u = O.solve(f, n, h, bc, layout, 0, 0, mode)
                err = np.abs(u - exact).max() / max(np.abs(exact).max(), np.abs(f).max() / w2 if w2 else 1.0)
                assert err < 1e-12, (cls, layout, axis, classes, w, mode, err)


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_spectral_superpositions(layout):
    """Random sums of eigenfunction products over random class triples, odd and even
    lengths, anisotropic spacing."""
    rng = np.random.default_rng(31 + layout)
    names = list(SPECTRAL)
    for trial in range(40):
        classes = [names[rng.integers(len(names))] for _ in range(3)]
        n = [int(v) for v in rng.choice([4, 5, 6, 7, 9, 10], size=3)]
        h = [float(v) for v in rng.uniform(0.05, 0.3, size=3)]
        f, exact = _eigen_case(rng, classes, n, h, layout, nterms=6)
        bc = [list(SPECTRAL[c]) for c in classes]
        u = O.solve(f, n, h, bc, layout)
        scale = max(np.abs(exact).max(), 1e-300)
        assert np.abs(u - exact).max() < 1e-12 * scale, (classes, n, layout)


def test_eigenmodes_satisfy_their_faces():
    """The test's own eigenfunctions: b'' = -w^2 b by finite differences, and the face
    conditions (value 0 at an odd face, slope 0 at an even face, period L)."""
    L, eps = 1.3, 1e-4
    for cls, (bl, br) in SPECTRAL.items():
        for fn, w in eigenmodes(cls, 6, L, O.NODE):
            x = np.linspace(0.1, 1.2, 7)
            d2 = (fn(x + eps) - 2 * fn(x) + fn(x - eps)) / eps ** 2
            assert np.allclose(d2, -w * w * fn(x), atol=1e-5 * max(1, w * w))
            slope = lambda x0: (fn(x0 + eps) - fn(x0 - eps)) / (2 * eps)
            if cls == "P":
                assert abs(fn(0.0) - fn(L)) < 1e-12 and abs(slope(0.0) - slope(L)) < 1e-5 * max(1, w)
                continue
            for face, code in ((0.0, bl), (L, br)):
                if code == 1:
                    assert abs(fn(face)) < 1e-12
                else:
                    assert abs(slope(face)) < 1e-5 * max(1, w)


# ---------------------------------------------------------------------------------
def _curl_field(rng, n, h, layout, modes):
    """Real field f = sum Re(A_t exp(i k_t . x)) and the exact u = sum Re(-(i k x A) e) / |k|^2
    on an all-periodic grid; arrays [3][z][y][x]."""
    xs = [grid(n[a], h[a], layout) for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    f = np.zeros((3,) + X.shape)
    u = np.zeros_like(f)
    for m in modes:
        k = np.array([2 * np.pi * m[a] / (n[a] * h[a]) for a in range(3)])
        Avec = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        phase = np.exp(1j * (k[0] * X + k[1] * Y + k[2] * Z))
        for c in range(3):
            f[c] += np.real(Avec[c] * phase)
        k2 = float(k @ k)
        if k2 == 0:
            continue
        ikxA = 1j * np.cross(k, Avec)
        for c in range(3):
            u[c] += np.real(-ikxA[c] * phase) / k2
    return f, u


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
@pytest.mark.parametrize("n", [[6, 7, 5], [8, 4, 6]])
def test_periodic_curl_closed_form(layout, n):
    """Biot-Savart on periodic axes: signed wavenumbers (modes above N/2 are negative
    frequencies), both curl orientations, every component."""
    rng = np.random.default_rng(7 + layout)
    h = [0.11, 0.09, 0.14]
    modes = []
    for _ in range(5):
        modes.append([int(rng.integers(-((n[a] - 1) // 2), (n[a] - 1) // 2 + 1)) for a in range(3)])
    f, exact = _curl_field(rng, n, h, layout, modes)
    bc = [[2, 2]] * 3
    for mode in (O.FAST, O.NAIVE):
        u = O.solve(f, n, h, bc, layout, 0, 1, mode)
        assert np.abs(u - exact).max() < 1e-12 * np.abs(exact).max(), (n, layout, mode)


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
def test_periodic_curl_nyquist(layout):
    """An even-length axis carrying its Nyquist mode: with the phase whose continuous
    derivative vanishes at the grid points, the exact solution has no derivative along
    that axis, which is what zeroing the Nyquist derivative gives."""
    n, h = [8, 6, 5], [0.1, 0.12, 0.15]
    xs = [grid(n[a], h[a], layout) for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    kn = np.pi / h[0]                       # Nyquist wavenumber of x (N = 8)
    ky, kz = 2 * np.pi / (n[1] * h[1]), 2 * np.pi * 2 / (n[2] * h[2])
    nyq = np.cos(kn * X) if layout == O.NODE else np.sin(kn * X)
    g = nyq * np.sin(ky * Y) * np.cos(kz * Z)
    # f = (g, g, g): curl f = (dy g - dz g, dz g - dx g, dx g - dy g) with dx g = 0 on the grid
    dyg = nyq * ky * np.cos(ky * Y) * np.cos(kz * Z)
    dzg = -nyq * kz * np.sin(ky * Y) * np.sin(kz * Z)
    k2 = kn ** 2 + ky ** 2 + kz ** 2
    exact = -np.stack([dyg - dzg, dzg, -dyg]) / k2
    f = np.stack([g, g, g])
    for mode in (O.FAST, O.NAIVE):
        u = O.solve(f, n, h, [[2, 2]] * 3, layout, 0, 1, mode)
        assert np.abs(u - exact).max() < 1e-12 * np.abs(exact).max(), (layout, mode)


# ---------------------------------------------------------------------------------
@pytest.mark.skipif(os.environ.get("FLUXMI_SLOW") != "1", reason="about 8 GB and 2 minutes; set FLUXMI_SLOW=1")
@pytest.mark.parametrize("case,maker", [("unbounded", A.app_b_unbounded), ("semi", A.app_b_semi)])
def test_paper_chat2_errors_256(case, maker):
    """App. B.2 / B.3 at N = 256 (the last printed points the oracle reaches on a host)."""
    with open(GOLDEN) as fh:
        g = json.load(fh)[case]
    f, phi, bc = maker(256)
    u = O.solve(f, [256] * 3, [1.0 / 256] * 3, bc, O.NODE, 0, 0)
    assert np.abs(u - phi).max() == pytest.approx(g["E_inf"]["256"], rel=1e-10)
