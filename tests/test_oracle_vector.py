"""The oracle's Biot-Savart with boundary conditions per component (Sec. V: the
derivative on a symmetric axis swaps DCT and DST, with the sign rule for each
direction of the swap), pinned by what does not use that rule:

* the method of images: a symmetric axis equals a periodic axis of the mirrored field
  (period 2L for equal faces, 4L for mixed ones), a semi-unbounded axis equals a fully
  unbounded axis of the field mirrored about its symmetric face; the doubled problems
  are the plain Biot-Savart solve with the complex derivative i w, pinned on its own;
* single Fourier modes on fully spectral boxes, where u = -curl(f) / |k|^2 exactly, with
  the derivatives written out by hand (spectral, and the central-difference symbols);
* shared periodic / unbounded faces: the same result as the plain Biot-Savart solve;
* faces that do not describe a mirror-symmetric vector field are rejected."""
import numpy as np
import pytest

import oracle as O

E, OD, P, U = O.EVEN, O.ODD, O.PER, O.UNB
SW = {E: OD, OD: E, P: P, U: U}


def _mirror(f, lo, hi, layout, how):
    """Extend f [..., nx] along x.  'sym2': period 2L (equal symmetric faces), returns
    the x range [-L, L); 'sym4': period 4L (mixed faces), [0, 4L); 'lo': unbounded
    [-L, L] mirrored about 0; 'hi': [0, 2L] mirrored about L."""
    s_lo = 1.0 if lo == E else -1.0
    s_hi = 1.0 if hi == E else -1.0
    if layout == O.CELL:
        if how in ("sym2", "lo"):
            return np.concatenate([s_lo * f[..., ::-1], f], axis=-1)
        if how == "hi":
            return np.concatenate([f, s_hi * f[..., ::-1]], axis=-1)
        g = np.concatenate([f, s_hi * f[..., ::-1]], axis=-1)  # [0, 2L)
        return np.concatenate([g, s_lo * g[..., ::-1]], axis=-1)  # mirrored about 2L
    # node layout: f holds N + 1 nodes
    if how in ("sym2", "lo"):
        return np.concatenate([s_lo * f[..., :0:-1], f], axis=-1)  # 2N + 1 nodes
    if how == "hi":
        return np.concatenate([f, s_hi * f[..., -2::-1]], axis=-1)
    g = np.concatenate([f, s_hi * f[..., -2::-1]], axis=-1)  # nodes 0 .. 2N
    tail = s_lo * g[..., -2:0:-1]  # nodes 2N + 1 .. 4N - 1 (g(4L - x) = s_lo g(x))
    return np.concatenate([g, tail, g[..., :1]], axis=-1)  # 4N + 1 (duplicate of node 0)


def _faces(xf, yz):
    """Per-component faces: x faces xf for the tangential components (y, z), swapped
    for the normal one (x); y and z faces yz for all."""
    norm = [SW[b] for b in xf]
    return [[norm, [yz, yz], [yz, yz]], [list(xf), [yz, yz], [yz, yz]], [list(xf), [yz, yz], [yz, yz]]]


CASES = [((E, E), "sym2"), ((OD, OD), "sym2"), ((E, OD), "sym4"), ((OD, E), "sym4"),
         ((E, U), "lo"), ((OD, U), "lo"), ((U, E), "hi"), ((U, OD), "hi")]


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
@pytest.mark.parametrize("xf,how", CASES)
@pytest.mark.parametrize("yz", [U, P])
def test_images(layout, xf, how, yz):
    n, h = [6, 5, 7], [0.1, 0.13, 0.09]
    bcv = _faces(xf, yz)
    rng = np.random.default_rng(7 * layout + 3 * yz + CASES.index((xf, how)))
    f = rng.standard_normal((3,) + O.user_shape(n, layout))
    for kind in (1, 2, 4):
        u = O.solve_vector(f, n, h, bcv, layout, 0, kind)
        parts = []
        for c in range(3):
            lo, hi = bcv[c][0]
            fc = f[c].copy()
            if layout == O.NODE:  # values on odd faces are not data
                if lo == OD:
                    fc[..., 0] = 0.0
                if hi == OD:
                    fc[..., -1] = 0.0
            parts.append(_mirror(fc, lo, hi, layout, how))
        mult = 4 if how == "sym4" else 2
        n2 = [mult * n[0], n[1], n[2]]
        xb = [P, P] if how.startswith("sym") else [U, U]
        u2 = O.solve(np.stack(parts), n2, h, [xb, [yz, yz], [yz, yz]], layout, 0, kind)
        nx = f.shape[-1]
        # the mirrored part comes first for 'sym2' / 'lo' (N points), last otherwise
        start = n[0] if how in ("sym2", "lo") else 0
        crop = u2[..., start:start + nx]
        err = np.abs(crop - u).max() / np.abs(u2).max()
        assert err < 1e-13, (layout, xf, yz, kind, err)


def _d(w, h, kind):
    """Derivative factor of wavenumber w: spectral, or the central-difference symbol."""
    if kind == 1:
        return w
    if kind == 2:
        return np.sin(w * h) / h
    if kind == 3:
        return (4 / 3 * np.sin(w * h) - 1 / 6 * np.sin(2 * w * h)) / h
    return (1.5 * np.sin(w * h) - 0.3 * np.sin(2 * w * h) + np.sin(3 * w * h) / 30) / h


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
@pytest.mark.parametrize("xf", [(E, E), (OD, OD), (E, OD), (OD, E)])
@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_single_mode_closed_form(layout, xf, kind):
    """f_b = A_b X_b(x) cos(ky y + a_b) cos(kz z + b_b) on x symmetric, y and z periodic:
    X_b = cos(kx x) for a component even on the left face, sin(kx x) for an odd one
    (kx = pi m / L for equal faces, pi (m + 1/2) / L for mixed ones).  Every derivative
    of a mode is the mode of the other parity times its factor, so u = -curl(f) / |k|^2
    with the derivatives written out here (no transform involved)."""
    n = [8, 6, 10]
    h = [0.11, 0.1, 0.07]
    L = [n[a] * h[a] for a in range(3)]
    bcv = _faces(xf, P)
    mixed = xf[0] != xf[1]
    kx = np.pi * ((2 + 0.5) if mixed else 3) / L[0]
    ky = 2 * np.pi * 2 / L[1]
    kz = 2 * np.pi * 1 / L[2]
    k2 = kx * kx + ky * ky + kz * kz
    off = 0.5 if layout == O.CELL else 0.0
    npts = [n[a] + (1 if layout == O.NODE else 0) for a in range(3)]
    x = (np.arange(npts[0]) + off) * h[0]
    y = (np.arange(npts[1]) + off) * h[1]
    z = (np.arange(npts[2]) + off) * h[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    A = [0.7, -1.3, 0.9]
    al = [0.3, -0.8, 1.1]
    be = [-0.4, 0.6, 0.2]
    # left-face symmetry of each component along x: cos for even, sin for odd
    even = [bcv[b][0][0] == E for b in range(3)]
    Dx, Dy, Dz = _d(kx, h[0], kind), _d(ky, h[1], kind), _d(kz, h[2], kind)

    def Xf(b, deriv=False):
        if not deriv:
            return np.cos(kx * X) if even[b] else np.sin(kx * X)
        return -Dx * np.sin(kx * X) if even[b] else Dx * np.cos(kx * X)

    def Yf(b, deriv=False):
        return -Dy * np.sin(ky * Y + al[b]) if deriv else np.cos(ky * Y + al[b])

    def Zf(b, deriv=False):
        return -Dz * np.sin(kz * Z + be[b]) if deriv else np.cos(kz * Z + be[b])

    def comp(b, dx=False, dy=False, dz=False):
        return A[b] * Xf(b, dx) * Yf(b, dy) * Zf(b, dz)

    f = np.stack([comp(b) for b in range(3)])
    curl = np.stack([comp(2, dy=True) - comp(1, dz=True),
                     comp(0, dz=True) - comp(2, dx=True),
                     comp(1, dx=True) - comp(0, dy=True)])
    exact = -curl / k2
    u = O.solve_vector(f, n, h, bcv, layout, 0, kind)
    err = np.abs(u - exact).max() / np.abs(exact).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("layout", [O.CELL, O.NODE])
@pytest.mark.parametrize("bc", [[[U, U], [P, P], [U, U]], [[P, P], [P, P], [P, P]], [[U, U]] * 3])
def test_shared_faces_equal_plain_biot_savart(layout, bc):
    n, h = [6, 5, 7], [0.1, 0.12, 0.09]
    rng = np.random.default_rng(11 + layout)
    f = rng.standard_normal((3,) + O.user_shape(n, layout))
    for kind in (1, 3):
        a = O.solve_vector(f, n, h, [bc, bc, bc], layout, 0, kind)
        b = O.solve(f, n, h, bc, layout, 0, kind)
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def test_swap_faces():
    bcv = _faces((E, OD), U)
    sw = O.swap_faces(bcv)
    assert sw[0][0] == [E, OD] and sw[1][0] == [OD, E] and sw[2][0] == [OD, E]
    assert sw[1][1] == [U, U] and sw[0][2] == [U, U]


VALID = [
    _faces((E, E), U),                # tangential even, normal odd
    _faces((OD, OD), P),              # tangential odd, normal even
    _faces((E, U), U),                # semi-unbounded
    [[[E, E], [OD, OD], [U, U]], [[OD, OD], [E, E], [U, U]], [[OD, OD], [OD, OD], [U, U]]],  # two symmetric axes
]
INVALID = [
    [[[E, E], [U, U], [U, U]]] * 3,                                                      # one symmetry for all
    [[[OD, OD], [U, U], [U, U]], [[E, E], [U, U], [U, U]], [[OD, OD], [U, U], [U, U]]],  # tangential differ
    [[[U, U], [U, U], [U, U]], [[P, P], [U, U], [U, U]], [[U, U], [U, U], [U, U]]],      # periodic and unbounded mixed
    [[[OD, U], [U, U], [U, U]], [[OD, U], [U, U], [U, U]], [[E, U], [U, U], [U, U]]],    # tangential differ (semi)
    [[[E, E], [U, U], [U, U]], [[OD, OD], [U, U], [U, U]], [[OD, OD], [P, P], [U, U]]],  # y faces differ
]


@pytest.mark.parametrize("bcv", VALID)
def test_mirror_symmetric_faces_accepted(bcv):
    n, h = [4, 4, 4], [0.1] * 3
    f = np.random.default_rng(1).standard_normal((3,) + O.user_shape(n, O.CELL))
    u = O.solve_vector(f, n, h, bcv, O.CELL, 0, 1)
    assert np.all(np.isfinite(u))


@pytest.mark.parametrize("bcv", INVALID)
def test_inconsistent_faces_rejected(bcv):
    n, h = [4, 4, 4], [0.1] * 3
    f = np.zeros((3,) + O.user_shape(n, O.CELL))
    with pytest.raises(ValueError):
        O.solve_vector(f, n, h, bcv, O.CELL, 0, 1)
