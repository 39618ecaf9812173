"""Closed-form fields used to pin the oracle (no part of the solver's arithmetic).

* The three validation cases of Sec. IV with the reference solutions of App. B
  (compact bump functions and a trigonometric product).
* Free-space potentials of Gaussian sources: 3-D (erf), 1 convolution direction
  (erfc-based), 2 convolution directions (Hankel integral / exponential integral), and
  the Biot-Savart velocity of a Gaussian column (curl of the 3-D potential).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special


# --- App. B compact bump: B(s) = exp(10 (1 - 1/(1 - s^2))) for |s| < 1 -------------
def bump(s):
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    m = np.abs(s) < 1
    out[m] = np.exp(10.0 - 10.0 / (1.0 - s[m] ** 2))
    return out


def bump_dd(s, scale):
    """d^2/dx^2 B(s(x)) for s = scale * x + c (chain rule)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    m = np.abs(s) < 1
    sm = s[m]
    b = np.exp(10.0 - 10.0 / (1.0 - sm ** 2))
    q1 = -20.0 * sm / (1.0 - sm ** 2) ** 2            # d/ds of the exponent
    q2 = -20.0 * (1.0 + 3.0 * sm ** 2) / (1.0 - sm ** 2) ** 3
    out[m] = b * (q1 ** 2 + q2) * scale ** 2
    return out


def _outer(X, Y, Z):
    return Z[:, None, None] * Y[None, :, None] * X[None, None, :]


def _lap(X, Xdd, Y, Ydd, Z, Zdd):
    return _outer(Xdd, Y, Z) + _outer(X, Ydd, Z) + _outer(X, Y, Zdd)


def app_b_spectral(N, L=1.0):
    """App. B.1: x even-even, y odd-even, z periodic; node-centred on [0, L]^3."""
    x = np.arange(N + 1) * (L / N)
    X = np.cos(np.pi * x / L)
    Y = np.sin(2.5 * np.pi * x / L)
    Z = np.sin(8.0 * np.pi * x / L)
    phi = _outer(X, Y, Z)
    f = -((np.pi / L) ** 2 + (2.5 * np.pi / L) ** 2 + (8.0 * np.pi / L) ** 2) * phi
    bc = [[0, 0], [1, 0], [2, 2]]
    return f, phi, bc


def app_b_unbounded(N, L=1.0):
    """App. B.2: fully unbounded, node-centred on [0, L]^3."""
    x = np.arange(N + 1) * (L / N)
    s = 2.0 * x / L - 1.0
    X, Xdd = bump(s), bump_dd(s, 2.0 / L)
    phi = _outer(X, X, X)
    f = _lap(X, Xdd, X, Xdd, X, Xdd)
    bc = [[3, 3], [3, 3], [3, 3]]
    return f, phi, bc


def app_b_semi(N, L=1.0):
    """App. B.3: x unbounded-left / even-right, y unbounded, z odd-left /
    unbounded-right; node-centred on [0, L]^3."""
    x = np.arange(N + 1) * (L / N)
    sx1, sx2 = (2 * x - 1.4 * L) / L, (2 * x - 2.6 * L) / L
    X = bump(sx1) + bump(sx2)
    Xdd = bump_dd(sx1, 2.0 / L) + bump_dd(sx2, 2.0 / L)
    sy = 2 * x / L - 1
    Y, Ydd = bump(sy), bump_dd(sy, 2.0 / L)
    sz1, sz2 = (2 * x - 0.6 * L) / L, (2 * x + 0.6 * L) / L
    Z = bump(sz1) - bump(sz2)
    Zdd = bump_dd(sz1, 2.0 / L) - bump_dd(sz2, 2.0 / L)
    phi = _outer(X, Y, Z)
    f = _lap(X, Xdd, Y, Ydd, Z, Zdd)
    bc = [[3, 0], [3, 3], [1, 3]]
    return f, phi, bc


# --- Gaussian sources ---------------------------------------------------------------
def cell_coords(N, lo, hi):
    h = (hi - lo) / N
    return lo + (np.arange(N) + 0.5) * h, h


def gaussian_potential_3d(r, sigma):
    """u solving lap(u) = exp(-r^2/(2 sigma^2)) in free space, u -> 0 at infinity."""
    Q = (2.0 * np.pi * sigma ** 2) ** 1.5
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-12
    out[small] = -sigma ** 2
    rs = r[~small]
    out[~small] = -Q * special.erf(rs / (np.sqrt(2.0) * sigma)) / (4.0 * np.pi * rs)
    return out


def gaussian_dphi_dr(r, sigma):
    Q = (2.0 * np.pi * sigma ** 2) ** 1.5
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    m = r > 1e-12
    rm = r[m]
    out[m] = -(Q / (4.0 * np.pi)) * (
        np.sqrt(2.0 / np.pi) * np.exp(-rm ** 2 / (2 * sigma ** 2)) / (sigma * rm)
        - special.erf(rm / (np.sqrt(2.0) * sigma)) / rm ** 2
    )
    return out


def gaussian_column_velocity(X, Y, Z, sigma):
    """u = curl((0, 0, phi)) solves lap(u) = curl((0, 0, g)) for the 3-D Gaussian g."""
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    d = gaussian_dphi_dr(r, sigma)
    with np.errstate(invalid="ignore", divide="ignore"):
        ux = np.where(r > 0, d * Y / r, 0.0)
        uy = np.where(r > 0, -d * X / r, 0.0)
    return np.stack([ux, uy, np.zeros_like(ux)])


def gaussian_1unb(z, k, sigma):
    """U solving U'' - k^2 U = exp(-z^2/(2 sigma^2)) on the line, bounded (k > 0), or
    U'' = exp(...) with U = int |z - z'|/2 f(z') dz' (k = 0)."""
    z = np.asarray(z, dtype=np.float64)
    if k == 0.0:
        return 0.5 * (z * sigma * np.sqrt(2 * np.pi) * special.erf(z / (sigma * np.sqrt(2)))
                      + 2 * sigma ** 2 * np.exp(-z ** 2 / (2 * sigma ** 2)))
    a = (k * sigma ** 2 - z) / (sigma * np.sqrt(2))
    b = (k * sigma ** 2 + z) / (sigma * np.sqrt(2))
    I = sigma * np.sqrt(np.pi / 2) * np.exp(-z ** 2 / (2 * sigma ** 2)) * (special.erfcx(a) + special.erfcx(b))
    return -I / (2.0 * k)


def gaussian_2unb_k0(rho, sigma):
    """U solving the 2-D Poisson equation for exp(-rho^2/(2 sigma^2)) with the free-space
    kernel ln(rho)/(2 pi):  U = sigma^2 ln(rho) + sigma^2/2 E1(rho^2/(2 sigma^2))."""
    rho = np.asarray(rho, dtype=np.float64)
    t = rho ** 2 / (2 * sigma ** 2)
    out = np.empty_like(rho)
    m = rho > 1e-12
    out[m] = sigma ** 2 * np.log(rho[m]) + 0.5 * sigma ** 2 * special.exp1(t[m])
    out[~m] = 0.5 * sigma ** 2 * (-np.euler_gamma + np.log(2 * sigma ** 2))
    return out


def gaussian_2unb_k(rho_table, k, sigma):
    """U(rho) solving U'' + U'/rho - k^2 U = exp(-rho^2/(2 sigma^2)) (Hankel transform)."""
    vals = []
    for r in rho_table:
        f = lambda q: -sigma ** 2 * np.exp(-q * q * sigma ** 2 / 2) * special.j0(q * r) * q / (q * q + k * k)
        v, _ = integrate.quad(f, 0, 12.0 / sigma, limit=400, epsabs=1e-14, epsrel=1e-12)
        vals.append(v)
    return np.array(vals)
