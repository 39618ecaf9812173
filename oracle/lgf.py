"""Lattice Green's function of the second-order (7-point) discrete Laplacian, LGF2 of
Sec. IV (the paper cites Martinsson & Rodin for it) -- test infrastructure only.

G solves  sum_a (G(n + e_a) - 2 G(n) + G(n - e_a)) / h_a^2 = delta_{n,0} / (h_x h_y h_z)
on the infinite lattice, so that u = sum_m G(n - m) f(m) h_x h_y h_z solves the
discrete Poisson equation exactly.  With the discrete heat kernel of each axis,
exp(-2 t / h^2) I_n(2 t / h^2),

    G(n) = -(1 / prod h) int_0^inf prod_a ive(n_a, 2 t / h_a^2) dt.

The integrand decays like prod h (4 pi t)^(-3/2); it is integrated with the trapezoidal
rule in u = ln t (exponentially convergent for this analytic integrand) after
subtracting g(t) = prod h (4 pi (t + c))^(-3/2), whose integral is added back in closed
form, so that the truncated remainder decays like t^(-5/2).  For arguments above 1e8 the
scaled Bessel function is its large-argument expansion.  Pinned in
tests/test_oracle_lgf.py by Watson's closed form of G(0), the discrete Laplacian of the
table, the far field -1/(4 pi |x|) and the E_inf values the paper prints for LGF2.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _ive_large(n, x, terms=10):
    """exp(-x) I_n(x) for x >> n^2: 1/sqrt(2 pi x) sum_k (-1)^k a_k(n) / x^k."""
    mu = 4.0 * np.asarray(n, dtype=float) ** 2
    term = np.ones(np.broadcast(n, x).shape)
    total = term.copy()
    for k in range(1, terms):
        term = term * -(mu - (2 * k - 1) ** 2) / (k * 8.0 * x)
        total = total + term
    return total / np.sqrt(2.0 * np.pi * x)


def ive(n, x):
    nb, xb = np.broadcast_arrays(np.asarray(n), np.asarray(x, dtype=float))
    out = np.empty(nb.shape)
    small = xb < 1e8
    out[small] = special.ive(nb[small], xb[small])
    out[~small] = _ive_large(nb[~small], xb[~small])
    return out


def lgf_table(ext, h, du=0.1, c=None):
    """G at the integer offsets 0 .. ext[a] - 1 along each axis: array [ext_z][ext_y][ext_x]
    (x fastest).  ext, h: (x, y, z)."""
    h = np.asarray(h, dtype=float)
    ext = [int(e) for e in ext]
    ph = float(np.prod(h))
    c = float(np.max(h)) ** 2 if c is None else float(c)
    u_lo = np.log(np.min(h) ** 2) - 36.0
    u_hi = np.log(np.max(h) ** 2 * (1.0 + max(ext) ** 2)) + 26.0
    u = np.arange(u_lo, u_hi + 0.5 * du, du)
    t = np.exp(u)
    w = du * t
    A = [ive(np.arange(e)[None, :], 2.0 * t[:, None] / h[a] ** 2) for a, e in enumerate(ext)]
    g = ph * (4.0 * np.pi * (t + c)) ** -1.5
    K = len(t)
    # sum_k w_k A_z[k, m2] A_y[k, m1] A_x[k, m0]
    azy = (A[2][:, :, None] * A[1][:, None, :]).reshape(K, -1)
    S = ((azy * w[:, None]).T @ A[0]).reshape(ext[2], ext[1], ext[0])
    integral = S - np.sum(w * g) + ph * 2.0 * (4.0 * np.pi) ** -1.5 / np.sqrt(c)
    return np.ascontiguousarray(-integral / ph)
