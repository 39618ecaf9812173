"""FP64 CPU reference solver — test infrastructure only.

Thin ctypes front-end over ``liboracle.so`` (built from ``oracle.cpp``).  Only the
test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package; the GPU library never calls it and shares no code with it.

The oracle follows FLUPS (arXiv 2211.07777): per-axis transforms chosen by the
boundary conditions (Table I, Sec. II-B), domain doubling for unbounded directions and
padding plus DCT/DST for semi-unbounded ones (Sec. II-C), multiplication by the Green's
spectrum (Eq. of Sec. II) or by the Green's spectrum times the spectral curl (Sec. V).

Boundary codes: 0 even, 1 odd, 2 periodic, 3 unbounded.  Layout: 0 cell, 1 node.
Green: 0 CHAT2 as printed in Sec. IV (sphere-mean self-term times the cell volume),
1 the sphere-mean self-term itself, 2..6 the regularised HEJ2..HEJ10 kernels, 7 HEJ0
(the HEJ kernels with three convolution directions or none), 8 LGF2, the lattice Green's
function of the second-order discrete Laplacian (oracle/lgf.py; three convolution
directions or none).  Kind: 0 Poisson, 1 Biot-Savart (spectral curl),
2 / 3 / 4 Biot-Savart with the finite-difference curl of order 2 / 4 / 6.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "oracle.cpp")

EVEN, ODD, PER, UNB = 0, 1, 2, 3
CELL, NODE = 0, 1
FAST, NAIVE, DIRECT = 0, 1, 2
# FFTW-numbered real-to-real kinds
REDFT00, REDFT01, REDFT10, REDFT11, RODFT00, RODFT01, RODFT10, RODFT11 = range(8)
CLASS_NAMES = ["P", "EE", "OO", "EO", "OE", "UU", "EU", "OU", "UE", "UO"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP, FP64)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH)
    ):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp", _SRC_PATH]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_fft.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        L.oracle_dft_naive.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        L.oracle_r2r.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        L.oracle_axis_info.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
        L.oracle_green_value.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_green_value.restype = ctypes.c_double
        L.oracle_solve.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_solve_vector.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_green_spectrum.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.oracle_spectral_dims.argtypes = [ip, dp, ip, ctypes.c_int, ip]
        L.oracle_direct_points.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, dp]
        L.oracle_transform.argtypes = [ip, dp, ip, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_lgf.argtypes = [dp, ctypes.c_long, ctypes.c_long, ctypes.c_long]
        L.oracle_set_lgf.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle error {rc}")


def fft(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _check(lib().oracle_fft(x.size, _dp(x.view(np.float64)), _dp(y.view(np.float64)), sign))
    return y


def dft_naive(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _check(lib().oracle_dft_naive(x.size, _dp(x.view(np.float64)), _dp(y.view(np.float64)), sign))
    return y


def r2r(kind, x, naive=False):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    _check(lib().oracle_r2r(kind, x.size, _dp(x), _dp(y), 1 if naive else 0))
    return y


def axis_info(N, h, node, bl, br):
    info = np.zeros(12, dtype=np.int32)
    _check(lib().oracle_axis_info(N, h, node, bl, br, _ip(info)))
    keys = ["cls", "nuser", "nspec", "nlog", "fwd", "bwd", "first", "kshift", "unb", "dft", "rev", "half2"]
    d = dict(zip(keys, (int(v) for v in info)))
    d["cls_name"] = CLASS_NAMES[d["cls"]]
    return d


def green_value(du, variant, cellvol, rho, k):
    return lib().oracle_green_value(du, variant, cellvol, rho, k)


def _prep(n, h, bc):
    n = np.ascontiguousarray(n, dtype=np.int32)
    h = np.ascontiguousarray(h, dtype=np.float64)
    bc = np.ascontiguousarray(np.asarray(bc).reshape(-1), dtype=np.int32)
    assert n.size == 3 and h.size == 3 and bc.size == 6
    return n, h, bc


def user_shape(n, layout):
    """(nz, ny, nx) of the user's array."""
    add = 1 if layout == NODE else 0
    return (int(n[2]) + add, int(n[1]) + add, int(n[0]) + add)


LGF2 = 8
_lgf_keep = {}


def _prepare_lgf(n, h, bc, green):
    """LGF2 with three convolution directions: tabulate the lattice Green's function at
    offsets up to 2N along each axis and hand it to the oracle."""
    if green != LGF2:
        return
    bcs = np.asarray(bc).reshape(3, 2)
    if not all((3 in bcs[a]) for a in range(3)):
        return  # spectral form, or a mix the oracle refuses
    from .lgf import lgf_table
    ext = tuple(2 * int(v) + 1 for v in n)
    key = (ext, tuple(float(v) for v in h))
    if key not in _lgf_keep:
        _lgf_keep.clear()
        _lgf_keep[key] = lgf_table(ext, h)
    t = _lgf_keep[key]
    lib().oracle_set_lgf(_dp(t), ext[0], ext[1], ext[2])


def solve(rhs, n, h, bc, layout, green=0, kind=0, mode=FAST):
    """Solve lap(u) = f (kind 0) or lap(u) = curl(f) (kind 1: spectral derivative; 2, 3, 4:
    finite-difference derivative of order 2, 4, 6).

    rhs: array [nz, ny, nx] (Poisson) or [3, nz, ny, nx] (Biot-Savart), FP64.
    n: intervals (node) or cells (cell) per axis (x, y, z); h: spacing per axis;
    bc: [[xl, xr], [yl, yr], [zl, zr]].
    """
    n, h, bc = _prep(n, h, bc)
    shp = user_shape(n, layout)
    ncomp = 3 if kind >= 1 else 1
    rhs = np.ascontiguousarray(rhs, dtype=np.float64).reshape((ncomp,) + shp)
    out = np.empty_like(rhs)
    _prepare_lgf(n, h, bc, green)
    _check(lib().oracle_solve(_ip(n), _dp(h), _ip(bc), layout, green, kind, mode, _dp(rhs), _dp(out)))
    return out if kind >= 1 else out[0]


def swap_faces(bcv):
    """The faces of the velocity for source faces bcv [3][3][2]: even and odd swapped."""
    sw = {EVEN: ODD, ODD: EVEN, PER: PER, UNB: UNB}
    return [[[sw[int(f)] for f in ax] for ax in comp] for comp in np.asarray(bcv).tolist()]


def solve_vector(rhs, n, h, bcv, layout, green=0, kind=1, mode=FAST):
    """Biot-Savart lap(u) = curl(f) with boundary conditions per component (Sec. V).

    bcv: [3][3][2], per component (x, y, z) the [[xl, xr], [yl, yr], [zl, zr]] faces.
    Periodic and unbounded faces are shared by the components; on a symmetric face of
    axis a the component along a has one symmetry and the two others the opposite one.
    Component p of the result has the faces of component p with even and odd swapped
    (swap_faces).  kind 1 spectral derivative, 2 / 3 / 4 finite differences.
    rhs: [3, nz, ny, nx] FP64."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    h = np.ascontiguousarray(h, dtype=np.float64)
    b = np.ascontiguousarray(np.asarray(bcv).reshape(-1), dtype=np.int32)
    assert n.size == 3 and h.size == 3 and b.size == 18
    shp = user_shape(n, layout)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64).reshape((3,) + shp)
    out = np.empty_like(rhs)
    _prepare_lgf(n, h, b[:6], green)
    _check(lib().oracle_solve_vector(_ip(n), _dp(h), _ip(b), layout, green, kind, mode, _dp(rhs), _dp(out)))
    return out


def direct_points(rhs, n, h, bc, layout, points, green=0):
    """u at the given user points [(ix, iy, iz), ...] by the direct convolution sum
    (Poisson; every axis fully or semi-unbounded).  rhs: [nz, ny, nx] FP64."""
    n, h, bc = _prep(n, h, bc)
    shp = user_shape(n, layout)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64).reshape(shp)
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int32).reshape(-1, 3))
    out = np.empty(len(pts))
    _prepare_lgf(n, h, bc, green)
    _check(lib().oracle_direct_points(_ip(n), _dp(h), _ip(bc), layout, green, _dp(rhs), len(pts),
                                      pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out)))
    return out


def spectral_dims(n, h, bc, layout):
    n, h, bc = _prep(n, h, bc)
    d = np.zeros(3, dtype=np.int32)
    _check(lib().oracle_spectral_dims(_ip(n), _dp(h), _ip(bc), layout, _ip(d)))
    return tuple(int(v) for v in d)  # (x, y, z)


def green_spectrum(n, h, bc, layout, green=0, mode=FAST):
    """Green's spectrum (with quadrature weight and 1/prod(nlog)), array [sz][sy][sx]."""
    n, h, bc = _prep(n, h, bc)
    dx, dy, dz = spectral_dims(n, h, bc, layout)
    out = np.empty((dz, dy, dx), dtype=np.complex128)
    _prepare_lgf(n, h, bc, green)
    _check(lib().oracle_green_spectrum(_ip(n), _dp(h), _ip(bc), layout, green, mode, _dp(out.view(np.float64))))
    return out


def forward(f, n, h, bc, layout):
    """Forward transforms of every axis (no spectral multiplication), unnormalised:
    complex spectrum [sz][sy][sx], full length along every axis."""
    n, h, bc = _prep(n, h, bc)
    shp = user_shape(n, layout)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(shp)
    dx, dy, dz = spectral_dims(n, h, bc, layout)
    out = np.empty((dz, dy, dx), dtype=np.complex128)
    _check(lib().oracle_transform(_ip(n), _dp(h), _ip(bc), layout, -1, _dp(f), _dp(out.view(np.float64))))
    return out


def backward(F, n, h, bc, layout):
    """Backward transforms of every axis with the crop and fix-ups, unnormalised: the real
    part on the user grid [nz][ny][nx]."""
    n, h, bc = _prep(n, h, bc)
    F = np.ascontiguousarray(F, dtype=np.complex128)
    out = np.empty(user_shape(n, layout))
    _check(lib().oracle_transform(_ip(n), _dp(h), _ip(bc), layout, +1, _dp(F.view(np.float64)), _dp(out)))
    return out


def num_threads():
    return lib().oracle_num_threads()


def set_num_threads(n):
    """OpenMP threads of later oracle calls."""
    lib().oracle_set_num_threads(int(n))
