"""The special functions that the device uses to generate Green's spectra (fm_special.h:
K0 / K1 for the two-unbounded-direction kernels, Si for HEJ0, exp(-x) I_n(x) for LGF2),
built for the host from the same source and checked against scipy over the argument
ranges the generation uses."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
from scipy import special

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "special", "special_host.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("special") / "libspecial.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out, SRC])
    L = ctypes.CDLL(out)
    L.sf_bessel_k.argtypes = [ctypes.c_int, ctypes.c_double]
    L.sf_bessel_k.restype = ctypes.c_double
    L.sf_sine_integral.argtypes = [ctypes.c_double]
    L.sf_sine_integral.restype = ctypes.c_double
    L.sf_scaled_bessel_row.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    return L


def test_bessel_k0_k1(lib):
    """K_nu(x), nu = 0, 1, against scipy's kv: x = k rho and k r_eq of the kernels with two
    convolution directions span about 1e-3 ... 1e3 (the kernel underflows beyond 700)."""
    xs = np.concatenate([np.geomspace(1e-4, 25, 300), np.geomspace(25, 600, 100)])
    for nu in (0, 1):
        got = np.array([lib.sf_bessel_k(nu, x) for x in xs])
        ref = special.kv(nu, xs)
        assert np.max(np.abs(got - ref) / ref) < 5e-15, nu


def test_sine_integral(lib):
    xs = np.concatenate([np.linspace(0, 10, 1001), np.geomspace(10, 2e5, 500)])
    got = np.array([lib.sf_sine_integral(x) for x in xs])
    ref = special.sici(xs)[0]
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)) < 2e-15


def test_scaled_bessel_rows(lib):
    """exp(-x) I_n(x), n < count, against scipy's ive (x < 1e9, where scipy's is defined)
    across the series, recurrence and large-argument regimes."""
    worst = 0.0
    for count in (3, 65, 1025):
        for x in np.concatenate([np.geomspace(1e-12, 1, 10), np.geomspace(1, 1e9, 40)]):
            row = np.zeros(count)
            lib.sf_scaled_bessel_row(x, count, row.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            ref = special.ive(np.arange(count), x)
            worst = max(worst, float(np.max(np.abs(row - ref)) / np.max(ref)))
    assert worst < 1e-13, worst
