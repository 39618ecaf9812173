"""CPU checks of the GPU library's host side: it loads, exports every entry point the
header declares, and plans every boundary class combination (no device needed)."""
import itertools
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F
from paper_2211_07777_amd import fluxmi as FX

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fluxmi.h")
PAIRS = [(2, 2), (0, 0), (1, 1), (0, 1), (1, 0), (3, 3), (0, 3), (1, 3), (3, 0), (3, 1)]


def test_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(fm_[a-z_]+)\s*\(", text))
    lib = F.library()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(FX.EXPORTED)


def test_error_strings():
    for code in range(-8, 1):
        assert F.error_string(code)


@pytest.mark.parametrize("layout", [0, 1])
def test_plans_every_combination_and_matches_oracle_table(layout):
    n, h = [6, 8, 10], [0.1, 0.2, 0.3]
    cost = {"P": 2, "EE": 0, "OO": 0, "EO": 0, "OE": 0, "UU": 3, "EU": 1, "OU": 1, "UE": 1, "UO": 1}
    for combo in itertools.product(PAIRS, repeat=3):
        for prec in (F.F64, F.F32):
            info = F.plan_inspect(n, h, combo, layout, F.CHAT2, prec)
            costs = [cost[info["axis_class"][a]] for a in info["order"]]
            assert costs == sorted(costs)
            for a in range(3):
                o = O.axis_info(n[a], h[a], layout, *combo[a])
                assert info["axis_class"][a] == o["cls_name"]
                if o["dft"]:
                    assert info["fft_len"][a] == o["nspec"]
                else:
                    assert info["spec_len"][a] == o["nspec"]
                    assert info["fft_len"][a] == o["nlog"] * (2 if o["unb"] else 1) // (2 if o["unb"] else 1)


def test_rejects_bad_arguments():
    with pytest.raises(F.FluxmiError) as e:
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[2, 0], [3, 3], [3, 3]], 0)
    assert e.value.status == -2
    with pytest.raises(F.FluxmiError) as e:
        F.plan_inspect([1, 8, 8], [0.1] * 3, [[3, 3]] * 3, 0)
    assert e.value.status == -3
    with pytest.raises(F.FluxmiError) as e:
        F.plan_inspect([22, 8, 8], [0.1] * 3, [[2, 2], [3, 3], [3, 3]], 0)  # factor 11
    assert e.value.status == -3
    with pytest.raises(F.FluxmiError) as e:
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[0, 0], [3, 3], [3, 3]], 0, kind=F.BIOT_SAVART, ncomp=3)
    assert e.value.status == -4
    with pytest.raises(F.FluxmiError) as e:
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[3, 3]] * 3, 0, kind=F.BIOT_SAVART, ncomp=1)
    assert e.value.status == -4


def test_regularised_kernels_need_three_or_no_unbounded_directions():
    for g in (F.HEJ2, F.HEJ4, F.HEJ6, F.HEJ8, F.HEJ10, F.HEJ0, F.LGF2):
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[3, 3]] * 3, 0, g)
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[0, 3], [3, 1], [3, 3]], 1, g)
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[2, 2], [0, 1], [1, 1]], 0, g)
        for bc in ([[3, 3], [2, 2], [2, 2]], [[3, 3], [3, 3], [0, 0]]):
            with pytest.raises(F.FluxmiError) as e:
                F.plan_inspect([8, 8, 8], [0.1] * 3, bc, 0, g)
            assert e.value.status == -4
    with pytest.raises(F.FluxmiError) as e:
        F.plan_inspect([8, 8, 8], [0.1] * 3, [[3, 3]] * 3, 0, 9)
    assert e.value.status == -4


def test_workspace_and_padding_sizes():
    # fully unbounded 512^3 cell, FP32, 3 components: two spectral buffers per component
    info = F.plan_inspect([512] * 3, [2 / 512] * 3, [[3, 3]] * 3, 0, F.CHAT2, F.F32, F.BIOT_SAVART, 3)
    v1 = 513 * 512 * 512 * 8
    v2 = 513 * 1024 * 512 * 8
    assert info["workspace_bytes"] == 3 * (v1 + v2)
    assert info["fft_len"] == [1024] * 3
    assert info["spec_len"] == [513, 1024, 1024]
    assert info["green_dims"] == [513, 513, 513]


@pytest.mark.parametrize("prec,values", [(F.F64, 256 * 8), (F.F32, 256 * 16)])
def test_tile_input_fits_register_stage(prec, values):
    # The inverse real-to-complex pass reads two Hermitian half-spectra (M/2 + 1 complex
    # values each) per FFT line: its tile must still fit the register stage of the
    # persistent kernels, or the tail of the tile is never loaded.
    n, h = [128, 128, 256], [1 / 128] * 3
    info = F.plan_inspect(n, h, [[2, 2], [0, 1], [3, 3]], 1, F.CHAT2, prec)
    assert info["order"] == [1, 0, 2]
    assert info["lines_per_tile"][3] * 65 <= values
    # every length a periodic axis may take, both layouts: the planner's own validator
    # rejects a tile that overflows the stage, so planning must succeed
    for m in (4, 8, 16, 32, 64, 96, 128, 256, 512, 1024, 2048, 4096):
        for layout in (0, 1):
            F.plan_inspect([m, 8, 6], [0.1] * 3, [[2, 2], [0, 1], [3, 3]], layout, F.CHAT2, prec)
            F.plan_inspect([6, m, 8], [0.1] * 3, [[3, 3], [2, 2], [3, 3]], layout, F.CHAT2, prec)


def test_biot_savart_512_plans_in_both_precisions():
    # three components of a 1024-point line do not fit 8 FP64 values per thread: the
    # fused pass falls back to the 16-value kernel class instead of failing
    for prec in (F.F32, F.F64):
        info = F.plan_inspect([512] * 3, [2 / 512] * 3, [[3, 3]] * 3, 0, F.CHAT2, prec, F.BIOT_SAVART, 3)
        assert info["fft_len"] == [1024] * 3
        assert 1 <= info["lines_per_tile"][2] <= 64


def _create_vector(n, h, bcv, layout=0, kind=1, prec=0):
    """fm_plan_create_vector's status on the host (no device: a problem that passes
    planning fails afterwards with FM_E_HIP and leaves no plan)."""
    import ctypes
    lib = F.library()
    n3 = (ctypes.c_int * 3)(*n)
    h3 = (ctypes.c_double * 3)(*h)
    b18 = (ctypes.c_int * 18)(*[int(v) for c in bcv for f in c for v in f])
    handle = ctypes.c_void_p()
    rc = lib.fm_plan_create_vector(ctypes.byref(handle), n3, h3, b18, layout, 0, prec, kind, None)
    assert handle.value is None or rc == 0
    return rc


def test_vector_plan_faces_checked_before_the_device():
    """Faces per component: a mirror-symmetric set with one, two or three symmetric axes
    plans (and then needs the device), one that is not mirror-symmetric is FM_E_BC, the
    Poisson kind is FM_E_KIND."""
    n, h = [8, 8, 8], [0.1] * 3
    U, E, OD, P = 3, 0, 1, 2
    one = [[[OD, OD], [U, U], [U, U]], [[E, E], [U, U], [U, U]], [[E, E], [U, U], [U, U]]]
    two = [[[OD, OD], [E, U], [P, P]], [[E, E], [OD, U], [P, P]], [[E, E], [E, U], [P, P]]]
    three = [[[OD, OD], [E, E], [E, E]], [[E, E], [OD, OD], [E, E]], [[E, E], [E, E], [OD, OD]]]
    for layout in (0, 1):
        for prec in (0, 1):
            assert _create_vector(n, h, one, layout, prec=prec) == -6   # planned; no device
            assert _create_vector(n, h, two, layout, prec=prec) == -6
    for layout in (0, 1):
        assert _create_vector(n, h, three, layout) == -6
    assert _create_vector(n, h, one, kind=0) == -4
    bad = [c[:] for c in one]
    bad[0] = [[E, E], [U, U], [U, U]]            # normal component with the tangential symmetry
    assert _create_vector(n, h, bad) == -2
    mixed = [[[U, U]] * 3, [[P, P], [U, U], [U, U]], [[U, U]] * 3]   # periodic and unbounded mixed
    assert _create_vector(n, h, mixed) == -2
