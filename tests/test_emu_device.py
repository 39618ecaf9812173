"""The library's device code and host code built for the CPU against an emulated HIP
runtime (tests/emu: every workgroup of every grid run as host threads, LDS and device
memory checked by AddressSanitizer, UndefinedBehaviorSanitizer on, streams as queues
that run only when the host synchronises), with the FP32 one-launch batched kernels and
the FP32 fused real-to-real kernel of length 32 switched back on (FM_FP32_ONE_LAUNCH).

Replayed: the twelve FP32 and twelve FP64 plans of the batched-equals-single GPU test
(random sizes from {4, 6, 8, 12, 16}, random faces, both layouts), each solved alone in
the default tiling, in every launch mode its passes accept, and with fm_solve_static,
and compared with the FP64 oracle (FP64 1e-12, FP32 1e-5 relative L-infinity); then each
precision's twelve in one fm_solve_batched call, compared bitwise with the single
solves.  Also the 12 x 10 x 9 cell grid with faces EU / EU / EE in both precisions (also
as its passes one call at a time with the second repeated, and as a one-plan batch) and
two more FP32 grids, which join their precision's batch; and Biot-Savart plans with
faces per component on one, two and three symmetric axes (8 x 6 x 8, both layouts and
precisions, the spectral curl and FD4), against the oracle's vector solve; and every
case twice through a server (three slots), its right-hand side copied from pinned memory
on a producer stream created before the server's, so that a solve not ordered after
that copy would read the NaN-filled input."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

PAIRS = [(2, 2), (0, 0), (1, 1), (0, 1), (1, 0), (3, 3), (0, 3), (1, 3), (3, 0), (3, 1)]


def replay_cases():
    lines = []
    for prec in (0, 1):  # FM_F64, FM_F32
        rng = np.random.default_rng(5)
        for i in range(12):
            n = [int(v) for v in rng.choice([4, 6, 8, 12, 16], size=3)]
            bc = [list(PAIRS[j]) for j in rng.integers(10, size=3)]
            layout = int(rng.integers(2))
            lines.append([prec] + n + [0.1, 0.08, 0.12] + sum(bc, []) + [layout, 40 + i])
    for prec in (0, 1):
        lines.append([prec, 12, 10, 9, 0.1, 0.1, 0.1, 0, 3, 0, 3, 0, 0, 0, 7])
    lines.append([1, 16, 16, 16, 0.1, 0.1, 0.1, 3, 3, 3, 3, 3, 3, 0, 8])
    lines.append([1, 16, 8, 16, 0.1, 0.1, 0.1, 2, 2, 0, 1, 3, 3, 1, 9])
    return "\n".join(" ".join(map(str, c)) for c in lines) + "\n"


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_device_code_under_cpu_emulation(tmp_path):
    import build_emu
    exe = build_emu.build(str(tmp_path / "build"))
    cases = tmp_path / "cases.txt"
    cases.write_text(replay_cases())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe, str(cases)], capture_output=True, text=True, env=env, timeout=900)
    out = res.stdout
    print(out[-3000:], res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "emulated cases done, 0 failure(s)" in out
    # the one-launch batches ran and every precision reached the per-wavefront kernels
    for prec, count in (("FP32", 15), ("FP64", 13)):
        assert f"{prec} batched: {count} plans, status 0, {count} bitwise equal" in out
    assert out.count(" vector ") == 12
    assert out.count("status 0 bitwise equal, one-plan batch status 0 bitwise equal") == 2
    assert "serving: 56 requests, status 0, 56 within tolerance" in out
    for prec in ("FP32", "FP64"):
        for mode in (1, 3, 4):
            assert f"{prec} mode {mode}" in out or (prec, mode) == ("FP64", 1)
