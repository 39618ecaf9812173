"""Build the GPU library (libfluxmi.so) in-tree with hipcc for gfx950.

The pass kernels are compiled once per (precision, length class) from fm_inst.hip
with -D flags, in parallel, then linked with the generation kernels and the host
planner.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfluxmi.so")
HEADERS = ["fm_pass.h", "fm_device.h", "fm_wave.h", "fm_launch.h", "fm_internal.h", "fm_special.h"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
LENGTHS = [0, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048, 4096]
PRECISIONS = ["float", "double"]


def _units():
    units = []
    for t in PRECISIONS:
        for m in LENGTHS:
            defs = [f"-DFM_T={t}", f"-DFM_MC={m}"]
            if t == "float":
                defs.append("-DFM_NO_BATCHED")  # FP32 batches run plan by plan
            units.append((os.path.join(CSRC, "fm_inst.hip"), f"inst_{t}_{m}.o", defs))
    # FP64 lines longer than 2048 (runtime-length class 1)
    units.append((os.path.join(CSRC, "fm_inst.hip"), "inst_double_long.o", ["-DFM_T=double", "-DFM_MC=1"]))
    units.append((os.path.join(CSRC, "fm_gen.hip"), "gen.o", []))
    units.append((os.path.join(CSRC, "fm_plan.cpp"), "plan.o", []))
    units.append((os.path.join(CSRC, "fm_serve.cpp"), "serve.o", []))
    units.append((os.path.join(CSRC, "fm_static.hip"), "static.o", []))
    return units


def _sources():
    return [os.path.join(CSRC, f) for f in ("fm_inst.hip", "fm_gen.hip", "fm_plan.cpp", "fm_serve.cpp",
                                            "fm_static.hip")] + \
        [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(os.path.dirname(HERE), "include", "fluxmi.h")]


def _compile(unit, force=True):
    src, obj, defs = unit
    out = os.path.join(OBJ, obj)
    if not force and os.path.exists(out):
        device = src.endswith(("fm_inst.hip", "fm_gen.hip"))  # include fm_device.h only
        heads = ["fm_pass.h", "fm_device.h", "fm_wave.h", "fm_launch.h", "fm_special.h"] if device else ["fm_pass.h", "fm_internal.h"]
        deps = [src] + [os.path.join(CSRC, h) for h in heads] + [os.path.abspath(__file__)]
        if not device:
            deps.append(os.path.join(os.path.dirname(HERE), "include", "fluxmi.h"))
        if os.path.getmtime(out) >= max(os.path.getmtime(d) for d in deps):
            return out
    cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {obj}:\n" + res.stdout + res.stderr)
    return out


def build_library(force: bool = True, jobs: int | None = None) -> str:
    """Compile libfluxmi.so; with force=False only the objects older than their sources
    (and only when some source is newer than the library)."""
    if not force and os.path.exists(LIB):
        if os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in _sources()):
            return LIB
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, force), _units()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build_library(force="--incremental" not in sys.argv))
