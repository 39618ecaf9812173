"""Build the CPU emulation of the device code (tests/emu) with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer: the library's kernels and host code
compiled against the emulated HIP runtime, the FP64 oracle and the replay driver.
Test infrastructure only.  Usage: build(out_dir) -> path of the driver executable."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.abspath(os.path.join(HERE, "..", ".."))
CSRC = os.path.join(ROOT, "paper_2211_07777_amd", "csrc")
# the length classes compiled (FFT lengths of grids up to 16 cells per axis); the rest
# are stubs (emu_stubs.cpp)
CLASSES = [0, 32, 48, 64, 96, 128]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
FLAGS = ["-std=c++20", "-O0", "-g", "-I" + os.path.join(HERE, "include"), "-DFM_FP32_ONE_LAUNCH",
         "-Wno-attributes"] + SAN


def _units():
    u = []
    for t in ("float", "double"):
        for mc in CLASSES:
            u.append((os.path.join(CSRC, "fm_inst.hip"), f"inst_{t}_{mc}.o", [f"-DFM_T={t}", f"-DFM_MC={mc}"]))
    for name in ("fm_gen.hip", "fm_static.hip", "fm_plan.cpp", "fm_serve.cpp"):
        u.append((os.path.join(CSRC, name), name.split(".")[0] + ".o", []))
    for name in ("emu_runtime.cpp", "emu_stubs.cpp", "emu_driver.cpp"):
        u.append((os.path.join(HERE, name), name.split(".")[0] + ".o", []))
    return u


def build(out_dir, jobs=8):
    os.makedirs(out_dir, exist_ok=True)

    def compile_one(unit):
        src, obj, defs = unit
        out = os.path.join(out_dir, obj)
        cmd = ["g++"] + FLAGS + defs + ["-x", "c++", "-c", src, "-o", out]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        return out

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, _units()))
    orc = os.path.join(out_dir, "oracle.o")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fopenmp", "-c", os.path.join(ROOT, "oracle", "oracle.cpp"),
                    "-o", orc], check=True)
    exe = os.path.join(out_dir, "emu_driver")
    subprocess.run(["g++"] + SAN + objs + [orc, "-fopenmp", "-pthread", "-o", exe], check=True)
    return exe


if __name__ == "__main__":
    import sys
    print(build(sys.argv[1] if len(sys.argv) > 1 else "/tmp/fluxmi_emu"))
