"""The host planning code (fm_plan.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, device entry points stubbed) and driven over thousands of
random and invalid problems, fm_plan_create's failure and cleanup path without a device,
and NULL / out-of-range arguments (tests/sanitize/host_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2211_07777_amd", "csrc")
ROCM = "/opt/rocm"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_planner_under_sanitizers(tmp_path):
    flags = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    objs = []
    for src in (os.path.join(CSRC, "fm_plan.cpp"), os.path.join(HERE, "sanitize", "stubs.cpp"),
                os.path.join(HERE, "sanitize", "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call(["g++"] + flags + ["-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    subprocess.check_call(["g++"] + flags + objs + ["-o", exe, "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                                                    "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(res.stdout[-2000:], res.stderr[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "planned" in res.stdout
