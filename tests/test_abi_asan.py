"""The host-side C++ of the library (problem builders, argument and option
checks) built with AddressSanitizer and UBSan and driven by
tests/native/host_paths.cpp, with buffers of exactly the documented sizes.
No GPU is touched; the device code is linked from the regular build."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_04406_amd", "csrc")
KOBJ = os.path.join(ROOT, "paper_2512_04406_amd", "_build", "kernels.hip.o")


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(_hipcc() is None or not os.path.exists(KOBJ),
                    reason="needs hipcc and the regular build (kernels object)")
def test_host_paths_under_address_and_ub_sanitizers(tmp_path):
    hipcc = _hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-std=c++17", "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src in ("api.cpp", "solver.cpp"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call([hipcc, *inc, *san, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    drv = str(tmp_path / "host_paths.o")
    subprocess.check_call([hipcc, *inc, *san, "-c", os.path.join(ROOT, "tests", "native", "host_paths.cpp"),
                           "-o", drv])
    exe = str(tmp_path / "host_paths")
    subprocess.check_call([hipcc, *san, "--offload-arch=gfx950", drv, *objs, KOBJ, "-o", exe,
                           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host paths ok" in r.stdout
