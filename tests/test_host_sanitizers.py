"""The library's host C++ (argument validation and the FP64 GauSum multiplier of fse_gausum.cpp) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: tests/host_sanitize/check_host.cpp is linked with
fse_api.cpp and fse_gausum.cpp built with both sanitizers (host code only) and the kernel objects built as usual,
and run; a memory error or undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1512_03210_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not available")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from paper_1512_03210_amd import build
    out = str(tmp_path)
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    common = ["-std=c++17", "-O1", "-g", "-I", os.path.join(ROOT, "include")]
    # the API source is HIP (it holds a device array): its host side under the sanitizers, its device side as usual
    host_san = [f for flag in san for f in ("-Xarch_host", flag)]
    _run([CLANG, "-x", "hip", "--offload-arch=gfx950", "--rocm-path=/opt/rocm", *common, *host_san, "-fPIC",
          "-c", os.path.join(CSRC, "fse_api.cpp"), "-o", os.path.join(out, "api.o")])
    _run([CLANG, *common, *san, "-fPIC", "-c", os.path.join(CSRC, "fse_gausum.cpp"), "-o", os.path.join(out, "gausum.o")])
    _run([CLANG, *common, *san, "-c", os.path.join(ROOT, "tests", "host_sanitize", "check_host.cpp"),
          "-o", os.path.join(out, "main.o")])
    # the kernels and their launchers as the library builds them
    objs = []
    for src in ("fse_launch_f64.hip", "fse_launch_f32.hip"):
        obj = os.path.join(build.BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(
                os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC)):
            os.makedirs(build.BUILD, exist_ok=True)
            obj = build._compile(src)
        objs.append(obj)
    exe = os.path.join(out, "check_host")
    _run([CLANG, *san, "--hip-link", "--offload-arch=gfx950", "--rocm-path=/opt/rocm", os.path.join(out, "main.o"),
          os.path.join(out, "api.o"), os.path.join(out, "gausum.o"), *objs,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-5000:]
    assert "host checks passed" in r.stdout
