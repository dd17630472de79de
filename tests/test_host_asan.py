"""The library's host logic (validation, layouts, descriptor and graph
building, the batch engine, serving-style admit/remove cycles, Scheme I's
driver, the 3-D solver) run on the CPU under AddressSanitizer.

The library sources are compiled host-only (no device code) and linked
against tests/hostcheck/hipstub.cpp, a stand-in HIP runtime in which "device"
memory is host memory, kernels are not run, and events, graphs and executable
graphs are tracked so that a use after destroy or a double destroy aborts.
tests/hostcheck/harness.cpp drives the same call sequences as bench.py and the
serving loop.  No GPU is involved."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG) and shutil.which("nm")),
                    reason="no ROCm toolchain")
def test_host_logic_under_address_sanitizer(tmp_path):
    csrc = os.path.join(ROOT, "paper_1909_02894_amd", "csrc")
    here = os.path.join(ROOT, "tests", "hostcheck")
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))

    def compile_one(f):
        obj = os.path.join(tmp_path, f[:-4] + ".o")
        cmd = [HIPCC, "--offload-host-only", "-O1", "-g", "-fPIC", "-std=c++17",
               "-Xarch_host", "-fsanitize=address", "-c", os.path.join(csrc, f), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(compile_one, srcs))
    stub = os.path.join(tmp_path, "hipstub.o")
    r = subprocess.run([HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-g", "-fPIC",
                        "-Xarch_host", "-fsanitize=address", "-c", os.path.join(here, "hipstub.cpp"), "-o", stub],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    # host-only objects name one fat-binary symbol per translation unit; give
    # each an empty definition (the stub runtime registers nothing)
    names = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True)
        names |= {ln.split()[-1] for ln in r.stdout.splitlines() if "__hip_fatbin_" in ln}
    fat = os.path.join(tmp_path, "fatbins.c")
    with open(fat, "w") as fh:
        fh.write("".join(f"char {n}[16];\n" for n in sorted(names)))
    fat_o = os.path.join(tmp_path, "fatbins.o")
    r = subprocess.run([CLANG, "-x", "c", "-c", fat, "-o", fat_o], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    objs.append(fat_o)
    exe = os.path.join(tmp_path, "harness")
    link = [CLANG, "-std=c++17", "-g", "-O1", "-fsanitize=address", "-I" + os.path.join(ROOT, "include"),
            "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", os.path.join(here, "harness.cpp"), *objs, stub,
            "-o", exe]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "serve ok" in r.stdout
