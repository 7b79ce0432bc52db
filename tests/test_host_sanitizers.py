"""The boundary's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no device).

The library's host sources (host.cpp, tables.cpp) are compiled again with both sanitizers on the
host side only (the gfx950 code objects stay as built), linked with the kernels' objects into a
separate shared library, and driven by `host_abi_driver.c`, itself sanitized: problem
validation, null contexts on every entry point, and the set-up's failure and clean-up path when
no device is present (its success path where one is).  Leaks are checked; the HIP runtime's own
allocations are suppressed."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2005_00331_amd")
CLANG = "/opt/rocm/llvm/bin/clang"


def _kernel_objects():
    from paper_2005_00331_amd import build as b
    objs = [os.path.join(PKG, "_build", os.path.splitext(s)[0] + ".o") for s in b.SOURCES]
    if not all(os.path.exists(o) for o in objs):
        b.build()
    return b, [o for o in objs if not o.endswith(("host.o", "tables.o"))]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    b, kobjs = _kernel_objects()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    objs = []
    for src in ("host.cpp", "tables.cpp"):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.run([b.HIPCC, *b.CXXFLAGS, *san, "-x", "hip", "-c", os.path.join(b.CSRC, src), "-o", obj],
                       check=True, capture_output=True)
        objs.append(obj)
    lib = str(tmp_path / "libmfpff_san.so")
    subprocess.run([b.HIPCC, "-shared", "-fPIC", f"--offload-arch={b.ARCH}", *san, *objs, *kobjs, "-o", lib],
                   check=True, capture_output=True)
    exe = str(tmp_path / "driver")
    subprocess.run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "host_abi_driver.c"),
                    "-o", exe, "-L", str(tmp_path), "-lmfpff_san", f"-Wl,-rpath,{tmp_path}", "-lm"],
                   check=True, capture_output=True)
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               LSAN_OPTIONS=f"suppressions={supp}", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
