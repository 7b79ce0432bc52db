"""Build libmfpff.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["cell_kernel.hip", "tile_kernel.hip", "rowcell_kernel.hip", "linecell_kernel.hip", "mfma_kernel.hip", "vector_ops.hip", "transfer.hip", "dense.hip", "tables.cpp", "host.cpp"]
LIB = os.path.join(HERE, "libmfpff.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MFPFF_ARCH", "gfx950")

CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # keep the compiler away from packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


VARIANTS = {
    # the library the package loads
    "release": ("_build", LIB, []),
    # debug kernel build: every computed node, cell and transfer index checked against its range
    # (bounds.h); loaded only by its own test, through MFPFF_LIB
    "bounds": ("_build_bounds", os.path.join(HERE, "libmfpff_bounds.so"), ["-DMFPFF_BOUNDS"]),
}


def build(verbose=False, jobs=8, variant="release"):
    """Compile every source to an object in the variant's build folder (in parallel), then link
    the variant's shared library."""
    sub, lib, extra = VARIANTS[variant]
    bdir = os.path.join(HERE, sub)
    os.makedirs(bdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC, *CXXFLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, variant="bounds" if "--bounds" in sys.argv else "release"))
