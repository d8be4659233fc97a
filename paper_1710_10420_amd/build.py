"""Build libprs.so (the HIP kernels and the C ABI) for gfx950, in-tree.

    python -m paper_1710_10420_amd.build

Kernels are compiled with -ffp-contract=off (only the explicit fmaf calls
fuse) and with packed FP32 instructions disabled.

The library is linked against the HIP runtime that PyTorch loads (torch
bundles its own libamdhip64.so), so that one process holds one HIP runtime:
device pointers and streams handed over by torch are then valid in the
library.  Without torch it falls back to the system runtime in /opt/rocm.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libprs.so")

SOURCES = ["prs_ensemble.hip", "prs_kernels.hip", "prs_kernels_f64.hip", "prs_api.cpp"]
ARCH = os.environ.get("PRS_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def hip_runtime_dir():
    """Directory of the libamdhip64.so the process will use."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is not None and spec.origin:
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    return "/opt/rocm/lib"


def clangxx():
    for cand in ("/opt/rocm/llvm/bin/clang++", shutil.which("amdclang++"), shutil.which("g++")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("no C++ linker found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-mcode-object-version=5",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def build(verbose=False):
    """Compile every source (always, even when a library exists) and link
    libprs.so atomically."""
    objs = []
    tmpdir = os.path.join(PKG, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    procs = []
    for src in SOURCES:                       # the sources compile in parallel
        obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), "--offload-arch=" + ARCH, "-c", os.path.join(CSRC, src), "-o", obj] + flags()
        if src.endswith(".cpp"):
            cmd = [hipcc(), "-x", "hip", "--offload-arch=" + ARCH, "-c",
                   os.path.join(CSRC, src), "-o", obj] + flags()
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, pr in procs if pr.wait() != 0]
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    rt = hip_runtime_dir()
    runtime = os.path.join(rt, "libamdhip64.so")
    cmd = [clangxx(), "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L" + rt, "-l:" + os.path.basename(runtime), "-Wl,-rpath," + rt, "-Wl,--no-undefined",
        "-lstdc++", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    write_isa_counts(objs)
    return LIB


ISA_COUNTS = os.path.join(PKG, "isa_counts.json")


def write_isa_counts(objs):
    """Instruction counts of every pass kernel's march loop in this build
    (isa.py), for the benchmark's issue-rate figure; removed when the tools
    are missing so that no stale counts survive a rebuild."""
    import json

    from paper_1710_10420_amd import isa
    try:
        counts = isa.counts_for_objects(objs)
    except (OSError, subprocess.CalledProcessError) as e:
        print("isa counts not written: %s" % e, file=sys.stderr)
        if os.path.exists(ISA_COUNTS):
            os.remove(ISA_COUNTS)
        return
    with open(ISA_COUNTS + ".tmp", "w") as f:
        json.dump(counts, f, indent=0, sort_keys=True)
    os.replace(ISA_COUNTS + ".tmp", ISA_COUNTS)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
