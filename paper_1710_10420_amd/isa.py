"""Instruction counts of the pass kernels' marching loops, read from the
gfx950 code this package builds.

The multi-step passes sit close to the vector-ALU issue limit as well as the
HBM limit, so the benchmark reports both fractions; the issue fraction needs
the number of vector instructions a wave issues per march iteration, which is
a property of the compiled code.  This module pulls the gfx950 code object
out of the compiled kernel objects (clang-offload-bundler), disassembles it
(llvm-objdump) and, for every pass kernel, counts the instructions of its
steady-state march loop: the span from the head of the loop (the target of
the most backward branches) to its last backward branch.

    python -m paper_1710_10420_amd.isa [object files ...]

prints the counts as JSON; build.py writes them to isa_counts.json next to
the library after every build, and the benchmark reads that file.
"""
import json
import os
import re
import subprocess
import sys
import tempfile

LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"

# k_<name>I<template args>EEv...: integer (Li<n>E), bool (Lb<0|1>E) and the
# field type (f float, d double)
_KERNEL = re.compile(r"^([0-9a-f]+) <_ZN3prs12_GLOBAL__N_1\d+(k_\w+?)I((?:Li\d+E|Lb[01]E)+)([fd])E")
_INSN = re.compile(r"^\s+([a-z_0-9]+)\b[^/]*//\s*([0-9A-F]+):")
_BRANCH_TARGET = re.compile(r"<[^>]*\+0x([0-9a-f]+)>")


def _tool(name):
    path = os.path.join(LLVM, name)
    if not os.path.exists(path):
        raise FileNotFoundError(path)
    return path


def disassemble(obj):
    """gfx950 disassembly of the device code embedded in a host object
    ("" when the object holds no device code)."""
    sections = subprocess.run([_tool("llvm-readelf"), "-S", obj], check=True, capture_output=True, text=True)
    if ".hip_fatbin" not in sections.stdout:
        return ""
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fatbin")
        dev = os.path.join(d, "dev.co")
        subprocess.run([_tool("llvm-objcopy"), "--dump-section=.hip_fatbin=" + fat, obj, os.path.join(d, "x")],
                       check=True, capture_output=True)
        subprocess.run([_tool("clang-offload-bundler"), "--unbundle", "--type=o", "--input=" + fat,
                        "--targets=" + TARGET, "--output=" + dev], check=True, capture_output=True)
        out = subprocess.run([_tool("llvm-objdump"), "-d", "--no-show-raw-insn", dev], check=True,
                             capture_output=True, text=True)
    return out.stdout


def _template_args(s):
    return [int(v) for v in re.findall(r"L[ib](\d+)E", s)]


def loop_counts(asm):
    """{kernel label: counts of its steady-state loop} for the prs kernels in
    a disassembly.  A label reads k_name<args,type>, e.g. k_tb2d<2,8,0,1,f>
    (VEC 2, 8 steps per pass, no diagnostics, unit spacing, float32)."""
    out = {}
    cur = None
    body = []

    def finish():
        if cur is None or not body:
            return
        base = body[0][0]
        # back-edges grouped by target; the march loop is unrolled by four
        # and its head is the target of the most back-edges (every unrolled
        # iteration may leave through it); ties go to the longer span
        edges = {}
        for addr, op, tgt in body:
            if tgt is not None and op.startswith("s_") and "branch" in op and base + tgt < addr:
                edges.setdefault(base + tgt, []).append(addr)
        if not edges:
            return
        head = max(edges, key=lambda t: (len(edges[t]), max(edges[t]) - t))
        best = (head, max(edges[head]))
        c = {"valu": 0, "salu": 0, "vmem_load": 0, "vmem_store": 0, "lds": 0, "other": 0}
        for addr, op, _ in body:
            if not best[0] <= addr <= best[1]:
                continue
            if op.startswith("v_"):
                c["valu"] += 1
            elif op.startswith("s_"):
                c["salu"] += 1
            elif op.startswith(("buffer_load", "global_load")):
                c["vmem_load"] += 1
            elif op.startswith(("buffer_store", "global_store")):
                c["vmem_store"] += 1
            elif op.startswith("ds_"):
                c["lds"] += 1
            else:
                c["other"] += 1
        out[cur] = c

    for line in asm.splitlines():
        m = _KERNEL.match(line)
        if m:
            finish()
            cur = "%s<%s,%s>" % (m.group(2), ",".join(str(v) for v in _template_args(m.group(3))), m.group(4))
            body = []
            continue
        if line and not line[0].isspace():
            finish()
            cur, body = None, []
            continue
        if cur is None:
            continue
        mi = _INSN.match(line)
        if not mi:
            continue
        tm = _BRANCH_TARGET.search(line)
        body.append((int(mi.group(2), 16), mi.group(1), int(tm.group(1), 16) if tm else None))
    finish()
    return out


def counts_for_objects(objs):
    res = {}
    for obj in objs:
        res.update(loop_counts(disassemble(obj)))
    return res


if __name__ == "__main__":
    print(json.dumps(counts_for_objects(sys.argv[1:]), indent=1, sort_keys=True))
