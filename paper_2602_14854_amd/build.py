"""Build the HIP shared library libdd_dlra.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["dd_api.hip", "dd_kernels_ts.hip", "dd_kernels_small.hip", "dd_wide.hip"]
LIB = os.path.join(HERE, "libdd_dlra.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Tall-skinny kernels (k_*, kw_*) stream their operands through registers;
# any private (scratch) memory there is a register spill or a local array the
# compiler could not keep in registers, both of which multiply HBM traffic.
_TS_KERNEL = re.compile(r"_ZN2dd\d+kw?_")


def scratch_report(text: str):
    """[(kernel, scratch bytes per lane)] from the compiler's
    kernel-resource-usage remarks."""
    out, name = [], None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name is not None:
            out.append((name, int(m.group(1))))
            name = None
    return out


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "csrc", src.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS[:-4], "-c", *FLAGS[-4:], "-Rpass-analysis=kernel-resource-usage", *inc,
               os.path.join(HERE, "csrc", src), "-o", obj]
        cmd = [c for c in cmd if c != "-shared"]
        objs.append(obj)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    ok = True
    spills = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0 or verbose:
            sys.stderr.write("\n".join(l for l in out.splitlines() if "kernel-resource-usage" not in l) + "\n")
        if p.returncode != 0:
            ok = False
            sys.stderr.write(f"compile of {src} failed\n")
        spills += [(k, b) for k, b in scratch_report(out) if b > 0 and _TS_KERNEL.match(k)]
    if not ok:
        raise RuntimeError("HIP compile failed")
    if spills:
        raise RuntimeError("tall-skinny kernels use scratch memory: " + ", ".join(f"{k} ({b} B/lane)" for k, b in spills))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
