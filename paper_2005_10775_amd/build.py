"""Builds libnlasm.so in-tree for gfx950 with hipcc.

The plan translation unit is compiled with -ffp-contract=off (the pair
predicate must round every operation separately); the numeric units keep
contraction on.  Packed FP32 instructions are disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnlasm.so")
ARCH = os.environ.get("NLA_OFFLOAD_ARCH", "gfx950")

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(os.path.dirname(HERE), "include")]
UNITS = {
    "nla_plan.hip": ["-ffp-contract=off"],
    "nla_numeric.hip": [],
    "nla_cg.hip": [],
    "nla_fp32.hip": [],
    "nla_mlp.hip": [],
}


def build(verbose=False, jobs=4):
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src, extra in UNITS.items():
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = ["hipcc", "-c"] + COMMON + extra + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout.decode())
    os.replace(tmp, LIB)
    return LIB


def _wait(procs):
    errs = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            errs.append("%s:\n%s" % (src, out.decode()))
        elif out and b"warning" in out:
            sys.stderr.write(out.decode())
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    print(build(verbose=True))
