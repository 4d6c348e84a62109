"""Build the gfx950 LBRMT library (``liblbrmt.so``) in-tree with hipcc.

``python -m paper_2402_12696_amd.build_lib`` or ``build()`` compiles every
``csrc/*.hip`` file for gfx950 and links them into
``paper_2402_12696_amd/liblbrmt.so``.  The reference-map kernels are compiled
without floating-point contraction (their discrete decisions are taken in plain
IEEE double); the lattice Boltzmann kernels fuse multiply-adds only within one
source expression, so all their launch variants round identically.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbrmt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]
PER_FILE = {
    # contraction only inside one source expression: every launch variant of
    # the lattice update then rounds identically
    "k_lb.hip": ["-ffp-contract=on"],
    "k_band.hip": ["-ffp-contract=off"],
    "k_diag.hip": ["-ffp-contract=off"],
    "k_adjoint.hip": ["-ffp-contract=off"],
}
SOURCES = ["k_lb.hip", "k_band.hip", "k_diag.hip", "k_adjoint.hip", "lbrmt_api.hip"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + out)
    return out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [HIPCC, *COMMON, *PER_FILE.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        out = _run(cmd)
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
