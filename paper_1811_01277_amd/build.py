"""Build the HIP library libelpahip.so in-tree for gfx950 with hipcc.

Each translation unit is compiled to an object in parallel (the kernel units
hold large fully unrolled step bodies), then the objects are linked.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libelpahip.so")
# the stripe kernel families are split by element type so that their many
# fully unrolled variants compile in parallel
SOURCES = ["elpa_hh.cpp", "hh_tune.cpp", "hh_ws.cpp", "hh_kernels.hip", "hh_stripe_r64.hip",
           "hh_stripe_r32.hip", "hh_stripe_c64.hip", "hh_split.hip", "hh_split_r64.hip",
           "hh_split_r32.hip", "hh_split_c64.hip", "hh_wy.hip", "hh_wy_r64.hip",
           "hh_wy_r32.hip", "hh_wy_c64.hip", "bt2.hip", "b2t.hip", "f2b.hip",
           "gen.hip", "dc.hip", "hh_noalloc.hip", "peak_probe.hip"]
ARCH = os.environ.get("ELPA_HIP_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed fp32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    if verbose and r.stderr.strip():
        # the host pass does not know the device feature flag; harmless
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + "." + tag + ".o") for s in SOURCES]
    cmds = [["hipcc", *FLAGS, "-c", os.path.join(CSRC, s), "-o", o]
            for s, o in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(max_workers=jobs or len(cmds)) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        tmp = LIB + ".tmp" + tag
        _run(["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp,
              "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"], verbose)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
