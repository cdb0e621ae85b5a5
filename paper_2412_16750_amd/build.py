"""Compile the HIP library ``libidmx.so`` for gfx950, in-tree.

hipcc cross-compiles, so this runs without a GPU.  The kernels file is built
eleven times (IDM_PART = 0..10) in parallel to shorten the build.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libidmx.so"
LIB_PATH = os.path.join(PKG, LIB_NAME)
ARCH = "gfx950"

HIP_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
    # strict FP: no contraction beyond the explicit fmaf() calls, so the
    # backward pass recomputes the forward states bit for bit
    "-ffp-contract=off",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source and link libidmx.so next to this file."""
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    cc = hipcc()
    units = []
    for part in range(11):
        units.append((os.path.join(CSRC, "idm_kernels.hip"), os.path.join(bdir, "idm_kernels_%d.o" % part),
                      ["-DIDM_PART=%d" % part]))
    units.append((os.path.join(CSRC, "idm_api.hip"), os.path.join(bdir, "idm_api.o"), []))
    for extra in ("ego_kernels.hip", "mlp_kernels.hip"):
        src = os.path.join(CSRC, extra)
        if os.path.exists(src):
            units.append((src, os.path.join(bdir, extra.replace(".hip", ".o")), []))

    def compile_one(u):
        src, obj, defs = u
        return _run([cc] + HIP_FLAGS + defs + ["-c", src, "-o", obj])

    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        outs = list(ex.map(compile_one, units))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [u[1] for u in units])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
