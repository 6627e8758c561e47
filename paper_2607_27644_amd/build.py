"""Builds librbp.so (HIP for gfx950) in the package directory.

Every source is compiled for gfx950 only, with FP contraction off (the decoder's
float operations are specified one by one) and with the packed-FP32 VALU
instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbp.so")
SOURCES = ["rbp_common.hip", "rbp_decode.hip", "rbp_mlp.hip", "rbp_spa.hip", "rbp_window.hip", "rbp_probe.hip"]
# Test build of the proposal network with FP32 operands (same kernels, FP32
# matrix cores): its gradients are checked element by element against the
# float64 reference.  Not part of the product path.
LIB_MLP_F32 = os.path.join(HERE, "librbp_mlp_f32.so")
MLP_F32_SOURCES = [("rbp_common.hip", []), ("rbp_mlp.hip", ["-DRBP_MLP_FP32"])]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(jobs, verbose):
    """jobs: (source, extra flags, object path); compiled in parallel."""
    procs = []
    for src, extra, obj in jobs:
        cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    for src, p in procs:
        out, _ = p.communicate()
        msgs = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
        if verbose and msgs:
            print("\n".join(msgs))


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of {os.path.basename(lib)} failed:\n{r.stdout}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    main = [(src, [], os.path.join(CSRC, src.replace(".hip", ".o"))) for src in SOURCES]
    f32 = [(src, extra, os.path.join(CSRC, src.replace(".hip", "_f32.o"))) for src, extra in MLP_F32_SOURCES]
    _compile(main + f32, verbose)
    _link([o for _, _, o in main], LIB)
    _link([o for _, _, o in f32], LIB_MLP_F32)
    for _, _, o in main + f32:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
