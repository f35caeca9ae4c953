"""Build the gfx950 shared library ``libfp.so`` in place.

Compiles ``csrc/fp_inst.hip`` once per (precision, reconstruction) pair and
``csrc/fp_api.hip`` in parallel with hipcc for gfx950, then links them.
Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfp.so")
ARCH = os.environ.get("FP_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]

UNITS = [("fp_inst.hip", ["-DFP_INST_PREC=0", "-DFP_INST_RECON=0"], "inst_p0_r0.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=0", "-DFP_INST_RECON=1"], "inst_p0_r1.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=1", "-DFP_INST_RECON=0"], "inst_p1_r0.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=1", "-DFP_INST_RECON=1"], "inst_p1_r1.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=0", "-DFP_INST_RECON=2"], "inst_p0_r2.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=1", "-DFP_INST_RECON=2"], "inst_p1_r2.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=0", "-DFP_INST_RECON=3"], "inst_p0_r3.o"),
         ("fp_inst.hip", ["-DFP_INST_PREC=1", "-DFP_INST_RECON=3"], "inst_p1_r3.o"),
         ("fp_api.hip", [], "api.o")]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.isabs(c) and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="fpbuild_") as tmp:
        procs = []
        for src, defs, obj in UNITS:
            cmd = [cc, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", os.path.join(tmp, obj)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        failed = []
        for cmd, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if p.returncode != 0:
                failed.append((cmd, text))
            elif verbose and text.strip():
                print(text)
        if failed:
            msg = "\n".join(" ".join(c) + "\n" + t for c, t in failed)
            raise RuntimeError("hipcc failed:\n" + msg)
        tmp_lib = LIB + ".tmp"
        cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}",
               *[os.path.join(tmp, o) for _, _, o in UNITS], "-o", tmp_lib]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
