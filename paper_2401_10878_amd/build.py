"""Build the gfx950 HIP library libhlbm.so in-tree.

    python -m paper_2401_10878_amd.build

hipcc for gfx950 only; no FMA contraction (the signed-distance arithmetic
that decides node ownership and contact detection is evaluated exactly as
written); packed FP32 instructions disabled.
"""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhlbm.so")
SOURCES = ["api.hip", "k_particles.hip", "k_detect.hip", "k_lattice.hip",
           "k_contacts.hip", "k_adjoint.hip", "k_fields.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unused-command-line-argument",
         "-Wno-unused-value", "-Wno-unused-result"]


HEADER = os.path.join(os.path.dirname(HERE), "include", "hlbm.h")


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the library's sources: every file in
    csrc/ and include/hlbm.h, by name and content.  Built into the library
    (hlbm_build_hash) so that the binding can refuse a stale build."""
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".h")))
    for f in files + [HEADER]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object in parallel, then link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    sh = source_hash()
    for s in SOURCES:
        o = os.path.join(objdir, s.replace(".hip", ".o"))
        objs.append(o)
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + [
            f'-DHLBM_SOURCE_HASH="{sh}"', "-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[[p.poll() is None for _, p in procs].index(True)][1].wait()
    for s, p in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
