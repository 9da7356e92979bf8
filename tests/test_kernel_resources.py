"""Register and scratch budget of the HIP kernels (compiled here, no GPU).

A private array indexed at run time, or a spill, puts per-lane scratch
memory behind every wavefront; on the lattice pass that once cost more HBM
traffic than the populations themselves.  Every kernel must compile without
scratch, and the FP32 / binary16 lattice kernels within 128 VGPRs (four
wavefronts per SIMD).  One exception, bounded: the contact treatment's
variant for ellipsoid types (launched only when such a type is in use), where
the inlined nearest-point bisection leaves the correction box in scratch
(at most 64 bytes per lane)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2401_10878_amd import build as B  # noqa: E402


def _usage(src, tmp_path):
    out = tmp_path / (os.path.basename(src) + ".o")
    flags = [f for f in B.FLAGS if f != "-shared"]
    r = subprocess.run([B.HIPCC] + flags + ["-c", src, "-o", str(out),
                        "-Rpass-analysis=kernel-resource-usage"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"(VGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1).split()[0]] = int(m.group(2))
    return kernels


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("src", B.SOURCES)
def test_no_scratch(src, tmp_path):
    k = _usage(os.path.join(B.CSRC, src), tmp_path)
    if src != "api.hip":
        assert k, "no kernels reported"
    for name, u in k.items():
        if "k_treatILb1ELb1E" in name:     # k_treat<POLY, ELL>: see above
            assert u.get("ScratchSize", 0) <= 64, (name, u)
            continue
        assert u.get("ScratchSize", 0) == 0, (name, u)
        if "k_lattice" in name and ("IfE" in name or "half" in name):
            assert u["VGPRs"] <= 128, (name, u)
