"""Division by a fixed divisor with a multiply-high and a shift, as the
kernels use it for block and tile coordinates (host build of the same
header, no GPU): every quotient must equal integer division for numerators
below 2^31."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2401_10878_amd import build as B  # noqa: E402

PROGRAM = r"""
#include "context.h"
#include <cstdio>
#include <cstdlib>
int main() {
  unsigned long long checked = 0;
  unsigned seed = 12345u;
  for (unsigned d = 1; d <= 70000; d = d < 4200 ? d + 1 : d + 97) {
    const hlbm::FastDiv f = hlbm::make_fastdiv(d);
    // around multiples of d (both sides) and pseudo-random numerators
    for (unsigned k = 0; k < 64; ++k) {
      seed = seed * 1664525u + 1013904223u;
      const unsigned long long base = (unsigned long long)d * ((seed >> 1) / d);
      for (int off = -2; off <= 2; ++off) {
        const long long n = (long long)base + off;
        if (n < 0 || n >= (1ll << 31)) continue;
        const unsigned q = hlbm::fdiv((unsigned)n, f);
        if (q != (unsigned)n / d) { printf("FAIL d=%u n=%lld q=%u\n", d, n, q); return 1; }
        ++checked;
      }
      const unsigned n = seed & 0x7fffffffu;
      if (hlbm::fdiv(n, f) != n / d) { printf("FAIL d=%u n=%u\n", d, n); return 1; }
      ++checked;
    }
    const unsigned top = 0x7fffffffu;
    if (hlbm::fdiv(top, f) != top / d) { printf("FAIL d=%u top\n", d); return 1; }
    if (hlbm::fdiv(0u, f) != 0u) { printf("FAIL d=%u zero\n", d); return 1; }
  }
  printf("OK %llu\n", checked);
  return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_fastdiv_matches_integer_division(tmp_path):
    src = tmp_path / "fastdiv_check.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "fastdiv_check"
    r = subprocess.run([B.HIPCC, "--cuda-host-only", "-O2", "-std=c++17",
                        "-I", B.CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
