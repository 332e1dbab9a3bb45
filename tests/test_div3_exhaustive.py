"""The fp32 division by 3 of the 3D three-term root (div3 in the 3D device
code): the product with RN(1/3) corrected once by its exact remainder with
two fused multiply-adds (Markstein's correction step), and x = +-0 passed
through.  It must equal the IEEE quotient x / 3 bit for bit for every
finite float; this runs the same sequence in C with the host's fmaf (IEEE
fused multiply-add, as the device's v_fma_f32) over all 2^32 bit patterns."""
import os
import subprocess
import tempfile

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static float div3(float x) {
  const float third = 0x1.555556p-2f;
  const float q0 = x * third;
  const float r = fmaf(-q0, 3.0f, x);
  const float q = fmaf(r, third, q0);
  return x == 0.0f ? x : q;
}
int main(void) {
  unsigned long long bad = 0, n = 0;
  #pragma omp parallel for reduction(+:bad, n) schedule(static)
  for (long long hi = 0; hi < 65536; ++hi) {
    for (uint32_t lo = 0; lo < 65536; ++lo) {
      const uint32_t u = ((uint32_t)hi << 16) | lo;
      float x;
      memcpy(&x, &u, 4);
      if (!isfinite(x)) continue;
      ++n;
      const float ref = x / 3.0f, got = div3(x);
      uint32_t a, b;
      memcpy(&a, &ref, 4);
      memcpy(&b, &got, 4);
      bad += a != b;
    }
  }
  printf("%llu %llu\n", n, bad);
  return 0;
}
"""


def test_div3_equals_ieee_division_for_every_finite_float():
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "div3.c")
        exe = os.path.join(d, "div3")
        with open(c, "w") as f:
            f.write(SRC)
        flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]
        try:
            subprocess.check_call(["gcc", *flags, "-mfma", c, "-o", exe, "-lm"])
        except (OSError, subprocess.CalledProcessError):
            pytest.skip("no gcc with FMA support")
        out = subprocess.check_output([exe], env=dict(os.environ, OMP_NUM_THREADS=str(min(8, os.cpu_count() or 1))))
    n, bad = (int(v) for v in out.split())
    assert n == (1 << 32) - (1 << 24)  # every bit pattern but the 2^24 inf / NaN ones
    assert bad == 0
