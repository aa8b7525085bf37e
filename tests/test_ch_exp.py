"""The generated kernels' branch-free exp (csrc/chem_exp.inc) against the C
library's exp on the host: the same source text is compiled for the CPU and
evaluated on 2e7 arguments spread over [-745, 709] plus the range the rate
expressions use most; every result must lie within 1 ulp of libm's."""
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2405_05974_amd", "csrc", "chem_exp.inc")

HARNESS = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#define __device__
#define __forceinline__ inline
%s
static int64_t ord(double v) {   // monotone integer image of a finite double
  int64_t b; std::memcpy(&b, &v, 8);
  return b < 0 ? INT64_MIN - b : b;
}
int main() {
  std::mt19937_64 g(2405);
  std::uniform_real_distribution<double> wide(-745.0, 709.0), rates(-120.0, 80.0);
  int64_t worst = 0; double at = 0.0; long n = 0;
  for (long i = 0; i < 20000000; ++i) {
    const double x = (i & 1) ? wide(g) : rates(g);
    const int64_t d = std::llabs(ord(ch_exp(x)) - ord(std::exp(x)));
    if (d > worst) { worst = d; at = x; }
    ++n;
  }
  std::printf("%%ld %%lld %%.17g\n", n, (long long)worst, at);
  return 0;
}
"""


def test_ch_exp_within_one_ulp_of_libm():
    text = open(INC).read()
    body = text[text.index('R"CHEXP(') + len('R"CHEXP('):text.rindex(')CHEXP"')]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "chexp.cpp")
        exe = os.path.join(d, "chexp")
        open(src, "w").write(HARNESS % body)
        subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", src, "-o", exe, "-lm"], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    n, worst, at = int(out[0]), int(out[1]), float(out[2])
    print(f"ch_exp vs libm exp: {n} arguments, worst {worst} ulp at x = {at!r}")
    assert n == 20000000
    assert worst <= 1
