"""The shower's FP64 logarithm (csrc/vsh_math.hpp) against the host's
extended-precision logl: at most 2 ulp over the whole exponent range, near
1, and on uniforms of the Philox conversion (the values the trial scales
take the log of)."""
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2403_08692_amd", "csrc")

PROG = r'''
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include "vsh_math.hpp"
int main() {
  double x;
  while (std::fread(&x, 8, 1, stdin) == 1) {
    const double f = vsh::log_fast(x);
    const long double r = logl((long double)x);
    const double rd = (double)r;
    double ulp = std::nextafter(std::fabs(rd), INFINITY) - std::fabs(rd);
    if (ulp == 0.0 || !std::isfinite(ulp)) ulp = 1e-300;
    const double err = (double)(((long double)f - r) / (long double)ulp);
    std::fwrite(&err, 8, 1, stdout);
  }
  return 0;
}
'''


def _ulp_errors(xs):
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        open(src, "w").write(PROG)
        subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I" + HDR, src, "-o", exe], check=True)
        out = subprocess.run([exe], input=np.ascontiguousarray(xs, np.float64).tobytes(), capture_output=True,
                             check=True).stdout
    return np.frombuffer(out, np.float64)


def test_log_fast_within_two_ulp():
    rng = np.random.default_rng(1)
    wide = np.exp(rng.uniform(-740, 709, 200_000))
    near1 = 1.0 + rng.uniform(-1e-3, 1e-3, 100_000)
    sub = rng.uniform(1e-320, 1e-308, 20_000)
    m = rng.integers(0, 2 ** 52, 200_000, dtype=np.uint64)
    uni = (2 * m.astype(np.float64) + 1) * 2.0 ** -53  # the Philox u(0,1) values
    edge = np.array([0.5, 1.0, 2.0, np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 1), 1e-300, 1.7e308,
                     2.0 ** -53, 1 - 2.0 ** -53, 91.2 ** 2, 0.25])
    xs = np.concatenate([wide, near1, sub, uni, edge])
    err = np.abs(_ulp_errors(xs))
    assert err.max() <= 2.0, (err.max(), xs[np.argmax(err)])
    assert np.mean(err) < 0.6
