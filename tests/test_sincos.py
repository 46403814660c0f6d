"""The dynamics kernels' single-precision sine and cosine (csrc/sincos.h),
compiled for the host and checked against FP64 sin / cos: within 3 units
in the last place of the float result (plus the reduction's absolute error,
which grows with |x|) over the range the Cody-Waite reduction serves, exact
quadrant signs at multiples of pi/2, large arguments, and NaN for Inf /
NaN."""
import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "sincos.h"
int main() {
  float x;
  while (std::scanf("%a", &x) == 1) {
    float s, c;
    pds::sincos_fast(x, &s, &c);
    std::printf("%a %a\n", (double)s, (double)c);
  }
  return 0;
}
"""


def _run(xs):
    d = "/tmp/pds_sincos_%d" % os.getpid()
    os.makedirs(d, exist_ok=True)
    src, exe = os.path.join(d, "t.cpp"), os.path.join(d, "t")
    with open(src, "w") as fh:
        fh.write(DRIVER)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2109_08815_amd", "csrc"),
                           "-o", exe, src])
    inp = "\n".join(float(x).hex() for x in np.asarray(xs, np.float32)) + "\n"
    out = subprocess.run([exe], input=inp.encode(), stdout=subprocess.PIPE, check=True).stdout.decode().split()
    v = np.array([float.fromhex(t) for t in out]).reshape(-1, 2)
    return v[:, 0], v[:, 1]


def test_sincos_accuracy():
    rng = np.random.default_rng(11)
    xs = np.concatenate([
        np.linspace(-7.0, 7.0, 20001),
        rng.uniform(-100.0, 100.0, 20000),
        rng.uniform(-8192.0, 8192.0, 20000),
        [0.0, -0.0, 1e-30, -1e-20, 8192.0, -8192.0],
    ]).astype(np.float32)
    s, c = _run(xs)
    x64 = xs.astype(np.float64)
    ulp = np.float64(np.finfo(np.float32).eps)
    # reduction error: |k| * |pi/2 - (A + B + C)| plus the rounding of r
    red = np.abs(x64) * 1e-15 + 2.0 ** -26
    for got, ref in ((s, np.sin(x64)), (c, np.cos(x64))):
        err = np.abs(got - ref)
        assert np.all(err <= 3.0 * ulp * np.maximum(np.abs(ref), 2.0 ** -24) + red), float(np.max(err))
    assert s[np.where(xs == 0.0)[0][0]] == 0.0 and c[np.where(xs == 0.0)[0][0]] == 1.0


def test_sincos_quadrants_and_fallback():
    k = np.arange(-40, 41)
    xs = (k * np.pi / 2).astype(np.float32)
    s, c = _run(xs)
    q = np.mod(k, 4)
    assert np.all(np.sign(np.round(s)) == np.array([0, 1, 0, -1])[q])
    assert np.all(np.sign(np.round(c)) == np.array([1, 0, -1, 0])[q])
    big = np.array([9000.0, -1e5, 1e6, -4e6], np.float32)
    sb, cb = _run(big)
    assert np.allclose(sb, np.sin(big.astype(np.float64)), atol=5e-7)
    assert np.allclose(cb, np.cos(big.astype(np.float64)), atol=5e-7)
    sn, cn = _run(np.array([np.inf, np.nan], np.float32))
    assert np.all(np.isnan(sn)) and np.all(np.isnan(cn))
