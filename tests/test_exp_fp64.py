"""The FP64 exponential of the global diagnostics (csrc/exp_fp64.hpp:
Cody-Waite reduction, degree-13 Taylor polynomial, ldexp), compiled for the
host from the same source the kernels use and checked against the C
library's exp, which is accurate to within one unit in the last place:
within 2 ulp on a sweep of FP32 inputs over the whole FP64 range, exact at 0,
and 0 / infinity beyond the range and at the infinities."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1707_08900_amd", "csrc", "exp_fp64.hpp")

DRIVER = r'''
#include "%s"
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
static double host_fma(double a, double b, double c) { return std::fma(a, b, c); }
static double ulps(double a, double b) {
    if (a == b) return 0.0;
    if (!std::isfinite(a) || !std::isfinite(b)) return 1e30;
    const double u = std::nextafter(std::fabs(b), INFINITY) - std::fabs(b);
    return std::fabs(a - b) / u;
}
int main() {
    double worst = 0.0, at = 0.0;
    long n = 0;
    for (int64_t i = 0; i < 4294967296LL; i += 211) {  // every 211th FP32 bit pattern
        const uint32_t bits = (uint32_t)i;
        float x;
        std::memcpy(&x, &bits, 4);
        if (!std::isfinite(x) || x < -744.0f || x > 709.5f) continue;
        const double e = ulps(fd6::exp_fp64_with((double)x, host_fma), std::exp((double)x));
        ++n;
        if (e > worst) worst = e, at = x;
    }
    std::printf("%%ld %%.3f %%.9g\n", n, worst, at);
    const double sp[] = {0.0, 1.0, -1.0, 709.7, -745.2, 800.0, -800.0, 3e38, -3e38,
                         INFINITY, -INFINITY};
    for (double x : sp) std::printf("%%.17g\n", fd6::exp_fp64_with(x, host_fma));
    return 0;
}
''' % HEADER


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    d = tmp_path_factory.mktemp("expfp64")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    r = subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    return out.stdout.split("\n")


def test_within_two_ulp(results):
    n, worst, at = results[0].split()
    print(f"{n} inputs, max {worst} ulp at {at}")
    assert int(n) > 5_000_000 and float(worst) <= 2.0


def test_special_values(results):
    vals = [float(v) for v in results[1:12]]
    assert vals[0] == 1.0
    assert abs(vals[1] - 2.718281828459045) <= 4.5e-16 and abs(vals[2] - 0.36787944117144233) <= 1e-16
    assert 0 < vals[3] < float("inf") and 0 <= vals[4] < 1e-300
    assert vals[5] == float("inf") and vals[6] == 0.0
    assert vals[7] == float("inf") and vals[8] == 0.0
    assert vals[9] == float("inf") and vals[10] == 0.0
