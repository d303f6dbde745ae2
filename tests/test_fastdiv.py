"""The invariant-divisor quotient used by the grid-transfer kernels (csrc/fastdiv.hpp), checked on the
host against plain integer division: every divisor up to 70,000 (the transfer passes divide by grid
extents) and some up to 2^32 - 1, dividends 0..4095, multiples of the divisor and their neighbours,
seeded random 32-bit values and 2^32 - 1.  Compiled with hipcc as a host program (no GPU needed).
"""
import os
import shutil
import subprocess

import pytest

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2605_21046_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <random>
#include "fastdiv.hpp"

static long check(unsigned d, std::mt19937_64& g) {
    const sg::FastDiv f = sg::make_fastdiv(d);
    long bad = 0;
    auto one = [&](unsigned long long n) {
        if (n > 0xffffffffull) return;
        if (sg::fast_quot(f, (unsigned)n) != (unsigned)n / d) ++bad;
    };
    for (unsigned n = 0; n < 4096; ++n) one(n);
    for (unsigned long long k = 1; k < 64; ++k) {
        const unsigned long long n = (unsigned long long)d * (k * 7919ull);
        one(n - 1); one(n); one(n + 1);
    }
    for (int i = 0; i < 64; ++i) one((unsigned)g());
    one(0xffffffffull);
    return bad;
}

int main() {
    std::mt19937_64 g(7);
    long bad = 0, divisors = 0;
    for (unsigned d = 1; d <= 70000; ++d, ++divisors) bad += check(d, g);
    const unsigned big[] = {65535u, 65536u, 65537u, 1u << 20, (1u << 31) - 1, 1u << 31, (1u << 31) + 1,
                            0xfffffffeu, 0xffffffffu};
    for (unsigned d : big) { bad += check(d, g); ++divisors; }
    for (int i = 0; i < 2000; ++i, ++divisors) bad += check((unsigned)(g() | 1u), g);
    std::printf("divisors %ld mismatches %ld\n", divisors, bad);
    return bad != 0;
}
"""


def test_fast_quotient_matches_integer_division(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    src = tmp_path / "fastdiv_check.cpp"
    exe = tmp_path / "fastdiv_check"
    src.write_text(PROGRAM)
    r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", CSRC, str(src),
                        "-o", str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and "mismatches 0" in run.stdout, run.stdout + run.stderr
