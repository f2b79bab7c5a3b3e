"""Host logic: the time differences' division by the time unit
(`div_ts` in paper_1607_06283_amd/csrc/kernels.h: a multiply by the rounded
reciprocal and one fused correction) against the IEEE division it replaces,
bit for bit, on integer time differences (small, multiples of 125, up to
2^53) over the unit values the tests and benches use, ill-conditioned units
and random ones; units outside [2^-100, 2^100] take the division itself.
The header is compiled into a small host program with hipcc (the host's
fma is the correctly rounded one)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_06283_amd", "csrc")

PROGRAM = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include "kernels.h"
static uint64_t s = 0x2545F4914F6CDD1Dull;
static uint64_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
int main(void) {
    double units[48];
    int nu = 0;
    const double fixed[] = {1000.0, 100.0, 10000.0, 1.0, 3.0, 7.0, 333.3, 1e-3, 0.1,
                            12345.678, 999.999, 1024.0, 3.0000000000000004,
                            1.9999999999999998, 65535.0, 1e6, 0x1p-100, 0x1p100};
    for (double v : fixed) units[nu++] = v;
    while (nu < 48)
        units[nu++] = ldexp(1.0 + (double)(rnd() >> 11) * 0x1p-53, (int)(rnd() % 41) - 20);
    long long n = 0, bad = 0, fast = 0;
    for (int k = 0; k < nu; ++k) {
        const rec::BuildConsts b = rec::make_build_consts(0.2, 0.2, units[k]);
        fast += b.its != 0.0;
        for (int it = 0; it < 400000; ++it) {
            const uint64_t r = rnd();
            int64_t a;
            switch (it & 3) {
                case 0: a = (int64_t)(r % 2000001) - 1000000; break;
                case 1: a = (int64_t)(r >> 24) - (int64_t)(1ull << 39); break;
                case 2: a = (int64_t)(r % 20001) * 125 - 1250000; break;
                default: a = (int64_t)(r >> 11) * ((r & 1) ? 1 : -1); break;
            }
            const double x = (double)a;
            const double got = rec::div_ts(x, b), ref = x / units[k];
            ++n;
            if (memcmp(&got, &ref, sizeof got) != 0) {
                if (bad < 5) printf("x=%lld ts=%.17g got %.17g ref %.17g\n", (long long)a,
                                    units[k], got, ref);
                ++bad;
            }
        }
    }
    printf("%lld %lld %lld\n", n, bad, fast);
    return bad != 0;
}
"""


def test_time_division_equals_ieee_division(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        hipcc = shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    src = tmp_path / "divts.cpp"
    exe = tmp_path / "divts"
    src.write_text(PROGRAM)
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-ffp-contract=off", "-I", CSRC, str(src), "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    n, bad, fast = (int(v) for v in out.stdout.split()[-3:])
    assert out.returncode == 0 and bad == 0, out.stdout
    assert n == 48 * 400000 and fast == 48  # every unit here takes the fused form
