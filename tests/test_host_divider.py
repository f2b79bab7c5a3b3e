"""Host logic: the multiply-high divider that splits a fused launch's tile
index into its tile row and column (`make_divider` / `divide` in
paper_1607_06283_amd/csrc/kernels.h; Granlund and Montgomery 1994) against
integer division, for every divisor up to 70000 and random divisors up to
2^31 - 1, at the boundaries of each quotient and at random dividends below
2^31.  The header is compiled into a small host program with hipcc."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_06283_amd", "csrc")

PROGRAM = r"""
#include <stdint.h>
#include <stdio.h>
#include "kernels.h"
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (uint32_t)(s >> 11); }
static long long bad = 0, n_checked = 0;
static void check(uint32_t d, int64_t n) {
    if (n < 0 || n > 0x7fffffff) return;
    const rec::Divider dv = rec::make_divider(d);
    const int q = rec::divide((int)n, dv);
    ++n_checked;
    if ((int64_t)q != n / (int64_t)d) {
        if (bad < 5) printf("d=%u n=%lld got %d\n", d, (long long)n, q);
        ++bad;
    }
}
int main(void) {
    for (uint32_t d = 1; d <= 70000; ++d) {
        const int64_t lim = 0x7fffffff;
        const int64_t qm = lim / d;
        const int64_t ns[] = {0, 1, d - 1, d, d + 1, 2 * (int64_t)d - 1, qm * d - 1, qm * d,
                              lim, lim - 1};
        for (int64_t n : ns) check(d, n);
        for (int k = 0; k < 24; ++k) check(d, rnd() & 0x7fffffff);
        for (int k = 0; k < 8; ++k) check(d, (int64_t)(rnd() % 4096) * d + (rnd() % 3) - 1);
    }
    for (int k = 0; k < 200000; ++k) {
        uint32_t d = rnd() & 0x7fffffff;
        if (!d) d = 1;
        check(d, rnd() & 0x7fffffff);
        check(d, d);
        check(d, (int64_t)d - 1);
    }
    printf("%lld %lld\n", n_checked, bad);
    return bad != 0;
}
"""


def test_divider_matches_integer_division(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        hipcc = shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    src = tmp_path / "div.cpp"
    exe = tmp_path / "div"
    src.write_text(PROGRAM)
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-I", CSRC, str(src), "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    checked, bad = (int(v) for v in out.stdout.split()[-2:])
    assert out.returncode == 0 and bad == 0, out.stdout
    assert checked > 2_000_000
