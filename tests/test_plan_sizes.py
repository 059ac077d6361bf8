"""The plan's length arithmetic (csrc/plan_sizes.hpp) on the CPU: a small
C++ program built with g++ prints the temporal FFT length and the band of
oversampled bins for a sweep of workloads, and the test checks what the
kernels rely on: the band holds every bin the interpolation's taps can
reach (|K| from 0 to the largest non-Nyquist lattice point, Section 3.1:
w_t bins around s = c|K| dt n_t/(2 pi)), it fits in the FFT without wrapping
onto itself, the bin count is even so that each sensor's row of FP32 band
values starts on a 16-byte boundary (the spread's 16-byte loads to LDS),
and the FFT length is even and 2,3,5-smooth."""
import math
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1510_01078_amd", "csrc")

# (sigma_t, Nt, w_t, kmax*c*dt) sweeps: the workloads' ranges plus short traces
CASES = []
for sig in (1.1, 1.25, 1.5, 2.0, 3.0):
    for nt in (2, 3, 16, 75, 128, 511, 1024, 1536, 2048):
        for wt in (2, 6, 8, 10, 12, 16):
            for kcd in (0.0, 0.3, 1.3, 1.95, 2.8):
                CASES.append((sig, nt, wt, kcd))


def _smooth_even(n):
    if n < 2 or n % 2:
        return False
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_temporal_band_layout(tmp_path):
    body = "\n".join(f"  emit({s!r}, {nt}, {wt}, {k!r});" for s, nt, wt, k in CASES)
    src = tmp_path / "band.cpp"
    src.write_text(
        '#include <cstdio>\n#include "plan_sizes.hpp"\n'
        "static void emit(double s, int nt, int wt, double kcd) {\n"
        "  const patsz::Band b = patsz::temporal_band(s, nt, wt, kcd, 1.0, 1.0);\n"
        '  std::printf("%d %d %d %d\\n", b.ok ? 1 : 0, b.n_t, b.b_lo, b.nb);\n'
        "}\nint main() {\n" + body + "\n  return 0;\n}\n")
    exe = tmp_path / "band"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True,
                   capture_output=True, timeout=120)
    rows = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout.split("\n")
    rows = [list(map(int, r.split())) for r in rows if r]
    assert len(rows) == len(CASES)
    n_ok = 0
    for (sig, nt, wt, kcd), (ok, n_t, b_lo, nb) in zip(CASES, rows):
        smax = kcd * n_t / (2 * math.pi)
        if not ok:
            # refused only when even the longest FFT cannot hold the band
            assert n_t >= 8192
            continue
        n_ok += 1
        assert _smooth_even(n_t) and n_t >= sigma_floor(sig, nt)
        assert nb % 2 == 0 and (nb * 8) % 16 == 0
        assert b_lo == -(wt // 2)
        # every tap of every interpolation point is inside the band
        assert b_lo + nb - 1 >= math.floor(smax) + wt // 2
        # at most one bin of rounding beyond what the taps need
        assert b_lo + nb - 1 <= math.floor(smax) + wt // 2 + 2
        # the band does not wrap onto itself in the FFT
        assert nb <= n_t and b_lo + nb - 1 < n_t
    assert n_ok > 0.9 * len(CASES)


def sigma_floor(sig, nt):
    return math.ceil(sig * nt - 1e-9)
