"""The float rate functions of the library divide by the constants 10, 18,
20 and 80 with one multiplication by the rounded reciprocal and Markstein's
correction (two fused multiply-adds) instead of a full division. This checks,
on the CPU and for every float in the range the rate arguments can take,
that the result equals the IEEE quotient bit for bit (x = -0 may give +0:
the quotient only enters exp and exprelr, which give 1 at either zero), which
is what keeps the library's exact solver identical to the oracle."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_constant_divisions_equal_ieee_quotient_exhaustively(tmp_path):
    exe = str(tmp_path / "div_const_check")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           os.path.join(HERE, "c", "div_const_check.c"), "-o", exe, "-lm"])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, check=True).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert [float(r[0]) for r in rows] == [10.0, 18.0, 20.0, 80.0]
    for c, tested, bad in rows:
        assert int(tested) > 3_000_000_000, c
        assert int(bad) == 0, c
