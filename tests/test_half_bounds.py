"""Host logic: outward rounding of BVH box bounds to IEEE half floats (ppt_half.h), checked
against numpy's float16 (round to nearest even) on special values, every float16 value and its
float32 neighbours, and random float32 values over the whole range.  A bound rounded the wrong way,
by more than one half-float step, or not exactly at a representable value fails."""
import os
import subprocess

import numpy as np
import pytest

CLANG = "/opt/rocm/llvm/bin/clang++"
HEADER_DIR = os.path.join(os.path.dirname(__file__), "..", "paper_2607_13265_amd", "csrc")
PROGRAM = r"""
#include "ppt_half.h"
#include <cstdio>
int main() {
    float x;
    while (std::fread(&x, 4, 1, stdin) == 1) {
        uint16_t r[2] = {ppt::half_down(x), ppt::half_up(x)};
        std::fwrite(r, 2, 2, stdout);
    }
    return 0;
}
"""


def _values():
    rng = np.random.default_rng(11)
    special = np.array([0.0, -0.0, 1e-9, -1e-9, 6e-8, -6e-8, 1.0, -1.0, 65504.0, -65504.0, 65519.0, 65520.0,
                        -65520.0, 7e4, -7e4, 1e30, -1e30, 3.3e38, -3.3e38, 2048.5, 3000.1, -3000.1], np.float32)
    h = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16)
    h = h[np.isfinite(h)].astype(np.float32)
    nb = np.concatenate([h, np.nextafter(h, np.float32(np.inf)), np.nextafter(h, np.float32(-np.inf))])
    mag = np.exp(rng.uniform(np.log(1e-10), np.log(3e38), 200000)).astype(np.float32)
    rnd = mag * rng.choice([-1.0, 1.0], mag.size).astype(np.float32)
    return np.concatenate([special, nb, rnd]).astype(np.float32)


def test_half_bounds_outward_and_tight(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ with _Float16 support not found")
    src, exe = tmp_path / "half.cpp", tmp_path / "half"
    src.write_text(PROGRAM)
    subprocess.run([CLANG, "-O2", "-std=c++17", "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    x = _values()
    out = subprocess.run([str(exe)], input=x.tobytes(), capture_output=True, check=True).stdout
    r = np.frombuffer(out, np.uint16).reshape(-1, 2)
    lo16, hi16 = r[:, 0].view(np.float16), r[:, 1].view(np.float16)
    lo, hi, xd = lo16.astype(np.float64), hi16.astype(np.float64), x.astype(np.float64)
    assert lo.size == x.size
    # outward: the stored interval contains the value
    assert np.all(lo <= xd) and np.all(hi >= xd)
    with np.errstate(over="ignore"):  # values beyond the half range round to infinity here
        # exact where the value is a half float (nearest rounding returns it unchanged)
        exact = np.float16(x).astype(np.float64) == xd
        # otherwise one half-float step wide: hi is the next half float above lo
        step = np.nextafter(lo16[~exact], np.float16(np.inf)).astype(np.float64)
    assert np.all(lo[exact] == xd[exact]) and np.all(hi[exact] == xd[exact])
    assert np.array_equal(step, hi[~exact])
    # beyond the half range the outer bound is infinite
    big = np.abs(xd) > 65504.0
    assert np.all(np.isinf(hi[big & (xd > 0)])) and np.all(np.isinf(lo[big & (xd < 0)]))
