"""Host check of the compile-time roots of unity that the mixed-radix register DFTs use as twiddle
constants: the exact integer reduction to the first octant and the Taylor series must give cos and
sin of 2 pi j / R for every j (a wrong quadrant, swap or sign would be off by O(1))."""
from __future__ import annotations

import math
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2203_02734_amd", "csrc")
RADICES = (3, 5, 6, 7, 9, 10, 12, 15, 20, 24, 25, 30, 100, 200, 1024)

SRC = r"""
#include <cstdio>
#include "wolf_device.hpp"
template <int R> void dump() {
  constexpr wolf::RootTable<R> t{};
  for (int j = 0; j < R; ++j) std::printf("%d %d %.17e %.17e\n", R, j, t.c[j], t.s[j]);
}
int main() { @CALLS@ return 0; }
"""


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    cc = hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("roots")
    src = d / "roots.hip"
    src.write_text(SRC.replace("@CALLS@", "".join(f"dump<{r}>();" for r in RADICES)))
    exe = d / "roots"
    r = subprocess.run([cc, "--offload-host-only", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    rows = {}
    for line in out.splitlines():
        rr, j, c, s = line.split()
        rows[(int(rr), int(j))] = (float(c), float(s))
    return rows


def test_every_root(table):
    assert len(table) == sum(RADICES)
    for (r, j), (c, s) in table.items():
        # the reference angle 2 pi j / r is itself rounded once (about 1e-16 relative)
        assert abs(c - math.cos(2 * math.pi * j / r)) < 4e-15, (r, j)
        assert abs(s - math.sin(2 * math.pi * j / r)) < 4e-15, (r, j)


def test_exact_symmetries(table):
    """Octant reduction is exact in integers: quarter turns and mirror angles agree bit for bit."""
    for r in RADICES:
        for j in range(r):
            c, s = table[(r, j)]
            c2, s2 = table[(r, (r - j) % r)]
            assert c == c2 and s == -s2, (r, j)  # conjugate pair
            if r % 4 == 0:
                c3, s3 = table[(r, (j + r // 4) % r)]
                assert c3 == -s and s3 == c, (r, j)  # quarter turn
    assert table[(4 * 256, 0)] == (1.0, 0.0)
    assert table[(12, 3)] == (0.0, 1.0) or abs(table[(12, 3)][0]) < 1e-300
