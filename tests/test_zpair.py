"""Host logic of the z filter's paired layout: the closed-form pair list that
lets one wavefront hold a lateral mode k and its negative -k (the bilinear
form r^T z in mode space pairs R(-k) with Z(k), Parseval on the lateral
transform of Eq. (16)).  The function is compiled from the library's own
header for the host with g++ and checked on every plane size up to 40 x 40:
each mode appears once, a pair is (k, -k), a flagged mode is its own
negative, and the pair count matches the count of modes."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1009_5300_amd", "csrc", "internal.h")

HARNESS = r"""
#include <cstdio>
#include <vector>
#define __host__
#define __device__
%s
int main() {
  int bad = 0;
  for (int nx = 1; nx <= 40; ++nx)
    for (int ny = 1; ny <= 40; ++ny) {
      const int nxy = nx * ny;
      auto neg = [&](int m) { return ((ny - m / nx) %% ny) * nx + (nx - m %% nx) %% nx; };
      std::vector<int> seen(nxy, 0);
      int covered = 0, j = 0, nself = 0;
      for (;; ++j) {
        bool s0 = false, s1 = false;
        const int a = zpair_mode(j, 0, ny, nx, s0), b = zpair_mode(j, 1, ny, nx, s1);
        if (a >= nxy) break;
        if (j > nxy) { ++bad; break; }
        if (s0 != (neg(a) == a)) ++bad;
        if (!s0 && (b >= nxy || neg(a) != b || s1)) ++bad;
        if (s0 && b < nxy && (!s1 || neg(b) != b)) ++bad;
        for (int m : {a, b})
          if (m < nxy) {
            if (seen[m]++) ++bad;
            ++covered;
          }
      }
      for (int m = 0; m < nxy; ++m) nself += neg(m) == m;
      if (covered != nxy || j != (nxy - nself) / 2 + (nself + 1) / 2) ++bad;
      if (bad) { printf("fail %%d x %%d\n", nx, ny); return 1; }
    }
  printf("ok\n");
  return 0;
}
"""


def _zpair_source():
    h = open(HEADER).read()
    m = re.search(r"__host__ __device__ inline int zpair_mode\(.*?\n}\n", h, flags=re.S)
    assert m, "zpair_mode not found in internal.h"
    return m.group(0)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_zfilter_pairs_cover_every_mode_once(tmp_path):
    src = tmp_path / "zpair.cpp"
    src.write_text(HARNESS % _zpair_source())
    exe = tmp_path / "zpair"
    subprocess.run(["g++", "-O1", "-std=c++17", "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
