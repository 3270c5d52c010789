"""The dedispersion kernels' workgroup -> (DM block, time tile) mapping
(XCD-aware, partial last DM block scheduled last) is a bijection onto the
tiles: the header is compiled for the host and every grid of up to 39 DM
blocks x 199 time tiles is checked, with and without a partial last block."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1307_5700_amd", "csrc")

PROG = r"""
#include <cstdio>
#include <vector>
#include "tile_map.h"
int main() {
  int bad = 0, grids = 0;
  for (int nd = 1; nd <= 39; ++nd)
    for (int nt = 1; nt <= 199; ++nt)
      for (int partial = 0; partial < 2; ++partial) {
        std::vector<int> hits(nd * nt, 0);
        for (int b = 0; b < nd * nt; ++b) {
          const mbtp::TileIdx t = mbtp::xcd_tile(b, nd, nt, partial != 0);
          if (t.dblock < 0 || t.dblock >= nd || t.ttile < 0 || t.ttile >= nt) { ++bad; continue; }
          hits[t.ttile * nd + t.dblock]++;
        }
        for (int h : hits) bad += h != 1;
        ++grids;
      }
  std::printf("%d %d\n", grids, bad);
  return bad != 0;
}
"""


def test_tile_map_is_a_bijection(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    src = tmp_path / "tile_map_check.cpp"
    src.write_text(PROG)
    exe = tmp_path / "tile_map_check"
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    grids, bad = map(int, r.stdout.split())
    assert grids == 39 * 199 * 2
    assert bad == 0 and r.returncode == 0
