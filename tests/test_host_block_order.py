"""Host check of the whole-GPU chain's helper block order (run_kernels.hpp).

block_at(v, H, nblk, bpl, jh) maps the positions 0 .. nblk - 1 that the H
helpers take in turn (helper w: w - 1, w - 1 + H, ...) to accept blocks;
helper_of_fine(b, ...) names the helper that holds fine block b, and the
helpers' ownership wait polls exactly those helpers. The order must be a
permutation of the blocks for every helper count, and the two functions must
agree, or a block is left out or two helpers write the same rows. Both are
host-callable, so they are compiled for the host alone and checked over
every helper count of depths 2..8 for both lane-group widths.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CHECK = r"""
#include <cstdio>
#include <vector>
#include "run_kernels.hpp"
int main() {
  long checked = 0;
  for (int NG : {8, 16}) {  // lane groups of a workgroup (GS = 32 and 16)
    const int bpl = (378 + NG - 1) / NG, jh = (189 + NG - 1) / NG;
    for (int L = 2; L <= 8; ++L) {
      const int nblk = L == 2 ? 8 : 72 + (L > 3 ? (L - 3) * bpl : 0);
      for (int H = 1; H <= nblk; ++H) {
        std::vector<int> seen(nblk, 0);
        for (int v = 0; v < nblk; ++v) {
          const int b = fmmdev::block_at(v, H, nblk, bpl, jh);
          if (b < 0 || b >= nblk || seen[b]++) {
            printf("not a permutation: NG %d L %d H %d v %d b %d\n", NG, L, H, v, b);
            return 1;
          }
          if (b >= 72 && fmmdev::helper_of_fine(b, H, nblk, bpl, jh) != 1 + v % H) {
            printf("owner mismatch: NG %d L %d H %d block %d\n", NG, L, H, b);
            return 1;
          }
          ++checked;
        }
      }
    }
  }
  printf("ok %ld\n", checked);
  return 0;
}
"""


def test_block_order_is_a_permutation(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not found")
    src = tmp_path / "block_order.hip"
    src.write_text(CHECK)
    exe = tmp_path / "block_order"
    cmd = [HIPCC, "--cuda-host-only", "-O1", "-std=c++17",
           "-I", os.path.join(ROOT, "paper_2006_16622_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0 and run.stdout.startswith("ok"), run.stdout + run.stderr
