"""Host check of the layout helpers shared by the kernels and the workspace plan
(csrc/cc3_internal.hpp): the padded row pitch of the triple-loop cubes and the
blocked K order of the split-BF16 mixed-all operands.  Compiled for the host with
hipcc and run on the CPU; no device is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "cc3_internal.hpp"
int main() {
  using namespace cc3;
  for (int nv = 1; nv <= 300; ++nv) {
    // rows padded to the next multiple of 8 values, and no further
    const int rp = cube_pitch(nv);
    if (rp < nv || rp % 8 != 0 || rp - nv >= 8) { printf("pitch %d\n", nv); return 1; }
    if (cube_slot(nv) != (int64_t)nv * nv * rp) { printf("slot %d\n", nv); return 1; }
    // the blocked K covers every pair (x, y) < nv once, in whole 8 x 8 blocks of 64
    const int64_t K = lp_kb_len(nv);
    if (K < (int64_t)nv * nv || K % 64 != 0) { printf("len %d\n", nv); return 1; }
    // the row pitch is never a power of two (rows that far apart share channels)
    const int64_t P = lp_kb_pitch(nv);
    if (P < K || (P & (P - 1)) == 0 || P % 8 != 0) { printf("pitch K %d\n", nv); return 1; }
    std::vector<char> seen(K, 0);
    for (int x = 0; x < nv; ++x)
      for (int y = 0; y < nv; ++y) {
        const int64_t k = lp_kb(x, y, nv);
        if (k < 0 || k >= K || seen[k]) { printf("kb %d %d %d\n", nv, x, y); return 1; }
        seen[k] = 1;
        if (k - lp_kb(x & ~7, y & ~7, nv) != (x & 7) * 8 + (y & 7)) {
          printf("block %d %d %d\n", nv, x, y);
          return 1;
        }
      }
  }
  printf("ok\n");
  return 0;
}
"""


def test_cube_pitch_and_blocked_k(tmp_path):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "layout.cpp"
    exe = tmp_path / "layout"
    src.write_text(PROGRAM)
    r = subprocess.run([HIPCC, "-std=c++17", "-I", os.path.join(ROOT, "paper_2007_01088_amd", "csrc"),
                        "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
