"""Host check of the single-launch two-pass work list (csrc/fused_order.hpp):
every (phase, transform, piece) appears exactly once, and every second-phase
item of a transform comes after all of its first-phase items -- the property
that makes every wait in the persistent kernel end (Sec. V-D, one global
synchronisation per transform).  Compiled with g++ as plain host code."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(HERE, "..", "paper_2410_05934_amd", "csrc", "fused_order.hpp")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "fused_order.hpp"
using namespace nttk;
int main() {
  long checked = 0;
  const unsigned P1[] = {1, 2, 8, 16}, P2[] = {1, 3, 16, 32};
  for (unsigned n_tr = 1; n_tr <= 70; ++n_tr)
    for (unsigned lag = 1; lag <= n_tr; ++lag)
      for (unsigned p1 : P1)
        for (unsigned p2 : P2) {
          const unsigned total = n_tr * (p1 + p2);
          std::vector<int> seen(total, 0);
          std::vector<long> last1(n_tr, -1), first2(n_tr, -1);
          for (unsigned i = 0; i < total; ++i) {
            FusedItem it = fused_item(i, n_tr, lag, p1, p2);
            if (it.t >= n_tr || it.phase > 1 || it.sub >= (it.phase ? p2 : p1)) {
              std::printf("bad item %u n_tr=%u lag=%u p1=%u p2=%u\n", i, n_tr, lag, p1, p2);
              return 1;
            }
            const unsigned key = it.t * (p1 + p2) + (it.phase ? p1 + it.sub : it.sub);
            if (seen[key]++) { std::printf("duplicate at %u\n", i); return 1; }
            if (it.phase == 0) last1[it.t] = i;
            else if (first2[it.t] < 0) first2[it.t] = i;
          }
          for (unsigned t = 0; t < n_tr; ++t)
            if (!(last1[t] >= 0 && first2[t] > last1[t])) {
              std::printf("order broken t=%u n_tr=%u lag=%u\n", t, n_tr, lag);
              return 1;
            }
          ++checked;
        }
  std::printf("ok %ld\n", checked);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_fused_work_list_is_a_dependency_respecting_permutation(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-DNTT_HD=inline",
                           f"-I{os.path.dirname(HDR)}", str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok")
