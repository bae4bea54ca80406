"""Host check of the contribution-record field packing (pf_record.hpp): the
view index and the two binding constraints round-trip for every value a
forward state can hold, including views 2048..4095, whose packed word has
bit 31 set.  The header is plain integer code; it is compiled here with the
host compiler and run on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_24994_amd", "csrc")

PROG = r"""
#include <cstdio>
#include "pf_record.hpp"
int main() {
  long bad = 0, n = 0;
  const int binds[] = {-2, -1, 0, 1, 7, 255, 256, 511, 1000, pf::REC_MAX_BIND};
  for (int v = 0; v < pf::REC_MAX_VIEWS; ++v)
    for (int b0 : binds)
      for (int b1 : binds) {
        const int w = pf::pack_view_bind(v, b0, b1);
        ++n;
        if (pf::rec_view(w) != v || pf::rec_bind0(w) != b0 || pf::rec_bind1(w) != b1) ++bad;
      }
  const int top = pf::pack_view_bind(4095, -2, -1);
  std::printf("%ld %ld %d %d\n", n, bad, pf::rec_view(top), top < 0 ? 1 : 0);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_view_and_bindings_round_trip(tmp_path):
    src = tmp_path / "rec.cpp"
    exe = tmp_path / "rec"
    src.write_text(PROG)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    n, bad, top_view, top_negative = map(int, out)
    assert n == 4096 * 100 and bad == 0
    # view 4095 sets bit 31 of the packed word and still decodes as 4095
    assert top_view == 4095 and top_negative == 1
