"""Host: the comparator network that orders the terms of the TD arithmetic
(Batcher's odd-even merge sort, csrc/sortnet.h) sorts every input.  By the 0-1
principle a comparator network that sorts every 0/1 sequence sorts every
sequence, so the check enumerates all 2^N 0/1 inputs for each N used (and a
few more), compiled with the host compiler from the same header."""
import pathlib
import shutil
import subprocess

import pytest

HDR = pathlib.Path(__file__).resolve().parents[1] / "paper_2301_09960_amd" / "csrc" / "sortnet.h"

SRC = r'''
#include <cstdio>
#include "sortnet.h"
template <int N> int check() {
  constexpr mp::SortNet<N> net{};
  for (unsigned m = 0; m < (1u << N); ++m) {
    int v[N];
    for (int q = 0; q < N; ++q) v[q] = (m >> q) & 1;
    for (int c = 0; c < net.count; ++c) {
      const int a = net.lo[c], b = net.hi[c];
      if (v[b] > v[a]) { const int t = v[a]; v[a] = v[b]; v[b] = t; }
    }
    for (int q = 1; q < N; ++q)
      if (v[q] > v[q - 1]) return 1;
  }
  std::printf("%d %d\n", N, net.count);
  return 0;
}
int main() {
  return check<2>() | check<3>() | check<4>() | check<5>() | check<6>() | check<7>() | check<8>() |
         check<9>() | check<10>() | check<12>() | check<16>();
}
'''


def test_sorting_network_sorts_every_input(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    (tmp_path / "check.cpp").write_text(SRC)
    exe = tmp_path / "check"
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{HDR.parent}", "-o", str(exe), str(tmp_path / "check.cpp")],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    counts = dict(tuple(map(int, line.split())) for line in out.stdout.split("\n") if line)
    # fewer comparators than an insertion sort (N (N - 1) / 2) from N = 4 on
    assert all(counts[n] < n * (n - 1) // 2 for n in counts if n >= 4)
    assert counts[8] == 19
