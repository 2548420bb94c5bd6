// Comparator network that sorts N values: Batcher's odd-even merge sort (the
// iterative form for any N; comparators that would reach past N are left out).
// Pure C++ and constexpr, so device code unrolls it into a fixed sequence of
// compare-exchanges on compile-time indices, and host tests can check it
// against every 0/1 input.  For N = 8: 19 comparators in 6 layers, against 28
// in 13 for an insertion sort.
#pragma once

namespace mp {

template <int N>
struct SortNet {
  static constexpr int kMax = 256;
  int lo[kMax] = {};
  int hi[kMax] = {};
  int count = 0;
  constexpr SortNet() {
    for (int p = 1; p < N; p <<= 1)
      for (int k = p; k >= 1; k >>= 1)
        for (int j = k % p; j + k < N; j += 2 * k)
          for (int i = 0; i < k && i + j + k < N; ++i)
            if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
              lo[count] = i + j;
              hi[count] = i + j + k;
              ++count;
            }
  }
};

}  // namespace mp
