// Host driver for the bin packing of the register-resident kernel: reads
// "B rpw cap maxper slots" and B system lengths from stdin, prints the
// full-capacity packing and the balanced one (capacity, then one line per
// bin with its system indices).
#include <cstdio>
#include <numeric>
#include <vector>

#include "pack.h"

static void print(const std::vector<int32_t>& bins,
                  const std::vector<int32_t>& items) {
  std::printf("%zu\n", bins.size() / 2);
  for (size_t b = 0; b < bins.size() / 2; ++b) {
    for (int j = 0; j < bins[2 * b + 1]; ++j)
      std::printf("%d ", items[bins[2 * b] + j]);
    std::printf("\n");
  }
}

int main() {
  int B, rpw, cap, maxper, slots;
  if (std::scanf("%d %d %d %d %d", &B, &rpw, &cap, &maxper, &slots) != 5)
    return 2;
  std::vector<int64_t> off(B + 1, 0);
  for (int i = 0; i < B; ++i) {
    int len;
    if (std::scanf("%d", &len) != 1) return 2;
    off[i + 1] = off[i] + len;
  }
  std::vector<int32_t> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return off[x + 1] - off[x] > off[y + 1] - off[y];
  });
  std::vector<int32_t> bins, items;
  btpack::pack_bins(order, off.data(), rpw, cap, maxper, bins, items);
  print(bins, items);
  const int c = btpack::balanced_capacity(order, off.data(), rpw, cap, maxper,
                                          slots, (int)(bins.size() / 2), bins,
                                          items);
  std::printf("%d\n", c);
  print(bins, items);
  return 0;
}
