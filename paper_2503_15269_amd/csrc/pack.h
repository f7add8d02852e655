// Packing of the systems of a batch into bins of the register-resident
// kernel (host code only, no HIP: also compiled on its own by the host tests).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace btpack {

// First-fit-decreasing packing of the systems, taken in ``order`` (longest
// first), into bins of at most ``cap`` rows and ``maxper`` systems; a system
// of len rows takes len rounded up to whole segments of ``rpw`` rows (the
// unit the kernel aligns systems to)
// (every system must fit: its padded length <= cap). Output: ``bins`` holds
// (first item, item count) per bin, ``items`` the system indices bin by bin.
// First fit = the lowest-numbered bin with room, found in a max-tree over
// the bins' free rows (a bin that holds ``maxper`` systems has none), so the
// packing is that of the plain scan in O(B log B).
inline void pack_bins(const std::vector<int32_t>& order, const int64_t* off,
                      int rpw, int cap, int maxper, std::vector<int32_t>& bins,
                      std::vector<int32_t>& items) {
  const size_t B = order.size();
  size_t P = 1;
  while (P < std::max<size_t>(B, 1)) P <<= 1;
  // leaves: free rows of bin i (bins not yet opened are empty: cap)
  std::vector<int> tree(2 * P, cap);
  std::vector<int> used, count;
  std::vector<std::vector<int32_t>> members;
  for (int32_t id : order) {
    const int len = (int)(off[id + 1] - off[id]);
    const int pad = (len + rpw - 1) / rpw * rpw;
    size_t v = 1;  // leftmost leaf with tree >= pad
    while (v < P) v = tree[2 * v] >= pad ? 2 * v : 2 * v + 1;
    const size_t b = v - P;
    if (b == used.size()) {
      used.push_back(0);
      count.push_back(0);
      members.emplace_back();
    }
    used[b] += pad;
    count[b] += 1;
    members[b].push_back(id);
    tree[v] = count[b] < maxper ? cap - used[b] : -1;
    for (v >>= 1; v >= 1; v >>= 1) tree[v] = std::max(tree[2 * v], tree[2 * v + 1]);
  }
  bins.clear();
  items.clear();
  for (size_t b = 0; b < members.size(); ++b) {
    bins.push_back((int32_t)items.size());
    bins.push_back((int32_t)members[b].size());
    items.insert(items.end(), members[b].begin(), members[b].end());
  }
}

// Bin capacity for ``slots`` workgroups resident at once, given the
// full-capacity packing (``nbins`` bins, passed in ``bins``/``items``). Bins
// of the full capacity can leave compute units idle: a batch of few rows
// fills only a few bins, and the last round of a longer queue is partial.
// The smallest capacity (whole segments, at least the longest system) that
// packs the systems into no more bins than those rounds of ``slots`` hold
// spreads the same rows over more workgroups with less work each; its
// packing replaces ``bins``/``items``. Returns the capacity taken.
inline int balanced_capacity(const std::vector<int32_t>& order,
                             const int64_t* off, int rpw, int full, int maxper,
                             int slots, int nbins, std::vector<int32_t>& bins,
                             std::vector<int32_t>& items) {
  if (slots < 1 || nbins < 1) return full;
  int64_t total = 0;
  int longest = 0;
  for (int32_t id : order) {
    const int len = (int)(off[id + 1] - off[id]);
    const int pad = (len + rpw - 1) / rpw * rpw;
    total += pad;
    longest = std::max(longest, pad);
  }
  const int64_t target = (int64_t)((nbins + slots - 1) / slots) * slots;
  const int64_t even = (total + target - 1) / target;
  int cap = (int)std::max<int64_t>(longest, (even + rpw - 1) / rpw * rpw);
  std::vector<int32_t> b2, i2;
  for (; cap < full; cap += rpw) {
    pack_bins(order, off, rpw, cap, maxper, b2, i2);
    if ((int64_t)(b2.size() / 2) <= target) {
      bins.swap(b2);
      items.swap(i2);
      return cap;
    }
  }
  return full;
}

}  // namespace btpack
