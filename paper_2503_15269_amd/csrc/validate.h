// Host-side argument validation and workspace layout of the btpcg C-ABI.
// Plain C++ with no HIP dependency, so that it is also compiled on its own
// with the host sanitizers (tests/validate_driver.cpp).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "btpcg.h"

// Variants of the register-resident bin kernel (3, 6, 12 entries per lane).
#define BT_FAST_VARIANTS 3

// Entries of a packed lower triangle of an n x n block, rows one after the
// other (row i holds entries (i, 0..i)), padded to whole 16-byte chunks of
// float32 (n = 12: 78 entries, 80 stored).
constexpr int li_packed_len(int n) { return (n * (n + 1) / 2 + 3) / 4 * 4; }

namespace btv {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Parameters inside the admissible set C_g of Section III-C and the
// library's limits.
inline bool params_ok(const bt_params* p) {
  if (!p) return false;
  if (!(std::isfinite(p->a) && std::isfinite(p->b))) return false;
  // admissible set C_g: 2a + b = 1, a >= 0, b >= -1
  if (std::fabs(2.0 * p->a + p->b - 1.0) > 1e-12) return false;
  if (p->a < 0.0 || p->b < -1.0 - 1e-12) return false;
  if (p->m < 1 || p->m > BT_MAX_M) return false;
  if (p->pc != BT_PC_POLY && p->pc != BT_PC_NONE) return false;
  if (p->prec != BT_F64 && p->prec != BT_F32 && p->prec != BT_F32_IR &&
      p->prec != BT_BF16X2_IR)
    return false;
  for (int i = 1; i < p->m; ++i)
    if (!std::isfinite(p->alpha[i])) return false;
  if (p->warm_start != 0 && p->warm_start != 1) return false;
  if (p->fallback_f64 != 0 && p->fallback_f64 != 1) return false;
  if (p->prec == BT_F32_IR || p->prec == BT_BF16X2_IR) {
    if (p->max_outer < 1) return false;
    if (!(p->inner_tol > 0.0 && p->inner_tol < 1.0)) return false;
  }
  return true;
}

inline size_t elem_bytes(const bt_params* p) {
  return p->prec == BT_F64 ? sizeof(double) : sizeof(float);
}

// Largest instance (block rows) the library accepts; keeps every row and
// element index of one instance inside int32.
constexpr int64_t kMaxRowsPerInstance = (int64_t)1 << 24;

// Validate offsets (B + 1 entries, offsets[0] = 0, every instance non-empty
// and at most kMaxRowsPerInstance rows, total below 2^31 rows); returns the
// total rows R, or -1, and the largest horizon in *maxN.
inline int64_t check_offsets(int B, const int64_t* off, int* maxN) {
  if (B < 1 || !off || !maxN || off[0] != 0) return -1;
  int64_t mx = 0;
  for (int i = 0; i < B; ++i) {
    if (off[i + 1] <= off[i]) return -1;
    const int64_t Ni = off[i + 1] - off[i];
    if (Ni > kMaxRowsPerInstance) return -1;
    if (off[i + 1] > ((int64_t)1 << 31) - 1) return -1;
    mx = std::max(mx, Ni);
  }
  *maxN = (int)mx;
  return off[B];
}

struct Layout {
  size_t off, order, rowinst, ctr, fail, bins, items, F, L, Li, Lp, Fhi, Flo,
      F64, L64, Li64, total;
};

// Float64 factors for the fallback of stagnating float32 refinement.
inline bool keeps_f64(const bt_params* p) {
  return p->fallback_f64 && p->prec == BT_F32_IR;
}

// The register-resident kernel can serve the handle (block size and
// precision; whether its systems fit its bins is decided at setup).
inline bool fast_capable(int n, const bt_params* p) {
  return (n == 12 || n == 24) && p->prec == BT_F32_IR;
}

// Workspace layout of a handle: every region 256-byte aligned.
inline Layout layout(int B, int64_t R, int n, size_t es, bool split,
                     bool packed, bool f64 = false) {
  Layout l{};
  size_t at = 0;
  l.off = at; at += align_up(sizeof(int64_t) * (B + 1));
  l.order = at; at += align_up(sizeof(int32_t) * B);
  l.rowinst = at; at += align_up(sizeof(int32_t) * (size_t)R);
  l.ctr = at; at += align_up(sizeof(int32_t) * 64);
  l.fail = at; at += align_up(sizeof(int32_t) * B);
  l.bins = at; at += BT_FAST_VARIANTS * align_up(sizeof(int32_t) * 2 * B);
  l.items = at; at += BT_FAST_VARIANTS * align_up(sizeof(int32_t) * B);
  const size_t blk = align_up(es * (size_t)R * n * n);
  l.F = at; at += blk;
  l.L = at; at += blk;
  l.Li = at; at += blk;
  l.Lp = at; at += packed ? align_up(es * (size_t)R * li_packed_len(n)) : 0;
  // bfloat16 splits of F and of the transposed blocks
  const size_t hblk = split ? align_up(2 * 2 * (size_t)R * n * n) : 0;
  l.Fhi = at; at += hblk;
  l.Flo = at; at += hblk;
  const size_t dblk = f64 ? align_up(sizeof(double) * (size_t)R * n * n) : 0;
  l.F64 = at; at += dblk;
  l.L64 = at; at += dblk;
  l.Li64 = at; at += dblk;
  l.total = at;
  return l;
}

}  // namespace btv
