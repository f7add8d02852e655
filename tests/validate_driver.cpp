// Host driver for the C-ABI's argument validation and workspace layout
// (csrc/validate.h), built with the address and undefined-behaviour
// sanitizers: valid and invalid parameters, offsets at and beyond the
// limits, layouts whose regions must be aligned, in order and disjoint.
#include <cmath>
#include <cstdio>
#include <limits>
#include <vector>

#include "validate.h"

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++fails;                                                \
    }                                                         \
  } while (0)

static bt_params defaults() {
  bt_params p{};
  p.a = 1.0;
  p.b = -1.0;
  p.m = 2;
  p.pc = BT_PC_POLY;
  for (int i = 0; i < BT_MAX_M; ++i) p.alpha[i] = 1.0;
  p.alpha[1] = 7.0;
  p.prec = BT_F64;
  p.max_outer = 30;
  p.inner_tol = 1e-4;
  return p;
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  bt_params p = defaults();
  CHECK(btv::params_ok(&p));
  CHECK(!btv::params_ok(nullptr));
  bt_params q = p; q.a = 0.5; q.b = 0.0; CHECK(btv::params_ok(&q));
  q = p; q.a = 0.0; q.b = 1.0; CHECK(btv::params_ok(&q));
  q = p; q.a = 0.5; q.b = 0.5; CHECK(!btv::params_ok(&q));  // 2a + b != 1
  q = p; q.a = -0.1; q.b = 1.2; CHECK(!btv::params_ok(&q));
  q = p; q.a = nan; CHECK(!btv::params_ok(&q));
  q = p; q.m = 0; CHECK(!btv::params_ok(&q));
  q = p; q.m = BT_MAX_M + 1; CHECK(!btv::params_ok(&q));
  q = p; q.pc = 7; CHECK(!btv::params_ok(&q));
  q = p; q.prec = 9; CHECK(!btv::params_ok(&q));
  q = p; q.alpha[1] = nan; CHECK(!btv::params_ok(&q));
  q = p; q.alpha[5] = nan; CHECK(btv::params_ok(&q));  // beyond m: unused
  q = p; q.warm_start = 2; CHECK(!btv::params_ok(&q));
  q = p; q.prec = BT_F32_IR; q.inner_tol = 0.0; CHECK(!btv::params_ok(&q));
  q = p; q.prec = BT_F32_IR; q.inner_tol = 1.0; CHECK(!btv::params_ok(&q));
  q = p; q.prec = BT_F32_IR; q.max_outer = 0; CHECK(!btv::params_ok(&q));

  int maxN = -1;
  const int64_t good[] = {0, 3, 10, 11};
  CHECK(btv::check_offsets(3, good, &maxN) == 11 && maxN == 7);
  const int64_t empty[] = {0, 3, 3, 5};
  CHECK(btv::check_offsets(3, empty, &maxN) == -1);
  const int64_t back[] = {0, 4, 2};
  CHECK(btv::check_offsets(2, back, &maxN) == -1);
  const int64_t start[] = {1, 4};
  CHECK(btv::check_offsets(1, start, &maxN) == -1);
  CHECK(btv::check_offsets(0, good, &maxN) == -1);
  CHECK(btv::check_offsets(1, nullptr, &maxN) == -1);
  const int64_t huge[] = {0, btv::kMaxRowsPerInstance + 1};
  CHECK(btv::check_offsets(1, huge, &maxN) == -1);
  const int64_t edge[] = {0, btv::kMaxRowsPerInstance};
  CHECK(btv::check_offsets(1, edge, &maxN) == btv::kMaxRowsPerInstance);
  std::vector<int64_t> many(257);
  for (int i = 0; i <= 256; ++i) many[i] = (int64_t)i * btv::kMaxRowsPerInstance;
  CHECK(btv::check_offsets(256, many.data(), &maxN) == -1);  // >= 2^31 rows
  const int64_t wrap[] = {0, 5, (int64_t)1 << 62, 4};
  CHECK(btv::check_offsets(3, wrap, &maxN) == -1);

  for (int n : {1, 5, 12, 24, 48, 64})
    for (int split = 0; split < 2; ++split)
      for (int packed = 0; packed < 2; ++packed) {
        const btv::Layout l = btv::layout(37, 1000, n, n % 2 ? 8 : 4, split,
                                          packed);
        const size_t r[] = {l.off, l.order, l.rowinst, l.ctr, l.fail, l.bins,
                            l.items, l.F, l.L, l.Li, l.Lp, l.Fhi, l.Flo,
                            l.total};
        for (size_t i = 0; i + 1 < sizeof r / sizeof r[0]; ++i) {
          CHECK(r[i] % btv::kAlign == 0);
          CHECK(r[i] <= r[i + 1]);
        }
        CHECK(l.F - l.items >= (size_t)BT_FAST_VARIANTS * 37 * 4);
        CHECK(l.total - l.Li >= (size_t)1000 * n * n * (n % 2 ? 8 : 4));
      }
  CHECK(li_packed_len(12) == 80 && li_packed_len(24) == 300);
  if (fails) return 1;
  std::puts("validate driver ok");
  return 0;
}
