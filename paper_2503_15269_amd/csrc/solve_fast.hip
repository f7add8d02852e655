// Register-resident PCG kernel (solve_fast.h): the public entry points and
// the n = 12 variants; the n = 24 variant is instantiated in solve_fast24.hip.
#include "solve_fast.h"


// The register-resident kernel covers block sizes 12 (3, 6 or 12 entries per
// lane) and 24 (6 entries per lane) with float32 inner iteration and float64
// refinement, the optimal weights (1,-1) and polynomial order 1..4.
bool bt_fast_supported(int n, int prec, int v) {
  if (prec != BT_F32_IR || v < 0 || v >= BT_FAST_VARIANTS) return false;
  if (n == 12) return true;
  if (n == 24) return btf::kEpt[v] == 6;
  return false;
}
bool bt_fast_params(const bt_params* p) {
  return p->pc == BT_PC_POLY && p->a == 1.0 && p->m >= 1 && p->m <= 4;
}

int bt_fast_threads(int v) { return 3072 / btf::kEpt[v]; }
int bt_fast_rows_per_seg(int n, int v) {
  if (n == 24) return btf::Geo<24, 6>::RPS;
  switch (btf::kEpt[v]) {
    case 3: return btf::Geo<12, 3>::RPS;
    case 6: return btf::Geo<12, 6>::RPS;
    default: return btf::Geo<12, 12>::RPS;
  }
}
int bt_fast_rows_per_bin(int n) { return n == 24 ? 128 : 256; }
int bt_fast_max_systems_per_bin() { return btf::MAXI; }

hipError_t bt_launch_fast(const SolveArgs& a, int v, int grid, hipStream_t s) {
  if (a.n == 24) return bt_launch_fast24(a, grid, s);
  switch (btf::kEpt[v]) {
    case 3: return btf::launch_ept<12, 3>(a, grid, s);
    case 6: return btf::launch_ept<12, 6>(a, grid, s);
    default: return btf::launch_ept<12, 12>(a, grid, s);
  }
}

int bt_fast_max_grid(int n, int v) {
  if (n == 24) return bt_fast_max_grid24();
  switch (btf::kEpt[v]) {
    case 3: return btf::max_grid<12, 3>();
    case 6: return btf::max_grid<12, 6>();
    default: return btf::max_grid<12, 12>();
  }
}
