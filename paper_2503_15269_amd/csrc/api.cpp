// C-ABI of the btpcg library: argument validation, workspace layout, kernel
// selection and launches. All device memory belongs to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "grid.h"
#include "internal.h"
#include "pack.h"

namespace {

using btv::align_up;
using btv::check_offsets;
using btv::elem_bytes;
using btv::keeps_f64;
using btv::fast_capable;
using btv::Layout;
using btv::layout;
using btv::params_ok;

int kernel_prec(const bt_params* p) {
  return p->prec == BT_F64 ? BT_F64 : BT_F32;
}

// Configuration indices of the register-resident bin kernel variants (after
// the generic ones).
int fast_index() { return bt_num_kernel_configs(); }
bool is_fast(int cfg) {
  return cfg >= fast_index() && cfg < fast_index() + BT_FAST_VARIANTS;
}
int num_configs() { return bt_num_kernel_configs() + BT_FAST_VARIANTS; }
KernelConfig fast_config(int v) { return {bt_fast_threads(v), 0, BT_F32}; }

KernelConfig config_at(int i) {
  return is_fast(i) ? fast_config(i - fast_index()) : bt_kernel_config_at(i);
}

// Smallest generic configuration of the right precision whose capacity holds
// the largest system; ties go to the smaller workgroup.
int auto_config(int prec, int64_t maxP) {
  int best = -1;
  int64_t bestcap = 0;
  for (int i = 0; i < bt_num_kernel_configs(); ++i) {
    const KernelConfig& c = bt_kernel_config_at(i);
    if (c.prec != prec) continue;
    const int64_t cap = (int64_t)c.nt * c.s;
    if (cap < maxP) continue;
    if (best < 0 || cap < bestcap ||
        (cap == bestcap && c.nt < bt_kernel_config_at(best).nt)) {
      best = i;
      bestcap = cap;
    }
  }
  return best;
}

int generic_config(const bt_handle* h) {
  return auto_config(kernel_prec(&h->p), (int64_t)h->maxN * h->n);
}

int config_for(const bt_handle* h) {
  if (h->cfg >= 0) return h->cfg;
  for (int v = 0; v < BT_FAST_VARIANTS; ++v)  // 3 entries per lane first
    if (h->nbins[v] > 0) return fast_index() + v;
  return generic_config(h);
}

int hip_status(hipError_t e) { return e == hipSuccess ? BT_OK : BT_EHIP; }

// full: also L (read by every kernel but the register-resident one).
int launch_setup(const bt_handle* h, hipStream_t s, bool full) {
  hipError_t e = bt_launch_setup_init(h->B, h->fail, h->ctr, s);
  if (e != hipSuccess) return BT_EHIP;
  SetupArgs a{};
  a.B = h->B;
  a.n = h->n;
  a.dtype = h->dtype;
  a.prec = h->p.prec;
  a.R = h->R;
  a.off = h->off;
  a.rowinst = h->rowinst;
  a.D = h->D;
  a.O = h->O;
  a.fail = h->fail;
  a.F = h->F;
  // the packed L^{-1} of the register-resident kernel on every setup; the
  // full L and L^{-1} of the other kernels on full setups (without a packed
  // copy to read back, the off-diagonal step needs the full one)
  a.Lp = h->Lp;
  a.L = full ? h->L : nullptr;
  a.Li = full || !h->Lp ? h->Li : nullptr;
  if (a.prec == BT_BF16X2_IR) a.prec = BT_F32_IR;  // float32 factors first
  h->full_valid = false;
  if (bt_launch_setup(a, s) != hipSuccess) return BT_EHIP;
  h->full_valid = full;
  if (h->Fhi)
    return hip_status(
        bt_mrhs_split((const float*)h->F, h->Fhi, h->Flo, h->R, h->n, s));
  return BT_OK;
}

SolveArgs base_args(const bt_handle* h) {
  SolveArgs a{};
  a.B = h->B;
  a.n = h->n;
  a.dtype = h->dtype;
  a.ir = h->p.prec == BT_F32_IR || h->p.prec == BT_BF16X2_IR;
  a.pc = h->p.pc;
  a.m = h->p.m;
  a.a = h->p.a;
  for (int i = 0; i < BT_MAX_M; ++i) a.alpha[i] = i == 0 ? 1.0 : h->p.alpha[i];
  a.inner_tol = h->p.inner_tol;
  a.max_outer = h->p.max_outer;
  a.warm = h->p.warm_start;
  a.off = h->off;
  a.order = h->order;
  a.ctr = h->ctr;
  a.fail = h->fail;
  a.F = h->F;
  a.L = h->L;
  a.Li = h->Li;
  a.D = h->D;
  a.O = h->O;
  return a;
}

int run(const bt_handle* h, SolveArgs& a, hipStream_t s) {
  int cfg = config_for(h);
  if (is_fast(cfg) && (a.mode != 0 || !a.ir)) cfg = generic_config(h);
  if (cfg < 0) return BT_EINVAL;
  if (!is_fast(cfg) && !h->full_valid) {  // first use of L
    const int rc = launch_setup(h, s, true);
    if (rc != BT_OK) return rc;
  }
  a.Lp = h->Lp;
  if (is_fast(cfg)) {
    const int v = cfg - fast_index();
    a.bins = h->bins[v];
    a.bin_items = h->bin_items[v];
    a.nbins = h->nbins[v];
    const int grid =
        std::max(1, std::min(h->nbins[v], bt_fast_max_grid(h->n, v)));
    return hip_status(bt_launch_fast(a, v, grid, s));
  }
  const int grid = std::max(1, std::min(h->B, bt_solve_max_grid(cfg)));
  return hip_status(bt_launch_solve(cfg, a, grid, s));
}

// After a float32 + refinement solve (fallback_f64): the systems whose
// refinement stagnated (info BT_ESTAGNATED) get float64 factors and blocks
// (setup kernels masked by info: workgroups without such a system return at
// once) and a float64 PCG from their current iterate (the generic kernel,
// every other system skipped). Enqueued unconditionally, so the call stays
// free of host waits; with nothing stagnated both passes only read info.
int fallback_f64(const bt_handle* h, const double* b, double* x, double tol,
                 int maxit, bt_info* info, hipStream_t s) {
  if (bt_launch_setup_init(h->B, h->fail, h->ctr, s) != hipSuccess)
    return BT_EHIP;
  SetupArgs g{};
  g.B = h->B;
  g.n = h->n;
  g.dtype = h->dtype;
  g.prec = BT_F64;
  g.R = h->R;
  g.off = h->off;
  g.rowinst = h->rowinst;
  g.D = h->D;
  g.O = h->O;
  g.fail = h->fail;
  g.F = h->F64;
  g.L = h->L64;
  g.Li = h->Li64;
  g.Lp = nullptr;
  g.mask = info;
  if (bt_launch_setup(g, s) != hipSuccess) return BT_EHIP;
  SolveArgs a = base_args(h);
  a.ir = 0;
  a.mode = 0;
  a.warm = 1;
  a.F = h->F64;
  a.L = h->L64;
  a.Li = h->Li64;
  a.Lp = nullptr;
  a.b = b;
  a.x = x;
  a.info = info;
  a.tol = tol;
  a.maxit = maxit;
  a.only_stagnated = 1;
  const int cfg = auto_config(BT_F64, (int64_t)h->maxN * h->n);
  if (cfg < 0) return BT_EINVAL;
  const int grid = std::max(1, std::min(h->B, bt_solve_max_grid(cfg)));
  return hip_status(bt_launch_solve(cfg, a, grid, s));
}

}  // namespace

extern "C" {

void bt_default_params(bt_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->a = 1.0;
  p->b = -1.0;
  p->m = 2;
  p->pc = BT_PC_POLY;
  for (int i = 0; i < BT_MAX_M; ++i) p->alpha[i] = 1.0;
  p->alpha[1] = 7.0;
  p->prec = BT_F64;
  p->max_outer = 30;
  p->inner_tol = 1e-4;
}

const char* bt_strerror(int code) {
  switch (code) {
    case BT_OK: return "ok";
    case BT_NOT_CONVERGED: return "iteration cap reached before the tolerance";
    case BT_EINVAL: return "invalid argument";
    case BT_ENOTSPD: return "a diagonal block is not positive definite (A is not SPD)";
    case BT_EBREAKDOWN: return "PCG breakdown: A or the preconditioner is not positive definite";
    case BT_ENONFINITE: return "non-finite value";
    case BT_EHIP: return "HIP runtime error";
    case BT_ENOSPACE: return "workspace too small";
    case BT_ETIMEOUT: return "a grid barrier gave up waiting (workgroups not all resident)";
    case BT_ESTAGNATED: return "float32 refinement stagnated (the system is too ill-conditioned for the float32 operator)";
    default: return "unknown status";
  }
}

size_t bt_workspace_bytes(int B, const int64_t* offsets_host, int n,
                          const bt_params* p) {
  int maxN = 0;
  if (!params_ok(p) || n < 1 || n > 64) return 0;
  const int64_t R = check_offsets(B, offsets_host, &maxN);
  if (R < 0) return 0;
  return layout(B, R, n, elem_bytes(p), p->prec == BT_BF16X2_IR,
                fast_capable(n, p), keeps_f64(p))
      .total;
}

int bt_batch_setup(bt_handle** h, int B, const int64_t* offsets_host, int n,
                   int dtype, const void* D, const void* O, const bt_params* p,
                   void* workspace, size_t ws_bytes, void* stream) {
  if (!h) return BT_EINVAL;
  *h = nullptr;
  if (!params_ok(p) || n < 1 || n > 64 || !D || !workspace) return BT_EINVAL;
  if (dtype != BT_DT_F64 && dtype != BT_DT_F32) return BT_EINVAL;
  int maxN = 0;
  const int64_t R = check_offsets(B, offsets_host, &maxN);
  if (R < 0) return BT_EINVAL;
  if (R > B && !O) return BT_EINVAL;
  // The single-workgroup solve kernels must hold the largest instance; a
  // single system may be larger (bt_solve_grid and the many-right-hand-side
  // solve span the grid instead).
  if (B > 1 && p->prec != BT_BF16X2_IR &&
      auto_config(kernel_prec(p), (int64_t)maxN * n) < 0)
    return BT_EINVAL;
  const Layout l = layout(B, R, n, elem_bytes(p), p->prec == BT_BF16X2_IR,
                          fast_capable(n, p), keeps_f64(p));
  if (ws_bytes < l.total) return BT_ENOSPACE;
  // the float64 fallback runs the generic kernel on the largest system
  if (keeps_f64(p) && auto_config(BT_F64, (int64_t)maxN * n) < 0)
    return BT_EINVAL;

  bt_handle* hh = new (std::nothrow) bt_handle();
  if (!hh) return BT_EHIP;
  hh->B = B;
  hh->n = n;
  hh->dtype = dtype;
  hh->maxN = maxN;
  hh->R = R;
  hh->p = *p;
  hh->D = D;
  hh->O = O;
  unsigned char* w = (unsigned char*)workspace;
  hh->off = (int64_t*)(w + l.off);
  hh->order = (int32_t*)(w + l.order);
  hh->rowinst = (int32_t*)(w + l.rowinst);
  hh->ctr = (int32_t*)(w + l.ctr);
  hh->fail = (int32_t*)(w + l.fail);
  for (int v = 0; v < BT_FAST_VARIANTS; ++v) {
    hh->bins[v] = (int32_t*)(w + l.bins + v * align_up(sizeof(int32_t) * 2 * B));
    hh->bin_items[v] = (int32_t*)(w + l.items + v * align_up(sizeof(int32_t) * B));
  }
  hh->F = w + l.F;
  hh->L = w + l.L;
  hh->Li = w + l.Li;
  hh->Lp = fast_capable(n, p) ? w + l.Lp : nullptr;
  if (p->prec == BT_BF16X2_IR) {
    hh->Fhi = (unsigned short*)(w + l.Fhi);
    hh->Flo = (unsigned short*)(w + l.Flo);
  }
  if (keeps_f64(p)) {
    hh->F64 = w + l.F64;
    hh->L64 = w + l.L64;
    hh->Li64 = w + l.Li64;
  }
  hh->off_host.assign(offsets_host, offsets_host + B + 1);

  // longest systems first (longest-processing-time order for the queue)
  std::vector<int32_t> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return offsets_host[x + 1] - offsets_host[x] >
           offsets_host[y + 1] - offsets_host[y];
  });
  std::vector<int32_t> bins[BT_FAST_VARIANTS], items[BT_FAST_VARIANTS];
  for (int v = 0; v < BT_FAST_VARIANTS; ++v) {
    if (bt_fast_params(p) && bt_fast_supported(n, p->prec, v) &&
        maxN <= bt_fast_rows_per_bin(n)) {
      const int rps = bt_fast_rows_per_seg(n, v);
      const int full = bt_fast_rows_per_bin(n);
      const int maxper = bt_fast_max_systems_per_bin();
      btpack::pack_bins(order, offsets_host, rps, full, maxper, bins[v],
                        items[v]);
      btpack::balanced_capacity(order, offsets_host, rps, full, maxper,
                                bt_fast_max_grid(n, v),
                                (int)(bins[v].size() / 2), bins[v], items[v]);
      hh->nbins[v] = (int)(bins[v].size() / 2);
    }
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> rowinst((size_t)R);
  for (int i = 0; i < B; ++i)
    for (int64_t g = offsets_host[i]; g < offsets_host[i + 1]; ++g)
      rowinst[(size_t)g] = i;
  bool ok =
      hipMemcpyAsync(hh->off, hh->off_host.data(), sizeof(int64_t) * (B + 1),
                     hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(hh->order, order.data(), sizeof(int32_t) * B,
                     hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(hh->rowinst, rowinst.data(), sizeof(int32_t) * R,
                     hipMemcpyHostToDevice, s) == hipSuccess;
  for (int v = 0; v < BT_FAST_VARIANTS && ok; ++v)
    if (hh->nbins[v] > 0)
      ok = hipMemcpyAsync(hh->bins[v], bins[v].data(),
                          sizeof(int32_t) * bins[v].size(),
                          hipMemcpyHostToDevice, s) == hipSuccess &&
           hipMemcpyAsync(hh->bin_items[v], items[v].data(),
                          sizeof(int32_t) * items[v].size(),
                          hipMemcpyHostToDevice, s) == hipSuccess;
  if (!ok || hipStreamSynchronize(s) != hipSuccess) {
    delete hh;
    return BT_EHIP;
  }
  const int rc = launch_setup(hh, s, !is_fast(config_for(hh)));
  if (rc != BT_OK) {
    delete hh;
    return rc;
  }
  *h = hh;
  return BT_OK;
}

int bt_refactor(bt_handle* h, void* stream) {
  if (!h) return BT_EINVAL;
  return launch_setup(h, (hipStream_t)stream, !is_fast(config_for(h)));
}

int bt_setup(bt_handle** h, int N, int n, int dtype, const void* D,
             const void* O, const bt_params* p, void* workspace,
             size_t ws_bytes, void* stream) {
  const int64_t off[2] = {0, (int64_t)N};
  if (N < 1) {
    if (h) *h = nullptr;
    return BT_EINVAL;
  }
  return bt_batch_setup(h, 1, off, n, dtype, D, O, p, workspace, ws_bytes,
                        stream);
}

int bt_precondition(const bt_handle* h, const double* r, double* z,
                    void* stream) {
  if (!h || !r || !z) return BT_EINVAL;
  SolveArgs a = base_args(h);
  a.mode = 1;
  a.warm = 0;
  a.b = r;
  a.x = z;
  a.info = nullptr;
  return run(h, a, (hipStream_t)stream);
}

// bt_solve with the start chosen by the caller (warm: x holds x0 on entry)
static int solve_from(const bt_handle* h, const double* b, double* x,
                      double tol, int maxit, bt_info* info, int warm,
                      void* stream) {
  if (!h || !b || !x || !info || !(tol >= 0.0) || maxit < 0) return BT_EINVAL;
  SolveArgs a = base_args(h);
  a.mode = 0;
  a.warm = warm;
  a.b = b;
  a.x = x;
  a.info = info;
  a.tol = tol;
  a.maxit = maxit;
  const int rc = run(h, a, (hipStream_t)stream);
  if (rc != BT_OK || !h->F64) return rc;
  return fallback_f64(h, b, x, tol, maxit, info, (hipStream_t)stream);
}

int bt_solve(const bt_handle* h, const double* b, double* x, double tol,
             int maxit, bt_info* info, void* stream) {
  return solve_from(h, b, x, tol, maxit, info, h ? h->p.warm_start : 0,
                    stream);
}

int bt_solve_batched(const bt_handle* h, const double* b, double* x,
                     double tol, int maxit, bt_info* info, void* stream) {
  return bt_solve(h, b, x, tol, maxit, info, stream);
}

int bt_solve_adjoint(const bt_handle* h, const double* x, const double* g,
                     double* lambda, double* dD, double* dO, double tol,
                     int maxit, bt_info* info, void* stream) {
  if (!h || !x || !g || !lambda) return BT_EINVAL;
  if (dO && h->R == h->B) dO = nullptr;  // no upper blocks at all
  int rc = solve_from(h, g, lambda, tol, maxit, info, 0, stream);
  if (rc != BT_OK) return rc;
  if (!dD && !dO) return BT_OK;
  return hip_status(bt_launch_adjoint_outer(h->B, h->n, h->R, h->off,
                                            h->rowinst, x,
                                            lambda, dD, dO,
                                            (hipStream_t)stream));
}

size_t bt_mrhs_workspace_bytes(const bt_handle* h, int nrhs) {
  if (!h || nrhs < 1) return 0;
  return bt_mrhs_scratch_bytes(h->R, h->n, nrhs);
}

int bt_solve_mrhs(const bt_handle* h, int nrhs, const double* b, double* x,
                  double tol, int maxit, bt_info* info, void* scratch,
                  size_t scratch_bytes, void* stream) {
  if (!h || !b || !x || !info || !scratch || !(tol >= 0.0) || maxit < 0)
    return BT_EINVAL;
  if (h->p.prec != BT_BF16X2_IR || h->B != 1 || h->p.pc != BT_PC_POLY)
    return BT_EINVAL;
  if (!(h->n == 16 || h->n == 32 || h->n == 48 || h->n == 64)) return BT_EINVAL;
  if (nrhs < 16 || nrhs > BT_MRHS_MAX || nrhs % 16 != 0) return BT_EINVAL;
  if (scratch_bytes < bt_mrhs_scratch_bytes(h->R, h->n, nrhs))
    return BT_ENOSPACE;
  return bt_mrhs_run(h->R, h->n, nrhs, h->Fhi, h->Flo, (const float*)h->Li,
                     h->D, h->O, h->dtype, b, x, tol, maxit, h->p.max_outer,
                     h->p.inner_tol, h->p.pc, h->p.a, h->p.m, h->p.alpha,
                     h->p.warm_start, scratch, info, (hipStream_t)stream);
}

size_t bt_direct_workspace_bytes(const bt_handle* h) {
  if (!h || !bt_direct_supported(h->n)) return 0;
  return bt_direct_scratch_bytes(h->R, h->n);
}

int bt_solve_direct(const bt_handle* h, const double* b, double* x,
                    bt_info* info, void* scratch, size_t scratch_bytes,
                    void* stream) {
  if (!h || !b || !x || !info || !scratch) return BT_EINVAL;
  if (!bt_direct_supported(h->n)) return BT_EINVAL;
  if (scratch_bytes < bt_direct_scratch_bytes(h->R, h->n)) return BT_ENOSPACE;
  return hip_status(bt_launch_direct(h->B, h->n, h->dtype, h->off, h->order,
                                     h->D, h->O, b, x, info, h->R, scratch,
                                     (hipStream_t)stream));
}

size_t bt_grid_workspace_bytes(const bt_handle* h) {
  return bt_grid_scratch_bytes(h);
}

int bt_solve_grid(const bt_handle* h, const double* b, double* x, double tol,
                  int maxit, bt_info* info, void* scratch,
                  size_t scratch_bytes, void* stream) {
  if (!h || !b || !x || !info || !scratch || h->B != 1 || !(tol >= 0.0) ||
      maxit < 0)
    return BT_EINVAL;
  if (scratch_bytes < bt_grid_scratch_bytes(h)) return BT_ENOSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (!h->full_valid) {  // the stopping test and BT_PC_NONE read L
    const int rc = launch_setup(h, s, true);
    if (rc != BT_OK) return rc;
  }
  return bt_grid_solve(h, b, x, tol, maxit, info, scratch, s);
}

int bt_solve_grid_noalloc(const bt_handle* h, const double* b, double* x,
                          double tol, int maxit, bt_info* info, void* stream) {
  if (!h || h->B != 1) return BT_EINVAL;
  const size_t need = bt_grid_scratch_bytes(h);
  if (need == 0) return BT_EINVAL;
  if (need > BT_GRID_NOALLOC_MAX_BYTES) return BT_ENOSPACE;
  void* ws = nullptr;
  if (bt_grid_static_scratch(&ws) != hipSuccess || !ws) return BT_EHIP;
  return bt_solve_grid(h, b, x, tol, maxit, info, ws,
                       BT_GRID_NOALLOC_MAX_BYTES, stream);
}

int bt_set_grid_wait(bt_handle* h, double seconds) {
  if (!h || !(seconds >= 0.0) || !std::isfinite(seconds)) return BT_EINVAL;
  h->grid_wait_s = seconds;
  return BT_OK;
}

int bt_kernel_config_count(void) { return num_configs(); }

int bt_kernel_config(int i, int* nt, int* s, int* prec) {
  if (i < 0 || i >= num_configs()) return BT_EINVAL;
  const KernelConfig c = config_at(i);
  if (nt) *nt = c.nt;
  if (s) *s = c.s;
  if (prec) *prec = c.prec;
  return BT_OK;
}

int bt_set_kernel_config(bt_handle* h, int i) {
  if (!h) return BT_EINVAL;
  if (i < 0) {
    h->cfg = -1;
    return BT_OK;
  }
  if (i >= num_configs()) return BT_EINVAL;
  if (is_fast(i)) {
    if (h->nbins[i - fast_index()] <= 0) return BT_EINVAL;
    h->cfg = i;
    return BT_OK;
  }
  const KernelConfig& c = bt_kernel_config_at(i);
  if (c.prec != kernel_prec(&h->p)) return BT_EINVAL;
  if ((int64_t)c.nt * c.s < (int64_t)h->maxN * h->n) return BT_EINVAL;
  h->cfg = i;
  return BT_OK;
}

int bt_get_kernel_config(const bt_handle* h) {
  if (!h) return -1;
  return config_for(h);
}

void bt_destroy(bt_handle* h) { delete h; }

}  // extern "C"
