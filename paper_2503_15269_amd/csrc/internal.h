// Internal declarations of the btpcg library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <stdint.h>

#include <vector>

#include "btpcg.h"
#include "validate.h"

#define BT_NO_FAIL 0x7fffffff

// Host-side handle. Device pointers point into the caller's workspace.

struct bt_handle {
  int B = 0, n = 0, dtype = 0, maxN = 0;
  int64_t R = 0;
  bt_params p{};
  const void* D = nullptr;
  const void* O = nullptr;
  int64_t* off = nullptr;   // [B+1] row offsets
  int32_t* order = nullptr; // [B] instances, longest first
  int32_t* rowinst = nullptr;  // [R] instance of each block row
  int32_t* ctr = nullptr;   // [64] queue counters of the persistent kernels
  int32_t* fail = nullptr;  // [B] first failing block row, BT_NO_FAIL if none
  // bins of the register-resident kernel, per variant: [B][2] (start, count)
  // and the systems of the bins, bin after bin; nbins 0: variant n/a
  int32_t* bins[BT_FAST_VARIANTS] = {};
  int32_t* bin_items[BT_FAST_VARIANTS] = {};
  int nbins[BT_FAST_VARIANTS] = {};
  void* F = nullptr;        // [R][n][n] scaled off-diagonal blocks
  void* L = nullptr;        // [R][n][n] Cholesky factors of D_k
  void* Li = nullptr;       // [R][n][n] their inverses
  // [R][li_packed_len(n)] the inverses as packed lower triangles, for the
  // register-resident kernel (handles it can serve; else null)
  void* Lp = nullptr;
  unsigned short* Fhi = nullptr;  // BT_BF16X2_IR: [2][R][n][n], F then F^T
  unsigned short* Flo = nullptr;  // blockwise, split into bfloat16 hi + lo
  // fallback_f64: float64 F, L, L^{-1} for systems whose float32 refinement
  // stagnated (computed, for those systems only, by the fallback pass)
  void* F64 = nullptr;
  void* L64 = nullptr;
  void* Li64 = nullptr;
  int cfg = -1;             // solve-kernel configuration, -1 = automatic
  // L is current (the register-resident kernel does not read it; for the
  // other kernels it is computed on first use)
  mutable bool full_valid = false;
  // grid-wide solve: longest wait at one of its grid barriers before the
  // solve gives up (BT_ETIMEOUT), in seconds
  double grid_wait_s = 2.0;
  std::vector<int64_t> off_host;
};

// Raise the dynamic-LDS limit of kernel ``fn`` to ``bytes`` on the current
// device, once per device: ``done`` holds one bit per device ordinal, set
// after the attribute call succeeded (device ordinals past 63 make the call
// every time). Safe to call from several host threads.
inline hipError_t lds_limit(const void* fn, size_t bytes,
                            std::atomic<uint64_t>& done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = dev >= 0 && dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

// Arguments of the persistent solve kernel (passed by value).
struct SolveArgs {
  int B, n, dtype;
  int mode;          // 0 solve, 1 apply the preconditioner once
  int ir;            // float inner iteration inside float64 refinement
  int pc, m;
  double a;
  double alpha[BT_MAX_M];
  double tol, inner_tol;
  int maxit, max_outer;
  int warm;          // mode 0: x holds an initial guess on entry
  const void* Lp;    // packed L^{-1} (null: the kernel reads Li)
  const int64_t* off;
  const int32_t* order;
  const int32_t* bins;       // register-resident kernel: [nbins][2] (start, count)
  const int32_t* bin_items;  // systems of the bins, bin after bin
  int nbins;
  int32_t* ctr;
  const int32_t* fail;
  const void* F;
  const void* L;
  const void* Li;
  const void* D;     // system of record
  const void* O;
  const double* b;   // right-hand side (mode 0) or r (mode 1)
  double* x;         // solution (mode 0) or z (mode 1)
  bt_info* info;
  // float64 fallback pass: only the systems whose info reports
  // BT_ESTAGNATED are solved (from their current x); their counts add to
  // the float32 solve's
  int only_stagnated;
};

// Arguments of the setup kernel. L or F null: not computed.
struct SetupArgs {
  int B, n, dtype, prec;
  void* Lp;                // packed L^{-1} out (null: not written); with Li
                           // null the off-diagonal step reads it back
  int64_t R;
  const int64_t* off;
  const int32_t* rowinst;  // [R] instance of each block row
  const void* D;
  const void* O;
  int32_t* fail;
  void* F;
  void* L;
  void* Li;
  // non-null: only the block rows of systems whose info reports
  // BT_ESTAGNATED are needed (a workgroup without any returns at once)
  const bt_info* mask;
};

// The paper's block gemvs per block row and PCG iteration, g_a(m) of
// Section IV-B (2m + 2 at a = 0, 5m + 1 for 0 < a < 1, 3m + 3 at a = 1);
// 3 without preconditioner (the product with A alone).
__host__ __device__ inline int bt_gemv_g(int pc, double a, int m) {
  if (pc == BT_PC_NONE) return 3;
  if (a == 0.0) return 2 * m + 2;
  if (a == 1.0) return 3 * m + 3;
  return 5 * m + 1;
}

// Block-times-vector products over the N block rows of one system, from the
// counts of what a solve executed: ``halves`` halves of an application of
// the off-diagonal operator C (the F_{k-1}^T half and the F_k half, each one
// product on N - 1 rows), ``tri`` triangular transforms (one product per
// row) and ``res`` float64 residuals of the record (D, O and O^T: 3N - 2).
__host__ __device__ inline int64_t bt_gemv_rows(int N, int64_t halves,
                                                int64_t tri, int64_t res) {
  return halves * (N - 1) + tri * N + res * (3 * (int64_t)N - 2);
}

// Power of two 2^-e with 2^e <= sqrt(n2) < 2^(e+1): scales a float64
// residual of squared norm n2 to norm in [1, 2) before it is rounded to
// float32, so the inner float32 solve sees neither underflow nor overflow
// whatever the scale of b; multiplying by a power of two is exact.
__host__ __device__ inline double bt_unit_scale(double n2) {
  if (!(n2 > 0.0) || !(n2 < INFINITY)) return 1.0;
  return ldexp(1.0, -ilogb(sqrt(n2)));
}

struct KernelConfig {
  int nt, s, prec;  // prec: BT_F64 for double kernels, BT_F32 for float ones;
                    // s = 0: the register-resident bin kernel
};

int bt_num_kernel_configs();
const KernelConfig& bt_kernel_config_at(int i);
hipError_t bt_launch_solve(int cfg, const SolveArgs& a, int grid,
                           hipStream_t s);
int bt_solve_max_grid(int cfg);
hipError_t bt_launch_setup(const SetupArgs& a, hipStream_t s);
bool bt_fast_supported(int n, int prec, int variant);
bool bt_fast_params(const bt_params* p);
int bt_fast_threads(int variant);
int bt_fast_rows_per_seg(int n, int variant);  // system alignment
int bt_fast_rows_per_bin(int n);
int bt_fast_max_systems_per_bin();
hipError_t bt_launch_fast(const SolveArgs& a, int variant, int grid,
                          hipStream_t s);
int bt_fast_max_grid(int n, int variant);
// the n = 24 variant (solve_fast24.hip)
hipError_t bt_launch_fast24(const SolveArgs& a, int grid, hipStream_t s);
int bt_fast_max_grid24();
hipError_t bt_launch_setup_init(int B, int32_t* fail, int32_t* ctr,
                                hipStream_t s);
size_t bt_mrhs_scratch_bytes(int64_t R, int n, int nrhs);
hipError_t bt_mrhs_split(const float* F, unsigned short* hi, unsigned short* lo,
                         int64_t R, int n, hipStream_t s);
int bt_mrhs_run(int64_t R, int n, int nrhs, const unsigned short* Fhi,
                const unsigned short* Flo, const float* Li, const void* D,
                const void* O, int dtype, const double* b, double* x,
                double tol, int maxit, int max_outer, double inner_tol,
                int pc, double a, int m, const double* alpha, int warm,
                void* scratch, bt_info* info, hipStream_t s);
size_t bt_direct_scratch_bytes(int64_t R, int n);
bool bt_direct_supported(int n);
hipError_t bt_launch_direct(int B, int n, int dtype, const int64_t* off,
                            const int32_t* order, const void* D, const void* O,
                            const double* b, double* x, bt_info* info,
                            int64_t R, void* scratch, hipStream_t s);
hipError_t bt_launch_adjoint_outer(int B, int n, int64_t R,
                                   const int64_t* off, const int32_t* rowinst,
                                   const double* x,
                                   const double* lam, double* dD, double* dO,
                                   hipStream_t s);
