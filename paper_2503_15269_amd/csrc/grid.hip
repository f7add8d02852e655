// Grid-wide PCG for one large system.
//
// The register-resident and persistent kernels give each system one
// workgroup, which leaves a single long horizon (hundreds of block rows) on
// one CU with the whole iteration latency-bound there. Here every step of
// the iteration is a kernel over all block rows instead, and the kernel
// boundaries are the grid-wide barriers the PCG recurrences need:
//   k_g_init   r = L^{-1} s (s = b, or the float64 residual under
//              refinement), z = M^{-1} r, rho and ||s||^2 partials
//   k_g_q      p = z + beta p, q = Ahat p = p - C p, sigma partials
//   k_g_u      x += alpha p, r -= alpha q, ||L r||^2 partials,
//              z = M^{-1} r, rho partials
//   k_g_x      x = L^{-T} xhat (or x += L^{-T} d under refinement)
//   k_g_res    float64 residual b - A x of the record, ||.||^2 partials
// Same scaled coordinates as the other solve kernels: Ahat = I - C,
// (C v)_k = -(F_{k-1}^T v_{k-1} + F_k v_{k+1}), and the preconditioner of
// eq. Mminv-polynomial-coefficients evaluated as y_0 = (I + aC) r,
// y_i = ((1-a)C + aC^2) y_{i-1}, z = sum alpha_i y_i (Section IV-B).
//
// A workgroup owns rb consecutive block rows. M^{-1} needs neighbours to a
// depth D (1 + 2(m-1) at a = 1): the workgroup loads r (or forms r - alpha q)
// on its rows plus D on each side into LDS and applies C there on windows
// that shrink by one row per application, so M^{-1} r of its own rows needs
// no further grid-wide exchange. Scalars never leave the device: each
// workgroup writes one partial per reduction, and every workgroup of the
// next kernel sums all partials in the same fixed order, so all of them
// take the same decisions (alpha, beta, stopping) without a broadcast.
// Workgroup 0 records the outcome in a small control block that the host
// reads every few iterations; kernels that find it settled return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "grid.h"
#include "internal.h"
#include "reduce.h"

namespace btg {

using btk::AccOf;

constexpr int NT = 256;    // threads per workgroup
constexpr int CHUNK = 8;   // iterations enqueued between host checks
// partial-sum slots, nwg doubles each
enum { P_RHO0 = 0, P_RHO1 = 1, P_SIG = 2, P_NR2 = 3, P_NB2 = 4, P_RES = 5,
       P_RHOF = 6, P_SLOTS = 7 };

struct Ctl {
  int status;  // BT_NOT_CONVERGED while the (inner) iteration runs
  int it;      // PCG steps of this (inner) solve
  // sums of the partial slots P_NB2, P_RES, P_NR2 (k_g_sums), read by the
  // host after the last kernel of a solve or refinement step
  double nb2, res, nr2;
};

template <typename T>
struct GArgs {
  int R, n, rb, depth, nwg, pc, m, ir, dtype;
  double a, tol, itol;
  // k_g_init reads src * sscale (a power of two: the right-hand side of the
  // inner solve at norm in [1, 2)); k_g_x adds L^{-T} d * xscale = 1/sscale
  double sscale, xscale;
  double alpha[BT_MAX_M];
  const T* F;
  const T* L;
  const T* Li;
  const void* D;  // record
  const void* O;
  const double* src;  // k_g_init: b or the float64 residual
  const double* b;
  double* x;          // float64 iterate / solution
  double* r64;        // float64 residual (refinement)
  T* pb[2];
  T* rbuf[2];
  T* q;
  T* z;
  T* xh;              // scaled iterate (direct) or correction d (refinement)
  double* part;       // [P_SLOTS][nwg]
  Ctl* ctl;
};

__device__ __forceinline__ double rec(const void* P, size_t i, int dtype) {
  return dtype == BT_DT_F64 ? ((const double*)P)[i]
                            : (double)((const float*)P)[i];
}

// Sums over the workgroup of K values per thread, every thread gets them:
// a wavefront butterfly (lane 0's result is taken), then the four
// wavefronts in a fixed order. Deterministic and the same in every
// workgroup for the same inputs. ``red`` holds at least 4 K doubles.
template <int K>
__device__ __forceinline__ void wg_sums(double (&v)[K], double* red) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[4 * k + wv] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k)
    v[k] = (red[4 * k] + red[4 * k + 1]) + (red[4 * k + 2] + red[4 * k + 3]);
  __syncthreads();
}

__device__ __forceinline__ double wg_sum(double v, double* red) {
  double t[1] = {v};
  wg_sums<1>(t, red);
  return t[0];
}

// Sums of K partial slots over all workgroups (fixed order).
template <int K>
__device__ __forceinline__ void slot_sums(const double* part,
                                          const int (&slot)[K], int nwg,
                                          double* red, double (&out)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (int i = threadIdx.x; i < nwg; i += NT) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] += part[slot[k] * nwg + i];
  }
  wg_sums<K>(out, red);
}

// Settle the solve (workgroup 0 writes; the others took the same decision).
__device__ __forceinline__ void settle(Ctl* ctl, int status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->status = status;
}

// Window geometry: own rows [k0, k1), window [w0, w1) with depth d.
struct Win {
  int k0, k1, w0, w1;
};
__device__ __forceinline__ Win window(int R, int rb, int d) {
  Win w;
  w.k0 = blockIdx.x * rb;
  w.k1 = min(R, w.k0 + rb);
  w.w0 = max(0, w.k0 - d);
  w.w1 = min(R, w.k1 + d);
  return w;
}

// The blocks F_b, b in [fb0, fb0 + cnt), of a workgroup: staged in LDS when
// they fit (then C reads them from there), else read from memory.
template <typename T>
struct FBlocks {
  const T* base;  // LDS copy, or F itself
  int fb0;        // first block of the LDS copy (0 for F itself)
  __device__ __forceinline__ const T* blk(int b, size_t nn) const {
    return base + (size_t)(b - fb0) * nn;
  }
};

constexpr size_t FSTAGE_MAX = 48 * 1024;  // bytes of staged blocks at most

template <typename T>
__device__ FBlocks<T> stage_F(const GArgs<T>& a, int b0, int b1, T* lds) {
  const size_t nn = (size_t)a.n * a.n;
  b0 = max(b0, 0);
  b1 = min(b1, a.R - 1);  // F_b exists for b <= R - 2
  FBlocks<T> f{a.F, 0};
  if (lds == nullptr || b1 <= b0) return f;
  const size_t cnt = (size_t)(b1 - b0) * nn;
  const T* src = a.F + (size_t)b0 * nn;
  for (size_t e = threadIdx.x; e < cnt; e += NT) lds[e] = src[e];
  __syncthreads();
  return FBlocks<T>{lds, b0};
}

// out = C v on rows [lo, hi); v valid on the rows it needs; both in the
// window layout (row k at (k - w0) n). Same arithmetic order as the other
// solve kernels: the F_{k-1}^T term, then the F_k term, in order j.
template <typename T>
__device__ void applyC(const GArgs<T>& a, const FBlocks<T>& F, const T* v,
                       T* out, int w0, int lo, int hi) {
  const int n = a.n;
  const size_t nn = (size_t)n * n;
  const int cnt = (hi - lo) * n;
  for (int e = threadIdx.x; e < cnt; e += NT) {
    const int k = lo + e / n, i = e % n;
    T acc = T(0);
    if (k > 0) {
      const T* Fm = F.blk(k - 1, nn) + i;
      const T* vm = v + (k - 1 - w0) * n;
#pragma unroll 4
      for (int j = 0; j < n; ++j) acc += Fm[(size_t)j * n] * vm[j];
    }
    if (k < a.R - 1) {
      const T* Fk = F.blk(k, nn) + (size_t)i * n;
      const T* vp = v + (k + 1 - w0) * n;
#pragma unroll 4
      for (int j = 0; j < n; ++j) acc += Fk[j] * vp[j];
    }
    out[(k - w0) * n + i] = -acc;
  }
}

// rows on which C v is known when v is known on [lo, hi)
__device__ __forceinline__ void shrink(int R, int& lo, int& hi) {
  if (lo > 0) ++lo;
  if (hi < R) --hi;
}

// z = M^{-1} r on the own rows; r known on the whole window (LDS), y, w1,
// w2, z window buffers. Returns with z valid on [k0, k1).
template <typename T>
__device__ void precond(const GArgs<T>& a, const FBlocks<T>& F, const Win& W,
                        const T* r, T* y, T* w1, T* w2, T* z) {
  const int n = a.n, w0 = W.w0;
  const T av = (T)a.a, om = (T)(1.0 - a.a);
  int lo = W.w0, hi = W.w1;
  // y_0 = r + a C r
  if (a.a != 0.0) {
    shrink(a.R, lo, hi);
    applyC(a, F, r, w1, w0, lo, hi);
    __syncthreads();
    for (int e = threadIdx.x; e < (hi - lo) * n; e += NT) {
      const int o = (lo - w0) * n + e;
      y[o] = r[o] + av * w1[o];
      z[o] = y[o];
    }
  } else {
    for (int e = threadIdx.x; e < (hi - lo) * n; e += NT) {
      const int o = (lo - w0) * n + e;
      y[o] = r[o];
      z[o] = r[o];
    }
  }
  __syncthreads();
  for (int m = 1; m < a.m; ++m) {
    shrink(a.R, lo, hi);
    applyC(a, F, y, w1, w0, lo, hi);
    __syncthreads();
    if (a.a != 0.0) {
      shrink(a.R, lo, hi);
      applyC(a, F, w1, w2, w0, lo, hi);
      __syncthreads();
    }
    const T al = (T)a.alpha[m];
    for (int e = threadIdx.x; e < (hi - lo) * n; e += NT) {
      const int o = (lo - w0) * n + e;
      y[o] = a.a != 0.0 ? om * w1[o] + av * w2[o] : w1[o];
      z[o] += al * y[o];
    }
    __syncthreads();
  }
}

// (M v)_k[i] for the lower-triangular block M_k (row i, columns 0..i)
template <typename T>
__device__ __forceinline__ T lower(const T* M, const T* v, int n, int k,
                                   int i) {
  const T* row = M + ((size_t)k * n + i) * n;
  T acc = T(0);
  for (int j = 0; j <= i; ++j) acc += row[j] * v[j];
  return acc;
}

// (M^T v)_k[i] for the lower-triangular block M_k (column i, rows i..n-1)
template <typename T>
__device__ __forceinline__ T lowerT(const T* M, const T* v, int n, int k,
                                    int i) {
  const T* blk = M + (size_t)k * n * n;
  T acc = T(0);
  for (int j = i; j < n; ++j) acc += blk[(size_t)j * n + i] * v[j];
  return acc;
}

// Partial of one reduction over the own rows into its slot.
template <typename T>
__device__ __forceinline__ void put_partial(const GArgs<T>& a, int slot,
                                            double v, double* red) {
  const double s = wg_sum(v, red);
  if (threadIdx.x == 0) a.part[slot * a.nwg + blockIdx.x] = s;
}

// The preconditioner on the own rows from r known on the window; for
// BT_PC_NONE (M = I on the original system) z = L^T L r, a row-local map.
// Returns the rho partial r'z (the accumulator of the precision).
template <typename T>
__device__ double precond_own(const GArgs<T>& a, const FBlocks<T>& F,
                              const Win& W, T* r, T* y, T* w1, T* w2, T* z) {
  const int n = a.n, w0 = W.w0;
  if (a.pc == BT_PC_NONE) {
    for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
      const int k = W.k0 + e / n, i = e % n;
      y[(k - w0) * n + i] = lower(a.L, r + (k - w0) * n, n, k, i);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
      const int k = W.k0 + e / n, i = e % n;
      z[(k - w0) * n + i] = lowerT(a.L, y + (k - w0) * n, n, k, i);
    }
    __syncthreads();
  } else {
    precond(a, F, W, r, y, w1, w2, z);
  }
  typename AccOf<T>::type acc;
  acc.zero();
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
    const int o = (W.k0 - w0) * n + e;
    acc.add_prod(r[o], z[o]);
    a.z[(size_t)W.k0 * n + e] = z[o];
  }
  return acc.value();
}

template <typename T>
__device__ __forceinline__ T* lds_vec(double* red, int slot, int len) {
  return reinterpret_cast<T*>(red + NT) + (size_t)slot * len;
}

// Entries of one window vector in LDS: rb rows and the halo on both sides
// (at least one row: k_g_q forms p on the neighbour rows).
__host__ __device__ __forceinline__ int wlen(int rb, int depth, int n) {
  return (rb + 2 * (depth > 1 ? depth : 1)) * n;
}

// Bytes of staged blocks: the window's (rb + 2 depth - 1) or, in k_g_q,
// rb + 1 blocks.
template <typename T>
__host__ __device__ __forceinline__ size_t fstage_bytes(int rb, int depth,
                                                        int n) {
  return (size_t)(rb + 2 * depth + 1) * n * n * sizeof(T);
}

// LDS for staged blocks (after the five window vectors), or null when they
// do not fit
template <typename T>
__device__ __forceinline__ T* lds_F(const GArgs<T>& a, double* red) {
  const int lmax = wlen(a.rb, a.depth, a.n);
  return fstage_bytes<T>(a.rb, a.depth, a.n) <= FSTAGE_MAX
             ? lds_vec<T>(red, 5, lmax)
             : nullptr;
}

// r = L^{-1} s on the window (s = a.src, float64, cast to T first),
// z = M^{-1} r, partials rho (both rho slots of step 0), ||s||^2.
template <typename T>
__global__ void __launch_bounds__(NT) k_g_init(GArgs<T> a) {
  extern __shared__ double red[];
  const Win W = window(a.R, a.rb, a.depth);
  const int n = a.n, len = (W.w1 - W.w0) * n;
  const int lmax = wlen(a.rb, a.depth, n);
  T* r = lds_vec<T>(red, 0, lmax);
  T* y = lds_vec<T>(red, 1, lmax);
  T* w1 = lds_vec<T>(red, 2, lmax);
  T* w2 = lds_vec<T>(red, 3, lmax);
  T* z = lds_vec<T>(red, 4, lmax);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl->status = BT_NOT_CONVERGED;
    a.ctl->it = 0;
  }
  const FBlocks<T> F = stage_F(a, W.w0, W.w1 - 1, lds_F(a, red));
  for (int e = threadIdx.x; e < len; e += NT)
    y[e] = (T)(a.src[(size_t)W.w0 * n + e] * a.sscale);
  __syncthreads();
  double nb = 0.0;
  for (int e = threadIdx.x; e < len; e += NT) {
    const int k = W.w0 + e / n, i = e % n;
    r[e] = lower(a.Li, y + (k - W.w0) * n, n, k, i);
    if (k >= W.k0 && k < W.k1) {
      const double s = a.src[(size_t)W.w0 * n + e] * a.sscale;
      nb += s * s;
      a.rbuf[0][(size_t)k * n + i] = r[e];
      a.xh[(size_t)k * n + i] = T(0);
    }
  }
  __syncthreads();
  put_partial(a, P_NB2, nb, red);
  const double rho = precond_own(a, F, W, r, y, w1, w2, z);
  const double s = wg_sum(rho, red);
  if (threadIdx.x == 0) {
    a.part[P_RHO0 * a.nwg + blockIdx.x] = s;
    a.part[P_RHOF * a.nwg + blockIdx.x] = s;
  }
}

// Step i: the stopping test on the state after step i - 1, beta,
// p = z + beta p (own rows and both neighbour rows), q = p - C p, sigma.
// Everything the step reads is requested before the decisions.
template <typename T>
__global__ void __launch_bounds__(NT) k_g_q(GArgs<T> a, int i) {
  extern __shared__ double red[];
  const int st = a.ctl->status;
  const Win W = window(a.R, a.rb, 1);
  const int n = a.n, len = (W.w1 - W.w0) * n;
  const int lmax = wlen(a.rb, a.depth, n);
  T* p = lds_vec<T>(red, 0, lmax);
  T* zb = lds_vec<T>(red, 1, lmax);
  T* cp = lds_vec<T>(red, 2, lmax);
  const T* pin = a.pb[(i + 1) & 1];
  T* pout = a.pb[i & 1];
  for (int e = threadIdx.x; e < len; e += NT) {
    const size_t g = (size_t)W.w0 * n + e;
    zb[e] = a.z[g];
    p[e] = i == 0 ? T(0) : pin[g];
  }
  const FBlocks<T> F = stage_F(a, W.k0 - 1, W.k1, lds_F(a, red));
  double S[5];
  slot_sums<5>(a.part, {i & 1, (i + 1) & 1, P_NB2, P_NR2, P_RHOF}, a.nwg,
               red, S);
  if (st != BT_NOT_CONVERGED) return;
  const double rho = S[0], rprev = S[1], nb2 = S[2], nr2 = S[3], rho0 = S[4];
  if (!a.ir) {
    if (i == 0) {
      if (!(nb2 < INFINITY)) { settle(a.ctl, BT_ENONFINITE); return; }
      if (nb2 == 0.0) { settle(a.ctl, BT_OK); return; }
    } else {
      if (nr2 <= a.tol * a.tol * nb2) { settle(a.ctl, BT_OK); return; }
      if (!(nr2 < INFINITY)) { settle(a.ctl, BT_ENONFINITE); return; }
    }
    if (!(rho > 0.0)) {
      settle(a.ctl, rho == rho ? BT_EBREAKDOWN : BT_ENONFINITE);
      return;
    }
  } else {  // inner solve of a refinement step: stop when r'z fell enough
    if (!(rho > 0.0)) { settle(a.ctl, BT_OK); return; }
    if (i > 0 && rho <= a.itol * a.itol * rho0) {
      settle(a.ctl, BT_OK);
      return;
    }
  }
  const T be = i == 0 ? T(0) : (T)(rho / rprev);
  for (int e = threadIdx.x; e < len; e += NT)
    p[e] = i == 0 ? zb[e] : zb[e] + be * p[e];
  __syncthreads();
  applyC(a, F, p, cp, W.w0, W.k0, W.k1);
  __syncthreads();
  typename AccOf<T>::type acc;
  acc.zero();
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
    const int o = (W.k0 - W.w0) * n + e;
    const size_t g = (size_t)W.k0 * n + e;
    const T qv = p[o] - cp[o];
    pout[g] = p[o];
    a.q[g] = qv;
    acc.add_prod(p[o], qv);
  }
  put_partial(a, P_SIG, acc.value(), red);
}

// Step i: alpha = rho / sigma, x += alpha p, r -= alpha q (own rows and the
// preconditioner's halo), ||L r||^2, z = M^{-1} r, rho.
template <typename T>
__global__ void __launch_bounds__(NT) k_g_u(GArgs<T> a, int i) {
  extern __shared__ double red[];
  if (a.ctl->status != BT_NOT_CONVERGED) return;
  const Win W = window(a.R, a.rb, a.depth);
  const int n = a.n, len = (W.w1 - W.w0) * n;
  const int lmax = wlen(a.rb, a.depth, n);
  T* r = lds_vec<T>(red, 0, lmax);
  T* y = lds_vec<T>(red, 1, lmax);
  T* w1 = lds_vec<T>(red, 2, lmax);
  T* w2 = lds_vec<T>(red, 3, lmax);
  T* z = lds_vec<T>(red, 4, lmax);
  const int st = a.ctl->status;
  const T* rin = a.rbuf[i & 1];
  T* rout = a.rbuf[(i + 1) & 1];
  const T* p = a.pb[i & 1];
  for (int e = threadIdx.x; e < len; e += NT) {
    const size_t g = (size_t)W.w0 * n + e;
    r[e] = rin[g];
    y[e] = a.q[g];
  }
  const FBlocks<T> F = stage_F(a, W.w0, W.w1 - 1, lds_F(a, red));
  double S[2];
  slot_sums<2>(a.part, {P_SIG, i & 1}, a.nwg, red, S);
  if (st != BT_NOT_CONVERGED) return;
  const double sigma = S[0], rho = S[1];
  if (!(sigma > 0.0)) {
    settle(a.ctl, a.ir ? BT_OK : (sigma == sigma ? BT_EBREAKDOWN
                                                 : BT_ENONFINITE));
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->it = i + 1;
  const T al = (T)(rho / sigma);
  for (int e = threadIdx.x; e < len; e += NT) {
    const int k = W.w0 + e / n;
    const size_t g = (size_t)W.w0 * n + e;
    r[e] = r[e] - al * y[e];
    if (k >= W.k0 && k < W.k1) {
      a.xh[g] += al * p[g];
      rout[g] = r[e];
    }
  }
  __syncthreads();
  if (!a.ir) {  // ||r|| = ||L rhat|| of the original system
    double t2 = 0.0;
    typename AccOf<T>::type acc;
    acc.zero();
    for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
      const int k = W.k0 + e / n, ii = e % n;
      const T t = lower(a.L, r + (k - W.w0) * n, n, k, ii);
      acc.add_prod(t, t);
    }
    t2 = acc.value();
    put_partial(a, P_NR2, t2, red);
  }
  const double rz = precond_own(a, F, W, r, y, w1, w2, z);
  put_partial(a, (i + 1) & 1, rz, red);
}

// x = L^{-T} xhat (add = 0) or x += L^{-T} d (add = 1), own rows.
template <typename T>
__global__ void __launch_bounds__(NT) k_g_x(GArgs<T> a, int add) {
  extern __shared__ double red[];
  const Win W = window(a.R, a.rb, 0);
  const int n = a.n;
  T* v = lds_vec<T>(red, 0, wlen(a.rb, a.depth, n));
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT)
    v[e] = a.xh[(size_t)W.k0 * n + e];
  __syncthreads();
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
    const int k = W.k0 + e / n, i = e % n;
    const double u =
        (double)lowerT(a.Li, v + (k - W.k0) * n, n, k, i) * a.xscale;
    const size_t g = (size_t)W.k0 * n + e;
    a.x[g] = add ? a.x[g] + u : u;
  }
}

// r64 = b - A x in float64 from the record, own rows, and ||r64||^2.
template <typename T>
__global__ void __launch_bounds__(NT) k_g_res(GArgs<T> a) {
  extern __shared__ double red[];
  const Win W = window(a.R, a.rb, 0);
  const int n = a.n;
  const size_t nn = (size_t)n * n;
  double s2 = 0.0, b2 = 0.0;
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
    const int k = W.k0 + e / n, i = e % n;
    const double* xk = a.x + (size_t)k * n;
    double acc = 0.0;
    const size_t db = (size_t)k * nn + (size_t)i * n;
    for (int j = 0; j < n; ++j) acc += rec(a.D, db + j, a.dtype) * xk[j];
    if (k > 0) {
      const size_t ob = (size_t)(k - 1) * nn + i;
      for (int j = 0; j < n; ++j)
        acc += rec(a.O, ob + (size_t)j * n, a.dtype) * xk[j - n];
    }
    if (k < a.R - 1) {
      const size_t ob = (size_t)k * nn + (size_t)i * n;
      for (int j = 0; j < n; ++j)
        acc += rec(a.O, ob + j, a.dtype) * xk[n + j];
    }
    const size_t g = (size_t)k * n + i;
    const double rv = a.b[g] - acc;
    if (a.r64) a.r64[g] = rv;
    s2 += rv * rv;
    b2 += a.b[g] * a.b[g];
  }
  put_partial(a, P_RES, s2, red);
  put_partial(a, P_NB2, b2, red);
}

// Sums of the partial slots the host needs (fixed order, one workgroup).
template <typename T>
__global__ void __launch_bounds__(NT) k_g_sums(GArgs<T> a) {
  extern __shared__ double red[];
  double S[3];
  slot_sums<3>(a.part, {P_NB2, P_RES, P_NR2}, a.nwg, red, S);
  if (threadIdx.x == 0) {
    a.ctl->nb2 = S[0];
    a.ctl->res = S[1];
    a.ctl->nr2 = S[2];
  }
}

template <typename T>
struct Plan {
  GArgs<T> a;
  size_t lds;
  int grid;
};

inline int depth_of(const bt_params& p) {
  if (p.pc == BT_PC_NONE) return 0;
  const int d1 = p.a != 0.0 ? 1 : 0, dh = p.a != 0.0 ? 2 : 1;
  return d1 + (p.m - 1) * dh;
}

inline int rows_per_wg(int64_t R) {
  return (int)std::max<int64_t>(4, std::min<int64_t>(16, R / 64));
}

// Scratch layout: seven T vectors (p twice, r twice, q, z, xhat), the
// float64 residual, the partial sums, the control block.
template <typename T>
struct Scratch {
  size_t r64, part, ctl, total;
  Scratch(int64_t R, int n) {
    const int nwg = (int)((R + rows_per_wg(R) - 1) / rows_per_wg(R));
    const size_t v = (size_t)R * n;
    r64 = (7 * v * sizeof(T) + 255) / 256 * 256;
    part = r64 + v * sizeof(double);
    ctl = part + (size_t)P_SLOTS * nwg * sizeof(double);
    total = ctl + sizeof(Ctl);
  }
};

template <typename T, typename K, typename... Args>
hipError_t launch(K kernel, const Plan<T>& pl, hipStream_t s, Args... args) {
  hipLaunchKernelGGL(kernel, dim3(pl.grid), dim3(NT), pl.lds, s, pl.a,
                     args...);
  return hipGetLastError();
}

template <typename T>
hipError_t set_lds(size_t lds) {
  // the size depends on the system, so the limit is set on every call that
  // needs more than the default (a few runtime calls per solve)
  if (lds <= 65536) return hipSuccess;
  const void* fns[] = {(const void*)k_g_init<T>, (const void*)k_g_q<T>,
                       (const void*)k_g_u<T>, (const void*)k_g_x<T>,
                       (const void*)k_g_res<T>, (const void*)k_g_sums<T>};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(
        f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
int run(const bt_handle* h, const double* b, double* x, double tol, int maxit,
        bt_info* info, void* ws, hipStream_t s) {
  const int64_t R = h->R;
  const int n = h->n;
  Plan<T> pl{};
  GArgs<T>& a = pl.a;
  a.R = (int)R;
  a.n = n;
  a.rb = rows_per_wg(R);
  a.nwg = (int)((R + a.rb - 1) / a.rb);
  a.depth = depth_of(h->p);
  a.pc = h->p.pc;
  a.m = h->p.m;
  a.a = h->p.a;
  for (int i = 0; i < BT_MAX_M; ++i) a.alpha[i] = i == 0 ? 1.0 : h->p.alpha[i];
  a.ir = 0;
  a.dtype = h->dtype;
  a.tol = tol;
  a.itol = h->p.inner_tol;
  a.sscale = a.xscale = 1.0;
  a.F = (const T*)h->F;
  a.L = (const T*)h->L;
  a.Li = (const T*)h->Li;
  a.D = h->D;
  a.O = h->O;
  a.b = b;
  a.x = x;
  const size_t v = (size_t)R * n;
  T* f = (T*)ws;
  a.pb[0] = f;
  a.pb[1] = f + v;
  a.rbuf[0] = f + 2 * v;
  a.rbuf[1] = f + 3 * v;
  a.q = f + 4 * v;
  a.z = f + 5 * v;
  a.xh = f + 6 * v;
  const Scratch<T> sl(R, n);
  a.r64 = (double*)((unsigned char*)ws + sl.r64);
  a.part = (double*)((unsigned char*)ws + sl.part);
  a.ctl = (Ctl*)((unsigned char*)ws + sl.ctl);
  pl.grid = a.nwg;
  pl.lds = NT * sizeof(double) +
           5 * (size_t)wlen(a.rb, a.depth, n) * sizeof(T);
  const size_t fb = fstage_bytes<T>(a.rb, a.depth, n);
  if (fb <= FSTAGE_MAX) pl.lds += fb;
  if (set_lds<T>(pl.lds) != hipSuccess) return BT_EHIP;

  Ctl ctl{};
  // parts: first sum the partial slots on the device (k_g_sums)
  auto sync_state = [&](bool parts) -> bool {
    if (parts && launch(k_g_sums<T>, pl, s) != hipSuccess) return false;
    if (hipMemcpyAsync(&ctl, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) !=
        hipSuccess)
      return false;
    return hipStreamSynchronize(s) == hipSuccess;
  };
  auto host_slot = [&](int slot) {
    return slot == P_NB2 ? ctl.nb2 : slot == P_RES ? ctl.res : ctl.nr2;
  };
  // inner loop: steps until the control block is settled or ``cap`` steps.
  // The first check comes after as many steps as the last inner solve on
  // this handle took (steps launched after the settling return at once),
  // later ones every CHUNK steps.
  auto iterate = [&](int cap, int* steps) -> bool {
    int i = 0;
    int chunk = std::max(CHUNK, h->grid_hint);
    for (;;) {
      const int stop = std::min(cap, i + chunk);
      chunk = CHUNK;
      for (; i < stop; ++i) {
        if (launch(k_g_q<T>, pl, s, i) != hipSuccess ||
            launch(k_g_u<T>, pl, s, i) != hipSuccess)
          return false;
      }
      if (!sync_state(false)) return false;
      if (ctl.status != BT_NOT_CONVERGED || i >= cap) break;
    }
    *steps = ctl.it;
    h->grid_hint = ctl.it;
    return true;
  };

  int status = BT_NOT_CONVERGED, total = 0, outer = 0;
  double nb2 = 0.0, nr2 = 0.0, nrt2 = 0.0;
  const bool refine = h->p.prec == BT_F32_IR || h->p.prec == BT_BF16X2_IR;
  // executed block products: halves of applications of C, triangular
  // transforms, float64 residuals (halo rows recomputed by a workgroup are
  // not counted)
  int64_t g_half = 0, g_tri = 0, g_res = 0;
  const bool none = a.pc == BT_PC_NONE;
  const int apc = none ? 0
                       : (a.a != 0.0 ? 1 : 0) + (a.m - 1) * (a.a != 0.0 ? 2 : 1);
  // one inner solve of ``steps`` steps: k_g_init (L^{-1} s, z = M^{-1} r),
  // per step q = Ahat p and z = M^{-1} r (and ||L r|| without refinement),
  // then k_g_x (L^{-T})
  auto count_inner = [&](int steps) {
    g_half += 2 * ((int64_t)apc * (steps + 1) + steps);
    g_tri += 2 + (none ? 2 * (int64_t)(steps + 1) : 0) + (a.ir ? 0 : steps);
  };
  const bool warm = h->p.warm_start != 0;
  // float32 without refinement also starts from the residual of x0 = 0,
  // which gives ||b|| before the iteration, so that its right-hand side can
  // be scaled (float64 needs no scaling and saves the pass)
  const bool from_res = warm || sizeof(T) == sizeof(float);
  if (!refine && from_res) {
    // from the initial guess x0 (held in x): plain PCG on the correction,
    // A d = r0 = b - A x0, with the test ||r|| <= tol ||b|| carried over to
    // the correction's right-hand side
    if (!warm && hipMemsetAsync(x, 0, v * sizeof(double), s) != hipSuccess)
      return BT_EHIP;
    if (launch(k_g_res<T>, pl, s) != hipSuccess || !sync_state(true))
      return BT_EHIP;
    ++g_res;
    nb2 = host_slot(P_NB2);
    const double nr02 = host_slot(P_RES);
    nr2 = nrt2 = nr02;
    outer = 1;
    if (!(nb2 < INFINITY) || !(nr02 < INFINITY)) {
      status = BT_ENONFINITE;
    } else if (nb2 == 0.0) {  // b = 0: x = 0
      if (hipMemsetAsync(x, 0, v * sizeof(double), s) != hipSuccess)
        return BT_EHIP;
      status = BT_OK;
      nr2 = nrt2 = 0.0;
    } else if (nr02 <= tol * tol * nb2) {
      status = BT_OK;
    } else {
      a.src = a.r64;
      a.tol = tol * std::sqrt(nb2 / nr02);
      a.sscale = bt_unit_scale(nr02);
      a.xscale = 1.0 / a.sscale;
      if (launch(k_g_init<T>, pl, s) != hipSuccess) return BT_EHIP;
      int steps = 0;
      if (!iterate(maxit, &steps)) return BT_EHIP;
      status = ctl.status;
      total = steps;
      count_inner(steps);
      double* r64 = a.r64;
      a.r64 = nullptr;
      if (launch(k_g_x<T>, pl, s, 1) != hipSuccess ||
          launch(k_g_res<T>, pl, s) != hipSuccess || !sync_state(true))
        return BT_EHIP;
      ++g_res;
      a.r64 = r64;
      nr2 = total > 0 ? host_slot(P_NR2) * a.xscale * a.xscale : nr02;
      nrt2 = host_slot(P_RES);
      if (status == BT_NOT_CONVERGED && total > 0 && nr2 <= tol * tol * nb2)
        status = BT_OK;
    }
  } else if (!refine) {
    // plain PCG in the precision of the factors
    a.src = b;
    if (launch(k_g_init<T>, pl, s) != hipSuccess) return BT_EHIP;
    int steps = 0;
    if (!iterate(maxit, &steps)) return BT_EHIP;
    status = ctl.status;
    total = steps;
    count_inner(steps);
    outer = 1;
    a.r64 = nullptr;
    if (launch(k_g_x<T>, pl, s, 0) != hipSuccess ||
        launch(k_g_res<T>, pl, s) != hipSuccess || !sync_state(true))
      return BT_EHIP;
    ++g_res;
    nb2 = host_slot(P_NB2);
    nr2 = total > 0 ? host_slot(P_NR2) : nb2;
    nrt2 = host_slot(P_RES);
    // the test after the last permitted step (the kernels run it at the
    // start of the next step, which is not launched)
    if (status == BT_NOT_CONVERGED && total > 0 && nr2 <= tol * tol * nb2)
      status = BT_OK;
  } else {
    // float inner PCG inside float64 refinement on the record
    a.ir = 1;
    if (!warm && hipMemsetAsync(x, 0, v * sizeof(double), s) != hipSuccess)
      return BT_EHIP;
    for (;;) {
      if (launch(k_g_res<T>, pl, s) != hipSuccess || !sync_state(true))
        return BT_EHIP;
      if (outer > 0 || warm) ++g_res;  // the first pass from 0 reads b only
      nr2 = host_slot(P_RES);
      if (outer == 0) nb2 = host_slot(P_NB2);
      nrt2 = nr2;
      if (warm && outer == 0 && nb2 == 0.0) {  // b = 0: x = 0
        if (hipMemsetAsync(x, 0, v * sizeof(double), s) != hipSuccess)
          return BT_EHIP;
        nr2 = nrt2 = 0.0;
        status = BT_OK;
        break;
      }
      if (nr2 <= tol * tol * nb2) { status = BT_OK; break; }
      if (!(nr2 < INFINITY)) { status = BT_ENONFINITE; break; }
      if (outer >= h->p.max_outer || total >= maxit) break;
      a.src = a.r64;
      a.sscale = bt_unit_scale(nr2);
      a.xscale = 1.0 / a.sscale;
      if (launch(k_g_init<T>, pl, s) != hipSuccess) return BT_EHIP;
      int steps = 0;
      if (!iterate(maxit - total, &steps)) return BT_EHIP;
      total += steps;
      count_inner(steps);
      if (launch(k_g_x<T>, pl, s, 1) != hipSuccess) return BT_EHIP;
      ++outer;
      if (steps == 0) {
        status = BT_EBREAKDOWN;
        if (launch(k_g_res<T>, pl, s) != hipSuccess || !sync_state(true))
          return BT_EHIP;
        ++g_res;
        nrt2 = nr2 = host_slot(P_RES);
        break;
      }
    }
  }
  bt_info hi{};
  hi.status = status;
  hi.iters = total;
  hi.outer = outer;
  hi.fail_index = -1;
  hi.relres = nb2 > 0.0 ? std::sqrt(nr2 / nb2) : 0.0;
  hi.relres_true = nb2 > 0.0 ? std::sqrt(nrt2 / nb2) : 0.0;
  hi.gemv_exec = bt_gemv_rows(a.R, g_half, g_tri, g_res);
  hi.gemv_paper = (int64_t)total * bt_gemv_g(a.pc, a.a, a.m);
  if (hipMemcpyAsync(info, &hi, sizeof(hi), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return BT_EHIP;
  return BT_OK;
}

}  // namespace btg

size_t bt_grid_scratch_bytes(const bt_handle* h) {
  if (!h || h->B != 1) return 0;
  return h->p.prec == BT_F64 ? btg::Scratch<double>(h->R, h->n).total
                             : btg::Scratch<float>(h->R, h->n).total;
}

int bt_grid_solve(const bt_handle* h, const double* b, double* x, double tol,
                  int maxit, bt_info* info, void* ws, hipStream_t s) {
  if (h->p.prec == BT_F64)
    return btg::run<double>(h, b, x, tol, maxit, info, ws, s);
  return btg::run<float>(h, b, x, tol, maxit, info, ws, s);
}

// ---------------------------------------------------------------------------
// Scratch held by the library for bt_solve_grid_noalloc (callers that cannot
// allocate device memory). One array per GPU the library runs on, kept until
// the process ends. On the host the array's name is only a stand-in, never
// a device address: host code uses the address that hipGetSymbolAddress
// returns for the current device, taken once per device and kept below.
// Every call on a GPU shares that GPU's array (calls that overlap on one GPU
// race); the grid kernels initialise everything they read before reading it
// (control block in k_g_init, partial slots before their sums, p and the
// correction at step 0), so nothing has to start at zero.
static __device__ __align__(256) unsigned char scratch[BT_GRID_NOALLOC_MAX_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_addr[64];  // per device ordinal
}  // namespace

hipError_t bt_grid_static_scratch(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}
