// Many right-hand sides at once: X = A^{-1} B for an [R][n][nrhs] panel of
// right-hand sides (one system, n a multiple of 16).
//
// Each right-hand side runs its own PCG (own alpha, beta, convergence), but
// the operator is applied to the whole panel, so each application of the
// scaled off-diagonal operator C (see solve.hip for the scaled form of the
// paper's preconditioner) is a pair of dense n x n by n x nrhs products per
// block row:  (C V)_k = -(F_{k-1}^T V_{k-1} + F_k V_{k+1}).
// These run on the matrix cores: v_mfma_f32_16x16x16_bf16 with the blocks
// stored split as F = Fhi + Flo (two bfloat16 arrays) and the panel split the
// same way on the fly; the product is hi*hi + hi*lo + lo*hi with float32
// accumulation (relative error ~1e-5), and the float64 refinement on the
// record removes what the inner float32 solve leaves.
//
// One inner iteration (m = 2 shown; the polynomial follows eq. Mminv-poly-
// nomial-coefficients at a = 1: y_0 = r + C r, y_i = C(C y_{i-1}))
//   p = z + beta p, q = p - C p,
//     sigma = p'q partials                  k_mr_app<EPI_QU>
//   alpha = rho / sigma                     k_mr_colsum<SIGMA>
//   r = r - alpha q, d += alpha p,
//     y0 = r + C r                          k_mr_app<EPI_Y0U>
//   w = C y0                                k_mr_app<EPI_W>
//   z = y0 + alpha_1 C w, rho = r'z parts   k_mr_app<EPI_Z>
//   beta, stopping test                     k_mr_colsum<RHO>
// The vector updates are fused into the products: a workgroup forms the
// updated p (or r) of its own row and of both neighbour rows from the old
// values, so p and r alternate between two panels (the neighbours' old
// values must survive until every workgroup has read them). Workgroups are
// mapped to rows so that each XCD gets a contiguous range of block rows and
// the neighbour rows' data is shared in its L2. Converged right-hand sides
// no longer update; a workgroup whose columns have all stopped returns at
// once. The host checks every few iterations whether any is left.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "internal.h"

namespace btm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WG = 256;       // 4 wavefronts, 16 right-hand sides each
constexpr int CPW = 16;       // columns per wavefront
constexpr int CPB = 64;       // columns per workgroup

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

enum { EPI_QU = 0, EPI_Y0 = 1, EPI_W = 2, EPI_Z = 3, EPI_Y0U = 4 };

struct MrArgs {
  int R, n, nrhs;
  const unsigned short* Fhi;  // [R][n][n]
  const unsigned short* Flo;
  const float* Li;            // [R][n][n]
  const void* D;              // record
  const void* O;
  int dtype;
  const double* b;            // [R][n][nrhs]
  double* x;
  float *p, *q, *r, *d, *y0, *w, *z;  // panels [R][n][nrhs]
  float *p2, *r2;             // second panels of p and r (alternating)
  double* part;               // [R][nrhs] per-row partial sums
  // per right-hand-side state
  double *rho, *rho0, *alpha, *beta, *nb2, *nr2;
  int *act, *done, *first, *inner, *total, *outer, *status;
  double alpha1;              // polynomial coefficient of the second term
  int m;
  double tol, itol2;
  int maxit;
};

// ---------------------------------------------------------------------------
// Y = C V on the matrix cores, with an epilogue. Grid (8 ceil(R / 8),
// nrhs / 64); block b works on row (b mod 8) ceil(R / 8) + b / 8, so that the
// workgroups of one XCD (dispatched round-robin) cover consecutive rows.
// For EPI_QU and EPI_Y0U the operand is an update formed on the fly:
//   QU:  V = p_new = z + beta p   (V1 = z, V2 = p old, out2 = p new)
//   Y0U: V = r_new = r - alpha q  (V1 = r old, V2 = q, out2 = r new)
// (for a column that has stopped the operand is the old value, unchanged).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_row(int b, int R) {
  const int chunk = (R + 7) / 8;
  return (b & 7) * chunk + (b >> 3);
}

template <int EPI>
__device__ __forceinline__ float operand(const MrArgs& a, const float* V1,
                                         const float* V2, size_t idx, int col,
                                         bool act) {
  if constexpr (EPI == EPI_QU) {
    return act ? __fmaf_rn((float)a.beta[col], V2[idx], V1[idx]) : V2[idx];
  } else if constexpr (EPI == EPI_Y0U) {
    return act ? __fmaf_rn(-(float)a.alpha[col], V2[idx], V1[idx]) : V1[idx];
  } else {
    return V1[idx];
  }
}

template <int NB, int EPI>
__global__ void __launch_bounds__(WG) k_mr_app(MrArgs a, const float* V,
                                              const float* V2, const float* aux,
                                              float* out, float* out2) {
  constexpr int MT = NB / 16;
  constexpr int NN = NB * NB;
  __shared__ __align__(16) unsigned short sFk[2][NN];   // hi, lo of F_k
  __shared__ __align__(16) unsigned short sFm[2][NN];   // hi, lo of F_{k-1}
  const int k = xcd_row(blockIdx.x, a.R);
  if (k >= a.R) return;
  const int t = threadIdx.x;
  const int wv = t >> 6, l = t & 63;
  const int c0 = blockIdx.y * CPB + wv * CPW;
  const int col = c0 + (l & 15);
  const int kq = 4 * (l >> 4);                 // k-offset of this lane
  const bool has_prev = k > 0, has_next = k < a.R - 1;
  // nothing to do once every column of this workgroup has stopped (the host
  // only checks every few iterations)
  if (!__syncthreads_or(a.act[blockIdx.y * CPB + (t & 63)])) return;
  {
    // 16-byte loads of the bfloat16 halves (NN is a multiple of 8)
    const uint4* fh = reinterpret_cast<const uint4*>(a.Fhi);
    const uint4* fl = reinterpret_cast<const uint4*>(a.Flo);
    constexpr int NC = NN / 8;
    for (int e = t; e < NC; e += WG) {
      if (has_next) {
        reinterpret_cast<uint4*>(sFk[0])[e] = fh[(size_t)k * NC + e];
        reinterpret_cast<uint4*>(sFk[1])[e] = fl[(size_t)k * NC + e];
      }
      if (has_prev) {
        reinterpret_cast<uint4*>(sFm[0])[e] = fh[(size_t)(k - 1) * NC + e];
        reinterpret_cast<uint4*>(sFm[1])[e] = fl[(size_t)(k - 1) * NC + e];
      }
    }
  }
  __syncthreads();
  const int ld = a.nrhs;
  const bool act = a.act[col] != 0;
  f32x4 acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < MT; ++ks) {
    const int kr = 16 * ks + kq;  // first of the 4 K rows of this lane
    if (has_next) {
      bf16x4 bh, bl;
      const size_t base = ((size_t)(k + 1) * NB + kr) * ld + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = operand<EPI>(a, V, V2, base + (size_t)i * ld, col, act);
        const unsigned short h = f2bf(v);
        bh[i] = (short)h;
        bl[i] = (short)f2bf(v - bf2f(h));
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int row = 16 * mt + (l & 15);
        bf16x4 ah, al;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ah[i] = (short)sFk[0][row * NB + kr + i];
          al[i] = (short)sFk[1][row * NB + kr + i];
        }
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[mt], 0, 0, 0);
      }
    }
    if (has_prev) {
      bf16x4 bh, bl;
      const size_t base = ((size_t)(k - 1) * NB + kr) * ld + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = operand<EPI>(a, V, V2, base + (size_t)i * ld, col, act);
        const unsigned short h = f2bf(v);
        bh[i] = (short)h;
        bl[i] = (short)f2bf(v - bf2f(h));
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int mcol = 16 * mt + (l & 15);   // row of F^T = column of F
        bf16x4 ah, al;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ah[i] = (short)sFm[0][(kr + i) * NB + mcol];
          al[i] = (short)sFm[1][(kr + i) * NB + mcol];
        }
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[mt], 0, 0, 0);
      }
    }
  }
  // epilogue: lane holds rows 16 mt + kq + i of column ``col``; C V = -acc
  double dp = 0.0;
  const float alc = (float)a.alpha[col];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * mt + kq + i;
      const size_t idx = ((size_t)k * NB + row) * ld + col;
      const float cv = -acc[mt][i];
      float o;
      if constexpr (EPI == EPI_QU) {
        const float pv = operand<EPI>(a, V, V2, idx, col, act);
        out2[idx] = pv;                  // p new
        o = pv - cv;                     // q = p - C p
        dp += (double)pv * (double)o;    // sigma = p'q
      } else if constexpr (EPI == EPI_Y0U) {
        const float rv = operand<EPI>(a, V, V2, idx, col, act);
        out2[idx] = rv;                  // r new
        if (act) a.d[idx] = __fmaf_rn(alc, aux[idx], a.d[idx]);  // d += alpha p
        o = rv + cv;                     // y0 = r + C r
      } else if constexpr (EPI == EPI_Y0) {
        o = aux[idx] + cv;               // y0 = r + C r
      } else if constexpr (EPI == EPI_W) {
        o = cv;                          // w = C y0
      } else {
        o = aux[idx] + (float)a.alpha1 * cv;  // z = y0 + alpha_1 C w
        dp += (double)a.r[idx] * (double)o;   // rho = r'z
      }
      out[idx] = o;
    }
  }
  if constexpr (EPI == EPI_QU || EPI == EPI_Z) {
    dp += __shfl_xor(dp, 16);
    dp += __shfl_xor(dp, 32);
    if (l < 16) a.part[(size_t)k * ld + col] = dp;
  }
}

// Per right-hand side: sum of the per-row partials in a fixed order, then
// the scalar step. One workgroup per right-hand side.
enum { SUM_SIGMA = 0, SUM_RHO = 1, SUM_RES = 2 };

template <int KIND>
__global__ void __launch_bounds__(256) k_mr_colsum(MrArgs a) {
  __shared__ double s[256];
  const int c = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < a.R; k += 256) v += a.part[(size_t)k * a.nrhs + c];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double tot = s[0];
  if constexpr (KIND == SUM_SIGMA) {
    if (a.act[c]) {
      if (!(tot > 0.0)) {
        a.act[c] = 0;
        a.alpha[c] = 0.0;
      } else {
        a.alpha[c] = a.rho[c] / tot;
        a.inner[c] += 1;
        a.total[c] += 1;
      }
    }
  } else if constexpr (KIND == SUM_RHO) {
    if (a.act[c]) {
      if (!(tot > 0.0)) {
        a.act[c] = 0;
      } else if (a.first[c]) {
        a.rho0[c] = tot;
      } else if (tot <= a.itol2 * a.rho0[c]) {
        a.act[c] = 0;
      }
      if (a.total[c] >= a.maxit) a.act[c] = 0;
      a.beta[c] = a.first[c] ? 0.0 : tot / a.rho[c];
      a.rho[c] = tot;
      a.first[c] = 0;
    }
  } else {  // SUM_RES: float64 residual of the record
    a.nr2[c] = tot;
    if (!a.done[c]) {
      const double t2 = a.tol * a.tol * a.nb2[c];
      if (tot <= t2) {
        a.status[c] = BT_OK;
        a.done[c] = 1;
      } else if (!(tot < INFINITY)) {
        a.status[c] = BT_ENONFINITE;
        a.done[c] = 1;
      } else if (a.total[c] >= a.maxit) {
        a.done[c] = 1;
      }
    }
    a.act[c] = a.done[c] ? 0 : 1;
    a.first[c] = 1;
    a.inner[c] = 0;
  }
}

// ||b||^2 per right-hand side into part (then summed by SUM_RES-like code).
__global__ void k_mr_bnorm(MrArgs a) {
  const int k = blockIdx.x;
  for (int c = threadIdx.x; c < a.nrhs; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < a.n; ++i) {
      const double v = a.b[((size_t)k * a.n + i) * a.nrhs + c];
      s += v * v;
    }
    a.part[(size_t)k * a.nrhs + c] = s;
  }
}

__global__ void k_mr_init_cols(MrArgs a) {
  __shared__ double s[256];
  const int c = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < a.R; k += 256) v += a.part[(size_t)k * a.nrhs + c];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nb = s[0];
    a.nb2[c] = nb;
    a.nr2[c] = nb;
    a.total[c] = 0;
    a.outer[c] = 0;
    a.status[c] = BT_NOT_CONVERGED;
    a.done[c] = 0;
    if (!(nb < INFINITY)) {
      a.status[c] = BT_ENONFINITE;
      a.done[c] = 1;
    } else if (nb == 0.0) {
      a.status[c] = BT_OK;
      a.done[c] = 1;
    }
  }
}

// Panel kernels of the refinement, one workgroup per (block row, 64
// columns): wavefront w takes the rows w, w + 4, ..., lane l the column
// 64 blockIdx.y + l; the n x n blocks sit in LDS and are read as broadcasts,
// the panels are read and written with consecutive lanes on consecutive
// columns.

// r64 = b - A x in float64 (x = 0 on the first pass: r64 = b), with
//   (A x)_k = D_k x_k + O_k x_{k+1} + O_{k-1}^T x_{k-1},
// and the squared column norms of r64 per block row into part.
template <int NB, typename Rec>
__global__ void __launch_bounds__(256) k_mr_resid(MrArgs a, double* r64,
                                                  int first) {
  constexpr int NN = NB * NB, MR = NB / 4;
  __shared__ Rec sD[NN], sO[NN], sOm[NN];
  __shared__ double red[4][64];
  const int k = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int c = blockIdx.y * CPB + lane, L = a.nrhs;
  const size_t pn = (size_t)NB * L;
  const bool hp = k > 0, hn = k < a.R - 1;
  const Rec* D = (const Rec*)a.D + (size_t)k * NN;
  const Rec* O = (const Rec*)a.O;
  for (int e = t; e < NN; e += 256) {
    sD[e] = D[e];
    sO[e] = hn ? O[(size_t)k * NN + e] : (Rec)0;
    sOm[e] = hp ? O[(size_t)(k - 1) * NN + e] : (Rec)0;
  }
  __syncthreads();
  const bool done = a.done[c] != 0;
  double acc[MR];
#pragma unroll
  for (int m = 0; m < MR; ++m) acc[m] = 0.0;
  if (!first && !done) {
    const double* xk = a.x + (size_t)k * pn + c;
    const double* xn = hn ? xk + pn : xk;
    const double* xm = hp ? xk - pn : xk;
#pragma unroll 4
    for (int j = 0; j < NB; ++j) {
      const double x0 = xk[(size_t)j * L];
      const double x1 = hn ? xn[(size_t)j * L] : 0.0;
      const double x2 = hp ? xm[(size_t)j * L] : 0.0;
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int i = w + 4 * m;
        double v = fma((double)sD[i * NB + j], x0, acc[m]);
        v = fma((double)sO[i * NB + j], x1, v);
        acc[m] = fma((double)sOm[j * NB + i], x2, v);
      }
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const size_t idx = (size_t)k * pn + (size_t)(w + 4 * m) * L + c;
    const double v = done ? 0.0 : a.b[idx] - acc[m];
    r64[idx] = v;
    ss = fma(v, v, ss);
  }
  red[w][lane] = ss;
  __syncthreads();
  if (w == 0)
    a.part[(size_t)k * L + c] = (red[0][lane] + red[1][lane]) +
                                (red[2][lane] + red[3][lane]);
}

// r = L^{-1} r64 (float), d = 0, p = 0 for the running columns.
template <int NB>
__global__ void __launch_bounds__(256) k_mr_tohat(MrArgs a, const double* r64) {
  constexpr int NN = NB * NB, MR = NB / 4;
  __shared__ float sL[NN];
  const int k = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int c = blockIdx.y * CPB + lane, L = a.nrhs;
  const size_t pn = (size_t)NB * L;
  for (int e = t; e < NN; e += 256) sL[e] = a.Li[(size_t)k * NN + e];
  __syncthreads();
  float acc[MR];
#pragma unroll
  for (int m = 0; m < MR; ++m) acc[m] = 0.f;
  if (a.act[c]) {
    const double* rk = r64 + (size_t)k * pn + c;
#pragma unroll 4
    for (int j = 0; j < NB; ++j) {
      const float rv = (float)rk[(size_t)j * L];
#pragma unroll
      for (int m = 0; m < MR; ++m)  // L^{-1} is zero above the diagonal
        acc[m] = __fmaf_rn(sL[(w + 4 * m) * NB + j], rv, acc[m]);
    }
  }
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const size_t idx = (size_t)k * pn + (size_t)(w + 4 * m) * L + c;
    a.r[idx] = acc[m];
    a.d[idx] = 0.f;
    a.p[idx] = 0.f;  // beta = 0 at the first step: p = z
  }
}

// x += L^{-T} d for the columns that ran an inner solve.
template <int NB>
__global__ void __launch_bounds__(256) k_mr_xupd(MrArgs a) {
  constexpr int NN = NB * NB, MR = NB / 4;
  __shared__ float sL[NN];
  const int k = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int c = blockIdx.y * CPB + lane, L = a.nrhs;
  const size_t pn = (size_t)NB * L;
  for (int e = t; e < NN; e += 256) sL[e] = a.Li[(size_t)k * NN + e];
  __syncthreads();
  if (a.done[c]) return;
  float acc[MR];
#pragma unroll
  for (int m = 0; m < MR; ++m) acc[m] = 0.f;
  const float* dk = a.d + (size_t)k * pn + c;
#pragma unroll 4
  for (int j = 0; j < NB; ++j) {
    const float dv = dk[(size_t)j * L];
#pragma unroll
    for (int m = 0; m < MR; ++m)  // (L^{-1})_{j i} = 0 for j < i
      acc[m] = __fmaf_rn(sL[j * NB + w + 4 * m], dv, acc[m]);
  }
#pragma unroll
  for (int m = 0; m < MR; ++m)
    a.x[(size_t)k * pn + (size_t)(w + 4 * m) * L + c] += (double)acc[m];
}

__global__ void k_mr_outer_done(MrArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.nrhs || a.done[c]) return;
  a.outer[c] += 1;
  if (a.inner[c] == 0) {
    a.status[c] = BT_EBREAKDOWN;
    a.done[c] = 1;
  }
}

__global__ void k_mr_zero_x(MrArgs a) {
  const size_t N = (size_t)a.R * a.n * a.nrhs;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x)
    a.x[i] = 0.0;
}

__global__ void k_mr_info(MrArgs a, bt_info* info) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.nrhs) return;
  const double nb = a.nb2[c];
  info[c].status = a.status[c];
  info[c].iters = a.total[c];
  info[c].outer = a.outer[c];
  info[c].fail_index = -1;
  const double rr = nb > 0.0 ? sqrt(a.nr2[c] / nb) : 0.0;
  info[c].relres = rr;
  info[c].relres_true = rr;
}

// F (float32) -> Fhi + Flo (bfloat16 pair).
__global__ void k_mr_split(const float* F, unsigned short* hi,
                           unsigned short* lo, size_t N) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const float v = F[i];
    const unsigned short h = f2bf(v);
    hi[i] = h;
    lo[i] = f2bf(v - bf2f(h));
  }
}

template <int NB, int EPI>
hipError_t app(const MrArgs& a, const float* V, const float* V2,
               const float* aux, float* out, float* out2, hipStream_t s) {
  const int rows = 8 * ((a.R + 7) / 8);
  hipLaunchKernelGGL((k_mr_app<NB, EPI>), dim3(rows, a.nrhs / CPB), dim3(WG),
                     0, s, a, V, V2, aux, out, out2);
  return hipGetLastError();
}

// z = M^{-1} r at a = 1 for the current r: y0 = r + C r, then per extra term
// y = C(C y), z = y0 + alpha_1 y (m <= 2 on this path; m = 1 reuses the Z
// epilogue with alpha_1 = 0). ``y0_done``: y0 already formed (by EPI_Y0U).
template <int NB>
hipError_t precond(const MrArgs& a, hipStream_t s, bool y0_done) {
  hipError_t e = hipSuccess;
  if (!y0_done) {
    e = app<NB, EPI_Y0>(a, a.r, nullptr, a.r, a.y0, nullptr, s);
    if (e != hipSuccess) return e;
  }
  MrArgs b = a;
  if (a.m == 1) b.alpha1 = 0.0;
  e = app<NB, EPI_W>(b, a.y0, nullptr, nullptr, a.w, nullptr, s);
  if (e != hipSuccess) return e;
  return app<NB, EPI_Z>(b, a.w, nullptr, a.y0, a.z, nullptr, s);
}

// One inner iteration up to and including y0 = r + C r of the new residual;
// swaps the p and r panels of ``a``.
template <int NB>
hipError_t inner_iteration(MrArgs& a, hipStream_t s) {
  hipError_t e = app<NB, EPI_QU>(a, a.z, a.p, nullptr, a.q, a.p2, s);
  if (e != hipSuccess) return e;
  std::swap(a.p, a.p2);
  hipLaunchKernelGGL((k_mr_colsum<SUM_SIGMA>), dim3(a.nrhs), dim3(256), 0, s, a);
  e = app<NB, EPI_Y0U>(a, a.r, a.q, a.p, a.y0, a.r2, s);
  if (e != hipSuccess) return e;
  std::swap(a.r, a.r2);
  return hipSuccess;
}

template <int NB>
int solve(const MrArgs& a0, double* r64, int max_outer, bt_info* info,
          hipStream_t s) {
  MrArgs a = a0;
  const size_t N = (size_t)a.R * a.n * a.nrhs;
  const int grid_ew = (int)std::min<size_t>((N + 255) / 256, 4096);
  int hany = 0;
  std::vector<int> flags(a.nrhs);
  // any right-hand side still running (its flag, read back after a sync)
  auto read_any = [&](int* out) -> bool {
    if (hipMemcpyAsync(flags.data(), a.act, sizeof(int) * a.nrhs,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return false;
    int o = 0;
    for (int v : flags) o |= v;
    *out = o;
    return true;
  };
  hipLaunchKernelGGL(k_mr_zero_x, dim3(grid_ew), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mr_bnorm, dim3(a.R), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_mr_init_cols, dim3(a.nrhs), dim3(256), 0, s, a);
  for (int outer = 0;; ++outer) {
    if (a.dtype == BT_DT_F64)
      hipLaunchKernelGGL((k_mr_resid<NB, double>), dim3(a.R, a.nrhs / CPB),
                         dim3(256), 0, s, a, r64, outer == 0 ? 1 : 0);
    else
      hipLaunchKernelGGL((k_mr_resid<NB, float>), dim3(a.R, a.nrhs / CPB),
                         dim3(256), 0, s, a, r64, outer == 0 ? 1 : 0);
    hipLaunchKernelGGL((k_mr_colsum<SUM_RES>), dim3(a.nrhs), dim3(256), 0, s, a);
    if (!read_any(&hany)) return BT_EHIP;
    if (hany == 0 || outer >= max_outer) break;
    hipLaunchKernelGGL((k_mr_tohat<NB>), dim3(a.R, a.nrhs / CPB), dim3(256),
                       0, s, a, r64);
    if (precond<NB>(a, s, false) != hipSuccess) return BT_EHIP;
    hipLaunchKernelGGL((k_mr_colsum<SUM_RHO>), dim3(a.nrhs), dim3(256), 0, s, a);
    for (int it = 0;; ++it) {
      if ((it & 7) == 7) {
        if (!read_any(&hany)) return BT_EHIP;
        if (hany == 0) break;
      }
      if (inner_iteration<NB>(a, s) != hipSuccess) return BT_EHIP;
      if (precond<NB>(a, s, true) != hipSuccess) return BT_EHIP;
      hipLaunchKernelGGL((k_mr_colsum<SUM_RHO>), dim3(a.nrhs), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL((k_mr_xupd<NB>), dim3(a.R, a.nrhs / CPB), dim3(256),
                       0, s, a);
    hipLaunchKernelGGL(k_mr_outer_done, dim3((a.nrhs + 63) / 64), dim3(64), 0,
                       s, a);
  }
  hipLaunchKernelGGL(k_mr_info, dim3((a.nrhs + 63) / 64), dim3(64), 0, s, a,
                     info);
  return hipGetLastError() == hipSuccess ? BT_OK : BT_EHIP;
}

}  // namespace btm

// Bytes of scratch for a multi-RHS solve: nine float32 panels, the float64
// residual panel, per-row partial sums and per-column state.
size_t bt_mrhs_scratch_bytes(int64_t R, int n, int nrhs) {
  const size_t pn = (size_t)R * n * nrhs;
  return 9 * pn * sizeof(float) + pn * sizeof(double) +
         (size_t)R * nrhs * sizeof(double) + 6 * (size_t)nrhs * sizeof(double) +
         8 * (size_t)nrhs * sizeof(int) + 256;
}

hipError_t bt_mrhs_split(const float* F, unsigned short* hi, unsigned short* lo,
                         size_t N, hipStream_t s) {
  const int grid = (int)std::min<size_t>((N + 255) / 256, 4096);
  hipLaunchKernelGGL(btm::k_mr_split, dim3(grid), dim3(256), 0, s, F, hi, lo, N);
  return hipGetLastError();
}

int bt_mrhs_run(int64_t R, int n, int nrhs, const unsigned short* Fhi,
                const unsigned short* Flo, const float* Li, const void* D,
                const void* O, int dtype, const double* b, double* x,
                double tol, int maxit, int max_outer, double inner_tol, int m,
                double alpha1, void* scratch, bt_info* info, hipStream_t s) {
  btm::MrArgs a{};
  a.R = (int)R;
  a.n = n;
  a.nrhs = nrhs;
  a.Fhi = Fhi;
  a.Flo = Flo;
  a.Li = Li;
  a.D = D;
  a.O = O;
  a.dtype = dtype;
  a.b = b;
  a.x = x;
  a.tol = tol;
  a.itol2 = inner_tol * inner_tol;
  a.maxit = maxit;
  a.m = m;
  a.alpha1 = alpha1;
  const size_t pn = (size_t)R * n * nrhs;
  unsigned char* w = (unsigned char*)scratch;
  float* f = (float*)w;
  a.p = f;
  a.q = f + pn;
  a.r = f + 2 * pn;
  a.d = f + 3 * pn;
  a.y0 = f + 4 * pn;
  a.w = f + 5 * pn;
  a.z = f + 6 * pn;
  a.p2 = f + 7 * pn;
  a.r2 = f + 8 * pn;
  double* r64 = (double*)(f + 9 * pn);
  a.part = r64 + pn;
  double* cs = a.part + (size_t)R * nrhs;
  a.rho = cs;
  a.rho0 = cs + nrhs;
  a.alpha = cs + 2 * nrhs;
  a.beta = cs + 3 * nrhs;
  a.nb2 = cs + 4 * nrhs;
  a.nr2 = cs + 5 * nrhs;
  int* is = (int*)(cs + 6 * nrhs);
  a.act = is;
  a.done = is + nrhs;
  a.first = is + 2 * nrhs;
  a.inner = is + 3 * nrhs;
  a.total = is + 4 * nrhs;
  a.outer = is + 5 * nrhs;
  a.status = is + 6 * nrhs;
  if (n == 48) return btm::solve<48>(a, r64, max_outer, info, s);
  if (n == 32) return btm::solve<32>(a, r64, max_outer, info, s);
  if (n == 16) return btm::solve<16>(a, r64, max_outer, info, s);
  if (n == 64) return btm::solve<64>(a, r64, max_outer, info, s);
  return BT_EINVAL;
}
