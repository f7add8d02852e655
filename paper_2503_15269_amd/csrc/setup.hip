// Setup kernels: the diagonal-block factors and the scaled off-diagonal
// splitting terms of the preconditioner (Section IV-A: the dense inverses of
// the D_k are the O(N n^3) part; every block row is independent).
//
// For each block row g (one workgroup per row), in float64:
//   L_g  = chol(D_g)                  (D_g = L_g L_g^T; failure => A not SPD)
//   Li_g = L_g^{-1}                   (so D_g^{-1} = Li_g^T Li_g)
//   F_g  = Li_g O_g Li_{g+1}^T        (rows with a successor in the system)
// Li_{g+1} is recomputed by the workgroup of row g from D_{g+1}, so one
// launch produces everything with no inter-workgroup dependency.
// The results are stored in the iteration's precision.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace btk {

__device__ __forceinline__ double load_rec(const void* P, size_t i,
                                           int dtype) {
  return dtype == BT_DT_F64 ? ((const double*)P)[i]
                            : (double)((const float*)P)[i];
}

__device__ __forceinline__ int find_instance(const int64_t* off, int B,
                                             int64_t g) {
  int lo = 0, hi = B;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// In-place Cholesky of the n x n matrix M (row-major, LDS); lower triangle
// receives L. Returns false (uniformly) if a pivot is not positive.
template <int NT>
__device__ bool chol_lds(double* M, int n, int* flag) {
  if (threadIdx.x == 0) *flag = 0;
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double d = M[j * n + j];
      if (d > 0.0 && d < INFINITY) M[j * n + j] = sqrt(d);
      else *flag = 1;
    }
    __syncthreads();
    if (*flag) return false;
    const double djj = M[j * n + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += NT) M[i * n + j] /= djj;
    __syncthreads();
    const int w = n - j - 1;
    for (int e = threadIdx.x; e < w * w; e += NT) {
      int ii = j + 1 + e / w, ll = j + 1 + e % w;
      if (ll <= ii) M[ii * n + ll] -= M[ii * n + j] * M[ll * n + j];
    }
  }
  __syncthreads();
  return true;
}

// Linv = L^{-1} by forward substitution, one column per thread.
template <int NT>
__device__ void trinv_lds(const double* L, double* Li, int n) {
  for (int c = threadIdx.x; c < n; c += NT) {
    for (int i = 0; i < c; ++i) Li[i * n + c] = 0.0;
    for (int i = c; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int p = c; p < i; ++p) t -= L[i * n + p] * Li[p * n + c];
      Li[i * n + c] = t / L[i * n + i];
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void store(void* P, size_t i, double v) {
  ((T*)P)[i] = (T)v;
}

template <int NT, typename T>
__global__ void __launch_bounds__(NT) k_setup(SetupArgs a) {
  extern __shared__ double sm[];
  __shared__ int flag;
  const int n = a.n;
  const int nn = n * n;
  const int64_t g = blockIdx.x;
  const int inst = find_instance(a.off, a.B, g);
  const int64_t r1 = a.off[inst + 1];
  const bool has_next = g + 1 < r1;
  double* M0 = sm;
  double* M1 = sm + nn;
  double* M2 = sm + 2 * nn;
  double* M3 = sm + 3 * nn;
  const size_t gb = (size_t)g * nn;

  for (int e = threadIdx.x; e < nn; e += NT) M0[e] = load_rec(a.D, gb + e, a.dtype);
  if (!chol_lds<NT>(M0, n, &flag)) {
    if (threadIdx.x == 0) atomicMin(&a.fail[inst], (int)(g - a.off[inst]));
    return;
  }
  trinv_lds<NT>(M0, M1, n);
  for (int e = threadIdx.x; e < nn; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    store<T>(a.L, gb + e, j <= i ? M0[e] : 0.0);
    store<T>(a.Li, gb + e, M1[e]);
  }
  if (!has_next) return;
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += NT)
    M0[e] = load_rec(a.D, gb + nn + e, a.dtype);
  if (!chol_lds<NT>(M0, n, &flag)) return;  // reported by row g+1
  trinv_lds<NT>(M0, M2, n);                  // Li_{g+1}
  const size_t ob = (size_t)(g - inst) * nn;
  for (int e = threadIdx.x; e < nn; e += NT) M0[e] = load_rec(a.O, ob + e, a.dtype);
  __syncthreads();
  // M3 = Li_g O_g
  for (int e = threadIdx.x; e < nn; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    double t = 0.0;
    for (int p = 0; p <= i; ++p) t += M1[i * n + p] * M0[p * n + j];
    M3[e] = t;
  }
  __syncthreads();
  // F_g = M3 Li_{g+1}^T
  for (int e = threadIdx.x; e < nn; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    double t = 0.0;
    for (int q = 0; q <= j; ++q) t += M3[i * n + q] * M2[j * n + q];
    store<T>(a.F, gb + e, t);
  }
}


// ---------------------------------------------------------------------------
// Small block sizes: one lane per block row, everything in registers.
// ---------------------------------------------------------------------------
template <int NB>
__device__ __forceinline__ constexpr int tri(int i, int j) {
  return i * (i + 1) / 2 + j;  // packed lower triangle, row-major
}

// L_g = chol(D_g) and Li_g = L_g^{-1} (in place, row by row), float64.
template <int NB, typename T, typename Rec>
__global__ void __launch_bounds__(64) k_factor_lane(SetupArgs a) {
  const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (g >= a.R) return;
  constexpr int NL = NB * (NB + 1) / 2;
  constexpr int NN = NB * NB;
  double M[NL];
  const Rec* D = (const Rec*)a.D + (size_t)g * NN;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) M[tri<NB>(i, j)] = (double)D[i * NB + j];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double s = M[tri<NB>(j, j)];
#pragma unroll
    for (int p = 0; p < j; ++p) s -= M[tri<NB>(j, p)] * M[tri<NB>(j, p)];
    if (!(s > 0.0 && s < INFINITY)) {
      ok = false;
      s = 1.0;
    }
    const double d = sqrt(s);
    const double rd = 1.0 / d;
    M[tri<NB>(j, j)] = d;
#pragma unroll
    for (int i = j + 1; i < NB; ++i) {
      double t = M[tri<NB>(i, j)];
#pragma unroll
      for (int p = 0; p < j; ++p) t -= M[tri<NB>(i, p)] * M[tri<NB>(j, p)];
      M[tri<NB>(i, j)] = t * rd;
    }
  }
  if (!ok) {
    const int inst = find_instance(a.off, a.B, g);
    atomicMin(&a.fail[inst], (int)(g - a.off[inst]));
  }
  T* L = (T*)a.L + (size_t)g * NN;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) L[i * NB + j] = (T)(j <= i ? M[tri<NB>(i, j)] : 0.0);
  // X = L^{-1}: X[i][j] = -(1/L[i][i]) sum_{k=j}^{i-1} L[i][k] X[k][j];
  // row i overwrites its own L entries in increasing j, each of which is
  // read for the last time by the step that overwrites it.
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const double di = 1.0 / M[tri<NB>(i, i)];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) s += M[tri<NB>(i, k)] * M[tri<NB>(k, j)];
      M[tri<NB>(i, j)] = -s * di;
    }
    M[tri<NB>(i, i)] = di;
  }
  T* Li = (T*)a.Li + (size_t)g * NN;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) Li[i * NB + j] = (T)(j <= i ? M[tri<NB>(i, j)] : 0.0);
}

// F_g = Li_g O_g Li_{g+1}^T for rows with a successor; one wavefront per row,
// operands staged in LDS as float64.
template <int NB, typename T, typename Rec>
__global__ void __launch_bounds__(256) k_scaled_offdiag(SetupArgs a) {
  constexpr int NN = NB * NB;
  __shared__ double sm[4][4][NN];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + w;
  bool valid = g < a.R;
  int inst = 0;
  if (valid) {
    inst = find_instance(a.off, a.B, g);
    valid = g + 1 < a.off[inst + 1];
  }
  double* Lg = sm[w][0];
  double* Om = sm[w][1];
  double* Ln = sm[w][2];
  double* Tm = sm[w][3];
  if (valid) {
    const T* lig = (const T*)a.Li + (size_t)g * NN;
    const Rec* og = (const Rec*)a.O + (size_t)(g - inst) * NN;
    for (int e = l; e < NN; e += 64) {
      Lg[e] = (double)lig[e];
      Ln[e] = (double)lig[NN + e];
      Om[e] = (double)og[e];
    }
  }
  __syncthreads();
  if (valid) {
    for (int e = l; e < NN; e += 64) {
      const int i = e / NB, j = e - (e / NB) * NB;
      double t = 0.0;
      for (int p = 0; p <= i; ++p) t += Lg[i * NB + p] * Om[p * NB + j];
      Tm[e] = t;
    }
  }
  __syncthreads();
  if (valid) {
    T* F = (T*)a.F + (size_t)g * NN;
    for (int e = l; e < NN; e += 64) {
      const int i = e / NB, j = e - (e / NB) * NB;
      double t = 0.0;
      for (int q = 0; q <= j; ++q) t += Tm[i * NB + q] * Ln[j * NB + q];
      F[e] = (T)t;
    }
  }
}

template <int NB, typename T, typename Rec>
hipError_t launch_lane(const SetupArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_factor_lane<NB, T, Rec>), dim3((a.R + 63) / 64),
                     dim3(64), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_scaled_offdiag<NB, T, Rec>), dim3((a.R + 3) / 4),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int NB>
hipError_t launch_lane_nb(const SetupArgs& a, hipStream_t s) {
  const bool f64 = a.prec == BT_F64;
  const bool r64 = a.dtype == BT_DT_F64;
  if (f64) return r64 ? launch_lane<NB, double, double>(a, s)
                      : launch_lane<NB, double, float>(a, s);
  return r64 ? launch_lane<NB, float, double>(a, s)
             : launch_lane<NB, float, float>(a, s);
}

__global__ void k_setup_init(int B, int32_t* fail, int32_t* ctr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < B) fail[t] = BT_NO_FAIL;
  if (t < 64) ctr[t] = 0;
}

// dD_g = -lambda_g x_g^T ; dO_(g-i) = -(lambda_g x_{g+1}^T + x_g lambda_{g+1}^T)
__global__ void __launch_bounds__(256)
    k_adjoint_outer(int B, int n, const int64_t* off, const double* x,
                    const double* lam, double* dD, double* dO) {
  const int64_t g = blockIdx.x;
  const int inst = find_instance(off, B, g);
  const bool has_next = g + 1 < off[inst + 1];
  const int nn = n * n;
  const double* xg = x + g * n;
  const double* lg = lam + g * n;
  for (int e = threadIdx.x; e < nn; e += 256) {
    const int i = e / n, j = e - (e / n) * n;
    if (dD) dD[(size_t)g * nn + e] = -lg[i] * xg[j];
    if (dO && has_next)
      dO[(size_t)(g - inst) * nn + e] = -(lg[i] * xg[n + j] + xg[i] * lg[n + j]);
  }
}

}  // namespace btk

hipError_t bt_launch_setup(const SetupArgs& a, hipStream_t s) {
  if (a.R <= 0) return hipSuccess;
  if (a.n == 12) return btk::launch_lane_nb<12>(a, s);
  if (a.n == 6) return btk::launch_lane_nb<6>(a, s);
  const size_t sm = 4 * sizeof(double) * (size_t)a.n * a.n;
  const bool f64 = a.prec == BT_F64;
  const bool big = a.n > 16;
  const void* fn =
      big ? (f64 ? (const void*)btk::k_setup<256, double>
                 : (const void*)btk::k_setup<256, float>)
          : (f64 ? (const void*)btk::k_setup<64, double>
                 : (const void*)btk::k_setup<64, float>);
  hipError_t e = hipFuncSetAttribute(
      fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  if (big) {
    if (f64)
      hipLaunchKernelGGL((btk::k_setup<256, double>), dim3(a.R), dim3(256), sm,
                         s, a);
    else
      hipLaunchKernelGGL((btk::k_setup<256, float>), dim3(a.R), dim3(256), sm,
                         s, a);
  } else {
    if (f64)
      hipLaunchKernelGGL((btk::k_setup<64, double>), dim3(a.R), dim3(64), sm,
                         s, a);
    else
      hipLaunchKernelGGL((btk::k_setup<64, float>), dim3(a.R), dim3(64), sm, s,
                         a);
  }
  return hipGetLastError();
}

hipError_t bt_launch_setup_init(int B, int32_t* fail, int32_t* ctr,
                                hipStream_t s) {
  int n = B > 64 ? B : 64;
  hipLaunchKernelGGL(btk::k_setup_init, dim3((n + 255) / 256), dim3(256), 0, s,
                     B, fail, ctr);
  return hipGetLastError();
}

hipError_t bt_launch_adjoint_outer(int B, int n, int64_t R, const int64_t* off,
                                   const double* x, const double* lam,
                                   double* dD, double* dO, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(btk::k_adjoint_outer, dim3(R), dim3(256), 0, s, B, n, off,
                     x, lam, dD, dO);
  return hipGetLastError();
}
