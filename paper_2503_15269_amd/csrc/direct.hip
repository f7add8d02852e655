// Batched direct solve by block Cholesky (block Thomas), the method the
// paper compares PCG against in Section IV-C:
//   S_0 = D_0,  S_k = D_k - M_k M_k^T,  L_k = chol(S_k),
//   M_k = O_{k-1}^T L_{k-1}^{-T}          (A = L L^T, L block bidiagonal)
//   forward  y_k = L_k^{-1} (b_k - M_k y_{k-1})
//   backward x_k = L_k^{-T} (y_k - M_{k+1}^T x_{k+1}).
// Each system is sequential in its horizon; the parallelism is the batch.
//
// Layout: one wavefront per system (one per workgroup: no barrier and no
// LDS at all), lane i < n holding row i of the current blocks in registers.
// Every entry a lane needs from another row (the pivots and columns of the
// Cholesky of S_k, the rows of L_{k-1} in the solve for M_k, the rows of M_k
// in M_k M_k^T, the finished entries of the substitutions) is read from the
// owning lane's register with v_readlane: the sequential horizon never waits
// on memory. The rows of L_k and M_k go to the caller's scratch for the
// backward sweep; the next block row's operands are loaded while the current
// one is factored. float64 throughout, from the system of record (float32
// or float64).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace btd {

struct DirectArgs {
  int B, n, dtype;
  const int64_t* off;
  const int32_t* order;
  const void* D;
  const void* O;
  const double* b;
  double* x;
  double* Lbuf;  // [R][n][n] rows of L_k
  double* Mbuf;  // [R][n][n] rows of M_k (unused for a system's first row)
  bt_info* info;
};

template <typename Rec>
__device__ __forceinline__ double ld(const void* P, size_t i) {
  return (double)((const Rec*)P)[i];
}

__device__ __forceinline__ double bcast(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned int)lo);
}

template <int NB, typename Rec>
__global__ void __launch_bounds__(64) k_direct(DirectArgs a) {
  constexpr int NN = NB * NB;
  // prefetch the next block row when its registers fit next to the others
  constexpr bool PRE = NB <= 16;
  const int i = threadIdx.x;
  const int slot = blockIdx.x;
  const int sys = a.order[slot];
  const int64_t r0 = a.off[sys];
  const int N = (int)(a.off[sys + 1] - r0);
  const int ob0 = (int)(r0 - sys);  // first upper block of the system
  const bool row = i < NB;
  const int ii = row ? i : NB - 1;   // lanes past the block repeat row NB - 1
  int fail = -1;
  double S[NB];        // row i of D_k, S_k, then L_k
  double Lp[NB];       // row i of L_{k-1}
  double rdp[NB];      // 1 / L_{k-1}[c][c] (the same in every lane)
  double yprev = 0.0;  // y_{k-1}[i]
  double Dn[PRE ? NB : 1], On[PRE ? NB : 1], bn = 0.0;

  // row ii of D_k, column ii of O_{k-1} (k > 0) and b_k[ii]
  auto load = [&](int k, double* Dr, double* Oc, double& bv) {
    const int64_t g = r0 + k;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      Dr[c] = ld<Rec>(a.D, (size_t)g * NN + (size_t)ii * NB + c);
    if (k > 0) {
      const size_t ob = (size_t)(ob0 + k - 1) * NN;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        Oc[c] = ld<Rec>(a.O, ob + (size_t)c * NB + ii);
    }
    bv = a.b[g * NB + ii];
  };
  if constexpr (PRE) load(0, Dn, On, bn);

  // ------------------------------------------------------------ forward
  for (int k = 0; k < N; ++k) {
    const int64_t g = r0 + k;
    double v;
    double m[NB];
    if constexpr (PRE) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        S[c] = Dn[c];
        m[c] = On[c];
      }
      v = bn;
      if (k + 1 < N) load(k + 1, Dn, On, bn);
    } else {
      load(k, S, m, v);
    }
    if (k > 0) {
      // row i of M_k: L_{k-1} m = column i of O_{k-1} (forward substitution
      // in place; L_{k-1}[c][p] from lane c)
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double t = m[c];
#pragma unroll
        for (int p = 0; p < c; ++p) t = fma(-bcast(Lp[p], c), m[p], t);
        m[c] = t * rdp[c];
      }
      // v -= M_k y_{k-1} (y_{k-1}[p] from lane p)
#pragma unroll
      for (int p = 0; p < NB; ++p) v = fma(-m[p], bcast(yprev, p), v);
      if (row) {
#pragma unroll
        for (int p = 0; p < NB; ++p)
          a.Mbuf[(size_t)g * NN + (size_t)i * NB + p] = m[p];
      }
      // S_k = D_k - M_k M_k^T (row i, lower part; row c of M_k from lane c)
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double t = S[c];
#pragma unroll
        for (int p = 0; p < NB; ++p) t = fma(-m[p], bcast(m[p], c), t);
        if (c <= ii) S[c] = t;
      }
    }
    // Cholesky of S_k, lane i keeping row i; pivots and column entries from
    // the owning lanes' registers. The forward substitution y_k = L_k^{-1} v
    // runs along: once column j of L_k is known, y_k[j] (lane j) is final and
    // the lanes below subtract its share.
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double djj = bcast(S[j], j);
      if (!(djj > 0.0 && djj < INFINITY)) {
        if (fail < 0) fail = k;
        djj = 1.0;
      }
      const double dj = sqrt(djj), rdj = 1.0 / dj;
      rdp[j] = rdj;
      if (ii > j) S[j] *= rdj;
      if (ii == j) {
        S[j] = dj;
        v *= rdj;  // y_k[j]
      }
      const double yj = bcast(v, j);
      if (ii > j) v = fma(-S[j], yj, v);
#pragma unroll
      for (int c = j + 1; c < NB; ++c) {
        const double lcj = bcast(S[j], c);  // L[c][j]
        if (ii >= c) S[c] = fma(-S[j], lcj, S[c]);
      }
    }
    yprev = v;  // y_k[i]
    // L_k for the next row's M (registers) and the backward sweep (scratch)
#pragma unroll
    for (int c = 0; c < NB; ++c) Lp[c] = c <= ii ? S[c] : 0.0;
    if (row) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        a.Lbuf[(size_t)g * NN + (size_t)i * NB + c] = Lp[c];
      a.x[g * NB + i] = v;  // y_k, replaced by x_k on the way back
    }
  }

  // ----------------------------------------------------------- backward
  // Lane i reads column i of L_k and of M_{k+1} (consecutive lanes read
  // consecutive entries); the next row's are loaded during the current one
  // when their registers fit.
  constexpr bool PREB = NB <= 32;
  double Lc[NB], Mc[NB], Lcn[PREB ? NB : 1], Mcn[PREB ? NB : 1], un = 0.0;
  auto load_b = [&](int k, double* L_, double* M_, double& u_) {
    const int64_t g = r0 + k;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      L_[c] = a.Lbuf[(size_t)g * NN + (size_t)c * NB + ii];
    if (k + 1 < N) {
      const size_t mb = (size_t)(g + 1) * NN;
#pragma unroll
      for (int c = 0; c < NB; ++c) M_[c] = a.Mbuf[mb + (size_t)c * NB + ii];
    }
    u_ = a.x[g * NB + ii];
  };
  if constexpr (PREB) load_b(N - 1, Lcn, Mcn, un);
  double xn = 0.0;  // x_{k+1}[i] (none for the last row)
  for (int k = N - 1; k >= 0; --k) {
    const int64_t g = r0 + k;
    double u;
    if constexpr (PREB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        Lc[c] = Lcn[c];
        Mc[c] = Mcn[c];
      }
      u = un;
      if (k > 0) load_b(k - 1, Lcn, Mcn, un);
    } else {
      load_b(k, Lc, Mc, u);
    }
    if (k + 1 < N) {  // u -= M_{k+1}^T x_{k+1} (x_{k+1}[c] from lane c)
#pragma unroll
      for (int c = 0; c < NB; ++c) u = fma(-Mc[c], bcast(xn, c), u);
    }
    // x_k = L_k^{-T} u by columns of L_k^T: once x_k[c] (lane c) is final,
    // the lanes above subtract L[c][i] x_k[c]
#pragma unroll
    for (int c = NB - 1; c >= 0; --c) {
      if (ii == c) u /= Lc[c];
      const double xc = bcast(u, c);
      if (ii < c) u = fma(-Lc[c], xc, u);
    }
    xn = u;
    if (row) a.x[g * NB + i] = u;
  }
  if (i == 0) {
    bt_info* inf = a.info + sys;
    inf->status = fail < 0 ? BT_OK : BT_ENOTSPD;
    inf->iters = 0;
    inf->outer = 0;
    inf->fail_index = fail;
    inf->relres = NAN;
    inf->relres_true = NAN;
    inf->gemv_exec = 0;
    inf->gemv_paper = 0;
  }
}

template <int NB>
hipError_t launch_nb(const DirectArgs& a, hipStream_t s) {
  if (a.dtype == BT_DT_F64)
    hipLaunchKernelGGL((k_direct<NB, double>), dim3(a.B), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_direct<NB, float>), dim3(a.B), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace btd

size_t bt_direct_scratch_bytes(int64_t R, int n) {
  return 2 * (size_t)R * n * n * sizeof(double);
}

bool bt_direct_supported(int n) {
  return (n >= 1 && n <= 16) || n == 24 || n == 32 || n == 48 || n == 64;
}

hipError_t bt_launch_direct(int B, int n, int dtype, const int64_t* off,
                            const int32_t* order, const void* D, const void* O,
                            const double* b, double* x, bt_info* info,
                            int64_t R, void* scratch, hipStream_t s) {
  btd::DirectArgs a{};
  a.B = B;
  a.n = n;
  a.dtype = dtype;
  a.off = off;
  a.order = order;
  a.D = D;
  a.O = O;
  a.b = b;
  a.x = x;
  a.Lbuf = (double*)scratch;
  a.Mbuf = a.Lbuf + (size_t)R * n * n;
  a.info = info;
  switch (n) {
    case 1: return btd::launch_nb<1>(a, s);
    case 2: return btd::launch_nb<2>(a, s);
    case 3: return btd::launch_nb<3>(a, s);
    case 4: return btd::launch_nb<4>(a, s);
    case 5: return btd::launch_nb<5>(a, s);
    case 6: return btd::launch_nb<6>(a, s);
    case 7: return btd::launch_nb<7>(a, s);
    case 8: return btd::launch_nb<8>(a, s);
    case 9: return btd::launch_nb<9>(a, s);
    case 10: return btd::launch_nb<10>(a, s);
    case 11: return btd::launch_nb<11>(a, s);
    case 12: return btd::launch_nb<12>(a, s);
    case 13: return btd::launch_nb<13>(a, s);
    case 14: return btd::launch_nb<14>(a, s);
    case 15: return btd::launch_nb<15>(a, s);
    case 16: return btd::launch_nb<16>(a, s);
    case 24: return btd::launch_nb<24>(a, s);
    case 32: return btd::launch_nb<32>(a, s);
    case 48: return btd::launch_nb<48>(a, s);
    default: return btd::launch_nb<64>(a, s);
  }
}
