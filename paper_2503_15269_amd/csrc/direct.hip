// Batched direct solve by block Cholesky (block Thomas), the method the
// paper compares PCG against in Section IV-C:
//   S_0 = D_0,  S_k = D_k - M_k M_k^T,  L_k = chol(S_k),
//   M_k = O_{k-1}^T L_{k-1}^{-T}          (A = L L^T, L block bidiagonal)
//   forward  y_k = L_k^{-1} (b_k - M_k y_{k-1})
//   backward x_k = L_k^{-T} (y_k - M_{k+1}^T x_{k+1}).
// Each system is sequential in its horizon; the parallelism is the batch.
//
// Layout: 16 lanes per system (lane i < n holds row i of the current blocks
// in registers), four systems per wavefront, one wavefront per workgroup (so
// a barrier only synchronises the wavefront), systems taken longest first so
// that the four systems of a wavefront have similar horizons. The rows of
// L_k and M_k are published in LDS for the other lanes of the system and
// kept in the caller's scratch for the backward sweep. float64 throughout,
// from the system of record (float32 or float64).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace btd {

constexpr int GL = 16;  // lanes per system
constexpr int SPW = 4;  // systems per wavefront

template <int NB>
struct Slab {            // LDS of one system
  double L[NB][NB + 1];  // rows of L_k (then L_{k-1} for the next step)
  double M[NB][NB + 1];  // rows of M_k
  double rd[NB];         // 1 / L_k[j][j]
  double v[NB];          // right-hand side of the triangular solves
};

struct DirectArgs {
  int B, n, dtype;
  const int64_t* off;
  const int32_t* order;
  const void* D;
  const void* O;
  const double* b;
  double* x;
  double* Lbuf;  // [R][n][n]
  double* Mbuf;  // [R][n][n] (row g holds M_g; unused for a system's first row)
  bt_info* info;
};

template <typename Rec>
__device__ __forceinline__ double ld(const void* P, size_t i) {
  return (double)((const Rec*)P)[i];
}

template <int NB, typename Rec>
__global__ void __launch_bounds__(64) k_direct(DirectArgs a) {
  constexpr int NN = NB * NB;
  __shared__ Slab<NB> slabs[SPW];
  const int lane = threadIdx.x, grp = lane / GL, i = lane % GL;
  const int base = grp * GL;
  const int slot = blockIdx.x * SPW + grp;
  const bool has_sys = slot < a.B;
  const int sys = has_sys ? a.order[slot] : 0;
  const int64_t r0 = a.off[sys];
  const int N = has_sys ? (int)(a.off[sys + 1] - r0) : 0;
  const int ob0 = (int)(r0 - sys);  // first upper block of the system
  const bool row = i < NB;          // a lane with a block row
  const int ii = row ? i : NB - 1;
  Slab<NB>& sl = slabs[grp];
  // longest horizon of the wavefront (uniform loop bound)
  int Nmax = N;
#pragma unroll
  for (int s = 16; s < 64; s <<= 1) Nmax = max(Nmax, __shfl_xor(Nmax, s));
  int fail = -1;
  double y[NB];   // y_{k-1}, then y_k (every lane of the system holds it all)
  double m[NB];   // row i of M_k
  double S[NB];   // row i of S_k, then of L_k
#pragma unroll
  for (int c = 0; c < NB; ++c) y[c] = 0.0;

  // ------------------------------------------------------------ forward
  for (int k = 0; k < Nmax; ++k) {
    const bool act = k < N;
    const int64_t g = r0 + (act ? k : 0);
    // (a finished system re-reads its first row: always valid memory)
#pragma unroll
    for (int c = 0; c < NB; ++c)
      S[c] = ld<Rec>(a.D, (size_t)g * NN + (size_t)ii * NB + c);
    double v = a.b[g * NB + ii];
    if (act && k > 0) {
      // row i of M_k: L_{k-1} m^T = column i of O_{k-1}
      const size_t ob = (size_t)(ob0 + k - 1) * NN;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double t = ld<Rec>(a.O, ob + (size_t)c * NB + ii);
#pragma unroll
        for (int p = 0; p < c; ++p) t = fma(-sl.L[c][p], m[p], t);
        m[c] = t * sl.rd[c];
      }
      // v -= M_k y_{k-1}
#pragma unroll
      for (int p = 0; p < NB; ++p) v = fma(-m[p], y[p], v);
    }
    __syncthreads();  // L_{k-1} no longer read
    if (act && k > 0) {
      if (row) {
#pragma unroll
        for (int p = 0; p < NB; ++p) {
          sl.M[i][p] = m[p];
          a.Mbuf[(size_t)g * NN + (size_t)i * NB + p] = m[p];
        }
      }
    }
    __syncthreads();
    if (act && k > 0) {
      // S_k = D_k - M_k M_k^T (row i)
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double t = S[c];
#pragma unroll
        for (int p = 0; p < NB; ++p) t = fma(-m[p], sl.M[c][p], t);
        S[c] = t;
      }
    }
    // Cholesky of S_k, lane i keeping row i
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double djj = __shfl(S[j], base + j);
      if (act && !(djj > 0.0 && djj < INFINITY)) {
        if (fail < 0) fail = k;
        djj = 1.0;
      }
      const double dj = sqrt(djj), rdj = 1.0 / dj;
      if (ii > j) S[j] *= rdj;
      if (ii == j) S[j] = dj;
      if (row && i >= j) sl.L[i][j] = S[j];
      if (i == 0) sl.rd[j] = rdj;
      __syncthreads();
#pragma unroll
      for (int c = j + 1; c < NB; ++c) {
        const double lcj = sl.L[c][j];
        if (ii >= c) S[c] = fma(-S[j], lcj, S[c]);
      }
    }
    // y_k = L_k^{-1} v, formed by every lane of the system
    if (row) sl.v[i] = v;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double t = sl.v[c];
#pragma unroll
      for (int p = 0; p < c; ++p) t = fma(-sl.L[c][p], y[p], t);
      y[c] = t * sl.rd[c];
    }
    if (act && row) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        a.Lbuf[(size_t)g * NN + (size_t)i * NB + c] = c <= i ? S[c] : 0.0;
      a.x[g * NB + i] = y[i];  // y_k, replaced by x_k on the way back
    }
  }

  // ----------------------------------------------------------- backward
  double xn[NB];  // x_{k+1}
#pragma unroll
  for (int c = 0; c < NB; ++c) xn[c] = 0.0;
  for (int k = Nmax - 1; k >= 0; --k) {
    const bool act = k < N;
    const int64_t g = r0 + (act ? k : 0);
    double u = 0.0;
    __syncthreads();  // the previous step's LDS reads are done
    if (act && row) {
      u = a.x[g * NB + i];
      if (k + 1 < N) {  // u -= M_{k+1}^T x_{k+1}
        const size_t mb = (size_t)(g + 1) * NN;
#pragma unroll
        for (int c = 0; c < NB; ++c) u = fma(-a.Mbuf[mb + (size_t)c * NB + i], xn[c], u);
      }
#pragma unroll
      for (int c = 0; c < NB; ++c)
        sl.L[i][c] = a.Lbuf[(size_t)g * NN + (size_t)i * NB + c];
      sl.v[i] = u;
    }
    __syncthreads();
    // x_k = L_k^{-T} u (back substitution, every lane of the system)
    double xk[NB];
#pragma unroll
    for (int c = NB - 1; c >= 0; --c) {
      double t = sl.v[c];
#pragma unroll
      for (int p = c + 1; p < NB; ++p) t = fma(-sl.L[p][c], xk[p], t);
      xk[c] = t / sl.L[c][c];
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < NB; ++c) xn[c] = xk[c];
      if (row) a.x[g * NB + i] = xk[i];
    }
  }
  if (has_sys && i == 0) {
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
  const int grid = (a.B + SPW - 1) / SPW;
  if (a.dtype == BT_DT_F64)
    hipLaunchKernelGGL((k_direct<NB, double>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_direct<NB, float>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace btd

size_t bt_direct_scratch_bytes(int64_t R, int n) {
  return 2 * (size_t)R * n * n * sizeof(double);
}

bool bt_direct_supported(int n) { return n >= 1 && n <= 16; }

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
    default: return btd::launch_nb<16>(a, s);
  }
}
