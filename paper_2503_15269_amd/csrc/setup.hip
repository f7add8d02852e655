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

#include <type_traits>

#include "internal.h"

namespace btk {

__device__ __forceinline__ double load_rec(const void* P, size_t i,
                                           int dtype) {
  return dtype == BT_DT_F64 ? ((const double*)P)[i]
                            : (double)((const float*)P)[i];
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

// Under a fallback mask only the block rows of systems whose float32
// refinement stagnated are needed: a workgroup whose rows [g0, g1) hold none
// returns at once (every thread takes part in the vote, so the return is
// uniform).
__device__ __forceinline__ bool rows_needed(const SetupArgs& a, int64_t g0,
                                            int64_t g1) {
  if (!a.mask) return true;
  bool any = false;
  for (int64_t g = g0 + threadIdx.x; g < g1 && g < a.R; g += blockDim.x)
    any = any || a.mask[a.rowinst[g]].status == BT_ESTAGNATED;
  return __syncthreads_or(any);
}

template <int NT, typename T>
__global__ void __launch_bounds__(NT) k_setup(SetupArgs a) {
  if (!rows_needed(a, blockIdx.x, (int64_t)blockIdx.x + 1)) return;
  extern __shared__ double sm[];
  __shared__ int flag;
  const int n = a.n;
  const int nn = n * n;
  const int64_t g = blockIdx.x;
  const int inst = a.rowinst[g];
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
    if (a.L) store<T>(a.L, gb + e, j <= i ? M0[e] : 0.0);
    store<T>(a.Li, gb + e, M1[e]);
  }
  if (!has_next || !a.F) return;
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

// 16-byte vectors of float or double entries (clang vector types, which
// stay in registers when held in arrays)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename S>
using Vec16 = typename std::conditional<sizeof(S) == 4, f32x4, f64x2>::type;

template <typename D>
__device__ __forceinline__ void put_chunk(D* dst, const f32x4& v) {
  dst[0] = (D)v.x;
  dst[1] = (D)v.y;
  dst[2] = (D)v.z;
  dst[3] = (D)v.w;
}
template <typename D>
__device__ __forceinline__ void put_chunk(D* dst, const f64x2& v) {
  dst[0] = (D)v.x;
  dst[1] = (D)v.y;
}
__device__ __forceinline__ void get_chunk(const float* src, f32x4& v) {
  v = f32x4{src[0], src[1], src[2], src[3]};
}
__device__ __forceinline__ void get_chunk(const double* src, f64x2& v) {
  v = f64x2{src[0], src[1]};
}

// Coalesced copies between global memory (blocks of NN entries, contiguous)
// and LDS (blocks padded to NN + 1 entries, so that lane-per-block reads hit
// distinct banks). 16-byte global accesses, issued in batches of 16 per lane.
template <int NN, typename S, typename D>
__device__ __forceinline__ void stage_in(const S* src, D* lds, int nblk) {
  constexpr int EPC = 16 / sizeof(S);  // entries per 16-byte chunk
  constexpr int PER = NN / EPC;        // chunks per lane (64 blocks)
  constexpr int BAT = 16;
  static_assert(NN % EPC == 0, "blocks are whole chunks");
  using V = Vec16<S>;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i0 = 0; i0 < PER; i0 += BAT) {
    V buf[BAT];
#pragma unroll
    for (int i = 0; i < BAT; ++i) {
      const int c = l + 64 * (i0 + i);
      buf[i] = V{};
      if (i0 + i < PER && c * EPC < nblk * NN)
        buf[i] = reinterpret_cast<const V*>(src)[c];
    }
#pragma unroll
    for (int i = 0; i < BAT; ++i) {
      const int c = l + 64 * (i0 + i);
      if (i0 + i < PER && c * EPC < nblk * NN) {
        const int e0 = c * EPC, blk = e0 / NN, off = e0 - blk * NN;
        put_chunk(lds + blk * (NN + 1) + off, buf[i]);
      }
    }
  }
}

// As stage_in, keeping only the lower triangles: entry (r, q <= r) of block
// blk goes to lds[blk (NL + 1) + r (r + 1) / 2 + q], NL = NB (NB + 1) / 2.
// A 16-byte chunk never spans two rows (NB is a multiple of its entries).
template <int NB, typename S, typename D>
__device__ __forceinline__ void stage_in_lower(const S* src, D* lds,
                                               int nblk) {
  constexpr int NN = NB * NB, NL = NB * (NB + 1) / 2;
  constexpr int EPC = 16 / sizeof(S);
  constexpr int PER = NN / EPC;
  constexpr int BAT = 16;
  static_assert(NB % EPC == 0, "chunks stay inside a row");
  using V = Vec16<S>;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i0 = 0; i0 < PER; i0 += BAT) {
    V buf[BAT];
#pragma unroll
    for (int i = 0; i < BAT; ++i) {
      const int c = l + 64 * (i0 + i);
      buf[i] = V{};
      if (i0 + i < PER && c * EPC < nblk * NN)
        buf[i] = reinterpret_cast<const V*>(src)[c];
    }
#pragma unroll
    for (int i = 0; i < BAT; ++i) {
      const int c = l + 64 * (i0 + i);
      if (i0 + i < PER && c * EPC < nblk * NN) {
        const int e0 = c * EPC, blk = e0 / NN, off = e0 - blk * NN;
        const int r = off / NB, q0 = off - r * NB;
        D* row = lds + blk * (NL + 1) + r * (r + 1) / 2;
#pragma unroll
        for (int k = 0; k < EPC; ++k)
          if (q0 + k <= r) row[q0 + k] = (D)buf[i][k];
      }
    }
  }
}

template <int NN, typename T>
__device__ __forceinline__ void stage_out(const T* lds, T* dst, int nblk) {
  constexpr int EPC = 16 / sizeof(T);
  constexpr int PER = NN / EPC;
  using V = Vec16<T>;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int c = l + 64 * i;
    if (c * EPC < nblk * NN) {
      const int e0 = c * EPC, blk = e0 / NN, off = e0 - blk * NN;
      V v;
      get_chunk(lds + blk * (NN + 1) + off, v);
      reinterpret_cast<V*>(dst)[c] = v;
    }
  }
}

// L_g = chol(D_g) and Li_g = L_g^{-1} (in place, row by row), float64; one
// lane per block row, a wavefront of 64 consecutive rows per workgroup. The
// blocks pass through LDS so that global reads and writes are coalesced.
template <int NB, typename T, typename Rec>
__global__ void __launch_bounds__(64) k_factor_lane(SetupArgs a) {
  constexpr int NL = NB * (NB + 1) / 2;
  constexpr int NN = NB * NB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t g0 = (int64_t)blockIdx.x * 64;
  if (!rows_needed(a, g0, g0 + 64)) return;
  const int l = threadIdx.x;
  const int64_t g = g0 + l;
  const int nblk = (int)(a.R - g0 < 64 ? a.R - g0 : 64);
  Rec* din = reinterpret_cast<Rec*>(smem_raw);
  T* tout = reinterpret_cast<T*>(smem_raw);
  double M[NL];
  const bool live = g < a.R;
  bool staged = false;
  if constexpr (NB % (16 / (int)sizeof(Rec)) == 0) {
    if (!a.L && !a.Li) {  // only the lower triangles pass through LDS
      stage_in_lower<NB>((const Rec*)a.D + (size_t)g0 * NN, din, nblk);
      __syncthreads();
      const Rec* dl = din + (size_t)(live ? l : 0) * (NL + 1);
#pragma unroll
      for (int t = 0; t < NL; ++t) M[t] = (double)dl[t];
      staged = true;
    }
  }
  if (!staged) {
    stage_in<NN>((const Rec*)a.D + (size_t)g0 * NN, din, nblk);
    __syncthreads();
    const Rec* dl = din + (size_t)(live ? l : 0) * (NN + 1);
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) M[tri<NB>(i, j)] = (double)dl[i * NB + j];
  }
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
  if (!ok && live) {
    const int inst = a.rowinst[g];
    atomicMin(&a.fail[inst], (int)(g - a.off[inst]));
  }
  T* tl = tout + (size_t)l * (NN + 1);
  __syncthreads();  // every lane has read its D block
  if (a.L) {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
        tl[i * NB + j] = (T)(j <= i ? M[tri<NB>(i, j)] : 0.0);
    __syncthreads();
    stage_out<NN>(tout, (T*)a.L + (size_t)g0 * NN, nblk);
    __syncthreads();
  }
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
  if (a.Lp) {
    // packed lower triangle, rows one after the other, zero padding
    constexpr int NP = li_packed_len(NB);
    T* tp = tout + (size_t)l * (NP + 1);
#pragma unroll
    for (int t = 0; t < NP; ++t) tp[t] = (T)(t < NL ? M[t] : 0.0);
    __syncthreads();
    stage_out<NP>(tout, (T*)a.Lp + (size_t)g0 * NP, nblk);
    if (!a.Li) return;
    __syncthreads();  // the staging area is reused for the full blocks
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
      tl[i * NB + j] = (T)(j <= i ? M[tri<NB>(i, j)] : 0.0);
  __syncthreads();
  stage_out<NN>(tout, (T*)a.Li + (size_t)g0 * NN, nblk);
}

template <int NB, typename T, typename Rec>
constexpr size_t factor_lds() {
  return (size_t)64 * (NB * NB + 1) *
         (sizeof(T) > sizeof(Rec) ? sizeof(T) : sizeof(Rec));
}
// packed mode: lower triangles of D in, packed L^{-1} out
template <int NB, typename T, typename Rec>
constexpr size_t factor_lds_packed() {
  constexpr size_t din = (size_t)64 * (NB * (NB + 1) / 2 + 1) * sizeof(Rec);
  constexpr size_t dout = (size_t)64 * (li_packed_len(NB) + 1) * sizeof(T);
  return din > dout ? din : dout;
}

// F_g = Li_g O_g Li_{g+1}^T for the rows g with a successor in their system,
// zero for the last row of each system. A wavefront covers RPW = 64 / TPR
// consecutive rows, TPR = NB / 3 lanes per row, lane q forming rows
// 3q .. 3q+2 of F_g in float64. The Li blocks of the wavefront's rows and the
// next one are contiguous in memory, and so are their O blocks (the upper
// block of row g is number g - i for instance i, and the last row of an
// instance has none): both ranges go to LDS with coalesced 16-byte loads,
// the lanes of a row then read the same LDS words (broadcast), and the F
// blocks return through LDS for coalesced stores.
// Per wavefront the LDS holds RPW + 1 slots of LB entries (full blocks, or
// the packed lower triangles with PK) and RPW full blocks (O, then F).
// With PK two wavefronts per workgroup keep a workgroup small enough that
// five fit on a CU (ten wavefronts).
template <int NB, typename T, bool PK>
struct OffdiagGeo {
  static constexpr int TPR = NB / 3;
  static constexpr int RPW = 64 / TPR;
  static constexpr int NN = NB * NB;
  static constexpr int LB = PK ? li_packed_len(NB) : NN;
  static constexpr int PW = (RPW + 1) * LB + RPW * NN;  // entries per wave
  static constexpr int WPB = PK ? 2
                             : PW * sizeof(T) > 40000 ? 1
                             : PW * sizeof(T) > 20000 ? 2 : 4;
  static constexpr size_t LDS = (size_t)WPB * PW * sizeof(T);
};

template <int NB, typename T, typename Rec, bool PK>
__global__ void __launch_bounds__((64 * OffdiagGeo<NB, T, PK>::WPB))
    k_offdiag_rows(SetupArgs a) {
  using G = OffdiagGeo<NB, T, PK>;
  constexpr int NN = G::NN, RPW = G::RPW, TPR = G::TPR;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  {
    const int64_t wg0 = (int64_t)blockIdx.x * G::WPB * RPW;
    if (!rows_needed(a, wg0, wg0 + G::WPB * RPW)) return;
  }
  T* Ls = reinterpret_cast<T*>(smem_raw) + (size_t)w * G::PW;
  T* Os = Ls + (size_t)(RPW + 1) * G::LB;
  const int64_t g0 = ((int64_t)blockIdx.x * G::WPB + w) * RPW;
  const int r = l / TPR, q = l % TPR;
  const int64_t g = g0 + r;
  const int64_t nO = a.R - a.B;  // upper blocks in all
  const int64_t ob0 = g0 < a.R ? g0 - a.rowinst[g0] : 0;
  // Li blocks g0 .. g0 + RPW (full, or packed lower triangles of LP entries)
  // and O blocks ob0 .. ob0 + RPW - 1, all loads of a lane issued before any
  // LDS store
  constexpr int LB = PK ? li_packed_len(NB) : NN;  // Li entries per block
  {
    using V = Vec16<T>;
    using W = Vec16<Rec>;
    constexpr int EPC = 16 / sizeof(T), EPR = 16 / sizeof(Rec);
    constexpr int CL = (RPW + 1) * NN / EPC, CO = RPW * NN / EPR;
    constexpr int PL = (CL + 63) / 64, PO = (CO + 63) / 64;
    constexpr int cl = (RPW + 1) * LB / EPC;  // chunks of the staged Li range
    const T* lsrc = (const T*)(PK ? a.Lp : a.Li);
    const V* srcl = reinterpret_cast<const V*>(lsrc + (size_t)g0 * LB);
    const W* srco = reinterpret_cast<const W*>((const Rec*)a.O + (size_t)ob0 * NN);
    V bl[PL];
    W bo[PO];
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int c = l + 64 * i;
      bl[i] = V{};
      if (c < cl && g0 + (c * EPC) / LB < a.R) bl[i] = srcl[c];
    }
#pragma unroll
    for (int i = 0; i < PO; ++i) {
      const int c = l + 64 * i;
      bo[i] = W{};
      if (c < CO && ob0 + (c * EPR) / NN < nO) bo[i] = srco[c];
    }
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int c = l + 64 * i;
      if (c < cl) reinterpret_cast<V*>(Ls)[c] = bl[i];
    }
#pragma unroll
    for (int i = 0; i < PO; ++i) {
      const int c = l + 64 * i;
      if (c < CO) put_chunk(Os + c * EPR, bo[i]);
    }
  }
  bool has_next = false;
  int lo = 0;  // position of this row's O block in the staged range
  if (g < a.R) {
    const int inst = a.rowinst[g];
    has_next = g + 1 < a.off[inst + 1];
    lo = has_next ? (int)(g - inst - ob0) : 0;
  }
  __syncthreads();
  T f[3][NB];
  if (has_next) {
    const T* lk = Ls + (size_t)r * LB;        // Li_g
    const T* ln = Ls + (size_t)(r + 1) * LB;  // Li_{g+1}
    const T* ok = Os + (size_t)lo * NN;       // O_g
    // entry (i, j) of a staged Li block (zero above the diagonal)
    auto li = [&](const T* blk, int i, int j) -> double {
      if constexpr (PK) return j <= i ? (double)blk[i * (i + 1) / 2 + j] : 0.0;
      return (double)blk[i * NB + j];
    };
    double t[3][NB];
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
      for (int j = 0; j < NB; ++j) t[e][j] = 0.0;
    // T = (rows 3q..3q+2 of Li_g) O_g; Li_g is zero above the diagonal
#pragma unroll 2
    for (int p = 0; p < NB; ++p) {
      double lp[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) lp[e] = li(lk, 3 * q + e, p);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double o = (double)ok[p * NB + j];
#pragma unroll
        for (int e = 0; e < 3; ++e) t[e][j] = fma(lp[e], o, t[e][j]);
      }
    }
    // F rows = T Li_{g+1}^T
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double s3[3] = {0.0, 0.0, 0.0};
      if constexpr (PK) {
        // row j of the packed Li_{g+1} (entries j(j+1)/2 .. j(j+1)/2 + j,
        // the columns c <= j), read as the aligned 16-byte chunks covering it
        using V = Vec16<T>;
        constexpr int EPC = 16 / sizeof(T);
        constexpr int KMAX = (NB + 2 * EPC - 2) / EPC;
        const int t0 = j * (j + 1) / 2, k0 = t0 / EPC, nk = (t0 + j) / EPC - k0;
        V ch[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
          if (k <= nk) ch[k] = reinterpret_cast<const V*>(ln)[k0 + k];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c > j) break;
          const int u = t0 + c - k0 * EPC;
          const double lv = (double)ch[u / EPC][u % EPC];
#pragma unroll
          for (int e = 0; e < 3; ++e) s3[e] = fma(t[e][c], lv, s3[e]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const double lv = li(ln, j, c);
#pragma unroll
          for (int e = 0; e < 3; ++e) s3[e] = fma(t[e][c], lv, s3[e]);
        }
      }
#pragma unroll
      for (int e = 0; e < 3; ++e) f[e][j] = (T)s3[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
      for (int j = 0; j < NB; ++j) f[e][j] = (T)0;
  }
  __syncthreads();  // every lane is done reading the staged O blocks
  {
    T* fo = Os + (size_t)r * NN + (size_t)(3 * q) * NB;
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
      for (int j = 0; j < NB; ++j) fo[e * NB + j] = f[e][j];
  }
  __syncthreads();
  {
    using V = Vec16<T>;
    constexpr int EPC = 16 / sizeof(T);
    constexpr int CF = RPW * NN / EPC;
    V* dst = reinterpret_cast<V*>((T*)a.F + (size_t)g0 * NN);
#pragma unroll
    for (int i = 0; i < (CF + 63) / 64; ++i) {
      const int c = l + 64 * i;
      if (c < CF && g0 + (c * EPC) / NN < a.R)
        dst[c] = reinterpret_cast<const V*>(Os)[c];
    }
  }
}

template <int NB, typename T, typename Rec, bool PK>
hipError_t launch_offdiag_pk(const SetupArgs& a, hipStream_t s) {
  using G = OffdiagGeo<NB, T, PK>;
  static std::atomic<uint64_t> attr{0};
  hipError_t e =
      lds_limit((const void*)k_offdiag_rows<NB, T, Rec, PK>, G::LDS, attr);
  if (e != hipSuccess) return e;
  const int64_t rows_per_block = (int64_t)G::WPB * G::RPW;
  hipLaunchKernelGGL((k_offdiag_rows<NB, T, Rec, PK>),
                     dim3((unsigned)((a.R + rows_per_block - 1) / rows_per_block)),
                     dim3(64 * G::WPB), G::LDS, s, a);
  return hipGetLastError();
}

template <int NB, typename T, typename Rec>
hipError_t launch_offdiag(const SetupArgs& a, hipStream_t s) {
  if ((NB == 12 || NB == 24) && !a.Li)  // only the packed L^{-1} is written
    return launch_offdiag_pk<NB, T, Rec, true>(a, s);
  return launch_offdiag_pk<NB, T, Rec, false>(a, s);
}

template <int NB, typename T, typename Rec>
hipError_t launch_lane(const SetupArgs& a, hipStream_t s) {
  const size_t lds = a.L || a.Li ? factor_lds<NB, T, Rec>()
                                 : factor_lds_packed<NB, T, Rec>();
  static std::atomic<uint64_t> attr{0};
  hipError_t e = lds_limit((const void*)k_factor_lane<NB, T, Rec>,
                           factor_lds<NB, T, Rec>(), attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factor_lane<NB, T, Rec>), dim3((a.R + 63) / 64),
                     dim3(64), lds, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_offdiag<NB, T, Rec>(a, s);
}

template <int NB>
hipError_t launch_offdiag_nb(const SetupArgs& a, hipStream_t s) {
  const bool f64 = a.prec == BT_F64;
  const bool r64 = a.dtype == BT_DT_F64;
  if (f64) return r64 ? launch_offdiag<NB, double, double>(a, s)
                      : launch_offdiag<NB, double, float>(a, s);
  return r64 ? launch_offdiag<NB, float, double>(a, s)
             : launch_offdiag<NB, float, float>(a, s);
}

// ---------------------------------------------------------------------------
// Larger blocks (n = 16 ... 64): half a wavefront (n <= 32) or a wavefront
// per block row for the factors, one workgroup per block row for F.
// ---------------------------------------------------------------------------

// L_g = chol(D_g), Li_g = L_g^{-1}, float64; two block rows per wavefront
// for n <= 32 (lanes 0..31 and 32..63), else one. Cholesky by columns with
// lane r holding row r in registers: after the pivot step of column j each
// lane publishes its entry of column j in LDS and updates the rest of its
// row from that column (broadcast reads). The inverse row by row: lane r
// holds row r of X = L^{-1}, row k is published once final and every later
// row subtracts its multiple.
template <int NB, typename T, typename Rec>
__global__ void __launch_bounds__(64) k_factor_wave(SetupArgs a) {
  // blocks per wavefront: two when a block row fits in half a wavefront
  constexpr int BPW = NB <= 32 ? 2 : 1, LW = 64 / BPW;
  constexpr int NN = NB * NB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (!rows_needed(a, (int64_t)blockIdx.x * BPW, (int64_t)blockIdx.x * BPW + BPW))
    return;
  const int sub = threadIdx.x / LW;        // which block of the wavefront
  const int r = threadIdx.x % LW;          // row of this lane in its block
  // per block: two column buffers (Cholesky step j uses col[j & 1]) and two
  // row buffers (inverse step k uses row[k & 1]); alternating buffers let a
  // step write while the previous one's readers may still be reading, so
  // each step needs one barrier. The buffers hold LW entries so that every
  // lane publishes its column entry without a branch (entries past the
  // block are never read): at n = 24 the branch-free step takes 121 instead
  // of 180 VGPRs, four wavefronts per SIMD instead of two.
  double* col = reinterpret_cast<double*>(smem_raw) + sub * 4 * LW;
  double* row = col + 2 * LW;
  const int64_t gb = (int64_t)blockIdx.x * BPW + sub;
  const bool real = gb < a.R;              // the last wavefront may hold one
  const int64_t g = real ? gb : a.R - 1;   // (always valid memory)
  const int rr = r < NB ? r : NB - 1;  // lanes past the block mirror the last row
  const int base = sub * LW;           // lane 0 of this block
  double m[NB];
  {
    const Rec* D = (const Rec*)a.D + (size_t)g * NN + (size_t)rr * NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) m[j] = (double)D[j];
  }
  bool ok = true;
  double myrd = 1.0;  // 1 / L[rr][rr]
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double djj = __shfl(m[j], base + j);  // pivot from lane j of the block
    if (!(djj > 0.0 && djj < INFINITY)) {
      ok = false;
      djj = 1.0;
    }
    const double dj = sqrt(djj), rd = 1.0 / dj;
    // the entries above the diagonal of a lane's row are never read, so the
    // updates below run unmasked (no branches in the unrolled loops)
    m[j] = rr == j ? dj : m[j] * rd;
    if (rr == j) myrd = rd;
    double* cj = col + (j & 1) * LW;
    cj[r] = m[j];  // column j of L (entries above j never read)
    __syncthreads();
#pragma unroll
    for (int c = j + 1; c < NB; ++c) m[c] = fma(-m[j], cj[c], m[c]);
  }
  if (!ok && r == 0 && real) {
    const int inst = a.rowinst[g];
    atomicMin(&a.fail[inst], (int)(g - a.off[inst]));
  }
  if (a.L && real && r < NB) {  // row r of L is in this lane's registers
    T* L = (T*)a.L + (size_t)g * NN + (size_t)r * NB;
#pragma unroll
    for (int c = 0; c < NB; ++c) L[c] = (T)(c <= r ? m[c] : 0.0);
  }
  // X = L^{-1} by the same scheme, lane r holding row r of X: at step k
  // row k is final (scaled by 1 / L[k][k]) and published; every row i > k
  // subtracts L[i][k] times it (L[i][k] is lane i's own m[k]). X overwrites
  // L in place: before step k, x[c] holds X[rr][c] for c < k and L[rr][c]
  // for c >= k; entry k of L is read for the last time at step k, where
  // entry k of X (so far the unit row's) takes its place.
  double (&x)[NB] = m;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double lk = x[k];                  // L[rr][k]
    x[k] = k == rr ? 1.0 : 0.0;
    const double sc = rr == k ? myrd : 1.0;  // row k becomes final
#pragma unroll
    for (int c = 0; c <= k; ++c) x[c] *= sc;
    double* rk = row + (k & 1) * LW;
    if (r == k) {
#pragma unroll
      for (int c = 0; c <= k; ++c) rk[c] = x[c];
    }
    __syncthreads();
    const double f = rr > k ? lk : 0.0;  // rows below k subtract it
#pragma unroll
    for (int c = 0; c <= k; ++c) x[c] = fma(-f, rk[c], x[c]);
  }
  if (r < NB && real) {
    if (a.Lp) {  // row r of the packed lower triangle
      T* Lp = (T*)a.Lp + (size_t)g * li_packed_len(NB) + (size_t)(r * (r + 1) / 2);
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c <= r) Lp[c] = (T)x[c];
    }
    if (a.Li) {
      T* Li = (T*)a.Li + (size_t)g * NN + (size_t)r * NB;
#pragma unroll
      for (int c = 0; c < NB; ++c) Li[c] = (T)x[c];
    }
  }
}

template <int NB>
constexpr int factor_wave_bpw() { return NB <= 32 ? 2 : 1; }

template <int NB>
constexpr size_t factor_wave_lds() {
  constexpr int bpw = factor_wave_bpw<NB>();  // LW = 64 / bpw entries
  return bpw * sizeof(double) * 4 * (size_t)(64 / bpw);
}

// F_g = Li_g O_g Li_{g+1}^T (zero for the last row of each instance), one
// 256-thread workgroup per block row, operands in LDS as float64.
template <int NB, typename T, typename Rec>
__global__ void __launch_bounds__(256) k_offdiag_block(SetupArgs a) {
  constexpr int NN = NB * NB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Lg = reinterpret_cast<double*>(smem_raw);
  double* Ln = Lg + NN;
  double* Og = Ln + NN;
  double* Tm = Og + NN;
  const int64_t g = blockIdx.x;
  if (!rows_needed(a, g, g + 1)) return;
  const int t = threadIdx.x;
  const int inst = a.rowinst[g];
  const bool has_next = g + 1 < a.off[inst + 1];
  T* F = (T*)a.F + (size_t)g * NN;
  if (!has_next) {
    for (int e = t; e < NN; e += 256) F[e] = (T)0;
    return;
  }
  const T* lig = (const T*)a.Li + (size_t)g * NN;
  const Rec* og = (const Rec*)a.O + (size_t)(g - inst) * NN;
  for (int e = t; e < NN; e += 256) {
    Lg[e] = (double)lig[e];
    Ln[e] = (double)lig[NN + e];
    Og[e] = (double)og[e];
  }
  __syncthreads();
  for (int e = t; e < NN; e += 256) {
    const int i = e / NB, j = e % NB;
    double s0 = 0.0;
#pragma unroll 8
    for (int p = 0; p < NB; ++p) s0 = fma(Lg[i * NB + p], Og[p * NB + j], s0);
    Tm[e] = s0;
  }
  __syncthreads();
  for (int e = t; e < NN; e += 256) {
    const int i = e / NB, j = e % NB;
    double s0 = 0.0;
#pragma unroll 8
    for (int q = 0; q < NB; ++q) s0 = fma(Tm[i * NB + q], Ln[j * NB + q], s0);
    F[e] = (T)s0;
  }
}

// F_g for n = 32, 48, 64 on the matrix cores (v_mfma_f64_16x16x4f64),
// one workgroup per block row with a wavefront per 16-wide strip. Operands
// in LDS as float64, rows padded to n + 2 entries so that the 16 rows a
// wavefront reads at once fall in distinct banks. Li is lower triangular
// (zeros above the diagonal), so the k-steps past a strip's diagonal are
// skipped: T = Li_g O_g by column strips (wave w: columns 16w.., every row
// strip I summing k < 16 (I + 1)), then F = T Li_{g+1}^T by row strips
// (wave w: rows 16w.., column strip J summing k < 16 (J + 1)); both splits
// give every wavefront the same number of steps.
// Layouts (16x16x4, float64): A operand lane l = A[l % 16][l / 16], B
// operand lane l = B[l / 16][l % 16], result lane l element i =
// D[4 i + l / 16][l % 16] (unlike the float32 shapes, whose element i is
// row 4 (l / 16) + i).
template <int NB>
constexpr size_t offdiag_mfma_lds() {
  return 4 * sizeof(double) * (size_t)NB * (NB + 2);
}

template <int NB, typename T, typename Rec>
__global__ void __launch_bounds__(64 * (NB / 16)) k_offdiag_mfma(SetupArgs a) {
  static_assert(NB % 16 == 0, "strips of 16");
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int W = NB / 16, NN = NB * NB, P = NB + 2, NT = 64 * W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Lg = reinterpret_cast<double*>(smem_raw);
  double* Og = Lg + NB * P;
  double* Ln = Og + NB * P;
  double* Tm = Ln + NB * P;
  const int64_t g = blockIdx.x;
  if (!rows_needed(a, g, g + 1)) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int inst = a.rowinst[g];
  const bool has_next = g + 1 < a.off[inst + 1];
  T* F = (T*)a.F + (size_t)g * NN;
  if (!has_next) {
    for (int e = t; e < NN; e += NT) F[e] = (T)0;
    return;
  }
  const T* lig = (const T*)a.Li + (size_t)g * NN;
  const Rec* og = (const Rec*)a.O + (size_t)(g - inst) * NN;
  for (int e = t; e < NN; e += NT) {
    const int r = e / NB, c = e - r * NB;
    Lg[r * P + c] = (double)lig[e];
    Ln[r * P + c] = (double)lig[NN + e];
    Og[r * P + c] = (double)og[e];
  }
  __syncthreads();
  const int li = l & 15, lk = l >> 4;
  // T, column strip w
#pragma unroll
  for (int I = 0; I < W; ++I) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4 * (I + 1); ++s) {
      const double av = Lg[(16 * I + li) * P + 4 * s + lk];
      const double bv = Og[(4 * s + lk) * P + 16 * w + li];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) Tm[(16 * I + 4 * i + lk) * P + 16 * w + li] = acc[i];
  }
  __syncthreads();
  // F, row strip w
#pragma unroll
  for (int J = 0; J < W; ++J) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4 * (J + 1); ++s) {
      const double av = Tm[(16 * w + li) * P + 4 * s + lk];
      const double bv = Ln[(16 * J + li) * P + 4 * s + lk];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      F[(size_t)(16 * w + 4 * i + lk) * NB + 16 * J + li] = (T)acc[i];
  }
}

template <int NB, typename T, typename Rec>
hipError_t launch_wave(const SetupArgs& a, hipStream_t s) {
  constexpr size_t flds = factor_wave_lds<NB>();
  static std::atomic<uint64_t> fattr{0};
  const hipError_t e0 =
      lds_limit((const void*)k_factor_wave<NB, T, Rec>, flds, fattr);
  if (e0 != hipSuccess) return e0;
  constexpr int bpw = factor_wave_bpw<NB>();
  hipLaunchKernelGGL((k_factor_wave<NB, T, Rec>),
                     dim3((unsigned)((a.R + bpw - 1) / bpw)), dim3(64), flds,
                     s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.F) return e;
  if (NB == 24) return launch_offdiag<24, T, Rec>(a, s);
  if constexpr (NB % 16 == 0) {
    constexpr size_t lds = offdiag_mfma_lds<NB>();
    static std::atomic<uint64_t> attr{0};
    e = lds_limit((const void*)k_offdiag_mfma<NB, T, Rec>, lds, attr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_offdiag_mfma<NB, T, Rec>), dim3((unsigned)a.R),
                       dim3(64 * (NB / 16)), lds, s, a);
    return hipGetLastError();
  }
  constexpr size_t lds = 4 * sizeof(double) * (size_t)NB * NB;
  static std::atomic<uint64_t> attr{0};
  e = lds_limit((const void*)k_offdiag_block<NB, T, Rec>, lds, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_offdiag_block<NB, T, Rec>), dim3((unsigned)a.R),
                     dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int NB>
hipError_t launch_wave_nb(const SetupArgs& a, hipStream_t s) {
  const bool f64 = a.prec == BT_F64;
  const bool r64 = a.dtype == BT_DT_F64;
  if (f64) return r64 ? launch_wave<NB, double, double>(a, s)
                      : launch_wave<NB, double, float>(a, s);
  return r64 ? launch_wave<NB, float, double>(a, s)
             : launch_wave<NB, float, float>(a, s);
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
// ADJ_ROWS consecutive block rows per workgroup, the rows' entries as one
// flat range (consecutive threads on consecutive entries of a row: coalesced
// stores; fewer, longer workgroups than one per row).
constexpr int ADJ_ROWS = 8;
__global__ void __launch_bounds__(256)
    k_adjoint_outer(int B, int n, int64_t R, const int64_t* off,
                    const int32_t* rowinst, const double* x, const double* lam,
                    double* dD, double* dO) {
  const int64_t g0 = (int64_t)blockIdx.x * ADJ_ROWS;
  const int rows = (int)(R - g0 < ADJ_ROWS ? R - g0 : ADJ_ROWS);
  const int nn = n * n;
  for (int e = threadIdx.x; e < rows * nn; e += 256) {
    const int rr = e / nn, w = e - rr * nn;
    const int i = w / n, j = w - i * n;
    const int64_t g = g0 + rr;
    const int inst = rowinst[g];
    const double* xg = x + g * n;
    const double* lg = lam + g * n;
    if (dD) dD[(size_t)g * nn + w] = -lg[i] * xg[j];
    if (dO && g + 1 < off[inst + 1])
      dO[(size_t)(g - inst) * nn + w] = -(lg[i] * xg[n + j] + xg[i] * lg[n + j]);
  }
}

// The same for a block size known at compile time (even): each thread
// writes two consecutive entries with one 16-byte store, and the index
// arithmetic divides by constants.
template <int NB>
__global__ void __launch_bounds__(256)
    k_adjoint_outer_nb(int64_t R, const int64_t* off, const int32_t* rowinst,
                       const double* x, const double* lam, double* dD,
                       double* dO) {
  static_assert(NB % 2 == 0, "pairs of entries");
  constexpr int NN = NB * NB, PR = NN / 2;
  const int64_t g0 = (int64_t)blockIdx.x * ADJ_ROWS;
  const int rows = (int)(R - g0 < ADJ_ROWS ? R - g0 : ADJ_ROWS);
  for (int e = threadIdx.x; e < rows * PR; e += 256) {
    const int rr = e / PR, w = 2 * (e - rr * PR);
    const int i = w / NB, j = w - i * NB;  // j even, j + 1 < NB
    const int64_t g = g0 + rr;
    const int inst = rowinst[g];
    const double* xg = x + g * NB;
    const double* lg = lam + g * NB;
    if (dD) {
      const double2 v = make_double2(-lg[i] * xg[j], -lg[i] * xg[j + 1]);
      *reinterpret_cast<double2*>(dD + (size_t)g * NN + w) = v;
    }
    if (dO && g + 1 < off[inst + 1]) {
      const double2 v =
          make_double2(-(lg[i] * xg[NB + j] + xg[i] * lg[NB + j]),
                       -(lg[i] * xg[NB + j + 1] + xg[i] * lg[NB + j + 1]));
      *reinterpret_cast<double2*>(dO + (size_t)(g - inst) * NN + w) = v;
    }
  }
}

}  // namespace btk

hipError_t bt_launch_setup(const SetupArgs& a0, hipStream_t s) {
  if (a0.R <= 0) return hipSuccess;
  if (a0.n == 12) return btk::launch_lane_nb<12>(a0, s);
  if (a0.n == 6) return btk::launch_lane_nb<6>(a0, s);
  switch (a0.n) {
    case 16: return btk::launch_wave_nb<16>(a0, s);
    case 24: return btk::launch_wave_nb<24>(a0, s);
    case 32: return btk::launch_wave_nb<32>(a0, s);
    case 48: return btk::launch_wave_nb<48>(a0, s);
    case 64: return btk::launch_wave_nb<64>(a0, s);
    default: break;
  }
  const SetupArgs& a = a0;
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
                                   const int32_t* rowinst, const double* x,
                                   const double* lam, double* dD, double* dO,
                                   hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int64_t grid = (R + btk::ADJ_ROWS - 1) / btk::ADJ_ROWS;
  // 16-byte stores need 16-byte aligned outputs
  const bool a16 = ((uintptr_t)dD % 16 == 0) && ((uintptr_t)dO % 16 == 0);
#define BT_ADJ_NB(NB)                                                        \
  case NB:                                                                  \
    hipLaunchKernelGGL(btk::k_adjoint_outer_nb<NB>, dim3((unsigned)grid),   \
                       dim3(256), 0, s, R, off, rowinst, x, lam, dD, dO);   \
    return hipGetLastError();
  if (a16) {
    switch (n) {
      BT_ADJ_NB(6)
      BT_ADJ_NB(12)
      BT_ADJ_NB(16)
      BT_ADJ_NB(24)
      BT_ADJ_NB(32)
      BT_ADJ_NB(48)
      BT_ADJ_NB(64)
      default: break;
    }
  }
#undef BT_ADJ_NB
  hipLaunchKernelGGL(btk::k_adjoint_outer, dim3((unsigned)grid), dim3(256), 0,
                     s, B, n, R, off, rowinst, x, lam, dD, dO);
  return hipGetLastError();
}
