// Batched direct solve by block Cholesky (block Thomas), the method the
// paper compares PCG against in Section IV-C:
//   S_0 = D_0,  S_k = D_k - M_k M_k^T,  L_k = chol(S_k),
//   M_k = O_{k-1}^T L_{k-1}^{-T}          (A = L L^T, L block bidiagonal)
//   forward  y_k = L_k^{-1} (b_k - M_k y_{k-1})
//   backward x_k = L_k^{-T} (y_k - M_{k+1}^T x_{k+1}).
// Each system is sequential in its horizon; the parallelism is the batch.
//
// Three layouts by block size, float64 throughout, from the system of record
// (float32 or float64); in each the next block row's operands are loaded
// while the current one is factored, and what the backward sweep needs goes
// to the caller's scratch:
//   n <= 16 (k_direct4): four systems per wavefront, lane c of a 16-lane row
//     holding column c of its system's blocks; entries of other columns come
//     with DPP broadcasts inside the FMAs, on unscaled Schur complements.
//   n = 24 (k_direct): one wavefront per system (no barrier, no LDS), lane i
//     holding row i; entries of other rows are read from the owning lane's
//     register with v_readlane, so the horizon never waits on memory.
//   n = 32, 48, 64 (k_direct_mfma): one workgroup per system, a wavefront
//     per 16-wide strip, the n^3 parts on the matrix cores (below).
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

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
  // what the backward sweep reads, per block row: the diagonal factor and
  // the coupling block, each kernel in its own form (n = 24: L_k and M_k;
  // n <= 16: their unscaled forms, with the pivots 1/d_c in Rbuf; n >= 32:
  // L_k^{-1} and Z_k = L_{k-1}^{-1} O_{k-1}); the coupling block of a
  // system's first row is unused
  double* Lbuf;  // [R][n][n]
  double* Mbuf;  // [R][n][n]
  double* Rbuf;  // [R][n] 1 / d_c, the pivots of S_k (n <= 16)
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

// ------------------------------------------------------------------------
// n <= 16: four systems per wavefront, one per row of 16 lanes, lane c of a
// row holding column c of that system's current blocks. A value from
// another column j is taken with the DPP broadcast row_newbcast:j (lane j
// of each row of 16 to the whole row), which the float64 FMA applies to its
// first operand in the same instruction: every step of the sequential
// horizon is register to register, with no readlane, LDS or memory on the
// chain, and each instruction serves four systems.
//
// Column c keeps the lower-triangle entries S[r][c] (r >= c) and, above the
// diagonal, the mirrored entries S[c][r], read from the lower triangle of
// D_k. The factorisation runs on unscaled Schur complements (pivots d_j,
// multipliers S[c][j] / d_j), so no square root is ever taken:
//   L[r][c] = Sc[r][c] / sqrt(d_c),  y_c = vh_c / sqrt(d_c)
// with Sc[r][c] the entries of column c at its own pivot and vh the
// right-hand side there; the solves below use Sc, vh and 1 / d_c directly.
// The solve for the next row's M^T = L_k^{-1} O_k and the update of its
// right-hand side run inside the pivot loop of row k (pivot j finishes
// column j of L_k, which is all step j of that solve needs), filling the
// latency of the pivot chain.

// row_newbcast is a 64-bit DPP form of the VOP1/VOP2 encodings; the
// compiler does not form it, and it leaves the wait states of inline asm to
// the author: each block starts with the two the DPP read of a VGPR written
// by the previous VALU instruction requires.
template <int L>
__device__ __forceinline__ double nb(double v) {  // lane L of the row
  double r;
  asm("s_nop 1\n\tv_mov_b64_dpp %0, %1 row_newbcast:%2 row_mask:0xf "
      "bank_mask:0xf"
      : "=v"(r)
      : "v"(v), "n"(L));
  return r;
}
template <int L>
__device__ __forceinline__ double fnb(double acc, double a, double b) {
  // acc - a[lane L of the row] * b
  asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf "
      "bank_mask:0xf"
      : "+v"(acc)
      : "v"(a), "v"(b), "n"(L));
  return acc;
}
// Four independent updates behind one pair of wait states (no instruction
// of the block writes a register another one broadcasts).
// acc_i -= acc_i[lane L] * b
template <int L>
__device__ __forceinline__ void self4(double& c0, double& c1, double& c2,
                                      double& c3, double b) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %0, -%4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %1, -%4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %2, -%4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %3, -%4 row_newbcast:%5 row_mask:0xf bank_mask:0xf"
      : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3)
      : "v"(b), "n"(L));
}
template <int L>
__device__ __forceinline__ double self1(double c, double b) {
  asm("s_nop 1\n\tv_fmac_f64_dpp %0, %0, -%1 row_newbcast:%2 row_mask:0xf "
      "bank_mask:0xf"
      : "+v"(c)
      : "v"(b), "n"(L));
  return c;
}
// acc_i -= a_i[lane L] * b
template <int L>
__device__ __forceinline__ void fnb4(double& c0, double& c1, double& c2,
                                     double& c3, double a0, double a1,
                                     double a2, double a3, double b) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, -%8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %5, -%8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %6, -%8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %7, -%8 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
      : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3)
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(b), "n"(L));
}
// acc_i -= a[lane L_i] * b
template <int L0, int L1, int L2, int L3>
__device__ __forceinline__ void gram4(double& c0, double& c1, double& c2,
                                      double& c3, double a, double b) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, -%5 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %4, -%5 row_newbcast:%7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %4, -%5 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %4, -%5 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
      : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3)
      : "v"(a), "v"(b), "n"(L0), "n"(L1), "n"(L2), "n"(L3));
}

// After code that may have written EXEC with a vector instruction (the
// predicated stores), the five wait states a DPP instruction needs.
__device__ __forceinline__ void dpp_exec_fence() {
  asm volatile("s_nop 4" ::: "memory");
}

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// 1 / sqrt(d) for d > 0: the hardware estimate and two Newton steps
// y <- y + y (1 - d y^2) / 2, each doubling the correct bits.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// 1 / d: the hardware estimate and two Newton steps y <- y + y (1 - d y).
__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-d, y, 1.0), y);
  return y;
}

// Waves per workgroup. Each wave is bound by its own instruction issue (a
// lone wave issues a float64 FMA about every 7.5 cycles, a DPP FMA behind
// its wait states about every 9 to 15), and waves sharing a CU slow each
// other down even on different SIMDs: one-wave workgroups, spread over as
// many CUs as the batch allows, measured fastest.
constexpr int kDirectWaves = 1;

template <int NB, typename Rec>
__global__ void __launch_bounds__(64 * kDirectWaves) k_direct4(DirectArgs a) {
  constexpr int NN = NB * NB;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const int cc = c < NB ? c : NB - 1;  // lanes past the block mirror NB - 1
  const int slot = (blockIdx.x * kDirectWaves + (threadIdx.x >> 6)) * 4 + q;
  const bool live = slot < a.B;
  const int sys = a.order[live ? slot : a.B - 1];
  const int64_t r0 = a.off[sys];
  const int Ns = (int)(a.off[sys + 1] - r0);
  const int N = live ? Ns : 0;
  const int Nw = max(max(__builtin_amdgcn_readlane(N, 0),
                         __builtin_amdgcn_readlane(N, 16)),
                     max(__builtin_amdgcn_readlane(N, 32),
                         __builtin_amdgcn_readlane(N, 48)));
  const int ob0 = (int)(r0 - sys);
  const bool wr = live && c < NB;
  int fail = -1;

  // Rows past the system's end repeat its last row (computed, never stored).
  // Lower-triangle entries of D_k for column cc: row cc left of the
  // diagonal, column cc from it down.
  auto load_d = [&](int k, double* Dr) {
    const int64_t g = r0 + min(k, Ns - 1);
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int e = r < cc ? cc * NB + r : r * NB + cc;
      Dr[r] = ld<Rec>(a.D, (size_t)g * NN + e);
    }
  };
  // column cc of O_k (between rows k and k + 1), b_{k+1}[cc]
  auto load_o = [&](int k, double* Oc, double& bv) {
    const int kc = min(k, Ns - 2);
    if (kc >= 0) {
      const size_t ob = (size_t)(ob0 + kc) * NN;
#pragma unroll
      for (int r = 0; r < NB; ++r) Oc[r] = ld<Rec>(a.O, ob + (size_t)r * NB + cc);
      bv = a.b[(r0 + kc + 1) * NB + cc];
    } else {
#pragma unroll
      for (int r = 0; r < NB; ++r) Oc[r] = 0.0;
      bv = 0.0;
    }
  };

  double S[NB], Dn[NB], On[NB], Za[NB], Zh[NB];
  double v = a.b[r0 * NB + cc], bn;
  load_d(0, S);
  load_d(1, Dn);
  load_o(0, On, bn);

  // ------------------------------------------------------------ forward
  for (int k = 0; k < Nw; ++k) {
    const int64_t g = r0 + k;
    const bool act = k < N, nxt = k + 1 < N;
    // Za: O_k column c, becoming L_k^{-1} O_k (times sqrt d) in the loop;
    // vn: b_{k+1} - M_{k+1} y_k
#pragma unroll
    for (int r = 0; r < NB; ++r) Za[r] = On[r];
    double vn = bn;
    load_o(k + 1, On, bn);

    // Pivot j: every column c > j takes S[r][j] S[c][j] / d_j off its rows
    // r > j (S[r][j] from lane j, S[c][j] its own mirrored entry), and v
    // takes v_j S[c][j] / d_j. Columns stop changing at their own pivot.
    double ido = 1.0;
    bool spd = true;
    sfor<0, NB>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const double d = nb<j>(S[j]);
      spd = spd && d > 0.0 && d < INFINITY;
      const double id = rcp_nr(d);
      ido = c == j ? id : ido;
      const double m = c > j ? S[j] * id : 0.0;
      sfor<0, (NB - 1 - j) / 4>([&](auto G) {
        constexpr int r = j + 1 + 4 * decltype(G)::value;
        self4<j>(S[r], S[r + 1], S[r + 2], S[r + 3], m);
      });
      sfor<j + 1 + 4 * ((NB - 1 - j) / 4), NB>([&](auto R) {
        constexpr int r = decltype(R)::value;
        S[r] = self1<j>(S[r], m);
      });
      // next row, step j: with Zh_j = Za_j / d_j (Za_j final: all earlier
      // columns of L_k taken off), L[r][j] z_j = Sc[r][j] Zh_j and
      // M[c][j] y_j = Zh_j[c] vh_j
      Zh[j] = Za[j] * id;
      sfor<0, (NB - 1 - j) / 4>([&](auto G) {
        constexpr int r = j + 1 + 4 * decltype(G)::value;
        fnb4<j>(Za[r], Za[r + 1], Za[r + 2], Za[r + 3], S[r], S[r + 1],
                S[r + 2], S[r + 3], Zh[j]);
      });
      sfor<j + 1 + 4 * ((NB - 1 - j) / 4), NB>([&](auto R) {
        constexpr int r = decltype(R)::value;
        Za[r] = fnb<j>(Za[r], S[r], Zh[j]);
      });
      vn = fnb<j>(vn, v, Zh[j]);
      v = self1<j>(v, m);
    });
    fail = (!spd && act && fail < 0) ? k : fail;
    if (wr && act) {
      // the column at its pivot below the diagonal, 1 / d_c, vh_c
#pragma unroll
      for (int r = 0; r < NB; ++r)
        a.Lbuf[(size_t)g * NN + (size_t)c * NB + r] = r > c ? S[r] : 0.0;
      a.Rbuf[g * NB + c] = ido;
      a.x[g * NB + c] = v;  // vh, replaced by x_k on the way back
    }
    if (wr && nxt) {
      // Za of row k + 1: M_{k+1}^T = Za / sqrt(d) row by row
#pragma unroll
      for (int r = 0; r < NB; ++r)
        a.Mbuf[(size_t)(g + 1) * NN + (size_t)c * NB + r] = Za[r];
    }
    dpp_exec_fence();
    // S_{k+1} = D_{k+1} - M M^T, (M M^T)[r][c] = sum_p Zh_p[r] Za_p[c]
#pragma unroll
    for (int r = 0; r < NB; ++r) S[r] = Dn[r];
    load_d(k + 2, Dn);
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      sfor<0, NB / 4>([&](auto G) {
        constexpr int r = 4 * decltype(G)::value;
        gram4<r, r + 1, r + 2, r + 3>(S[r], S[r + 1], S[r + 2], S[r + 3],
                                      Zh[p], Za[p]);
      });
      sfor<4 * (NB / 4), NB>([&](auto R) {
        constexpr int r = decltype(R)::value;
        S[r] = fnb<r>(S[r], Zh[p], Za[p]);
      });
    }
    v = vn;
  }

  // ----------------------------------------------------------- backward
  // sqrt(d_c) u_c = vh_c - sum_p Za_{k+1}[p][c] x_{k+1,p} (row c of the
  // stored Za, at p n + c), then x_c = (that - sum_{r>c} Sc[r][c] x_r) / d_c.
  auto load_b = [&](int k, double* L_, double* Zr, double& id, double& u) {
    const int kc = min(k, Ns - 1);
    const int64_t g = r0 + kc;
#pragma unroll
    for (int r = 0; r < NB; ++r) L_[r] = a.Lbuf[(size_t)g * NN + (size_t)cc * NB + r];
    if (kc + 1 < Ns) {
#pragma unroll
      for (int p = 0; p < NB; ++p)
        Zr[p] = a.Mbuf[(size_t)(g + 1) * NN + (size_t)p * NB + cc];
    } else {
#pragma unroll
      for (int p = 0; p < NB; ++p) Zr[p] = 0.0;
    }
    id = a.Rbuf[g * NB + cc];
    u = a.x[g * NB + cc];
  };
  // two block rows in flight: the backward step is short next to the
  // latency of its loads
  constexpr int PD = 2;
  double Lb[PD][NB], Zb[PD][NB], idb[PD], ub[PD];
  sfor<0, PD>([&](auto I) {
    constexpr int t = decltype(I)::value;
    if (Nw - 1 - t >= 0) load_b(Nw - 1 - t, Lb[t], Zb[t], idb[t], ub[t]);
  });
  double xn = 0.0;  // x_{k+1}[c]
  for (int k0 = Nw - 1; k0 >= 0; k0 -= PD) {
    sfor<0, PD>([&](auto I) {
      constexpr int t = decltype(I)::value;
      const int k = k0 - t;
      if (k < 0) return;
      const int64_t g = r0 + k;
      const bool act = k < N;
      double L0[NB], Zr[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        L0[r] = Lb[t][r];
        Zr[r] = Zb[t][r];
      }
      double u = ub[t];
      const double id = idb[t];
      if (k - PD >= 0) load_b(k - PD, Lb[t], Zb[t], idb[t], ub[t]);
      xn = k + 1 < N ? xn : 0.0;
      double u1 = 0.0;  // two chains over the columns of Za_{k+1}
      sfor<0, NB>([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p % 2 == 0)
          u = fnb<p>(u, xn, Zr[p]);
        else
          u1 = fnb<p>(u1, xn, Zr[p]);
      });
      u += u1;
      // x_r = u_r / d_r (lane r), then the columns above take Sc[r][c] x_r
      sfor<0, NB>([&](auto J) {
        constexpr int r = NB - 1 - decltype(J)::value;
        u = fnb<r>(u, u * id, L0[r]);
      });
      xn = u * id;
      if (wr && act) a.x[g * NB + c] = xn;
      dpp_exec_fence();
    });
  }
  if (live && c == 0) {
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

// ------------------------------------------------------------------------
// n = 32, 48, 64: one workgroup per system, a wavefront per 16-wide strip,
// the n^3 parts of each block row on the matrix cores
// (v_mfma_f64_16x16x4f64), the blocks in LDS (rows padded to n + 2 entries,
// so the 16 rows a wavefront reads at once fall in distinct banks):
//   S_k = D_k - Z_k^T Z_k                 (Z_k = L_{k-1}^{-1} O_{k-1})
//   L_k = chol(S_k), blocked by 16: the diagonal block factored (and
//        inverted) by the column-in-lane DPP code of the small sizes, the
//        panel below it times the inverse's transpose, the trailing blocks
//        updated, all products on MFMA
//   L_k^{-1} by block diagonals: X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj
//   y_k = L_k^{-1} (b_k - Z_k^T y_{k-1}),   Z_{k+1} = L_k^{-1} O_k
// and backward x_k = L_k^{-T} (y_k - Z_{k+1} x_{k+1}): with the inverse
// stored, both sweeps are products, never substitutions.
// MFMA 16x16x4 float64 layouts: A operand lane l = A[l % 16][l / 16], B
// operand lane l = B[l / 16][l % 16], result lane l element i =
// D[4 i + l / 16][l % 16].
typedef double mf_d4 __attribute__((ext_vector_type(4)));

template <int NB>
struct MfLds {
  static constexpr int P = NB + 2;  // padded row stride
  static constexpr int W = NB / 16;
  static constexpr int TP = 17;     // stride of a wave's scratch tile
  double S[NB * P];                 // D_k, S_k, then L_k (lower blocks)
  double I[NB * P];                 // L_k^{-1} (lower blocks)
  double Z[NB * P];                 // Z_k, then Z_{k+1}
  double O[NB * P];                 // O_k
  double T[W][16 * TP];             // per-wavefront tile hand-off
  double v[NB], y[NB];
  int fail;
};

// acc += (NEG ? -1 : 1) Xb Yb over K entries (a multiple of 4): Xb the 16
// rows xr.. and columns xc.. of X (TX: of X^T, read as X[xc + kk][xr + i]),
// Yb the rows yr.. and 16 columns yc.. of Y (TY: of Y^T). PX, PY: strides.
template <int PX, int PY, bool TX, bool TY, bool NEG>
__device__ __forceinline__ mf_d4 mm(const double* X, int xr, int xc,
                                    const double* Y, int yr, int yc, int K,
                                    mf_d4 acc, int li, int lk) {
#pragma unroll 4
  for (int s = 0; s < K; s += 4) {
    const int kk = s + lk;
    double av = TX ? X[(xc + kk) * PX + xr + li] : X[(xr + li) * PX + xc + kk];
    if (NEG) av = -av;
    const double bv = TY ? Y[(yc + li) * PY + yr + kk] : Y[(yr + kk) * PY + yc + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

template <int P>
__device__ __forceinline__ mf_d4 tile_ld(const double* X, int r0, int c0,
                                         int li, int lk) {
  mf_d4 t;
#pragma unroll
  for (int i = 0; i < 4; ++i) t[i] = X[(r0 + 4 * i + lk) * P + c0 + li];
  return t;
}
template <int P>
__device__ __forceinline__ void tile_st(double* X, int r0, int c0, mf_d4 t,
                                        int li, int lk) {
#pragma unroll
  for (int i = 0; i < 4; ++i) X[(r0 + 4 * i + lk) * P + c0 + li] = t[i];
}

// Order the LDS accesses of one wavefront (a hand-off through its scratch
// tile between lanes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Diagonal block (b, b) of S, 16 x 16, by lanes 0..15 of one wavefront (the
// column-in-lane pivot loop of the small sizes, unscaled): lane c ends with
// column c of L_bb written into S and column c of L_bb^{-1} into I. Returns
// false in every lane if a pivot is not positive.
template <int P>
__device__ __forceinline__ bool diag_block(double* S, double* I, int b,
                                           int c) {
  const int cc = c & 15;
  double Sd[16];
#pragma unroll
  for (int r = 0; r < 16; ++r)
    Sd[r] = r >= cc ? S[(b + r) * P + b + cc] : S[(b + cc) * P + b + r];
  double dso = 1.0;
  bool spd = true;
  sfor<0, 16>([&](auto J) {
    constexpr int j = decltype(J)::value;
    const double d = nb<j>(Sd[j]);
    spd = spd && d > 0.0 && d < INFINITY;
    dso = cc == j ? d : dso;
    const double m = cc > j ? Sd[j] * rcp_nr(d) : 0.0;
    sfor<0, (15 - j) / 4>([&](auto G) {
      constexpr int r = j + 1 + 4 * decltype(G)::value;
      self4<j>(Sd[r], Sd[r + 1], Sd[r + 2], Sd[r + 3], m);
    });
    sfor<j + 1 + 4 * ((15 - j) / 4), 16>([&](auto R) {
      constexpr int r = decltype(R)::value;
      Sd[r] = self1<j>(Sd[r], m);
    });
  });
  const double rs = rsqrt_nr(dso);  // 1 / L[cc][cc]
  double Lc[16], X[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    Lc[r] = r > cc ? Sd[r] * rs : (r == cc ? dso * rs : 0.0);
    X[r] = r == cc ? 1.0 : 0.0;
  }
  // column cc of L^{-1}: L X = e_cc by forward substitution, the entries of
  // L from their columns' lanes
  sfor<0, 16>([&](auto Pp) {
    constexpr int p = decltype(Pp)::value;
    X[p] *= nb<p>(rs);
    sfor<p + 1, 16>([&](auto R) {
      constexpr int r = decltype(R)::value;
      X[r] = fnb<p>(X[r], Lc[r], X[p]);
    });
  });
  if (c < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      S[(b + r) * P + b + c] = Lc[r];
      I[(b + r) * P + b + c] = X[r];
    }
  }
  dpp_exec_fence();
  return spd;
}

template <int NB, typename Rec>
__global__ void __launch_bounds__(NB * 4) k_direct_mfma(DirectArgs a) {
  using M = MfLds<NB>;
  constexpr int P = M::P, W = M::W, NT = 64 * W, NN = NB * NB;
  constexpr int PF = (NN + NT - 1) / NT;  // prefetched entries per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  M& sm = *reinterpret_cast<M*>(smem_raw);
  // the wavefront index, uniform across the wavefront (the diagonal block's
  // DPP code runs under a test of it)
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l = t & 63, li = l & 15, lk = l >> 4;
  const int sys = a.order[blockIdx.x];
  const int64_t r0 = a.off[sys];
  const int N = (int)(a.off[sys + 1] - r0);
  const int ob0 = (int)(r0 - sys);
  if (t == 0) sm.fail = -1;

  // entries e = t + NT i of D_k (lower triangle: the upper is never read)
  // and O_{k} into registers
  double pd[PF], po[PF];
  auto fetch = [&](int k) {
    const int64_t g = r0 + k;
    const bool hasO = k + 1 < N;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = min(t + NT * i, NN - 1);
      pd[i] = ld<Rec>(a.D, (size_t)g * NN + e);
      po[i] = hasO ? ld<Rec>(a.O, (size_t)(ob0 + k) * NN + e) : 0.0;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = t + NT * i;
      if (e < NN) {
        const int r = e / NB, cl = e - r * NB;
        sm.S[r * P + cl] = pd[i];
        sm.O[r * P + cl] = po[i];
      }
    }
  };
  fetch(0);
  for (int k = 0; k < N; ++k) {
    const int64_t g = r0 + k;
    stage();
    if (k + 1 < N) fetch(k + 1);
    __syncthreads();
    // S_k = D_k - Z_k^T Z_k (lower tiles) and v = b_k - Z_k^T y_{k-1}
    if (t < NB) {
      double v = a.b[g * NB + t];
      if (k > 0)
        for (int p = 0; p < NB; ++p) v = fma(-sm.Z[p * P + t], sm.y[p], v);
      sm.v[t] = v;
    }
    if (k > 0) {
      for (int tile = w; tile < W * (W + 1) / 2; tile += W) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= tile) ++I;
        const int J = tile - I * (I + 1) / 2;
        mf_d4 acc = tile_ld<P>(sm.S, 16 * I, 16 * J, li, lk);
        acc = mm<P, P, true, false, true>(sm.Z, 16 * I, 0, sm.Z, 0, 16 * J, NB,
                                          acc, li, lk);
        tile_st<P>(sm.S, 16 * I, 16 * J, acc, li, lk);
      }
    }
    __syncthreads();
    // blocked Cholesky of S_k with the inverses of the diagonal blocks
    for (int jb = 0; jb < W; ++jb) {
      if (w == 0) {
        const bool spd = diag_block<P>(sm.S, sm.I, 16 * jb, l);
        if (!spd && l == 0 && sm.fail < 0) sm.fail = k;
      }
      __syncthreads();
      // panel: L_ib,jb = S_ib,jb L_jb,jb^{-T}
      for (int ib = jb + 1 + w; ib < W; ib += W) {
        mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mm<P, P, false, true, false>(sm.S, 16 * ib, 16 * jb, sm.I,
                                           16 * jb, 16 * jb, 16, acc, li, lk);
        tile_st<P>(sm.S, 16 * ib, 16 * jb, acc, li, lk);
      }
      __syncthreads();
      // trailing: S_ib,jc -= L_ib,jb L_jc,jb^T for ib >= jc > jb
      const int rem = W - 1 - jb;
      for (int tile = w; tile < rem * (rem + 1) / 2; tile += W) {
        int u = 0;
        while ((u + 1) * (u + 2) / 2 <= tile) ++u;
        const int ib = jb + 1 + u, jc = jb + 1 + (tile - u * (u + 1) / 2);
        mf_d4 acc = tile_ld<P>(sm.S, 16 * ib, 16 * jc, li, lk);
        acc = mm<P, P, false, true, true>(sm.S, 16 * ib, 16 * jb, sm.S,
                                          16 * jb, 16 * jc, 16, acc, li, lk);
        tile_st<P>(sm.S, 16 * ib, 16 * jc, acc, li, lk);
      }
      __syncthreads();
    }
    // L_k^{-1} below the diagonal blocks, one block diagonal at a time
    for (int d = 1; d < W; ++d) {
      for (int jb = w; jb + d < W; jb += W) {
        const int ib = jb + d;
        mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int kb = jb; kb < ib; ++kb)
          acc = mm<P, P, false, false, false>(sm.S, 16 * ib, 16 * kb, sm.I,
                                              16 * kb, 16 * jb, 16, acc, li,
                                              lk);
        tile_st<M::TP>(sm.T[w], 0, 0, acc, li, lk);
        wave_lds_sync();
        mf_d4 x = {0.0, 0.0, 0.0, 0.0};
        x = mm<P, M::TP, false, false, true>(sm.I, 16 * ib, 16 * ib, sm.T[w],
                                             0, 0, 16, x, li, lk);
        tile_st<P>(sm.I, 16 * ib, 16 * jb, x, li, lk);
        wave_lds_sync();
      }
      __syncthreads();
    }
    // y_k = L_k^{-1} v, then Z_{k+1} = L_k^{-1} O_k
    if (t < NB) {
      double y = 0.0;
      for (int j = 0; j <= t; ++j) y = fma(sm.I[t * P + j], sm.v[j], y);
      sm.y[t] = y;
      a.x[g * NB + t] = y;  // y_k, replaced by x_k on the way back
    }
    if (k + 1 < N) {
      for (int tile = w; tile < W * W; tile += W) {
        const int I = tile / W, J = tile - I * W;
        mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mm<P, P, false, false, false>(sm.I, 16 * I, 0, sm.O, 0, 16 * J,
                                            16 * (I + 1), acc, li, lk);
        tile_st<P>(sm.Z, 16 * I, 16 * J, acc, li, lk);
      }
    }
    __syncthreads();
    // L_k^{-1} and Z_{k+1} for the backward sweep (zeros above the diagonal)
    for (int e = t; e < NN; e += NT) {
      const int r = e / NB, cl = e - r * NB;
      a.Lbuf[(size_t)g * NN + e] = cl <= r ? sm.I[r * P + cl] : 0.0;
      if (k + 1 < N) a.Mbuf[(size_t)(g + 1) * NN + e] = sm.Z[r * P + cl];
    }
  }

  // ----------------------------------------------------------- backward
  // x_k = L_k^{-T} (y_k - Z_{k+1} x_{k+1}); the blocks of row k - 1 are
  // loaded while row k is computed
  auto bfetch = [&](int k) {
    const int64_t g = r0 + k;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = min(t + NT * i, NN - 1);
      pd[i] = a.Lbuf[(size_t)g * NN + e];
      po[i] = k + 1 < N ? a.Mbuf[(size_t)(g + 1) * NN + e] : 0.0;
    }
  };
  __syncthreads();
  bfetch(N - 1);
  for (int k = N - 1; k >= 0; --k) {
    const int64_t g = r0 + k;
    stage();  // L_k^{-1} into S, Z_{k+1} into O
    if (k > 0) bfetch(k - 1);
    __syncthreads();
    if (t < NB) {
      double u = a.x[g * NB + t];
      if (k + 1 < N)
        for (int j = 0; j < NB; ++j) u = fma(-sm.O[t * P + j], sm.y[j], u);
      sm.v[t] = u;
    }
    __syncthreads();
    if (t < NB) {
      double x = 0.0;
      for (int j = t; j < NB; ++j) x = fma(sm.S[j * P + t], sm.v[j], x);
      a.x[g * NB + t] = x;
      sm.y[t] = x;  // x_k for the row above
    }
    __syncthreads();
  }
  if (t == 0) {
    bt_info* inf = a.info + sys;
    const int fail = sm.fail;
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
  if constexpr (NB <= 16) {
    const int per = 4 * kDirectWaves;  // systems per workgroup
    const dim3 grid((a.B + per - 1) / per), block(64 * kDirectWaves);
    if (a.dtype == BT_DT_F64)
      hipLaunchKernelGGL((k_direct4<NB, double>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_direct4<NB, float>), grid, block, 0, s, a);
    return hipGetLastError();
  } else if constexpr (NB % 16 == 0) {
    constexpr size_t lds = sizeof(MfLds<NB>);
    static std::atomic<uint64_t> attr_d{0}, attr_f{0};
    const hipError_t e =
        a.dtype == BT_DT_F64
            ? lds_limit((const void*)k_direct_mfma<NB, double>, lds, attr_d)
            : lds_limit((const void*)k_direct_mfma<NB, float>, lds, attr_f);
    if (e != hipSuccess) return e;
    if (a.dtype == BT_DT_F64)
      hipLaunchKernelGGL((k_direct_mfma<NB, double>), dim3(a.B), dim3(NB * 4),
                         lds, s, a);
    else
      hipLaunchKernelGGL((k_direct_mfma<NB, float>), dim3(a.B), dim3(NB * 4),
                         lds, s, a);
    return hipGetLastError();
  } else {
    if (a.dtype == BT_DT_F64)
      hipLaunchKernelGGL((k_direct<NB, double>), dim3(a.B), dim3(64), 0, s, a);
    else
      hipLaunchKernelGGL((k_direct<NB, float>), dim3(a.B), dim3(64), 0, s, a);
    return hipGetLastError();
  }
}

}  // namespace btd

size_t bt_direct_scratch_bytes(int64_t R, int n) {
  return (size_t)R * (2 * (size_t)n * n + n) * sizeof(double);
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
  a.Rbuf = a.Mbuf + (size_t)R * n * n;
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
