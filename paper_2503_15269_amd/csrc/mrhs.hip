// Many right-hand sides at once: X = A^{-1} B for an [R][n][nrhs] panel of
// right-hand sides (one system, n a multiple of 16).
//
// Each right-hand side runs its own PCG (own alpha, beta, convergence), but
// the operator is applied to the whole panel, so each application of the
// scaled off-diagonal operator C (see solve.hip for the scaled form of the
// paper's preconditioner) is a pair of dense n x n by n x nrhs products per
// block row:  (C V)_k = -(F_{k-1}^T V_{k-1} + F_k V_{k+1}).
// These run on the matrix cores: v_mfma_f32_16x16x32_bf16 (16x16x16 for an
// odd last tile) with the blocks stored split as F = Fhi + Flo (two bfloat16
// arrays) and the panel split the same way on the fly; the product is
// hi*hi + hi*lo + lo*hi with float32 accumulation (relative error ~1e-5), and
// the float64 refinement on the record removes what the inner float32 solve
// leaves.
//
// One inner iteration (m = 2 shown; the polynomial follows eq. Mminv-poly-
// nomial-coefficients at a = 1: y_0 = r + C r, y_i = C(C y_{i-1}))
//   p = z + beta p, q = p - C p,
//     sigma = p'q partials                  k_mr_qu
//   alpha = rho / sigma                     k_mr_colsum<SIGMA>
//   r = r - alpha q, d += alpha p,
//     y0 = r + C r, w = C y0,
//     z = y0 + alpha_1 C w, rho = r'z parts k_mr_post
//   beta, stopping test                     k_mr_colsum<RHO>
// The vector updates are fused into the products: a workgroup forms the
// updated p (or r) of its own row and of the neighbour rows from the old
// values, so p and r alternate between two panels (the neighbours' old
// values must survive until every workgroup has read them), and k_mr_post
// recomputes the y0 and w rows its z row depends on instead of storing them.
// Workgroups are mapped to rows so that each XCD gets a contiguous range of
// block rows and the neighbour rows' data is shared in its L2. Converged
// right-hand sides no longer update; a workgroup whose columns have all
// stopped returns at once. The host checks every few iterations whether any
// is left.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "internal.h"

namespace btm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int WG = 256;       // 4 wavefronts, 16 right-hand sides each
// A block in LDS: row r holds its NB / 4 groups of four columns as 16-byte
// chunks (the four hi halves, then the four lo halves), so one 16-byte read
// gives both A operands of a K step; rows are padded by one chunk, which
// puts the 8 rows a quarter-wavefront reads at once on distinct banks.
template <int NB>
struct Lds {
  static constexpr int RS = 2 * NB + 8;  // row stride (bfloat16 entries)
  static constexpr int BLK = NB * RS;    // one block
};
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

struct MrArgs {
  int R, n, nrhs;
  const unsigned short* Fhi;  // [R][n][n] bfloat16 split of F_k
  const unsigned short* Flo;
  const unsigned short* Ghi;  // [R][n][n] the same for G_k = F_k^T
  const unsigned short* Glo;
  const float* Li;            // [R][n][n]
  const void* D;              // record
  const void* O;
  int dtype;
  const double* b;            // [R][n][nrhs]
  double* x;
  float *p, *q, *r, *d, *z;   // panels [R][n][nrhs]
  float *p2, *r2;             // second panels of p and r (alternating)
  double* part;               // [R][nrhs] per-row partial sums
  // per right-hand-side state
  double *rho, *rho0, *alpha, *beta, *nb2, *nr2;
  int *act, *done, *first, *inner, *total, *outer, *status;
  double alpha1;              // polynomial coefficient of the second term
  int m;
  int pc;                     // BT_PC_POLY
  double aw;                  // splitting weight a
  double al[BT_MAX_M];        // polynomial coefficients (al[0] = 1)
  int nz;                     // applications of C in z = M^{-1} r
  double tol, itol2;
  int maxit;
};

// ---------------------------------------------------------------------------
// Matrix-core building blocks. A 16 x 16 tile of a product is accumulated by
// v_mfma_f32_16x16x16_bf16: lane l holds rows 4 (l / 16) + i (i = 0..3) of
// column l mod 16 of the accumulator, and the B operand of a K step wants
// exactly those rows of the same column, so the result of one product feeds
// the next one without data movement. Pan<NB> is one block row of a panel
// in that layout (16 columns per wavefront); Spl<NB> the same entries split
// x = hi + lo into bfloat16, so a product is hi*hi + hi*lo + lo*hi. The A
// operand (a block) is read from LDS as 4 consecutive entries of a row, so
// products with F_k^T use the stored transposed blocks G_k.
// ---------------------------------------------------------------------------
template <int NB>
struct Pan {
  f32x4 v[NB / 16];  // rows 16 t + 4 (l / 16) + i of column l mod 16
};

template <int NB>
struct Spl {
  bf16x4 h[NB / 16], lo[NB / 16];
};

template <int NB>
__device__ __forceinline__ Spl<NB> split(const Pan<NB>& p) {
  Spl<NB> s;
#pragma unroll
  for (int t = 0; t < NB / 16; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const __bf16 h = (__bf16)p.v[t][i];  // round to nearest even
      const __bf16 lo = (__bf16)(p.v[t][i] - (float)h);
      s.h[t][i] = __builtin_bit_cast(short, h);
      s.lo[t][i] = __builtin_bit_cast(short, lo);
    }
  return s;
}

// hi*hi + hi*lo + lo*hi into acc for one K step of 16; A: the 16-byte chunk
// (4 hi, 4 lo entries of a block row) at ``e`` in LDS
__device__ __forceinline__ f32x4 mma16(const unsigned short* A, int e,
                                       bf16x4 bh, bf16x4 bl, f32x4 acc) {
  const uint4 c = *reinterpret_cast<const uint4*>(A + e);
  const bf16x4 ah = __builtin_bit_cast(bf16x4, make_uint2(c.x, c.y));
  const bf16x4 al = __builtin_bit_cast(bf16x4, make_uint2(c.z, c.w));
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
}

// The same for one K step of 32 (v_mfma_f32_16x16x32_bf16, twice the K of
// one instruction above): the instruction pairs the 8 entries of A's lane
// group g with the 8 entries of B's lane group g (measured on gfx950 with
// integer operands), so items 0..3 may carry K rows 4g.. of one 16-row tile
// and items 4..7 those of the next. The panel's tiles ks and ks + 1 then form
// the B operand as they are, and the A operand is the two 16-byte chunks of
// the block row at ``e0`` and ``e1`` (16 columns apart).
__device__ __forceinline__ f32x4 mma32(const unsigned short* A, int e0, int e1,
                                       bf16x4 bh0, bf16x4 bl0, bf16x4 bh1,
                                       bf16x4 bl1, f32x4 acc) {
  const uint4 c0 = *reinterpret_cast<const uint4*>(A + e0);
  const uint4 c1 = *reinterpret_cast<const uint4*>(A + e1);
  const bf16x8 ah = __builtin_bit_cast(bf16x8, make_uint4(c0.x, c0.y, c1.x, c1.y));
  const bf16x8 al = __builtin_bit_cast(bf16x8, make_uint4(c0.z, c0.w, c1.z, c1.w));
  const bf16x8 bh = __builtin_bit_cast(
      bf16x8, (s16x8)__builtin_shufflevector(bh0, bh1, 0, 1, 2, 3, 4, 5, 6, 7));
  const bf16x8 bl = __builtin_bit_cast(
      bf16x8, (s16x8)__builtin_shufflevector(bl0, bl1, 0, 1, 2, 3, 4, 5, 6, 7));
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
}

template <int NB, bool HM, bool HP>
__device__ __forceinline__ void cprod_t(const unsigned short* Am,
                                        const Spl<NB>& Vm,
                                        const unsigned short* Ap,
                                        const Spl<NB>& Vp, int l,
                                        f32x4 (&acc)[NB / 16]) {
  constexpr int MT = NB / 16, RS = Lds<NB>::RS;
  const int kq = 4 * (l >> 4);  // first K row of this lane in a K step
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  // K steps of 32 over pairs of tiles, one of 16 for an odd last tile
#pragma unroll
  for (int ks = 0; ks < MT; ks += 2) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      // chunk of columns 16 ks + kq .. + 3 of row 16 mt + l mod 16
      const int e = (16 * mt + (l & 15)) * RS + 2 * (16 * ks + kq);
      if (ks + 1 < MT) {
        if constexpr (HP)
          acc[mt] = mma32(Ap, e, e + 32, Vp.h[ks], Vp.lo[ks], Vp.h[ks + 1],
                          Vp.lo[ks + 1], acc[mt]);
        if constexpr (HM)
          acc[mt] = mma32(Am, e, e + 32, Vm.h[ks], Vm.lo[ks], Vm.h[ks + 1],
                          Vm.lo[ks + 1], acc[mt]);
      } else {
        if constexpr (HP) acc[mt] = mma16(Ap, e, Vp.h[ks], Vp.lo[ks], acc[mt]);
        if constexpr (HM) acc[mt] = mma16(Am, e, Vm.h[ks], Vm.lo[ks], acc[mt]);
      }
    }
  }
}

// acc = [Am V_m] + [Ap V_p], each term only if its (wavefront-uniform) flag
// is set; Am and Ap point at row-major blocks in LDS (Lds<NB> layout). With Am = G_{j-1} = F_{j-1}^T, Ap = F_j and V_m, V_p
// the rows j -+ 1 this is -(C V)_j.
template <int NB>
__device__ __forceinline__ void cprod(bool hm, const unsigned short* Am,
                                      const Spl<NB>& Vm, bool hp,
                                      const unsigned short* Ap,
                                      const Spl<NB>& Vp, int l,
                                      f32x4 (&acc)[NB / 16]) {
  if (hm && hp) cprod_t<NB, true, true>(Am, Vm, Ap, Vp, l, acc);
  else if (hp) cprod_t<NB, false, true>(Am, Vm, Ap, Vp, l, acc);
  else if (hm) cprod_t<NB, true, false>(Am, Vm, Ap, Vp, l, acc);
  else cprod_t<NB, false, false>(Am, Vm, Ap, Vp, l, acc);
}

// Grid (8 ceil(R / 8), nrhs / 64); block b works on row (b mod 8) ceil(R / 8)
// + b / 8, so that the workgroups of one XCD (dispatched round-robin) cover
// consecutive rows.
__device__ __forceinline__ int xcd_row(int b, int R) {
  const int chunk = (R + 7) / 8;
  return (b & 7) * chunk + (b >> 3);
}

// NS blocks of split arrays on their way to LDS: all global loads are issued
// first (into registers), then written into the Lds<NB> layout, so a
// workgroup waits for memory once. 16-byte pieces of 8 entries (NB is a
// multiple of 8). A block index outside [0, R - 2] is clamped: that slot is
// then never read.
template <int NB, int NS>
struct Blocks {
  static constexpr int NN = NB * NB, NC = NN / 8, PER = (NC + WG - 1) / WG;
  uint4 vh[NS * PER], vl[NS * PER];

  __device__ __forceinline__ void load(const MrArgs& a, int s,
                                       const unsigned short* hi,
                                       const unsigned short* lo, int b) {
    b = min(max(b, 0), max(a.R - 2, 0));
    const uint4* sh = reinterpret_cast<const uint4*>(hi) + (size_t)b * NC;
    const uint4* sl = reinterpret_cast<const uint4*>(lo) + (size_t)b * NC;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = min((int)threadIdx.x + q * WG, NC - 1);  // stored if < NC
      vh[s * PER + q] = sh[e];
      vl[s * PER + q] = sl[e];
    }
  }
  __device__ __forceinline__ void store(int s, unsigned short* dst) const {
    constexpr int PR = NB / 8;  // pieces per row
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * WG;
      if (NC % WG == 0 || e < NC) {
        // 8 entries = two chunks of 4: (hi 0..3, lo 0..3), (hi 4..7, lo 4..7)
        const int o = (e / PR) * Lds<NB>::RS + 16 * (e % PR);
        const uint4 h = vh[s * PER + q], w = vl[s * PER + q];
        *reinterpret_cast<uint4*>(dst + o) = make_uint4(h.x, h.y, w.x, w.y);
        *reinterpret_cast<uint4*>(dst + o + 8) = make_uint4(h.z, h.w, w.z, w.w);
      }
    }
  }
};

// Panel access through buffer instructions: a resource over block row j
// ([n][nrhs] floats), the lane's column offset in a register and the row
// offset inside the block as a scalar, so no per-access address arithmetic.
struct PRow {
  __amdgpu_buffer_rsrc_t rs;
};

template <int NB>
__device__ __forceinline__ PRow prow(const float* X, int j, int ld) {
  const float* base = X + (size_t)j * NB * ld;
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0,
                                            NB * ld * 4, 0x00020000)};
}

// entry (16 tt + 4 (l / 16) + i, column) of the row; ``voff`` = byte offset
// of the lane's first entry
__device__ __forceinline__ float pld(PRow r, int voff, int ld, int tt, int i) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
      r.rs, voff, (16 * tt + i) * ld * 4, 0));
}

__device__ __forceinline__ void pst(PRow r, int voff, int ld, int tt, int i,
                                    float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r.rs, voff,
                                        (16 * tt + i) * ld * 4, 0);
}

// Columns past nrhs (a workgroup covers 64; nrhs is a multiple of 16): the
// lane's panel offset points past every block row, so buffer loads give 0
// and stores are dropped, and the per-column state is not read.
__device__ __forceinline__ int col_voff(int col, int kq, int ld, int nrhs) {
  return col < nrhs ? 4 * (kq * ld + col) : 0x40000000;
}
__device__ __forceinline__ bool col_act(const MrArgs& a, int col) {
  return col < a.nrhs && a.act[col] != 0;
}

// ---------------------------------------------------------------------------
// p = z + beta p (new p of the row and both neighbours, formed on the fly),
// q = p - C p = Ahat p, sigma = p'q partials. For a column that has stopped
// p keeps its old value.
// ---------------------------------------------------------------------------
template <int NB>
__global__ void __launch_bounds__(WG) k_mr_qu(MrArgs a, const float* pold,
                                             float* pnew) {
  constexpr int MT = NB / 16, BLK = Lds<NB>::BLK;
  __shared__ __align__(16) unsigned short sF[2 * BLK];  // G_{k-1}, F_k
  const int k = xcd_row(blockIdx.x, a.R);
  if (k >= a.R) return;
  const int t = threadIdx.x, l = t & 63;
  const int col = blockIdx.y * CPB + (t >> 6) * CPW + (l & 15);
  const int kq = 4 * (l >> 4);
  // nothing to do once every column of this workgroup has stopped (the host
  // only checks every few iterations)
  if (!__syncthreads_or(col_act(a, blockIdx.y * CPB + (t & 63)))) return;
  const int ld = a.nrhs;
  const int voff = col_voff(col, kq, ld, a.nrhs);
  const bool act = col_act(a, col);
  const float be = act ? (float)a.beta[col] : 0.f;
  auto load = [&](int j) {
    const PRow po = prow<NB>(pold, j, ld), zr = prow<NB>(a.z, j, ld);
    Pan<NB> p;
#pragma unroll
    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float pv = pld(po, voff, ld, tt, i);
        const float pn = __fmaf_rn(be, pv, pld(zr, voff, ld, tt, i));
        p.v[tt][i] = act ? pn : pv;
      }
    return p;
  };
  const bool hm = k > 0, hp = k < a.R - 1;
  // panel rows first, then the blocks: one wait for memory
  const Pan<NB> zero{};
  const Pan<NB> pm = hm ? load(k - 1) : zero;
  const Pan<NB> pp = hp ? load(k + 1) : zero;
  const Pan<NB> p0 = load(k);
  {
    Blocks<NB, 2> blk;
    blk.load(a, 0, a.Ghi, a.Glo, k - 1);
    blk.load(a, 1, a.Fhi, a.Flo, k);
    blk.store(0, sF);
    blk.store(1, sF + BLK);
  }
  __syncthreads();
  const Spl<NB> sm = split(pm), sp = split(pp);
  f32x4 acc[MT];
  cprod<NB>(hm, sF, sm, hp, sF + BLK, sp, l, acc);
  const PRow pw = prow<NB>(pnew, k, ld), qw = prow<NB>(a.q, k, ld);
  double dp = 0.0;
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float pv = p0.v[tt][i];
      const float o = pv + acc[tt][i];  // q = p - C p, C p = -acc
      pst(pw, voff, ld, tt, i, pv);
      pst(qw, voff, ld, tt, i, o);
      dp += (double)pv * (double)o;
    }
  dp += __shfl_xor(dp, 16);
  dp += __shfl_xor(dp, 32);
  if (l < 16 && col < a.nrhs) a.part[(size_t)k * ld + col] = dp;
}

// ---------------------------------------------------------------------------
// Everything of an inner iteration after alpha, for one block row k:
//   r' = r - alpha q and d += alpha p (UPD; r' = r otherwise),
//   y0 = r' + C r',  w = C y0,  z = y0 + alpha_1 C w,  rho = r''z partials,
// writing r' (UPD) and z of row k. z_k needs w at rows k +- 1, which need y0
// at rows k - 2, k, k + 2, which need r' at rows k - 3 .. k + 3: the
// workgroup recomputes these neighbour values itself (twice the matrix-core
// work of separate passes for y0, w and z) so that y0 and w never leave the
// registers and each panel is read once from memory. LDS holds six blocks:
// G_{k-3}, F_{k-2}, G_{k-1}, F_k, G_{k+1}, F_{k+2} for the y0 rows, then
// G_{k-2}, F_{k-1}, G_k, F_{k+1} replace the first, second, fifth and sixth
// for the w rows; z uses G_{k-1}, F_k (for M = 1, z = y0 and only those two
// are staged). Dynamic LDS: (M = 1 ? 2 : 6) blocks in the Lds<NB> layout.
// ---------------------------------------------------------------------------
template <int NB, int M, bool UPD>
__global__ void __launch_bounds__(WG) k_mr_post(MrArgs a) {
  constexpr int MT = NB / 16;
  extern __shared__ __align__(16) unsigned short sF[];
  auto S = [&](int slot) { return sF + slot * Lds<NB>::BLK; };
  const int k = xcd_row(blockIdx.x, a.R);
  if (k >= a.R) return;
  const int t = threadIdx.x, l = t & 63;
  const int col = blockIdx.y * CPB + (t >> 6) * CPW + (l & 15);
  const int kq = 4 * (l >> 4);
  if (!__syncthreads_or(col_act(a, blockIdx.y * CPB + (t & 63)))) return;
  // slots for M = 2: 0 G_{k-3}, 1 F_{k-2}, 2 G_{k-1}, 3 F_k, 4 G_{k+1},
  // 5 F_{k+2}; for M = 1 only G_{k-1}, F_k, in slots 0 and 1
  constexpr int SG = M >= 2 ? 2 : 0;  // slot of G_{k-1}; F_k follows
  const int ld = a.nrhs;
  const int voff = col_voff(col, kq, ld, a.nrhs);
  const bool act = col_act(a, col);
  const float al = UPD && act ? (float)a.alpha[col] : 0.f;
  auto load = [&](int j) {  // r' of row j
    const PRow rr = prow<NB>(a.r, j, ld);
    Pan<NB> p;
    if constexpr (UPD) {
      const PRow qr = prow<NB>(a.q, j, ld);
#pragma unroll
      for (int tt = 0; tt < MT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float rv = pld(rr, voff, ld, tt, i);
          const float rn = __fmaf_rn(-al, pld(qr, voff, ld, tt, i), rv);
          p.v[tt][i] = act ? rn : rv;
        }
    } else {
#pragma unroll
      for (int tt = 0; tt < MT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) p.v[tt][i] = pld(rr, voff, ld, tt, i);
    }
    return p;
  };
  // y0 of row j from r' of row j and the split r' of rows j - 1, j + 1,
  // with G_{j-1}, F_j in slots sg, sg + 1 (absent rows: flags off)
  auto y0_of = [&](int j, int sg, const Spl<NB>& rm, const Pan<NB>& r0,
                   const Spl<NB>& rp) {
    f32x4 acc[MT];
    cprod<NB>(j >= 1, S(sg), rm, j <= a.R - 2, S(sg + 1), rp, l, acc);
    Pan<NB> y;
#pragma unroll
    for (int tt = 0; tt < MT; ++tt) y.v[tt] = r0.v[tt] - acc[tt];
    return y;
  };
  const bool hm1 = k >= 1, hp1 = k <= a.R - 2;
  const bool hm2 = M >= 2 && k >= 2, hp2 = M >= 2 && k + 2 <= a.R - 1;
  const Pan<NB> zero{};
  const Spl<NB> szero{};
  // panel rows first, then the blocks: one wait for memory
  const Pan<NB> r0 = load(k);
  const Pan<NB> rm1 = hm1 ? load(k - 1) : zero;
  const Pan<NB> rp1 = hp1 ? load(k + 1) : zero;
  const Pan<NB> rm2 = hm2 ? load(k - 2) : zero;
  const Pan<NB> rm3 = hm2 && k >= 3 ? load(k - 3) : zero;
  const Pan<NB> rp2 = hp2 ? load(k + 2) : zero;
  const Pan<NB> rp3 = hp2 && k + 3 <= a.R - 1 ? load(k + 3) : zero;
  if constexpr (UPD) {  // r' and d += alpha p of the own row
    const PRow rw = prow<NB>(a.r2, k, ld), dr = prow<NB>(a.d, k, ld),
               pr = prow<NB>(a.p, k, ld);
#pragma unroll
    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pst(rw, voff, ld, tt, i, r0.v[tt][i]);
        const float dv = pld(dr, voff, ld, tt, i);
        const float dn = __fmaf_rn(al, pld(pr, voff, ld, tt, i), dv);
        pst(dr, voff, ld, tt, i, act ? dn : dv);
      }
  }
  {
    Blocks<NB, M >= 2 ? 6 : 2> blk;
    blk.load(a, SG, a.Ghi, a.Glo, k - 1);
    blk.load(a, SG + 1, a.Fhi, a.Flo, k);
    if constexpr (M >= 2) {
      blk.load(a, 0, a.Ghi, a.Glo, k - 3);
      blk.load(a, 1, a.Fhi, a.Flo, k - 2);
      blk.load(a, 4, a.Ghi, a.Glo, k + 1);
      blk.load(a, 5, a.Fhi, a.Flo, k + 2);
    }
#pragma unroll
    for (int q = 0; q < (M >= 2 ? 6 : 2); ++q) blk.store(q, S(q));
  }
  __syncthreads();
  const Spl<NB> sm1 = split(rm1), sp1 = split(rp1);
  const Pan<NB> y0 = y0_of(k, SG, sm1, r0, sp1);
  Pan<NB> z = y0;
  if constexpr (M >= 2) {
    Pan<NB> y0m = zero, y0p = zero;
    if (hm2) y0m = y0_of(k - 2, 0, split(rm3), rm2, sm1);
    if (hp2) y0p = y0_of(k + 2, 4, sp1, rp2, split(rp3));
    // the w rows need G_{k-2}, F_{k-1}, G_k, F_{k+1}
    __syncthreads();  // every wavefront is done with the y0 blocks
    {
      Blocks<NB, 4> late;
      late.load(a, 0, a.Ghi, a.Glo, k - 2);
      late.load(a, 1, a.Fhi, a.Flo, k - 1);
      late.load(a, 2, a.Ghi, a.Glo, k);
      late.load(a, 3, a.Fhi, a.Flo, k + 1);
      late.store(0, S(0));
      late.store(1, S(1));
      late.store(2, S(4));
      late.store(3, S(5));
    }
    __syncthreads();
    const Spl<NB> s0 = split(y0);
    f32x4 acc[MT];
    Spl<NB> swm{}, swp{};
    if (hm1) {  // w_{k-1} = -(F_{k-2}^T y0_{k-2} + F_{k-1} y0_k)
      cprod<NB>(hm2, S(0), hm2 ? split(y0m) : szero, true, S(1), s0, l, acc);
      Pan<NB> w;
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) w.v[tt] = -acc[tt];
      swm = split(w);
    }
    if (hp1) {  // w_{k+1} = -(F_k^T y0_k + F_{k+1} y0_{k+2})
      cprod<NB>(true, S(4), s0, hp2, S(5), hp2 ? split(y0p) : szero, l, acc);
      Pan<NB> w;
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) w.v[tt] = -acc[tt];
      swp = split(w);
    }
    cprod<NB>(hm1, S(2), swm, hp1, S(3), swp, l, acc);
    const float a1 = (float)a.alpha1;
#pragma unroll
    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) z.v[tt][i] = y0.v[tt][i] + a1 * -acc[tt][i];
  }
  const PRow zw = prow<NB>(a.z, k, ld);
  double dp = 0.0;
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pst(zw, voff, ld, tt, i, z.v[tt][i]);
      dp += (double)r0.v[tt][i] * (double)z.v[tt][i];
    }
  dp += __shfl_xor(dp, 16);
  dp += __shfl_xor(dp, 32);
  if (l < 16 && col < a.nrhs) a.part[(size_t)k * ld + col] = dp;
}

// ---------------------------------------------------------------------------
// The preconditioner for any splitting and order (eq. Mminv-polynomial-
// coefficients in the scaled form, G = I + a C, H = (1 - a) C + a C^2),
// evaluated by Horner's rule from panel passes of one kind:
//   out_k = cx X_k + cy Y_k + cc (C V)_k
// (X, Y, V optional), with the rho partials r'_k . out_k when ``rho``.
// ---------------------------------------------------------------------------
template <int NB>
__global__ void __launch_bounds__(WG) k_mr_lin(MrArgs a, const float* X,
                                              float cx, const float* Y,
                                              float cy, const float* V,
                                              float cc, float* out, int rho) {
  constexpr int MT = NB / 16, BLK = Lds<NB>::BLK;
  __shared__ __align__(16) unsigned short sF[2 * BLK];  // G_{k-1}, F_k
  const int k = xcd_row(blockIdx.x, a.R);
  if (k >= a.R) return;
  const int t = threadIdx.x, l = t & 63;
  const int col = blockIdx.y * CPB + (t >> 6) * CPW + (l & 15);
  const int kq = 4 * (l >> 4);
  if (!__syncthreads_or(col_act(a, blockIdx.y * CPB + (t & 63)))) return;
  const int ld = a.nrhs;
  const int voff = col_voff(col, kq, ld, a.nrhs);
  auto load = [&](const float* P, int j) {
    const PRow pr = prow<NB>(P, j, ld);
    Pan<NB> v;
#pragma unroll
    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) v.v[tt][i] = pld(pr, voff, ld, tt, i);
    return v;
  };
  const bool hm = V && k > 0, hp = V && k < a.R - 1;
  const Pan<NB> zero{};
  const Pan<NB> vm = hm ? load(V, k - 1) : zero;
  const Pan<NB> vp = hp ? load(V, k + 1) : zero;
  const Pan<NB> x = X ? load(X, k) : zero;
  const Pan<NB> y = Y ? load(Y, k) : zero;
  f32x4 acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (V) {
    {
      Blocks<NB, 2> blk;
      blk.load(a, 0, a.Ghi, a.Glo, k - 1);
      blk.load(a, 1, a.Fhi, a.Flo, k);
      blk.store(0, sF);
      blk.store(1, sF + BLK);
    }
    __syncthreads();
    cprod<NB>(hm, sF, split(vm), hp, sF + BLK, split(vp), l, acc);
  }
  const PRow ow = prow<NB>(out, k, ld);
  const PRow rr = prow<NB>(a.r, k, ld);
  double dp = 0.0;
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // C V = -acc
      const float o = cx * x.v[tt][i] + cy * y.v[tt][i] - cc * acc[tt][i];
      pst(ow, voff, ld, tt, i, o);
      if (rho) dp += (double)pld(rr, voff, ld, tt, i) * (double)o;
    }
  if (rho) {
    dp += __shfl_xor(dp, 16);
    dp += __shfl_xor(dp, 32);
    if (l < 16 && col < a.nrhs) a.part[(size_t)k * ld + col] = dp;
  }
}

// r' = r - alpha q into r2 and d += alpha p, for the running columns (the
// others keep r and d).
template <int NB>
__global__ void __launch_bounds__(WG) k_mr_rupd(MrArgs a) {
  constexpr int MT = NB / 16;
  const int k = xcd_row(blockIdx.x, a.R);
  if (k >= a.R) return;
  const int t = threadIdx.x, l = t & 63;
  const int col = blockIdx.y * CPB + (t >> 6) * CPW + (l & 15);
  const int kq = 4 * (l >> 4);
  const int ld = a.nrhs;
  const int voff = col_voff(col, kq, ld, a.nrhs);
  const bool act = col_act(a, col);
  const float al = act ? (float)a.alpha[col] : 0.f;
  const PRow rr = prow<NB>(a.r, k, ld), qr = prow<NB>(a.q, k, ld),
             rw = prow<NB>(a.r2, k, ld), dr = prow<NB>(a.d, k, ld),
             pr = prow<NB>(a.p, k, ld);
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float rv = pld(rr, voff, ld, tt, i);
      pst(rw, voff, ld, tt, i, act ? __fmaf_rn(-al, pld(qr, voff, ld, tt, i), rv) : rv);
      if (act) {
        const float dv = pld(dr, voff, ld, tt, i);
        pst(dr, voff, ld, tt, i, __fmaf_rn(al, pld(pr, voff, ld, tt, i), dv));
      }
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
    const double prev = a.nr2[c];  // before the last correction
    a.nr2[c] = tot;
    if (!a.done[c]) {
      const double t2 = a.tol * a.tol * a.nb2[c];
      if (tot <= t2) {
        a.status[c] = BT_OK;
        a.done[c] = 1;
      } else if (!(tot < INFINITY)) {
        a.status[c] = BT_ENONFINITE;
        a.done[c] = 1;
      } else if (a.outer[c] > 0 && tot > 0.25 * prev) {
        // the correction cut the float64 residual by less than 2x
        a.status[c] = BT_ESTAGNATED;
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

__global__ void k_mr_init_cols(MrArgs a, int warm) {
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
  if (warm && s[0] == 0.0)  // b = 0: x = 0 whatever the initial guess
    for (size_t e = threadIdx.x; e < (size_t)a.R * a.n; e += 256)
      a.x[e * a.nrhs + c] = 0.0;
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
  const bool cv = c < L;  // a column of the panel (nrhs % 64 may be nonzero)
  const bool done = !cv || a.done[c] != 0;
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
    if (cv) r64[idx] = v;
    ss = fma(v, v, ss);
  }
  red[w][lane] = ss;
  __syncthreads();
  if (w == 0 && cv)
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
  if (c >= L) return;  // past the panel (no barrier follows)
  float acc[MR];
#pragma unroll
  for (int m = 0; m < MR; ++m) acc[m] = 0.f;
  if (a.act[c]) {
    // the column's residual scaled by a power of two to norm in [1, 2)
    // before it is rounded to float32 (undone in k_mr_xupd)
    const double sc = bt_unit_scale(a.nr2[c]);
    const double* rk = r64 + (size_t)k * pn + c;
#pragma unroll 4
    for (int j = 0; j < NB; ++j) {
      const float rv = (float)(rk[(size_t)j * L] * sc);
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
  if (c >= L || a.done[c]) return;
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
  const double unscale = 1.0 / bt_unit_scale(a.nr2[c]);
#pragma unroll
  for (int m = 0; m < MR; ++m)
    a.x[(size_t)k * pn + (size_t)(w + 4 * m) * L + c] +=
        (double)acc[m] * unscale;
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

__global__ void k_mr_info(MrArgs a, bt_info* info, int warm) {
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
  // per refinement step: z = M^{-1} r (nz applications of C) and the two
  // triangular transforms; per inner iteration: 1 + nz applications; a
  // float64 residual after every step (and before the first from a guess)
  const int64_t halves =
      2 * ((int64_t)a.nz * a.outer[c] + (int64_t)(1 + a.nz) * a.total[c]);
  info[c].gemv_exec =
      bt_gemv_rows(a.R, halves, 2 * a.outer[c], a.outer[c] + (warm ? 1 : 0));
  info[c].gemv_paper = (int64_t)a.total[c] * bt_gemv_g(a.pc, a.aw, a.m);
}

// F (float32) -> hi + lo (bfloat16 pair): entries [0, R NN) the split of the
// blocks F_k, entries [R NN, 2 R NN) the split of G_k = F_k^T.
__global__ void k_mr_split(const float* F, unsigned short* hi,
                           unsigned short* lo, size_t RNN, int n) {
  const size_t nn = (size_t)n * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * RNN;
       i += (size_t)gridDim.x * blockDim.x) {
    float v;
    if (i < RNN) {
      v = F[i];
    } else {  // G_k[r][c] = F_k[c][r]
      const size_t g = i - RNN, k = g / nn, e = g - k * nn;
      const size_t r = e / n, c = e - r * n;
      v = F[k * nn + c * n + r];
    }
    const unsigned short h = f2bf(v);
    hi[i] = h;
    lo[i] = f2bf(v - bf2f(h));
  }
}

// workgroups over the columns (64 each; the last may be partly past nrhs)
inline int cblk(const MrArgs& a) { return (a.nrhs + CPB - 1) / CPB; }

template <int NB>
hipError_t qu(const MrArgs& a, hipStream_t s) {
  const int rows = 8 * ((a.R + 7) / 8);
  hipLaunchKernelGGL((k_mr_qu<NB>), dim3(rows, cblk(a)), dim3(WG), 0, s,
                     a, a.p, a.p2);
  return hipGetLastError();
}

template <int NB, int M, bool UPD>
hipError_t post_m(const MrArgs& a, hipStream_t s) {
  constexpr size_t lds = (M >= 2 ? 6 : 2) * Lds<NB>::BLK * sizeof(unsigned short);
  // above 64 KiB of LDS the limit must be raised
  static std::atomic<uint64_t> attr{0};
  const hipError_t e = lds_limit((const void*)k_mr_post<NB, M, UPD>, lds, attr);
  if (e != hipSuccess) return e;
  const int rows = 8 * ((a.R + 7) / 8);
  hipLaunchKernelGGL((k_mr_post<NB, M, UPD>), dim3(rows, cblk(a)),
                     dim3(WG), lds, s, a);
  return hipGetLastError();
}

// z = M^{-1} r' at a = 1 (m <= 2 on this path) and the rho partials, with
// r' = r - alpha q and d += alpha p first if ``upd``.
template <int NB, bool UPD>
hipError_t post(const MrArgs& a, hipStream_t s) {
  return a.m >= 2 ? post_m<NB, 2, UPD>(a, s) : post_m<NB, 1, UPD>(a, s);
}

// The fused kernels cover the optimal splitting (a = 1) at m <= 2; every
// other preconditioner of the family takes the panel passes below.
inline bool fused(const MrArgs& a) {
  return a.pc == BT_PC_POLY && a.aw == 1.0 && a.m <= 2;
}

template <int NB>
hipError_t lin(const MrArgs& a, const float* X, double cx, const float* Y,
               double cy, const float* V, double cc, float* out, int rho,
               hipStream_t s) {
  const int rows = 8 * ((a.R + 7) / 8);
  hipLaunchKernelGGL((k_mr_lin<NB>), dim3(rows, cblk(a)), dim3(WG), 0, s, a,
                     X, (float)cx, Y, (float)cy, V, (float)cc, out, rho);
  return hipGetLastError();
}

// z = M^{-1} r (r = a.r) and the rho partials, any splitting weight a and
// order m: y0 = G r = r + a C r, then Horner's rule on sum_i al_i H^i y0,
//   t <- al_i y0 + H t  (i = m - 2 .. 0, starting from t = al_{m-1} y0),
// H t = (1 - a) C t + a C (C t): a pass u = C t, then al_i y0 + (1 - a) u
// + a C u (at a = 0 one pass, al_i y0 + C t). q, p2 and r2 are free here
// (q was used up by the update of r, p2 and r2 hold the previous p and r);
// a pass never writes a panel whose neighbour rows it reads.
template <int NB>
hipError_t precond_general(const MrArgs& a, hipStream_t s) {
  hipError_t e;
  const double aw = a.aw;
  const int m = a.m;
  const float* y0 = a.r;
  if (aw != 0.0 || m == 1) {
    float* dst = m == 1 ? a.z : a.q;
    e = lin<NB>(a, a.r, 1, nullptr, 0, aw != 0.0 ? a.r : nullptr, aw, dst,
                m == 1, s);
    if (e != hipSuccess || m == 1) return e;
    y0 = dst;
  }
  const float* t = y0;
  double ct = a.al[m - 1];  // t stands for ct times the panel t
  for (int i = m - 2, side = 0; i >= 0; --i, side ^= 1) {
    const double ai = i == 0 ? 1.0 : a.al[i];
    if (aw == 0.0) {
      // t is y0 (= r) or the panel written by the previous pass: write the
      // other temporary
      float* dst = i == 0 ? a.z : (side ? a.r2 : a.p2);
      e = lin<NB>(a, y0, ai, nullptr, 0, t, ct, dst, i == 0, s);
      t = dst;
    } else {
      // u = C t into p2, then the new t into r2 (t, if not y0, was r2: its
      // last reader is the first pass)
      float* dst = i == 0 ? a.z : a.r2;
      e = lin<NB>(a, nullptr, 0, nullptr, 0, t, ct, a.p2, 0, s);
      if (e != hipSuccess) return e;
      e = lin<NB>(a, y0, ai, a.p2, 1.0 - aw, a.p2, aw, dst, i == 0, s);
      t = dst;
    }
    if (e != hipSuccess) return e;
    ct = 1.0;
  }
  return hipSuccess;
}

// z = M^{-1} r and the rho partials at the start of a refinement step
template <int NB>
hipError_t precond_first(const MrArgs& a, hipStream_t s) {
  return fused(a) ? post<NB, false>(a, s) : precond_general<NB>(a, s);
}

// One inner iteration up to the rho partials of the new residual; swaps the
// p and r panels of ``a``.
template <int NB>
hipError_t inner_iteration(MrArgs& a, hipStream_t s) {
  hipError_t e = qu<NB>(a, s);
  if (e != hipSuccess) return e;
  std::swap(a.p, a.p2);
  hipLaunchKernelGGL((k_mr_colsum<SUM_SIGMA>), dim3(a.nrhs), dim3(256), 0, s, a);
  if (fused(a)) {
    e = post<NB, true>(a, s);
    if (e != hipSuccess) return e;
    std::swap(a.r, a.r2);
    return hipSuccess;
  }
  const int rows = 8 * ((a.R + 7) / 8);
  hipLaunchKernelGGL((k_mr_rupd<NB>), dim3(rows, cblk(a)), dim3(WG), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  std::swap(a.r, a.r2);
  return precond_general<NB>(a, s);
}

template <int NB>
int solve(const MrArgs& a0, double* r64, int max_outer, int warm,
          bt_info* info, hipStream_t s) {
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
  // x holds the initial guess on entry (warm), else the iteration starts at 0
  if (!warm) hipLaunchKernelGGL(k_mr_zero_x, dim3(grid_ew), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mr_bnorm, dim3(a.R), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_mr_init_cols, dim3(a.nrhs), dim3(256), 0, s, a, warm);
  for (int outer = 0;; ++outer) {
    if (a.dtype == BT_DT_F64)
      hipLaunchKernelGGL((k_mr_resid<NB, double>), dim3(a.R, cblk(a)),
                         dim3(256), 0, s, a, r64, outer == 0 && !warm);
    else
      hipLaunchKernelGGL((k_mr_resid<NB, float>), dim3(a.R, cblk(a)),
                         dim3(256), 0, s, a, r64, outer == 0 && !warm);
    hipLaunchKernelGGL((k_mr_colsum<SUM_RES>), dim3(a.nrhs), dim3(256), 0, s, a);
    if (!read_any(&hany)) return BT_EHIP;
    if (hany == 0 || outer >= max_outer) break;
    hipLaunchKernelGGL((k_mr_tohat<NB>), dim3(a.R, cblk(a)), dim3(256),
                       0, s, a, r64);
    if (precond_first<NB>(a, s) != hipSuccess) return BT_EHIP;
    hipLaunchKernelGGL((k_mr_colsum<SUM_RHO>), dim3(a.nrhs), dim3(256), 0, s, a);
    for (int it = 0;; ++it) {
      if ((it & 7) == 7) {
        if (!read_any(&hany)) return BT_EHIP;
        if (hany == 0) break;
      }
      if (inner_iteration<NB>(a, s) != hipSuccess) return BT_EHIP;
      hipLaunchKernelGGL((k_mr_colsum<SUM_RHO>), dim3(a.nrhs), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL((k_mr_xupd<NB>), dim3(a.R, cblk(a)), dim3(256),
                       0, s, a);
    hipLaunchKernelGGL(k_mr_outer_done, dim3((a.nrhs + 63) / 64), dim3(64), 0,
                       s, a);
  }
  hipLaunchKernelGGL(k_mr_info, dim3((a.nrhs + 63) / 64), dim3(64), 0, s, a,
                     info, warm);
  return hipGetLastError() == hipSuccess ? BT_OK : BT_EHIP;
}

}  // namespace btm

// Bytes of scratch for a multi-RHS solve: seven float32 panels, the float64
// residual panel, per-row partial sums and per-column state.
size_t bt_mrhs_scratch_bytes(int64_t R, int n, int nrhs) {
  const size_t pn = (size_t)R * n * nrhs;
  return 7 * pn * sizeof(float) + pn * sizeof(double) +
         (size_t)R * nrhs * sizeof(double) + 6 * (size_t)nrhs * sizeof(double) +
         8 * (size_t)nrhs * sizeof(int) + 256;
}

hipError_t bt_mrhs_split(const float* F, unsigned short* hi, unsigned short* lo,
                         int64_t R, int n, hipStream_t s) {
  const size_t RNN = (size_t)R * n * n;
  const int grid = (int)std::min<size_t>((2 * RNN + 255) / 256, 4096);
  hipLaunchKernelGGL(btm::k_mr_split, dim3(grid), dim3(256), 0, s, F, hi, lo,
                     RNN, n);
  return hipGetLastError();
}

int bt_mrhs_run(int64_t R, int n, int nrhs, const unsigned short* Fhi,
                const unsigned short* Flo, const float* Li, const void* D,
                const void* O, int dtype, const double* b, double* x,
                double tol, int maxit, int max_outer, double inner_tol,
                int pc, double aw, int m, const double* alpha, int warm,
                void* scratch, bt_info* info, hipStream_t s) {
  btm::MrArgs a{};
  a.R = (int)R;
  a.n = n;
  a.nrhs = nrhs;
  a.Fhi = Fhi;
  a.Flo = Flo;
  a.Ghi = Fhi + (size_t)R * n * n;
  a.Glo = Flo + (size_t)R * n * n;
  a.Li = Li;
  a.D = D;
  a.O = O;
  a.dtype = dtype;
  a.b = b;
  a.x = x;
  a.tol = tol;
  a.itol2 = inner_tol * inner_tol;
  a.maxit = maxit;
  a.pc = pc;
  a.aw = aw;
  a.m = m;
  a.al[0] = 1.0;
  for (int i = 1; i < BT_MAX_M; ++i) a.al[i] = i < m ? alpha[i] : 0.0;
  a.alpha1 = a.al[1];
  a.nz = (aw != 0.0 ? 1 : 0) + (m - 1) * (aw == 0.0 ? 1 : 2);
  const size_t pn = (size_t)R * n * nrhs;
  unsigned char* w = (unsigned char*)scratch;
  float* f = (float*)w;
  a.p = f;
  a.q = f + pn;
  a.r = f + 2 * pn;
  a.d = f + 3 * pn;
  a.z = f + 4 * pn;
  a.p2 = f + 5 * pn;
  a.r2 = f + 6 * pn;
  double* r64 = (double*)(f + 7 * pn);
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
  if (n == 48) return btm::solve<48>(a, r64, max_outer, warm, info, s);
  if (n == 32) return btm::solve<32>(a, r64, max_outer, warm, info, s);
  if (n == 16) return btm::solve<16>(a, r64, max_outer, warm, info, s);
  if (n == 64) return btm::solve<64>(a, r64, max_outer, warm, info, s);
  return BT_EINVAL;
}
