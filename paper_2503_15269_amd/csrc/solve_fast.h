// Register-resident PCG kernel for small block sizes (float32 inner PCG in
// float64 iterative refinement).
//
// Same method and coordinates as the generic kernel (solve.hip): the
// iteration runs on Ahat = L^{-1} A L^{-T} = I - C with the scaled
// off-diagonal blocks F_k = L_k^{-1} O_k L_{k+1}^{-T},
//   (C v)_k = -(F_{k-1}^T v_{k-1} + F_k v_{k+1}),
// and the preconditioner of eq. Mminv-polynomial-coefficients is the
// polynomial  sum_i alpha_i ((1-a) C + a C^2)^i (I + a C),  evaluated as
// y_0 = G r, y_i = H y_{i-1}, z = sum alpha_i y_i.
//
// Layout on the chip. A workgroup owns a "bin" of systems whose block rows
// (each system padded to a whole wavefront of rows) total at most RPB (256
// rows for NB = 12, 128 for NB = 24). TPR = NB / EPT neighbouring lanes share
// a block row k; lane q owns entries EPT q .. EPT q + EPT - 1 of every vector
// row and keeps the same rows of F_k in registers (EPT * NB floats), read
// from memory once per bin. EPT (3, 6 or 12 entries per lane) trades lanes
// for registers: the workgroup has RPB * TPR threads, and fewer, wider lanes
// spend fewer instructions on shuffles and reductions per entry but hide
// less latency; the autotuner picks. One application of C then needs, per
// lane:
//   * the forward product F_k v_{k+1}: its EPT rows times the next vector
//     row, read from LDS (16-byte broadcast reads);
//   * the transposed product F_{k-1}^T v_{k-1}: the lanes of row k-1 form
//     partial sums over their own rows for all NB columns (own vector
//     entries, no LDS), reduce-scatter them inside the row with DPP moves
//     (for eight lanes the half-row mirror, partner q xor 7, first; then the
//     quad permutations xor 2 and xor 1), and hand the EPT finished sums of
//     lane q to lane q of row k through LDS.
// The column order of the F registers is permuted per lane (chunk c of lane q
// holds columns EPT (c xor q) .. +EPT-1) so that the reduce-scatter needs no
// selects. In LDS a vector row is stored in 16-byte slots of 3 entries
// (entry j at 4 (j / 3) + j % 3). Systems start on a segment boundary, a
// segment being the 16 lanes of a DPP row at n = 12 (16 / TPR block rows)
// and a wavefront at n = 24, so every per-system quantity (scalars,
// convergence masks) is uniform within a segment; a system is padded to
// whole segments (on the ragged batch at n = 12, EPT = 6: 2.6 % padding rows
// instead of the 11 % of whole wavefronts). Reductions are a DPP sum over
// each segment, one partial per segment in LDS, and a fixed-order sum over
// the system's segments that every row of the system forms alike; a
// converged system stops updating while the
// others in its bin go on. F is zero for the last row of a system, so systems
// sharing a bin, or a wavefront, do not couple.
// (kernel and launch templates; instantiated by solve_fast.hip for n = 12
// and solve_fast24.hip for n = 24, which are built with different
// instruction-scheduling strategies)
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "reduce.h"

namespace btf {

using btk::AccD;
using btk::AccX;

constexpr int SL = 4;      // reduction slots (reuse distance)
constexpr int MAXI = 64;   // systems per bin, upper bound
constexpr int MAXS = 64;   // segments per workgroup, upper bound

template <int NB, int EPT>
struct Geo {
  static constexpr int TPR = NB / EPT;            // lanes per block row
  // Systems are aligned to segments of SEG lanes: a DPP row at n = 12 (less
  // padding on ragged batches), a wavefront at n = 24 (per-system values stay
  // in scalar registers, which the larger F needs).
  static constexpr int SEG = NB == 12 ? 16 : 64;
  static constexpr int RPS = SEG / TPR;           // block rows per segment
  static constexpr int RPB = NB == 12 ? 256 : 128;  // block rows per bin
  static constexpr int NT = RPB * TPR;            // threads per workgroup
  static constexpr int NW = NT / 64;              // wavefronts
  static constexpr int NSEG = NT / SEG;           // segments
  static constexpr int SUB = EPT / 3;             // 16-byte slots per lane
  static constexpr int ROW = NB / 3 * 4;          // floats per staged row
  static_assert(NB % EPT == 0 && EPT % 3 == 0, "EPT divides NB, 3 | EPT");
  static_assert(TPR == 1 || TPR == 2 || TPR == 4 || TPR == 8,
                "1, 2, 4 or 8 lanes per block row");
  static_assert(NSEG <= MAXS && (SEG == 64 ? NSEG <= 16 : NSEG % 16 == 0),
                "segment slots: 16-lane rows read them 16 at a time");
};


template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// wave-uniform values into scalar registers
__device__ __forceinline__ int uni(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ double uni(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(u & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned int)lo);
}

// One block row of NB entries from a 16-byte aligned address (16-byte
// loads).
template <int NB, typename T>
__device__ __forceinline__ void load_row(const T* src, T (&v)[NB]) {
  if constexpr (sizeof(T) == 4) {
    static_assert(NB % 4 == 0, "whole 16-byte chunks");
#pragma unroll
    for (int c = 0; c < NB / 4; ++c) {
      const float4 t = reinterpret_cast<const float4*>(src)[c];
      v[4 * c] = t.x;
      v[4 * c + 1] = t.y;
      v[4 * c + 2] = t.z;
      v[4 * c + 3] = t.w;
    }
  } else {
    static_assert(NB % 2 == 0, "whole 16-byte chunks");
#pragma unroll
    for (int c = 0; c < NB / 2; ++c) {
      const double2 t = reinterpret_cast<const double2*>(src)[c];
      v[2 * c] = t.x;
      v[2 * c + 1] = t.y;
    }
  }
}

template <int NB, int EPT>
struct Smem {
  using G = Geo<NB, EPT>;
  float V[2][G::RPB * G::ROW];  // staged vector rows
  float T[2][G::RPB * G::ROW];  // transposed sums for row k+1
  float Z[G::ROW];              // zeros: the "previous row" of a first row
  double xs[G::RPB * NB];       // float64 iterate of the bin
  AccX redF[SL][MAXS];   // per-segment partials
  double redD[SL][MAXS];
  int active;   // running count of (wavefront, flag) events, never reset
  int bin;
  int cnt;
  int inst[MAXI];
  int lstart[MAXI];
  int nrows[MAXI];
};

template <int NB, int EPT>
struct Ctx {
  using G = Geo<NB, EPT>;
  Smem<NB, EPT>& sm;
  int lrow, q, seg;  // block row in the bin, lane in the row, segment
  int s0, s1;        // the system's segments (an idle lane: its own)
  int k, N;          // row within the system, system length (0: idle lane)
  bool row_ok;       // a real block row (not padding, not idle)
  int sf, sd, seen;
  // what the system executed: halves of applications of C, triangular
  // transforms, float64 residuals (uniform over the system's lanes)
  int nh, ntr, nrs;
  float Fr[EPT][NB]; // own rows of F_k, columns in lane order

  __device__ Ctx(Smem<NB, EPT>& s) : sm(s) {}

  // Float offset of 16-byte chunk ``ch`` of staged row ``row``. At n = 12
  // with two lanes per row, a quarter-wavefront's 16-byte accesses cover 8
  // rows of 64 bytes, two chunks each, and rows r and r + 4 would meet in the
  // same banks; rows 4..7 of every 8 swap their chunk pairs (ch xor 1), so
  // the 16 accesses tile all 64 banks.
  static constexpr bool SWZ = NB == 12 && G::TPR == 2;
  __device__ __forceinline__ static int slot(int row, int ch) {
    return row * G::ROW + 4 * (ch ^ (SWZ ? (row >> 2) & 1 : 0));
  }

  // A 16-byte chunk from LDS, of which three entries are used. In the
  // two-lane layout the fourth is kept alive so the read stays
  // ds_read_b128: the compiler would narrow it to a 12-byte read, whose
  // accesses meet in the banks (about twice the conflict cycles, measured);
  // elsewhere the narrow read costs no conflicts and fewer registers.
  __device__ __forceinline__ static float4 ld16(const float* p) {
    const float4 u = *reinterpret_cast<const float4*>(p);
    if constexpr (SWZ) asm volatile("" ::"v"(u.w));
    return u;
  }

  // own entries into staged row ``row`` of ``base`` (SUB 16-byte slots)
  __device__ __forceinline__ void put(float* base, int row,
                                      const float (&v)[EPT]) const {
#pragma unroll
    for (int h = 0; h < G::SUB; ++h)
      *reinterpret_cast<float4*>(base + slot(row, G::SUB * q + h)) =
          make_float4(v[3 * h], v[3 * h + 1], v[3 * h + 2], 0.f);
  }

  __device__ __forceinline__ int col(int x) const {  // lane-order column
    return EPT * ((x / EPT) ^ q) + x % EPT;
  }

  // Sum partial column sums P (lane column order, one per column of the
  // row's block) over the TPR lanes of the row; lane q receives the sums of
  // its own columns EPT q .. EPT q + EPT - 1. Every lane must take part.
  template <typename T>
  __device__ __forceinline__ void rscatter(const T (&P)[NB], T (&S)[EPT]) const {
    static_assert(G::TPR <= 4, "1, 2 or 4 lanes per block row");
    if constexpr (G::TPR == 4) {
      T K[2 * EPT];
#pragma unroll
      for (int y = 0; y < 2 * EPT; ++y)
        K[y] = P[y] + btk::dpp<btk::DPP_QUAD_2301>(P[2 * EPT + y]);
#pragma unroll
      for (int z = 0; z < EPT; ++z)
        S[z] = K[z] + btk::dpp<btk::DPP_QUAD_1032>(K[EPT + z]);
    } else if constexpr (G::TPR == 2) {
#pragma unroll
      for (int z = 0; z < EPT; ++z)
        S[z] = P[z] + btk::dpp<btk::DPP_QUAD_1032>(P[EPT + z]);
    } else {
#pragma unroll
      for (int z = 0; z < EPT; ++z) S[z] = P[z];
    }
  }

  // Natural column order -> lane column order (chunk cc of EPT entries
  // takes natural chunk cc xor q), one bit of q at a time with selects; the
  // map is its own inverse.
  template <typename T>
  __device__ __forceinline__ void to_lane_order(T (&v)[NB]) const {
    if constexpr (G::TPR >= 2) {
      const bool b0 = (q & 1) != 0;
#pragma unroll
      for (int cc = 0; cc < G::TPR; cc += 2)
#pragma unroll
        for (int z = 0; z < EPT; ++z) {
          const T u = v[EPT * cc + z], w = v[EPT * (cc + 1) + z];
          v[EPT * cc + z] = b0 ? w : u;
          v[EPT * (cc + 1) + z] = b0 ? u : w;
        }
    }
    if constexpr (G::TPR >= 4) {
      const bool b1 = (q & 2) != 0;
#pragma unroll
      for (int cc = 0; cc < G::TPR; cc += 4)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int z = 0; z < EPT; ++z) {
            const T u = v[EPT * (cc + h) + z], w = v[EPT * (cc + h + 2) + z];
            v[EPT * (cc + h) + z] = b1 ? w : u;
            v[EPT * (cc + h + 2) + z] = b1 ? u : w;
          }
    }
    static_assert(G::TPR <= 4, "1, 2 or 4 lanes per block row");
  }

  // Own rows EPT q .. EPT q + EPT - 1 of F_k into registers, lane column
  // order (zero for the last row of a system, which has no F_k): 16-byte
  // loads of the contiguous rows, then the chunk permutation.
  __device__ __forceinline__ void load_F(const float* F, int64_t g) {
    const bool has_next = row_ok && k < N - 1;
    const float keep = has_next ? 1.f : 0.f;
    const float* fk = F + (size_t)(has_next ? g : 0) * NB * NB +
                      (size_t)q * EPT * NB;  // always valid
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      load_row(fk + e * NB, Fr[e]);
#pragma unroll
      for (int x = 0; x < NB; ++x) Fr[e][x] *= keep;
      to_lane_order(Fr[e]);
    }
  }

  // Own rows i = EPT q + e of L_k^{-1} (natural column order, zero above the
  // diagonal), from the full blocks or the packed lower triangles. A packed
  // row is read as NB consecutive entries from its start (past its end they
  // belong to the next rows or the padding of the same block) and masked.
  template <bool PK>
  __device__ __forceinline__ void load_li_rows(const float* Li, int64_t g,
                                               float (&Lv)[EPT][NB]) const {
    constexpr size_t LP = li_packed_len(NB);
    if constexpr (PK) {
      const int i0 = q * EPT;
      const float* base = Li + (size_t)g * LP + (size_t)(i0 * (i0 + 1) / 2);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const float* row = base + e * i0 + e * (e + 1) / 2;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const float v = row[j];
          Lv[e][j] = j <= i0 + e ? v : 0.f;
        }
      }
    } else {
      const float* base = Li + (size_t)g * NB * NB + (size_t)q * EPT * NB;
#pragma unroll
      for (int e = 0; e < EPT; ++e) load_row(base + e * NB, Lv[e]);
    }
  }

  // ---- one application of C in two halves around a barrier -------------
  // partial sum of the transposed product for lane-order column x: own rows
  // of F_k times own entries of v
  __device__ __forceinline__ float tprod(int x, const float (&v)[EPT]) const {
    float s = Fr[0][x] * v[0];
#pragma unroll
    for (int e = 1; e < EPT; ++e) s = __fmaf_rn(Fr[e][x], v[e], s);
    return s;
  }

  template <int BUF>
  __device__ __forceinline__ void prep(const float (&v)[EPT]) {
    ++nh;
    float S[EPT];
    if constexpr (G::TPR == 8) {
      // Partner q xor 7 (mirror inside the 8-lane half row), then xor 2, then
      // xor 1. The upper half of the partial sums is formed first and each
      // lower slot is folded in as soon as it is formed, which keeps at most
      // 5 of the 8 column chunks live.
      float Ph[4 * EPT], K1[4 * EPT], K[2 * EPT];
#pragma unroll
      for (int y = 0; y < 4 * EPT; ++y) Ph[y] = tprod(4 * EPT + y, v);
#pragma unroll
      for (int y = 0; y < 4 * EPT; ++y)
        K1[y] = tprod(y, v) + dpp<btk::DPP_ROW_HALF_MIRROR>(
                                  Ph[EPT * (3 - y / EPT) + y % EPT]);
#pragma unroll
      for (int y = 0; y < 2 * EPT; ++y)
        K[y] = K1[y] + dpp<btk::DPP_QUAD_2301>(K1[2 * EPT + y]);
#pragma unroll
      for (int z = 0; z < EPT; ++z)
        S[z] = K[z] + dpp<btk::DPP_QUAD_1032>(K[EPT + z]);
    } else if constexpr (G::TPR == 4) {
      float P[NB];
#pragma unroll
      for (int x = 0; x < NB; ++x) P[x] = tprod(x, v);
      float K[2 * EPT];
#pragma unroll
      for (int y = 0; y < 2 * EPT; ++y)
        K[y] = P[y] + dpp<btk::DPP_QUAD_2301>(P[2 * EPT + y]);
#pragma unroll
      for (int z = 0; z < EPT; ++z)
        S[z] = K[z] + dpp<btk::DPP_QUAD_1032>(K[EPT + z]);
    } else if constexpr (G::TPR == 2) {
      float P[NB];
#pragma unroll
      for (int x = 0; x < NB; ++x) P[x] = tprod(x, v);
#pragma unroll
      for (int z = 0; z < EPT; ++z)
        S[z] = P[z] + dpp<btk::DPP_QUAD_1032>(P[EPT + z]);
    } else {
#pragma unroll
      for (int z = 0; z < EPT; ++z) S[z] = tprod(z, v);
    }
    put(sm.V[BUF], lrow, v);
    put(sm.T[BUF], lrow, S);
  }

  template <int BUF>
  __device__ __forceinline__ void finish(float (&y)[EPT]) {
    ++nh;
    const int rp = k < N - 1 ? lrow + 1 : lrow;
    float acc[EPT];
    {
#pragma unroll
      for (int h = 0; h < G::SUB; ++h) {
        const float* tr = k > 0 ? sm.T[BUF] + slot(lrow - 1, G::SUB * q + h)
                                : sm.Z + 4 * (G::SUB * q + h);
        const float4 u = ld16(tr);
        acc[3 * h] = u.x;
        acc[3 * h + 1] = u.y;
        acc[3 * h + 2] = u.z;
      }
    }
#pragma unroll
    for (int c = 0; c < G::TPR; ++c) {
#pragma unroll
      for (int h = 0; h < G::SUB; ++h) {
        const float4 u = ld16(sm.V[BUF] + slot(rp, G::SUB * (c ^ q) + h));
        const float uc[3] = {u.x, u.y, u.z};
#pragma unroll
        for (int e = 0; e < EPT; ++e)
#pragma unroll
          for (int z = 0; z < 3; ++z)
            acc[e] = __fmaf_rn(Fr[e][EPT * c + 3 * h + z], uc[z], acc[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) y[e] = -acc[e];
  }

  // ``on``: this lane's system still iterates (uniform over its segment); the
  // barrier is always taken, the arithmetic only when needed.
  template <int BUF>
  __device__ __forceinline__ void C(const float (&v)[EPT], float (&y)[EPT],
                                    bool on = true) {
    if (on) prep<BUF>(v);
    __syncthreads();
    if (on) finish<BUF>(y);
  }

  // ---- reductions --------------------------------------------------------
  // Every value below is uniform over a segment, and the sums over a system
  // are bitwise equal in all of its lanes.
  template <typename A>
  __device__ __forceinline__ static A seg_sum(A v) {
    if constexpr (G::SEG == 64) return btk::wave_sum(v);
    else return btk::row16_sum(v);
  }
  // a segment-uniform value; whole-wavefront segments keep it in scalar
  // registers
  template <typename V>
  __device__ __forceinline__ static V seg_uni(V v) {
    if constexpr (G::SEG == 64) return uni(v);
    else return v;
  }
  __device__ __forceinline__ void put_seg(const AccX& acc) {
    const AccX t = seg_sum(acc);
    if ((threadIdx.x & (G::SEG - 1)) == 0) sm.redF[sf][seg] = t;
  }
  // Sum of the system's segment partials: lane l of each DPP row adds slots
  // l, l + 16, .. that lie in [s0, s1) in that order, and the row's
  // butterfly adds the 16 (a fixed tree: deterministic, and the same in
  // every row of the system).
  __device__ __forceinline__ double take() {  // after the barrier
    const int l = threadIdx.x & 15;
    AccX v;
    v.zero();
#pragma unroll
    for (int i = 0; i < G::NSEG; i += 16) {
      const AccX u = sm.redF[sf][l + i];
      if (l + i >= s0 && l + i < s1) v.merge(u);
    }
    v = btk::row16_sum(v);
    sf = (sf + 1) % SL;
    return seg_uni(v.value());
  }
  __device__ __forceinline__ double take_if(bool on) {  // after the barrier
    if (on) return take();
    sf = (sf + 1) % SL;  // keep the slot rotation in step with the others
    return 0.0;
  }
  __device__ __forceinline__ double dot(const float (&x)[EPT],
                                        const float (&y)[EPT], bool on = true) {
    if (on) {
      AccX acc;
      acc.zero();
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc.add_prod(x[e], y[e]);
      put_seg(acc);
    }
    __syncthreads();
    return take_if(on);
  }
  __device__ __forceinline__ double sumd(double v) {
    AccD a;
    a.s = v;
    const AccD t = seg_sum(a);
    if ((threadIdx.x & (G::SEG - 1)) == 0) sm.redD[sd][seg] = t.s;
    __syncthreads();
    const int l = threadIdx.x & 15;
    AccD u;
    u.zero();
#pragma unroll
    for (int i = 0; i < G::NSEG; i += 16) {
      const double w = sm.redD[sd][l + i];
      if (l + i >= s0 && l + i < s1) u.s += w;
    }
    u = btk::row16_sum(u);
    sd = (sd + 1) % SL;
    return seg_uni(u.s);
  }
  // Any wavefront that raised its flag since the last check bumped the
  // counter; every lane compares with the value it saw last time. The next
  // bump happens only after a further barrier, so all lanes read the same.
  __device__ __forceinline__ bool any_after_barrier() {
    const int now = uni(sm.active);
    const bool any = now != seen;
    seen = now;
    return any;
  }
  __device__ __forceinline__ void put_flag(bool f) {  // every lane calls
    const bool any = __builtin_amdgcn_ballot_w64(f) != 0;
    if ((threadIdx.x & 63) == 0 && any) atomicAdd(&sm.active, 1);
  }

  // z = M^{-1} r at the optimal weights (a, b) = (1, -1), in the scaled
  // coordinates: G = I + C, H = C^2, so y_0 = r + C r, y_i = C (C y_{i-1}),
  // z = y_0 + sum_i alpha_i y_i. C(r) is applied by the caller (fused with a
  // reduction) and passed in as ``cr``.
  template <int M>
  __device__ __forceinline__ void precond_rest(const SolveArgs& a,
                                               const float (&r)[EPT],
                                               const float (&cr)[EPT],
                                               float (&z)[EPT],
                                               bool on = true) {
    float y[EPT], w[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      y[e] = r[e] + cr[e];
      z[e] = y[e];
    }
#pragma unroll
    for (int m = 1; m < M; ++m) {
      C<0>(y, w, on);
      C<1>(w, y, on);
      const float al = (float)a.alpha[m];
#pragma unroll
      for (int e = 0; e < EPT; ++e) z[e] = __fmaf_rn(al, y[e], z[e]);
    }
  }
};

template <int NB, int EPT, int M, typename Rec, bool PK>
__global__ void __launch_bounds__((Geo<NB, EPT>::NT)) k_fast_ir(SolveArgs a) {
  using G = Geo<NB, EPT>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Smem<NB, EPT>& sm = *reinterpret_cast<Smem<NB, EPT>*>(smem_raw);
  Ctx<NB, EPT> c(sm);
  const int t = threadIdx.x;
  c.lrow = t / G::TPR;
  c.q = t % G::TPR;
  c.seg = c.seg_uni(t / G::SEG);  // scalar for whole-wavefront segments
  c.sf = 0;
  c.sd = 0;
  if (t == 0) sm.active = 0;
  if (t < G::ROW) sm.Z[t] = 0.f;
  __syncthreads();
  c.seen = 0;
  const size_t nn = (size_t)NB * NB;
  constexpr size_t LP = li_packed_len(NB);  // packed L_k^{-1} entries
  const double itol2 = uni(a.inner_tol * a.inner_tol);  // scalar registers
  const float* F = (const float*)a.F;
  // L^{-1}: packed lower triangles (PK) or full blocks
  const float* Li = (const float*)(PK ? a.Lp : a.Li);

  for (;;) {
    if (t == 0) sm.bin = atomicAdd(&a.ctr[2], 1);
    __syncthreads();
    const int bin = sm.bin;
    if (bin >= a.nbins) break;
    if (t == 0) {
      const int start = a.bins[2 * bin], cnt = a.bins[2 * bin + 1];
      int at = 0;
      for (int j = 0; j < cnt; ++j) {
        const int id = a.bin_items[start + j];
        const int Nj = (int)(a.off[id + 1] - a.off[id]);
        sm.inst[j] = id;
        sm.lstart[j] = at;
        sm.nrows[j] = Nj;
        at += (Nj + G::RPS - 1) / G::RPS * G::RPS;
      }
      sm.cnt = cnt;
    }
    __syncthreads();

    // ---- geometry of this lane ------------------------------------------
    int j = -1;
    for (int jj = 0; jj < sm.cnt; ++jj) {
      const int ls = sm.lstart[jj];
      const int pad = (sm.nrows[jj] + G::RPS - 1) / G::RPS * G::RPS;
      if (c.lrow >= ls && c.lrow < ls + pad) j = jj;
    }
    const bool sys = j >= 0;  // uniform within the segment
    int inst = 0;
    bool lead = false;
    if (sys) {
      const int ls = sm.lstart[j];
      const int pad = (sm.nrows[j] + G::RPS - 1) / G::RPS * G::RPS;
      c.N = sm.nrows[j];
      c.k = c.lrow - ls;
      inst = sm.inst[j];
      c.s0 = ls / G::RPS;
      c.s1 = (ls + pad) / G::RPS;
      lead = (c.k == 0 && c.q == 0);
    } else {
      c.N = 0;
      c.k = 0;
      c.s0 = c.seg;
      c.s1 = c.seg + 1;
    }
    c.N = c.seg_uni(c.N);
    c.s0 = c.seg_uni(c.s0);
    c.s1 = c.seg_uni(c.s1);
    c.row_ok = sys && c.k < c.N;
    const int64_t g = sys ? a.off[inst] + c.k : 0;  // global block row
    const int64_t ob = g - inst;                     // its upper block

    // ---- per-system state ----------------------------------------------
    const int fail = sys ? a.fail[inst] : BT_NO_FAIL;
    const int e0 = c.q * EPT;
    double nbp = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const double bv = c.row_ok ? a.b[g * NB + e0 + e] : 0.0;
      nbp += bv * bv;
      sm.xs[c.lrow * NB + e0 + e] = 0.0;
    }
    const double nb2 = c.sumd(nbp);
    int status = BT_NOT_CONVERGED;
    bool done = !sys;
    if (sys && fail != BT_NO_FAIL) {
      status = BT_ENOTSPD;
      done = true;
    } else if (sys && !(nb2 < INFINITY)) {
      status = BT_ENONFINITE;
      done = true;
    } else if (sys && nb2 == 0.0) {
      status = BT_OK;
      done = true;
    }
    const double tol2 = a.tol * a.tol * nb2;
    int outer = 0, total = 0;
    double nr2 = nb2;
    double nr2_prev = INFINITY;  // before the last correction
    double unscale = 1.0;  // 1 / the scale of the current inner solve
    c.nh = 0;
    c.ntr = 0;
    c.nrs = 0;
    if (a.warm) {  // initial guess x0 (held in x on entry) of running systems
      if (!done && c.row_ok) {
#pragma unroll
        for (int e = 0; e < EPT; ++e)
          sm.xs[c.lrow * NB + e0 + e] = a.x[g * NB + e0 + e];
      }
      __syncthreads();  // neighbour rows of xs are read by the residual
    }

    // Refinement loop. F_k lives in registers only during an inner solve;
    // the residual and the two transforms in between use those registers to
    // issue all of a lane's loads at once (wide, row-contiguous), and the
    // transposed products O_k^T x_k and L_k^{-T} d are formed as partial
    // column sums over the lane's own rows, summed across the row's lanes
    // with DPP (the hand-off that F_k^T uses).
    float d[EPT];   // correction of the last inner solve (scaled coordinates)
    bool ran = false;  // an inner solve ran since the last correction
#pragma unroll
    for (int e = 0; e < EPT; ++e) d[e] = 0.f;
    const Rec* Dg = (const Rec*)a.D + (size_t)g * nn + (size_t)e0 * NB;
    const bool has_next = c.row_ok && c.k < c.N - 1;
    for (;;) {
      // ---- x64 += L^{-T} d (undoing the scale) ------------------------
      {
        float P[NB];  // column sums over the lane's rows, natural order
#pragma unroll
        for (int x = 0; x < NB; ++x) P[x] = 0.f;
        if (ran && c.row_ok) {
          float Lv[EPT][NB];
          c.template load_li_rows<PK>(Li, g, Lv);
#pragma unroll
          for (int e = 0; e < EPT; ++e)
#pragma unroll
            for (int j = 0; j < NB; ++j) P[j] = __fmaf_rn(Lv[e][j], d[e], P[j]);
        }
        c.to_lane_order(P);
        float S[EPT];
        c.rscatter(P, S);
        if (ran) {
          if (c.row_ok) {
#pragma unroll
            for (int e = 0; e < EPT; ++e)
              sm.xs[c.lrow * NB + e0 + e] += (double)S[e] * unscale;
          }
          ++c.ntr;
          ++outer;
          ran = false;
        }
        __syncthreads();  // xs complete before the residual reads it
      }

      // ---- float64 residual of the record, scaled by a power of two to
      // norm in [1, 2) before the float32 inner solve ----------------------
      float r64f[EPT];
      {
        const bool need = !done && (outer > 0 || a.warm);  // segment-uniform
        const double* xk = sm.xs + c.lrow * NB;
        double acc[EPT];
        double P[NB];  // column sums of O_k^T x_k over own rows, natural
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = 0.0;
#pragma unroll
        for (int x = 0; x < NB; ++x) P[x] = 0.0;
        if (need && c.row_ok) {
          // rows e0 .. e0 + EPT - 1 of D_k and O_k, 16-byte loads, in
          // batches of RB rows issued before their sums: enough loads in
          // flight without spilling next to the F registers (n = 12, EPT = 6:
          // two rows, 43 -> 36 spilled VGPRs and 2.5 % faster than three;
          // n = 24: one row, 286 -> 92 spilled VGPRs)
          constexpr int RB = sizeof(Rec) != 4 || NB > 12 ? 1
                             : EPT % 2 == 0             ? 2
                                                        : 3;
          static_assert(EPT % RB == 0, "whole batches");
          const double* xn = sm.xs + (c.lrow + 1) * NB;
#pragma unroll
          for (int e1 = 0; e1 < EPT; e1 += RB) {
            Rec Dv[RB][NB], Ov[RB][NB];
#pragma unroll
            for (int e = 0; e < RB; ++e) load_row(Dg + (e1 + e) * NB, Dv[e]);
            if (has_next) {
              const Rec* Og = (const Rec*)a.O + (size_t)ob * nn + (size_t)e0 * NB;
#pragma unroll
              for (int e = 0; e < RB; ++e) load_row(Og + (e1 + e) * NB, Ov[e]);
            }
#pragma unroll
            for (int e = 0; e < RB; ++e)
#pragma unroll
              for (int j = 0; j < NB; ++j)
                acc[e1 + e] += (double)Dv[e][j] * xk[j];
            if (has_next) {
#pragma unroll
              for (int e = 0; e < RB; ++e) {
                const double xo = xk[e0 + e1 + e];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                  const double o = (double)Ov[e][j];
                  acc[e1 + e] += o * xn[j];
                  P[j] += o * xo;
                }
              }
            }
          }
        }
        // O_k^T x_k to the lanes of row k + 1 (float64 through the T area)
        double* Td = reinterpret_cast<double*>(&sm.T[0][0]);
        {
          c.to_lane_order(P);
          double S[EPT];
          c.rscatter(P, S);
#pragma unroll
          for (int e = 0; e < EPT; ++e) Td[c.lrow * NB + e0 + e] = S[e];
        }
        __syncthreads();
        double rp = 0.0;
        double r64v[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          double r64 = 0.0;
          if (c.row_ok && !done) {
            const double bv = a.b[g * NB + e0 + e];
            if (need) {
              const double up = c.k > 0 ? Td[(c.lrow - 1) * NB + e0 + e] : 0.0;
              r64 = bv - (acc[e] + up);
            } else {
              r64 = bv;  // x = 0
            }
          }
          rp += r64 * r64;
          r64v[e] = r64;
        }
        const double s = c.sumd(rp);
        if (need) {
          nr2 = s;
          ++c.nrs;
        }
        const double sc = bt_unit_scale(nr2);
        unscale = 1.0 / sc;
#pragma unroll
        for (int e = 0; e < EPT; ++e) r64f[e] = (float)(r64v[e] * sc);
      }
      if (!done) {
        if (nr2 <= tol2) {
          status = BT_OK;
          done = true;
        } else if (!(nr2 < INFINITY)) {
          status = BT_ENONFINITE;
          done = true;
        } else if (outer > 0 && nr2 > 0.25 * nr2_prev) {
          // the correction cut the float64 residual by less than 2x
          status = BT_ESTAGNATED;
          done = true;
        } else if (outer >= a.max_outer || total >= a.maxit) {
          done = true;
        }
        nr2_prev = nr2;
      }

      // ---- inner system  Ahat d = L^{-1} r64  for the systems still running
      float r[EPT], p[EPT], z[EPT], qv[EPT];
      {
        c.put(sm.V[0], c.lrow, r64f);
        c.put_flag(!done);
        __syncthreads();
        if (!c.any_after_barrier()) break;  // every system of the bin is done
        if (!done) ++c.ntr;
        const float* rk = sm.V[0];
        float Lv[EPT][NB];
        if (c.row_ok && !done) {
          c.template load_li_rows<PK>(Li, g, Lv);
        } else {
#pragma unroll
          for (int e = 0; e < EPT; ++e)
#pragma unroll
            for (int j = 0; j < NB; ++j) Lv[e][j] = 0.f;
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < NB; ++j)
            acc = __fmaf_rn(Lv[e][j], rk[c.slot(c.lrow, j / 3) + j % 3], acc);
          r[e] = acc;
          d[e] = 0.f;
        }
      }
      c.load_F(F, g);  // F_k for this inner solve
      // z = M^{-1} r for the inner right-hand side
      {
        float cr[EPT];
        c.template C<1>(r, cr, !done);
        c.template precond_rest<M>(a, r, cr, z, !done);
      }
      // Inner PCG, arranged so that each iteration has two reductions and
      // five barriers: rho = r'z shares its barrier with the staging of z,
      // q = Ahat p follows from Ahat z by q = Ahat z + beta q, and the inner
      // solve stops when r'z (the squared residual in the M^{-1} norm) fell
      // by inner_tol^2.
      bool act = !done;
      bool first = true;
      double rho = 0.0, rho0 = 0.0;
      int inner = 0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {  // beta = 0 at the first step: p = z
        p[e] = 0.f;
        qv[e] = 0.f;
      }
      for (;;) {
        // a system that has stopped keeps taking the barriers (with its
        // bin) but no longer does arithmetic
        if (act) {
          AccX acc;
          acc.zero();
#pragma unroll
          for (int e = 0; e < EPT; ++e) acc.add_prod(r[e], z[e]);
          c.template prep<0>(z);
          c.put_seg(acc);
        }
        c.put_flag(act);
        __syncthreads();
        const double rho1 = c.take_if(act);
        if (!c.any_after_barrier()) break;
        if (act) {
          if (!(rho1 > 0.0)) act = false;
          else if (first) rho0 = rho1;
          else if (rho1 <= itol2 * rho0) act = false;
          if (total >= a.maxit) act = false;
        }
        float u[EPT];
        if (act) c.template finish<0>(u);
#pragma unroll
        for (int e = 0; e < EPT; ++e) u[e] = z[e] - u[e];
        if (act) {
          // the step sizes only scale float32 vectors: a float32 quotient
          // (reciprocal and product) is accurate enough
          const float be = first ? 0.f : __fdividef((float)rho1, (float)rho);
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            p[e] = __fmaf_rn(be, p[e], z[e]);
            qv[e] = __fmaf_rn(be, qv[e], u[e]);
          }
          rho = rho1;
        }
        first = false;
        const double sigma = c.dot(p, qv, act);
        if (act && !(sigma > 0.0)) act = false;
        if (act) {
          const float al = __fdividef((float)rho, (float)sigma);
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            d[e] = __fmaf_rn(al, p[e], d[e]);
            r[e] = __fmaf_rn(-al, qv[e], r[e]);
          }
          ++inner;
          ++total;
        }
        float cr[EPT];
        c.template C<1>(r, cr, act);
        c.template precond_rest<M>(a, r, cr, z, act);
      }
      if (!done) {
        ran = true;  // the correction is applied at the top of the loop
        if (inner == 0) {
          status = BT_EBREAKDOWN;
          done = true;
          ran = false;
          ++outer;
        }
      }
    }

    if (c.row_ok) {
#pragma unroll
      for (int e = 0; e < EPT; ++e)
        a.x[g * NB + e0 + e] = sm.xs[c.lrow * NB + e0 + e];
    }
    if (lead) {
      bt_info* inf = a.info + inst;
      inf->status = status;
      inf->iters = total;
      inf->outer = outer;
      inf->fail_index = status == BT_ENOTSPD ? fail : -1;
      const double rr = nb2 > 0.0 ? sqrt(nr2 / nb2) : 0.0;
      inf->relres = status == BT_ENOTSPD ? NAN : rr;
      inf->relres_true = status == BT_ENOTSPD ? NAN : rr;
      inf->gemv_exec = bt_gemv_rows(c.N, c.nh, c.ntr, c.nrs);
      inf->gemv_paper = (int64_t)total * bt_gemv_g(a.pc, a.a, a.m);
    }
    __syncthreads();
  }
  if (t == 0) {
    __threadfence();
    const int dn = atomicAdd(&a.ctr[3], 1);
    if (dn == (int)gridDim.x - 1) {
      atomicExch(&a.ctr[2], 0);
      atomicExch(&a.ctr[3], 0);
    }
  }
}

template <int NB, int EPT, int M, typename Rec, bool PK>
hipError_t launch_one(const SolveArgs& a, int grid, hipStream_t s) {
  using G = Geo<NB, EPT>;
  static std::atomic<uint64_t> attr{0};
  const hipError_t e = lds_limit((const void*)k_fast_ir<NB, EPT, M, Rec, PK>,
                                 sizeof(Smem<NB, EPT>), attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fast_ir<NB, EPT, M, Rec, PK>), dim3(grid),
                     dim3(G::NT), sizeof(Smem<NB, EPT>), s, a);
  return hipGetLastError();
}

template <int NB, int EPT, typename Rec, bool PK>
hipError_t launch_m(const SolveArgs& a, int grid, hipStream_t s) {
  switch (a.m) {
    case 1: return launch_one<NB, EPT, 1, Rec, PK>(a, grid, s);
    case 2: return launch_one<NB, EPT, 2, Rec, PK>(a, grid, s);
    case 3: return launch_one<NB, EPT, 3, Rec, PK>(a, grid, s);
    default: return launch_one<NB, EPT, 4, Rec, PK>(a, grid, s);
  }
}

// L^{-1} as full blocks or packed lower triangles
template <int NB, int EPT, typename Rec>
hipError_t launch_rec(const SolveArgs& a, int grid, hipStream_t s) {
  if constexpr (NB == 12 || NB == 24) {
    if (a.Lp) return launch_m<NB, EPT, Rec, true>(a, grid, s);
  }
  return launch_m<NB, EPT, Rec, false>(a, grid, s);
}

template <int NB, int EPT>
hipError_t launch_ept(const SolveArgs& a, int grid, hipStream_t s) {
  if (a.dtype == BT_DT_F64) return launch_rec<NB, EPT, double>(a, grid, s);
  return launch_rec<NB, EPT, float>(a, grid, s);
}

template <int NB, int EPT>
int max_grid() {
  using G = Geo<NB, EPT>;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, (const void*)k_fast_ir<NB, EPT, 2, float, false>, G::NT,
          sizeof(Smem<NB, EPT>)) != hipSuccess ||
      per < 1)
    per = 1;
  return cus * per;
}

// entries per lane of each variant (the variant index is the public one)
constexpr int kEpt[BT_FAST_VARIANTS] = {3, 6, 12};

}  // namespace btf
