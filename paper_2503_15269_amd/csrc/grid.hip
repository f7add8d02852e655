// Grid-wide PCG for one large system, in one persistent launch.
//
// The register-resident and queue kernels give each system one workgroup,
// which leaves a single long horizon (hundreds of block rows) on one CU with
// the whole iteration latency-bound there. Here the block rows of the one
// system are cut into windows of rb consecutive rows spread over the whole
// GPU, and one launch runs the complete solve: the phases below, separated
// by grid-wide barriers, with every decision (alpha, beta, stopping, the
// refinement loop) taken on the device.
//   init   r = L^{-1} f (f = b, or the float64 residual), u = M^{-1} r,
//          w = Ahat u, partials of r'u, w'u and ||f||^2
//   step   alpha, beta from the sums; p = u + beta p, s = w + beta s,
//          x += alpha p, r -= alpha s, u = M^{-1} r, w = Ahat u, partials
//          of r'u, w'u (and ||L r||^2 for the stopping test)
//   x      x = L^{-T} xhat (or x += L^{-T} d under refinement)
//   res    float64 residual b - A x of the record, ||.||^2 partials
// The step is the conjugate gradient iteration in the arrangement of
// Chronopoulos and Gear (1989): s = A p is carried by its own recurrence and
// sigma = p'A p = w'u - beta r'u / alpha_prev, so both dot products of an
// iteration come from one reduction and a step costs one grid barrier
// instead of two. In exact arithmetic its iterates are those of textbook
// PCG (the same alpha, beta, r, x); in floating point they differ by
// rounding. Same scaled
// coordinates as the other solve kernels: Ahat = I - C,
// (C v)_k = -(F_{k-1}^T v_{k-1} + F_k v_{k+1}), and the preconditioner of
// eq. Mminv-polynomial-coefficients evaluated as y_0 = (I + aC) r,
// y_i = ((1-a)C + aC^2) y_{i-1}, z = sum alpha_i y_i (Section IV-B).
//
// M^{-1} needs neighbours to a depth D (1 + 2(m-1) at a = 1) and w = Ahat u
// one more: the workgroup forms r - alpha s on its window's rows plus D + 1
// on each side in LDS and applies C there on windows that shrink by one row
// per application, so u and w of its own rows need no further exchange.
// When a workgroup keeps one window for the whole solve, the window's blocks
// F (and its own rows' L_k for ||L r||) are staged in LDS once per inner
// solve; with n <= 16 fixed at compile time and at most one window entry
// per thread, each thread also keeps the F entries of its own entry (row i
// of F_k, column i of F_{k-1}) in registers, so an application of C reads
// only the vector from LDS. The updates of y, z and w run inside the
// applications of C that produce their operands.
// Scalars never leave the device: each window writes one partial per
// reduction, and every workgroup sums all partials in the same fixed order,
// so all of them take the same decisions without a broadcast.
//
// Grid barrier: an arrival counter in the scratch, reset before the solve;
// barrier j is passed once it reaches (j + 1) times the workgroups. The data
// windows exchange is written and read with agent-coherent accesses, and
// every thread waits for its stores to complete before its workgroup
// arrives, so no cache has to be written back or invalidated. The wait is
// bounded by a wall-clock limit (checked with the abort flag on the first
// poll and every 16th): a workgroup that gives up raises an abort flag,
// every other workgroup sees it at its next wait and returns, and the solve
// reports BT_ETIMEOUT. The grid
// never exceeds the workgroups that fit on the device at once, and each
// workgroup loops over several windows when there are more windows than
// that.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>

#include "grid.h"
#include "internal.h"
#include "reduce.h"

namespace btg {

using btk::AccOf;

constexpr int NT = 256;  // threads per workgroup
// partial-sum slots, nwin doubles each: gamma = r'u, delta = w'u and
// ||L r||^2 by step parity, ||src||^2, the float64 residual, gamma of the
// first step
enum { P_G = 0, P_D = 2, P_N = 4, P_NB2 = 6, P_RES = 7, P_GF = 8,
       P_SLOTS = 9 };

// Barrier state in the scratch (reset by k_g_reset before every solve).
struct Bar {
  unsigned count;  // arrivals so far in this solve: barrier j is passed
                   // when it reaches (j + 1) * (workgroups)
  int abort;       // a workgroup gave up waiting
  int pad[2];
};

template <typename T>
struct GArgsBase {
  int R, n, rb, depth, nwin, pc, m, dtype;
  int refine, warm, from_res, max_outer, maxit;
  double a, tol, itol;
  double alpha[BT_MAX_M];
  long long spin_limit;  // wall-clock ticks (100 MHz) a barrier waits at most
  const T* F;
  const T* L;
  const T* Li;
  const void* D;  // record
  const void* O;
  const int32_t* fail;  // first failing block row of the factorisation
  const double* b;
  double* x;          // float64 iterate / solution
  double* r64;        // float64 residual
  T* rbuf[2];         // residual r, by step parity
  T* sbuf[2];         // s = A p, by step parity
  T* wbuf[2];         // w = A u, by step parity
  T* u;               // u = M^{-1} r
  T* p;               // search direction
  T* xh;              // scaled iterate (direct) or correction d (refinement)
  double* part;       // [P_SLOTS][nwin]
  Bar* bar;
  bt_info* info;
};

// The arguments with the block size fixed at compile time (NS > 0: the
// loops over a block's entries unroll completely) or read at run time.
template <typename T, int NS>
struct GArgs : GArgsBase<T> {
  __host__ __device__ __forceinline__ int nv() const {
    return NS > 0 ? NS : this->n;
  }
};

// Per-solve state that every workgroup holds identically.
struct St {
  const double* src;   // right-hand side of the next init phase
  double sscale;       // init reads src * sscale (a power of two)
  double xscale;       // x phase adds L^{-T} d * xscale
  double tol_in;       // stopping tolerance of the inner iteration
  int ir;              // inner solve of a refinement step
};

__device__ __forceinline__ double rec(const void* P, size_t i, int dtype) {
  return dtype == BT_DT_F64 ? ((const double*)P)[i]
                            : (double)((const float*)P)[i];
}

// Data that one window writes and others read (vector rows next to a
// window's own, partial sums, x for the residual) goes through agent-scope
// relaxed atomic loads and stores: coherent across the XCDs' separate L2
// caches without writing back or invalidating whole caches, so read-only
// operands (F, L, D, O) stay cached across the barriers.
template <typename V>
__device__ __forceinline__ V ld_sh(const V* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ void st_sh(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums over the workgroup of K values per thread, every thread gets them:
// the wavefront sum of the DPP tree, then the four wavefronts in a fixed
// order. Deterministic and the same in every workgroup for the same inputs.
// ``red`` holds at least 4 K doubles.
template <int K>
__device__ __forceinline__ void wg_sums(double (&v)[K], double* red) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    btk::AccD t;
    t.s = v[k];
    v[k] = btk::wave_sum(t).s;
  }
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

// Sums of K partial slots over all windows (fixed order).
template <int K>
__device__ __forceinline__ void slot_sums(const double* part,
                                          const int (&slot)[K], int nwin,
                                          double* red, double (&out)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (int i = threadIdx.x; i < nwin; i += NT) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] += ld_sh(part + slot[k] * nwin + i);
  }
  wg_sums<K>(out, red);
}

// Grid-wide barrier with a bounded wait; false once the solve is aborted.
// Every thread first waits until its shared stores have completed (they are
// agent-coherent), then one thread per workgroup adds its arrival to the
// counter (no reply needed) and waits until the counter reaches this
// barrier's target: no workgroup has to reset or release anything.
struct Sync {
  Bar* bar;
  unsigned nwg;
  unsigned target;  // arrivals that complete the next barrier (thread 0)
  long long limit;
  __device__ bool operator()(int* flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      int ok = 1;
      target += nwg;
      __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      const long long t0 = (long long)wall_clock64();
      unsigned polls = 0;
      while ((int)(__hip_atomic_load(&bar->count, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) -
                   target) < 0) {
        // the abort flag and the clock on the first poll and every 16th
        // (a limit of 0 gives up as soon as the workgroup has to wait)
        if ((polls++ & 15u) == 0 &&
            (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) != 0 ||
             (long long)wall_clock64() - t0 >= limit)) {
          __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) != 0)
        ok = 0;
      *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
  }
};

// Window geometry: own rows [k0, k1), window [w0, w1) with depth d.
struct Win {
  int k0, k1, w0, w1;
};
__device__ __forceinline__ Win window(int R, int rb, int d, int wi) {
  Win w;
  w.k0 = wi * rb;
  w.k1 = min(R, w.k0 + rb);
  w.w0 = max(0, w.k0 - d);
  w.w1 = min(R, w.k1 + d);
  return w;
}

// The blocks F_b, b in [fb0, fb0 + cnt), of a window: staged in LDS when
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

// ``copy`` false: the blocks are already in ``lds`` (staged by an earlier
// phase of the same window), only the descriptor is formed.
template <typename T, int NS>
__device__ FBlocks<T> stage_F(const GArgs<T, NS>& a, int b0, int b1, T* lds,
                              bool copy = true) {
  const size_t nn = (size_t)a.nv() * a.nv();
  b0 = max(b0, 0);
  b1 = min(b1, a.R - 1);  // F_b exists for b <= R - 2
  FBlocks<T> f{a.F, 0};
  if (lds == nullptr || b1 <= b0) return f;
  if (copy) {
    const size_t cnt = (size_t)(b1 - b0) * nn;
    const T* src = a.F + (size_t)b0 * nn;
    for (size_t e = threadIdx.x; e < cnt; e += NT) lds[e] = src[e];
    __syncthreads();
  }
  return FBlocks<T>{lds, b0};
}

// The blocks of one thread's entry (k, i) of its window, held in registers
// for a whole inner solve: row i of F_k and column i of F_{k-1} (zeros
// where the block does not exist). Used when n is fixed at compile time,
// the workgroup keeps one window and the window has at most one entry per
// thread (entry o = thread o); otherwise ``on`` is false and C reads the
// blocks from LDS or memory.
template <typename T, int NS>
struct FReg {
  static constexpr bool kUsed = NS > 0 && NS <= 16;  // registers suffice
  static constexpr int L = kUsed ? NS : 1;
  T fp[L];
  T fm[L];
  bool on;
};

// n consecutive entries of a window vector in LDS, as 16-byte reads when
// every row of the window starts on a 16-byte boundary.
template <typename T, int NS>
__device__ __forceinline__ void ld_row(const T* p, T (&v)[FReg<T, NS>::L]) {
  if constexpr ((NS * sizeof(T)) % 16 == 0) {
    const T* q = (const T*)__builtin_assume_aligned(p, 16);
#pragma unroll
    for (int j = 0; j < NS; ++j) v[j] = q[j];
  } else {
#pragma unroll
    for (int j = 0; j < FReg<T, NS>::L; ++j) v[j] = p[j];
  }
}

// C v on rows [lo, hi), v valid on the rows it needs, in the window layout
// (row k at (k - w0) n): ``ep(o, c)`` receives entry o of the window and its
// value c = (C v)[o], and stores what the caller needs (C v itself, or a
// combination with other vectors at the same entry). The F_{k-1}^T and F_k
// terms are summed in two chains and then added.
template <typename T, int NS, typename Ep>
__device__ __forceinline__ void applyC(const GArgs<T, NS>& a,
                                       const FBlocks<T>& F,
                                       const FReg<T, NS>& fr, const T* v,
                                       int w0, int lo, int hi, Ep&& ep) {
  if constexpr (FReg<T, NS>::kUsed) {
    if (fr.on) {
      const int o = threadIdx.x, k = w0 + o / NS;
      if (k >= lo && k < hi) {
        T am = T(0), ap = T(0), x[FReg<T, NS>::L];
        if (k > 0) {
          ld_row<T, NS>(v + (k - 1 - w0) * NS, x);
#pragma unroll
          for (int j = 0; j < NS; ++j) am += fr.fm[j] * x[j];
        }
        if (k < a.R - 1) {
          ld_row<T, NS>(v + (k + 1 - w0) * NS, x);
#pragma unroll
          for (int j = 0; j < NS; ++j) ap += fr.fp[j] * x[j];
        }
        ep(o, -(am + ap));
      }
      return;
    }
  }
  const int n = a.nv();
  const size_t nn = (size_t)n * n;
  const int cnt = (hi - lo) * n;
  for (int e = threadIdx.x; e < cnt; e += NT) {
    const int k = lo + e / n, i = e % n;
    T am = T(0), ap = T(0);
    if (k > 0) {
      const T* Fm = F.blk(k - 1, nn) + i;
      const T* vm = v + (k - 1 - w0) * n;
#pragma unroll
      for (int j = 0; j < n; ++j) am += Fm[(size_t)j * n] * vm[j];
    }
    if (k < a.R - 1) {
      const T* Fk = F.blk(k, nn) + (size_t)i * n;
      const T* vp = v + (k + 1 - w0) * n;
#pragma unroll
      for (int j = 0; j < n; ++j) ap += Fk[j] * vp[j];
    }
    ep((k - w0) * n + i, -(am + ap));
  }
}

// rows on which C v is known when v is known on [lo, hi)
__device__ __forceinline__ void shrink(int R, int& lo, int& hi) {
  if (lo > 0) ++lo;
  if (hi < R) --hi;
}

// z = M^{-1} r on the own rows; r known on the whole window (LDS), y, w1,
// w2, z window buffers. Returns with z valid on [k0, k1). The updates of
// y and z run inside the applications of C that produce their operands.
template <typename T, int NS>
__device__ void precond(const GArgs<T, NS>& a, const FBlocks<T>& F,
                        const FReg<T, NS>& fr, const Win& W, const T* r, T* y,
                        T* w1, T* w2, T* z) {
  const int n = a.nv(), w0 = W.w0;
  const T av = (T)a.a, om = (T)(1.0 - a.a);
  int lo = W.w0, hi = W.w1;
  const T* cur = r;  // y_{i}, the operand of the next application
  if (a.a != 0.0) {  // y_0 = r + a C r
    shrink(a.R, lo, hi);
    applyC(a, F, fr, r, w0, lo, hi, [&](int o, T c) {
      const T yv = r[o] + av * c;
      y[o] = yv;
      z[o] = yv;
    });
    cur = y;
  } else {  // y_0 = r
    for (int e = threadIdx.x; e < (hi - lo) * n; e += NT) {
      const int o = (lo - w0) * n + e;
      z[o] = r[o];
    }
  }
  __syncthreads();
  for (int m = 1; m < a.m; ++m) {
    const T al = (T)a.alpha[m];
    if (a.a != 0.0) {  // y_m = (1 - a) C y + a C (C y)
      shrink(a.R, lo, hi);
      applyC(a, F, fr, cur, w0, lo, hi, [&](int o, T c) { w1[o] = c; });
      __syncthreads();
      shrink(a.R, lo, hi);
      applyC(a, F, fr, w1, w0, lo, hi, [&](int o, T c) {
        const T yv = om * w1[o] + av * c;
        y[o] = yv;
        z[o] += al * yv;
      });
      cur = y;
    } else {  // y_m = C y_{m-1}, into the buffer the operand is not in
      T* nxt = cur == w2 ? y : w2;
      shrink(a.R, lo, hi);
      applyC(a, F, fr, cur, w0, lo, hi, [&](int o, T c) {
        nxt[o] = c;
        z[o] += al * c;
      });
      cur = nxt;
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

// Partial of one reduction over the window's own rows into its slot.
template <typename T, int NS>
__device__ __forceinline__ void put_partial(const GArgs<T, NS>& a, int slot,
                                            int wi, double v, double* red) {
  const double s = wg_sum(v, red);
  if (threadIdx.x == 0) st_sh(a.part + slot * a.nwin + wi, s);
}

template <typename T>
__device__ __forceinline__ T* lds_vec(double* red, int slot, int len) {
  return reinterpret_cast<T*>(red + NT) + (size_t)slot * len;
}

// Entries of one window vector in LDS: rb rows and the halo on both sides
// (at least one row: the q phase forms p on the neighbour rows).
__host__ __device__ __forceinline__ int wlen(int rb, int depth, int n) {
  return (rb + 2 * (depth > 1 ? depth : 1)) * n;
}

// Bytes of staged blocks: the window's (rb + 2 depth - 1) or, in the q
// phase, rb + 1 blocks.
template <typename T>
__host__ __device__ __forceinline__ size_t fstage_bytes(int rb, int depth,
                                                        int n) {
  return (size_t)(rb + 2 * depth + 1) * n * n * sizeof(T);
}

// LDS for staged blocks (after the five window vectors), or null when they
// do not fit
template <typename T, int NS>
__device__ __forceinline__ T* lds_F(const GArgs<T, NS>& a, double* red) {
  const int lmax = wlen(a.rb, a.depth + 1, a.nv());
  return fstage_bytes<T>(a.rb, a.depth + 1, a.nv()) <= FSTAGE_MAX
             ? lds_vec<T>(red, 5, lmax)
             : nullptr;
}

// LDS of a workgroup: the reduction scratch, the five window vectors and,
// when they fit, the staged blocks F.
template <typename T>
__host__ __device__ __forceinline__ size_t lds_base_bytes(int rb, int depth,
                                                          int n) {
  const size_t fb = fstage_bytes<T>(rb, depth, n);
  return NT * sizeof(double) + 5 * (size_t)wlen(rb, depth, n) * sizeof(T) +
         (fb <= FSTAGE_MAX ? fb : 0);
}

// The factors L_k of a window's own rows, for the stopping norm ||L r||,
// staged after the blocks F when both fit and the workgroup's LDS stays
// within 64 KB (two workgroups per CU).
constexpr size_t LDS_WITH_L_MAX = 64 * 1024;
template <typename T>
__host__ __device__ __forceinline__ size_t lstage_bytes(int rb, int n) {
  return (size_t)rb * n * n * sizeof(T);
}
template <typename T>
__host__ __device__ __forceinline__ bool lstage_fits(int rb, int depth,
                                                     int n) {
  return fstage_bytes<T>(rb, depth, n) <= FSTAGE_MAX &&
         lds_base_bytes<T>(rb, depth, n) + lstage_bytes<T>(rb, n) <=
             LDS_WITH_L_MAX;
}
template <typename T, int NS>
__device__ __forceinline__ T* lds_L(const GArgs<T, NS>& a, double* red) {
  const int n = a.nv();
  if (!lstage_fits<T>(a.rb, a.depth + 1, n)) return nullptr;
  return lds_F(a, red) + fstage_bytes<T>(a.rb, a.depth + 1, n) / sizeof(T);
}

// Row i of the lower-triangular block at ``row`` times v (columns 0..i),
// over a loop of fixed length when n is known at compile time.
template <typename T, int NS>
__device__ __forceinline__ T lower_row(const T* row, const T* v, int n,
                                       int i) {
  T acc = T(0);
  if constexpr (NS > 0) {
#pragma unroll
    for (int j = 0; j < NS; ++j)
      if (j <= i) acc += row[j] * v[j];
  } else {
    for (int j = 0; j <= i; ++j) acc += row[j] * v[j];
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Phases on one window. Each ends with a barrier of the workgroup, so the
// next window may reuse the LDS.
// ---------------------------------------------------------------------------

// u = M^{-1} r on own rows +- 1 and w = Ahat u = u - C u on own rows, from
// r in LDS on the window (depth D + 1); u and w to memory, partials of r'u
// and w'u (and ||L r||^2 when ``nrm``) into the slots of parity ``par``.
// ``Ls``: the own rows' factors L_k staged in LDS, or null (read from L).
template <typename T, int NS>
__device__ void u_and_w(const GArgs<T, NS>& a, const FBlocks<T>& F,
                        const FReg<T, NS>& fr, const Win& W, int par, bool nrm,
                        int wi, T* r, T* y, T* w1, T* w2, T* z, const T* Ls,
                        double* red) {
  const int n = a.nv(), w0 = W.w0;
  if (a.pc == BT_PC_NONE) {  // u = L^T L r, row-local, on own rows +- 1
    const int lo = max(W.k0 - 1, 0), hi = min(W.k1 + 1, a.R);
    for (int e = threadIdx.x; e < (hi - lo) * n; e += NT) {
      const int k = lo + e / n, i = e % n;
      y[(k - w0) * n + i] = lower(a.L, r + (k - w0) * n, n, k, i);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (hi - lo) * n; e += NT) {
      const int k = lo + e / n, i = e % n;
      z[(k - w0) * n + i] = lowerT(a.L, y + (k - w0) * n, n, k, i);
    }
    __syncthreads();
  } else {
    precond(a, F, fr, W, r, y, w1, w2, z);
  }
  typename AccOf<T>::type g, d, t2;
  g.zero();
  d.zero();
  t2.zero();
  // C u on own rows, w = u - C u, and the partials at each entry
  applyC(a, F, fr, z, w0, W.k0, W.k1, [&](int o, T c) {
    const int e = o - (W.k0 - w0) * n;
    const size_t gi = (size_t)W.k0 * n + e;
    const T zv = z[o], wv = zv - c;
    a.u[gi] = zv;
    st_sh(a.wbuf[par] + gi, wv);
    g.add_prod(r[o], zv);
    d.add_prod(wv, zv);
    if (nrm) {  // ||r|| = ||L rhat|| of the original system
      const int k = W.k0 + e / n, i = e % n;
      const T* rk = r + (k - w0) * n;
      const T tv = Ls ? lower_row<T, NS>(Ls + ((size_t)(k - W.k0) * n + i) * n,
                                         rk, n, i)
                      : lower(a.L, rk, n, k, i);
      t2.add_prod(tv, tv);
    }
  });
  double v[3] = {g.value(), d.value(), t2.value()};
  wg_sums<3>(v, red);
  if (threadIdx.x == 0) {
    st_sh(a.part + (P_G + par) * a.nwin + wi, v[0]);
    st_sh(a.part + (P_D + par) * a.nwin + wi, v[1]);
    if (nrm) st_sh(a.part + (P_N + par) * a.nwin + wi, v[2]);
  }
}

// Start of an inner solve: r = L^{-1} (src * sscale) on the window, xhat = 0,
// u, w and their partials (parity 0), ||src * sscale||^2.
// ``resident``: the workgroup keeps this one window for the whole inner
// solve, so the blocks staged here (F, and the own rows' L_k for the
// stopping norm) serve every step.
template <typename T, int NS>
__device__ void ph_init(const GArgs<T, NS>& a, const St& st, int wi,
                        bool resident, FReg<T, NS>& fr, double* red) {
  const Win W = window(a.R, a.rb, a.depth + 1, wi);
  const int n = a.nv(), len = (W.w1 - W.w0) * n;
  const int lmax = wlen(a.rb, a.depth + 1, n);
  T* r = lds_vec<T>(red, 0, lmax);
  T* y = lds_vec<T>(red, 1, lmax);
  T* w1 = lds_vec<T>(red, 2, lmax);
  T* w2 = lds_vec<T>(red, 3, lmax);
  T* z = lds_vec<T>(red, 4, lmax);
  const FBlocks<T> F = stage_F(a, W.w0, W.w1 - 1, lds_F(a, red));
  fr.on = false;
  if constexpr (FReg<T, NS>::kUsed) {
    if (resident && len <= NT) {  // this thread's blocks into registers
      fr.on = true;
      const int o = threadIdx.x, k = W.w0 + o / NS, i = o % NS;
      const size_t nn = (size_t)NS * NS;
      const bool in = o < len;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        fr.fp[j] = in && k < a.R - 1 ? F.blk(k, nn)[i * NS + j] : T(0);
        fr.fm[j] = in && k > 0 ? F.blk(k - 1, nn)[j * NS + i] : T(0);
      }
    }
  }
  if (resident && !st.ir) {
    T* Ls = lds_L(a, red);
    if (Ls) {
      const size_t cnt = (size_t)(W.k1 - W.k0) * n * n;
      const T* src = a.L + (size_t)W.k0 * n * n;
      for (size_t e = threadIdx.x; e < cnt; e += NT) Ls[e] = src[e];
    }
  }
  for (int e = threadIdx.x; e < len; e += NT)
    y[e] = (T)(ld_sh(st.src + (size_t)W.w0 * n + e) * st.sscale);
  __syncthreads();
  double nb = 0.0;
  for (int e = threadIdx.x; e < len; e += NT) {
    const int k = W.w0 + e / n, i = e % n;
    r[e] = lower(a.Li, y + (k - W.w0) * n, n, k, i);
    if (k >= W.k0 && k < W.k1) {
      const double s = ld_sh(st.src + (size_t)W.w0 * n + e) * st.sscale;
      nb += s * s;
      st_sh(a.rbuf[0] + (size_t)k * n + i, r[e]);
      a.xh[(size_t)k * n + i] = T(0);
    }
  }
  __syncthreads();
  put_partial(a, P_NB2, wi, nb, red);
  u_and_w(a, F, fr, W, 0, false, wi, r, y, w1, w2, z, (const T*)nullptr, red);
  if (threadIdx.x == 0)
    st_sh(a.part + P_GF * a.nwin + wi, ld_sh(a.part + P_G * a.nwin + wi));
  __syncthreads();
}

// Decision at the start of step i from the sums of the previous phase: the
// stopping test on r_i (textbook order: ||r|| first, then r'u, then
// p'Ap), beta and alpha. ``gprev`` and ``aprev`` hold gamma and alpha of
// step i - 1 and are updated. Returns BT_NOT_CONVERGED to go on.
constexpr int kCapped = 100;  // dec_step: the step cap is reached

template <typename T, int NS>
__device__ int dec_step(const GArgs<T, NS>& a, const St& st, int i, bool capped,
                        double* red, double* gprev, double* aprev, T* al,
                        T* be) {
  const int par = i & 1;
  double S[5];
  slot_sums<5>(a.part, {P_G + par, P_D + par, P_N + par, P_NB2, P_GF},
               a.nwin, red, S);
  const double gam = S[0], del = S[1], nr2 = S[2], nb2 = S[3], g0 = S[4];
  if (!st.ir) {
    if (i == 0) {
      if (!(nb2 < INFINITY)) return BT_ENONFINITE;
      if (nb2 == 0.0) return BT_OK;
    } else {
      if (nr2 <= st.tol_in * st.tol_in * nb2) return BT_OK;
      if (!(nr2 < INFINITY)) return BT_ENONFINITE;
    }
    if (!(gam > 0.0)) return gam == gam ? BT_EBREAKDOWN : BT_ENONFINITE;
  } else {  // inner solve of a refinement step: stop when r'u fell enough
    if (!(gam > 0.0)) return BT_OK;
    if (i > 0 && gam <= a.itol * a.itol * g0) return BT_OK;
  }
  if (capped) return kCapped;
  const double beta = i == 0 ? 0.0 : gam / *gprev;
  const double sigma = i == 0 ? del : del - beta * gam / *aprev;  // p'A p
  if (!(sigma > 0.0))
    return st.ir ? BT_OK : (sigma == sigma ? BT_EBREAKDOWN : BT_ENONFINITE);
  const double alpha = gam / sigma;
  *gprev = gam;
  *aprev = alpha;
  *al = (T)alpha;
  *be = (T)beta;
  return BT_NOT_CONVERGED;
}

// The vector data a step reads on one window, fetched before the step's
// decision so that its loads overlap the partial sums' (windows of at most
// PF NT entries; larger ones load in ph_step).
constexpr int PF = 2;
template <typename T>
struct Pre {
  T r[PF], w[PF], s[PF], u[PF], p[PF];
};

template <typename T, int NS>
__device__ __forceinline__ bool prefetchable(const GArgs<T, NS>& a) {
  return wlen(a.rb, a.depth + 1, a.nv()) <= PF * NT;
}

template <typename T, int NS>
__device__ void ph_step_fetch(const GArgs<T, NS>& a, int i, int wi, Pre<T>& f) {
  const Win W = window(a.R, a.rb, a.depth + 1, wi);
  const int n = a.nv(), len = (W.w1 - W.w0) * n;
  const int cur = i & 1, nxt = cur ^ 1;
#pragma unroll
  for (int t = 0; t < PF; ++t) {
    const int e = threadIdx.x + t * NT;
    if (e < len) {
      const int k = W.w0 + e / n;
      const size_t g = (size_t)W.w0 * n + e;
      f.r[t] = ld_sh(a.rbuf[cur] + g);
      f.w[t] = ld_sh(a.wbuf[cur] + g);
      f.s[t] = i == 0 ? T(0) : ld_sh(a.sbuf[nxt] + g);
      if (k >= W.k0 && k < W.k1) {
        f.u[t] = a.u[g];
        f.p[t] = i == 0 ? T(0) : a.p[g];
      }
    }
  }
}

// Step i: p = u + beta p, xhat += alpha p (own rows); s = w + beta s and
// r -= alpha s on the window (depth D + 1); u, w of the new r and the
// partials of step i + 1. ``f``: the window's data fetched ahead, or null.
template <typename T, int NS>
__device__ void ph_step(const GArgs<T, NS>& a, const St& st, int i, T al, T be,
                        int wi, const Pre<T>* f, bool resident,
                        const FReg<T, NS>& fr, double* red) {
  const Win W = window(a.R, a.rb, a.depth + 1, wi);
  const int n = a.nv(), len = (W.w1 - W.w0) * n;
  const int lmax = wlen(a.rb, a.depth + 1, n);
  const int cur = i & 1, nxt = cur ^ 1;
  T* r = lds_vec<T>(red, 0, lmax);
  T* y = lds_vec<T>(red, 1, lmax);
  T* w1 = lds_vec<T>(red, 2, lmax);
  T* w2 = lds_vec<T>(red, 3, lmax);
  T* z = lds_vec<T>(red, 4, lmax);
  auto one = [&](int e, T rv, T wv, T sv0, T uv, T pv0) {
    const int k = W.w0 + e / n;
    const size_t g = (size_t)W.w0 * n + e;
    const T sv = i == 0 ? wv : wv + be * sv0;
    r[e] = rv - al * sv;
    if (k >= W.k0 && k < W.k1) {
      const T pv = i == 0 ? uv : uv + be * pv0;
      a.p[g] = pv;
      a.xh[g] += al * pv;
      st_sh(a.sbuf[cur] + g, sv);
      st_sh(a.rbuf[nxt] + g, r[e]);
    }
  };
  if (f) {
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = threadIdx.x + t * NT;
      if (e < len) one(e, f->r[t], f->w[t], f->s[t], f->u[t], f->p[t]);
    }
  } else {
    for (int e = threadIdx.x; e < len; e += NT) {
      const int k = W.w0 + e / n;
      const size_t g = (size_t)W.w0 * n + e;
      const bool own = k >= W.k0 && k < W.k1;
      one(e, ld_sh(a.rbuf[cur] + g), ld_sh(a.wbuf[cur] + g),
          i == 0 ? T(0) : ld_sh(a.sbuf[nxt] + g), own ? a.u[g] : T(0),
          own && i > 0 ? a.p[g] : T(0));
    }
  }
  const FBlocks<T> F =
      stage_F(a, W.w0, W.w1 - 1, lds_F(a, red), !resident);
  const T* Ls = resident && !st.ir ? lds_L(a, red) : nullptr;
  __syncthreads();
  u_and_w(a, F, fr, W, nxt, !st.ir, wi, r, y, w1, w2, z, Ls, red);
  __syncthreads();
}

// x = L^{-T} xhat * xscale (add = 0) or x += L^{-T} d * xscale, own rows.
template <typename T, int NS>
__device__ void ph_x(const GArgs<T, NS>& a, const St& st, int add, int wi,
                     double* red) {
  const Win W = window(a.R, a.rb, 0, wi);
  const int n = a.nv();
  T* v = lds_vec<T>(red, 0, wlen(a.rb, a.depth + 1, n));
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT)
    v[e] = a.xh[(size_t)W.k0 * n + e];
  __syncthreads();
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
    const int k = W.k0 + e / n, i = e % n;
    const double u =
        (double)lowerT(a.Li, v + (k - W.k0) * n, n, k, i) * st.xscale;
    const size_t g = (size_t)W.k0 * n + e;
    st_sh(a.x + g, add ? ld_sh(a.x + g) + u : u);
  }
  __syncthreads();
}

// r64 = b - A x in float64 from the record, own rows, ||r64||^2 and ||b||^2.
template <typename T, int NS>
__device__ void ph_res(const GArgs<T, NS>& a, int wi, double* red) {
  const Win W = window(a.R, a.rb, 0, wi);
  const int n = a.nv();
  const size_t nn = (size_t)n * n;
  double s2 = 0.0, b2 = 0.0;
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * n; e += NT) {
    const int k = W.k0 + e / n, i = e % n;
    const double* xk = a.x + (size_t)k * n;
    double acc = 0.0;
    const size_t db = (size_t)k * nn + (size_t)i * n;
    for (int j = 0; j < n; ++j) acc += rec(a.D, db + j, a.dtype) * ld_sh(xk + j);
    if (k > 0) {
      const size_t ob = (size_t)(k - 1) * nn + i;
      for (int j = 0; j < n; ++j)
        acc += rec(a.O, ob + (size_t)j * n, a.dtype) * ld_sh(xk + j - n);
    }
    if (k < a.R - 1) {
      const size_t ob = (size_t)k * nn + (size_t)i * n;
      for (int j = 0; j < n; ++j)
        acc += rec(a.O, ob + j, a.dtype) * ld_sh(xk + n + j);
    }
    const size_t g = (size_t)k * n + i;
    const double rv = a.b[g] - acc;
    st_sh(a.r64 + g, rv);
    s2 += rv * rv;
    b2 += a.b[g] * a.b[g];
  }
  put_partial(a, P_RES, wi, s2, red);
  put_partial(a, P_NB2, wi, b2, red);
  __syncthreads();
}

// x = 0 on the window's own rows.
template <typename T, int NS>
__device__ void ph_zero_x(const GArgs<T, NS>& a, int wi) {
  const Win W = window(a.R, a.rb, 0, wi);
  for (int e = threadIdx.x; e < (W.k1 - W.k0) * a.nv(); e += NT)
    st_sh(a.x + (size_t)W.k0 * a.nv() + e, 0.0);
}

__global__ void k_g_reset(Bar* bar) {
  bar->count = 0u;
  bar->abort = 0;
}

// The whole solve. Every workgroup runs the same control flow and takes
// the same decisions; workgroup 0 writes the outcome.
template <typename T, int NS>
__global__ void __launch_bounds__(NT) k_g_solve(GArgs<T, NS> a) {
  extern __shared__ __align__(16) double red[];
  __shared__ int s_flag;
  Sync sync{a.bar, gridDim.x, 0u, a.spin_limit};
  const int wg = blockIdx.x, nwg = gridDim.x;
  auto each = [&](auto&& f) {
    for (int wi = wg; wi < a.nwin; wi += nwg) f(wi);
  };
  // executed block products: halves of applications of C, triangular
  // transforms, float64 residuals (halo rows a window recomputes are not
  // counted)
  long long g_half = 0, g_tri = 0, g_res = 0;
  const bool none = a.pc == BT_PC_NONE;
  const int apc = none ? 0
                       : (a.a != 0.0 ? 1 : 0) + (a.m - 1) * (a.a != 0.0 ? 2 : 1);
  int status = BT_NOT_CONVERGED, total = 0, outer = 0;
  double nb2 = 0.0, nr2 = 0.0, nrt2 = 0.0;
  bool aborted = false;
  auto barrier = [&]() {
    if (!aborted && !sync(&s_flag)) aborted = true;
    return !aborted;
  };
  auto sums2 = [&](int s0, int s1, double* v0, double* v1) {
    double S[2];
    slot_sums<2>(a.part, {s0, s1}, a.nwin, red, S);
    *v0 = S[0];
    *v1 = S[1];
  };
  St st{a.b, 1.0, 1.0, a.tol, 0};
  // one inner PCG solve from the right-hand side in st; returns the steps
  // taken, or -1 when aborted
  // a workgroup with one window fetches its data before the decision and
  // keeps the window's blocks in LDS from the init phase on
  const bool pre = prefetchable(a) && a.nwin <= nwg;
  FReg<T, NS> fr;
  fr.on = false;
  auto pcg = [&](int cap, int* settled) -> int {
    each([&](int wi) { ph_init(a, st, wi, pre, fr, red); });
    if (!barrier()) return -1;
    int steps = 0;
    double gprev = 0.0, aprev = 0.0;
    for (int i = 0;; ++i) {
      Pre<T> f;
      if (pre && wg < a.nwin) ph_step_fetch(a, i, wg, f);
      T al, be;
      const int d = dec_step(a, st, i, i >= cap, red, &gprev, &aprev, &al, &be);
      if (d != BT_NOT_CONVERGED) {
        *settled = d == kCapped ? BT_NOT_CONVERGED : d;
        break;
      }
      steps = i + 1;
      each([&](int wi) {
        ph_step(a, st, i, al, be, wi, pre ? &f : nullptr, pre, fr, red);
      });
      if (!barrier()) return -1;
    }
    // per step (and at the start): u = M^{-1} r and w = A u
    g_half += 2 * ((long long)(apc + 1) * (steps + 1));
    g_tri += 2 + (none ? 2 * (long long)(steps + 1) : 0) + (st.ir ? 0 : steps);
    return steps;
  };

  if (a.fail[0] != BT_NO_FAIL) {  // a D_k is not positive definite
    each([&](int wi) { ph_zero_x(a, wi); });
    status = BT_ENOTSPD;
  } else if (!a.refine) {
    int add = 0;
    outer = 1;
    if (a.from_res) {
      // from the initial guess x0 (held in x; 0 when not warm): plain PCG
      // on the correction A d = r0 = b - A x0, the test ||r|| <= tol ||b||
      // carried over to the correction's right-hand side
      if (!a.warm) {
        each([&](int wi) { ph_zero_x(a, wi); });
        barrier();
      }
      if (!aborted) each([&](int wi) { ph_res(a, wi, red); });
      barrier();
      ++g_res;
      double nr02 = 0.0;
      if (!aborted) sums2(P_NB2, P_RES, &nb2, &nr02);
      nr2 = nrt2 = nr02;
      if (aborted) {
      } else if (!(nb2 < INFINITY) || !(nr02 < INFINITY)) {
        status = BT_ENONFINITE;
      } else if (nb2 == 0.0) {  // b = 0: x = 0
        each([&](int wi) { ph_zero_x(a, wi); });
        status = BT_OK;
        nr2 = nrt2 = 0.0;
      } else if (nr02 <= a.tol * a.tol * nb2) {
        status = BT_OK;
      } else {
        st.src = a.r64;
        st.tol_in = a.tol * sqrt(nb2 / nr02);
        st.sscale = bt_unit_scale(nr02);
        st.xscale = 1.0 / st.sscale;
        add = 1;
      }
    }
    if (status == BT_NOT_CONVERGED && !aborted) {
      int settled = BT_NOT_CONVERGED;
      const int steps = pcg(a.maxit, &settled);
      if (steps >= 0) {
        total = steps;
        status = settled;
        double nr2s = 0.0, unused = 0.0;
        sums2(P_N + (steps & 1), P_NB2, &nr2s, &unused);
        each([&](int wi) { ph_x(a, st, add, wi, red); });
        if (barrier()) {
          each([&](int wi) { ph_res(a, wi, red); });
          if (barrier()) {
            ++g_res;
            double b2 = 0.0;
            sums2(P_NB2, P_RES, &b2, &nrt2);
            const double nr02 = nr2;
            nb2 = b2;
            nr2 = total > 0 ? nr2s * st.xscale * st.xscale
                            : (a.from_res ? nr02 : b2);
            // the test after the last permitted step (the q phase runs it
            // at the start of the next step, which the cap did not reach)
            if (status == BT_NOT_CONVERGED && total > 0 &&
                nr2 <= a.tol * a.tol * nb2)
              status = BT_OK;
          }
        }
      }
    }
  } else {
    // float inner PCG inside float64 refinement on the record
    st.ir = 1;
    st.src = a.r64;
    if (!a.warm) {
      each([&](int wi) { ph_zero_x(a, wi); });
      barrier();
    }
    double nr2_prev = INFINITY;  // before the last correction
    while (!aborted) {
      each([&](int wi) { ph_res(a, wi, red); });
      if (!barrier()) break;
      if (outer > 0 || a.warm) ++g_res;  // the first pass from 0 reads b only
      double b2 = 0.0;
      sums2(P_NB2, P_RES, &b2, &nr2);
      if (outer == 0) nb2 = b2;
      nrt2 = nr2;
      if (a.warm && outer == 0 && nb2 == 0.0) {  // b = 0: x = 0
        each([&](int wi) { ph_zero_x(a, wi); });
        nr2 = nrt2 = 0.0;
        status = BT_OK;
        break;
      }
      if (nr2 <= a.tol * a.tol * nb2) { status = BT_OK; break; }
      if (!(nr2 < INFINITY)) { status = BT_ENONFINITE; break; }
      // a correction that cut the float64 residual by less than 2x
      if (outer > 0 && nr2 > 0.25 * nr2_prev) { status = BT_ESTAGNATED; break; }
      if (outer >= a.max_outer || total >= a.maxit) break;
      nr2_prev = nr2;
      st.sscale = bt_unit_scale(nr2);
      st.xscale = 1.0 / st.sscale;
      int settled = BT_NOT_CONVERGED;
      const int steps = pcg(a.maxit - total, &settled);
      if (steps < 0) break;
      total += steps;
      each([&](int wi) { ph_x(a, st, 1, wi, red); });
      if (!barrier()) break;
      ++outer;
      if (steps == 0) {
        status = BT_EBREAKDOWN;
        each([&](int wi) { ph_res(a, wi, red); });
        if (!barrier()) break;
        ++g_res;
        sums2(P_RES, P_NB2, &nr2, &b2);
        nrt2 = nr2;
        break;
      }
    }
  }
  if (aborted) status = BT_ETIMEOUT;
  if (wg == 0 && threadIdx.x == 0) {
    const bool spd = status != BT_ENOTSPD;
    bt_info* inf = a.info;
    inf->status = status;
    inf->iters = total;
    inf->outer = spd ? outer : 0;
    inf->fail_index = spd ? -1 : a.fail[0];
    inf->relres = !spd ? NAN : nb2 > 0.0 ? sqrt(nr2 / nb2) : 0.0;
    inf->relres_true = !spd ? NAN : nb2 > 0.0 ? sqrt(nrt2 / nb2) : 0.0;
    inf->gemv_exec = spd ? bt_gemv_rows(a.R, g_half, g_tri, g_res) : 0;
    inf->gemv_paper = (int64_t)total * bt_gemv_g(a.pc, a.a, a.m);
  }
}

inline int depth_of(const bt_params& p) {
  if (p.pc == BT_PC_NONE) return 0;
  const int d1 = p.a != 0.0 ? 1 : 0, dh = p.a != 0.0 ? 2 : 1;
  return d1 + (p.m - 1) * dh;
}

// Rows per window. Larger windows mean fewer workgroups, cheaper grid
// barriers and less halo recomputed per own row: 4..16 rows (R / 64) up to
// 1024 block rows, then about one window per CU (R / 256, at most 64 rows;
// N = 8192, n = 12: 0.81 -> 0.56 ms, N = 32768: 2.66 -> 1.53 ms against
// 16 rows; that growth keeps the five window vectors within 64 KB of LDS).
// With n = 6 or 12 (block size fixed at compile time) a window of at most
// one entry per thread keeps each thread's F entries in registers; that is
// worth more (N = 2048, n = 12: 0.35 -> 0.28 ms) as long as every window
// still gets a workgroup of its own, so the window shrinks to fit when its
// windows then number at most one per CU (256).
constexpr int64_t kWindowsPerGrid = 256;
inline int rows_per_win(int64_t R, int n, int depth) {
  const int halo = 2 * std::max(depth + 1, 1);
  int64_t rb = std::max<int64_t>(4, std::min<int64_t>(16, R / 64));
  if (R / kWindowsPerGrid > rb) {  // grow towards one window per CU
    const int64_t lds_cap = (64 * 1024 - NT * (int64_t)sizeof(double)) /
                                (5 * n * (int64_t)sizeof(double)) - halo;
    rb = std::max(rb, std::min<int64_t>({64, R / kWindowsPerGrid, lds_cap}));
  }
  if (n == 6 || n == 12) {
    const int fit = NT / n - halo;
    if (fit >= 4 && fit < rb && (R + fit - 1) / fit <= kWindowsPerGrid) rb = fit;
  }
  return (int)rb;
}

// Scratch layout: nine T vectors (r, s and w twice, u, p, xhat), the
// float64 residual, the partial sums, the barrier.
constexpr int NVEC = 9;
template <typename T>
struct Scratch {
  size_t r64, part, bar, total;
  Scratch(int64_t R, int n, int depth) {
    const int rb = rows_per_win(R, n, depth);
    const int nwin = (int)((R + rb - 1) / rb);
    const size_t v = (size_t)R * n;
    r64 = (NVEC * v * sizeof(T) + 255) / 256 * 256;
    part = r64 + v * sizeof(double);
    bar = (part + (size_t)P_SLOTS * nwin * sizeof(double) + 255) / 256 * 256;
    total = bar + sizeof(Bar);
  }
};

// Workgroups of k_g_solve that fit on the device at once with ``lds`` bytes
// of LDS each (the grid never exceeds it: the barrier needs them all).
template <typename T, int NS>
int coresident(size_t lds) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, (const void*)k_g_solve<T, NS>, NT, lds) != hipSuccess)
    return 0;
  return cus * per;
}

// One persistent launch of k_g_solve with the block size fixed at compile
// time (NS > 0) or read at run time (NS = 0).
template <typename T, int NS>
int launch(const GArgsBase<T>& base, size_t lds, hipStream_t s) {
  GArgs<T, NS> a;
  static_cast<GArgsBase<T>&>(a) = base;
  // dynamic LDS beyond 64 KB needs the kernel's limit raised, to what the
  // 160 KB of a workgroup leave beside the kernel's static LDS
  if (lds > 65536) {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void*)k_g_solve<T, NS>) != hipSuccess)
      return BT_EHIP;
    const size_t cap = 160 * 1024 - fa.sharedSizeBytes;
    if (lds > cap) return BT_EINVAL;
    static std::atomic<uint64_t> attr{0};
    if (lds_limit((const void*)k_g_solve<T, NS>, cap, attr) != hipSuccess)
      return BT_EHIP;
  }
  const int res = coresident<T, NS>(lds);
  if (res < 1) return BT_EHIP;
  const int grid = std::min(a.nwin, res);
  hipLaunchKernelGGL(k_g_reset, dim3(1), dim3(1), 0, s, a.bar);
  if (hipGetLastError() != hipSuccess) return BT_EHIP;
  // a cooperative launch: all workgroups resident at once (the barrier
  // needs them; its bounded wait turns a violation into BT_ETIMEOUT)
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)k_g_solve<T, NS>, dim3(grid),
                                    dim3(NT), args, (unsigned)lds, s) ==
                 hipSuccess
             ? BT_OK
             : BT_EHIP;
}

template <typename T>
int run(const bt_handle* h, const double* b, double* x, double tol, int maxit,
        bt_info* info, void* ws, long long spin_limit, hipStream_t s) {
  const int64_t R = h->R;
  const int n = h->n;
  GArgsBase<T> a{};
  a.R = (int)R;
  a.n = n;
  a.rb = rows_per_win(R, n, depth_of(h->p));
  a.nwin = (int)((R + a.rb - 1) / a.rb);
  a.depth = depth_of(h->p);
  a.pc = h->p.pc;
  a.m = h->p.m;
  a.a = h->p.a;
  for (int i = 0; i < BT_MAX_M; ++i) a.alpha[i] = i == 0 ? 1.0 : h->p.alpha[i];
  a.dtype = h->dtype;
  a.tol = tol;
  a.itol = h->p.inner_tol;
  a.refine = h->p.prec == BT_F32_IR || h->p.prec == BT_BF16X2_IR;
  a.warm = h->p.warm_start != 0;
  // float32 without refinement also starts from the residual of x0 = 0,
  // which gives ||b|| before the iteration, so that its right-hand side can
  // be scaled (float64 needs no scaling and saves the pass)
  a.from_res = !a.refine && (a.warm || sizeof(T) == sizeof(float));
  a.max_outer = h->p.max_outer;
  a.maxit = maxit;
  a.spin_limit = spin_limit;
  a.F = (const T*)h->F;
  a.L = (const T*)h->L;
  a.Li = (const T*)h->Li;
  a.D = h->D;
  a.O = h->O;
  a.fail = h->fail;
  a.b = b;
  a.x = x;
  a.info = info;
  const size_t v = (size_t)R * n;
  T* f = (T*)ws;
  a.rbuf[0] = f;
  a.rbuf[1] = f + v;
  a.sbuf[0] = f + 2 * v;
  a.sbuf[1] = f + 3 * v;
  a.wbuf[0] = f + 4 * v;
  a.wbuf[1] = f + 5 * v;
  a.u = f + 6 * v;
  a.p = f + 7 * v;
  a.xh = f + 8 * v;
  const Scratch<T> sl(R, n, a.depth);
  a.r64 = (double*)((unsigned char*)ws + sl.r64);
  a.part = (double*)((unsigned char*)ws + sl.part);
  a.bar = (Bar*)((unsigned char*)ws + sl.bar);
  size_t lds = lds_base_bytes<T>(a.rb, a.depth + 1, n);
  if (lstage_fits<T>(a.rb, a.depth + 1, n)) lds += lstage_bytes<T>(a.rb, n);
  switch (n) {
    case 6: return launch<T, 6>(a, lds, s);
    case 12: return launch<T, 12>(a, lds, s);
    case 24: return launch<T, 24>(a, lds, s);
    default: return launch<T, 0>(a, lds, s);
  }
}

}  // namespace btg

size_t bt_grid_scratch_bytes(const bt_handle* h) {
  if (!h || h->B != 1) return 0;
  const int depth = btg::depth_of(h->p);
  return h->p.prec == BT_F64 ? btg::Scratch<double>(h->R, h->n, depth).total
                             : btg::Scratch<float>(h->R, h->n, depth).total;
}

int bt_grid_solve(const bt_handle* h, const double* b, double* x, double tol,
                  int maxit, bt_info* info, void* ws, hipStream_t s) {
  // the barrier's wait limit in ticks of the device's wall clock
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) !=
          hipSuccess ||
      khz <= 0)
    khz = 100000;  // 100 MHz
  const double ticks = h->grid_wait_s * 1e3 * khz;
  const long long lim = ticks < 9e18 ? (long long)ticks : (long long)9e18;
  if (h->p.prec == BT_F64)
    return btg::run<double>(h, b, x, tol, maxit, info, ws, lim, s);
  return btg::run<float>(h, b, x, tol, maxit, info, ws, lim, s);
}

// ---------------------------------------------------------------------------
// Scratch held by the library for bt_solve_grid_noalloc (callers that cannot
// allocate device memory). One array per GPU the library runs on, kept until
// the process ends. On the host the array's name is only a stand-in, never
// a device address: host code uses the address that hipGetSymbolAddress
// returns for the current device, taken once per device and kept below.
// Every call on a GPU shares that GPU's array (calls that overlap on one GPU
// race); the solve initialises everything it reads before reading it (the
// barrier state in k_g_reset, partial slots before their sums, p and the
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
