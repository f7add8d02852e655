// Persistent PCG kernel: one workgroup per system, systems taken from a
// device queue (longest first), the whole iteration on the device.
//
// Representation. With D_k = L_k L_k^T (Cholesky) and L = blkdiag(L_k), the
// iteration runs on the congruent system  Ahat = L^{-1} A L^{-T} = I - C,
// where C is block tridiagonal with zero diagonal blocks and
//   (C v)_k = -(F_{k-1}^T v_{k-1} + F_k v_{k+1}),
//   F_k = L_k^{-1} O_k L_{k+1}^{-T}.
// With J = B_d^{-1} C_d (the diagonal splitting of Section II-C) one has
// J = L^{-T} C L^T, and the parametric pair of Section III-A obeys
//   G_ab = (I + a J) B_d^{-1},  H_ab = I - G_ab A = (1-a) J + a J^2
// (for a = 1 this is the identity of the footnote to Theorem 3.6,
// M_m^{-1}(1,-1) = M_{2m}^{-1}(0,1)). Hence
//   M_m^{-1} = L^{-T} [ sum_i alpha_i Hh^i Gh ] L^{-1},
//   Gh = I + a C,  Hh = (1-a) C + a C^2,
// and PCG on (A, M^{-1}) from x0 = 0 equals PCG on (Ahat, Gh/Hh polynomial)
// from 0 under x = L^{-T} xhat, r = L rhat: same alpha_j, beta_j, same
// iteration count in exact arithmetic. The preconditioner is evaluated in
// the order of Section IV-B: y_0 = G r, y_i = H y_{i-1}, z = sum alpha_i y_i.
// Only F (one n x n block per row) is touched in the inner loop, instead of
// the D, O, D^{-1}, E_k and three H blocks of the explicit form.
//
// Stopping tests. BT_F64 / BT_F32: ||r|| = ||L rhat|| <= tol ||b||, the
// test of textbook PCG on the original system. BT_F32_IR: the outer loop
// tests the float64 residual b - A x of the record; each float32 inner
// solve stops when ||rhat|| fell by inner_tol.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "reduce.h"

namespace btk {

constexpr int SLOTS = 4;

template <typename T>
struct Shared {
  T* vb0;                            // staging buffers for neighbour access
  T* vb1;
  double* vd;                        // float64 view over both buffers
  typename AccOf<T>::type* redT;     // [SLOTS][NW]
  AccD* redD;                        // [SLOTS][NW]
  int cur;                           // buffer written last
  int slotT, slotD;
};

__device__ __forceinline__ double rec_load(const void* P, size_t i,
                                           int dtype) {
  return dtype == BT_DT_F64 ? ((const double*)P)[i]
                            : (double)((const float*)P)[i];
}

// (C v)_k[i] with v staged in LDS (instance-local layout [N][n]).
template <typename T>
__device__ __forceinline__ T apply_C(const T* __restrict__ F,
                                     const T* __restrict__ v, int N, int n,
                                     int k, int i) {
  T acc = T(0);
  const size_t nn = (size_t)n * n;
  if (k > 0) {
    const T* Fm = F + (size_t)(k - 1) * nn;  // column i of F_{k-1}
    const T* vm = v + (k - 1) * n;
    for (int j = 0; j < n; ++j) acc += Fm[j * n + i] * vm[j];
  }
  if (k < N - 1) {
    const T* Fk = F + (size_t)k * nn + (size_t)i * n;  // row i of F_k
    const T* vp = v + (k + 1) * n;
    for (int j = 0; j < n; ++j) acc += Fk[j] * vp[j];
  }
  return -acc;
}

// (M v)_k[i] for lower-triangular blocks M_k (row i, columns 0..i).
template <typename T>
__device__ __forceinline__ T apply_lower(const T* __restrict__ M,
                                         const T* __restrict__ v, int n,
                                         int k, int i) {
  const T* row = M + ((size_t)k * n + i) * n;
  const T* vk = v + k * n;
  T acc = T(0);
  for (int j = 0; j <= i; ++j) acc += row[j] * vk[j];
  return acc;
}

// (M^T v)_k[i] for lower-triangular blocks M_k (column i, rows i..n-1).
template <typename T>
__device__ __forceinline__ T apply_lowerT(const T* __restrict__ M,
                                          const T* __restrict__ v, int n,
                                          int k, int i) {
  const T* blk = M + (size_t)k * n * n;
  const T* vk = v + k * n;
  T acc = T(0);
  for (int j = i; j < n; ++j) acc += blk[j * n + i] * vk[j];
  return acc;
}

template <typename T, int NT, int S>
struct Inst {
  int N, n, P;
  int64_t r0;
  int inst;
  int k[S], i[S];
  bool act[S];
  const T* F;
  const T* L;
  const T* Li;

  __device__ __forceinline__ void init(const SolveArgs& a, int which) {
    inst = which;
    r0 = a.off[which];
    N = (int)(a.off[which + 1] - r0);
    n = a.n;
    P = N * n;
    const size_t off = (size_t)r0 * n * n;
    F = (const T*)a.F + off;
    L = (const T*)a.L + off;
    Li = (const T*)a.Li + off;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      int p = threadIdx.x + s * NT;
      act[s] = p < P;
      k[s] = act[s] ? p / n : 0;
      i[s] = act[s] ? p - k[s] * n : 0;
    }
  }
  __device__ __forceinline__ int pidx(int s) const {
    return threadIdx.x + s * NT;
  }
};

template <typename T, int NT, int S>
struct Ops {
  using Acc = typename AccOf<T>::type;
  Shared<T>& sh;
  const Inst<T, NT, S>& in;
  // what the system executed: halves of applications of C, triangular
  // transforms, float64 residuals (the same in every thread)
  int nh = 0, ntr = 0, nrs = 0;

  __device__ Ops(Shared<T>& s, const Inst<T, NT, S>& i) : sh(s), in(i) {}

  __device__ __forceinline__ int64_t gemv_exec() const {
    return bt_gemv_rows(in.N, nh, ntr, nrs);
  }

  // Write v into the other staging buffer and publish it to the workgroup.
  __device__ __forceinline__ const T* stage(const T (&v)[S]) {
    sh.cur ^= 1;
    T* b = sh.cur ? sh.vb1 : sh.vb0;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) b[in.pidx(s)] = v[s];
    __syncthreads();
    return b;
  }

  __device__ __forceinline__ void C(const T* v, T (&out)[S]) {
    nh += 2;
#pragma unroll
    for (int s = 0; s < S; ++s)
      out[s] = in.act[s] ? apply_C<T>(in.F, v, in.N, in.n, in.k[s], in.i[s])
                         : T(0);
  }

  __device__ __forceinline__ double dot(const T (&x)[S], const T (&y)[S]) {
    Acc acc;
    acc.zero();
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) acc.add_prod(x[s], y[s]);
    Acc* slot = sh.redT + sh.slotT * (NT / 64);
    sh.slotT = (sh.slotT + 1) % SLOTS;
    return block_sum<NT>(acc, slot).value();
  }

  __device__ __forceinline__ double sumd(double v) {
    AccD acc;
    acc.s = v;
    AccD* slot = sh.redD + sh.slotD * (NT / 64);
    sh.slotD = (sh.slotD + 1) % SLOTS;
    return block_sum<NT>(acc, slot).value();
  }

  // z = M^{-1} r in the scaled coordinates. If ``rs`` is not null it holds
  // r already staged; for BT_PC_NONE ``t`` must hold L r (then z = L^T t).
  __device__ __forceinline__ void precond(const SolveArgs& a, const T (&r)[S], const T* rs,
                          const T (&t)[S], T (&z)[S]) {
    if (a.pc == BT_PC_NONE) {
      const T* ts = stage(t);
      ++ntr;
#pragma unroll
      for (int s = 0; s < S; ++s)
        z[s] = in.act[s] ? apply_lowerT<T>(in.L, ts, in.n, in.k[s], in.i[s])
                         : T(0);
      return;
    }
    const T av = (T)a.a;
    T y[S], w1[S], w2[S];
    // y_0 = Gh r = r + a C r
    if (a.a != 0.0) {
      const T* v = rs ? rs : stage(r);
      C(v, w1);
#pragma unroll
      for (int s = 0; s < S; ++s) y[s] = r[s] + av * w1[s];
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) y[s] = r[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) z[s] = y[s];
    // y_i = Hh y_{i-1} = (1-a) C y + a C^2 y ; z += alpha_i y_i
    for (int m = 1; m < a.m; ++m) {
      C(stage(y), w1);
      if (a.a != 0.0) {
        C(stage(w1), w2);
        const T om = (T)(1.0 - a.a);
#pragma unroll
        for (int s = 0; s < S; ++s) y[s] = om * w1[s] + av * w2[s];
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) y[s] = w1[s];
      }
      const T al = (T)a.alpha[m];
#pragma unroll
      for (int s = 0; s < S; ++s) z[s] += al * y[s];
    }
  }

  // Stage x (float64, per element) across both buffers; the caller must make
  // sure nobody still reads the T buffers.
  __device__ __forceinline__ const double* stage_d(const double (&x)[S]) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) sh.vd[in.pidx(s)] = x[s];
    __syncthreads();
    return sh.vd;
  }

  // Float64 residual of the record: r = b - A x, x staged in LDS.
  __device__ __forceinline__ double resid(const SolveArgs& a, const double* xs,
                                          int s) {
    const int n = in.n, k = in.k[s], i = in.i[s];
    const size_t row = (size_t)(in.r0 + k);
    double acc = 0.0;
    const size_t nn = (size_t)n * n;
    size_t base = row * nn + (size_t)i * n;
    for (int j = 0; j < n; ++j)
      acc += rec_load(a.D, base + j, a.dtype) * xs[k * n + j];
    const size_t oblk = (size_t)(in.r0 - in.inst);  // first O block
    if (k > 0) {
      size_t ob = (oblk + k - 1) * nn;
      for (int j = 0; j < n; ++j)
        acc += rec_load(a.O, ob + (size_t)j * n + i, a.dtype) *
               xs[(k - 1) * n + j];
    }
    if (k < in.N - 1) {
      size_t ob = (oblk + k) * nn + (size_t)i * n;
      for (int j = 0; j < n; ++j)
        acc += rec_load(a.O, ob + j, a.dtype) * xs[(k + 1) * n + j];
    }
    return a.b[row * n + i] - acc;
  }
};

__device__ __forceinline__ void write_info(bt_info* info, int status,
                                           int iters, int outer, int fail,
                                           double relres, double relres_true,
                                           int64_t gemv_exec = 0,
                                           int64_t gemv_paper = 0) {
  if (threadIdx.x == 0) {
    info->status = status;
    info->iters = iters;
    info->outer = outer;
    info->fail_index = fail;
    info->relres = relres;
    info->relres_true = relres_true;
    info->gemv_exec = gemv_exec;
    info->gemv_paper = gemv_paper;
  }
}

// ------------------------------------------------------------------------
// One system, BT_F64 or BT_F32 (no refinement).
// ------------------------------------------------------------------------
template <typename T, int NT, int S>
__device__ __forceinline__ void solve_direct(const SolveArgs& a, Shared<T>& sh,
                             const Inst<T, NT, S>& in) {
  Ops<T, NT, S> op(sh, in);
  const double* b = a.b + in.r0 * in.n;
  double* x = a.x + in.r0 * in.n;
  bt_info* info = a.info + in.inst;

  // ||b||^2; from an initial guess x0 (held in x on entry) the iteration
  // solves for the correction: r0 = b - A x0 in float64 from the record
  T r[S], xh[S], p[S], q[S], z[S], t[S];
  double x0[S], r0[S];
  double nbp = 0.0, nrp = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double bv = in.act[s] ? b[in.pidx(s)] : 0.0;
    nbp += bv * bv;
    x0[s] = a.warm && in.act[s] ? x[in.pidx(s)] : 0.0;
    r0[s] = bv;
  }
  if (a.warm) {
    const double* xd = op.stage_d(x0);
    ++op.nrs;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) {
        r0[s] = op.resid(a, xd, s);
        nrp += r0[s] * r0[s];
      }
  }
  const double nb2 = op.sumd(nbp);
  const double nr02 = a.warm ? op.sumd(nrp) : nb2;
  __syncthreads();  // the T buffers overlap the float64 view
  // rhat = L^{-1} r0, r0 scaled by a power of two to norm in [1, 2) (exact;
  // keeps float32 iterations clear of underflow and overflow)
  const double sc = bt_unit_scale(nr02), unscale = 1.0 / sc;
  {
    T bt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) bt[s] = (T)(r0[s] * sc);
    const T* bs = op.stage(bt);
    ++op.ntr;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      r[s] = in.act[s] ? apply_lower<T>(in.Li, bs, in.n, in.k[s], in.i[s])
                       : T(0);
      xh[s] = T(0);
    }
  }
  if (!(nb2 < INFINITY)) {  // NaN or Inf in b
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) x[in.pidx(s)] = 0.0;
    write_info(info, BT_ENONFINITE, 0, 1, -1, NAN, NAN);
    return;
  }
  if (nb2 == 0.0) {
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) x[in.pidx(s)] = 0.0;
    write_info(info, BT_OK, 0, 1, -1, 0.0, 0.0);
    return;
  }
  const double tol2 = a.tol * a.tol * nb2;

  int status = BT_NOT_CONVERGED, it = 0;
  double nr2 = nr02;
  if (nr02 <= tol2) status = BT_OK;  // the test before any step
  // t = L r is only needed for BT_PC_NONE at the start (r = rhat, L r = r0)
  if (a.pc == BT_PC_NONE) {
#pragma unroll
    for (int s = 0; s < S; ++s) t[s] = in.act[s] ? (T)(r0[s] * sc) : T(0);
  }
  op.precond(a, r, nullptr, t, z);
  double rho = op.dot(r, z);
#pragma unroll
  for (int s = 0; s < S; ++s) p[s] = z[s];
  if (status == BT_NOT_CONVERGED && !(rho > 0.0))
    status = (rho == rho) ? BT_EBREAKDOWN : BT_ENONFINITE;

  while (status == BT_NOT_CONVERGED && it < a.maxit) {
    // q = Ahat p = p - C p
    op.C(op.stage(p), q);
#pragma unroll
    for (int s = 0; s < S; ++s) q[s] = p[s] - q[s];
    const double sigma = op.dot(p, q);
    if (!(sigma > 0.0)) {
      status = (sigma == sigma) ? BT_EBREAKDOWN : BT_ENONFINITE;
      break;
    }
    ++it;
    const T al = (T)(rho / sigma);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      xh[s] += al * p[s];
      r[s] -= al * q[s];
    }
    // ||r|| = ||L rhat||
    const T* rs = op.stage(r);
    ++op.ntr;
#pragma unroll
    for (int s = 0; s < S; ++s)
      t[s] = in.act[s] ? apply_lower<T>(in.L, rs, in.n, in.k[s], in.i[s])
                       : T(0);
    nr2 = op.dot(t, t) * (unscale * unscale);
    if (nr2 <= tol2) {
      status = BT_OK;
      break;
    }
    if (!(nr2 < INFINITY)) {
      status = BT_ENONFINITE;
      break;
    }
    if (it >= a.maxit) break;
    op.precond(a, r, rs, t, z);
    const double rho1 = op.dot(r, z);
    if (!(rho1 > 0.0)) {
      status = (rho1 == rho1) ? BT_EBREAKDOWN : BT_ENONFINITE;
      break;
    }
    const T be = (T)(rho1 / rho);
#pragma unroll
    for (int s = 0; s < S; ++s) p[s] = z[s] + be * p[s];
    rho = rho1;
  }

  // x = x0 + L^{-T} xhat, then the float64 residual of the record
  double xo[S];
  {
    const T* xs = op.stage(xh);
    ++op.ntr;
#pragma unroll
    for (int s = 0; s < S; ++s)
      xo[s] = in.act[s]
                  ? x0[s] + (double)apply_lowerT<T>(in.Li, xs, in.n, in.k[s],
                                                    in.i[s]) *
                                unscale
                  : 0.0;
  }
  const double* xd = op.stage_d(xo);
  ++op.nrs;
  double rp = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (in.act[s]) {
      x[in.pidx(s)] = xo[s];
      double rv = op.resid(a, xd, s);
      rp += rv * rv;
    }
  const double rt2 = op.sumd(rp);
  write_info(info, status, it, 1, -1, sqrt(nr2 / nb2), sqrt(rt2 / nb2),
             op.gemv_exec(), (int64_t)it * bt_gemv_g(a.pc, a.a, a.m));
}

// ------------------------------------------------------------------------
// One system, float32 inner PCG inside float64 iterative refinement.
// ------------------------------------------------------------------------
template <typename T, int NT, int S>
__device__ __forceinline__ void solve_ir(const SolveArgs& a, Shared<T>& sh,
                         const Inst<T, NT, S>& in) {
  Ops<T, NT, S> op(sh, in);
  const double* b = a.b + in.r0 * in.n;
  double* x = a.x + in.r0 * in.n;
  bt_info* info = a.info + in.inst;

  double x64[S], r64[S];
  double nbp = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double bv = in.act[s] ? b[in.pidx(s)] : 0.0;
    r64[s] = bv;
    x64[s] = a.warm && in.act[s] ? x[in.pidx(s)] : 0.0;  // initial guess
    nbp += bv * bv;
  }
  const double nb2 = op.sumd(nbp);
  if (!(nb2 < INFINITY) || nb2 == 0.0) {
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s]) x[in.pidx(s)] = 0.0;
    if (nb2 == 0.0) write_info(info, BT_OK, 0, 0, -1, 0.0, 0.0);
    else write_info(info, BT_ENONFINITE, 0, 0, -1, NAN, NAN);
    return;
  }
  const double tol2 = a.tol * a.tol * nb2;
  const double itol2 = a.inner_tol * a.inner_tol;
  int status = BT_NOT_CONVERGED, total = 0, outer = 0;
  double nr2 = nb2;
  double nr2_prev = INFINITY;  // before the last correction
  double unscale = 1.0;  // 1 / the scale of the current inner solve
  T r[S], d[S], p[S], q[S], z[S], t[S];
#pragma unroll
  for (int s = 0; s < S; ++s) t[s] = T(0);

  for (;;) {
    if (outer > 0 || a.warm) {
      const double* xd = op.stage_d(x64);
      ++op.nrs;
      double rp = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (in.act[s]) {
          r64[s] = op.resid(a, xd, s);
          rp += r64[s] * r64[s];
        }
      nr2 = op.sumd(rp);
      __syncthreads();  // the T buffers overlap the float64 view
    }
    if (nr2 <= tol2) {
      status = BT_OK;
      break;
    }
    if (!(nr2 < INFINITY)) {
      status = BT_ENONFINITE;
      break;
    }
    // a correction that cut the float64 residual by less than 2x: the
    // float32 operator is too coarse for this system
    if (outer > 0 && nr2 > 0.25 * nr2_prev) {
      status = BT_ESTAGNATED;
      break;
    }
    if (outer >= a.max_outer || total >= a.maxit) break;
    nr2_prev = nr2;
    ++outer;

    // inner system: Ahat dhat = L^{-1} r64, the residual scaled by a power
    // of two to norm in [1, 2) before it is rounded to the inner precision
    const double sc = bt_unit_scale(nr2);
    unscale = 1.0 / sc;
    {
      T rt[S];
#pragma unroll
      for (int s = 0; s < S; ++s) rt[s] = (T)(r64[s] * sc);
      const T* rs = op.stage(rt);
      ++op.ntr;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        r[s] = in.act[s] ? apply_lower<T>(in.Li, rs, in.n, in.k[s], in.i[s])
                         : T(0);
        d[s] = T(0);
      }
    }
    if (a.pc == BT_PC_NONE) {
#pragma unroll
      for (int s = 0; s < S; ++s) t[s] = (T)(r64[s] * sc);
    }
    const double n0 = op.dot(r, r);
    const double itarget = itol2 * n0;
    op.precond(a, r, nullptr, t, z);
    double rho = op.dot(r, z);
#pragma unroll
    for (int s = 0; s < S; ++s) p[s] = z[s];
    int inner = 0;
    while (rho > 0.0 && total < a.maxit) {
      op.C(op.stage(p), q);
#pragma unroll
      for (int s = 0; s < S; ++s) q[s] = p[s] - q[s];
      const double sigma = op.dot(p, q);
      if (!(sigma > 0.0)) break;
      ++inner;
      ++total;
      const T al = (T)(rho / sigma);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        d[s] += al * p[s];
        r[s] -= al * q[s];
      }
      const double rr = op.dot(r, r);
      if (rr <= itarget || total >= a.maxit) break;
      const T* rs = nullptr;
      if (a.pc == BT_PC_NONE) {
        rs = op.stage(r);
        ++op.ntr;
#pragma unroll
        for (int s = 0; s < S; ++s)
          t[s] = in.act[s] ? apply_lower<T>(in.L, rs, in.n, in.k[s], in.i[s])
                           : T(0);
      }
      op.precond(a, r, rs, t, z);
      const double rho1 = op.dot(r, z);
      if (!(rho1 > 0.0)) break;
      const T be = (T)(rho1 / rho);
#pragma unroll
      for (int s = 0; s < S; ++s) p[s] = z[s] + be * p[s];
      rho = rho1;
    }
    if (inner == 0) {  // no progress possible in float32
      status = BT_EBREAKDOWN;
      break;
    }
    // x64 += L^{-T} dhat (undoing the scale)
    const T* ds = op.stage(d);
    ++op.ntr;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (in.act[s])
        x64[s] += (double)apply_lowerT<T>(in.Li, ds, in.n, in.k[s], in.i[s]) *
                  unscale;
  }

#pragma unroll
  for (int s = 0; s < S; ++s)
    if (in.act[s]) x[in.pidx(s)] = x64[s];
  write_info(info, status, total, outer, -1, sqrt(nr2 / nb2),
             sqrt(nr2 / nb2), op.gemv_exec(),
             (int64_t)total * bt_gemv_g(a.pc, a.a, a.m));
}

// ------------------------------------------------------------------------
// z = M^{-1} r once.
// ------------------------------------------------------------------------
template <typename T, int NT, int S>
__device__ __forceinline__ void precond_once(const SolveArgs& a, Shared<T>& sh,
                             const Inst<T, NT, S>& in) {
  Ops<T, NT, S> op(sh, in);
  const double* rin = a.b + in.r0 * in.n;
  double* zout = a.x + in.r0 * in.n;
  T r[S], z[S], t[S];
  {
    T rt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      rt[s] = in.act[s] ? (T)rin[in.pidx(s)] : T(0);
      t[s] = rt[s];  // L rhat = r
    }
    const T* rs = op.stage(rt);
#pragma unroll
    for (int s = 0; s < S; ++s)
      r[s] = in.act[s] ? apply_lower<T>(in.Li, rs, in.n, in.k[s], in.i[s])
                       : T(0);
  }
  op.precond(a, r, nullptr, t, z);
  const T* zs = op.stage(z);
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (in.act[s])
      zout[in.pidx(s)] =
          (double)apply_lowerT<T>(in.Li, zs, in.n, in.k[s], in.i[s]);
}

constexpr int MODE_DIRECT = 0, MODE_IR = 1, MODE_PRECOND = 2;

template <typename T, int NT, int S, int MODE>
__global__ void __launch_bounds__(NT) k_solve(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using Acc = typename AccOf<T>::type;
  Shared<T> sh;
  sh.vb0 = (T*)smem;
  sh.vb1 = sh.vb0 + S * NT;
  sh.vd = (double*)smem;
  unsigned char* tail = smem + 2 * sizeof(T) * S * NT;
  if (2 * sizeof(T) < sizeof(double)) tail = smem + sizeof(double) * S * NT;
  sh.redT = (Acc*)tail;
  sh.redD = (AccD*)(tail + sizeof(Acc) * SLOTS * (NT / 64));
  sh.cur = 0;
  sh.slotT = 0;
  sh.slotD = 0;
  __shared__ int s_q;

  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd(&a.ctr[0], 1);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= a.B) break;
    const int which = a.order[q];
    // float64 fallback pass: the other systems keep their result
    bt_info prev{};
    if constexpr (MODE == MODE_DIRECT) {
      if (a.only_stagnated) {
        prev = a.info[which];
        if (prev.status != BT_ESTAGNATED) continue;
      }
    }
    Inst<T, NT, S> in;
    in.init(a, which);
    if (a.fail[which] != BT_NO_FAIL) {
      double* x = a.x + in.r0 * in.n;
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (in.act[s]) x[in.pidx(s)] = 0.0;
      if constexpr (MODE != MODE_PRECOND)
        write_info(a.info + which, BT_ENOTSPD, 0, 0, a.fail[which], NAN, NAN);
      continue;
    }
    if constexpr (MODE == MODE_PRECOND) {
      precond_once<T, NT, S>(a, sh, in);
    } else if constexpr (MODE == MODE_IR) {
      solve_ir<T, NT, S>(a, sh, in);
    } else {
      solve_direct<T, NT, S>(a, sh, in);
      if (a.only_stagnated && threadIdx.x == 0) {
        // thread 0 wrote the float64 outcome; the float32 steps count too
        bt_info* inf = a.info + which;
        inf->iters += prev.iters;
        inf->outer = prev.outer + 1;
        inf->gemv_exec += prev.gemv_exec;
        inf->gemv_paper += prev.gemv_paper;
      }
    }
    __syncthreads();
  }
  // The last workgroup to leave rewinds the queue for the next launch.
  if (threadIdx.x == 0) {
    __threadfence();
    const int done = atomicAdd(&a.ctr[1], 1);
    if (done == (int)gridDim.x - 1) {
      atomicExch(&a.ctr[0], 0);
      atomicExch(&a.ctr[1], 0);
    }
  }
}

template <typename T, int NT, int S>
size_t smem_bytes() {
  using Acc = typename AccOf<T>::type;
  size_t vec = 2 * sizeof(T) * S * NT;
  if (vec < sizeof(double) * S * NT) vec = sizeof(double) * S * NT;
  return vec + (sizeof(Acc) + sizeof(AccD)) * SLOTS * (NT / 64);
}

template <typename T, int NT, int S, int MODE>
hipError_t launch_mode(const SolveArgs& a, int grid, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  const size_t sm = smem_bytes<T, NT, S>();
  const hipError_t e = lds_limit((const void*)k_solve<T, NT, S, MODE>, sm, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve<T, NT, S, MODE>), dim3(grid), dim3(NT), sm, st,
                     a);
  return hipGetLastError();
}

template <typename T, int NT, int S>
hipError_t launch(const SolveArgs& a, int grid, hipStream_t st) {
  if (a.mode == 1) return launch_mode<T, NT, S, MODE_PRECOND>(a, grid, st);
  if constexpr (sizeof(T) == sizeof(float)) {
    if (a.ir) return launch_mode<T, NT, S, MODE_IR>(a, grid, st);
  }
  return launch_mode<T, NT, S, MODE_DIRECT>(a, grid, st);
}

// Co-resident workgroups of the solve kernel on the whole device (the grid
// never needs more: workgroups pull systems from the queue).
template <typename T, int NT, int S>
int max_grid() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess)
    cus = 256;
  const void* fn = sizeof(T) == sizeof(float)
                       ? (const void*)k_solve<T, NT, S, MODE_IR>
                       : (const void*)k_solve<T, NT, S, MODE_DIRECT>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, NT,
                                                   smem_bytes<T, NT, S>()) !=
          hipSuccess ||
      per < 1)
    per = 1;
  return cus * per;
}

struct Entry {
  KernelConfig cfg;
  hipError_t (*launch)(const SolveArgs&, int, hipStream_t);
  int (*grid)();
};

#define BT_ENTRY(T, NT, S, P) \
  { {NT, S, P}, &launch<T, NT, S>, &max_grid<T, NT, S> }

static const Entry kEntries[] = {
    BT_ENTRY(double, 256, 1, BT_F64),  BT_ENTRY(double, 256, 2, BT_F64),
    BT_ENTRY(double, 1024, 2, BT_F64), BT_ENTRY(double, 1024, 4, BT_F64),
    BT_ENTRY(double, 1024, 8, BT_F64), BT_ENTRY(float, 256, 1, BT_F32),
    BT_ENTRY(float, 256, 2, BT_F32),   BT_ENTRY(float, 256, 4, BT_F32),
    BT_ENTRY(float, 512, 4, BT_F32),   BT_ENTRY(float, 1024, 2, BT_F32),
    BT_ENTRY(float, 1024, 3, BT_F32),  BT_ENTRY(float, 1024, 4, BT_F32),
    BT_ENTRY(float, 1024, 8, BT_F32),
};

}  // namespace btk

int bt_num_kernel_configs() {
  return (int)(sizeof(btk::kEntries) / sizeof(btk::kEntries[0]));
}

const KernelConfig& bt_kernel_config_at(int i) { return btk::kEntries[i].cfg; }

hipError_t bt_launch_solve(int cfg, const SolveArgs& a, int grid,
                           hipStream_t s) {
  return btk::kEntries[cfg].launch(a, grid, s);
}

int bt_solve_max_grid(int cfg) { return btk::kEntries[cfg].grid(); }
