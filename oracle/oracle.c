/*
 * FP64 CPU oracle for PCG on SPD block-tridiagonal systems with the
 * multi-splitting polynomial preconditioner of Yang, Ohtsuka, Plancher and
 * Jones, "Polynomial and Parallelizable Preconditioning for Block Tridiagonal
 * Positive Definite Matrices" (arXiv 2503.15269).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plainly written reference
 * that the GPU library is checked against. Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark may load it. It shares no code,
 * header, table or helper with the GPU library.
 *
 * Conventions. A has N diagonal blocks D_k (n x n, SPD) and upper blocks
 * O_k = A[k][k+1] (n x n), k = 0..N-2; the lower blocks are O_k^T (eq. (1)).
 * Blocks are row-major. Block indices are 0-based here; the paper's are
 * 1-based, so the paper's even-indexed blocks are our odd k.
 * Vectors are [N][n]. Everything is double precision, plain loops, no
 * blocking or reordering beyond what each definition states.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_ENOTSPD (-2)
#define OR_EBREAKDOWN (-3)
#define OR_EINVAL (-1)

#define BLK(P, k, n) ((P) + (size_t)(k) * (size_t)(n) * (size_t)(n))
#define VEC(P, k, n) ((P) + (size_t)(k) * (size_t)(n))

/* ------------------------------------------------------------------ */
/* Dense n x n building blocks (textbook).                             */
/* ------------------------------------------------------------------ */

/* Cholesky A = L L^T; L lower triangular, zeros above. 0 or -1 if not SPD. */
static int chol(int n, const double *A, double *L) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int p = 0; p < j; ++p) s -= L[j * n + p] * L[j * n + p];
    if (!(s > 0.0)) return -1;
    double d = sqrt(s);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int p = 0; p < j; ++p) t -= L[i * n + p] * L[j * n + p];
      L[i * n + j] = t / d;
    }
  }
  return 0;
}

/* x <- L^{-1} x (forward substitution). */
static void lsolve(int n, const double *L, double *x) {
  for (int i = 0; i < n; ++i) {
    double t = x[i];
    for (int p = 0; p < i; ++p) t -= L[i * n + p] * x[p];
    x[i] = t / L[i * n + i];
  }
}

/* x <- L^{-T} x (back substitution with the transpose). */
static void ltsolve(int n, const double *L, double *x) {
  for (int i = n - 1; i >= 0; --i) {
    double t = x[i];
    for (int p = i + 1; p < n; ++p) t -= L[p * n + i] * x[p];
    x[i] = t / L[i * n + i];
  }
}

/* y += s * M x ; M n x n. */
static void gemv_acc(int n, double s, const double *M, const double *x,
                     double *y) {
  for (int i = 0; i < n; ++i) {
    double t = 0.0;
    for (int j = 0; j < n; ++j) t += M[i * n + j] * x[j];
    y[i] += s * t;
  }
}

/* y += s * M^T x. */
static void gemvt_acc(int n, double s, const double *M, const double *x,
                      double *y) {
  for (int i = 0; i < n; ++i) {
    double t = 0.0;
    for (int j = 0; j < n; ++j) t += M[j * n + i] * x[j];
    y[i] += s * t;
  }
}

/* C = A B (n x n). */
static void gemm(int n, const double *A, const double *B, double *C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int p = 0; p < n; ++p) t += A[i * n + p] * B[p * n + j];
      C[i * n + j] = t;
    }
}

/* C = A^T B. */
static void gemm_tn(int n, const double *A, const double *B, double *C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int p = 0; p < n; ++p) t += A[p * n + i] * B[p * n + j];
      C[i * n + j] = t;
    }
}

/* C = A B^T. */
static void gemm_nt(int n, const double *A, const double *B, double *C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double t = 0.0;
      for (int p = 0; p < n; ++p) t += A[i * n + p] * B[j * n + p];
      C[i * n + j] = t;
    }
}

/* Ainv = A^{-1} for SPD A, through its Cholesky factor: column j of the
 * inverse solves A c = e_j. Returns -1 if A is not SPD. */
static int inv_spd(int n, const double *A, double *Ainv, double *work) {
  double *L = work, *c = work + (size_t)n * n;
  if (chol(n, A, L)) return -1;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) c[i] = (i == j) ? 1.0 : 0.0;
    lsolve(n, L, c);
    ltsolve(n, L, c);
    for (int i = 0; i < n; ++i) Ainv[i * n + j] = c[i];
  }
  return 0;
}

static double dot(size_t len, const double *x, const double *y) {
  double s = 0.0;
  for (size_t i = 0; i < len; ++i) s += x[i] * y[i];
  return s;
}

/* ------------------------------------------------------------------ */
/* The matrix A of eq. (1).                                            */
/* ------------------------------------------------------------------ */

/* y = A x : y_k = O_{k-1}^T x_{k-1} + D_k x_k + O_k x_{k+1}. */
void or_spmv(int N, int n, const double *D, const double *O, const double *x,
             double *y) {
  for (int k = 0; k < N; ++k) {
    double *yk = VEC(y, k, n);
    for (int i = 0; i < n; ++i) yk[i] = 0.0;
    gemv_acc(n, 1.0, BLK(D, k, n), VEC(x, k, n), yk);
    if (k > 0) gemvt_acc(n, 1.0, BLK(O, k - 1, n), VEC(x, k - 1, n), yk);
    if (k < N - 1) gemv_acc(n, 1.0, BLK(O, k, n), VEC(x, k + 1, n), yk);
  }
}

/* ------------------------------------------------------------------ */
/* Direct solve: block Cholesky (block Thomas), Section IV-C.          */
/* A = L L^T with L block lower bidiagonal: diagonal blocks Lk (lower   */
/* triangular), sub-diagonal blocks W_k = O_k^T L_k^{-T}, and the       */
/* Schur recursion S_0 = D_0, S_{k+1} = D_{k+1} - W_k W_k^T.            */
/* Sequential in k, as the paper notes.                                 */
/* ------------------------------------------------------------------ */

/* Factor. Lf: [N][n][n], W: [N-1][n][n]. Returns 0, or -(k+1) if the
 * k-th Schur block is not positive definite (A not SPD). */
int or_btchol_factor(int N, int n, const double *D, const double *O,
                     double *Lf, double *W) {
  size_t nn = (size_t)n * n;
  double *S = (double *)malloc(sizeof(double) * nn);
  double *col = (double *)malloc(sizeof(double) * n);
  int rc = 0;
  memcpy(S, D, sizeof(double) * nn);
  for (int k = 0; k < N; ++k) {
    if (chol(n, S, BLK(Lf, k, n))) { rc = -(k + 1); break; }
    if (k == N - 1) break;
    /* W_k = O_k^T L_k^{-T}: row i of W_k solves L_k w = (O_k^T)_{row i}^T,
     * i.e. W_k^T = L_k^{-1} O_k, column by column. */
    const double *Ok = BLK(O, k, n);
    double *Wk = BLK(W, k, n);
    for (int j = 0; j < n; ++j) {          /* column j of L_k^{-1} O_k */
      for (int i = 0; i < n; ++i) col[i] = Ok[i * n + j];
      lsolve(n, BLK(Lf, k, n), col);
      for (int i = 0; i < n; ++i) Wk[j * n + i] = col[i]; /* transpose */
    }
    /* S_{k+1} = D_{k+1} - W_k W_k^T */
    const double *Dn = BLK(D, k + 1, n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int p = 0; p < n; ++p) t += Wk[i * n + p] * Wk[j * n + p];
        S[i * n + j] = Dn[i * n + j] - t;
      }
  }
  free(S);
  free(col);
  return rc;
}

/* Solve with the factors: L y = b forward, then L^T x = y backward. */
void or_btchol_solve(int N, int n, const double *Lf, const double *W,
                     const double *b, double *x) {
  double *y = x; /* in place */
  for (int k = 0; k < N; ++k) {
    double *yk = VEC(y, k, n);
    for (int i = 0; i < n; ++i) yk[i] = b[(size_t)k * n + i];
    if (k > 0) gemv_acc(n, -1.0, BLK(W, k - 1, n), VEC(y, k - 1, n), yk);
    lsolve(n, BLK(Lf, k, n), yk);
  }
  for (int k = N - 1; k >= 0; --k) {
    double *xk = VEC(x, k, n);
    if (k < N - 1) gemvt_acc(n, -1.0, BLK(W, k, n), VEC(x, k + 1, n), xk);
    ltsolve(n, BLK(Lf, k, n), xk);
  }
}

/* Factor and solve in one call. Returns the factor status. */
int or_btchol(int N, int n, const double *D, const double *O, const double *b,
              double *x) {
  size_t nn = (size_t)n * n;
  double *Lf = (double *)malloc(sizeof(double) * nn * N);
  double *W = (double *)malloc(sizeof(double) * nn * (N > 1 ? N - 1 : 1));
  int rc = or_btchol_factor(N, n, D, O, Lf, W);
  if (rc == 0) or_btchol_solve(N, n, Lf, W, b, x);
  free(Lf);
  free(W);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Preconditioner at the optimal weights (a,b) = (1,-1):               */
/* closed form of G_opt and H_opt, Section IV-A, eq. (GH-opt-closed-form)*/
/*   E_k   = D_k^{-1} O_k D_{k+1}^{-1}                                  */
/*   G_opt : diagonal D_k^{-1}, upper -E_k, lower -E_k^T                 */
/*   H_opt : (k,k)   E_{k-1}^T O_{k-1} + E_k O_k^T                       */
/*           (k,k+2) E_k O_{k+1}        (k+2,k) E_{k+1}^T O_k^T          */
/*   super/sub-diagonal blocks of H_opt are zero.                         */
/* ------------------------------------------------------------------ */

/* Outputs: Dinv [N], E [N-1], Hd [N], Hu [N-2], Hl [N-2] blocks.
 * Returns 0 or -(k+1) if D_k is not SPD. */
int or_setup_opt(int N, int n, const double *D, const double *O, double *Dinv,
                 double *E, double *Hd, double *Hu, double *Hl) {
  size_t nn = (size_t)n * n;
  double *work = (double *)malloc(sizeof(double) * (nn + n));
  double *T = (double *)malloc(sizeof(double) * nn);
  double *U = (double *)malloc(sizeof(double) * nn);
  int rc = 0;
  for (int k = 0; k < N; ++k)
    if (inv_spd(n, BLK(D, k, n), BLK(Dinv, k, n), work)) {
      rc = -(k + 1);
      goto done;
    }
  for (int k = 0; k < N - 1; ++k) {           /* E_k */
    gemm(n, BLK(Dinv, k, n), BLK(O, k, n), T);
    gemm(n, T, BLK(Dinv, k + 1, n), BLK(E, k, n));
  }
  for (int k = 0; k < N; ++k) {               /* Hd_k */
    double *H = BLK(Hd, k, n);
    for (size_t e = 0; e < nn; ++e) H[e] = 0.0;
    if (k > 0) {
      gemm_tn(n, BLK(E, k - 1, n), BLK(O, k - 1, n), U);
      for (size_t e = 0; e < nn; ++e) H[e] += U[e];
    }
    if (k < N - 1) {
      gemm_nt(n, BLK(E, k, n), BLK(O, k, n), U);
      for (size_t e = 0; e < nn; ++e) H[e] += U[e];
    }
  }
  for (int k = 0; k < N - 2; ++k) {
    gemm(n, BLK(E, k, n), BLK(O, k + 1, n), BLK(Hu, k, n));      /* (k,k+2) */
    /* (k+2,k): E_{k+1}^T O_k^T = (O_k E_{k+1})^T */
    gemm(n, BLK(O, k, n), BLK(E, k + 1, n), U);
    double *L = BLK(Hl, k, n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) L[i * n + j] = U[j * n + i];
  }
done:
  free(work);
  free(T);
  free(U);
  return rc;
}

/* y = G_opt r: y_k = D_k^{-1} r_k - E_{k-1}^T r_{k-1} - E_k r_{k+1}. */
void or_apply_Gopt(int N, int n, const double *Dinv, const double *E,
                   const double *r, double *y) {
  for (int k = 0; k < N; ++k) {
    double *yk = VEC(y, k, n);
    for (int i = 0; i < n; ++i) yk[i] = 0.0;
    gemv_acc(n, 1.0, BLK(Dinv, k, n), VEC(r, k, n), yk);
    if (k > 0) gemvt_acc(n, -1.0, BLK(E, k - 1, n), VEC(r, k - 1, n), yk);
    if (k < N - 1) gemv_acc(n, -1.0, BLK(E, k, n), VEC(r, k + 1, n), yk);
  }
}

/* y = H_opt v: y_k = Hd_k v_k + Hu_k v_{k+2} + Hl_{k-2} v_{k-2}. */
void or_apply_Hopt(int N, int n, const double *Hd, const double *Hu,
                   const double *Hl, const double *v, double *y) {
  for (int k = 0; k < N; ++k) {
    double *yk = VEC(y, k, n);
    for (int i = 0; i < n; ++i) yk[i] = 0.0;
    gemv_acc(n, 1.0, BLK(Hd, k, n), VEC(v, k, n), yk);
    if (k + 2 < N) gemv_acc(n, 1.0, BLK(Hu, k, n), VEC(v, k + 2, n), yk);
    if (k >= 2) gemv_acc(n, 1.0, BLK(Hl, k - 2, n), VEC(v, k - 2, n), yk);
  }
}

/* ------------------------------------------------------------------ */
/* The three splittings A = B - C of Section II-C, applied through their */
/* definitions (eqs. def-diagonal-splitting and def-stair-splittings).   */
/* B_d = blkdiag(D_k).                                                  */
/* B_l keeps the full block row at the paper's even rows (our odd k)    */
/*     and only D_k elsewhere; B_r is the complement pattern.           */
/* C_x = B_x - A, so (C_x v)_k = -(O_{k-1}^T v_{k-1} + O_k v_{k+1}) in  */
/* the rows where B_x keeps only D_k, and 0 in the full rows.           */
/* ------------------------------------------------------------------ */

/* Cholesky factors of every D_k, used by all B^{-1} applications. */
static int factor_diag(int N, int n, const double *D, double *Ld) {
  for (int k = 0; k < N; ++k)
    if (chol(n, BLK(D, k, n), BLK(Ld, k, n))) return -(k + 1);
  return 0;
}

static void dsolve(int n, const double *Lk, double *x) {
  lsolve(n, Lk, x);
  ltsolve(n, Lk, x);
}

/* off_k(v) = O_{k-1}^T v_{k-1} + O_k v_{k+1} (the off-diagonal row of A). */
static void offrow(int N, int n, const double *O, const double *v, int k,
                   double *out) {
  for (int i = 0; i < n; ++i) out[i] = 0.0;
  if (k > 0) gemvt_acc(n, 1.0, BLK(O, k - 1, n), VEC(v, k - 1, n), out);
  if (k < N - 1) gemv_acc(n, 1.0, BLK(O, k, n), VEC(v, k + 1, n), out);
}

/* which: 'd', 'l', 'r'. Row k of B_which is full iff full_row(which,k). */
static int full_row(char which, int k) {
  if (which == 'l') return (k % 2) == 1;  /* paper's even rows */
  if (which == 'r') return (k % 2) == 0;  /* paper's odd rows  */
  return 0;
}

/* y = B^{-1} v for B in {B_d, B_l, B_r}. In B_l and B_r the diagonal-only
 * rows are solved first; the full rows then only reference them. */
static void apply_Binv(char which, int N, int n, const double *Ld,
                       const double *O, const double *v, double *y,
                       double *tmp) {
  for (int k = 0; k < N; ++k)
    if (!full_row(which, k)) {
      memcpy(VEC(y, k, n), VEC(v, k, n), sizeof(double) * n);
      dsolve(n, BLK(Ld, k, n), VEC(y, k, n));
    }
  for (int k = 0; k < N; ++k)
    if (full_row(which, k)) {
      offrow(N, n, O, y, k, tmp);
      double *yk = VEC(y, k, n);
      for (int i = 0; i < n; ++i) yk[i] = v[(size_t)k * n + i] - tmp[i];
      dsolve(n, BLK(Ld, k, n), yk);
    }
}

/* y = C v for C in {C_d, C_l, C_r}. */
static void apply_C(char which, int N, int n, const double *O, const double *v,
                    double *y) {
  for (int k = 0; k < N; ++k) {
    double *yk = VEC(y, k, n);
    if (full_row(which, k)) {
      for (int i = 0; i < n; ++i) yk[i] = 0.0;
    } else {
      offrow(N, n, O, v, k, yk);
      for (int i = 0; i < n; ++i) yk[i] = -yk[i];
    }
  }
}

/* Parametric pair of eq. (def-GH-ab-multi-splitting), weights W_l = W_r = aI,
 * W_d = bI:
 *   G_ab r = a (B_l^{-1} r + B_r^{-1} r) + b B_d^{-1} r
 *   H_ab v = a (B_l^{-1} C_l v + B_r^{-1} C_r v) + b B_d^{-1} C_d v      */
typedef struct {
  int N, n;
  double a, b;
  const double *O;
  double *Ld;
  double *t1, *t2, *t3, *tmp;
} split_ctx;

static int split_init(split_ctx *c, int N, int n, double a, double b,
                      const double *D, const double *O) {
  size_t nn = (size_t)n * n, len = (size_t)N * n;
  c->N = N; c->n = n; c->a = a; c->b = b; c->O = O;
  c->Ld = (double *)malloc(sizeof(double) * nn * N);
  c->t1 = (double *)malloc(sizeof(double) * len);
  c->t2 = (double *)malloc(sizeof(double) * len);
  c->t3 = (double *)malloc(sizeof(double) * len);
  c->tmp = (double *)malloc(sizeof(double) * n);
  return factor_diag(N, n, D, c->Ld);
}

static void split_free(split_ctx *c) {
  free(c->Ld); free(c->t1); free(c->t2); free(c->t3); free(c->tmp);
}

static void split_G(split_ctx *c, const double *r, double *y) {
  size_t len = (size_t)c->N * c->n;
  apply_Binv('l', c->N, c->n, c->Ld, c->O, r, c->t1, c->tmp);
  apply_Binv('r', c->N, c->n, c->Ld, c->O, r, c->t2, c->tmp);
  apply_Binv('d', c->N, c->n, c->Ld, c->O, r, c->t3, c->tmp);
  for (size_t i = 0; i < len; ++i)
    y[i] = c->a * (c->t1[i] + c->t2[i]) + c->b * c->t3[i];
}

static void split_H(split_ctx *c, const double *v, double *y, double *cv) {
  size_t len = (size_t)c->N * c->n;
  apply_C('l', c->N, c->n, c->O, v, cv);
  apply_Binv('l', c->N, c->n, c->Ld, c->O, cv, c->t1, c->tmp);
  apply_C('r', c->N, c->n, c->O, v, cv);
  apply_Binv('r', c->N, c->n, c->Ld, c->O, cv, c->t2, c->tmp);
  apply_C('d', c->N, c->n, c->O, v, cv);
  apply_Binv('d', c->N, c->n, c->Ld, c->O, cv, c->t3, c->tmp);
  for (size_t i = 0; i < len; ++i)
    y[i] = c->a * (c->t1[i] + c->t2[i]) + c->b * c->t3[i];
}

/* Exported single applications (used by the tests). */
int or_apply_Gab(int N, int n, double a, double b, const double *D,
                 const double *O, const double *r, double *y) {
  split_ctx c;
  int rc = split_init(&c, N, n, a, b, D, O);
  if (rc == 0) split_G(&c, r, y);
  split_free(&c);
  return rc;
}

int or_apply_Hab(int N, int n, double a, double b, const double *D,
                 const double *O, const double *v, double *y) {
  split_ctx c;
  double *cv = (double *)malloc(sizeof(double) * (size_t)N * n);
  int rc = split_init(&c, N, n, a, b, D, O);
  if (rc == 0) split_H(&c, v, y, cv);
  split_free(&c);
  free(cv);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Preconditioner object: z = M^{-1} r,                                */
/*   M^{-1} = (I + alpha_1 H + ... + alpha_{m-1} H^{m-1}) G             */
/* (eqs. Mabinv and Mminv-polynomial-coefficients), evaluated the way   */
/* Section IV-B prescribes: y_0 = G r, y_i = H y_{i-1}, z = sum.        */
/* ------------------------------------------------------------------ */

#define OR_PC_OPT 0   /* (a,b) = (1,-1) with the closed-form blocks */
#define OR_PC_SPLIT 1 /* any (a,b), through the splitting definitions */
#define OR_PC_NONE 2  /* z = r (no preconditioner) */

typedef struct {
  int kind, N, n, m;
  double alpha[16];
  /* closed form */
  double *Dinv, *E, *Hd, *Hu, *Hl;
  /* split form */
  split_ctx sc;
  double *cv;
  double *y, *ynext;
} pc_t;

static int pc_init(pc_t *pc, int kind, int N, int n, double a, double b,
                   int m, const double *alpha, const double *D,
                   const double *O) {
  size_t nn = (size_t)n * n, len = (size_t)N * n;
  memset(pc, 0, sizeof(*pc));
  pc->kind = kind; pc->N = N; pc->n = n; pc->m = m;
  pc->alpha[0] = 1.0;
  for (int i = 1; i < m && i < 16; ++i) pc->alpha[i] = alpha ? alpha[i] : 1.0;
  pc->y = (double *)malloc(sizeof(double) * len);
  pc->ynext = (double *)malloc(sizeof(double) * len);
  if (kind == OR_PC_OPT) {
    int nm1 = N > 1 ? N - 1 : 1, nm2 = N > 2 ? N - 2 : 1;
    pc->Dinv = (double *)malloc(sizeof(double) * nn * N);
    pc->E = (double *)malloc(sizeof(double) * nn * nm1);
    pc->Hd = (double *)malloc(sizeof(double) * nn * N);
    pc->Hu = (double *)malloc(sizeof(double) * nn * nm2);
    pc->Hl = (double *)malloc(sizeof(double) * nn * nm2);
    return or_setup_opt(N, n, D, O, pc->Dinv, pc->E, pc->Hd, pc->Hu, pc->Hl);
  }
  if (kind == OR_PC_SPLIT) {
    pc->cv = (double *)malloc(sizeof(double) * len);
    return split_init(&pc->sc, N, n, a, b, D, O);
  }
  return 0;
}

static void pc_free(pc_t *pc) {
  free(pc->Dinv); free(pc->E); free(pc->Hd); free(pc->Hu); free(pc->Hl);
  if (pc->kind == OR_PC_SPLIT) split_free(&pc->sc);
  free(pc->cv); free(pc->y); free(pc->ynext);
}

static void pc_apply(pc_t *pc, const double *r, double *z) {
  size_t len = (size_t)pc->N * pc->n;
  if (pc->kind == OR_PC_NONE) {
    memcpy(z, r, sizeof(double) * len);
    return;
  }
  /* y_0 = G r */
  if (pc->kind == OR_PC_OPT) or_apply_Gopt(pc->N, pc->n, pc->Dinv, pc->E, r, pc->y);
  else split_G(&pc->sc, r, pc->y);
  memcpy(z, pc->y, sizeof(double) * len);
  for (int i = 1; i < pc->m; ++i) {
    /* y_i = H y_{i-1} */
    if (pc->kind == OR_PC_OPT)
      or_apply_Hopt(pc->N, pc->n, pc->Hd, pc->Hu, pc->Hl, pc->y, pc->ynext);
    else split_H(&pc->sc, pc->y, pc->ynext, pc->cv);
    double *t = pc->y; pc->y = pc->ynext; pc->ynext = t;
    for (size_t e = 0; e < len; ++e) z[e] += pc->alpha[i] * pc->y[e];
  }
}

/* z = M^{-1} r, one application (tests). Returns the setup status. */
int or_precond(int kind, int N, int n, double a, double b, int m,
               const double *alpha, const double *D, const double *O,
               const double *r, double *z) {
  pc_t pc;
  int rc = pc_init(&pc, kind, N, n, a, b, m, alpha, D, O);
  if (rc == 0) pc_apply(&pc, r, z);
  pc_free(&pc);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Preconditioned conjugate gradient (textbook form; the paper cites    */
/* Saad's and Nocedal-Wright's statements of it, Sections I and IV-C).  */
/* x_0 = 0, or the initial guess x0 when x0 is not NULL (then          */
/* r_0 = b - A x_0). Stops when ||r_j||_2 <= tol ||b||_2 on the         */
/* recursive residual. Iteration count = number of products A p.        */
/*                                                                      */
/* out[0] = iterations, out[1] = ||r_final||/||b||, out[2] = last ratio */
/* ||r_j||/(tol||b||), out[3] = the ratio one iteration earlier.         */
/* hist (optional, maxit+1 entries): ||r_j||/||b|| for j = 0..iters.    */
/* Returns OR_OK, OR_NOT_CONVERGED, OR_EBREAKDOWN or OR_ENOTSPD.        */
/* ------------------------------------------------------------------ */
int or_pcg(int N, int n, const double *D, const double *O, const double *bv,
           int kind, double a, double b, int m, const double *alpha,
           double tol, int maxit, double *x, double *out, double *hist,
           const double *x0) {
  size_t len = (size_t)N * n;
  pc_t pc;
  int rc = pc_init(&pc, kind, N, n, a, b, m, alpha, D, O);
  for (int i = 0; i < 4; ++i) out[i] = 0.0;
  for (size_t i = 0; i < len; ++i) x[i] = x0 ? x0[i] : 0.0;
  if (rc) { pc_free(&pc); return OR_ENOTSPD; }
  double *r = (double *)malloc(sizeof(double) * len);
  double *z = (double *)malloc(sizeof(double) * len);
  double *p = (double *)malloc(sizeof(double) * len);
  double *q = (double *)malloc(sizeof(double) * len);
  memcpy(r, bv, sizeof(double) * len);
  if (x0) { /* r_0 = b - A x_0 */
    or_spmv(N, n, D, O, x0, q);
    for (size_t i = 0; i < len; ++i) r[i] -= q[i];
  }
  double nb = sqrt(dot(len, bv, bv));
  double nr = sqrt(dot(len, r, r));
  int j = 0, status = OR_NOT_CONVERGED;
  double prev_ratio = 0.0;
  if (hist) hist[0] = (nb > 0.0) ? nr / nb : 0.0;
  if (nr <= tol * nb) {
    status = OR_OK;
    goto finish;
  }
  pc_apply(&pc, r, z);
  memcpy(p, z, sizeof(double) * len);
  double rho = dot(len, r, z);
  if (!(rho > 0.0)) { status = OR_EBREAKDOWN; goto finish; }
  for (j = 1; j <= maxit; ++j) {
    or_spmv(N, n, D, O, p, q);
    double sigma = dot(len, p, q);
    if (!(sigma > 0.0)) { status = OR_EBREAKDOWN; break; }
    double alp = rho / sigma;
    for (size_t i = 0; i < len; ++i) x[i] += alp * p[i];
    for (size_t i = 0; i < len; ++i) r[i] -= alp * q[i];
    prev_ratio = nr / (tol * nb);
    nr = sqrt(dot(len, r, r));
    if (hist) hist[j] = nr / nb;
    if (nr <= tol * nb) { status = OR_OK; break; }
    if (j == maxit) break;
    pc_apply(&pc, r, z);
    double rho1 = dot(len, r, z);
    if (!(rho1 > 0.0)) { status = OR_EBREAKDOWN; break; }
    double beta = rho1 / rho;
    for (size_t i = 0; i < len; ++i) p[i] = z[i] + beta * p[i];
    rho = rho1;
  }
  if (j > maxit) j = maxit;
finish:
  out[0] = (double)j;
  out[1] = (nb > 0.0) ? nr / nb : 0.0;
  out[2] = (nb > 0.0) ? nr / (tol * nb) : 0.0;
  out[3] = prev_ratio;
  free(r); free(z); free(p); free(q);
  pc_free(&pc);
  return status;
}

/* ------------------------------------------------------------------ */
/* Adjoint of x = A^{-1} b for a loss L(x) with gradient g = dL/dx:     */
/*   lambda = A^{-1} g (A is symmetric), dL/db = lambda,                 */
/*   dL/dA = -lambda x^T restricted to the block-tridiagonal pattern:    */
/*   dL/dD_k = -lambda_k x_k^T,                                          */
/*   dL/dO_k = -(lambda_k x_{k+1}^T + x_k lambda_{k+1}^T)                */
/* (O_k enters A at (k,k+1) and, transposed, at (k+1,k)).                */
/* lambda comes from the direct block Cholesky solve.                   */
/* ------------------------------------------------------------------ */
int or_adjoint(int N, int n, const double *D, const double *O, const double *x,
               const double *g, double *lam, double *dD, double *dO) {
  int rc = or_btchol(N, n, D, O, g, lam);
  if (rc) return rc;
  for (int k = 0; k < N; ++k) {
    double *G = BLK(dD, k, n);
    const double *lk = VEC(lam, k, n), *xk = VEC(x, k, n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) G[i * n + j] = -lk[i] * xk[j];
  }
  for (int k = 0; k < N - 1; ++k) {
    double *G = BLK(dO, k, n);
    const double *lk = VEC(lam, k, n), *xk = VEC(x, k, n);
    const double *l1 = VEC(lam, k + 1, n), *x1 = VEC(x, k + 1, n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        G[i * n + j] = -(lk[i] * x1[j] + xk[i] * l1[j]);
  }
  return 0;
}
