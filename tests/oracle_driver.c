/* Host driver that runs every entry point of the oracle on small SPD
 * block-tridiagonal systems (built here from a fixed-seed generator), for
 * the address and undefined-behaviour sanitizer build of oracle.c. Exits
 * non-zero when a call reports an unexpected status or a result is not
 * finite; the sanitizers abort on any invalid access. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void or_spmv(int N, int n, const double *D, const double *O, const double *x,
             double *y);
int or_btchol(int N, int n, const double *D, const double *O, const double *b,
              double *x);
int or_setup_opt(int N, int n, const double *D, const double *O, double *Dinv,
                 double *E, double *Hd, double *Hu, double *Hl);
void or_apply_Gopt(int N, int n, const double *Dinv, const double *E,
                   const double *r, double *y);
void or_apply_Hopt(int N, int n, const double *Hd, const double *Hu,
                   const double *Hl, const double *v, double *y);
int or_apply_Gab(int N, int n, double a, double b, const double *D,
                 const double *O, const double *r, double *y);
int or_apply_Hab(int N, int n, double a, double b, const double *D,
                 const double *O, const double *v, double *y);
int or_precond(int kind, int N, int n, double a, double b, int m,
               const double *alpha, const double *D, const double *O,
               const double *r, double *z);
int or_pcg(int N, int n, const double *D, const double *O, const double *bv,
           int kind, double a, double b, int m, const double *alpha,
           double tol, int maxit, double *x, double *out, double *hist,
           const double *x0);
int or_adjoint(int N, int n, const double *D, const double *O, const double *x,
               const double *g, double *lam, double *dD, double *dO);

static unsigned long long st = 88172645463325252ULL;
static double unif(void) { /* xorshift64, in [-1, 1) */
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return (double)(st >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int finite_all(const double *v, size_t len) {
  for (size_t i = 0; i < len; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* D_k = 4 n I + small symmetric noise, O_k = small noise: SPD by diagonal
 * dominance. */
static int run_case(int N, int n) {
  const size_t nn = (size_t)n * n, len = (size_t)N * n;
  const size_t no = N > 1 ? (size_t)(N - 1) * nn : 1;
  double *D = malloc(sizeof(double) * N * nn), *O = malloc(sizeof(double) * no);
  double *b = malloc(sizeof(double) * len), *x = malloc(sizeof(double) * len);
  double *y = malloc(sizeof(double) * len), *z = malloc(sizeof(double) * len);
  double *lam = malloc(sizeof(double) * len);
  double *dD = malloc(sizeof(double) * N * nn), *dO = malloc(sizeof(double) * no);
  double *Dinv = malloc(sizeof(double) * N * nn), *E = malloc(sizeof(double) * no);
  double *Hd = malloc(sizeof(double) * N * nn);
  double *Hu = malloc(sizeof(double) * (N > 2 ? (N - 2) * nn : 1));
  double *Hl = malloc(sizeof(double) * (N > 2 ? (N - 2) * nn : 1));
  double *hist = malloc(sizeof(double) * (10 * len + 2));
  double out[4], alpha[4] = {1.0, 1.0, 7.0, 1.0};
  int bad = 0;
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) {
        const double v = (i == j ? 4.0 * n : 0.0) + 0.5 * unif();
        D[k * nn + i * n + j] = v;
        D[k * nn + j * n + i] = v;
      }
  for (size_t e = 0; e + 1 < no + 1 && N > 1 && e < (size_t)(N - 1) * nn; ++e)
    O[e] = 0.5 * unif();
  for (size_t e = 0; e < len; ++e) b[e] = unif();
  or_spmv(N, n, D, O, b, y);
  bad |= !finite_all(y, len);
  bad |= or_btchol(N, n, D, O, b, x) != 0;
  bad |= or_setup_opt(N, n, D, O, Dinv, E, Hd, Hu, Hl) != 0;
  or_apply_Gopt(N, n, Dinv, E, b, y);
  or_apply_Hopt(N, n, Hd, Hu, Hl, y, z);
  bad |= !finite_all(z, len);
  const double ab[5][2] = {{1, -1}, {0.5, 0}, {0, 1}, {0.25, 0.5},
                           {1.0 / 3, 1.0 / 3}};
  for (int t = 0; t < 5; ++t) {
    bad |= or_apply_Gab(N, n, ab[t][0], ab[t][1], D, O, b, y) != 0;
    bad |= or_apply_Hab(N, n, ab[t][0], ab[t][1], D, O, y, z) != 0;
    bad |= !finite_all(z, len);
  }
  for (int kind = 0; kind < 3; ++kind)
    for (int m = 1; m <= 4; ++m) {
      bad |= or_precond(kind, N, n, kind == 1 ? 0.5 : 1.0,
                        kind == 1 ? 0.0 : -1.0, m, alpha, D, O, b, z) != 0;
      const int rc = or_pcg(N, n, D, O, b, kind, kind == 1 ? 0.5 : 1.0,
                            kind == 1 ? 0.0 : -1.0, m, alpha, 1e-10,
                            (int)(10 * len), x, out, hist, NULL);
      bad |= rc != 0;
      bad |= or_pcg(N, n, D, O, b, kind, 1.0, -1.0, m, alpha, 1e-10,
                    (int)(10 * len), z, out, NULL, x) != 0; /* from x0 */
    }
  bad |= or_adjoint(N, n, D, O, x, b, lam, dD, dO) != 0;
  bad |= !finite_all(dD, (size_t)N * nn);
  free(D); free(O); free(b); free(x); free(y); free(z); free(lam); free(dD);
  free(dO); free(Dinv); free(E); free(Hd); free(Hu); free(Hl); free(hist);
  return bad;
}

int main(void) {
  const int cases[][2] = {{1, 1}, {1, 5}, {2, 1}, {2, 3}, {3, 2}, {7, 4},
                          {16, 6}, {9, 12}};
  for (size_t c = 0; c < sizeof cases / sizeof cases[0]; ++c)
    if (run_case(cases[c][0], cases[c][1])) {
      fprintf(stderr, "case N=%d n=%d failed\n", cases[c][0], cases[c][1]);
      return 1;
    }
  puts("oracle driver ok");
  return 0;
}
