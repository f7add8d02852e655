/*
 * btpcg — preconditioned conjugate gradient for SPD block-tridiagonal systems
 * on AMD Instinct MI355X (gfx950).
 *
 * Problem (Yang, Ohtsuka, Plancher, Jones, arXiv 2503.15269, Section II-A,
 * eq. (1)): solve A x = b where A is symmetric positive definite and block
 * tridiagonal with N diagonal blocks D_k (n x n, SPD) and upper blocks
 * O_k = A[k][k+1] (n x n, k = 0..N-2); the lower blocks are O_k^T. All
 * blocks are dense.
 *
 * Preconditioner: the parametric multi-splitting polynomial preconditioner
 *   M_m^{-1} = (I + alpha_1 H_ab + ... + alpha_{m-1} H_ab^{m-1}) G_ab
 * (Section III-A, eq. Mabinv; Section III-E, eq. Mminv-polynomial-
 * coefficients) with the weights (a, b) of the diagonal and the two stair
 * splittings on the admissible set 2a + b = 1, a >= 0, b >= -1 (Section
 * III-C, the set C_g). The optimal weights are (a, b) = (1, -1) (Theorem 3.6).
 *
 * Layouts (all row-major, all device memory unless stated):
 *   D : [R][n][n]   diagonal blocks of every instance, rows concatenated
 *   O : [R-B][n][n] upper blocks; instance i owns blocks
 *                   offsets[i]-i .. offsets[i+1]-i-2
 *   b, x, r, z, g, lambda : [R][n] float64
 *   dD : [R][n][n] float64, dO : [R-B][n][n] float64
 * where B is the number of independent instances and R the total number of
 * block rows; instance i owns rows offsets[i] .. offsets[i+1]-1.
 * D and O are the system of record, in float64 or float32 (``dtype``);
 * float32 values are promoted exactly wherever double precision is used.
 *
 * Ownership: every buffer, including the workspace, belongs to the caller.
 * A handle only refers to them: D, O and the workspace must stay alive and
 * unchanged while the handle is used. The library never allocates device
 * memory. The handle itself is a small host object freed by bt_destroy.
 *
 * Execution: every call that takes a stream enqueues its work on that
 * stream (a hipStream_t; NULL is the null stream) and returns without
 * waiting. The return value reports argument validation and launch errors
 * only. Per-instance outcomes (convergence, iteration counts, a failed
 * factorisation) are written by the device into a bt_info array. Calls on one
 * handle must be ordered on one stream; two calls in flight at once on the
 * same handle share its scratch counters and race.
 */
#ifndef BTPCG_H
#define BTPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (return values and bt_info.status). */
#define BT_OK 0             /* converged / success */
#define BT_NOT_CONVERGED 1  /* iteration cap reached; x holds the last iterate */
#define BT_EINVAL (-1)      /* invalid argument (sizes, pointers, parameters) */
#define BT_ENOTSPD (-2)     /* Cholesky of a diagonal block failed: A not SPD */
#define BT_EBREAKDOWN (-3)  /* p'Ap <= 0 or r'z <= 0: A or M^{-1} not SPD */
#define BT_ENONFINITE (-4)  /* a non-finite value appeared */
#define BT_EHIP (-5)        /* HIP runtime error */
#define BT_ENOSPACE (-6)    /* workspace too small */
#define BT_ETIMEOUT (-7)    /* bt_solve_grid: a grid barrier waited longer
                               than its limit (bt_set_grid_wait) and the
                               solve gave up; x is not a solution */
#define BT_ESTAGNATED (-8)  /* float32 + refinement: a refinement step
                               reduced the float64 residual by less than a
                               factor 2 (the float32 operator is too coarse
                               for the system's conditioning); x holds the
                               last iterate. With bt_params.fallback_f64 set,
                               bt_solve and bt_solve_batched finish such a
                               system in float64 instead. */

/* Arithmetic of the iteration. */
#define BT_F64 0     /* float64 throughout */
#define BT_F32 1     /* float32 iteration (dot products of float32
                        vectors summed in float64); no refinement */
#define BT_F32_IR 2  /* float32 inner PCG inside a float64 iterative
                        refinement on the system of record */
#define BT_BF16X2_IR 3 /* as BT_F32_IR; in addition the off-diagonal blocks are
                        kept split as bfloat16 pairs (hi + lo) for the
                        many-right-hand-side solve, whose block products run
                        on the matrix cores (hi*hi + hi*lo + lo*hi, float32
                        accumulation) */

/* Storage type of D and O. */
#define BT_DT_F64 0
#define BT_DT_F32 1

/* Preconditioner family. */
#define BT_PC_POLY 0 /* M_m^{-1} of eq. Mminv-polynomial-coefficients */
#define BT_PC_NONE 1 /* no preconditioner (plain CG; not in the paper) */

#define BT_MAX_M 8

typedef struct bt_params {
  double a, b;            /* splitting weights; 2a+b = 1, a >= 0, b >= -1.
                             (1,-1): optimal (Theorem 3.6); (0,1): block
                             Jacobi (Section III-D) */
  int m;                  /* polynomial order, 1..BT_MAX_M */
  int pc;                 /* BT_PC_POLY or BT_PC_NONE */
  double alpha[BT_MAX_M]; /* alpha[i] multiplies H^i, i = 1..m-1; alpha[0]
                             is ignored (the leading term is I) */
  int prec;               /* BT_F64, BT_F32 or BT_F32_IR */
  int max_outer;          /* BT_F32_IR: cap on refinement steps */
  double inner_tol;       /* BT_F32_IR: each inner solve stops when its
                             residual fell by this factor */
  int warm_start;         /* 0: x0 = 0. 1: x holds the initial guess x0 on
                             entry to bt_solve, bt_solve_batched,
                             bt_solve_grid and bt_solve_mrhs; PCG then starts
                             from r0 = b - A x0 (float64, from the system of
                             record) and the test stays ||r|| <= tol ||b||.
                             b = 0 still gives x = 0. bt_solve_adjoint and
                             bt_precondition ignore it. */
  int fallback_f64;       /* BT_F32_IR: 1 keeps float64 factors and scaled
                             off-diagonal blocks of every system in the
                             workspace (3 R n^2 float64 more), and
                             bt_solve / bt_solve_batched finish each system
                             whose refinement stagnated (BT_ESTAGNATED) by a
                             float64 PCG from its current iterate, on the
                             device, in the same call and stream: the
                             float64 setup and solve passes skip every
                             system that did not stagnate. 0: such a system
                             stops with BT_ESTAGNATED. Other precisions
                             ignore it. */
} bt_params;

/* Defaults: a = 1, b = -1, m = 2, alpha = {1, 7} (the paper's "PolyCoeff"
 * choice, Section V), BT_PC_POLY, BT_F64, max_outer = 30, inner_tol = 1e-4,
 * warm_start = 0, fallback_f64 = 0. */
void bt_default_params(bt_params* p);

/* Per-instance outcome, written on the device (48 bytes). */
typedef struct bt_info {
  int32_t status;      /* BT_OK, BT_NOT_CONVERGED, BT_ENOTSPD, BT_EBREAKDOWN,
                          BT_ENONFINITE, BT_ESTAGNATED, BT_ETIMEOUT */
  int32_t iters;       /* PCG iterations = products with A (summed over the
                          inner solves under BT_F32_IR) */
  int32_t outer;       /* refinement steps (BT_F32_IR), else 1 */
  int32_t fail_index;  /* block row (within the instance) of a failed D_k
                          factorisation, else -1 */
  double relres;       /* ||r|| / ||b|| seen by the final stopping test */
  double relres_true;  /* ||b - A x|| / ||b|| in float64 from the record */
  int64_t gemv_exec;   /* block-times-vector products the solve executed,
                          summed over the instance's N block rows: two per
                          row and application of the off-diagonal operator
                          (one on the first and last row), one per row and
                          triangular transform with L_k^{-1} or L_k, three
                          per row and float64 residual of the record (two on
                          the first and last row). Halo rows that a kernel
                          recomputes are not counted. 0 for the direct
                          solve. */
  int64_t gemv_paper;  /* the paper's count iters * g_a(m) of Section IV-B
                          (block gemvs per block row: g = 2m+2 at a = 0,
                          5m+1 for 0 < a < 1, 3m+3 at a = 1; 3 without
                          preconditioner, the product with A alone); 0 for
                          the direct solve */
} bt_info;

typedef struct bt_handle bt_handle;

/* Bytes of workspace for a batch: B instances with row offsets
 * ``offsets_host`` (host memory, B+1 entries, offsets[0] = 0, increasing),
 * block size n and parameters p. Returns 0 on invalid arguments. */
size_t bt_workspace_bytes(int B, const int64_t* offsets_host, int n,
                          const bt_params* p);

/* Set up a batch of B independent systems (Section IV-A: the diagonal-block
 * inverses and the off-diagonal splitting terms of the preconditioner).
 * offsets_host: host array, B+1 entries. D, O: device, see the layouts above.
 * The workspace (device, >= bt_workspace_bytes) receives the factors.
 * On success *h receives a new handle. Errors: BT_EINVAL (B < 1, n < 1 or
 * n > 64, an empty instance, an instance too large for one workgroup
 * (N_i * n above 8192 elements; allowed with BT_BF16X2_IR, whose
 * many-right-hand-side solve spans the grid, while the other calls on such
 * a handle then fail with BT_EINVAL), parameters outside C_g, m outside
 * 1..BT_MAX_M, NULL pointers),
 * BT_ENOSPACE, BT_EHIP. A non-SPD D_k is reported by the next solve
 * (status BT_ENOTSPD, fail_index). */
int bt_batch_setup(bt_handle** h, int B, const int64_t* offsets_host, int n,
                   int dtype, const void* D, const void* O,
                   const bt_params* p, void* workspace, size_t ws_bytes,
                   void* stream);

/* Recompute the factors of an existing handle from the current contents of
 * its D and O buffers (same shapes, same pointers), e.g. after the caller
 * overwrote them with a new system. Enqueues kernels only (no copies), so it
 * can be captured into a HIP graph together with a solve. A replayed capture
 * recomputes what the captured call computed: for a handle served by the
 * register-resident kernel, the blocks that kernel reads. After replays with
 * new D and O, call bt_refactor once without a graph before using the handle
 * with bt_precondition, bt_solve_grid or another kernel configuration. */
int bt_refactor(bt_handle* h, void* stream);

/* Single system: bt_batch_setup with B = 1 and offsets {0, N}. */
int bt_setup(bt_handle** h, int N, int n, int dtype, const void* D,
             const void* O, const bt_params* p, void* workspace,
             size_t ws_bytes, void* stream);

/* z = M^{-1} r for every instance (one application of the preconditioner,
 * eq. Mminv-polynomial-coefficients). r, z: device [R][n] float64. */
int bt_precondition(const bt_handle* h, const double* r, double* z,
                    void* stream);

/* Solve A x = b (eq. 1 of Section II-A) for every instance by the conjugate
 * gradient method preconditioned with M_m^{-1} (the iteration the paper
 * cites in Section I and whose per-iteration cost Section IV-B counts: one
 * product with A and one application of M_m^{-1}, evaluated as y_0 = G r,
 * y_i = H y_{i-1}), from x0 = 0 (or x0 = x under warm_start) until
 * ||b - A x|| <= tol ||b|| (recursive residual; under BT_F32_IR the test is
 * on the float64 residual of the record) or maxit iterations.
 * b, x: device [R][n] float64. info: device, B entries.
 * Errors (returned): BT_EINVAL (NULL pointers, tol < 0, maxit < 0), BT_EHIP.
 * Per-instance outcomes go to info. */
int bt_solve(const bt_handle* h, const double* b, double* x, double tol,
             int maxit, bt_info* info, void* stream);

/* Same as bt_solve; the name of the batched entry point. B independent
 * instances of eq. 1 (Section II-A), each with its own horizon N_i, run in
 * one persistent launch and each converges on its own (the paper's
 * Section IV-C counts one workgroup per block row; here one workgroup holds
 * whole instances). */
int bt_solve_batched(const bt_handle* h, const double* b, double* x,
                     double tol, int maxit, bt_info* info, void* stream);

/* Adjoint of x = A^{-1} b for an upstream gradient g = dL/dx. The solve is
 * the same preconditioned iteration as bt_solve (A is symmetric, Section
 * II-A, so A^{-T} = A^{-1}); the gradient identities are those of any
 * linear solve (the paper has no adjoint):
 * lambda = A^{-1} g,
 * dL/db = lambda, dL/dD_k = -lambda_k x_k^T,
 * dL/dO_k = -(lambda_k x_{k+1}^T + x_k lambda_{k+1}^T).
 * x, g, lambda: device [R][n]; dD: device [R][n][n]; dO: device
 * [R-B][n][n]; all float64. dD or dO may be NULL to skip them. */
int bt_solve_adjoint(const bt_handle* h, const double* x, const double* g,
                     double* lambda, double* dD, double* dO, double tol,
                     int maxit, bt_info* info, void* stream);

/* Many right-hand sides (the block products with many right-hand sides of
 * the task's precision pattern): solve A X = B for ``nrhs`` columns at once,
 * each column an independent PCG with the handle's preconditioner, the
 * operator applied to the whole [n][nrhs] panel of a block row with matrix-
 * core products. Requires a handle set up with prec BT_BF16X2_IR, B = 1,
 * n in {16, 32, 48, 64}, pc BT_PC_POLY with any splitting weights, order
 * and coefficients (BT_PC_NONE, plain CG on A, would need the factors L_k,
 * which this path does not keep: BT_EINVAL). nrhs a multiple of 16,
 * 16..BT_MRHS_MAX. At a = 1 with m <= 2 the preconditioner is fused into
 * two passes per inner iteration; otherwise it is evaluated by Horner's
 * rule from panel passes (one per application of C).
 * b, x: device [R][n][nrhs] float64 (right-hand-side index fastest).
 * info: device, nrhs entries. scratch: device, >= bt_mrhs_workspace_bytes.
 * Unlike the other calls this one waits on the stream between refinement
 * steps (convergence checks), so it cannot be captured into a graph.
 * Errors: BT_EINVAL, BT_ENOSPACE, BT_EHIP. */
#define BT_MRHS_MAX 4096
size_t bt_mrhs_workspace_bytes(const bt_handle* h, int nrhs);
int bt_solve_mrhs(const bt_handle* h, int nrhs, const double* b, double* x,
                  double tol, int maxit, bt_info* info, void* scratch,
                  size_t scratch_bytes, void* stream);

/* Direct solve by block Cholesky (block Thomas, Section IV-C: the
 * O(N n^3) sequential-in-N method the paper weighs PCG against), for every
 * instance of the handle, in float64 from the system of record:
 * S_0 = D_0, S_k = D_k - M_k M_k^T, L_k = chol(S_k), M_k = O_{k-1}^T
 * L_{k-1}^{-T}; forward and backward substitution. Independent of the
 * preconditioner parameters; n in 1..16, 24, 32, 48 or 64. For n <= 16
 * four instances share a wavefront, one per row of 16 lanes, lane c holding
 * column c of the current blocks, with values moved between columns by DPP
 * broadcasts fused into the float64 FMAs; for n = 24, one wavefront per
 * instance, lane i holding row i, with readlane broadcasts; for n = 32, 48
 * and 64, one workgroup per instance with the n^3 products on the matrix
 * cores (float64 16x16x4 MFMA tiles in LDS). No square roots are taken for
 * n <= 16 (unscaled Schur complements, pivots 1 / d).
 * b, x: device [R][n] float64. info:
 * device, B entries (status BT_OK or BT_ENOTSPD with fail_index = the block
 * row whose Schur complement is not positive definite; iters = 0; relres
 * fields NaN, not computed). scratch: device, >= bt_direct_workspace_bytes
 * (the factors of every block row, (2 n^2 + n) R float64). Asynchronous
 * on the stream.
 * Errors: BT_EINVAL (another n, NULL pointers), BT_ENOSPACE, BT_EHIP. */
size_t bt_direct_workspace_bytes(const bt_handle* h);
int bt_solve_direct(const bt_handle* h, const double* b, double* x,
                    bt_info* info, void* scratch, size_t scratch_bytes,
                    void* stream);

/* One system spread over the whole GPU (the preconditioned conjugate
 * gradient iteration of bt_solve with the preconditioner of eq.
 * Mminv-polynomial-coefficients evaluated as in Section IV-B; the parallel
 * layout follows the n_blk workgroups over block rows of Section IV-C): the
 * block rows are cut into windows spread over all CUs, so a single long
 * horizon is not confined to one workgroup and systems above the
 * single-workgroup capacity of bt_solve (N n > 8192) can be solved. One
 * persistent (cooperative) launch runs the whole solve, the refinement loop
 * included, with grid-wide barriers between the steps and every decision
 * taken on the device; the call is asynchronous on the stream. Same
 * parameters, stopping tests and results as bt_solve for a handle of one
 * system (B = 1): BT_F64 / BT_F32 iterate in that precision, BT_F32_IR (and
 * BT_BF16X2_IR) run float32 PCG inside float64 refinement on the record.
 * b, x: device [N][n] float64; info: device, 1 entry (status BT_ETIMEOUT if
 * a barrier gave up, see bt_set_grid_wait). scratch: device,
 * >= bt_grid_workspace_bytes(h) (nine vectors of the iteration precision,
 * one float64 vector, per-window partial sums and the barrier state).
 * Errors: BT_EINVAL (B != 1, NULL pointers, tol < 0, maxit < 0),
 * BT_ENOSPACE, BT_EHIP; a D_k that is not positive definite gives
 * info.status BT_ENOTSPD with fail_index. */
size_t bt_grid_workspace_bytes(const bt_handle* h);
int bt_solve_grid(const bt_handle* h, const double* b, double* x, double tol,
                  int maxit, bt_info* info, void* scratch,
                  size_t scratch_bytes, void* stream);

/* Longest wait, in seconds, of one grid barrier of bt_solve_grid on this
 * handle before the solve gives up with BT_ETIMEOUT (default 2 s; a barrier
 * normally waits microseconds). Every workgroup then returns, so the kernel
 * always ends. Errors: BT_EINVAL (NULL handle, seconds < 0 or not finite). */
int bt_set_grid_wait(bt_handle* h, double seconds);

/* bt_solve_grid for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same solve, kernels and results as bt_solve_grid, but the scratch is
 * a static device array the library holds, BT_GRID_NOALLOC_MAX_BYTES per GPU
 * (allocated with the library's code object on each GPU it runs on, kept
 * until the process ends), instead of a workspace argument. The call
 * allocates no device memory. A system whose grid scratch
 * (bt_grid_workspace_bytes) exceeds the maximum is refused with BT_ENOSPACE
 * before any work is enqueued (float64: about 100 000 unknowns N n, float32
 * and refinement: about 190 000). Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two host threads, or two streams
 * in flight) race. The current device must be the one the stream belongs
 * to. Like bt_solve_grid it is asynchronous on the stream. Errors: as
 * bt_solve_grid, plus BT_ENOSPACE for a system above the maximum. */
#define BT_GRID_NOALLOC_MAX_BYTES ((size_t)8 << 20)
int bt_solve_grid_noalloc(const bt_handle* h, const double* b, double* x,
                          double tol, int maxit, bt_info* info, void* stream);

/* Kernel configurations for the solve (workgroup size x vector elements per
 * thread), for the autotuner. bt_kernel_config_count() entries; entry i has
 * threads nt[i], elements per thread s[i] and iteration precision prec[i].
 * bt_set_kernel_config selects entry i for a handle (-1: automatic); it fails
 * with BT_EINVAL when the entry cannot hold the handle's largest instance or
 * has another precision. */
int bt_kernel_config_count(void);
int bt_kernel_config(int i, int* nt, int* s, int* prec);
int bt_set_kernel_config(bt_handle* h, int i);
int bt_get_kernel_config(const bt_handle* h);

void bt_destroy(bt_handle* h);
const char* bt_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* BTPCG_H */
