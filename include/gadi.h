/*
 * gadi.h -- C ABI of libgadi.so, a GADI-IR sparse solver for AMD MI355X (gfx950).
 *
 * Method: three-precision iterative refinement around the general
 * alternating-direction implicit (GADI) iteration (Algorithm 1, Section 2.1 of
 * Ge and Zhang, "Three-precision iterative refinement with parameter
 * regularization and prediction for solving large sparse linear systems").
 * With the Hermitian/skew-Hermitian splitting A = H + S of Section 4.1,
 * H = (A + A^T)/2, S = (A - A^T)/2, one outer sweep is
 *   1. r = b - A x                               (residual, u_f = double)
 *   2. (alpha I + H) z = r                       (CG,   u_r = inner precision)
 *   3. (alpha I + S) y = (2 - omega) alpha z     (CGNE, u_r = inner precision)
 *   4. x = x + y                                 (update, u = double)
 * repeated until ||r||_2 <= tol ||r_0||_2 (the RES of Section 4.1).
 *
 * Conventions for every entry point:
 *   - Nothing aborts or throws across the ABI; each call returns a gadi_status.
 *   - Pointers flagged "device" are HIP device pointers on the current device;
 *     "host" pointers are ordinary host memory.  Vectors are contiguous,
 *     unit-stride, length n.
 *   - Work is enqueued on the stream bound with gadi_set_stream (default: the
 *     null stream).  Calls that return results to the host synchronise that
 *     stream before returning.
 *   - Handles are not thread-safe: calls on one handle must not overlap.
 */
#ifndef GADI_H
#define GADI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GADI_OK = 0,
  GADI_EINVAL = 1,      /* bad argument or malformed CSR */
  GADI_ENOTSPD = 2,     /* an inner operator showed non-positive curvature */
  GADI_EOVERFLOW16 = 3, /* a scaled half-precision quantity left the finite range,
                           or (FP8 mode) an entry of H or S beyond the E4M3 range */
  GADI_EDIVERGED = 4,   /* non-finite residual or ||r|| > 1e6 ||r_0|| */
  GADI_EMAXIT = 5,      /* outer sweep limit reached */
  GADI_EHIP = 6,        /* a HIP runtime call failed */
  GADI_ENOMEM = 7,      /* host or device allocation failed */
  GADI_EBARRIER = 8,    /* a device-wide barrier timed out (the kernel bailed out) */
  GADI_EPRUNED = 9      /* batched with prune_dominated only: the trial was stopped because its work
                           exceeded that of a converged trial of the same system */
} gadi_status;

/* Square CSR matrix, int32 indices, float64 values, read-only and owned by the
 * caller; the library copies what it needs during gadi_setup.  Column indices
 * within a row must be strictly increasing.  on_device != 0 means the three
 * arrays are device pointers. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t* row_ptr; /* [n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz */
  const int32_t* col_idx; /* [nnz], 0 <= col < n */
  const double* val;      /* [nnz] */
  int32_t on_device;
} gadi_csr;

/* Splittings A = M + N.  Only the Hermitian/skew-Hermitian splitting of the
 * paper's experiments (Section 4.1 equation) is provided. */
typedef enum { GADI_SPLIT_HSS = 0 } gadi_splitting;

/* Precision triple (u_r, u, u_f) of Algorithm 1: u_r of the inner solves
 * (steps 2-3), u of the solution and its update (step 4), u_f of the residual
 * (step 1).  "half" inner solves store matrices and Krylov vectors in fp16 and
 * compute in fp32; a single-precision u_f computes the residual with an fp32
 * copy of A; a single-precision u stores x in fp32.  The last three modes
 * exist to reproduce the precision study of Section 4.1 (Table 3d); only
 * gadi_ir_solve accepts them (the batched sweep takes the first three).
 * GADI_PREC_FP8_IR is the FP8 storage the paper names as future work
 * (Section 5): the off-diagonal values of H and S in OCP FP8 E4M3 (sign, 4
 * exponent bits with bias 7, 3 mantissa bits, largest finite 448; rounded to
 * nearest-even from double once, unscaled), the diagonal of H and the Krylov
 * vectors in fp16, fp32 arithmetic, double u and u_f.  Entries beyond 448 in
 * magnitude give EOVERFLOW16 on the first FP8 solve of a handle. */
typedef enum {
  GADI_PREC_FP64 = 0,    /* (double, double, double): plain GADI               */
  GADI_PREC_FP16_IR = 1, /* (half, double, double)                              */
  GADI_PREC_FP32_IR = 2, /* (single, double, double)                            */
  GADI_PREC_H_D_S = 3,   /* (half, double, single)                              */
  GADI_PREC_H_S_S = 4,   /* (half, single, single)                              */
  GADI_PREC_S_S_S = 5,   /* (single, single, single)                            */
  GADI_PREC_FP8_IR = 6   /* (fp8 values / half vectors, double, double)          */
} gadi_precision;

typedef struct {
  gadi_precision prec;
  double eps_inner;   /* inner stop: ||g - K z||_2 <= eps_inner ||g||_2 (recurrence residual) */
  int32_t maxit_outer;  /* sweep limit (EMAXIT when reached)                   */
  int32_t maxit_inner;  /* per inner solve                                      */
  int32_t on_device;    /* 1: b and x are device pointers; 0: host pointers     */
  int32_t record_history; /* 1: keep RES per sweep, read with gadi_get_history  */
  int32_t prune_dominated; /* batched only: a trial stops with GADI_EPRUNED once its
                              work (phases: CG steps + 2 CGNE steps + 5 per sweep)
                              exceeds that of a converged trial of the same system;
                              the best trial of every system is unaffected */
  int32_t grid_per_system; /* batched only: alpha/omega hold nsys * ntrial values,
                              system-major (a separate trial grid per system) */
} gadi_options;

typedef struct {
  int32_t status;       /* gadi_status of the solve */
  int32_t outer_sweeps; /* corrections applied */
  int64_t inner_H;      /* total CG steps on alpha I + H */
  int64_t inner_S;      /* total CGNE steps on alpha I + S */
  double relres;        /* final ||r||_2 / ||r_0||_2 (FP64 residual with the true A) */
  double seconds;       /* device time of the solve kernel */
  double alpha, omega;  /* parameters used */
  int32_t fell_back;    /* 1 if the caller's fallback rule replaced predicted parameters */
  int64_t barriers;     /* device-wide barriers executed by the solve kernel */
  double barrier_seconds; /* time block 0 spent inside device-wide barriers */
} gadi_solve_info;

typedef struct gadi_handle gadi_handle;
typedef struct gadi_mlp gadi_mlp;

/* Fill `o` with defaults for `prec`: eps_inner 1e-6 (FP64) or 3e-2 (every
 * reduced-precision mode), maxit_outer 20000, maxit_inner 2000, host pointers,
 * no history, no pruning. */
void gadi_default_options(gadi_options* o, gadi_precision prec);

/* Validate A, form H and S (Section 4.1 splitting) on the union pattern of A and
 * A^T, pack A, H, S into the device layout and return a handle.  EINVAL on a
 * malformed CSR, n above 2^29 - 1024, more than 2^31 - 1 stored entries or an
 * unsupported splitting; ENOMEM / EHIP on allocation failure.
 * The handle owns all device memory it allocates. */
gadi_status gadi_setup(const gadi_csr* A, gadi_splitting split, gadi_handle** out);

/* Bind a hipStream_t (passed as void*) for all later work on the handle. */
gadi_status gadi_set_stream(gadi_handle* h, void* stream);

/* Run GADI-IR (Algorithm 1) from x_0 = x.  b: [n] float64, x: [n] float64 in/out
 * (host or device per opts->on_device).  alpha > 0 and 0 <= omega < 2 (the
 * convergence domain of Theorem 1), tol >= 0.  On return x holds the last
 * iterate and info (may be NULL) is filled; the return value equals
 * info->status.  EINVAL for bad parameters.
 * The whole solve is one persistent cooperative kernel launch on the handle's
 * stream.  The first solve per handle and precision also times the candidate
 * launch shapes and inner-solver forms (see gadi_solver_form) and builds the
 * half layout of H and S it reads; both allocate, so that first call must not
 * be captured in a graph.  GADI_BARRIER=relay|xcc|direct selects the device-wide
 * barrier (default direct: XCC-hierarchical without a master block); all three
 * give bit-identical results. */
gadi_status gadi_ir_solve(gadi_handle* h, const double* b, double* x, double alpha, double omega,
                          double tol, const gadi_options* opts, gadi_solve_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * gadi_ir_solve with the same kernels and results, its workspace taken from a
 * fixed file-scope device array of 256 MiB per device instead of memory the
 * handle allocates.  No hipMalloc, hipFree or allocating library call is made.
 * Restrictions: b and x are device pointers (opts->on_device must be 1; with
 * opts == NULL the FP16-IR defaults apply to device pointers), prec is
 * GADI_PREC_FP16_IR or GADI_PREC_FP64 (the operators gadi_setup stores), and
 * record_history must be 0.  The launch shape is the one gadi_ir_solve's
 * autotuner chose for this handle and precision, else one 1024-thread block per
 * compute unit with the one-reduction inner solves.  ENOMEM (nothing enqueued)
 * if the padded system needs more than the array holds: 104 bytes per padded
 * row plus 1 MiB, i.e. at most 2,573,753 padded rows.  info->seconds is not
 * measured (0).  Every call on a device shares that device's array: calls that
 * overlap on one device (several handles or streams) race; each call clears the
 * array's vectors before use and synchronises its stream before returning. */
gadi_status gadi_ir_solve_noalloc(gadi_handle* h, const double* b, double* x, double alpha, double omega,
                                  double tol, const gadi_options* opts, gadi_solve_info* info);

/* Per-block timing of the last gadi_ir_solve launch, for load-balance
 * studies: wait_seconds[i] the time block i spent inside device-wide barriers,
 * total_seconds[i] its time in the launch (host arrays of `cap` entries, either
 * may be NULL).  Returns the number of blocks filled (0 if none). */
int32_t gadi_get_block_profile(gadi_handle* h, double* wait_seconds, double* total_seconds, int32_t cap);

/* Per-block timing of each of the first 96 phases (the compute between two
 * device-wide barriers) of the last gadi_ir_solve launch: seconds[p * blocks +
 * b] for phase p and block b (blocks = gadi_solver_blocks), ids[p] the phase
 * kind (the order of gadi_get_phase_profile).  Host arrays for up to
 * max_phases phases; returns the number of phases filled. */
int32_t gadi_get_phase_block_profile(gadi_handle* h, double* seconds, int32_t* ids, int32_t max_phases);

/* RES history of the last solve with record_history = 1: copies up to `cap`
 * values (RES before each sweep) into `out` (host) and returns the count. */
int32_t gadi_get_history(gadi_handle* h, double* out, int32_t cap);

/* Many systems, many (alpha, omega) trials each, in one persistent launch.
 * hs[nsys]: handles set up beforehand; b[s], x[s]: per-system host vectors
 * (x[s] receives the last iterate of trial 0 of system s and may be NULL);
 * alpha[t], omega[t] for t < ntrial (ntrial <= 16): the same trial grid for
 * every system, or alpha[s * ntrial + t] with opts->grid_per_system.
 * info[s * ntrial + t] receives each trial's record (status GADI_EPRUNED for a
 * trial stopped by opts->prune_dominated).  Trials start from x_0 = 0.  Returns
 * GADI_OK, GADI_EMAXIT if some trial reached the sweep limit, or an error.  The
 * parameter sweep of the paper's training-set generation (Section 3.3.2) uses
 * this call. */
gadi_status gadi_ir_solve_batched(gadi_handle* const* hs, int32_t nsys, const double* const* b,
                                  double* const* x, const double* alpha, const double* omega,
                                  int32_t ntrial, double tol, const gadi_options* opts,
                                  gadi_solve_info* info);

/* One product with the packed operators, for kernel-level checks and
 * bandwidth measurement.  x, y are device pointers of length n.
 *   which = 0: y = A x               float64 in/out
 *   which = 1: y = (alpha I + H) x   fp16 in/out (half values), fp32 arithmetic
 *   which = 2: y = (I + S / alpha) x fp16 in/out, fp32 arithmetic
 *   which = 3: y = (alpha I + H) x   float64 in/out, float64 operator
 *   which = 4: y = (alpha I + H) x   fp16 in/out, E4M3 off-diagonal values of H
 *              (the FP8 mode's operator; the first FP8 call on a handle encodes
 *              them, which allocates and synchronises: not under graph capture)
 * On a uniform stencil layout H and S are read from their half layout (the
 * positive offsets only; the products are the same bit for bit), which the
 * first such call per value type builds if no solve has: that call allocates,
 * so it must not be captured in a graph either.
 * Enqueued on the bound stream; does not synchronise. */
gadi_status gadi_spmv(gadi_handle* h, int32_t which, double alpha, const void* x, void* y);

/* Copy the packed fp16 values of H (which = 1) or S (which = 2) back in CSR
 * order of the union pattern: out_val[k] for the k-th stored entry of row i in
 * ascending column order, including the diagonal.  out_rp [n+1], out_col and
 * out_val [split nnz] are host arrays; pass NULL out_col/out_val to query the
 * count through *nnz_out. */
gadi_status gadi_get_split_fp16(gadi_handle* h, int32_t which, int32_t* out_rp, int32_t* out_col,
                                uint16_t* out_val, int64_t* nnz_out);

/* Copy the E4M3 codes of the off-diagonal values of H (which = 1) or S
 * (which = 2), as the FP8 mode stores them, back in CSR order of the union
 * pattern without the diagonal: out_val[k] for the k-th off-diagonal entry of
 * row i in ascending column order.  Encodes them first if no FP8 solve or
 * product has.  out_rp [n+1], out_col, out_val [off-diagonal count] are host
 * arrays; pass NULL out_col/out_val to query the count through *nnz_out.
 * EOVERFLOW16 if an entry is beyond the E4M3 range. */
gadi_status gadi_get_split_fp8(gadi_handle* h, int32_t which, int32_t* out_rp, int32_t* out_col,
                               uint8_t* out_val, int64_t* nnz_out);

/* Predictor features (the row sums computed on the device from the packed
 * splitting): out[8] = [ln n, dim, log10 mean(beta), log10(max(beta) h/2) with
 * h = 1/(grid+1) (the cell Peclet number), log10 lambda_min(H) with
 * lambda_min(H) = dim (2 - 2 cos(pi h)) (closed form for the h^2-scaled
 * Laplacian), log10 max_i(H_ii + R_i^H) (Gershgorin bound of lambda_max(H)),
 * log10 max_i R_i^S, log10 min_i R_i^S], R_i the off-diagonal absolute row
 * sums; log10 arguments floored at 1e-12.  dim, grid and beta[dim] describe the
 * convection-diffusion problem (Section 4.1) and are caller-supplied. */
gadi_status gadi_features(gadi_handle* h, int32_t dim, int32_t grid, const double* beta, float* out);

/* ---- (alpha, omega) predictor: 8 -> 64 -> 64 -> 2 MLP, fp32, ReLU ----------
 * Stands in for the parameter-prediction step of Section 3.3.  Targets are
 * (log10 alpha, omega).  Weights are one flat fp32 vector of 4866 values in
 * the order W1[64,8], b1[64], W2[64,64], b2[64], W3[2,64], b3[2]. */
gadi_status gadi_mlp_create(uint64_t seed, gadi_mlp** out);
gadi_status gadi_mlp_destroy(gadi_mlp* m);
/* host weights in/out (4866 floats) */
gadi_status gadi_mlp_set_weights(gadi_mlp* m, const float* w);
gadi_status gadi_mlp_get_weights(gadi_mlp* m, float* w);
/* feature standardisation: x_std = (x - mu) / sd, mu/sd [8] host */
gadi_status gadi_mlp_set_norm(gadi_mlp* m, const float* mu, const float* sd);
/* Feature range [lo, hi] (host [8] each): raw features are clamped to it before
 * standardisation, so predictions never extrapolate beyond the training set.
 * gadi_train_mlp sets it to the training features' range; default unbounded. */
gadi_status gadi_mlp_set_bounds(gadi_mlp* m, const float* lo, const float* hi);
gadi_status gadi_mlp_get_bounds(gadi_mlp* m, float* lo, float* hi);
/* Read the standardisation in use (mu, sd [8] host out). */
gadi_status gadi_mlp_get_norm(gadi_mlp* m, float* mu, float* sd);
/* Forward pass on the device: X [B,8] host (raw features), Y [B,2] host out. */
gadi_status gadi_mlp_forward(gadi_mlp* m, const float* X, int32_t B, float* Y);
/* Loss (MSE over B*2 outputs) and gradient [4866] for standardised inputs
 * Xs [B,8] and targets Y [B,2] (host), computed by the device kernels. */
gadi_status gadi_mlp_loss_grad(gadi_mlp* m, const float* Xs, const float* Y, int32_t B, float* loss,
                               float* grad);
/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8) for `epochs` full-batch
 * steps on raw features X [n,8] and targets Y [n,2] (host); computes and stores
 * the standardisation and the feature range from X.  loss_out[epochs] (may be NULL) gets the loss
 * before each step.  All arithmetic runs in the device kernels. */
gadi_status gadi_train_mlp(gadi_mlp* m, const float* X, const float* Y, int32_t n, int32_t epochs,
                           float lr, float* loss_out);
/* Predict (alpha, omega) for one raw feature vector (gadi_features' layout).
 * The network's outputs are y0 = log10(alpha / alpha_ref) and y1 = omega, with
 * alpha_ref = sqrt(lambda_min(H) lambda_max(H)) = 10^((f[4] + f[5]) / 2) taken
 * from the unclamped features, so that the spectral scale follows the system
 * size even where the network's inputs are clamped to the training range.
 * alpha is clamped to [1e-3, 10] and omega to [0, 1.99]. */
gadi_status gadi_predict_params(gadi_mlp* m, const float* features, double* alpha, double* omega);

/* Release the handle and its device memory. */
gadi_status gadi_destroy(gadi_handle* h);

/* Static description of a status code. */
const char* gadi_status_str(gadi_status s);

/* Per-phase profile of the last gadi_ir_solve on the handle, measured by block
 * 0 of the solve kernel (compute time between reductions, barrier waits
 * excluded): seconds[10] and counts[10] for the phases 0 residual, 1 CG
 * start, 2 CG product, 3 CG update, 4 CGNE start, 5 CGNE first product,
 * 6 CGNE second product, 7 CGNE update, 8 solution update, 9 unused. */
gadi_status gadi_get_phase_profile(gadi_handle* h, double* seconds, int64_t* counts);

/* Device layout of the packed matrices, out[7] = {n, padded rows, off-diagonal
 * entries of the union pattern of A and A^T, stored slots (entries plus
 * padding / phantom zeros), stored slots in diagonal-style slices (no column
 * index stored), structural entries in explicit slices (int32 column each),
 * offsets per slice when every slice is diagonal-style with the same offsets
 * (4 or 6; 0 otherwise)}. */
gadi_status gadi_get_layout(gadi_handle* h, int64_t* out);

/* Launch shape of the last gadi_ir_solve on this handle: returns the number of
 * blocks and stores the threads per block in *threads (may be NULL); 0 before
 * the first solve.  The shape is chosen per handle and precision by a timed
 * trial of candidate shapes on the first solve (override with the environment
 * variables GADI_SOLVE_BLOCK, GADI_BLOCKS_PER_CU and GADI_SOLVE_FORM). */
int32_t gadi_solver_blocks(gadi_handle* h, int32_t* threads);

/* Inner-solver form of the last gadi_ir_solve on this handle (-1 before the
 * first solve): 0 Hestenes-Stiefel CG and CGNE, 1 Chronopoulos-Gear CG and
 * CGNE (one reduction per step, neighbour values recomputed), 2 pipelined CG
 * (the product on K w, one phase per step) with Craig's CGNE, 3 Hestenes-Stiefel
 * CG with Craig's CGNE.  All of them compute
 * the inner iterations of Algorithm 1; the timed trial picks one per handle and
 * precision with the launch shape (override: GADI_SOLVE_FORM). */
int32_t gadi_solver_form(gadi_handle* h);

/* ------------------------------------------------------------------------
 * GADI-AB for the continuous Sylvester equation A X + X B = C (Section 4.3):
 * GADI with L(X) = A X + X B split into M(X) = A X and N(X) = X B.  One sweep:
 *   R = C - A X - X B                      (double)
 *   (alpha I + A) Z = R                    (one tridiagonal solve per column)
 *   Y (alpha I + B) = (2 - omega) alpha Z  (one tridiagonal solve per row)
 *   X <- X + Y                             (double)
 * The inner solves run in the precision prec selects (GADI_PREC_FP64,
 * GADI_PREC_FP32_IR or GADI_PREC_FP16_IR: right-hand sides scaled by a power
 * of two and rounded to half, A and B rounded to half, fp32 arithmetic); each
 * is exact up to rounding (LU factors shared by all columns / rows, the
 * recurrences split into chunks of rows that are joined by their boundary
 * values).  Residual and update are in double. */
typedef struct gadi_sylv gadi_sylv;

/* A (m x m) and B (n x n) tridiagonal, host arrays: sub[k-1], diag[k],
 * sup[k-1] with T[i+1][i] = sub[i] and T[i][i+1] = sup[i] (copied).  EINVAL
 * for m or n outside [1, 2^15] or missing arrays. */
gadi_status gadi_sylv_setup(int32_t m, int32_t n, const double* a_sub, const double* a_diag, const double* a_sup,
                            const double* b_sub, const double* b_diag, const double* b_sup, gadi_sylv** out);
/* Solve from X (in: X_0, out: the last iterate) until ||R||_F <= tol ||R_0||_F.
 * C and X are m x n row-major doubles, host or device pointers per
 * opts->on_device; opts->prec, eps_inner (unused: the inner solves are direct),
 * maxit_outer, record_history apply.  info: sweeps, relres, device seconds;
 * inner_H / inner_S count the column and row solves.  Status as gadi_ir_solve. */
gadi_status gadi_sylv_solve(gadi_sylv* h, const double* C, double* X, double alpha, double omega, double tol,
                            const gadi_options* opts, gadi_solve_info* info);
/* RES per sweep of the last solve with record_history (as gadi_get_history). */
int32_t gadi_sylv_get_history(gadi_sylv* h, double* out, int32_t cap);
gadi_status gadi_sylv_set_stream(gadi_sylv* h, void* hip_stream);
gadi_status gadi_sylv_destroy(gadi_sylv* h);

/* ---- Gaussian-process regression of alpha on the problem size (Section 3.3) ----
 * The paper's predictor maps the size n of small systems of one structure to
 * their best alpha and extrapolates to large n.  Model (host code, double):
 *   y(x) = b0 + b1 x + f(x) + e,  f ~ GP(0, sf2 exp(-(x - x')^2 / (2 l^2))),
 *   e ~ N(0, sn2),
 * the linear mean by least squares, the GP on its residuals (none when every
 * residual is at most 1e-12 max(1, max |y|)).  l, sn2 / sf2
 * maximise the log marginal likelihood over a fixed grid (l: 25 log-spaced
 * values in [0.1 s, 10 s], s the spread of x; sn2 / sf2: 13 log-spaced values
 * in [1e-6, 1]); sf2 is profiled out.  The callers take x = log2 n,
 * y = log10 alpha. */
typedef struct gadi_gpr gadi_gpr;

/* Fit to m points (host arrays x[m], y[m], finite; 1 <= m <= 256).  On
 * success *out owns the model.  EINVAL for bad arguments or when no grid point
 * gives a positive definite kernel matrix. */
gadi_status gadi_gpr_fit(const double* x, const double* y, int32_t m, gadi_gpr** out);

/* Latent posterior mean (and standard deviation if sd is not NULL) at q host
 * points xq[q]; mean and sd are host arrays of q entries. */
gadi_status gadi_gpr_predict(const gadi_gpr* g, const double* xq, int32_t q, double* mean, double* sd);

/* out[6] = b0, b1, l, sf2, sn2, log marginal likelihood of the residuals
 * (+inf when the data are exactly linear and the GP part is zero). */
gadi_status gadi_gpr_params(const gadi_gpr* g, double* out);

gadi_status gadi_gpr_destroy(gadi_gpr* g);

#ifdef __cplusplus
}
#endif

#endif /* GADI_H */
