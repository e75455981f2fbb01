/*
 * mlpcp.h -- multilevel principal component pursuit on AMD MI355X (gfx950).
 *
 * C ABI of the hot path of multilevel inexact ALM for robust PCA (PCP) and
 * for its compressive (masked) form, after Hovhannisyan, Panagakis, Parpas and
 * Zafeiriou, "Fast Multilevel Algorithms for Compressive Principle Component
 * Pursuit" (arXiv 2206.13369): every iteration restricts the m x n data to an
 * m x n_H coarse model, thresholds its singular values there, lifts the result
 * back with the prolongation and then applies the elementwise soft threshold,
 * the observation mask and the dual (gradient) step.
 *
 * Conventions shared by every entry point
 *  - Matrices are DEVICE pointers to row-major float32 storage unless noted;
 *    a leading dimension ld counts elements between consecutive rows and must
 *    be >= the number of columns.  m counts rows, n columns, m >= n is
 *    required (the paper assumes n <= m; transpose wide data first).
 *  - The caller owns every buffer.  The library keeps no per-call state; it
 *    keeps a per-device cache of the operator constants (restriction stencil
 *    and the n_H x n_H orthonormalising factor) for each (n, levels) pair it
 *    has seen, built on first use and kept until the process ends.
 *  - The restriction used is R = P (P^T P)^{-1/2}, where P is the composite
 *    linear-interpolation operator of Sec. 3.1, eq. (Rx), read through the
 *    worked n = 6 example (first row duplicated; last row = last coarse
 *    point); odd widths use vertex-centred interpolation, n_H = (n + 1) / 2.
 *    R has orthonormal columns spanning the same range as P.
 *  - "levels" counts halvings of n (levels = 0: R = I, the plain method).
 *  - Every call returns an int status (mlpcp_status): 0 = OK, > 0 = warning
 *    with valid outputs, < 0 = error; outputs are undefined after an error.
 *    All arguments are validated on the host before anything is launched, so
 *    a call with invalid arguments touches no GPU state.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).
 *    restrict / prolong / shrink are asynchronous on it.  The solvers and
 *    svt_prox synchronise it (the host loop reads the feasibility gap and the
 *    rank every iteration).
 *  - The solvers' host loops read each iteration's statistics from a record
 *    the device writes to pinned, host-mapped memory, spinning on the host
 *    thread until it arrives: each host thread that runs a solver holds one
 *    such record (a page of pinned memory) from its first solve until the
 *    process ends.  If that allocation fails the statistics are copied back
 *    instead.  Solves from different host threads on different streams may
 *    run at the same time.
 */
#ifndef MLPCP_H
#define MLPCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLPCP_OK = 0,
  MLPCP_NOT_CONVERGED = 1,    /* warning: max_iter reached, outputs valid      */
  MLPCP_E_INVALID_ARG = -1,   /* NULL pointer, non-positive lambda/tol, ...     */
  MLPCP_E_SHAPE = -2,         /* m < n, ld < columns, non-positive sizes        */
  MLPCP_E_LEVELS = -3,        /* levels < 0 or too deep for n (n_H < 1)         */
  MLPCP_E_NONFINITE = -4,     /* NaN/Inf in an observed entry of D, S0 or Y0,   */
                              /* or the feasibility gap became NaN or Inf       */
  MLPCP_E_EIG = -5,           /* the Jacobi eigensolver hit its sweep cap       */
  MLPCP_E_WORKSPACE = -6,     /* caller workspace smaller than required         */
  MLPCP_E_HIP = -7,           /* a HIP runtime call failed                       */
  MLPCP_E_UNSUPPORTED = -8    /* option outside the implemented set             */
} mlpcp_status;

/* Arithmetic of the two products of the coarse SVT (the precision form):
 *   MLPCP_FP32    Gram M_P^T M_P from float32 operands with float64 products and sums;
 *                 reconstruction N = M_P K on float32 MFMA (tall path) or with
 *                 float64 sums (wider coarse models).
 *   MLPCP_BF16X3  reconstruction in split bfloat16: x = hi + lo, each product taken
 *                 as hi*hi + hi*lo + lo*hi on MFMA with float32 accumulation.  The
 *                 Gram is split the same way while the threshold tau is far enough
 *                 above the rounding floor of the split product (tau^2 / trace of the
 *                 coarse Gram above a bound set by the unit roundoff and m, n_H), and
 *                 takes the MLPCP_FP32 path below it, so the singular values near
 *                 tau, which decide the rank, keep float32-data accuracy.
 *   MLPCP_BF16    as MLPCP_BF16X3, with one more tier on top: the Gram operands are
 *                 rounded to plain bfloat16 while tau is far above that rounding.
 * The eigensolve, the threshold and the rank decision stay in float64, the
 * elementwise update in float32.  The split reconstruction applies on the tall path
 * (n_H <= 64, multilevel); wider coarse models keep their float64 sums.
 * mlpcp_info reports how many iterations ran each reduced-precision Gram.       */
typedef enum { MLPCP_FP32 = 0, MLPCP_BF16 = 1, MLPCP_BF16X3 = 2 } mlpcp_precision;

/* Solver options.  Penalty schedule mu_{k+1} = min(rho mu_k, mu_max_factor * mu_0)
 * (the paper only asks for an increasing sequence, Alg. 1 and Alg. 4).
 * Stopping test: feasibility gap FG = ||P_Q(D - L - S)||_F / ||P_Q D||_F <= tol,
 * the measure of the experiments section, checked every iteration.           */
typedef struct {
  int levels;              /* restriction levels (0 = plain inexact ALM)      */
  double tol;              /* FG tolerance, > 0                               */
  int max_iter;            /* > 0                                             */
  double rho;              /* penalty growth factor, >= 1                     */
  double mu_max_factor;    /* mu_max = mu_max_factor * mu_0, >= 1             */
  int prec;                /* mlpcp_precision (other values: E_INVALID_ARG)   */
  int check_every;         /* FG check cadence; 1 is implemented              */
  int r_norm;              /* restriction normalisation: 0 = R = P (P^T P)^{-1/2}  */
                           /* (orthonormal), 1 = P / ||P||_2, 2 = P (the literal */
                           /* interpolation operator; ablation of the reading)  */
  int svt_method;          /* coarse SVT on models 128..512 wide (padded):     */
                           /* 0 = the matrix-function form (f(G) = (I - tau    */
                           /* G^{-1/2})_+ by scaled Newton-Schulz products, no  */
                           /* eigenvectors) in every iteration that Gershgorin */
                           /* discs do not settle at rank 0 (tested after a    */
                           /* zero rank); 1 = always the Jacobi eigensolver.   */
                           /* Other values: E_INVALID_ARG                      */
} mlpcp_opts;

/* Per-solve report.  history (optional, caller host memory): if fg_history is
 * non-NULL it receives the FG of each iteration (history_len entries at most),
 * rank_history likewise the rank kept by each coarse SVT.                    */
typedef struct {
  int iters;               /* iterations performed                            */
  double fg;               /* final feasibility gap                           */
  int rank;                /* singular values kept by the last coarse SVT     */
  double mu_final;         /* penalty used by the last iteration              */
  double tau_margin;       /* min_i |sigma_i - tau| / tau at the last SVT; a  */
                           /* lower bound where the eigensolver certified the */
                           /* spectrum below tau^2 by Gershgorin bounds       */
                           /* instead of diagonalising it; -1 when the last   */
                           /* SVT took the matrix-function form, which does   */
                           /* not resolve the singular values one by one      */
  int eig_sweeps;          /* Jacobi sweeps of the last eigensolve (0 when    */
                           /* the certificate settled it)                     */
  double* fg_history;      /* in: optional host array                         */
  int* rank_history;       /* in: optional host array                         */
  int history_len;         /* in: length of the two arrays                    */
  int gram_bf16_iters;     /* iterations whose Gram ran in plain bfloat16     */
  int gram_split_iters;    /* iterations whose Gram ran in split bfloat16     */
  int* sweeps_history;     /* in: optional host array (history_len entries):  */
                           /* Jacobi sweeps of each iteration's eigensolve    */
  double mu0;              /* initial penalty used (the computed default when */
                           /* the call passed mu0 <= 0)                       */
  int partial_eig_iters;   /* iterations whose SVT came from the rank-        */
                           /* predicted partial eigensolve (the previous rank */
                           /* at most 56 on a model at least 1024 wide):      */
                           /* subspace iteration on a 64-column block,        */
                           /* Rayleigh-Ritz, and a Cholesky certificate that  */
                           /* no other eigenvalue of the Gram reaches tau^2;  */
                           /* the full Jacobi eigensolve otherwise            */
  int msvt_iters;          /* iterations whose SVT took the matrix-function   */
                           /* form (see mlpcp_opts.svt_method)                */
  int msvt_flags;          /* of those, iterations whose Gram norm bounds      */
                           /* exceeded the growth their step counts assumed;  */
                           /* the rest of the solve then took the eigensolver */
  int msvt_products;       /* n_H x n_H x n_H float64 products those SVTs ran  */
} mlpcp_info;

/* Fills defaults: levels 0, tol 1e-6, max_iter 500, rho 1.5, mu_max_factor 1e7,
 * FP32, check_every 1, orthonormal restriction, svt_method 0.                */
void mlpcp_default_opts(mlpcp_opts* opts);

/* Coarse width n_H after `levels` halvings of n (Sec. 3.1: composite of
 * interpolation operators); < 0 (mlpcp_status) if levels is invalid.         */
int mlpcp_coarse_dim(int n, int levels);

/* Device workspace (bytes) a solve of an m x n problem needs with these
 * options (including the default-mu0 phase); 0 if the arguments are invalid.
 * The solvers and svt_prox accept ws = NULL, in which case they allocate (and
 * free) it themselves.                                                       */
size_t mlpcp_workspace_bytes(int m, int n, const mlpcp_opts* opts);

/* Robust PCA, eq. (rpca): min ||L||_* + lambda ||S||_1 s.t. D = L + S, by
 * inexact ALM (Alg. 1, opts->levels = 0) or multilevel inexact ALM (Alg. 4).
 *  D      m x n input, leading dimension ldd.
 *  lambda weight of the l1 term, > 0.
 *  mu0    initial penalty (Alg. 1 / Alg. 4 require one).  mu0 <= 0 selects
 *         the customary default 1.25 / ||P_Q D||_2, computed on the device
 *         before the iterations (float64 Gram of P_Q D, its top eigenvalue by
 *         repeated squaring, a Rayleigh quotient; relative error below 1e-7);
 *         info->mu0 reports the value used.  NaN/Inf: MLPCP_E_INVALID_ARG.
 *  S0, Y0 optional m x n (ld = n) initial sparse part and multiplier; NULL =
 *         zeros.  They may alias the S and Y outputs.
 *  L, S   outputs, m x n, ld = n.  Y: optional output multiplier (NULL = not
 *         returned).  L, S, Y must not alias D or each other.
 *  ws     device workspace of ws_bytes >= mlpcp_workspace_bytes(), or NULL.
 *  info   optional report (may be NULL).
 * Returns MLPCP_OK when FG <= tol, MLPCP_NOT_CONVERGED after max_iter (the
 * outputs then hold the last iterate).  Degenerate and invalid data:
 *  - P_Q D = 0: L = S = 0 (Y = 0), zero iterations, MLPCP_OK;
 *  - a NaN or Inf in an observed entry of D, S0 or Y0: MLPCP_E_NONFINITE
 *    before any iteration (detected by the initial pass over the data).
 * L must not alias S0 or Y0 (it stages P_Q D for the default mu0).           */
int mlpcp_pcp_solve(int m, int n, const float* D, int ldd, float lambda, double mu0,
                    const mlpcp_opts* opts, const float* S0, const float* Y0,
                    float* L, float* S, float* Y, void* ws, size_t ws_bytes,
                    mlpcp_info* info, void* stream);

/* Compressive PCP in its constrained form (Sec. 2): find L, S with
 * P_Q[L + S] = P_Q[D], minimising ||L||_* + lambda ||P_Q S||_1, by the masked
 * (multilevel) inexact ALM: the sparse part is free off Q, so off Q the dual
 * stays zero and the coarse data carries the previous L.
 *  Q  m x n uint8 mask (ld = n): nonzero = observed.  D off Q is ignored (its
 *     values never reach the result; the memory must still be readable).
 * Outputs: L is the completed low-rank estimate (all entries); S and Y are
 * zero off Q.  Other arguments as mlpcp_pcp_solve; S0 and Y0 off Q are ignored.
 * With Q all ones the result equals mlpcp_pcp_solve's.                       */
int mlpcp_cpcp_solve(int m, int n, const float* D, int ldd, const uint8_t* Q,
                     float lambda, double mu0, const mlpcp_opts* opts,
                     const float* S0, const float* Y0, float* L, float* S, float* Y,
                     void* ws, size_t ws_bytes, mlpcp_info* info, void* stream);

/* Coarse singular value thresholding lifted back (Alg. 4, the coarse SVT and
 * its prolongation, eq. coarse-aug-lagr): L = SVT_tau(M R) R^T, the proximal
 * map of tau ||.||_* restricted to matrices whose rows lie in range(R).
 *  M m x n (ldm), tau > 0, L m x n output (ld = n), rank: optional host int
 *  receiving the number of singular values above tau.                        */
int mlpcp_svt_prox(int m, int n, const float* M, int ldm, int levels, float tau,
                   float* L, int* rank, void* ws, size_t ws_bytes, void* stream);

/* mlpcp_svt_prox without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and result as mlpcp_svt_prox, with the workspace, and
 * the restriction operator of the last (n, levels) served, in a static device array
 * of 64 MiB that the library holds on each GPU it runs on until the process ends.
 * Sizes whose operator plus workspace exceed it return MLPCP_E_WORKSPACE before
 * anything is launched.  The first call on a device looks up the array's device
 * address once; a call with a new (n, levels) rebuilds the operator in the array.
 * Every call on one GPU shares its array: calls that overlap on one GPU (other
 * threads, other streams) race and must be serialised by the caller.  Kernel timing
 * (mlpcp_profile_enable) must be off.  Synchronises the stream.               */
int mlpcp_svt_prox_static(int m, int n, const float* M, int ldm, int levels, float tau,
                          float* L, int* rank, void* stream);

/* Elementwise soft threshold S_tau[x] = sign(x) max(|x| - tau, 0) (the sparse
 * step of Alg. 1), on `count` contiguous floats.  Y may alias X.  tau >= 0.
 * NaN inputs propagate.                                                      */
int mlpcp_shrink(size_t count, const float* X, float tau, float* Y, void* stream);

/* Restriction XH = X R (m x n -> m x n_H; Alg. 4, coarse data), asynchronous.
 *  X m x n (ldx >= n), XH m x n_H (ldh >= n_H).  Coarse widths up to 1024
 *  (MLPCP_E_UNSUPPORTED beyond).                                             */
int mlpcp_restrict(int m, int n, const float* X, int ldx, int levels, float* XH, int ldh,
                   void* stream);

/* Prolongation X = XH R^T (m x n_H -> m x n; Alg. 4, lift), asynchronous.
 *  XH m x n_H (ldh >= n_H), X m x n (ldx >= n).  Coarse widths up to 512
 *  (MLPCP_E_UNSUPPORTED beyond).                                             */
int mlpcp_prolong(int m, int n, const float* XH, int ldh, int levels, float* X, int ldx,
                  void* stream);

/* ---- Differentiation form: one explicit iteration and its adjoint -------------
 * One iteration of multilevel inexact ALM (Alg. 4; Alg. 1 at levels = 0) in the
 * paper's explicit form, for unrolled (differentiable) solvers:
 *   M = D - S + Y/mu;  L = SVT_{1/mu}(M R) R^T;  S' = S_{lam/mu}[D - L + Y/mu];
 *   Y' = Y + mu (D - L - S').
 *  D m x n (ldd); S, Y m x n (ld = n), NULL = zeros; L, S_next, Y_next outputs
 *  m x n (ld = n); rank: optional host int.  Synchronises the stream.          */
size_t mlpcp_step_workspace_bytes(int m, int n, int levels);
int mlpcp_ialm_step(int m, int n, int levels, const float* D, int ldd, const float* S, const float* Y,
                    float lambda, double mu, float* L, float* S_next, float* Y_next, int* rank,
                    void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of mlpcp_ialm_step at (D, S, Y, lambda), mu held fixed.
 * Recomputes the step internally (checkpoint/recompute), then propagates the output
 * adjoints L_bar, S_bar, Y_bar (m x n, ld = n, NULL = zero) back:
 *   D_bar      (m x n, ldd)  += dLoss/dD contribution of this step (accumulated),
 *   S_bar_prev (m x n, ld n)  = dLoss/dS,   Y_bar_prev (m x n, ld n) = dLoss/dY,
 *   *lambda_bar (host)       += dLoss/dlambda contribution (NULL = not wanted).
 * The SVT adjoint is the derivative of the singular value thresholding map written
 * in the coarse singular basis; dropped singular directions enter only through
 * A v_j, so no coefficient divides by a small singular value and every coefficient
 * is bounded (sigma_i > tau >= sigma_j).  The soft-threshold adjoint is the mask
 * 1[|E| > lambda/mu] and, for lambda, -sign(E)/mu on that mask.  Synchronises.   */
int mlpcp_ialm_step_vjp(int m, int n, int levels, const float* D, int ldd, const float* S, const float* Y,
                        float lambda, double mu, const float* L_bar, const float* S_bar, const float* Y_bar,
                        float* D_bar, float* S_bar_prev, float* Y_bar_prev, double* lambda_bar,
                        void* ws, size_t ws_bytes, void* stream);

/* ---- Unconstrained CPCP by Frank-Wolfe Thresholding ---------------------------
 * eq. (cpcp):  min 1/2 ||P_Q[L + S - D]||_F^2 + lam_L ||L||_* + lam_S ||S||_1,
 * by FW-T (Alg. 3, levels = 0) or multilevel FW-T (Alg. 6, levels > 0) on the
 * epigraph form eq. (cpcp-fw): L = S = 0, t_L = t_S = 0, U = f / lam at start;
 * each iteration takes the nuclear linear oracle -u w^T (top singular pair of the
 * gradient G = P_Q[L + S - D]; ML-FWT: of the coarse gradient G R, lifted by R^T,
 * radius 1/||R||_2 = 1), the l1 oracle at the largest |G_ij|, the gates
 * lam >= -<G, M>, the exact line search over both segments (a convex quadratic
 * on the unit square), the threshold S = S_{lam_S}[S_half - P_Q[L + S_half - D]]
 * with t_S = ||S||_1, and the bounds U = f / lam.
 * Stopping: relative objective change |f_{k-1} - f_k| / f_{k-1} <= tol (the paper
 * runs to a 1e-3 tolerance without defining it).
 *  D    m x n (ldd >= n), m >= n, m * n < 2^31.
 *  Q    m x n uint8 mask (ld = n), nonzero = observed; NULL = fully observed.
 *  lam_L, lam_S > 0 (the arithmetic uses these float values).
 *  levels  0 = FW-T (power iteration for the top pair, n <= 8192 with
 *          16-byte-aligned D and L and ldd % 4 == 0, else n <= 2048);
 *          > 0 = ML-FWT, n_H <= 64, n <= 8192.  Other shapes: MLPCP_E_UNSUPPORTED.
 *  L, S outputs m x n (ld = n): the last iterate; S is zero off Q.
 *  ws   device workspace >= mlpcp_fwt_workspace_bytes(m, n, levels, Q != NULL),
 *       or NULL (allocated and freed inside).
 *  info optional report; its history arrays (host, optional) receive per
 *       iteration f, the step sizes alpha, beta and the top singular value.
 * Returns MLPCP_OK when the stopping test holds (also when P_Q D = 0: zero
 * iterations, L = S = 0), MLPCP_NOT_CONVERGED after max_iter.  Synchronises.   */
typedef struct {
  int iters;               /* iterations performed                            */
  int converged;           /* 1 if the stopping test held                     */
  double f;                /* objective f(L, S, t_L, t_S) of the last iterate */
  double t_L, t_S;         /* its epigraph variables (t_S = ||S||_1)          */
  double rel_change;       /* last |f_{k-1} - f_k| / f_{k-1}                  */
  double gap;              /* Frank-Wolfe gap <grad f, x - v> of the last step */
  long long power_steps;   /* power-iteration steps in total (FW-T)          */
  double* f_history;       /* in: optional host arrays of history_len entries */
  double* alpha_history;
  double* beta_history;
  double* sigma_history;
  int history_len;
} mlpcp_fwt_info;

size_t mlpcp_fwt_workspace_bytes(int m, int n, int levels, int masked);
int mlpcp_cpcp_fwt(int m, int n, const float* D, int ldd, const uint8_t* Q, float lam_L, float lam_S,
                   int levels, double tol, int max_iter, float* L, float* S, void* ws, size_t ws_bytes,
                   mlpcp_fwt_info* info, void* stream);

/* Static description of a status code (never NULL).                          */
const char* mlpcp_status_string(int status);

/* Kernel timing, for diagnostics and benchmarking.  Kernels are grouped into
 * classes (read() reports them in a fixed order: init_restrict, gram,
 * coarse_CGC, jacobi_pairs, jacobi_apply, jacobi_misc, svt_prep, epilogue,
 * reduce, finalize, coarse_svt_small, fw_pass, fw_power, fw_small, fw_top,
 * other).  enable(mask) resets the counters and brackets every
 * launch of class i with HIP events on the caller's stream when bit i of mask is
 * set (mask 0 = off, -1 = all); the elapsed times are accumulated per class.
 * read() copies up to `cap` classes into `out` (static names) and returns the
 * number of classes.  Each timed launch adds two event records to the stream.  */
typedef struct {
  const char* name;
  long long launches;
  double total_ms;
} mlpcp_kernel_time;

int mlpcp_profile_enable(int mask);
int mlpcp_profile_read(mlpcp_kernel_time* out, int cap);

#ifdef __cplusplus
}
#endif

#endif /* MLPCP_H */
