// Internal declarations shared by the HIP translation units of libmlpcp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/mlpcp.h"

namespace mlpcp {

// Status propagation -----------------------------------------------------------------
#define MLPCP_HIP(call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return MLPCP_E_HIP;             \
  } while (0)

#define MLPCP_TRY(call)                                   \
  do {                                                    \
    int s_ = (call);                                      \
    if (s_ < 0) return s_;                                \
  } while (0)

constexpr int kEigBlock = 32;          // Jacobi block width b; inner problems are 2b x 2b
constexpr int kEigInner = 2 * kEigBlock;
constexpr int kPad = 64;               // padding of n_H for the Gram / eigensolver tiles
constexpr int kMaxStencil = 2;         // nonzeros per fine row of the composite interpolation
constexpr int kQfWidth = 16;           // coarse widths up to this also get the dense float32 operator P C
constexpr int kMaxEigSweeps = 40;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// bfloat16 helpers for the precision form: round-to-nearest-even split x = hi + lo
__device__ __forceinline__ unsigned short f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Operator constants of the coarse model for one (n, levels) pair, on one device.
//  P (n x nH) composite interpolation:
//   rows  : fine row j -> kMaxStencil (coarse index, weight) pairs (weight 0 pads)
//   cols  : CSC, coarse column c -> fine rows col_ptr[c] .. col_ptr[c+1]
//  C = (P^T P)^{-1/2} (nH x nH, float64, row-major ld = nH), identity when levels = 0.
struct Operator {
  int n = 0, levels = 0, nH = 0;
  int max_col_nnz = 0;
  int nnz = 0;                // nonzeros of P
  bool contig = false;        // every column's fine rows are consecutive (ascending)
  int* row_idx = nullptr;     // [n * kMaxStencil]
  float* row_w = nullptr;     // [n * kMaxStencil]
  int* col_ptr = nullptr;     // [nH + 1]
  int* col_row = nullptr;     // [nnz]
  float* col_w = nullptr;     // [nnz]
  double* C = nullptr;        // [nH * nH] (nullptr when levels == 0)
  float* Qf = nullptr;        // [kQfWidth * n]: (P C)^T in float32, zero rows beyond nH (nH <= kQfWidth only)
  void* mem = nullptr;        // device block holding the tables and C (owned by the cache)
};

// Returns the cached operator for (n, levels, r_norm) on the current device, building it
// on first use (host stencil tables, then C on the GPU with the Jacobi eigensolver).
// r_norm 0: C = (P^T P)^{-1/2} (orthonormal R = P C); 1: C = I / ||P||_2; 2: C = I (the
// literal interpolation operator).
int get_operator(int n, int levels, hipStream_t stream, const Operator** out, int r_norm = 0);
// The same operator built into caller memory: `mem` (operator_bytes: the tables and C,
// kept) and `tmp` (operator_tmp_bytes: the eigensolve that forms C, free again on
// return).  Synchronises `stream`.
size_t operator_bytes(int n, int levels);
size_t operator_tmp_bytes(int n, int levels);
int build_operator_at(int n, int levels, int r_norm, hipStream_t stream, Operator* op, void* mem, void* tmp);

// Builds the composite interpolation stencil on the host (also used by host tests
// through mlpcp_coarse_dim and by get_operator).
int coarse_dim_checked(int n, int levels);
void build_stencil_host(int n, int levels, std::vector<int>& row_idx, std::vector<float>& row_w,
                        std::vector<int>& col_ptr, std::vector<int>& col_row, std::vector<float>& col_w,
                        std::vector<double>* dense_P);

// ---- symmetric eigensolver (eig.hip) ---------------------------------------------
// Workspace for an N x N problem (N multiple of kPad).
size_t eig_workspace_bytes(int N);
// A: N x N float64 symmetric (ld = N), overwritten.  On return V (N x N, ld = N) holds
// the eigenvectors as columns (unsorted), lam[i] = A_ii, perm[k] = index of the k-th
// largest eigenvalue.  n <= N is the true size (rows/cols >= n must be zero).
// warm: V holds an orthogonal starting basis on entry (e.g. the previous eigenvectors,
// identity on the padding); otherwise V is initialised to the identity.
// sweeps_out receives the number of sweeps.  Synchronises `stream`.
// cert_tau2 > 0 (N > kEigInner only): threshold certificate for an SVT at tau^2 =
// cert_tau2 -- when, at the start of a sweep, every row's Gershgorin bound
// sum_j |a_ij| lies below tau^2, all eigenvalues do and the iteration stops there (A,
// V and lam as they stand; the SVT of such a matrix is zero).  For N >= 1024 also the
// partial form: pairs of two rows certified at the start of a sweep are not rotated,
// so the certified block (all its eigenvalues below tau^2) is left undiagonalised, its
// diagonal entries in lam and its columns of V spanning that invariant subspace.
// On return gb[i] (N doubles, caller's memory) holds the bound of each certified row
// and -1 for the others (all -1 below N = 1024 unless every row is certified).
// Per-iteration statistics written on the device, read by the host once per iteration.
struct IterStats {
  double fg2;      // sum of squared residuals on Q
  double nrm2;     // ||P_Q D||_F^2 (init)
  double margin;   // min |sigma - tau| / tau
  double trace;    // sum of the coarse eigenvalues (||M_H||_F^2)
  int rank;
  int sweeps;      // Jacobi sweeps of the one-workgroup coarse SVT (-1: sweep cap hit)
  double lam_r;    // smallest eigenvalue kept (0 at rank 0)
  double lam_65;   // 65th largest eigenvalue (0 below width 65)
  int kform;       // 1: the wide reconstruction factor T holds K itself (n_H columns,
                   // the matrix-function SVT); 0: T T^T = K with `rank` columns
  int msvt_flag;   // matrix-function SVT: bit 0 / bit 1 set when its norm bound alpha /
                   // beta exceeded the cap its step counts assumed
  double msvt_alpha, msvt_beta;   // those norm bounds
};

// A record the device publishes to pinned, host-mapped memory: the values first, then,
// behind a system-scope fence, the sequence number of the request that wrote them.
struct ProbeRecord {
  double v[3];
  unsigned long long seq;
};

// Spins on host memory until *seqp == want; every 1024 polls a stream query ends the wait
// with MLPCP_E_HIP on an error, or when the stream has drained without publishing.
int wait_seq(const unsigned long long* seqp, unsigned long long want, hipStream_t s);

// Sweep count placeholder: the count is in IterStats::sweeps after the next sync.
constexpr int kSweepsOnDevice = -100;

// The whole coarse SVT of a coarse model of width n_H <= kEigInner in one workgroup:
// G_H = C G C (C null: plain, G_H = G), optional warm start from V, Jacobi, ordering,
// weights sw, T = C V_sorted diag(sw), Tt, and K = T T^T (if K is non-null); writes V,
// lam (diagonal), perm, sw and the rank / margin / trace / sweeps fields of st.
// Buffers are kEigInner x kEigInner with leading dimension ld (= kEigInner).
// certify: the threshold certificate of eig_sym at tau^2 (a matrix whose rows all have
// Gershgorin bounds below tau^2 is not diagonalised; the margin is then taken from
// the bounds).  With certify and K, the SVT operator may instead come from the
// second-order perturbation expansion around the current diagonal, tested on the warm
// start and after every Jacobi sweep (T, Tt, lam, perm, sw are then left as they are;
// V holds the rotated basis and st->sweeps the sweeps run before it).  With certify the
// basis in V (written, and read back by a warm start) is C V, not V; without it, V.
int coarse_svt_small(int nH, int ld, const double* G, const double* C, double* V, bool warm, double tau,
                     bool certify, double* lam, int* perm, double* sw, double* T, double* Tt, double* K,
                     IterStats* st, hipStream_t stream);

// Top eigenpair of C G C (G: n_H x n_H float64 Gram, ld = kEigInner, n_H <= kEigInner;
// C: n_H x n_H, ld = n_H, or null for the identity) in one workgroup: writes z = C x
// (kEigInner entries, zero past n_H) for the unit top eigenvector x, and lam = x^T (C G C) x.
int coarse_top_small(int nH, const double* G, const double* C, double* z, double* lam, hipStream_t stream);

int eig_sym(int n, int N, double* A, double* V, double* lam, int* perm, void* ws,
            hipStream_t stream, int* sweeps_out, bool warm, int sweep_hint = 0, double cert_tau2 = 0.0,
            double* gb = nullptr);

// ---- rank-predicted partial eigensolve (subspace.hip) ----------------------------------
// Workspace of svt_partial for an N x N Gram.
size_t subspace_workspace_bytes(int N);
// Whether svt_partial may be tried: N a multiple of 64, at least 128, and the previous
// rank in [1, 56].
bool subspace_eligible(int N, int r_prev);
// The eigenpairs of G (N x N, ld N, float64) above tau^2 from a 64-column block started at
// the columns perm[0..63] of V (first_iters subspace steps before the first Rayleigh-Ritz
// step), with a certificate that G has no other eigenvalue at or above tau^2.
// *ok = true: V[:, 0..r) holds them (descending), lam their values and -1 beyond, perm the
// identity, gb (N entries) -1 within the first r and the certified bound beyond,
// *trace_dev (device) = trace(G).  *ok = false: V, lam, perm, gb untouched (the caller
// runs the full eigensolver).  *iters = subspace steps taken; *ratio = the block's last
// Ritz value over its r-th (the convergence factor of the next solve's steps).
// Synchronises `s`.
int svt_partial(int N, const double* G, double tau, int first_iters, double* V, double* lam, int* perm, double* gb,
                double* trace_dev, void* ws, hipStream_t s, bool* ok, int* iters, double* ratio);
// Subspace steps for a convergence factor rho = lambda_65 / lambda_r: enough to bring the
// residual of the leading pairs down by about 1e-10.
int subspace_steps(double rho);

// ---- matrix-function SVT (msvt.hip) -----------------------------------------------------
constexpr int kMsvtMaxWidth = 512;
// Step counts and coefficients of one matrix-function SVT, fixed on the host.
struct MsvtPlan {
  double alpha_cap, beta_cap;   // norm bounds the step counts assume
  int n_sign, n_inv;            // scaled Newton-Schulz steps of the two phases
  double a_sign[64], a_inv[64];
};
// Whether an N x N Gram may take the matrix-function SVT: N a multiple of 64 in
// [128, kMsvtMaxWidth].
bool msvt_eligible(int N);
size_t msvt_workspace_bytes(int N);
// Plan for threshold tau given estimates (upper bounds) of the two norm bounds.
int msvt_plan(double tau, double alpha_est, double beta_est, MsvtPlan* mp);
// G_H = C G C (N x N, ld N; G exactly symmetric, zero past n_H; C n_H x n_H, ld n_H) on
// the matrix-function SVT's product kernel, the result exactly symmetric.  prep: (re)build
// the padded C and C^2 first.  *products (nullable) += the products launched.  No sync.
int msvt_cgc(int nH, int N, const double* G, const double* C, bool prep, double* GH, void* ws, hipStream_t s,
             int* products);
// Gershgorin certificate that every eigenvalue of G (n_H x n_H block, ld ldg) is below
// tau^2 (then st takes rank 0 in factor form and a margin bound), and the largest
// absolute row sum and the trace of G.  Synchronises `s`.
int msvt_probe(int nH, int N, const double* G, int ldg, double tau, IterStats* st, void* ws, hipStream_t s,
               bool* certified, double* gmax, double* trace, ProbeRecord* pub_host = nullptr,
               ProbeRecord* pub_dev = nullptr, unsigned long long seq = 0);
// K (N x N, ld ldk == N) = C f(G) C with f(l) = (1 - tau / sqrt(l))_+ on the eigenvalues
// of G (n_H x n_H block of an N x N buffer, ld ldg; C n_H x n_H, ld n_H, or null for the
// identity), zero beyond n_H; st: rank, trace, kform = 1, the flags and bounds.  prep:
// (re)build the padded C and C^2 kept in the workspace (once per operator).  *products
// (nullable) += the N x N x N products launched.  No sync.
int svt_msvt(int nH, int N, const double* G, int ldg, double tau, const double* C, bool prep, const MsvtPlan& mp,
             double* K, int ldk, IterStats* st, void* ws, hipStream_t s, int* products);

// ---- Gram (gram.hip) ---------------------------------------------------------------
// G = A^T A for A m x k (float32, ld = lda, k <= kp, kp multiple of kPad), accumulated
// in float64; G is kp x kp float64 (ld = kp), rows/cols >= k zero.
size_t gram_workspace_bytes(int m, int kp);
int gram_f64(int m, int k, int kp, const float* A, int lda, double* G, void* ws,
             hipStream_t stream, int prec = 0);
// G = A^T B (A, B m x k float32), float64 accumulation; uses at most
// gram_workspace_bytes(m, kp) of workspace.
int cross_f64(int m, int k, int kp, const float* A, int lda, const float* B, int ldb, double* G, void* ws,
              hipStream_t stream);

// ---- small dense float64 products (dense.hip) ----------------------------------------
// C(MxN) = alpha * op(A) op(B), float64 row-major with explicit leading dimensions.
int gemm_f64(bool transA, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
             const double* B, int ldb, double* C, int ldc, hipStream_t stream);
// C = alpha op(A) op(B) + beta C.
int gemm_f64_acc(bool transA, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
                 const double* B, int ldb, double beta, double* C, int ldc, hipStream_t stream);
// The lower block triangle of C (the 64 x 64 tiles on and below the diagonal; n x n,
// ld ldc) += alpha A B^T, plus alpha B A^T when sym; A, B n x 64 float64 (ld 64).
int rank64_lower_f64(int n, const double* A, const double* B, double alpha, bool sym, double* C, int ldc,
                     hipStream_t stream);
// Upper Cholesky factor inverse of the leading p x p block of S (p <= 64): Rinv = R^{-1}
// with S = R^T R (64 x 64, identity beyond p); *fail = 1 if a pivot is not above
// floor_rel times the largest diagonal entry.  One wave.
int chol_inv64(int p, const double* S, int lds, double floor_rel, double* Rinv, int ldr, int* fail,
               hipStream_t stream);
// Out(m x k2, float32, ldo) = In(m x k1, float32, ldi) * W(k1 x k2, float64, ldw),
// accumulated in float64.
int rmul_f32_by_f64(int m, int k1, int k2, const float* In, int ldi, const double* W, int ldw,
                    float* Out, int ldo, hipStream_t stream);

// ---- spectral norm of the observed data (spectral.hip) --------------------------------
// Workspace of spectral_norm_sq for an m x n matrix.
size_t spectral_workspace_bytes(int m, int n);
// *out (host) = ||A||_2^2 for A m x n float32 (ld = lda): float64 Gram, its top eigenvalue
// by repeated squaring and a Rayleigh quotient.  Synchronises `stream`.
int spectral_norm_sq(int m, int n, const float* A, int lda, void* ws, hipStream_t stream, double* out);
// out (m x n, ld = n) = Q ? D : 0.
int stage_masked(int m, int n, const float* D, int ldd, const uint8_t* Q, float* out, hipStream_t stream);

// ---- stencil kernels (operators.hip) ---------------------------------------------------
// XP = X P  (m x n -> m x nH, float32; the interpolation stencil, no C factor).
int apply_P(const Operator& op, int m, const float* X, int ldx, float* XP, int ldp, hipStream_t s);
// X = N P^T (m x nH -> m x n).
int apply_Pt(const Operator& op, int m, const float* N, int ldn, float* X, int ldx, hipStream_t s);

}  // namespace mlpcp
