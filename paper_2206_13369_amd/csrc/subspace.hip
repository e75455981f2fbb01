// Rank-predicted partial eigensolve for the singular value threshold of a wide Gram
// matrix G (N x N, float64): the SVT needs only the eigenpairs above tau^2 (the paper
// remarks after Alg. 1 that only the leading singular values have to be computed), so
// when the previous iteration kept r_prev <= kSubMaxRank of them, this iteration's are
// taken from a block of kSubCols = 64 vectors started at the previous leading
// eigenvectors:
//
//  1. subspace iteration X <- orth(G X) (orth: Cholesky QR, applied twice), on f64 MFMA;
//  2. Rayleigh-Ritz: H = X^T G X = Q Theta Q^T by the one-workgroup Jacobi solver,
//     X <- X Q ordered by Ritz value, W = G X, and the residual of the r Ritz pairs above
//     tau^2: e = ||W_U - X_U Theta_U||_F; more subspace steps while e is too large;
//  3. certificate that nothing outside span(X_U) reaches tau^2: with
//     B = (I - X_U X_U^T) G (I - X_U X_U^T) = G - X_U Z^T - Z X_U^T, Z = W_U - X_U Theta_U / 2,
//     the blocked Cholesky factorisation of c I - B must succeed for
//     c = tau^2 - e - (rounding allowance).  Then every eigenvalue of B is below c; in the
//     basis (X_U, its complement) G is diag(Theta_U, B') plus an off-diagonal coupling of
//     norm at most e, so (Weyl) r eigenvalues of G lie within e of Theta_U, above tau^2,
//     and all others below c + e < tau^2: the rank is r and the SVT is that of
//     (Theta_U, X_U) up to the coupling.
//
// Acceptance also asks e <= max(kSubResTol tau^2, rounding floor of the products): the
// thresholded map f(l) = (1 - tau / sqrt(l))_+ has slope at most 1/(2 tau^2) above tau^2,
// so the coupling moves the SVT by about kSubResTol / 2 relative.  When any test fails
// the caller runs the full Jacobi eigensolver instead, the same SVT by another route.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "profile.h"

namespace mlpcp {

namespace {

constexpr int kSubCols = 64;
constexpr int kSubMaxRank = 56;
constexpr int kSubMoreIters = 2;    // steps added when the residual is still too large
constexpr int kSubMaxIters = 12;
constexpr double kSubResTol = 1.0e-8;

struct SubLayout {
  size_t off_M, off_X, off_W, off_Y, off_X2, off_W2, off_P, off_S, off_R, off_H, off_Q, off_Qs, off_th, off_thr,
      off_rho, off_perm, off_flag, off_ews, total;
};

SubLayout sub_layout(int N) {
  SubLayout l;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += align256(b);
    return o;
  };
  const size_t tall = (size_t)N * kSubCols * sizeof(double);
  const size_t sq = (size_t)kSubCols * kSubCols * sizeof(double);
  l.off_M = take((size_t)N * N * sizeof(double));
  l.off_X = take(tall);
  l.off_W = take(tall);
  l.off_Y = take(tall);
  l.off_X2 = take(tall);
  l.off_W2 = take(tall);
  l.off_P = take(tall);
  l.off_S = take(sq);
  l.off_R = take(sq);
  l.off_H = take(sq);
  l.off_Q = take(sq);
  l.off_Qs = take(sq);
  l.off_th = take(kSubCols * sizeof(double));
  l.off_thr = take(kSubCols * sizeof(double));
  l.off_rho = take((kSubCols + 1) * sizeof(double));
  l.off_perm = take(kSubCols * sizeof(int));
  l.off_flag = take(4 * sizeof(int));
  l.off_ews = take(eig_workspace_bytes(kSubCols));
  l.total = off;
  return l;
}

unsigned grid_of(size_t total) { return (unsigned)std::min<size_t>((total + 255) / 256, 4096); }

// X (N x 64, ld 64) = columns perm[0..63] of V (N x N, ld N)
__global__ void k_gather_cols(int N, const double* __restrict__ V, const int* __restrict__ perm,
                              double* __restrict__ X) {
  const size_t total = (size_t)N * kSubCols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / kSubCols;
    const int j = (int)(e % kSubCols);
    X[e] = V[i * N + perm[j]];
  }
}

// H <- (H + H^T) / 2 (64 x 64)
__global__ void k_sym64(double* __restrict__ H) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kSubCols * kSubCols; e += gridDim.x * blockDim.x) {
    const int r = e / kSubCols, c = e % kSubCols;
    if (r < c) {
      const double v = 0.5 * (H[r * kSubCols + c] + H[c * kSubCols + r]);
      H[r * kSubCols + c] = v;
      H[c * kSubCols + r] = v;
    }
  }
}

// Ritz order (descending): Qs = Q[:, perm], th = thr[perm]
__global__ void k_sort_ritz(const double* __restrict__ Q, const double* __restrict__ thr, const int* __restrict__ perm,
                            double* __restrict__ Qs, double* __restrict__ th) {
  for (int e = threadIdx.x; e < kSubCols * kSubCols; e += blockDim.x) {
    const int r = e / kSubCols, c = e % kSubCols;
    Qs[e] = Q[r * kSubCols + perm[c]];
  }
  if (threadIdx.x < kSubCols) th[threadIdx.x] = thr[perm[threadIdx.x]];
}

// rho[j] = ||W[:, j] - th[j] X[:, j]||^2 (block j < 64); block 64: rho[64] = trace(G)
__global__ void __launch_bounds__(256) k_sub_resid(int N, const double* __restrict__ W, const double* __restrict__ X,
                                                   const double* __restrict__ th, const double* __restrict__ G,
                                                   double* __restrict__ rho) {
  __shared__ double r1[256];
  const int j = blockIdx.x;
  double a = 0.0;
  if (j < kSubCols) {
    const double t = th[j];
    for (int i = threadIdx.x; i < N; i += 256) {
      const double d = fma(-t, X[(size_t)i * kSubCols + j], W[(size_t)i * kSubCols + j]);
      a = fma(d, d, a);
    }
  } else {
    for (int i = threadIdx.x; i < N; i += 256) a += G[(size_t)i * N + i];
  }
  r1[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) r1[threadIdx.x] += r1[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rho[j] = r1[0];
}

// Z = W_U - X_U Theta_U / 2 for the first r columns, zero beyond (N x 64)
__global__ void k_make_Z(int N, int r, const double* __restrict__ W, const double* __restrict__ X,
                         const double* __restrict__ th, double* __restrict__ Z) {
  const size_t total = (size_t)N * kSubCols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % kSubCols);
    Z[e] = j < r ? fma(-0.5 * th[j], X[e], W[e]) : 0.0;
  }
}

// XU = X with the columns from r on zeroed (N x 64)
__global__ void k_keep_cols(int N, int r, const double* __restrict__ X, double* __restrict__ XU) {
  const size_t total = (size_t)N * kSubCols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
    XU[e] = (int)(e % kSubCols) < r ? X[e] : 0.0;
}

// M = c I - G (N x N)
__global__ void k_shift_neg(int N, double c, const double* __restrict__ G, double* __restrict__ M) {
  const size_t total = (size_t)N * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
    M[e] = ((e / N) == (e % N) ? c : 0.0) - G[e];
}

// The result in the eigensolver's output convention: V[:, 0..r) = X_U, lam = Theta_U
// there and -1 elsewhere, perm = identity, gb = the certified bound beyond the first r
// (-1 within)
__global__ void k_sub_out(int N, int r, const double* __restrict__ X2, const double* __restrict__ th, double bound,
                          double* __restrict__ V, double* __restrict__ lam, int* __restrict__ perm,
                          double* __restrict__ gb) {
  const size_t total = (size_t)N * kSubCols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / kSubCols;
    const int j = (int)(e % kSubCols);
    V[i * N + j] = X2[e];
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    lam[i] = i < r ? th[i] : -1.0;
    perm[i] = i;
    if (gb) gb[i] = i < r ? -1.0 : bound;
  }
}

// X = orth(W) by one Cholesky QR step (X = W R^{-1}, W^T W = R^T R); fail flag on a lost
// pivot.  Between subspace steps one step suffices (the next product and step restore
// what rounding took from orthogonality); before the Rayleigh-Ritz step it is applied
// twice, which leaves X orthonormal to rounding.
int chol_qr(int N, const double* W, double* X, double* S, double* Rinv, int* fail, hipStream_t s) {
  MLPCP_TRY(gemm_f64(true, false, kSubCols, kSubCols, N, 1.0, W, kSubCols, W, kSubCols, S, kSubCols, s));
  MLPCP_TRY(chol_inv64(kSubCols, S, kSubCols, 1.0e-15, Rinv, kSubCols, fail, s));
  MLPCP_TRY(gemm_f64(false, false, N, kSubCols, kSubCols, 1.0, W, kSubCols, Rinv, kSubCols, X, kSubCols, s));
  return MLPCP_OK;
}

}  // namespace

size_t subspace_workspace_bytes(int N) { return sub_layout(N).total; }

int subspace_steps(double rho) {
  if (!(rho > 0.0) || !(rho < 1.0)) return kSubMaxIters;
  const int q = (int)std::ceil(std::log(1.0e-10) / std::log(rho));
  return std::max(2, std::min(q, kSubMaxIters));
}

bool subspace_eligible(int N, int r_prev) {
  return N >= 2 * kSubCols && N % kSubCols == 0 && r_prev >= 1 && r_prev <= kSubMaxRank;
}

int svt_partial(int N, const double* G, double tau, int first_iters, double* V, double* lam, int* perm, double* gb,
                double* trace_dev, void* ws, hipStream_t s, bool* ok, int* iters_out, double* ratio_out) {
  *ok = false;
  *iters_out = 0;
  *ratio_out = 1.0;
  first_iters = std::max(1, std::min(first_iters, kSubMaxIters));
  if (!subspace_eligible(N, 1)) return MLPCP_E_INVALID_ARG;
  const SubLayout l = sub_layout(N);
  char* b = static_cast<char*>(ws);
  auto at = [&](size_t o) { return reinterpret_cast<double*>(b + o); };
  double *M = at(l.off_M), *X = at(l.off_X), *W = at(l.off_W), *Y = at(l.off_Y), *X2 = at(l.off_X2),
         *W2 = at(l.off_W2), *P = at(l.off_P), *S = at(l.off_S), *Rinv = at(l.off_R), *H = at(l.off_H),
         *Q = at(l.off_Q), *Qs = at(l.off_Qs), *th = at(l.off_th), *thr = at(l.off_thr), *rho = at(l.off_rho);
  int* permH = reinterpret_cast<int*>(b + l.off_perm);
  int* flag = reinterpret_cast<int*>(b + l.off_flag);
  void* ews = b + l.off_ews;
  const size_t tall = (size_t)N * kSubCols;
  const double tau2 = tau * tau;
  const double eps = std::ldexp(1.0, -52);
  {
    ProfScope ps(KC_JACOBI_MISC, s);
    MLPCP_HIP(hipMemsetAsync(flag, 0, 4 * sizeof(int), s));
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_of(tall)), dim3(256), 0, s, N, V, perm, X);
    MLPCP_HIP(hipGetLastError());
  }
  int iters = 0, r = 0;
  double e = 0.0;
  double hth[kSubCols], hrho[kSubCols + 1];
  int hflag[4];
  for (int step = first_iters;; step = kSubMoreIters) {
    {
      ProfScope ps(KC_JACOBI_MISC, s);
      for (int it = 0; it < step; ++it) {
        MLPCP_TRY(gemm_f64(false, false, N, kSubCols, N, 1.0, G, N, X, kSubCols, W, kSubCols, s));
        if (it + 1 < step) {
          MLPCP_TRY(chol_qr(N, W, X, S, Rinv, &flag[0], s));
        } else {
          MLPCP_TRY(chol_qr(N, W, Y, S, Rinv, &flag[0], s));
          MLPCP_TRY(chol_qr(N, Y, X, S, Rinv, &flag[0], s));
        }
      }
      iters += step;
      MLPCP_TRY(gemm_f64(false, false, N, kSubCols, N, 1.0, G, N, X, kSubCols, W, kSubCols, s));
      MLPCP_TRY(gemm_f64(true, false, kSubCols, kSubCols, N, 1.0, X, kSubCols, W, kSubCols, H, kSubCols, s));
      hipLaunchKernelGGL(k_sym64, dim3(4), dim3(1024), 0, s, H);
      MLPCP_HIP(hipGetLastError());
    }
    int sweeps = 0;
    MLPCP_TRY(eig_sym(kSubCols, kSubCols, H, Q, thr, permH, ews, s, &sweeps, false));
    {
      ProfScope ps(KC_JACOBI_MISC, s);
      hipLaunchKernelGGL(k_sort_ritz, dim3(1), dim3(1024), 0, s, Q, thr, permH, Qs, th);
      MLPCP_TRY(gemm_f64(false, false, N, kSubCols, kSubCols, 1.0, X, kSubCols, Qs, kSubCols, X2, kSubCols, s));
      MLPCP_TRY(gemm_f64(false, false, N, kSubCols, kSubCols, 1.0, W, kSubCols, Qs, kSubCols, W2, kSubCols, s));
      hipLaunchKernelGGL(k_sub_resid, dim3(kSubCols + 1), dim3(256), 0, s, N, W2, X2, th, G, rho);
      MLPCP_HIP(hipGetLastError());
    }
    MLPCP_HIP(hipMemcpyAsync(hth, th, sizeof(hth), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipMemcpyAsync(hrho, rho, sizeof(hrho), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipStreamSynchronize(s));
    *iters_out = iters;
    if (hflag[0]) return MLPCP_OK;   // the block lost rank: leave it to the full solver
    r = 0;
    double e2 = 0.0;
    for (int i = 0; i < kSubCols; ++i) {
      if (!std::isfinite(hth[i]) || !std::isfinite(hrho[i])) return MLPCP_OK;
      if (hth[i] > tau2) {
        ++r;
        e2 += hrho[i];
      }
    }
    if (r < 1 || r > kSubMaxRank) return MLPCP_OK;
    // the convergence factor of the next solve's subspace steps, lambda_65 / lambda_r,
    // estimated by the block's last and r-th Ritz values
    *ratio_out = hth[r - 1] > 0.0 ? std::max(hth[kSubCols - 1], 0.0) / hth[r - 1] : 1.0;
    e = std::sqrt(e2);
    // the residual cannot fall below the rounding of the products G X (length-N sums
    // over r columns, entries up to ||G|| = theta_1), the level a full eigensolve's
    // backward error also has
    const double floor_e = 64.0 * std::sqrt((double)N * r) * eps * std::fabs(hth[0]);
    const bool small = e <= std::max(kSubResTol * tau2, floor_e);
    if (small) break;
    if (iters + kSubMoreIters > kSubMaxIters) return MLPCP_OK;
    // continue from the Ritz basis
    MLPCP_HIP(hipMemcpyAsync(X, X2, tall * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  if (!(hth[r - 1] - e > tau2)) return MLPCP_OK;
  // rounding allowance of forming c I - B (products of length 64 and N over entries of
  // size up to ||G|| <= trace G) and of the Cholesky factorisation (N^2 eps relative)
  const double trG = std::max(hrho[kSubCols], 0.0);
  const double allow = 80.0 * N * eps * trG + (double)N * N * eps * tau2;
  const double c = tau2 - e - allow;
  if (!(c > 0.0)) return MLPCP_OK;
  {
    ProfScope ps(KC_JACOBI_MISC, s);
    double* Z = W;   // W is free now
    double* XU = Y;
    hipLaunchKernelGGL(k_make_Z, dim3(grid_of(tall)), dim3(256), 0, s, N, r, W2, X2, th, Z);
    hipLaunchKernelGGL(k_keep_cols, dim3(grid_of(tall)), dim3(256), 0, s, N, r, X2, XU);
    hipLaunchKernelGGL(k_shift_neg, dim3(grid_of((size_t)N * N)), dim3(256), 0, s, N, c, G, M);
    MLPCP_HIP(hipGetLastError());
    // only the lower block triangle is formed and factorised
    MLPCP_TRY(rank64_lower_f64(N, XU, Z, 1.0, true, M, N, s));
    for (int kb = 0; kb < N; kb += kSubCols) {
      double* Mkk = M + (size_t)kb * N + kb;
      MLPCP_TRY(chol_inv64(kSubCols, Mkk, N, 1.0e-14, Rinv, kSubCols, &flag[1], s));
      const int rem = N - kb - kSubCols;
      if (rem > 0) {
        // panel of the lower factor, L21 = M21 R^{-1}, then the trailing update M22 -= L21 L21^T
        MLPCP_TRY(gemm_f64(false, false, rem, kSubCols, kSubCols, 1.0, Mkk + (size_t)kSubCols * N, N, Rinv, kSubCols,
                           P, kSubCols, s));
        double* M22 = Mkk + (size_t)kSubCols * N + kSubCols;
        MLPCP_TRY(rank64_lower_f64(rem, P, P, -1.0, false, M22, N, s));
      }
    }
  }
  MLPCP_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  if (hflag[1]) return MLPCP_OK;
  {
    ProfScope ps(KC_JACOBI_MISC, s);
    hipLaunchKernelGGL(k_sub_out, dim3(grid_of(tall)), dim3(256), 0, s, N, r, X2, th, c + e, V, lam, perm, gb);
    MLPCP_HIP(hipGetLastError());
    if (trace_dev)
      MLPCP_HIP(hipMemcpyAsync(trace_dev, rho + kSubCols, sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  *ok = true;
  return MLPCP_OK;
}

}  // namespace mlpcp
