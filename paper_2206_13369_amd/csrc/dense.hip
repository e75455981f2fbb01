// Small dense float64 helpers used around the eigensolver: C = op(A) op(B) for the
// n_H x n_H products (C G C, the warm start V^T A V, the orthonormalising factor) on
// float64 MFMA (a latency-oriented kernel for coarse sizes, a 32 x 32-tile one for
// outputs of thousands of tiles), and a right multiplication of a tall float32
// matrix by a small float64 matrix.
#include "common.h"

namespace mlpcp {

namespace {

constexpr int T = 16;     // output tile (one 16 x 16 MFMA block)
constexpr int KC = 256;   // K chunk staged in LDS at once

typedef double d4_t __attribute__((ext_vector_type(4)));

// One 16 x 16 tile of C per block.  Both K panels of a chunk (op(A) rows i0.., op(B)
// columns j0..) are loaded with all their loads in flight, then the four waves each
// take a quarter of the chunk's K on MFMA and their accumulators are summed through
// LDS: the products here are small (n_H <= a few hundred), so latency, not MFMA
// throughput, bounds them, and this keeps a 256^3 product at one load round trip per
// chunk over 256 blocks.
__global__ void __launch_bounds__(256) k_gemm_f64(int transA, int transB, int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                  int ldc, double beta) {
  __shared__ double sA[T][KC + 1];   // sA[r][c] = op(A)[i0 + r][k0 + c]
  __shared__ double sB[KC][T + 1];   // sB[r][c] = op(B)[k0 + r][j0 + c]
  __shared__ double red[4][T * T];
  const int i0 = blockIdx.y * T, j0 = blockIdx.x * T;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += KC) {
    constexpr int PER = T * KC / 256;   // elements of each panel per thread
    double ra[PER], rb[PER];
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int e = tid + 256 * x;
      // coalesced order: the index that is contiguous in memory runs fastest
      const int ar = transA ? e % T : e / KC, ac = transA ? e / T : e % KC;
      const int br = transB ? e % KC : e / T, bc = transB ? e / KC : e % T;
      const int gi = i0 + ar, gk = k0 + ac, gk2 = k0 + br, gj = j0 + bc;
      ra[x] = (gi < M && gk < K) ? (transA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk]) : 0.0;
      rb[x] = (gk2 < K && gj < N) ? (transB ? B[(size_t)gj * ldb + gk2] : B[(size_t)gk2 * ldb + gj]) : 0.0;
    }
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int e = tid + 256 * x;
      const int ar = transA ? e % T : e / KC, ac = transA ? e / T : e % KC;
      const int br = transB ? e % KC : e / T, bc = transB ? e / KC : e % T;
      sA[ar][ac] = ra[x];
      sB[br][bc] = rb[x];
    }
    __syncthreads();
    // wave w: k in [w KC/4, (w+1) KC/4); v_mfma_f64_16x16x4f64: lane l holds
    // op(A)[l%16][k + l/16] and op(B)[k + l/16][l%16]
    const int kq = wave * (KC / 4);
#pragma unroll 4
    for (int ks = 0; ks < KC / 16; ++ks) {
      const int k = kq + ks * 4 + (lane >> 4);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[lane & 15][k], sB[k][lane & 15], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // output register v of lane l: row 4v + l/16, column l%16
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][(4 * v + (lane >> 4)) * T + (lane & 15)] = acc[v];
  __syncthreads();
  {
    const int r = tid / T, c = tid % T, gi = i0 + r, gj = j0 + c;
    if (gi < M && gj < N) {
      const double v = alpha * (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]);
      C[(size_t)gi * ldc + gj] = beta != 0.0 ? fma(beta, C[(size_t)gi * ldc + gj], v) : v;
    }
  }
}

// Wide products (the plain method's warm start at n in the thousands): 32 x 32 tiles
// with K staged 32 at a time, so each panel element is fetched N/32 (not N/16) times;
// with thousands of blocks in flight the load latency is hidden across blocks.
constexpr int TW = 32;
__global__ void __launch_bounds__(256) k_gemm_f64_wide(int transA, int transB, int M, int N, int K, double alpha,
                                                       const double* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                       int ldc, double beta) {
  __shared__ double sA[TW][TW + 1];
  __shared__ double sB[TW][TW + 1];
  const int i0 = blockIdx.y * TW, j0 = blockIdx.x * TW;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += TW) {
    for (int e = tid; e < TW * TW; e += 256) {
      const int r = e / TW, c = e % TW;
      const int gi = i0 + r, gk = k0 + c;  // sA[r][c] = op(A)[gi][gk]
      double va = 0.0;
      if (gi < M && gk < K) va = transA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      sA[r][c] = va;
      const int gk2 = k0 + r, gj = j0 + c;  // sB[r][c] = op(B)[gk2][gj]
      double vb = 0.0;
      if (gk2 < K && gj < N) vb = transB ? B[(size_t)gj * ldb + gk2] : B[(size_t)gk2 * ldb + gj];
      sB[r][c] = vb;
    }
    __syncthreads();
    // wave (wi, wj) owns a 16 x 16 sub-tile
#pragma unroll
    for (int ks = 0; ks < TW / 4; ++ks) {
      const double a = sA[wi * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
      const double b = sB[ks * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int gj = j0 + wj * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = i0 + wi * 16 + 4 * v + (lane >> 4);
    if (gi < M && gj < N) {
      const double x = alpha * acc[v];
      C[(size_t)gi * ldc + gj] = beta != 0.0 ? fma(beta, C[(size_t)gi * ldc + gj], x) : x;
    }
  }
}

// Upper Cholesky factor of the leading p x p block of the symmetric S (p <= 64, ld lds)
// and its inverse: S = R^T R, Rinv = R^{-1} (64 x 64, ld ldr, the identity beyond p).
// 256 threads; thread t holds row i = t / 4 of the working matrix at the columns
// q + 4c (q = t % 4, c < 16) in registers.  Right-looking: at step k the four owners of
// row k publish it in LDS (one barrier per step), every thread forms R's row k entries
// it needs and updates its trailing entries.  The inverse by back substitution, four
// threads per column of R^{-1} (partial sums over k = q mod 4 combined by lane
// shuffles), the 64 steps unrolled so the column stays in registers.  *fail = 1 (never
// cleared here) if a pivot is not above floor_rel times the largest diagonal entry of S
// (or is NaN); that pivot is then taken as 1, so the outputs stay finite.
__global__ void __launch_bounds__(256) k_chol_inv64(int p, const double* __restrict__ S, int lds, double floor_rel,
                                                    double* __restrict__ Rinv, int ldr, int* __restrict__ fail) {
  __shared__ double row[2][64];
  __shared__ double R[64][65];
  __shared__ double dg[64];
  __shared__ double rdi[64];   // 1 / R_kk
  const int t = threadIdx.x;
  const int i = t >> 2, q = t & 3;
  double a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int j = q + 4 * c;
    a[c] = (i < p && j < p) ? S[(size_t)i * lds + j] : (i == j ? 1.0 : 0.0);
    if (j == i) dg[i] = a[c];
  }
  __syncthreads();
  double dmax = 0.0;
  for (int k = 0; k < p; ++k) dmax = fmax(dmax, dg[k]);
  bool bad = false;
  for (int k = 0; k < 64; ++k) {
    double* rk = row[k & 1];
    if (i == k) {
#pragma unroll
      for (int c = 0; c < 16; ++c) rk[q + 4 * c] = a[c];
    }
    __syncthreads();
    double piv = rk[k];
    if (!(piv > floor_rel * dmax)) {
      bad = true;
      piv = 1.0;
    }
    // 1 / sqrt(piv) from the hardware estimate and two Newton steps (the step's only
    // long dependency chain); then 1 / piv and sqrt(piv) by multiplications
    double y = __builtin_amdgcn_rsq(piv);
    y = y * fma(-0.5 * piv * y, y, 1.5);
    y = y * fma(-0.5 * piv * y, y, 1.5);
    const double ipiv = y * y, rkk = piv * y;
    if (t < 64) R[k][t] = t < k ? 0.0 : (t == k ? rkk : rk[t] * y);
    if (t == k) rdi[k] = y;
    // trailing update, branch-free: entries outside (i > k, j > k) keep their value
    const double f = i > k ? rk[i] * ipiv : 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int j = q + 4 * c;
      const double upd = fma(-f, rk[j], a[c]);
      a[c] = j > k ? upd : a[c];
    }
  }
  __syncthreads();
  // column l = t / 4 of R^{-1}: T_il = (delta_il - sum_{i < k <= l} R_ik T_kl) / R_ii
  const int l = i;
  double tv[16];   // T_kl for k = q + 4c
#pragma unroll
  for (int c = 0; c < 16; ++c) tv[c] = 0.0;
#pragma unroll
  for (int ii = 63; ii >= 0; --ii) {
    double s0 = 0.0, s1 = 0.0;   // two chains over the sixteen terms
#pragma unroll
    for (int c = 0; c < 16; c += 2) {
      const int k0 = q + 4 * c, k1 = k0 + 4;
      const double r0 = R[ii][k0], r1 = R[ii][k1];
      s0 = fma((k0 > ii && k0 <= l) ? r0 : 0.0, tv[c], s0);
      s1 = fma((k1 > ii && k1 <= l) ? r1 : 0.0, tv[c + 1], s1);
    }
    double sum = s0 + s1;
    sum += __shfl_xor(sum, 1, 4);
    sum += __shfl_xor(sum, 2, 4);
    const double v = ii <= l ? ((ii == l ? 1.0 : 0.0) - sum) * rdi[ii] : 0.0;
    if (q == (ii & 3)) tv[ii >> 2] = v;
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) Rinv[(size_t)(q + 4 * c) * ldr + l] = tv[c];
  if (t == 0 && bad) *fail = 1;
}

// The lower block triangle of C (64 x 64 tiles on and below the diagonal, n x n, ld ldc)
// += alpha A B^T (+ alpha B A^T when sym), A and B n x 64 (ld 64): the rank-64 updates of
// a blocked Cholesky factorisation, which reads only that triangle.  One block per tile
// (blockIdx.x enumerates the tiles (ti, tj), tj <= ti); K = 64 in two halves staged in
// LDS; wave w owns the 32 x 32 quadrant (w / 2, w % 2), four 16 x 16 MFMA tiles.
__global__ void __launch_bounds__(256) k_rank64_lower(int n, const double* __restrict__ A,
                                                      const double* __restrict__ B, double alpha, int sym,
                                                      double* __restrict__ C, int ldc) {
  __shared__ double sI[64][33];   // rows of the first operand at tile row ti (32 of K)
  __shared__ double sJ[64][33];   // rows of the second operand at tile column tj
  const int b = blockIdx.x;
  int ti = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int tj = b - ti * (ti + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  d4_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int pass = 0; pass < (sym ? 2 : 1); ++pass) {
    const double* P1 = pass ? B : A;   // rows at ti
    const double* P2 = pass ? A : B;   // rows at tj
    for (int k0 = 0; k0 < 64; k0 += 32) {
      for (int e = tid; e < 64 * 32; e += 256) {
        const int r = e >> 5, c = e & 31;
        const int gi = ti * 64 + r, gj = tj * 64 + r;
        sI[r][c] = gi < n ? P1[(size_t)gi * 64 + k0 + c] : 0.0;
        sJ[r][c] = gj < n ? P2[(size_t)gj * 64 + k0 + c] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 32; ks += 4) {
        const int k = ks + (lane >> 4);
        const double a0 = sI[wi * 32 + (lane & 15)][k], a1 = sI[wi * 32 + 16 + (lane & 15)][k];
        const double b0 = sJ[wj * 32 + (lane & 15)][k], b1 = sJ[wj * 32 + 16 + (lane & 15)][k];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  // output register v of lane l: row 4v + l/16, column l%16 of each 16 x 16 tile
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = ti * 64 + wi * 32 + 16 * x + 4 * v + (lane >> 4);
        const int gj = tj * 64 + wj * 32 + 16 * y + (lane & 15);
        if (gi < n && gj < n) C[(size_t)gi * ldc + gj] += alpha * acc[x][y][v];
      }
}

// one block per row; threads stride over the output columns
__global__ void k_rmul(int m, int k1, int k2, const float* __restrict__ In, int ldi, const double* __restrict__ W,
                       int ldw, float* __restrict__ Out, int ldo) {
  const int row = blockIdx.x;
  if (row >= m) return;
  const float* x = In + (size_t)row * ldi;
  for (int col = threadIdx.x; col < k2; col += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < k1; ++c) acc += (double)x[c] * W[(size_t)c * ldw + col];
    Out[(size_t)row * ldo + col] = (float)acc;
  }
}

}  // namespace

int gemm_f64(bool transA, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
             const double* B, int ldb, double* C, int ldc, hipStream_t stream) {
  return gemm_f64_acc(transA, transB, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, stream);
}

int chol_inv64(int p, const double* S, int lds, double floor_rel, double* Rinv, int ldr, int* fail,
               hipStream_t stream) {
  if (p < 1 || p > 64) return MLPCP_E_INVALID_ARG;
  hipLaunchKernelGGL(k_chol_inv64, dim3(1), dim3(256), 0, stream, p, S, lds, floor_rel, Rinv, ldr, fail);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int gemm_f64_acc(bool transA, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
                 const double* B, int ldb, double beta, double* C, int ldc, hipStream_t stream) {
  const size_t tiles = (size_t)((N + T - 1) / T) * ((M + T - 1) / T);
  if (tiles > 2048) {   // more 16 x 16 tiles than a few per compute unit: panel re-reads dominate
    dim3 grid((N + TW - 1) / TW, (M + TW - 1) / TW);
    hipLaunchKernelGGL(k_gemm_f64_wide, grid, dim3(256), 0, stream, (int)transA, (int)transB, M, N, K, alpha, A, lda,
                       B, ldb, C, ldc, beta);
  } else {
    dim3 grid((N + T - 1) / T, (M + T - 1) / T);
    hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, stream, (int)transA, (int)transB, M, N, K, alpha, A, lda, B,
                       ldb, C, ldc, beta);
  }
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int rank64_lower_f64(int n, const double* A, const double* B, double alpha, bool sym, double* C, int ldc,
                     hipStream_t stream) {
  if (n <= 0) return MLPCP_OK;
  const int nt = (n + 63) / 64;
  hipLaunchKernelGGL(k_rank64_lower, dim3(nt * (nt + 1) / 2), dim3(256), 0, stream, n, A, B, alpha, sym ? 1 : 0, C,
                     ldc);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int rmul_f32_by_f64(int m, int k1, int k2, const float* In, int ldi, const double* W, int ldw, float* Out, int ldo,
                    hipStream_t stream) {
  if (m == 0 || k2 == 0) return MLPCP_OK;
  hipLaunchKernelGGL(k_rmul, dim3(m), dim3(64), 0, stream, m, k1, k2, In, ldi, W, ldw, Out, ldo);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

}  // namespace mlpcp
