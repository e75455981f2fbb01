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
                                                  int ldc) {
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
    if (gi < M && gj < N) C[(size_t)gi * ldc + gj] = alpha * (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]);
  }
}

// Wide products (the plain method's warm start at n in the thousands): 32 x 32 tiles
// with K staged 32 at a time, so each panel element is fetched N/32 (not N/16) times;
// with thousands of blocks in flight the load latency is hidden across blocks.
constexpr int TW = 32;
__global__ void __launch_bounds__(256) k_gemm_f64_wide(int transA, int transB, int M, int N, int K, double alpha,
                                                       const double* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                       int ldc) {
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
    if (gi < M && gj < N) C[(size_t)gi * ldc + gj] = alpha * acc[v];
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
  const size_t tiles = (size_t)((N + T - 1) / T) * ((M + T - 1) / T);
  if (tiles > 2048) {   // more 16 x 16 tiles than a few per compute unit: panel re-reads dominate
    dim3 grid((N + TW - 1) / TW, (M + TW - 1) / TW);
    hipLaunchKernelGGL(k_gemm_f64_wide, grid, dim3(256), 0, stream, (int)transA, (int)transB, M, N, K, alpha, A, lda,
                       B, ldb, C, ldc);
  } else {
    dim3 grid((N + T - 1) / T, (M + T - 1) / T);
    hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, stream, (int)transA, (int)transB, M, N, K, alpha, A, lda, B,
                       ldb, C, ldc);
  }
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
