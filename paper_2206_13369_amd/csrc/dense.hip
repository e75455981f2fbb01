// Small dense float64 helpers used around the eigensolver: C = op(A) op(B) for the
// n_H x n_H products (C G C, the warm start V^T A V, the orthonormalising factor) on
// float64 MFMA, and a right multiplication of a tall float32 matrix by a small
// float64 matrix.
#include "common.h"

namespace mlpcp {

namespace {

constexpr int T = 32;

typedef double d4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm_f64(int transA, int transB, int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                  int ldc) {
  __shared__ double sA[T][T + 1];
  __shared__ double sB[T][T + 1];
  const int i0 = blockIdx.y * T, j0 = blockIdx.x * T;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += T) {
    for (int e = tid; e < T * T; e += 256) {
      const int r = e / T, c = e % T;
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
    // wave (wi, wj) owns the 16 x 16 sub-tile; v_mfma_f64_16x16x4f64: lane l holds
    // op(A)[l%16][k0 + l/16] and op(B)[k0 + l/16][l%16]
#pragma unroll
    for (int ks = 0; ks < T / 4; ++ks) {
      const double a = sA[wi * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
      const double b = sB[ks * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // output register v of lane l: row 4v + l/16, column l%16
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
  dim3 grid((N + T - 1) / T, (M + T - 1) / T);
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, stream, (int)transA, (int)transB, M, N, K, alpha, A, lda, B,
                     ldb, C, ldc);
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
