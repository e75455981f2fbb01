// Spectral norm of the observed data, ||P_Q D||_2, for the default initial penalty
// mu_0 = 1.25 / ||P_Q D||_2 of the solvers (inexact ALM needs an initial penalty,
// Alg. 1 / Alg. 4; this is its customary scale).  Computed once per solve, before the
// iterations:
//   G = A^T A            float64 Gram of A = P_Q D on MFMA (the solver's Gram kernels)
//   B_0 = G / tr(G),  B_{s+1} = B_s^2 / tr(B_s^2)   repeated squaring, float64 MFMA
//   x = the column of B_S with the largest diagonal entry,  lambda = x^T G x / x^T x.
// B_S = sum_j (lambda_j / lambda_1)^(2^S) v_j v_j^T / norm, so x lies in the span of the
// eigenvectors whose eigenvalues are within a factor (1 - delta) of lambda_1 up to a
// weight exp(-2^S delta); the Rayleigh quotient's relative error is then at most
// max_delta delta exp(-2^(S+1) delta) = 1 / (e 2^(S+1)), about 1e-8 for S = 24, whatever the
// gaps between the top eigenvalues.
#include <algorithm>

#include "common.h"
#include "profile.h"

namespace mlpcp {

namespace {

constexpr int kSquarings = 24;

// out (m x n, ld n) = Q ? D : 0
__global__ void k_stage_masked(int m, int n, const float* __restrict__ D, int ldd, const uint8_t* __restrict__ Q,
                               float* __restrict__ out) {
  const size_t total = (size_t)m * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / n, j = e % n;
    out[e] = Q[e] ? D[i * ldd + j] : 0.0f;
  }
}

__device__ double block_sum256(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// Out = In / tr(In) on the leading n x n block (ld = ld); every block forms the trace
// itself (n diagonal reads), so one launch does the whole normalisation.
__global__ void __launch_bounds__(256) k_trace_scale(int n, int ld, const double* __restrict__ In,
                                                      double* __restrict__ Out) {
  __shared__ double red[256];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) t += In[(size_t)i * ld + i];
  const double tr = block_sum256(t, red);
  const double inv = 1.0 / tr;
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t i = e / n, j = e % n;
    Out[i * ld + j] = In[i * ld + j] * inv;
  }
}

// One workgroup: j* = argmax_j B_jj, x = B[:, j*] (B symmetric: row j*), y = G x,
// out[0] = x^T y / x^T x.  Waves take rows of G with coalesced loads.
__global__ void __launch_bounds__(1024) k_top_rq(int n, int ld, const double* __restrict__ B,
                                                  const double* __restrict__ G, double* __restrict__ out) {
  __shared__ double sval[1024];
  __shared__ int sidx[1024];
  __shared__ double sxy[16], sxx[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double best = -1.0;
  int bi = 0;
  for (int j = tid; j < n; j += 1024) {
    const double v = B[(size_t)j * ld + j];
    if (v > best) {
      best = v;
      bi = j;
    }
  }
  sval[tid] = best;
  sidx[tid] = bi;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) {
      const double o = sval[tid + w];
      const int oi = sidx[tid + w];
      if (o > sval[tid] || (o == sval[tid] && oi < sidx[tid])) {
        sval[tid] = o;
        sidx[tid] = oi;
      }
    }
    __syncthreads();
  }
  const double* x = B + (size_t)sidx[0] * ld;
  double xy = 0.0, xx = 0.0;
  for (int i = wave; i < n; i += 16) {
    const double* g = G + (size_t)i * ld;
    double acc = 0.0;
    for (int k = lane; k < n; k += 64) acc = fma(g[k], x[k], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) {
      xy = fma(x[i], acc, xy);
      xx = fma(x[i], x[i], xx);
    }
  }
  if (lane == 0) {
    sxy[wave] = xy;
    sxx[wave] = xx;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 16; ++w) {
      a += sxy[w];
      b += sxx[w];
    }
    out[0] = a / b;
  }
}

struct SpecLayout {
  int np;
  size_t off_G, off_B0, off_B1, off_out, off_gram, total;
};

SpecLayout spec_layout(int m, int n) {
  SpecLayout l;
  l.np = round_up(n, kPad);
  const size_t nn = (size_t)l.np * l.np * sizeof(double);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += align256(b);
    return o;
  };
  l.off_G = take(nn);
  l.off_B0 = take(nn);
  l.off_B1 = take(nn);
  l.off_out = take(sizeof(double));
  l.off_gram = take(gram_workspace_bytes(m, l.np));
  l.total = off;
  return l;
}

}  // namespace

size_t spectral_workspace_bytes(int m, int n) { return spec_layout(m, n).total; }

int stage_masked(int m, int n, const float* D, int ldd, const uint8_t* Q, float* out, hipStream_t s) {
  const size_t total = (size_t)m * n;
  const unsigned grid = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_stage_masked, dim3(grid), dim3(256), 0, s, m, n, D, ldd, Q, out);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int spectral_norm_sq(int m, int n, const float* A, int lda, void* ws, hipStream_t s, double* out) {
  const SpecLayout l = spec_layout(m, n);
  char* base = static_cast<char*>(ws);
  double* G = reinterpret_cast<double*>(base + l.off_G);
  double* B[2] = {reinterpret_cast<double*>(base + l.off_B0), reinterpret_cast<double*>(base + l.off_B1)};
  double* dout = reinterpret_cast<double*>(base + l.off_out);
  ProfScope ps(KC_OTHER, s);
  MLPCP_HIP(hipMemsetAsync(G, 0, (size_t)l.np * l.np * sizeof(double), s));
  MLPCP_TRY(gram_f64(m, n, l.np, A, lda, G, base + l.off_gram, s, 0));
  const unsigned grid = (unsigned)std::min<size_t>(((size_t)n * n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_trace_scale, dim3(grid), dim3(256), 0, s, n, l.np, G, B[0]);
  for (int k = 0; k < kSquarings; ++k) {
    MLPCP_TRY(gemm_f64(false, false, n, n, n, 1.0, B[0], l.np, B[0], l.np, B[1], l.np, s));
    hipLaunchKernelGGL(k_trace_scale, dim3(grid), dim3(256), 0, s, n, l.np, B[1], B[0]);
  }
  hipLaunchKernelGGL(k_top_rq, dim3(1), dim3(1024), 0, s, n, l.np, B[0], G, dout);
  MLPCP_HIP(hipGetLastError());
  MLPCP_HIP(hipMemcpyAsync(out, dout, sizeof(double), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  return MLPCP_OK;
}

}  // namespace mlpcp
