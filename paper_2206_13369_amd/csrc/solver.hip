// Multilevel inexact ALM (Alg. 4; Alg. 1 when levels = 0) for PCP and its masked
// (compressive) form, and the standalone coarse SVT.
//
// Per iteration t (penalty mu_t, threshold tau = 1/mu_t):
//   gram      G   = M_P^T M_P, M_P = X_t P                  (coarse data without C)
//   coarse    G_H = C G C = (X_t R)^T (X_t R),  R = P C     (Gram of the coarse data)
//   eig       G_H = V diag(lam) V^T (float64 Jacobi)
//   svt prep  sigma = sqrt(lam), r = #{sigma > tau}, w = (sigma - tau)/sigma,
//             T = C V_r diag(sqrt w)  (n_H x r)
//   epilogue  L_{t+1} = M_P T T^T P^T  (= U_H S_tau[Sigma_H] V_H^T R^T, the coarse SVT
//             lifted back), then per element on Q, with E = D - L + Y_t/mu_t:
//                 S = S_{lam/mu_t}[E],  Y_{t+1} = mu_t clip(E, lam/mu_t)
//             (the dual update Y_t + mu_t (D - L - S) in closed form), the
//             feasibility-gap partial sum of (D - L - S)^2 = (clip(E) - Y_t/mu_t)^2, and
//             the next coarse data X_{t+1} = D - S + Y_{t+1}/mu_{t+1}; off Q,
//             X_{t+1} = L_{t+1} and S = Y = 0.  X_{t+1} is restricted (X_{t+1} P) in the
//             same pass.
// State between iterations: one m x n float32 matrix holding W = E - D = -L + Y_t/mu_t
// on Q and L off Q, kept in the caller's S buffer, plus M_P.  W is small where D carries
// large corruptions, so the updates are written in terms of W and clip(D + W) and never
// subtract two large float32 numbers.  A final pass recomputes L from the last coarse
// factors and writes L, S = S[D + W] and Y.
#include <mutex>

#include "common.h"
#include "profile.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

namespace mlpcp {

namespace {

constexpr int kThreads = 256;
// LDS per block of the wide epilogue and the initial pass (sets the rows per block):
// small panels give more blocks per compute unit (c2, 2000 x 2000 at n_H = 250: two rows
// per block, 0.70 ms of epilogue per solve against 0.83 ms at 28 KB and 1.35 ms at 60 KB)
constexpr size_t kLdsBudget = 20 * 1024;
// Below this width the full Jacobi eigensolver measured faster than the partial one
// (a 256-wide plain Gram at rank 7-9: 125 ms per solve with the full solver, 142 ms with
// the partial one, whose 64 x 64 Rayleigh-Ritz solve and Cholesky steps are latency
// bound); at 2048 the partial one wins (445 -> 300 ms).
constexpr int kPartialMinWidth = 1024;

enum Mode { MODE_STEP = 0, MODE_FINAL = 1, MODE_RECON = 2 };

__device__ __forceinline__ float shrinkf(float e, float thr) {
  const float a = fabsf(e) - thr;
  return a > 0.0f ? copysignf(a, e) : 0.0f;
}

__device__ __forceinline__ bool qbit(const uint32_t* __restrict__ bits, int nw, int i, int j) {
  return (bits[(size_t)i * nw + (j >> 5)] >> (j & 31)) & 1u;
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// restrict the TM x n panel sX (LDS, ld ls) into MP rows i0.. (ld ldp), c < nH
__device__ __forceinline__ void restrict_panel(const float* sX, int ls, int rows, int n, int nH,
                                               float* __restrict__ MP, int ldp, int i0,
                                               const int* __restrict__ col_ptr, const int* __restrict__ col_row,
                                               const float* __restrict__ col_w) {
  if (nH <= 16 && (ls & 1)) {
    // thread -> coarse column c = t / 16 and rows t % 16, + 16, ...: a wave's lanes read
    // one tap of four columns in sixteen rows, from distinct banks (odd row stride)
    const int c = threadIdx.x >> 4, r0 = threadIdx.x & 15;
    if (c >= nH) return;
    const int t0 = col_ptr[c], t1 = col_ptr[c + 1];
    for (int i = r0; i < rows; i += 16) {
      const float* x = sX + (size_t)i * ls;
      float acc = 0.0f;
      for (int t = t0; t < t1; ++t) acc = fmaf(col_w[t], x[col_row[t]], acc);
      MP[(size_t)(i0 + i) * ldp + c] = acc;
    }
    return;
  }
  if (nH <= kThreads) {
    // thread -> coarse column c and rows r0, r0 + rstep, ...: each tap's index and weight
    // are read once for up to four of the thread's rows (same sum order per output)
    const int rstep = kThreads / nH;
    const int r0 = threadIdx.x / nH, c = threadIdx.x % nH;
    if (r0 >= rstep) return;
    const int t0 = col_ptr[c], t1 = col_ptr[c + 1];
    for (int rb = r0; rb < rows; rb += 4 * rstep) {
      float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int t = t0; t < t1; ++t) {
        const int jr = col_row[t];
        const float w = col_w[t];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int i = rb + k * rstep;
          if (i < rows) acc[k] = fmaf(w, sX[(size_t)i * ls + jr], acc[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = rb + k * rstep;
        if (i < rows) MP[(size_t)(i0 + i) * ldp + c] = acc[k];
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < rows * nH; e += kThreads) {
    const int i = e / nH, c = e % nH;
    const float* x = sX + (size_t)i * ls;
    float acc = 0.0f;
    const int t1 = col_ptr[c + 1];
    for (int t = col_ptr[c]; t < t1; ++t) acc = fmaf(col_w[t], x[col_row[t]], acc);
    MP[(size_t)(i0 + i) * ldp + c] = acc;
  }
}

__global__ void k_pack_mask(int m, int n, const uint8_t* __restrict__ Q, int nw, uint32_t* __restrict__ bits) {
  const size_t total = (size_t)m * nw;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / nw;
    const int w = (int)(idx % nw);
    uint32_t v = 0;
    const int j0 = w * 32;
    const int jn = min(32, n - j0);
    for (int b = 0; b < jn; ++b) v |= (Q[i * n + j0 + b] != 0 ? 1u : 0u) << b;
    bits[idx] = v;
  }
}

// Initial coarse data: X_0 = P_Q(D - S0 + Y0/mu0) (or X_0 = M for the standalone SVT),
// M_P = X_0 P (PLAIN: M_P = X_0), and partial sums of ||P_Q D||^2 (NaN if an observed
// entry of D, S0 or Y0 is not finite).
template <bool PLAIN, bool MASKED, bool VEC>
__global__ void __launch_bounds__(kThreads) k_init(int m, int n, int nH, int TM, const float* __restrict__ D,
                                                   int ldd, const uint32_t* __restrict__ bits, int nw,
                                                   const float* __restrict__ S0, const float* __restrict__ Y0,
                                                   float inv_mu0, float* __restrict__ MP, int ldp,
                                                   const int* __restrict__ col_ptr, const int* __restrict__ col_row,
                                                   const float* __restrict__ col_w, double* __restrict__ partial) {
  extern __shared__ float sm[];
  __shared__ double red[kThreads];
  const int i0 = blockIdx.x * TM;
  const int rows = min(TM, m - i0);
  const int ls = PLAIN ? n : (n | 1);   // odd LDS row stride of the staged panel
  double acc = 0.0;
  if (VEC && !PLAIN) {
    // groups of four columns (D, S0, Y0 16-byte aligned rows): one mask word, one float4
    // of each operand per group, four groups per thread in flight
    const int n4 = n >> 2;
    const int total = rows * n4;
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * kThreads) {
      float4 d4[4], s4[4], y4[4];
      uint32_t qb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kThreads;
        if (e < total) {
          const int gi = i0 + e / n4, j0 = 4 * (e % n4);
          qb[u] = MASKED ? (bits[(size_t)gi * nw + (j0 >> 5)] >> (j0 & 31)) & 0xFu : 0xFu;
          d4[u] = *reinterpret_cast<const float4*>(D + (size_t)gi * ldd + j0);
          s4[u] = S0 ? *reinterpret_cast<const float4*>(S0 + (size_t)gi * n + j0) : make_float4(0.f, 0.f, 0.f, 0.f);
          y4[u] = Y0 ? *reinterpret_cast<const float4*>(Y0 + (size_t)gi * n + j0) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kThreads;
        if (e < total) {
          const int i = e / n4, j0 = 4 * (e % n4);
          const float dv[4] = {d4[u].x, d4[u].y, d4[u].z, d4[u].w};
          const float sv[4] = {s4[u].x, s4[u].y, s4[u].z, s4[u].w};
          const float yv[4] = {y4[u].x, y4[u].y, y4[u].z, y4[u].w};
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float x = 0.0f;
            if ((qb[u] >> v) & 1u) {
              acc += (double)dv[v] * (double)dv[v];
              x = dv[v];
              if (S0) x -= sv[v];
              if (Y0) x += yv[v] * inv_mu0;
              acc += (double)(x - x);   // 0, or NaN when D, S0 or Y0 is not finite here
            }
            sm[(size_t)i * ls + j0 + v] = x;
          }
        }
      }
    }
  } else {
    // element e = i n + j, stepped by kThreads without a division per element
    int i = threadIdx.x / n, j = threadIdx.x % n;
    const int di = kThreads / n, dj = kThreads % n;
    for (int e = threadIdx.x; e < rows * n; e += kThreads) {
      const int gi = i0 + i;
      float x = 0.0f;
      if (!MASKED || qbit(bits, nw, gi, j)) {
        const float d = D[(size_t)gi * ldd + j];
        acc += (double)d * (double)d;
        x = d;
        if (S0) x -= S0[(size_t)gi * n + j];
        if (Y0) x += Y0[(size_t)gi * n + j] * inv_mu0;
        acc += (double)(x - x);   // 0, or NaN when D, S0 or Y0 is not finite here
      }
      if (PLAIN)
        MP[(size_t)gi * ldp + j] = x;
      else
        sm[(size_t)i * ls + j] = x;
      j += dj;
      i += di;
      if (j >= n) {
        j -= n;
        ++i;
      }
    }
  }
  if (!PLAIN) {
    __syncthreads();
    restrict_panel(sm, ls, rows, n, nH, MP, ldp, i0, col_ptr, col_row, col_w);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
}

// sigma_k = sqrt(max(lam_perm[k], 0)), r = #{sigma > tau}, sw[k] = sqrt((sigma-tau)/sigma).
// gb (nullable): Gershgorin row bounds of the indices the eigensolver certified below
// tau^2 (else -1); such an index enters the margin through its bound,
// (tau - sqrt(gb)) / tau, a lower bound on the distance of the certified block's
// singular values from tau.
__global__ void __launch_bounds__(kThreads) k_svt_prep(const double* __restrict__ lam, const int* __restrict__ perm,
                                                       int nH, double tau, const double* __restrict__ gb,
                                                       double* __restrict__ sw, IterStats* __restrict__ st,
                                                       const double* __restrict__ trace) {
  __shared__ int cnt[kThreads];
  __shared__ double mg[kThreads];
  __shared__ double tr[kThreads];
  int c = 0;
  double mgn = 1.0e300, trc = 0.0;
  for (int k = threadIdx.x; k < nH; k += kThreads) {
    trc += fmax(lam[perm[k]], 0.0);
    const double sg = sqrt(fmax(lam[perm[k]], 0.0));
    if (sg > tau) {
      ++c;
      sw[k] = sqrt((sg - tau) / sg);
    } else {
      sw[k] = 0.0;
    }
    const double g = gb != nullptr ? gb[perm[k]] : -1.0;
    mgn = fmin(mgn, g >= 0.0 ? (tau - sqrt(g)) / tau : fabs(sg - tau) / tau);
  }
  cnt[threadIdx.x] = c;
  mg[threadIdx.x] = mgn;
  tr[threadIdx.x] = trc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      cnt[threadIdx.x] += cnt[threadIdx.x + w];
      mg[threadIdx.x] = fmin(mg[threadIdx.x], mg[threadIdx.x + w]);
      tr[threadIdx.x] += tr[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->rank = cnt[0];
    st->kform = 0;
    st->margin = mg[0];
    st->trace = trace ? *trace : tr[0];
    st->lam_r = cnt[0] > 0 ? lam[perm[cnt[0] - 1]] : 0.0;
    st->lam_65 = nH > 64 ? lam[perm[64]] : 0.0;
  }
}

// T[c][k] = sum_j C[c][j] V[j][perm[k]] * sw[k] (C = I when PLAIN), k < r;  Tt = T^T.
// Kept in float64: L = (M_P T) T^T extracts a part of the coarse data that can be far
// smaller than the data itself, so both the factor and the sums stay in float64.
template <bool PLAIN>
__global__ void k_build_T(int nH, int N, const double* __restrict__ C, const double* __restrict__ V,
                          const int* __restrict__ perm, const double* __restrict__ sw,
                          const IterStats* __restrict__ st, double* __restrict__ T, double* __restrict__ Tt,
                          int ldT) {
  const int r = st->rank;
  const size_t total = (size_t)nH * nH;   // columns past the rank are written as zero
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / nH), k = (int)(idx % nH);
    double tv = 0.0;
    if (k < r) {
      const int col = perm[k];
      double v;
      if (PLAIN) {
        v = V[(size_t)c * N + col];
      } else {
        v = 0.0;
        for (int j = 0; j < nH; ++j) v += C[(size_t)c * nH + j] * V[(size_t)j * N + col];
      }
      tv = v * sw[k];
    }
    T[(size_t)c * ldT + k] = tv;
    Tt[(size_t)k * ldT + c] = tv;
  }
}

struct EpiArgs {
  int m, n, nH, TM, ldp, nw, ldT;
  const float* D;
  int ldd;
  const uint32_t* bits;
  const float* MPcur;
  float* MPnext;
  const double* T;
  const double* Tt;
  const double* Kw;   // K form: the n_H x n_H product operator (wide path, n_H padded <= 512)
  float* Abuf;        // factor form: A = M_P T (m x rank, ld ldp)
  float* Nbuf;        // N = M_P K (m x n_H, ld ldp), formed before the wide epilogue
  const IterStats* st;
  const float* Zin;   // state (E on Q, L off Q)
  float* Zout;        // may equal Zin
  const float* Y0;    // first iteration: initial multiplier (nullable)
  float* Lout;        // FINAL / RECON
  float* Sout;        // FINAL (may equal Zin)
  float* Yout;        // FINAL (nullable)
  float mu, inv_mu, mu_prev, inv_mu_next, lam, thr;
  float thr_prev;     // lam / mu_{t-1}
  float ratio_prev;   // mu_{t-1} / mu_t
  float grow;         // 1 + mu_t / mu_{t+1}
  int first;
  const int* row_idx;
  const float* row_w;
  const int* col_ptr;
  const int* col_row;
  const float* col_w;
  double* partial;
};

// C (M x N, float32, ldc) = A (M x K, float32, lda) B (K x N, float64, ldb) on float64
// MFMA, the sums rounded to float32 once: the reconstruction products of the wide path
// (N = M_P K, or A = M_P T and N = A T^T in the factor form).  K and N are capped on the
// device by *kcap / *ncap when non-null (the rank of the factor form; output columns at
// or past *ncap are left untouched).  One 32 x 32 output tile per block, four waves of
// one 16 x 16 tile each (v_mfma_f64_16x16x4f64); K in steps of 32 staged in LDS, the next
// step's operands loaded into registers while the current one is multiplied.
__global__ void __launch_bounds__(256) k_recon_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                                    const double* __restrict__ B, int ldb, float* __restrict__ C,
                                                    int ldc, const int* __restrict__ kcap,
                                                    const int* __restrict__ ncap) {
  __shared__ double sA[32][33];
  __shared__ double sB[32][33];
  const int Ke = kcap ? min(K, *kcap) : K;
  const int Ne = ncap ? min(N, *ncap) : N;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;   // row tiles on x (m can be large)
  if (j0 >= Ne) return;   // whole block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  // thread's four staging elements: rows tid / 32 + 8 q, column tid % 32
  const int sr = tid >> 5, scol = tid & 31;
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = sr + 8 * q;
      const int gi = i0 + r, gk = k0 + scol;
      ra[q] = (gi < M && gk < Ke) ? (double)A[(size_t)gi * lda + gk] : 0.0;
      const int gk2 = k0 + r, gj = j0 + scol;
      rb[q] = (gk2 < Ke && gj < N) ? B[(size_t)gk2 * ldb + gj] : 0.0;
    }
  };
  if (Ke > 0) load(0);
  for (int k0 = 0; k0 < Ke; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sA[sr + 8 * q][scol] = ra[q];
      sB[sr + 8 * q][scol] = rb[q];
    }
    __syncthreads();
    if (k0 + 32 < Ke) load(k0 + 32);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const double av = sA[wi * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
      const double bv = sB[ks * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // output register v of lane l: row 4 v + l / 16, column l % 16
  const int gj = j0 + wj * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = i0 + wi * 16 + 4 * v + (lane >> 4);
    if (gi < M && gj < N) C[(size_t)gi * ldc + gj] = (float)acc[v];
  }
}

template <int MODE, bool PLAIN, bool MASKED>
__global__ void __launch_bounds__(kThreads) k_epilogue(EpiArgs a) {
  extern __shared__ float sm[];
  __shared__ double red[kThreads];
  const int nHp = a.ldp;
  float* sN = sm;                               // TM x nHp: N panel
  float* sX = sN + (size_t)a.TM * nHp;          // TM x n  : next coarse data (not PLAIN)
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * a.TM;
  const int rows = min(a.TM, a.m - i0);
  const int nH = a.nH, n = a.n;

  // 1. N panel (N = M_P K, formed on MFMA by k_recon_gemm before this launch)
  for (int e = tid; e < rows * nH; e += kThreads) {
    const int i = e / nH, c = e % nH;
    sN[i * nHp + c] = a.Nbuf[(size_t)(i0 + i) * a.ldp + c];
  }
  __syncthreads();
  // 2. fine elements
  double racc = 0.0;
  for (int e = tid; e < rows * n; e += kThreads) {
    const int i = e / n, j = e % n;
    const int gi = i0 + i;
    float L;
    if (PLAIN) {
      L = sN[i * nHp + j];
    } else {
      const int* ri = a.row_idx + j * kMaxStencil;
      const float* rw = a.row_w + j * kMaxStencil;
      L = 0.0f;
#pragma unroll
      for (int s = 0; s < kMaxStencil; ++s) L = fmaf(rw[s], sN[i * nHp + ri[s]], L);
    }
    const size_t gij = (size_t)gi * n + j;
    if (MODE == MODE_RECON) {
      a.Lout[gij] = L;
      continue;
    }
    const bool q = MASKED ? qbit(a.bits, a.nw, gi, j) : true;
    if (MODE == MODE_FINAL) {
      a.Lout[gij] = L;
      if (q) {
        const float e = a.D[(size_t)gi * a.ldd + j] + a.Zin[gij];   // E = D + W
        a.Sout[gij] = shrinkf(e, a.thr);
        if (a.Yout) a.Yout[gij] = fminf(fmaxf(a.mu * e, -a.lam), a.lam);
      } else {
        a.Sout[gij] = 0.0f;
        if (a.Yout) a.Yout[gij] = 0.0f;
      }
      continue;
    }
    float x;
    if (q) {
      // state W = E - D = -L + Y/mu (small), so no update below cancels large terms
      const float d = a.D[(size_t)gi * a.ldd + j];
      float ym;   // Y_t / mu_t
      if (a.first) {
        ym = a.Y0 ? a.Y0[gij] * a.inv_mu : 0.0f;
      } else {
        const float et = d + a.Zin[gij];                          // E_t
        ym = fminf(fmaxf(et, -a.thr_prev), a.thr_prev) * a.ratio_prev;   // clip(E_t) mu_{t-1}/mu_t
      }
      const float wv = ym - L;                                    // W_{t+1}
      const float c = fminf(fmaxf(d + wv, -a.thr), a.thr);        // clip(E_{t+1}, lam/mu_t)
      const float res = c - ym;                                   // D - L - S
      racc += (double)res * (double)res;
      a.Zout[gij] = wv;
      x = c * a.grow - wv;                                        // D - S + Y_{t+1}/mu_{t+1}
    } else {
      a.Zout[gij] = L;
      x = L;
    }
    if (PLAIN)
      a.MPnext[(size_t)gi * a.ldp + j] = x;
    else
      sX[(size_t)i * n + j] = x;
  }
  if (MODE != MODE_STEP) return;
  if (!PLAIN) {
    __syncthreads();
    restrict_panel(sX, n, rows, n, nH, a.MPnext, a.ldp, i0, a.col_ptr, a.col_row, a.col_w);
  }
  const double s = block_sum(racc, red);
  if (tid == 0) a.partial[blockIdx.x] = s;
}

// W[j][k] = V[j][perm[k]] * sw[k] for k < r (zero beyond): the right factor of
// T = C W, formed on MFMA by gemm_f64.
__global__ void k_build_W(int nH, int N, const double* __restrict__ V, const int* __restrict__ perm,
                          const double* __restrict__ sw, const IterStats* __restrict__ st, double* __restrict__ W) {
  const int r = st->rank;
  const size_t total = (size_t)nH * nH;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nH), k = (int)(idx % nH);
    W[(size_t)j * N + k] = k < r ? V[(size_t)j * N + perm[k]] * sw[k] : 0.0;
  }
}

// Tt = T^T (n_H x n_H block, ld N)
__global__ void k_transpose(int nH, int N, const double* __restrict__ T, double* __restrict__ Tt) {
  const size_t total = (size_t)nH * nH;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / nH), k = (int)(idx % nH);
    Tt[(size_t)k * N + c] = T[(size_t)c * N + k];
  }
}

// K = T T^T (n_H x n_H, float64, ld = ldK), the coarse SVT operator of the tall path:
// L = M_P K P^T.  Entries beyond n_H are zero.
__global__ void k_build_K(int nH, int ldK, const double* __restrict__ T, int ldT, const IterStats* __restrict__ st,
                          double* __restrict__ K) {
  const int r = st->rank;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ldK * ldK) return;
  const int c = idx / ldK, d = idx % ldK;
  double acc = 0.0;
  if (c < nH && d < nH)
    for (int k = 0; k < r; ++k) acc = fma(T[(size_t)c * ldT + k], T[(size_t)d * ldT + k], acc);
  K[idx] = acc;
}

// Epilogue for coarse widths n_H <= kTallNH (the tall, HBM-bound workloads).  A
// persistent grid: each block stages the interpolation stencil (and, at PREC 0, K in
// float64) in LDS once, then loops over tiles of at most kTallRows rows: N = M_P K,
// L = N P^T, the elementwise update (float4 accesses when VEC), and the restriction
// of the next coarse data.  Same arithmetic as k_epilogue.
//
// N = M_P K on MFMA, wave w owning output columns 16w..16w+15 and keeping its K
// fragments in registers for the whole grid-stride loop:
//  * PREC 0: v_mfma_f32_16x16x4_f32 on float32 M_P and K (K rounded from float64);
//    lane l holds A[l%16][4s + l/16] and B[4s + l/16][16w + l%16] at step s;
//  * PREC 2: both split into bfloat16 hi + lo with the three products hi*hi + hi*lo +
//    lo*hi on v_mfma_f32_16x16x32_bf16; lane l holds A[l%16][32s + 8(l/16) + q] and
//    B[32s + 8(l/16) + q][16w + l%16], q < 8.
// Both accumulate in float32; the output register v of lane l is row 4(l/16) + v,
// column 16w + l%16.  PREC 0 serves the float32 solver, PREC 2 the precision form.
constexpr int kTallNH = 64;
constexpr int kTallRows = 16;          // rows per tile (one MFMA row block)
constexpr int kRowBatch = 2;           // rows whose loads a thread issues together
constexpr int kLdA = kTallNH + 8;      // padded LDS row of the M_P tile
constexpr int kLdN = kTallNH + 4;      // padded LDS row of the N tile

template <int MODE, bool MASKED, bool VEC, int PREC, bool NARROW>
__global__ void __launch_bounds__(kThreads) k_epilogue_tall(EpiArgs a, const double* __restrict__ K, int ntiles,
                                                           int nnz) {
  extern __shared__ double smd[];
  __shared__ double red[kThreads];
  static_assert(PREC == 0 || PREC == 2, "reconstruction precision");
  const int n = a.n, nH = a.nH, TM = a.TM;
  float* sMP = reinterpret_cast<float*>(smd);                // 16 x kLdA
  float* sN = sMP + kTallRows * kLdA;                        // 16 x kLdN
  // TM x ls, ls = n | 1 odd: the restriction's lanes (one row each) read the same
  // stencil column of sixteen rows from distinct banks
  const int ls = n | 1;
  float* sX = sN + kTallRows * kLdN;
  int* sRi = reinterpret_cast<int*>(sX + (size_t)TM * ls);   // n x 2
  float* sRw = reinterpret_cast<float*>(sRi + 2 * n);       // n x 2
  int* sCp = reinterpret_cast<int*>(sRw + 2 * n);           // nH + 1
  int* sCr = sCp + (nH + 1);                                // nnz
  float* sCw = reinterpret_cast<float*>(sCr + nnz);         // nnz
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < 2 * n; e += kThreads) {
    sRi[e] = a.row_idx[e];
    sRw[e] = a.row_w[e];
  }
  if (MODE == MODE_STEP) {
    for (int e = tid; e <= nH; e += kThreads) sCp[e] = a.col_ptr[e];
    for (int e = tid; e < nnz; e += kThreads) {
      sCr[e] = a.col_row[e];
      sCw[e] = a.col_w[e];
    }
  }
  const bool wave_on = 16 * wave < nH;
  const int kcol = 16 * wave + (lane & 15);
  float kf[16];                // PREC 0: B fragments, k = 4s + l/16
  bf16x8_t kh[2], kl[2];       // PREC 2: B fragments, k = 32s + 8(l/16) + q
  if (PREC == 0) {
#pragma unroll
    for (int s = 0; s < 16; ++s) kf[s] = (float)K[(4 * s + (lane >> 4)) * kTallNH + kcol];
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double kv = K[(32 * s + 8 * (lane >> 4) + q) * kTallNH + kcol];
        const unsigned short h = f2bf((float)kv);
        kh[s][q] = __builtin_bit_cast(__bf16, h);
        kl[s][q] = __builtin_bit_cast(__bf16, f2bf((float)(kv - (double)bf2f(h))));
      }
  }
  const int ksteps = PREC == 0 ? (nH + 3) / 4 : (nH > 32 ? 2 : 1);
  // fixed-column assignment of the elementwise pass (vector path, n / 4 <= kThreads):
  // thread -> column group ec_j0, rows ec_r0, ec_r0 + ec_rstep, ...
  const int grow = n / 4;
  const bool fixed_cols = VEC && grow <= kThreads;
  const int ec_rstep = fixed_cols ? kThreads / grow : 1;
  const int ec_r0 = fixed_cols ? tid / grow : 0;
  const int ec_j0 = fixed_cols ? 4 * (tid % grow) : 0;
  const bool ec_on = fixed_cols && ec_r0 < ec_rstep;
  int st_i0[4], st_i1[4];
  float st_w0[4], st_w1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = ec_on ? ec_j0 + v : 0;
    st_i0[v] = a.row_idx[2 * j];
    st_i1[v] = a.row_idx[2 * j + 1];
    st_w0[v] = a.row_w[2 * j];
    st_w1[v] = a.row_w[2 * j + 1];
  }
  // restriction.  n_H <= 16: thread -> row rc_r of the 16-row tile and coarse column
  // rc_g (a wave's lanes read one tap of four columns in sixteen rows: with the odd row
  // stride, distinct banks).  Wider: thread -> coarse column rc_c, rows rc_r0 + k rc_rstep
  // (at least 4 rows per pass, each tap's index and weight read once for all of them;
  // measured faster there, 89 against 100 us per launch at n_H = 50)
  const int rc_r = tid & (kTallRows - 1), rc_g = tid / kTallRows;
  const int rc_rstep = kThreads / nH;
  const int rc_r0 = tid / nH, rc_c = tid % nH;
  const bool rc_on = rc_r0 < rc_rstep;
  double racc = 0.0;
  // the M_P rows of the block's next tile are fetched into registers one tile ahead
  constexpr int MPR = kTallRows * kTallNH / kThreads;
  float mpv[MPR];
  auto fetch_mp = [&](int tile) {
    const int r0 = tile * TM, nr = min(TM, a.m - r0);
#pragma unroll
    for (int e = 0; e < MPR; ++e) {
      const int x = tid + kThreads * e;
      const int i = x / kTallNH, c = x % kTallNH;
      mpv[e] = (i < nr && c < nH) ? a.MPcur[(size_t)(r0 + i) * a.ldp + c] : 0.0f;
    }
  };
  if (blockIdx.x < ntiles) fetch_mp(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int i0 = tile * TM;
    const int rows = min(TM, a.m - i0);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < MPR; ++e) {
      const int x = tid + kThreads * e;
      sMP[(x / kTallNH) * kLdA + x % kTallNH] = mpv[e];
    }
    if (tile + (int)gridDim.x < ntiles) fetch_mp(tile + gridDim.x);
    __syncthreads();
    if (wave_on) {                                          // N = M_P K
      f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
      if (PREC == 0) {
        const float* ap = sMP + (lane & 15) * kLdA + (lane >> 4);
#pragma unroll
        for (int s = 0; s < 16; ++s)
          if (s < ksteps) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[4 * s], kf[s], acc, 0, 0, 0);
      } else {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          if (s < ksteps) {
            const float* ap = sMP + (lane & 15) * kLdA + 32 * s + 8 * (lane >> 4);
            const float4 x0 = *reinterpret_cast<const float4*>(ap);
            const float4 x1 = *reinterpret_cast<const float4*>(ap + 4);
            const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            bf16x8_t ah, al;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const unsigned short h = f2bf(xv[q]);
              ah[q] = __builtin_bit_cast(__bf16, h);
              al[q] = __builtin_bit_cast(__bf16, f2bf(xv[q] - bf2f(h)));
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, kh[s], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, kl[s], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, kh[s], acc, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sN[(4 * (lane >> 4) + v) * kLdN + kcol] = acc[v];
    }
    __syncthreads();
    constexpr int V = VEC ? 4 : 1;
    // one element group (V consecutive columns of one row): N -> L through the row
    // stencil, then the elementwise update
    // the loads of one element group (V consecutive columns of row i), then its update
    auto load_group = [&](int i, int j0, float (&dv)[V], float (&zv)[V], uint32_t& qb) {
      if (MODE == MODE_RECON) return;
      const int gi = i0 + i;
      const size_t gij = (size_t)gi * n + j0;
      qb = 0xFu;
      if (MASKED) qb = (a.bits[(size_t)gi * a.nw + (j0 >> 5)] >> (j0 & 31)) & (VEC ? 0xFu : 1u);
      if (VEC) {
        const float4 d4 = *reinterpret_cast<const float4*>(a.D + (size_t)gi * a.ldd + j0);
        dv[0] = d4.x; dv[V > 1 ? 1 : 0] = d4.y; dv[V > 2 ? 2 : 0] = d4.z; dv[V > 3 ? 3 : 0] = d4.w;
        if (MODE == MODE_FINAL || !a.first) {
          const float4 z4 = *reinterpret_cast<const float4*>(a.Zin + gij);
          zv[0] = z4.x; zv[V > 1 ? 1 : 0] = z4.y; zv[V > 2 ? 2 : 0] = z4.z; zv[V > 3 ? 3 : 0] = z4.w;
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) zv[v] = 0.0f;
        }
      } else {
        dv[0] = a.D[(size_t)gi * a.ldd + j0];
        zv[0] = (MODE == MODE_FINAL || !a.first) ? a.Zin[gij] : 0.0f;
      }
    };
    auto element_group = [&](int i, int j0, const float (&Lv)[V], const float (&dv)[V], const float (&zv)[V],
                             uint32_t qb) {
      const int gi = i0 + i;
      const size_t gij = (size_t)gi * n + j0;
      if (MODE == MODE_RECON) {
        if (VEC) {
          *reinterpret_cast<float4*>(a.Lout + gij) =
              make_float4(Lv[0], Lv[V > 1 ? 1 : 0], Lv[V > 2 ? 2 : 0], Lv[V > 3 ? 3 : 0]);
        } else {
          a.Lout[gij] = Lv[0];
        }
        return;
      }
      float o1[V], o2[V], o3[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const bool q = (qb >> v) & 1u;
        if (MODE == MODE_FINAL) {
          const float ev = dv[v] + zv[v];
          o1[v] = Lv[v];
          o2[v] = q ? shrinkf(ev, a.thr) : 0.0f;
          o3[v] = q ? fminf(fmaxf(a.mu * ev, -a.lam), a.lam) : 0.0f;
        } else {
          float ym;
          if (a.first) {
            ym = a.Y0 ? a.Y0[gij + v] * a.inv_mu : 0.0f;
          } else {
            ym = fminf(fmaxf(dv[v] + zv[v], -a.thr_prev), a.thr_prev) * a.ratio_prev;
          }
          const float wv = ym - Lv[v];
          const float c = fminf(fmaxf(dv[v] + wv, -a.thr), a.thr);
          const float res = c - ym;
          if (q) racc += (double)res * (double)res;
          o1[v] = q ? wv : Lv[v];                   // next state
          o2[v] = q ? c * a.grow - wv : Lv[v];      // next coarse data X_{t+1}
        }
      }
      if (MODE == MODE_FINAL) {
        if (VEC) {
          *reinterpret_cast<float4*>(a.Lout + gij) = make_float4(o1[0], o1[V > 1 ? 1 : 0], o1[V > 2 ? 2 : 0], o1[V > 3 ? 3 : 0]);
          *reinterpret_cast<float4*>(a.Sout + gij) = make_float4(o2[0], o2[V > 1 ? 1 : 0], o2[V > 2 ? 2 : 0], o2[V > 3 ? 3 : 0]);
          if (a.Yout)
            *reinterpret_cast<float4*>(a.Yout + gij) = make_float4(o3[0], o3[V > 1 ? 1 : 0], o3[V > 2 ? 2 : 0], o3[V > 3 ? 3 : 0]);
        } else {
          a.Lout[gij] = o1[0];
          a.Sout[gij] = o2[0];
          if (a.Yout) a.Yout[gij] = o3[0];
        }
      } else {
        if (VEC)
          *reinterpret_cast<float4*>(a.Zout + gij) = make_float4(o1[0], o1[V > 1 ? 1 : 0], o1[V > 2 ? 2 : 0], o1[V > 3 ? 3 : 0]);
        else
          a.Zout[gij] = o1[0];
#pragma unroll
        for (int v = 0; v < V; ++v) sX[(size_t)i * ls + j0 + v] = o2[v];
      }
    };
    if (fixed_cols) {
      // every thread keeps the same V columns for all rows of the tile (stencil in
      // registers, no index arithmetic per element); the loads of kRowBatch rows are
      // issued together
      constexpr int RB = kRowBatch;
      if (ec_on)
        for (int i = ec_r0; i < rows; i += RB * ec_rstep) {
          float dv[RB][V], zv[RB][V];
          uint32_t qb[RB];
#pragma unroll
          for (int u = 0; u < RB; ++u)
            if (i + u * ec_rstep < rows) load_group(i + u * ec_rstep, ec_j0, dv[u], zv[u], qb[u]);
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const int ii = i + u * ec_rstep;
            if (ii >= rows) break;
            const float* nrow = sN + ii * kLdN;
            float Lv[V];
#pragma unroll
            for (int v = 0; v < V; ++v) Lv[v] = fmaf(st_w1[v], nrow[st_i1[v]], st_w0[v] * nrow[st_i0[v]]);
            element_group(ii, ec_j0, Lv, dv[u], zv[u], qb[u]);
          }
        }
    } else {
      const int groups = rows * n / V;
      for (int g = tid; g < groups; g += kThreads) {
        const int e = g * V;
        const int i = e / n, j0 = e % n;
        float dv[V], zv[V];
        uint32_t qb = 0;
        load_group(i, j0, dv, zv, qb);
        const float* nrow = sN + i * kLdN;
        float Lv[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int j = j0 + v;
          Lv[v] = fmaf(sRw[2 * j + 1], nrow[sRi[2 * j + 1]], sRw[2 * j] * nrow[sRi[2 * j]]);
        }
        element_group(i, j0, Lv, dv, zv, qb);
      }
    }
    if (MODE == MODE_STEP) {
      __syncthreads();
      // restrict X_{t+1} (same accumulation order in both forms: taps in order)
      if (NARROW) {   // n_H <= kTallRows
        if (rc_r < rows && rc_g < nH) {
          const float* x = sX + (size_t)rc_r * ls;
          float acc = 0.0f;
          const int t0 = sCp[rc_g], t1 = sCp[rc_g + 1];
          // taps in chunks of 8: their indices and weights are read together, then the data
          for (int t = t0; t < t1; t += 8) {
            int cols[8];
            float ws[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              cols[u] = t + u < t1 ? sCr[t + u] : 0;
              ws[u] = t + u < t1 ? sCw[t + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (t + u < t1) acc = fmaf(ws[u], x[cols[u]], acc);
          }
          a.MPnext[(size_t)(i0 + rc_r) * a.ldp + rc_g] = acc;
        }
      } else if (rc_on) {
        float acc[kTallRows / 4] = {};
        const int t0 = sCp[rc_c], t1 = sCp[rc_c + 1];
        for (int t = t0; t < t1; t += 8) {
          int cols[8];
          float ws[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            cols[u] = t + u < t1 ? sCr[t + u] : 0;
            ws[u] = t + u < t1 ? sCw[t + u] : 0.0f;
          }
#pragma unroll
          for (int k = 0; k < kTallRows / 4; ++k) {
            const int i = rc_r0 + k * rc_rstep;
            if (i < rows) {
              const float* x = sX + (size_t)i * ls;
#pragma unroll
              for (int u = 0; u < 8; ++u)
                if (t + u < t1) acc[k] = fmaf(ws[u], x[cols[u]], acc[k]);
            }
          }
        }
#pragma unroll
        for (int k = 0; k < kTallRows / 4; ++k) {
          const int i = rc_r0 + k * rc_rstep;
          if (i < rows) a.MPnext[(size_t)(i0 + i) * a.ldp + rc_c] = acc[k];
        }
      }
    }
  }
  if (MODE != MODE_STEP) return;
  const double sum = block_sum(racc, red);
  if (tid == 0) a.partial[blockIdx.x] = sum;
}

// sums partial[0..cnt) in a fixed order into *out
__global__ void __launch_bounds__(kThreads) k_reduce(const double* __restrict__ partial, int cnt,
                                                     double* __restrict__ out) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < cnt; i += kThreads) s += partial[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

// The per-iteration record the host's stop test reads: the iteration statistics and,
// written after them, the sequence number of the iteration that filled them in.
struct HostStats {
  IterStats st;
  unsigned long long seq;
};

// k_reduce (sum of the blocks' residual partials into st->fg2), then the whole iteration
// record copied to host-mapped memory with its sequence number last, behind a
// system-scope fence: the host can read the record as soon as it sees the number,
// without a copy or a stream synchronisation.
__global__ void __launch_bounds__(kThreads) k_reduce_publish(const double* __restrict__ partial, int cnt,
                                                             IterStats* __restrict__ st, HostStats* host,
                                                             unsigned long long seq) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < cnt; i += kThreads) s += partial[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) {
    st->fg2 = t;
    IterStats c = *st;
    c.fg2 = t;
    host->st = c;
    __threadfence_system();
    *reinterpret_cast<volatile unsigned long long*>(&host->seq) = seq;
  }
}

// One page of pinned, host-mapped memory per host thread for the records the host waits
// on (allocated on the thread's first solve, kept until the process ends; a solve runs to
// completion on its calling thread, so the page is never shared).  Null when the
// allocation fails: the values then come back by a copy and a stream synchronisation.
struct HostPage {
  HostStats stats;
  ProbeRecord probe;
};

struct HostSlot {
  HostPage* host = nullptr;   // host address
  HostPage* dev = nullptr;    // the same memory as the device addresses it
  unsigned long long next = 0;
};

HostSlot* host_slot() {
  thread_local HostSlot slot;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, sizeof(HostPage), hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable) ==
        hipSuccess) {
      HostPage* pg = static_cast<HostPage*>(h);
      pg->stats.seq = 0;
      pg->probe.seq = 0;
      if (hipHostGetDevicePointer(&d, h, 0) == hipSuccess) {
        slot.host = pg;
        slot.dev = static_cast<HostPage*>(d);
      }
    }
    (void)hipGetLastError();
  }
  return slot.host ? &slot : nullptr;
}

// The record with sequence number want, once published.
int wait_published(const HostStats* h, unsigned long long want, hipStream_t s, IterStats* out) {
  MLPCP_TRY(wait_seq(&h->seq, want, s));
  std::memcpy(out, const_cast<const IterStats*>(&h->st), sizeof(IterStats));
  return MLPCP_OK;
}

unsigned grid_for(size_t total) {
  size_t b = (total + kThreads - 1) / kThreads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// ---------------------------------------------------------------------------------
struct Plan {
  int m, n, nH, nHp, levels, TM, nblk, nw;
  bool plain, masked;
  size_t lds_epi, lds_init;
  // tall path (n_H <= kTallNH, not plain): persistent grid over TM_tall-row tiles
  bool tall;
  int TM_tall, ntiles_tall, grid_tall, nnz;
  // leading dimension of the coarse data M_P (m x n_H float32): n_H rounded up to 16 on
  // the tall path (the rows are then 64-byte aligned and nothing beyond is stored),
  // nHp on the wide path (whose epilogue stages M_P rows at that width)
  int ldmp;
  size_t lds_tall;
  // precision of the Gram (0 float64 products, 1 bfloat16, 2 split bfloat16) and of
  // the tall reconstruction N = M_P K (0 float32 MFMA, 2 split bfloat16)
  int gram_prec, recon_prec;
  size_t off_mp0, off_mp1, off_bits, off_G, off_GH, off_tmp, off_V, off_lam, off_gb, off_perm, off_sw, off_T, off_Tt,
      off_K, off_part, off_gram, off_eig, off_stats, off_sub, off_ms, off_Kw, off_N, off_A, total;
  bool sub;   // workspace for the rank-predicted partial eigensolve (solves on the wide path)
  bool ms;    // workspace for the matrix-function SVT (solves on the wide path, n_H <= 512)
  bool kw;    // wide path with the K form of the reconstruction (n_H padded <= 512):
              // N = M_P K, K = C f(G) C; wider models keep the factor form N = (M_P T) T^T
};

int device_cus() {
  static std::atomic<int> cached[64];   // 0 until the first query (zero-initialised static)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cached[dev].load(std::memory_order_relaxed);
  if (!c) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
    cached[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

// Precision form (mlpcp_opts.prec) -> (Gram, reconstruction) kernel precisions.  The
// Gram's precision is chosen per iteration (gram_prec_for; this is the first
// iteration's).  The reconstruction is always split: N = M_P K is a short
// (n_H-term) sum whose bfloat16 rounding would reach L directly at ~3e-3.
void prec_split(int prec, int& gram, int& recon) {
  gram = prec == MLPCP_BF16 ? 1 : prec == MLPCP_BF16X3 ? 2 : 0;
  recon = prec == MLPCP_FP32 ? 0 : 2;
}

// Gram precision of one iteration of a precision-form solve, from rho = tau^2 / trace
// (trace of the previous iteration's coarse Gram; the first iteration has rho = inf).
// A Gram in reduced precision moves the singular values it yields; the iteration may
// use it while that shift stays below 1% of the threshold tau, so that the values
// near tau -- the ones that decide the rank and carry the weights (sigma - tau) --
// are those of the float32 data:
//  * bfloat16 operands are the exact Gram of A + E, |E_ij| <= u |A_ij| (u = 2^-8,
//    independent errors), which moves each sigma by at most ||E||_2 ~
//    (u / sqrt 3)(1/sqrt(n_H) + 1/sqrt(m)) ||A||_F:  rho >= (u^2/3)(..)^2 / 0.01^2;
//  * split operands drop the lo*lo products: the Gram of A + E minus Lo^T Lo, with
//    |Lo_ij| <= u |A_ij|, a symmetric error of norm ~ (u^2/3)(..)^2 trace, plus the
//    float32 rounding of the 32-row chunk sums, ~2^-24 trace / sqrt(m / 32); an
//    eigenvalue error d moves sigma ~ tau by d / (2 tau):  rho >= d / (2 * 0.01 trace);
//  * below both, the Gram takes the float64-product path of the float32 solver.
// tau falls geometrically with mu, so a solve walks down the tiers: the first
// iterations in bfloat16, the middle ones split, the last ones, which fix the result
// and the rank, exact.  MLPCP_BF16X3 skips the bfloat16 tier.
int gram_prec_for(int prec, double tau, double trace_prev, int m, int nH) {
  if (prec == MLPCP_FP32) return 0;
  if (std::isinf(trace_prev)) return prec == MLPCP_BF16 ? 1 : 2;
  if (!(trace_prev > 0.0)) return 0;
  constexpr double u = 1.0 / 256.0, eta = 0.01;
  const double rho = tau * tau / trace_prev;
  const double e1 = 1.0 / std::sqrt((double)nH) + 1.0 / std::sqrt((double)m);
  const double rho_bf16 = (u * u / 3.0) * e1 * e1 / (eta * eta);
  const double d_split = (u * u / 3.0) * e1 * e1 + std::ldexp(1.0, -24) / std::sqrt(std::max(1.0, m / 32.0));
  const double rho_split = d_split / (2.0 * eta);
  if (prec == MLPCP_BF16 && rho >= rho_bf16) return 1;
  if (rho >= rho_split) return 2;
  return 0;
}

}  // namespace

int wait_seq(const unsigned long long* seqp, unsigned long long want, hipStream_t s) {
  for (unsigned spins = 1;; ++spins) {
    if (__atomic_load_n(seqp, __ATOMIC_ACQUIRE) == want) return MLPCP_OK;
    if ((spins & 1023u) == 0u) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) return __atomic_load_n(seqp, __ATOMIC_ACQUIRE) == want ? MLPCP_OK : MLPCP_E_HIP;
      if (q != hipErrorNotReady) return MLPCP_E_HIP;
    }
    __builtin_ia32_pause();
  }
}

namespace {

int make_plan(int m, int n, int levels, bool masked, Plan& p, int prec = MLPCP_FP32, bool partial = false) {
  p.m = m;
  prec_split(prec, p.gram_prec, p.recon_prec);
  p.n = n;
  p.levels = levels;
  p.nH = coarse_dim_checked(n, levels);
  if (p.nH < 1) return MLPCP_E_LEVELS;
  p.nHp = round_up(p.nH, kPad);
  p.plain = (levels == 0);
  p.masked = masked;
  p.nw = (n + 31) / 32;
  const size_t per_row = (size_t)4 * (p.nHp + (p.plain ? 0 : n));
  int TM = (int)(kLdsBudget / per_row);
  if (TM < 1) return MLPCP_E_UNSUPPORTED;
  if (TM > 64) TM = 64;
  p.TM = TM;
  p.nblk = (m + TM - 1) / TM;
  p.lds_epi = (size_t)TM * per_row;
  p.lds_init = p.plain ? 0 : (size_t)TM * (n | 1) * 4;
  p.tall = !p.plain && p.nHp <= kTallNH;
  p.nnz = 0;
  p.TM_tall = 0;
  p.ntiles_tall = 0;
  p.grid_tall = 0;
  p.lds_tall = 0;
  if (p.tall) {
    p.nnz = 2 * n;   // upper bound: at most two weights per fine row
    const size_t fixed = (size_t)4 * kTallRows * (kLdA + kLdN) + (size_t)16 * n + (size_t)4 * (p.nH + 1) +
                         (size_t)8 * p.nnz;
    const size_t per = (size_t)4 * (n | 1);
    const size_t budget = 76 * 1024;   // at least two blocks per 160 KB CU
    int tm = budget > fixed ? (int)((budget - fixed) / per) : 0;
    if (tm > kTallRows) tm = kTallRows;
    if (tm < 1) {
      p.tall = false;
    } else {
      p.TM_tall = tm;
      p.ntiles_tall = (m + tm - 1) / tm;
      p.lds_tall = fixed + (size_t)tm * per;
      // resident blocks per CU from LDS (160 KB, plus the static reduction array)
      const int per_cu = (int)std::min<size_t>(4, (160 * 1024) / (p.lds_tall + kThreads * 8 + 256));
      p.grid_tall = std::min(p.ntiles_tall, std::max(per_cu, 1) * device_cus());
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t nn = (size_t)p.nHp * p.nHp;
  p.ldmp = p.tall ? round_up(p.nH, 16) : p.nHp;
  p.off_mp0 = take((size_t)m * p.ldmp * 4);
  p.off_mp1 = take((size_t)m * p.ldmp * 4);
  p.off_bits = take(masked ? (size_t)m * p.nw * 4 : 0);
  p.off_G = take(nn * 8);
  p.off_GH = take(p.plain ? 0 : nn * 8);
  p.off_tmp = take(p.plain ? 0 : nn * 8);
  p.off_V = take(nn * 8);
  p.off_lam = take((size_t)p.nHp * 8);
  p.off_gb = take((size_t)p.nHp * 8 + 8);   // + the partial eigensolve's trace of G
  p.off_perm = take((size_t)p.nHp * 4);
  p.off_sw = take((size_t)p.nHp * 8);
  p.off_T = take(nn * 8);
  p.off_Tt = take(nn * 8);
  p.off_K = take(p.tall ? (size_t)kTallNH * kTallNH * 8 : 0);
  p.off_part = take((size_t)std::max(p.nblk, 4096) * 8);
  p.off_gram = take(gram_workspace_bytes(m, p.nHp));
  p.off_eig = take(eig_workspace_bytes(p.nHp));
  p.off_stats = take(sizeof(IterStats));
  p.sub = partial && p.nHp >= kPartialMinWidth && subspace_eligible(p.nHp, 1);
  p.off_sub = take(p.sub ? subspace_workspace_bytes(p.nHp) : 0);
  p.ms = partial && !p.tall && msvt_eligible(p.nHp);
  p.off_ms = take(p.ms ? msvt_workspace_bytes(p.nHp) : 0);
  p.kw = !p.tall && p.nHp <= kMsvtMaxWidth;
  p.off_Kw = take(p.kw ? nn * 8 : 0);
  p.off_N = take(p.tall ? 0 : (size_t)m * p.ldmp * 4);
  p.off_A = take(p.tall || p.kw ? 0 : (size_t)m * p.ldmp * 4);
  p.total = off + 256;  // slack for aligning the caller's base pointer
  return MLPCP_OK;
}

struct WS {
  char* base = nullptr;
  void* owned = nullptr;
  ~WS() {
    if (owned) (void)hipFree(owned);
  }
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(base + off);
  }
};

int bind_workspace(const Plan& p, void* ws, size_t ws_bytes, WS& w) {
  if (ws) {
    if (ws_bytes < p.total) return MLPCP_E_WORKSPACE;
    w.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  } else {
    MLPCP_HIP(hipMalloc(&w.owned, p.total));
    w.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(w.owned) + 255) & ~uintptr_t(255));
  }
  return MLPCP_OK;
}

int valid_opts(const mlpcp_opts& o) {
  if (!(o.tol > 0.0) || !std::isfinite(o.tol) || o.max_iter < 1 || !(o.rho >= 1.0) || !std::isfinite(o.rho) ||
      !(o.mu_max_factor >= 1.0) || !std::isfinite(o.mu_max_factor))
    return MLPCP_E_INVALID_ARG;
  if (o.prec != MLPCP_FP32 && o.prec != MLPCP_BF16 && o.prec != MLPCP_BF16X3) return MLPCP_E_INVALID_ARG;
  if (o.check_every != 1 || o.r_norm < 0 || o.r_norm > 2) return MLPCP_E_UNSUPPORTED;
  if (o.svt_method != 0 && o.svt_method != 1) return MLPCP_E_INVALID_ARG;
  return MLPCP_OK;
}

// Eigensolver state carried across the iterations of a solve: the previous rank (which
// decides whether the partial eigensolve is tried) and whether V holds a full orthogonal
// basis (after a partial solve only its leading columns are meaningful, so the next full
// Jacobi starts cold).
struct EigState {
  int r_prev = 0;
  double margin_prev = 0.0;   // the previous SVT's min |sigma - tau| / tau
  double rho = 1.0;           // convergence factor lambda_65 / lambda_r of the previous spectrum
  bool v_full = false;
  int partial_iters = 0;      // iterations whose SVT the partial eigensolve gave
  bool last_partial = false;
  bool ms_on = false;         // the matrix-function SVT may be used (opts and workspace)
  bool ms_prep = false;       // its padded C and C^2 are built
  int ms_iters = 0;           // iterations whose SVT it gave
  int ms_flags = 0;           // iterations whose norm bounds exceeded the assumed caps
  int ms_products = 0;        // N x N x N products those iterations launched
  double trace_prev = 0.0;    // trace of the previous coarse Gram
  double ms_alpha = 0.0, ms_beta = 0.0;   // its norm bounds at the previous iteration (0: none)
};

// Growth allowed for the norm bounds of the matrix-function SVT from one iteration to the
// next (they follow ||G||_2, which moves slowly along a solve); a larger step flags the
// iteration and the rest of the solve takes the eigensolver.
constexpr double kMsvtGrowth = 4.0;

// The partial eigensolve is tried when the previous rank was small and either the
// previous SVT came from it too or the previous spectrum kept a clear gap at the
// threshold: with eigenvalues within a few percent of tau^2 the block's steps converge
// too slowly to pay (the full solver then runs).  (After a partial solve the margin's
// part beyond the block is the certificate's bound, a lower bound close to zero, so it
// cannot serve as the gate.)
constexpr double kPartialMinMargin = 0.05;

// One coarse SVT on M_P (buffer `mp`): Gram, C G C, eigensolve, weights, T.
// certify: let the eigensolver leave undiagonalised what Gershgorin bounds put below
// tau^2 (the whole matrix, whose SVT is then zero, or on wide matrices a block of it);
// V and lam are then not the eigendecomposition, so callers that need it (the SVT's
// derivative) pass false.
int coarse_svt(const Plan& p, const Operator& op, const WS& w, const float* mp, double tau, hipStream_t s,
               int* sweeps, bool warm, bool certify, int gram_prec = -1, EigState* es = nullptr) {
  if (gram_prec < 0) gram_prec = p.gram_prec;
  double* G = w.at<double>(p.off_G);
  double* V = w.at<double>(p.off_V);
  double* lam = w.at<double>(p.off_lam);
  int* perm = w.at<int>(p.off_perm);
  double* sw = w.at<double>(p.off_sw);
  double* T = w.at<double>(p.off_T);
  double* Tt = w.at<double>(p.off_Tt);
  IterStats* st = w.at<IterStats>(p.off_stats);
  MLPCP_TRY(gram_f64(p.m, p.nH, p.nHp, mp, p.ldmp, G, w.at<void>(p.off_gram), s, gram_prec));
  if (p.nHp == kEigInner) {
    // one workgroup from the Gram to the reconstruction factors; sweeps come back in st
    *sweeps = kSweepsOnDevice;
    return coarse_svt_small(p.nH, p.nHp, G, p.plain ? nullptr : op.C, V, warm, tau, certify, lam, perm, sw, T, Tt,
                            p.tall ? w.at<double>(p.off_K) : (p.kw ? w.at<double>(p.off_Kw) : nullptr), st, s);
  }
  double* GH = G;
  const bool ms_path = es && es->ms_on && p.ms && certify;
  if (!p.plain) {
    GH = w.at<double>(p.off_GH);
    if (ms_path) {
      // on the matrix-function SVT's products (exactly symmetric result)
      MLPCP_TRY(msvt_cgc(p.nH, p.nHp, G, op.C, !es->ms_prep, GH, w.at<void>(p.off_ms), s, &es->ms_products));
      es->ms_prep = true;
    } else {
      ProfScope ps(KC_COARSE, s);
      double* tmp = w.at<double>(p.off_tmp);
      MLPCP_TRY(gemm_f64(false, false, p.nH, p.nH, p.nH, 1.0, op.C, p.nH, G, p.nHp, tmp, p.nHp, s));
      MLPCP_TRY(gemm_f64(false, false, p.nH, p.nH, p.nH, 1.0, tmp, p.nHp, op.C, p.nH, GH, p.nHp, s));
    }
  }
  // Matrix-function SVT (no eigenvectors).  After an iteration of rank 0 the Gershgorin
  // discs are tested first (one sync): when they put every eigenvalue below tau^2 the SVT
  // is zero; otherwise their bounds cap the norm bounds of the iteration's first phase.
  // After a nonzero rank the caps are the previous iteration's bounds times the allowed
  // growth, with no sync.
  if (ms_path) {
    const double t = tau * tau;
    double a_est, b_est;
    if (es->r_prev == 0 || !(es->ms_alpha > 0.0)) {
      bool cert = false;
      double gmax = 0.0, trace = 0.0;
      HostSlot* hsl = host_slot();
      const unsigned long long want = hsl ? ++hsl->next : 0;
      MLPCP_TRY(msvt_probe(p.nH, p.nHp, GH, p.nHp, tau, st, w.at<void>(p.off_ms), s, &cert, &gmax, &trace,
                           hsl ? &hsl->host->probe : nullptr, hsl ? &hsl->dev->probe : nullptr, want));
      if (cert) {
        es->v_full = false;
        *sweeps = 0;
        return MLPCP_OK;
      }
      // ||G - t I||_2 <= (max row sum of |G|) + t; ||Gt||_2 = max(||G||_2, t)
      a_est = gmax + t;
      b_est = kMsvtGrowth * std::max(gmax, t);
      (void)trace;
    } else {
      a_est = kMsvtGrowth * es->ms_alpha;
      b_est = kMsvtGrowth * es->ms_beta;
    }
    MsvtPlan mp;
    MLPCP_TRY(msvt_plan(tau, a_est, b_est, &mp));
    MLPCP_TRY(svt_msvt(p.nH, p.nHp, GH, p.nHp, tau, p.plain ? nullptr : op.C, false, mp, w.at<double>(p.off_Kw),
                       p.nHp, st, w.at<void>(p.off_ms), s, &es->ms_products));
    es->v_full = false;
    es->last_partial = false;
    ++es->ms_iters;
    *sweeps = 0;
    return MLPCP_OK;
  }
  double* gb = certify ? w.at<double>(p.off_gb) : nullptr;
  // rank-predicted partial eigensolve (the previous rank was small), else the full one
  bool partial = false;
  double* trace = nullptr;
  const bool was_partial = es && es->last_partial;
  if (es) es->last_partial = false;
  if (es && p.sub && certify && subspace_eligible(p.nHp, es->r_prev) &&
      (was_partial || es->margin_prev >= kPartialMinMargin)) {
    int it = 0;
    double ratio = 1.0;
    double* tr_out = w.at<double>(p.off_gb) + p.nHp;
    MLPCP_TRY(svt_partial(p.nHp, GH, tau, subspace_steps(es->rho), V, lam, perm, gb, tr_out, w.at<void>(p.off_sub), s,
                          &partial, &it, &ratio));
    trace = partial ? tr_out : nullptr;
    if (partial) {
      es->rho = ratio;
      es->v_full = false;
      ++es->partial_iters;
      es->last_partial = true;
      *sweeps = 0;
    }
  }
  if (!partial) {
    const bool warm_ok = warm && (!es || es->v_full);
    // the previous eigensolve's sweep count (in *sweeps on entry) sizes the first batch
    MLPCP_TRY(eig_sym(p.nH, p.nHp, GH, V, lam, perm, w.at<void>(p.off_eig), s, sweeps, warm_ok,
                      warm_ok ? *sweeps : 0, certify ? tau * tau : 0.0, gb));
    if (es) es->v_full = true;
  }
  ProfScope ps(KC_SVT, s);
  hipLaunchKernelGGL(k_svt_prep, dim3(1), dim3(kThreads), 0, s, lam, perm, p.nH, tau, gb, sw, st, trace);
  const size_t tot = (size_t)p.nH * p.nH;
  if (p.plain)
    hipLaunchKernelGGL(k_build_T<true>, dim3(grid_for(tot)), dim3(kThreads), 0, s, p.nH, p.nHp, op.C, V, perm, sw,
                       st, T, Tt, p.nHp);
  else {
    // T = C W on MFMA, W = V_sorted diag(sw) (columns beyond the rank zero)
    double* W = w.at<double>(p.off_tmp);
    hipLaunchKernelGGL(k_build_W, dim3(grid_for(tot)), dim3(kThreads), 0, s, p.nH, p.nHp, V, perm, sw, st, W);
    MLPCP_TRY(gemm_f64(false, false, p.nH, p.nH, p.nH, 1.0, op.C, p.nH, W, p.nHp, T, p.nHp, s));
    hipLaunchKernelGGL(k_transpose, dim3(grid_for(tot)), dim3(kThreads), 0, s, p.nH, p.nHp, T, Tt);
  }
  if (p.tall)
    hipLaunchKernelGGL(k_build_K, dim3((kTallNH * kTallNH + kThreads - 1) / kThreads), dim3(kThreads), 0, s, p.nH,
                       kTallNH, T, p.nHp, st, w.at<double>(p.off_K));
  else if (p.kw)   // K = T T^T for the K form of the reconstruction (T is zero past the rank)
    MLPCP_TRY(gemm_f64(false, false, p.nH, p.nH, p.nH, 1.0, T, p.nHp, Tt, p.nHp, w.at<double>(p.off_Kw), p.nHp, s));
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

// After the stream sync that read `hs`: the sweep count of the last coarse SVT (from
// the device when the one-workgroup path ran) and MLPCP_E_EIG if it hit the cap.
int resolve_sweeps(int& sweeps, const IterStats& hs) {
  if (sweeps == kSweepsOnDevice) sweeps = hs.sweeps;
  return sweeps < 0 ? MLPCP_E_EIG : MLPCP_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <int MODE, bool MASKED, bool VEC>
int launch_tall_one(const Plan& p, const EpiArgs& a, const double* K, int nnz, int grid, hipStream_t s) {
  const bool narrow = p.nH <= kTallRows;
  auto fn = p.recon_prec == 2 ? (narrow ? k_epilogue_tall<MODE, MASKED, VEC, 2, true> : k_epilogue_tall<MODE, MASKED, VEC, 2, false>)
                              : (narrow ? k_epilogue_tall<MODE, MASKED, VEC, 0, true> : k_epilogue_tall<MODE, MASKED, VEC, 0, false>);
  MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)p.lds_tall));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), p.lds_tall, s, a, K, p.ntiles_tall, nnz);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

// Launches the epilogue of the given mode; returns the number of FG partials written.
template <int MODE>
int launch_epilogue(const Plan& p, const EpiArgs& a, const double* K, int nnz, hipStream_t s, int* partials) {
  if (!p.tall) {
    // N = M_P K (K form) or A = M_P T, N = A T^T (factor form, rank columns)
    ProfScope ps(KC_RECON, s);
    const dim3 gb(256);
    const dim3 gg((p.m + 31) / 32, (p.nH + 31) / 32);
    if (p.kw) {
      hipLaunchKernelGGL(k_recon_gemm, gg, gb, 0, s, p.m, p.nH, p.nH, a.MPcur, p.ldmp, a.Kw, p.nHp, a.Nbuf, p.ldmp,
                         nullptr, nullptr);
    } else {
      const int* rk = &a.st->rank;
      hipLaunchKernelGGL(k_recon_gemm, gg, gb, 0, s, p.m, p.nH, p.nH, a.MPcur, p.ldmp, a.T, p.nHp, a.Abuf, p.ldmp,
                         nullptr, rk);
      hipLaunchKernelGGL(k_recon_gemm, gg, gb, 0, s, p.m, p.nH, p.nH, a.Abuf, p.ldmp, a.Tt, p.nHp, a.Nbuf, p.ldmp,
                         rk, nullptr);
    }
    MLPCP_HIP(hipGetLastError());
  }
  ProfScope ps(MODE == MODE_STEP ? KC_EPILOGUE : KC_FINAL, s);
  if (p.tall) {
    const int grid = p.grid_tall;
    *partials = grid;
    const bool vec = (p.n % 4 == 0) && aligned16(a.Lout) && aligned16(a.Zin) && aligned16(a.Zout) &&
                     aligned16(a.Sout) && aligned16(a.Yout) && (MODE == MODE_RECON || (a.ldd % 4 == 0 && aligned16(a.D)));
    EpiArgs b = a;
    b.TM = p.TM_tall;
    if (vec) {
      if (p.masked) return launch_tall_one<MODE, true, true>(p, b, K, nnz, grid, s);
      return launch_tall_one<MODE, false, true>(p, b, K, nnz, grid, s);
    }
    if (p.masked) return launch_tall_one<MODE, true, false>(p, b, K, nnz, grid, s);
    return launch_tall_one<MODE, false, false>(p, b, K, nnz, grid, s);
  }
  *partials = p.nblk;
  const dim3 g(p.nblk), b(kThreads);
  if (p.plain) {
    if (p.masked)
      hipLaunchKernelGGL((k_epilogue<MODE, true, true>), g, b, p.lds_epi, s, a);
    else
      hipLaunchKernelGGL((k_epilogue<MODE, true, false>), g, b, p.lds_epi, s, a);
  } else {
    if (p.masked)
      hipLaunchKernelGGL((k_epilogue<MODE, false, true>), g, b, p.lds_epi, s, a);
    else
      hipLaunchKernelGGL((k_epilogue<MODE, false, false>), g, b, p.lds_epi, s, a);
  }
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

// The reconstruction operands and products of the wide epilogue.
void bind_recon(const Plan& p, const WS& w, EpiArgs& a) {
  a.T = w.at<double>(p.off_T);
  a.Tt = w.at<double>(p.off_Tt);
  a.Kw = p.kw ? w.at<double>(p.off_Kw) : nullptr;
  a.Nbuf = p.tall ? nullptr : w.at<float>(p.off_N);
  a.Abuf = (p.tall || p.kw) ? nullptr : w.at<float>(p.off_A);
}

int launch_init(const Plan& p, const Operator& op, const float* D, int ldd, const uint32_t* bits,
                const float* S0, const float* Y0, float inv_mu0, float* mp, double* partial, hipStream_t s) {
  const dim3 g(p.nblk), b(kThreads);
  ProfScope ps(KC_INIT, s);
  auto a16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  const bool vec = !p.plain && p.n % 4 == 0 && ldd % 4 == 0 && a16(D) && (!S0 || a16(S0)) && (!Y0 || a16(Y0));
#define MLPCP_INIT(PL, MK, VC)                                                                                     \
  hipLaunchKernelGGL((k_init<PL, MK, VC>), g, b, p.lds_init, s, p.m, p.n, p.nH, p.TM, D, ldd, bits, p.nw, S0, Y0, \
                     inv_mu0, mp, p.ldmp, op.col_ptr, op.col_row, op.col_w, partial)
  if (p.plain) {
    if (p.masked)
      MLPCP_INIT(true, true, false);
    else
      MLPCP_INIT(true, false, false);
  } else if (vec) {
    if (p.masked)
      MLPCP_INIT(false, true, true);
    else
      MLPCP_INIT(false, false, true);
  } else {
    if (p.masked)
      MLPCP_INIT(false, true, false);
    else
      MLPCP_INIT(false, false, false);
  }
#undef MLPCP_INIT
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int solve(int m, int n, const float* D, int ldd, const uint8_t* Q, float lambda, double mu0,
          const mlpcp_opts* optp, const float* S0, const float* Y0, float* L, float* S, float* Y, void* ws,
          size_t ws_bytes, mlpcp_info* info, void* stream, bool masked) {
  mlpcp_opts o;
  if (optp)
    o = *optp;
  else
    mlpcp_default_opts(&o);
  if (m < 1 || n < 1 || m < n || ldd < n) return MLPCP_E_SHAPE;
  if (!D || !L || !S || (masked && !Q)) return MLPCP_E_INVALID_ARG;
  if (!(lambda > 0.0f) || !std::isfinite(lambda) || !std::isfinite(mu0)) return MLPCP_E_INVALID_ARG;
  MLPCP_TRY(valid_opts(o));
  if (coarse_dim_checked(n, o.levels) < 1) return MLPCP_E_LEVELS;
  if (L == S || L == Y || (Y && S == Y) || (const float*)L == D || (const float*)S == D) return MLPCP_E_INVALID_ARG;
  if ((S0 && (const float*)L == S0) || (Y0 && (const float*)L == Y0)) return MLPCP_E_INVALID_ARG;
  Plan p;
  MLPCP_TRY(make_plan(m, n, o.levels, masked, p, o.prec, true));
  const size_t need = std::max(p.total, spectral_workspace_bytes(m, n) + 256);
  if (ws && ws_bytes < need) return MLPCP_E_WORKSPACE;

  hipStream_t s = static_cast<hipStream_t>(stream);
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, o.levels, s, &op, o.r_norm));
  Plan pw = p;
  pw.total = need;
  WS w;
  MLPCP_TRY(bind_workspace(pw, ws, ws_bytes, w));
  // default initial penalty mu_0 = 1.25 / ||P_Q D||_2 (the workspace serves this phase
  // first; P_Q D is staged in the L output, which aliases no input)
  double sigma2 = 0.0;
  if (mu0 <= 0.0) {
    const float* A = D;
    int lda = ldd;
    if (masked) {
      MLPCP_TRY(stage_masked(m, n, D, ldd, Q, L, s));
      A = L;
      lda = n;
    }
    MLPCP_TRY(spectral_norm_sq(m, n, A, lda, w.base, s, &sigma2));
    mu0 = (sigma2 > 0.0 && std::isfinite(sigma2)) ? 1.25 / std::sqrt(sigma2) : 1.0;
  }
  float* mp[2] = {w.at<float>(p.off_mp0), w.at<float>(p.off_mp1)};
  uint32_t* bits = masked ? w.at<uint32_t>(p.off_bits) : nullptr;
  double* part = w.at<double>(p.off_part);
  IterStats* st = w.at<IterStats>(p.off_stats);
  if (!p.plain) MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_GH), 0, (size_t)p.nHp * p.nHp * 8, s));
  if (masked) {
    const size_t words = (size_t)m * p.nw;
    hipLaunchKernelGGL(k_pack_mask, dim3(grid_for(words)), dim3(kThreads), 0, s, m, n, Q, p.nw, bits);
  }
  MLPCP_TRY(launch_init(p, *op, D, ldd, bits, S0, Y0, (float)(1.0 / mu0), mp[0], part, s));
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, part, p.nblk, &st->nrm2);
  MLPCP_HIP(hipGetLastError());
  IterStats hs;
  MLPCP_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  if (info) {
    info->mu0 = mu0;
    info->partial_eig_iters = 0;
  }
  // an observed entry of D, S0 or Y0 that is NaN or infinite: nothing is iterated
  if (!std::isfinite(hs.nrm2)) {
    if (info) {
      info->iters = 0;
      info->fg = NAN;
    }
    return MLPCP_E_NONFINITE;
  }
  // P_Q D = 0: the solution is L = S = 0 (and Y = 0), with no iteration
  if (hs.nrm2 == 0.0) {
    MLPCP_HIP(hipMemsetAsync(L, 0, (size_t)m * n * sizeof(float), s));
    MLPCP_HIP(hipMemsetAsync(S, 0, (size_t)m * n * sizeof(float), s));
    if (Y) MLPCP_HIP(hipMemsetAsync(Y, 0, (size_t)m * n * sizeof(float), s));
    MLPCP_HIP(hipStreamSynchronize(s));
    if (info) {
      info->iters = 0;
      info->fg = 0.0;
      info->rank = 0;
      info->mu_final = mu0;
      info->tau_margin = 0.0;
      info->eig_sweeps = 0;
      info->gram_bf16_iters = 0;
      info->gram_split_iters = 0;
    }
    return MLPCP_OK;
  }
  if (!(mu0 > 0.0)) return MLPCP_E_NONFINITE;
  const double nrmD = std::sqrt(hs.nrm2);

  const double mu_max = o.mu_max_factor * mu0;
  double mu = mu0, mu_prev = mu0;
  double fg = INFINITY;
  int t = 0, rank = 0, sweeps = 0;
  double margin = 0.0;
  bool converged = false;
  int status = MLPCP_OK;
  double trace_prev = INFINITY;
  int bf16_iters = 0, split_iters = 0;
  EigState es;
  es.ms_on = o.svt_method == 0 && p.ms;
  HostSlot* slot = host_slot();
  for (t = 0; t < o.max_iter; ++t) {
    const double mu_next = std::min(o.rho * mu, mu_max);
    const int gp = gram_prec_for(o.prec, 1.0 / mu, trace_prev, m, p.nH);
    bf16_iters += gp == 1;
    split_iters += gp == 2;
    MLPCP_TRY(coarse_svt(p, *op, w, mp[t & 1], 1.0 / mu, s, &sweeps, t > 0, true, gp, &es));
    EpiArgs a{};
    a.m = m; a.n = n; a.nH = p.nH; a.TM = p.TM; a.ldp = p.ldmp; a.nw = p.nw; a.ldT = p.nHp;
    a.D = D; a.ldd = ldd; a.bits = bits;
    a.MPcur = mp[t & 1]; a.MPnext = mp[(t + 1) & 1];
    bind_recon(p, w, a); a.st = st;
    a.Zin = S; a.Zout = S; a.Y0 = Y0;
    a.mu = (float)mu; a.inv_mu = (float)(1.0 / mu); a.mu_prev = (float)mu_prev;
    a.inv_mu_next = (float)(1.0 / mu_next); a.lam = lambda; a.thr = (float)(lambda / mu);
    a.thr_prev = (float)(lambda / mu_prev); a.ratio_prev = (float)(mu_prev / mu); a.grow = (float)(1.0 + mu / mu_next);
    a.first = (t == 0);
    a.row_idx = op->row_idx; a.row_w = op->row_w;
    a.col_ptr = op->col_ptr; a.col_row = op->col_row; a.col_w = op->col_w;
    a.partial = part;
    int nparts = 0;
    MLPCP_TRY(launch_epilogue<MODE_STEP>(p, a, w.at<double>(p.off_K), op->nnz, s, &nparts));
    if (slot) {
      const unsigned long long want = ++slot->next;
      {
        ProfScope ps(KC_REDUCE, s);
        hipLaunchKernelGGL(k_reduce_publish, dim3(1), dim3(kThreads), 0, s, part, nparts, st, &slot->dev->stats,
                           want);
      }
      MLPCP_HIP(hipGetLastError());
      MLPCP_TRY(wait_published(&slot->host->stats, want, s, &hs));
    } else {
      {
        ProfScope ps(KC_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, part, nparts, &st->fg2);
      }
      MLPCP_HIP(hipGetLastError());
      MLPCP_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
      MLPCP_HIP(hipStreamSynchronize(s));
    }
    prof_drain();
    MLPCP_TRY(resolve_sweeps(sweeps, hs));
    fg = std::sqrt(hs.fg2) / nrmD;
    rank = hs.rank;
    es.r_prev = rank;
    es.margin_prev = hs.margin;
    if (!es.last_partial) es.rho = hs.lam_r > 0.0 ? std::max(hs.lam_65, 0.0) / hs.lam_r : 1.0;
    margin = hs.margin;
    trace_prev = hs.trace;
    es.trace_prev = hs.trace;
    if (hs.kform) {
      es.ms_alpha = hs.msvt_alpha;
      es.ms_beta = hs.msvt_beta;
      if (hs.msvt_flag) {
        ++es.ms_flags;
        es.ms_on = false;
      }
    }
    if (info && info->fg_history && t < info->history_len) info->fg_history[t] = fg;
    if (info && info->rank_history && t < info->history_len) info->rank_history[t] = rank;
    if (info && info->sweeps_history && t < info->history_len) info->sweeps_history[t] = sweeps;
    if (!std::isfinite(fg)) {
      status = MLPCP_E_NONFINITE;
      ++t;
      break;
    }
    if (fg <= o.tol) {
      converged = true;
      ++t;
      break;
    }
    mu_prev = mu;
    mu = mu_next;
  }
  if (status == MLPCP_OK) {
    // t iterations done; the last one used mu (if converged) -- recompute its L
    const int last = t - 1;
    const double mu_last = converged ? mu : mu_prev;
    EpiArgs a{};
    a.m = m; a.n = n; a.nH = p.nH; a.TM = p.TM; a.ldp = p.ldmp; a.nw = p.nw; a.ldT = p.nHp;
    a.D = D; a.ldd = ldd; a.bits = bits;
    a.MPcur = mp[last & 1]; a.MPnext = nullptr;
    bind_recon(p, w, a); a.st = st;
    a.Zin = S; a.Lout = L; a.Sout = S; a.Yout = Y;
    a.mu = (float)mu_last; a.lam = lambda; a.thr = (float)(lambda / mu_last);
    a.row_idx = op->row_idx; a.row_w = op->row_w;
    int nparts = 0;
    MLPCP_TRY(launch_epilogue<MODE_FINAL>(p, a, w.at<double>(p.off_K), op->nnz, s, &nparts));
    MLPCP_HIP(hipStreamSynchronize(s));
    if (!converged) status = MLPCP_NOT_CONVERGED;
    mu = mu_last;
  }
  if (info) {
    info->iters = t;
    info->fg = fg;
    info->rank = rank;
    info->mu_final = mu;
    info->tau_margin = margin;
    info->eig_sweeps = sweeps;
    info->gram_bf16_iters = bf16_iters;
    info->gram_split_iters = split_iters;
    info->partial_eig_iters = es.partial_iters;
    info->msvt_iters = es.ms_iters;
    info->msvt_flags = es.ms_flags;
    info->msvt_products = es.ms_products;
  }
  return status;
}


// ===================================================================================
// Differentiation form: one explicit iteration of Alg. 4 (Alg. 1 at levels = 0) and
// its vector-Jacobian product, for unrolled solvers.
//
// Step (penalty mu, tau = 1/mu, theta = lam/mu):
//   M = D - S + Y/mu;  A = M R;  F = SVT_tau(A);  L = F R^T;
//   E = D - L + Y/mu;  S' = S_theta[E];  Y' = Y + mu (D - L - S').
// Adjoint, given Lb, S'b, Y'b:
//   Yb += Y'b;  Db += mu Y'b;  Lb -= mu Y'b;  S'b -= mu Y'b
//   Eb = S'b 1[|E| > theta];  lam_b -= sum(S'b sign(E) 1[|E| > theta]) / mu
//   Db += Eb;  Lb -= Eb;  Yb += Eb/mu
//   Fb = Lb R;  Ab = SVT-VJP(A, Fb);  Mb = Ab R^T
//   Db += Mb;  Sb = -Mb;  Yb += Mb/mu
// SVT-VJP with A = U diag(sigma) V^T, f = (sigma - tau)_+, kept set K = {sigma > tau},
// dropped set D: with Phat = V^T A^T Fb V (so that U_i^T Fb V_j = Phat_ij / sigma_i),
//   Ab = A V Omega V^T + Fb V diag(w) V^T,  w = f / sigma,
//   Omega_ij (i, j in K)     = (M_ij - Gb_ij w_j) / sigma_i,
//       Gb_ij = Phat_ij / sigma_i,  M_ij = sym(Gb)_ij + skew(Gb)_ij (f_i + f_j)/(sigma_i + sigma_j)
//   Omega_ij (i in K, j in D) = Omega_ji = (sigma_i - tau)(Phat_ij + Phat_ji) / (sigma_i (sigma_i^2 - sigma_j^2))
//   Omega_ij (i, j in D)     = 0.
// This is the singular-value-function derivative (the SVT Jacobian) with every term in
// a dropped left singular vector u_j rewritten through sigma_j u_j = A v_j: no division
// by a small or zero sigma_j remains, and every coefficient is bounded because
// sigma_i > tau >= sigma_j (the gap guard holds exactly).  With A = M_P C and
// Fb = Fb_P C (Fb_P = Lb P), Phat = Tf^T (M_P^T Fb_P) Tf and
// Mb P-side = M_P (Tf Omega Tf^T) + Fb_P (Tf diag(w) Tf^T), Tf = C V.

__global__ void k_step_elem(int m, int n, const float* __restrict__ D, int ldd, const float* __restrict__ L,
                            const float* __restrict__ Y, float mu, float inv_mu, float thr,
                            float* __restrict__ Sn, float* __restrict__ Yn) {
  const size_t total = (size_t)m * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / n;
    const int j = (int)(idx % n);
    const float d = D[i * ldd + j];
    const float y = Y ? Y[idx] : 0.0f;
    const float e = d - L[idx] + y * inv_mu;
    const float sv = shrinkf(e, thr);
    Sn[idx] = sv;
    Yn[idx] = y + mu * (d - L[idx] - sv);
  }
}

__global__ void __launch_bounds__(kThreads) k_vjp_elem1(int m, int n, const float* __restrict__ D, int ldd,
                                                        const float* __restrict__ L, const float* __restrict__ Y,
                                                        const float* __restrict__ Lb, const float* __restrict__ Sb,
                                                        const float* __restrict__ Yb, float mu, float inv_mu,
                                                        float thr, float* __restrict__ Ltot,
                                                        float* __restrict__ Db, float* __restrict__ Yacc,
                                                        double* __restrict__ lam_part) {
  __shared__ double red[kThreads];
  const size_t total = (size_t)m * n;
  double lacc = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / n;
    const int j = (int)(idx % n);
    const float d = D[i * ldd + j];
    const float y = Y ? Y[idx] : 0.0f;
    const float e = d - L[idx] + y * inv_mu;
    const float yb = Yb ? Yb[idx] : 0.0f;
    const float sb = (Sb ? Sb[idx] : 0.0f) - mu * yb;
    const bool on = fabsf(e) > thr;
    const float eb = on ? sb : 0.0f;
    if (on) lacc -= (double)sb * (e > 0.0f ? 1.0 : -1.0) * (double)inv_mu;
    Ltot[idx] = (Lb ? Lb[idx] : 0.0f) - mu * yb - eb;
    Db[i * ldd + j] += mu * yb + eb;
    Yacc[idx] = yb + eb * inv_mu;
  }
  const double t = block_sum(lacc, red);
  if (threadIdx.x == 0) lam_part[blockIdx.x] = t;
}

__global__ void k_vjp_elem2(int m, int n, const float* __restrict__ Xb, float inv_mu, float* __restrict__ Db, int ldd,
                            float* __restrict__ Sbp, float* __restrict__ Ybp) {
  const size_t total = (size_t)m * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / n;
    const int j = (int)(idx % n);
    const float xb = Xb[idx];
    Db[i * ldd + j] += xb;
    Sbp[idx] = -xb;
    Ybp[idx] = Ybp[idx] + xb * inv_mu;   // Ybp holds the accumulated Y adjoint on entry
  }
}

// Tf[c][k] = sum_j C[c][j] V[j][perm[k]] (C = I when PLAIN), all k < nH; Tw = Tf diag(w)
template <bool PLAIN>
__global__ void k_build_Tf(int nH, int N, const double* __restrict__ C, const double* __restrict__ V,
                           const int* __restrict__ perm, const double* __restrict__ lam, double tau,
                           const IterStats* __restrict__ st, double* __restrict__ Tf, double* __restrict__ Tw) {
  const int r = st->rank;
  const size_t total = (size_t)nH * nH;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / nH), k = (int)(idx % nH);
    const int col = perm[k];
    double v;
    if (PLAIN) {
      v = V[(size_t)c * N + col];
    } else {
      v = 0.0;
      for (int j = 0; j < nH; ++j) v += C[(size_t)c * nH + j] * V[(size_t)j * N + col];
    }
    const double sg = sqrt(fmax(lam[col], 0.0));
    const double wk = (k < r && sg > 0.0) ? (sg - tau) / sg : 0.0;
    Tf[(size_t)c * N + k] = v;
    Tw[(size_t)c * N + k] = v * wk;
  }
}

// Omega (sorted basis, nH x nH, ld N) from Phat, the singular values and tau.
__global__ void k_vjp_coef(int nH, int N, const double* __restrict__ lam, const int* __restrict__ perm, double tau,
                           const IterStats* __restrict__ st, const double* __restrict__ Ph,
                           double* __restrict__ Om) {
  const int r = st->rank;
  const size_t total = (size_t)nH * nH;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / nH), j = (int)(idx % nH);
    const double si = sqrt(fmax(lam[perm[i]], 0.0)), sj = sqrt(fmax(lam[perm[j]], 0.0));
    const bool ki = i < r, kj = j < r;
    const double pij = Ph[(size_t)i * N + j], pji = Ph[(size_t)j * N + i];
    double o = 0.0;
    if (ki && kj) {
      const double gij = pij / si, gji = pji / sj;
      const double fi = si - tau, fj = sj - tau;
      const double cp = (fi + fj) / (si + sj);
      const double mij = (i == j) ? gij : 0.5 * (gij + gji) + 0.5 * (gij - gji) * cp;
      o = (mij - gij * (fj / sj)) / si;
    } else if (ki) {
      o = (si - tau) * (pij + pji) / (si * (si - sj) * (si + sj));
    } else if (kj) {
      o = (sj - tau) * (pij + pji) / (sj * (sj - si) * (sj + si));
    }
    Om[(size_t)i * N + j] = o;
  }
}

// Out(m x k2) = In1 W1 + In2 W2 (float32 inputs, float64 weights and sums), one row per block
__global__ void k_rmul2(int m, int k1, int k2, const float* __restrict__ In1, int ld1, const double* __restrict__ W1,
                        const float* __restrict__ In2, int ld2, const double* __restrict__ W2, int ldw,
                        float* __restrict__ Out, int ldo) {
  const int row = blockIdx.x;
  if (row >= m) return;
  const float* x1 = In1 + (size_t)row * ld1;
  const float* x2 = In2 + (size_t)row * ld2;
  for (int col = threadIdx.x; col < k2; col += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < k1; ++c)
      acc += (double)x1[c] * W1[(size_t)c * ldw + col] + (double)x2[c] * W2[(size_t)c * ldw + col];
    Out[(size_t)row * ldo + col] = (float)acc;
  }
}

struct StepPlan {
  Plan p;
  size_t off_L, off_Ltot, off_Fb, off_Xbp, off_Xb, off_Z, off_Ph, off_Om, off_Tf, off_Tw, off_t1, off_WA, off_WF,
      off_lp, total;
  int lp_blocks;
};

int make_step_plan(int m, int n, int levels, StepPlan& sp) {
  MLPCP_TRY(make_plan(m, n, levels, false, sp.p));
  size_t off = sp.p.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t mn = (size_t)m * n, mh = (size_t)m * sp.p.nHp, nn = (size_t)sp.p.nHp * sp.p.nHp;
  sp.off_L = take(mn * 4);
  sp.off_Ltot = take(mn * 4);
  sp.off_Fb = take(mh * 4);
  sp.off_Xbp = take(mh * 4);
  sp.off_Xb = take(mn * 4);
  sp.off_Z = take(nn * 8);
  sp.off_Ph = take(nn * 8);
  sp.off_Om = take(nn * 8);
  sp.off_Tf = take(nn * 8);
  sp.off_Tw = take(nn * 8);
  sp.off_t1 = take(nn * 8);
  sp.off_WA = take(nn * 8);
  sp.off_WF = take(nn * 8);
  sp.lp_blocks = (int)grid_for(mn);
  sp.off_lp = take((size_t)sp.lp_blocks * 8);
  sp.total = off + 256;
  return MLPCP_OK;
}

// Forward part shared by step and step_vjp: M_P, coarse SVT, L (into Lout).
int step_forward_core(const StepPlan& sp, const Operator& op, const WS& w, const float* D, int ldd, const float* S,
                      const float* Y, double mu, float* Lout, hipStream_t s) {
  const Plan& p = sp.p;
  float* mp = w.at<float>(p.off_mp0);
  if (!p.plain) MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_GH), 0, (size_t)p.nHp * p.nHp * 8, s));
  MLPCP_TRY(launch_init(p, op, D, ldd, nullptr, S, Y, (float)(1.0 / mu), mp, nullptr, s));
  int sweeps = 0;
  MLPCP_TRY(coarse_svt(p, op, w, mp, 1.0 / mu, s, &sweeps, false, false));
  EpiArgs a{};
  a.m = p.m; a.n = p.n; a.nH = p.nH; a.TM = p.TM; a.ldp = p.ldmp; a.nw = p.nw; a.ldT = p.nHp;
  a.MPcur = mp; bind_recon(p, w, a);
  a.st = w.at<IterStats>(p.off_stats);
  a.Lout = Lout;
  a.row_idx = op.row_idx; a.row_w = op.row_w;
  int nparts = 0;
  MLPCP_TRY(launch_epilogue<MODE_RECON>(p, a, w.at<double>(p.off_K), op.nnz, s, &nparts));
  return MLPCP_OK;
}

int step_args_ok(int m, int n, int levels, const float* D, int ldd, float lambda, double mu) {
  if (m < 1 || n < 1 || m < n || ldd < n) return MLPCP_E_SHAPE;
  if (!D) return MLPCP_E_INVALID_ARG;
  if (!(lambda > 0.0f) || !std::isfinite(lambda) || !(mu > 0.0) || !std::isfinite(mu)) return MLPCP_E_INVALID_ARG;
  if (coarse_dim_checked(n, levels) < 1) return MLPCP_E_LEVELS;
  return MLPCP_OK;
}

int svt_prox_args(int m, int n, const float* M, int ldm, int levels, float tau, const float* L) {
  if (m < 1 || n < 1 || m < n || ldm < n) return MLPCP_E_SHAPE;
  if (!M || !L) return MLPCP_E_INVALID_ARG;
  if (!(tau > 0.0f) || !std::isfinite(tau)) return MLPCP_E_INVALID_ARG;
  if (coarse_dim_checked(n, levels) < 1) return MLPCP_E_LEVELS;
  return MLPCP_OK;
}

// L = SVT_tau(M R) R^T with the workspace bound to `w` (plan `p`).  Synchronises.
int svt_prox_core(const Plan& p, const Operator& op, const WS& w, const float* M, int ldm, float tau, float* L,
                  int* rank, hipStream_t s) {
  float* mp = w.at<float>(p.off_mp0);
  if (!p.plain) MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_GH), 0, (size_t)p.nHp * p.nHp * 8, s));
  MLPCP_TRY(launch_init(p, op, M, ldm, nullptr, nullptr, nullptr, 0.0f, mp, nullptr, s));
  int sweeps = 0;
  MLPCP_TRY(coarse_svt(p, op, w, mp, (double)tau, s, &sweeps, false, true));
  EpiArgs a{};
  a.m = p.m; a.n = p.n; a.nH = p.nH; a.TM = p.TM; a.ldp = p.ldmp; a.nw = p.nw; a.ldT = p.nHp;
  a.MPcur = mp; bind_recon(p, w, a);
  a.st = w.at<IterStats>(p.off_stats);
  a.Lout = L;
  a.row_idx = op.row_idx; a.row_w = op.row_w;
  int nparts = 0;
  MLPCP_TRY(launch_epilogue<MODE_RECON>(p, a, w.at<double>(p.off_K), op.nnz, s, &nparts));
  IterStats hs;
  MLPCP_HIP(hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  MLPCP_TRY(resolve_sweeps(sweeps, hs));
  if (rank) *rank = hs.rank;
  return MLPCP_OK;
}

// ---- the allocation-free entry point ------------------------------------------------
// Its workspace (and the operator of the last (n, levels) it served) lives in one
// file-scope device array per GPU.  In host code `scratch` is only a symbol: its device
// address on the current GPU comes from hipGetSymbolAddress, taken once per device on
// the first call there and kept; kernels and copies get that address, never the name.
constexpr size_t kScratchBytes = (size_t)64 << 20;

struct StaticScratch {
  void* ptr = nullptr;
  int op_n = -1, op_levels = -1;   // operator currently built at the start of the array
  Operator op;
};

std::mutex g_scratch_mutex;
StaticScratch g_scratch[64];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

int static_scratch(StaticScratch** out) {
  int dev = 0;
  MLPCP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return MLPCP_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  StaticScratch& sc = g_scratch[dev];
  if (!sc.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return MLPCP_E_HIP;
    sc.ptr = p;
  }
  *out = &sc;
  return MLPCP_OK;
}

}  // namespace

}  // namespace mlpcp

using namespace mlpcp;

extern "C" {

size_t mlpcp_workspace_bytes(int m, int n, const mlpcp_opts* optp) {
  mlpcp_opts o;
  if (optp)
    o = *optp;
  else
    mlpcp_default_opts(&o);
  if (m < 1 || n < 1 || m < n) return 0;
  Plan p;
  if (make_plan(m, n, o.levels, true, p, MLPCP_FP32, true) != MLPCP_OK) return 0;
  // the default-mu_0 phase (mu0 <= 0) runs in the same workspace before the iterations
  return std::max(p.total, spectral_workspace_bytes(m, n) + 256);
}

int mlpcp_pcp_solve(int m, int n, const float* D, int ldd, float lambda, double mu0, const mlpcp_opts* opts,
                    const float* S0, const float* Y0, float* L, float* S, float* Y, void* ws, size_t ws_bytes,
                    mlpcp_info* info, void* stream) {
  return solve(m, n, D, ldd, nullptr, lambda, mu0, opts, S0, Y0, L, S, Y, ws, ws_bytes, info, stream, false);
}

int mlpcp_cpcp_solve(int m, int n, const float* D, int ldd, const uint8_t* Q, float lambda, double mu0,
                     const mlpcp_opts* opts, const float* S0, const float* Y0, float* L, float* S, float* Y,
                     void* ws, size_t ws_bytes, mlpcp_info* info, void* stream) {
  return solve(m, n, D, ldd, Q, lambda, mu0, opts, S0, Y0, L, S, Y, ws, ws_bytes, info, stream, true);
}

int mlpcp_svt_prox(int m, int n, const float* M, int ldm, int levels, float tau, float* L, int* rank, void* ws,
                   size_t ws_bytes, void* stream) {
  MLPCP_TRY(svt_prox_args(m, n, M, ldm, levels, tau, L));
  Plan p;
  MLPCP_TRY(make_plan(m, n, levels, false, p));
  if (ws && ws_bytes < p.total) return MLPCP_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, levels, s, &op));
  WS w;
  MLPCP_TRY(bind_workspace(p, ws, ws_bytes, w));
  return svt_prox_core(p, *op, w, M, ldm, tau, L, rank, s);
}

int mlpcp_svt_prox_static(int m, int n, const float* M, int ldm, int levels, float tau, float* L, int* rank,
                          void* stream) {
  MLPCP_TRY(svt_prox_args(m, n, M, ldm, levels, tau, L));
  Plan p;
  MLPCP_TRY(make_plan(m, n, levels, false, p));
  const size_t op_bytes = align256(operator_bytes(n, levels));
  if (op_bytes + std::max(p.total, operator_tmp_bytes(n, levels)) > kScratchBytes) return MLPCP_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  StaticScratch* sc = nullptr;
  MLPCP_TRY(static_scratch(&sc));
  char* base = static_cast<char*>(sc->ptr);
  // the operator sits at the start of the array, the solver's workspace after it
  if (sc->op_n != n || sc->op_levels != levels) {
    sc->op_n = -1;
    MLPCP_TRY(build_operator_at(n, levels, 0, s, &sc->op, base, base + op_bytes));
    sc->op_n = n;
    sc->op_levels = levels;
  }
  WS w;
  w.base = base + op_bytes;
  return svt_prox_core(p, sc->op, w, M, ldm, tau, L, rank, s);
}

}  // extern "C"

extern "C" {

size_t mlpcp_step_workspace_bytes(int m, int n, int levels) {
  if (m < 1 || n < 1 || m < n) return 0;
  StepPlan sp;
  if (make_step_plan(m, n, levels, sp) != MLPCP_OK) return 0;
  return sp.total;
}

int mlpcp_ialm_step(int m, int n, int levels, const float* D, int ldd, const float* S, const float* Y, float lambda,
                    double mu, float* L, float* S_next, float* Y_next, int* rank, void* ws, size_t ws_bytes,
                    void* stream) {
  MLPCP_TRY(step_args_ok(m, n, levels, D, ldd, lambda, mu));
  if (!L || !S_next || !Y_next) return MLPCP_E_INVALID_ARG;
  StepPlan sp;
  MLPCP_TRY(make_step_plan(m, n, levels, sp));
  if (ws && ws_bytes < sp.total) return MLPCP_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, levels, s, &op));
  WS w;
  Plan tmp = sp.p;
  tmp.total = sp.total;
  MLPCP_TRY(bind_workspace(tmp, ws, ws_bytes, w));
  MLPCP_TRY(step_forward_core(sp, *op, w, D, ldd, S, Y, mu, L, s));
  hipLaunchKernelGGL(k_step_elem, dim3(grid_for((size_t)m * n)), dim3(kThreads), 0, s, m, n, D, ldd, L, Y,
                     (float)mu, (float)(1.0 / mu), (float)(lambda / mu), S_next, Y_next);
  MLPCP_HIP(hipGetLastError());
  IterStats hs;
  MLPCP_HIP(hipMemcpyAsync(&hs, w.at<IterStats>(sp.p.off_stats), sizeof(hs), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  if (sp.p.nHp == kEigInner && hs.sweeps < 0) return MLPCP_E_EIG;
  if (rank) *rank = hs.rank;
  return MLPCP_OK;
}

int mlpcp_ialm_step_vjp(int m, int n, int levels, const float* D, int ldd, const float* S, const float* Y,
                        float lambda, double mu, const float* L_bar, const float* S_bar, const float* Y_bar,
                        float* D_bar, float* S_bar_prev, float* Y_bar_prev, double* lambda_bar, void* ws,
                        size_t ws_bytes, void* stream) {
  MLPCP_TRY(step_args_ok(m, n, levels, D, ldd, lambda, mu));
  if (!D_bar || !S_bar_prev || !Y_bar_prev) return MLPCP_E_INVALID_ARG;
  StepPlan sp;
  MLPCP_TRY(make_step_plan(m, n, levels, sp));
  if (ws && ws_bytes < sp.total) return MLPCP_E_WORKSPACE;
  const Plan& p = sp.p;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, levels, s, &op));
  WS w;
  Plan tmp = sp.p;
  tmp.total = sp.total;
  MLPCP_TRY(bind_workspace(tmp, ws, ws_bytes, w));
  float* Lw = w.at<float>(sp.off_L);
  // recompute the forward step
  MLPCP_TRY(step_forward_core(sp, *op, w, D, ldd, S, Y, mu, Lw, s));
  ProfScope ps(KC_OTHER, s);
  const float inv_mu = (float)(1.0 / mu), thr = (float)(lambda / mu);
  float* Ltot = w.at<float>(sp.off_Ltot);
  double* lp = w.at<double>(sp.off_lp);
  hipLaunchKernelGGL(k_vjp_elem1, dim3(sp.lp_blocks), dim3(kThreads), 0, s, m, n, D, ldd, Lw, Y, L_bar, S_bar, Y_bar,
                     (float)mu, inv_mu, thr, Ltot, D_bar, Y_bar_prev, lp);
  // Fb_P = Ltot P
  const float* FbP = Ltot;
  int ldF = n;
  if (!p.plain) {
    float* fb = w.at<float>(sp.off_Fb);
    MLPCP_TRY(apply_P(*op, m, Ltot, n, fb, p.nHp, s));
    FbP = fb;
    ldF = p.nHp;
  }
  const float* MP = w.at<float>(p.off_mp0);
  double* Z = w.at<double>(sp.off_Z);
  MLPCP_HIP(hipMemsetAsync(Z, 0, (size_t)p.nHp * p.nHp * 8, s));
  MLPCP_TRY(cross_f64(m, p.nH, p.nHp, MP, p.ldmp, FbP, ldF, Z, w.at<void>(p.off_gram), s));
  double* V = w.at<double>(p.off_V);
  double* lam = w.at<double>(p.off_lam);
  int* perm = w.at<int>(p.off_perm);
  const IterStats* st = w.at<IterStats>(p.off_stats);
  double* Tf = w.at<double>(sp.off_Tf);
  double* Tw = w.at<double>(sp.off_Tw);
  const size_t tot = (size_t)p.nH * p.nH;
  if (p.plain)
    hipLaunchKernelGGL(k_build_Tf<true>, dim3(grid_for(tot)), dim3(kThreads), 0, s, p.nH, p.nHp, op->C, V, perm, lam,
                       1.0 / mu, st, Tf, Tw);
  else
    hipLaunchKernelGGL(k_build_Tf<false>, dim3(grid_for(tot)), dim3(kThreads), 0, s, p.nH, p.nHp, op->C, V, perm,
                       lam, 1.0 / mu, st, Tf, Tw);
  double* t1 = w.at<double>(sp.off_t1);
  double* Ph = w.at<double>(sp.off_Ph);
  const int h = p.nH, N = p.nHp;
  MLPCP_TRY(gemm_f64(true, false, h, h, h, 1.0, Tf, N, Z, N, t1, N, s));     // Tf^T Z
  MLPCP_TRY(gemm_f64(false, false, h, h, h, 1.0, t1, N, Tf, N, Ph, N, s));   // (Tf^T Z) Tf
  double* Om = w.at<double>(sp.off_Om);
  hipLaunchKernelGGL(k_vjp_coef, dim3(grid_for(tot)), dim3(kThreads), 0, s, h, N, lam, perm, 1.0 / mu, st, Ph, Om);
  double* WA = w.at<double>(sp.off_WA);
  double* WF = w.at<double>(sp.off_WF);
  MLPCP_TRY(gemm_f64(false, false, h, h, h, 1.0, Tf, N, Om, N, t1, N, s));   // Tf Omega
  MLPCP_TRY(gemm_f64(false, true, h, h, h, 1.0, t1, N, Tf, N, WA, N, s));    // (Tf Omega) Tf^T
  MLPCP_TRY(gemm_f64(false, true, h, h, h, 1.0, Tw, N, Tf, N, WF, N, s));    // Tf diag(w) Tf^T
  float* Xb = w.at<float>(sp.off_Xb);
  if (p.plain) {
    hipLaunchKernelGGL(k_rmul2, dim3(m), dim3(kThreads), 0, s, m, h, h, MP, p.ldmp, WA, FbP, ldF, WF, N, Xb, n);
  } else {
    float* Xbp = w.at<float>(sp.off_Xbp);
    hipLaunchKernelGGL(k_rmul2, dim3(m), dim3(kThreads), 0, s, m, h, h, MP, p.ldmp, WA, FbP, ldF, WF, N, Xbp, p.nHp);
    MLPCP_TRY(apply_Pt(*op, m, Xbp, p.nHp, Xb, n, s));
  }
  hipLaunchKernelGGL(k_vjp_elem2, dim3(grid_for((size_t)m * n)), dim3(kThreads), 0, s, m, n, Xb, inv_mu, D_bar, ldd,
                     S_bar_prev, Y_bar_prev);
  MLPCP_HIP(hipGetLastError());
  if (lambda_bar) {
    double* lsum = w.at<double>(p.off_part);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, lp, sp.lp_blocks, lsum);
    double hl = 0.0;
    MLPCP_HIP(hipMemcpyAsync(&hl, lsum, sizeof(double), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipStreamSynchronize(s));
    *lambda_bar += hl;
  } else {
    MLPCP_HIP(hipStreamSynchronize(s));
  }
  if (p.nHp == kEigInner) {
    IterStats hs;
    MLPCP_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipStreamSynchronize(s));
    if (hs.sweeps < 0) return MLPCP_E_EIG;
  }
  return MLPCP_OK;
}

}  // extern "C"
