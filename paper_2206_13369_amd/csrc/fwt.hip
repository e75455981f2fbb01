// Frank-Wolfe Thresholding (Alg. 3) and multilevel Frank-Wolfe Thresholding (Alg. 6)
// for the unconstrained CPCP problem, eq. (cpcp), in its epigraph form eq. (cpcp-fw):
//
//   f(L, S, t_L, t_S) = 1/2 ||P_Q[L + S - D]||_F^2 + lam_L t_L + lam_S t_S,
//   ||L||_* <= t_L <= U_L,  ||S||_1 <= t_S <= U_S.
//
// One iteration: gradient G = P_Q[L + S - D] (eq. cpcp-grad-LS); nuclear linear oracle
// M_L = -u w^T from the top singular pair of G (FW-T) or of the coarse gradient G R
// lifted by R^T (ML-FWT, radius 1/||R||_2 = 1 for the orthonormal R); l1 oracle at the
// largest |G_ij|; the gates lam >= -<G, M>; exact line search over the two segments
// (a convex quadratic over the unit square); the threshold step on S; the bounds
// U = f / lam.
//
// Structure used by the GPU path (both facts hold exactly in the algorithm):
//  * After a threshold step, S = S_{lam_S}[D - L] on Q and 0 off Q (the S_half terms
//    of the threshold argument cancel on Q; off Q S starts at zero and the l1 atom
//    lives on Q), so G = -P_Q clamp(D - L, -lam_S, lam_S).  S is never stored between
//    iterations: each pass recomputes it from D and L.  Evaluating G in this clipped
//    form also keeps |G| <= lam_S exactly, so rounding cannot open the l1 gate.
//  * ML-FWT atoms are -u (R v_H)^T, so L = Z P^T with Z (m x n_H) in the coarse space
//    (P the interpolation stencil, R = P C, C = (P^T P)^{-1/2}, direction z = C v_H).
//    The line-search inner products that involve the new atom reduce to per-row sums
//    over the coarse columns with the tridiagonal P^T diag(Q_i) P, precomputed once.
//
// Per iteration the ML path streams D and the bit-packed mask once (5/8 + 4 bytes per
// entry); the plain path reads and writes the dense L and the gradient, and runs power
// iterations G^T G x (4 bytes per entry each) for its top singular pair.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "profile.h"

namespace mlpcp {
namespace {

constexpr int kFT = 256;          // threads per block of the streaming kernels
constexpr int kNSums = 8;         // E2, ES, T5..T9, (pad) per block
constexpr int kNTerms = 4;        // S1..S4 per block
constexpr int kPowMax = 500;      // power-iteration steps per FW iteration (cap)
constexpr double kPowEps = 1e-6;  // ||v_new - v_old|| that ends the power iteration

// Device state of one solve, read by the kernels and copied to the host once per
// iteration.
struct FwState {
  double f, t_L, t_S, U_L, U_S;
  double E2, T5, T6, T7, T8, T9;   // sums at the current iterate (see k_fw_finalize)
  double gmax;                     // max |G|
  long long gidx;                  // its flat index i * n + j (smallest among equals)
  double sigma, alpha, beta, gap, coefL;
  int takeL, takeS, thresholded, pad;
  // power iteration (plain path)
  int pow_active, pow_steps;
  double pow_delta;
};

__device__ __forceinline__ float shrinkf(float x, float t) {
  const float a = fabsf(x) - t;
  return a > 0.0f ? copysignf(a, x) : 0.0f;
}
__device__ __forceinline__ float clampf(float x, float t) { return fminf(fmaxf(x, -t), t); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// fixed-order block reduction of NV doubles per thread; result valid in thread 0
template <int NV>
__device__ void block_sums(double (&v)[NV], double* red /* [NV][kFT/64] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k * (kFT / 64) + wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < kFT / 64; ++w) s += red[k * (kFT / 64) + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// (value, index) argmax with ties to the smaller index, across the block
__device__ void block_argmax(float& best, long long& bidx, float* rv, long long* ri) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(best, o, 64);
    const long long oi = __shfl_xor(bidx, o, 64);
    if (ov > best || (ov == best && oi < bidx)) {
      best = ov;
      bidx = oi;
    }
  }
  if (lane == 0) {
    rv[wid] = best;
    ri[wid] = bidx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kFT / 64; ++w)
      if (rv[w] > best || (rv[w] == best && ri[w] < bidx)) {
        best = rv[w];
        bidx = ri[w];
      }
  }
  __syncthreads();
}

// Per-entry arithmetic shared by every kernel that revisits an iterate: from D, L and
// the mask bit, the iterate's S and G.  THR: S has been thresholded (every iteration
// after the first); otherwise S = 0.
template <bool THR>
__device__ __forceinline__ void entry(float d, float l, bool q, float lamS, float& s, float& g) {
  const float x = d - l;
  if (!q) {
    s = 0.0f;
    g = 0.0f;
  } else if (THR) {
    s = shrinkf(x, lamS);
    g = -clampf(x, lamS);
  } else {
    s = 0.0f;
    g = -x;
  }
}

struct Sums {
  double E2 = 0, ES = 0, T5 = 0, T6 = 0, T7 = 0, T8 = 0, T9 = 0;
  float best = -1.0f;
  long long bidx = 0;
  __device__ __forceinline__ void add(float l, float s, float g, bool q, long long idx) {
    if (!q) return;
    const double L = l, S = s, G = g;
    E2 += G * G;
    ES += fabs(S);
    T5 += L * L;
    T6 += G * L;
    T7 += L * S;
    T8 += S * S;
    T9 += G * S;
    const float a = fabsf(g);
    if (a > best || (a == best && idx < bidx)) {
      best = a;
      bidx = idx;
    }
  }
};

__device__ void store_sums(Sums& sm, double* red, float* rv, long long* ri, double* partial, float* pmax,
                           long long* pidx) {
  double v[7] = {sm.E2, sm.ES, sm.T5, sm.T6, sm.T7, sm.T8, sm.T9};
  block_sums<7>(v, red);
  block_argmax(sm.best, sm.bidx, rv, ri);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 7; ++k) partial[(size_t)blockIdx.x * kNSums + k] = v[k];
    pmax[blockIdx.x] = sm.best;
    pidx[blockIdx.x] = sm.bidx;
  }
}

__device__ __forceinline__ bool mask_bit(const uint32_t* __restrict__ bits, int nw, int i, int j) {
  return (bits[(size_t)i * nw + (j >> 5)] >> (j & 31)) & 1u;
}

// packed stencil tap of fine column j: first coarse index (high 16 bits) and the
// numerator of its dyadic weight w0 = num * 2^-levels (low 16 bits); the second tap is
// the next coarse column with weight 1 - w0 (rows of the composite interpolation are
// adjacent pairs that sum to one)
__device__ __forceinline__ void unpack_tap(uint32_t t, float scale, int& c, float& w0) {
  c = (int)(t >> 16);
  w0 = (float)(t & 0xFFFFu) * scale;
}

__device__ __forceinline__ float lift(const float* zrow, int c, float w0, int nH) {
  const float a = w0 * zrow[c];
  return (w0 < 1.0f && c + 1 < nH) ? fmaf(1.0f - w0, zrow[c + 1], a) : a;
}

// ---------------------------------------------------------------------------------
// Multilevel pass over a batch of R rows at a time: Z update (the line-search step of
// the previous iteration), entries (S, G), the sums and the argmax, and the restriction
// GP = G P of the new gradient.
struct PassML {
  int m, n, nH, R, nw, levels;
  const float* D;
  int ldd;
  const uint32_t* bits;
  float* Z;
  int ldz;
  float* GP;
  int ldg;
  const uint32_t* taps;   // [n]
  const int* first;       // [nH + 1]: first fine column whose first tap is c
  const double* T;        // direction z = T[c * ldT] (column 0)
  int ldT;
  const double* gz;       // [m]: G w of the previous iterate (u = gz / sigma)
  const FwState* st;
  float lamS;
  double* partial;
  float* pmax;
  long long* pidx;
};

template <bool MASKED, int VEC, bool THR>
__global__ void __launch_bounds__(kFT) k_fw_pass_ml(PassML a) {
  extern __shared__ char smem_raw[];
  uint32_t* sTap = reinterpret_cast<uint32_t*>(smem_raw);                 // [n]
  int* sFirst = reinterpret_cast<int*>(sTap + a.n);                        // [nH + 1]
  float* sz = reinterpret_cast<float*>(sFirst + a.nH + 1);                 // [nH]
  float* sZ = sz + a.nH;                                                   // [R][nH]
  float* sG = sZ + (size_t)a.R * a.nH;                                     // [R][n]
  __shared__ double red[8 * (kFT / 64)];
  __shared__ float rv[kFT / 64];
  __shared__ long long ri[kFT / 64];
  const int tid = threadIdx.x;
  const float scale = ldexpf(1.0f, -a.levels);
  for (int j = tid; j < a.n; j += kFT) sTap[j] = a.taps[j];
  for (int c = tid; c <= a.nH; c += kFT) sFirst[c] = a.first[c];
  for (int c = tid; c < a.nH; c += kFT) sz[c] = (float)a.T[(size_t)c * a.ldT];
  const double alpha = THR ? a.st->alpha : 0.0;
  const double coefL = THR ? a.st->coefL : 0.0;   // alpha U_L / sigma if the atom is taken
  __syncthreads();
  Sums sm;
  const int nv = a.n / VEC;
  const int nbatch = (a.m + a.R - 1) / a.R;
  for (int b = blockIdx.x; b < nbatch; b += gridDim.x) {
    const int i0 = b * a.R;
    const int rows = min(a.R, a.m - i0);
    // Z <- (1 - alpha) Z - alpha U_L u z^T  (first iteration: Z = 0)
    for (int t = tid; t < rows * a.nH; t += kFT) {
      const int r = t / a.nH, c = t - r * a.nH;
      const int i = i0 + r;
      float zv = 0.0f;
      if (THR) {
        zv = (float)((1.0 - alpha) * (double)a.Z[(size_t)i * a.ldz + c] - coefL * a.gz[i] * (double)sz[c]);
        a.Z[(size_t)i * a.ldz + c] = zv;
      }
      sZ[r * a.nH + c] = zv;
    }
    __syncthreads();
    for (int f = tid; f < rows * nv; f += kFT) {
      const int r = f / nv, s = f - r * nv;
      const int i = i0 + r, j = s * VEC;
      const float* drow = a.D + (size_t)i * a.ldd;
      float d[VEC];
      if constexpr (VEC == 4) {
        const float4 v = *reinterpret_cast<const float4*>(drow + j);
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      } else {
        d[0] = drow[j];
      }
      uint32_t qb = 0xFu;
      if (MASKED) qb = (a.bits[(size_t)i * a.nw + (j >> 5)] >> (j & 31)) & (VEC == 4 ? 0xFu : 0x1u);
      const float* zr = sZ + r * a.nH;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        int c;
        float w0;
        unpack_tap(sTap[j + e], scale, c, w0);
        const float l = lift(zr, c, w0, a.nH);
        const bool q = (qb >> e) & 1u;
        float sv, gv;
        entry<THR>(d[e], l, q, a.lamS, sv, gv);
        sm.add(l, sv, gv, q, (long long)i * a.n + j + e);
        sG[r * a.n + j + e] = gv;
      }
    }
    __syncthreads();
    // GP[i][c] = sum_j G_ij P_jc: fine columns whose first tap is c (weight w0) and
    // those whose first tap is c - 1 (weight 1 - w0), in a fixed order
    for (int t = tid; t < rows * a.nH; t += kFT) {
      const int r = t / a.nH, c = t - r * a.nH;
      const float* g = sG + r * a.n;
      double acc = 0.0;
      for (int j = sFirst[c]; j < sFirst[c + 1]; ++j) acc += (double)((float)(sTap[j] & 0xFFFFu) * scale) * g[j];
      if (c > 0)
        for (int j = sFirst[c - 1]; j < sFirst[c]; ++j)
          acc += (double)(1.0f - (float)(sTap[j] & 0xFFFFu) * scale) * g[j];
      a.GP[(size_t)(i0 + r) * a.ldg + c] = (float)acc;
    }
    __syncthreads();
  }
  store_sums(sm, red, rv, ri, a.partial, a.pmax, a.pidx);
}

// ---------------------------------------------------------------------------------
// Plain pass: dense L update, entries, sums, argmax; writes L and the gradient G.
struct PassPlain {
  int m, n, nw;
  const float* D;
  int ldd;
  const uint32_t* bits;
  float* L;               // ld = n
  float* G;               // ld = n
  const double* w;        // [n] direction of the previous iterate
  const double* gz;       // [m]
  const FwState* st;
  float lamS;
  double* partial;
  float* pmax;
  long long* pidx;
};

template <bool MASKED, int VEC, bool THR>
__global__ void __launch_bounds__(kFT) k_fw_pass_plain(PassPlain a) {
  __shared__ double red[8 * (kFT / 64)];
  __shared__ float rv[kFT / 64];
  __shared__ long long ri[kFT / 64];
  const double alpha = THR ? a.st->alpha : 0.0;
  const double coefL = THR ? a.st->coefL : 0.0;
  const float oma = (float)(1.0 - alpha);
  Sums sm;
  const unsigned nv = (unsigned)(a.n / VEC);
  const unsigned total = (unsigned)a.m * nv;   // < 2^31 (checked on the host)
  for (unsigned f = blockIdx.x * kFT + threadIdx.x; f < total; f += gridDim.x * kFT) {
    const int i = (int)(f / nv);
    const int j = (int)(f - (unsigned)i * nv) * VEC;
    const float* drow = a.D + (size_t)i * a.ldd;
    float* lrow = a.L + (size_t)i * a.n;
    float d[VEC], l[VEC];
    if constexpr (VEC == 4) {
      const float4 v = *reinterpret_cast<const float4*>(drow + j);
      d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      if (THR) {
        const float4 x = *reinterpret_cast<const float4*>(lrow + j);
        l[0] = x.x; l[1] = x.y; l[2] = x.z; l[3] = x.w;
      } else {
        l[0] = l[1] = l[2] = l[3] = 0.0f;
      }
    } else {
      d[0] = drow[j];
      l[0] = THR ? lrow[j] : 0.0f;
    }
    uint32_t qb = 0xFu;
    if (MASKED) qb = (a.bits[(size_t)i * a.nw + (j >> 5)] >> (j & 31)) & (VEC == 4 ? 0xFu : 0x1u);
    const double cu = THR ? coefL * a.gz[i] : 0.0;
    float g[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      // L <- (1 - alpha) L - alpha U_L u_i w_j  (first iteration: L = 0)
      l[e] = THR ? (float)((double)(oma * l[e]) - cu * a.w[j + e]) : 0.0f;
      const bool q = (qb >> e) & 1u;
      float sv;
      entry<THR>(d[e], l[e], q, a.lamS, sv, g[e]);
      sm.add(l[e], sv, g[e], q, (long long)i * a.n + j + e);
    }
    if constexpr (VEC == 4) {
      *reinterpret_cast<float4*>(lrow + j) = make_float4(l[0], l[1], l[2], l[3]);
      *reinterpret_cast<float4*>(a.G + (size_t)i * a.n + j) = make_float4(g[0], g[1], g[2], g[3]);
    } else {
      lrow[j] = l[0];
      a.G[(size_t)i * a.n + j] = g[0];
    }
  }
  store_sums(sm, red, rv, ri, a.partial, a.pmax, a.pidx);
}

// Sums the pass partials in a fixed order; f, t_S and the bounds U = f / lam at the
// current iterate.
__global__ void __launch_bounds__(64) k_fw_finalize(const double* __restrict__ partial,
                                                    const float* __restrict__ pmax,
                                                    const long long* __restrict__ pidx, int nb, double lamL,
                                                    double lamS, int thr, FwState* st) {
  const int lane = threadIdx.x;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  float best = -1.0f;
  long long bi = 0;
  for (int b = lane; b < nb; b += 64) {
    for (int k = 0; k < 7; ++k) v[k] += partial[(size_t)b * kNSums + k];
    if (pmax[b] > best || (pmax[b] == best && pidx[b] < bi)) {
      best = pmax[b];
      bi = pidx[b];
    }
  }
  for (int k = 0; k < 7; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(best, o, 64);
    const long long oi = __shfl_xor(bi, o, 64);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    st->E2 = v[0];
    st->t_S = v[1];
    st->T5 = v[2];
    st->T6 = v[3];
    st->T7 = v[4];
    st->T8 = v[5];
    st->T9 = v[6];
    st->gmax = (double)best;
    st->gidx = bi;
    st->thresholded = thr;
    st->f = 0.5 * v[0] + lamL * st->t_L + lamS * v[1];
    st->U_L = st->f / lamL;
    st->U_S = st->f / lamS;
  }
}

// ---------------------------------------------------------------------------------
// Line-search terms.  For the direction w (unit, fine) of the nuclear atom, per row i:
//   gz_i = sum_j G_ij w_j,  lz_i = sum_j Q_ij L_ij w_j,  dz_i = sum_j Q_ij D_ij w_j,
//   qz_i = sum_j Q_ij w_j^2,
// and the block sums S1 = sum gz^2, S2 = sum gz^2 qz, S3 = sum gz lz, S4 = sum gz dz.

// multilevel: w = P z, so with A_ic = sum_j Q_ij P_jc^2, B_ic = sum_j Q_ij P_jc P_j,c+1
// (P^T diag(Q_i) P is tridiagonal) and QDP = (Q o D) P:
//   gz_i = GP_i . z,  dz_i = QDP_i . z,  qz_i = z^T Mq_i z,  lz_i = z^T Mq_i Z_i^T.
struct TermsML {
  int m, nH;
  const float *Z, *GP, *Aq, *Bq, *QDP;
  int ld;                 // leading dimension of all five
  const double* T;        // z = column 0
  int ldT;
  double* gz;
  double* partial;
};

__global__ void __launch_bounds__(kFT) k_fw_terms_ml(TermsML a) {
  extern __shared__ double sz[];   // [nH]
  __shared__ double red[4 * (kFT / 64)];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < a.nH; c += kFT) sz[c] = a.T[(size_t)c * a.ldT];
  __syncthreads();
  double acc[4] = {0, 0, 0, 0};
  for (int i = blockIdx.x * (kFT / 64) + wid; i < a.m; i += gridDim.x * (kFT / 64)) {
    const size_t o = (size_t)i * a.ld;
    double g = 0, l = 0, d = 0, q = 0;
    for (int c = lane; c < a.nH; c += 64) {
      const double zc = sz[c];
      const double A = a.Aq[o + c], B = a.Bq[o + c];
      const double zn = c + 1 < a.nH ? sz[c + 1] : 0.0;
      const double Zc = a.Z[o + c];
      const double Zn = c + 1 < a.nH ? (double)a.Z[o + c + 1] : 0.0;
      const double Zp = c > 0 ? (double)a.Z[o + c - 1] : 0.0;
      const double Bp = c > 0 ? (double)a.Bq[o + c - 1] : 0.0;
      g += zc * a.GP[o + c];
      d += zc * a.QDP[o + c];
      l += zc * (A * Zc + B * Zn + Bp * Zp);
      q += A * zc * zc + 2.0 * B * zc * zn;
    }
    g = wave_sum(g);
    l = wave_sum(l);
    d = wave_sum(d);
    q = wave_sum(q);
    if (lane == 0) {
      a.gz[i] = g;
      acc[0] += g * g;
      acc[1] += g * g * q;
      acc[2] += g * l;
      acc[3] += g * d;
    }
  }
  block_sums<4>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.partial[(size_t)blockIdx.x * kNTerms + k] = acc[k];
}

// plain: one wave per row over the fine columns (G recomputed from D and L)
struct TermsPlain {
  int m, n, nw;
  const float* D;
  int ldd;
  const uint32_t* bits;
  const float* L;
  const double* w;
  float lamS;
  int thr;
  double* gz;
  double* partial;
};

template <bool MASKED, bool THR>
__global__ void __launch_bounds__(kFT) k_fw_terms_plain(TermsPlain a) {
  extern __shared__ double sw[];   // [n]
  __shared__ double red[4 * (kFT / 64)];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < a.n; j += kFT) sw[j] = a.w[j];
  __syncthreads();
  double acc[4] = {0, 0, 0, 0};
  for (int i = blockIdx.x * (kFT / 64) + wid; i < a.m; i += gridDim.x * (kFT / 64)) {
    const float* drow = a.D + (size_t)i * a.ldd;
    const float* lrow = a.L + (size_t)i * a.n;
    double g = 0, l = 0, d = 0, q = 0;
    for (int j = lane; j < a.n; j += 64) {
      const bool qq = MASKED ? mask_bit(a.bits, a.nw, i, j) : true;
      if (!qq) continue;
      const float dv = drow[j], lv = lrow[j];
      float sv, gv;
      entry<THR>(dv, lv, true, a.lamS, sv, gv);
      const double wj = sw[j];
      g += (double)gv * wj;
      l += (double)lv * wj;
      d += (double)dv * wj;
      q += wj * wj;
    }
    g = wave_sum(g);
    l = wave_sum(l);
    d = wave_sum(d);
    q = wave_sum(q);
    if (lane == 0) {
      a.gz[i] = g;
      acc[0] += g * g;
      acc[1] += g * g * q;
      acc[2] += g * l;
      acc[3] += g * d;
    }
  }
  block_sums<4>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) a.partial[(size_t)blockIdx.x * kNTerms + k] = acc[k];
}

// ---------------------------------------------------------------------------------
// The step: gates, the exact line search and the t_L update (one thread, float64).
__device__ void box_qp(double haa, double hab, double hbb, double ga, double gb, double& ra, double& rb) {
  auto phi = [&](double x, double y) { return 0.5 * (haa * x * x + 2.0 * hab * x * y + hbb * y * y) + ga * x + gb * y; };
  auto c01 = [](double x) { return fmin(1.0, fmax(0.0, x)); };
  double ba = 0.0, bb = 0.0, bv = phi(0.0, 0.0);
  auto consider = [&](double x, double y) {
    const double v = phi(x, y);
    if (v < bv) {
      bv = v;
      ba = x;
      bb = y;
    }
  };
  consider(1.0, 0.0);
  consider(0.0, 1.0);
  consider(1.0, 1.0);
  if (haa > 0.0) {
    consider(c01(-(ga + hab * 0.0) / haa), 0.0);
    consider(c01(-(ga + hab * 1.0) / haa), 1.0);
  }
  if (hbb > 0.0) {
    consider(0.0, c01(-(gb + hab * 0.0) / hbb));
    consider(1.0, c01(-(gb + hab * 1.0) / hbb));
  }
  const double det = haa * hbb - hab * hab;
  if (det > 0.0) {
    const double x = (-ga * hbb + gb * hab) / det;
    const double y = (-gb * haa + ga * hab) / det;
    if (x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0) consider(x, y);
  }
  ra = ba;
  rb = bb;
}

struct SolveArgs {
  int m, n, nH, levels;
  const double* partial;  // terms partials
  int nb;
  const float* D;
  int ldd;
  // the iterate's L at the argmax: plain L (ld n) or Z (ldz) with the stencil taps
  const float* L;
  const float* Z;
  int ldz;
  const uint32_t* taps;
  const double* T;        // ML direction z (column 0)
  int ldT;
  const double* w;        // plain direction
  const double* gz;
  double lamL, lamS;
  FwState* st;
};

__global__ void __launch_bounds__(64) k_fw_solve(SolveArgs a) {
  const int lane = threadIdx.x;
  double v[4] = {0, 0, 0, 0};
  for (int b = lane; b < a.nb; b += 64)
    for (int k = 0; k < 4; ++k) v[k] += a.partial[(size_t)b * kNTerms + k];
  for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
  if (lane != 0) return;
  FwState* st = a.st;
  const double S1 = v[0], S2 = v[1], S3 = v[2], S4 = v[3];
  const double sigma = sqrt(S1);
  const double U_L = st->U_L, U_S = st->U_S;
  const bool takeL = !(a.lamL >= sigma);
  const bool takeS = !(a.lamS >= st->gmax);
  // the iterate at the argmax entry (observed whenever max |G| > 0)
  const long long gi = st->gidx;
  const int is = (int)(gi / a.n), js = (int)(gi - (long long)is * a.n);
  const float dstar = a.D[(size_t)is * a.ldd + js];
  float lstar;
  double wstar;
  if (a.levels > 0) {
    const float scale = ldexpf(1.0f, -a.levels);
    int c;
    float w0;
    unpack_tap(a.taps[js], scale, c, w0);
    const float* zr = a.Z + (size_t)is * a.ldz;
    lstar = lift(zr, c, w0, a.nH);
    wstar = (double)w0 * a.T[(size_t)c * a.ldT];
    if (w0 < 1.0f && c + 1 < a.nH) wstar += (double)(1.0f - w0) * a.T[(size_t)(c + 1) * a.ldT];
  } else {
    lstar = a.L[(size_t)is * a.n + js];
    wstar = a.w[js];
  }
  float sstar, gstar;
  if (st->thresholded)
    entry<true>(dstar, lstar, true, (float)a.lamS, sstar, gstar);
  else
    entry<false>(dstar, lstar, true, (float)a.lamS, sstar, gstar);
  double T1 = 0, T2 = 0, T3 = 0, T4 = 0, VLs = 0, VtL = 0;
  if (takeL) {
    T1 = U_L * U_L * S2 / S1;
    T2 = -U_L * S3 / sigma;
    T3 = -U_L * sigma;
    T4 = -U_L * (sigma - S3 / sigma + S4 / sigma);
    VLs = -U_L * (a.gz[is] / sigma) * wstar;
    VtL = U_L;
  }
  const double sg = gstar > 0.0f ? 1.0 : (gstar < 0.0f ? -1.0 : 0.0);
  const double VSs = takeS ? -U_S * sg : 0.0;
  const double VtS = takeS ? U_S : 0.0;
  const double Ls = lstar, Ss = sstar, Gs = gstar;
  const double haa = T1 - 2.0 * T2 + st->T5;
  const double hab = -T4 + st->T7 + (VLs - Ls) * VSs;
  const double hbb = st->T8 + VSs * VSs - 2.0 * VSs * Ss;
  const double ga = T3 - st->T6 + a.lamL * (VtL - st->t_L);
  const double gb = -st->T9 + Gs * VSs + a.lamS * (VtS - st->t_S);
  double al, be;
  box_qp(haa, hab, hbb, ga, gb, al, be);
  st->sigma = sigma;
  st->takeL = takeL;
  st->takeS = takeS;
  st->alpha = al;
  st->beta = be;
  st->gap = -(ga + gb);
  st->coefL = takeL ? al * U_L / sigma : 0.0;
  st->t_L = st->t_L + al * (VtL - st->t_L);
}

// ---------------------------------------------------------------------------------
// Plain top singular pair: power iteration x <- G^T G x / ||G^T G x|| on the stored
// gradient, warm-started from the previous direction.  Each step: per-block partial
// sums of G^T (G x) over its rows (fixed order), a column reduction over the blocks,
// then the normalisation and the convergence test.  All kernels return at once when
// the iteration has converged (device-gated steps, queued in batches by the host).
struct PowArgs {
  int m, n, gs, rpb;      // group size (threads per row), rows per block
  const float* G;
  double* x;              // [n] current direction (unit)
  double* partial;        // [nb][n]
  double* y;              // [n]
  double* ypart;          // [nbc]
  FwState* st;
};

template <int VEC, int NS>
__global__ void __launch_bounds__(kFT) k_fw_power(PowArgs a) {
  if (!a.st->pow_active) return;
  extern __shared__ double sx[];   // [n] x, then [n] the block's G^T G x
  __shared__ double wsum[kFT / 64];
  const int tid = threadIdx.x;
  const int g = tid / a.gs, l = tid - g * a.gs;
  const int R = kFT / a.gs;
  const int nv = a.n / VEC;
  for (int j = tid; j < a.n; j += kFT) sx[j] = a.x[j];
  __syncthreads();
  double acc[NS * VEC];
#pragma unroll
  for (int k = 0; k < NS * VEC; ++k) acc[k] = 0.0;
  const int r0 = blockIdx.x * a.rpb;
  const int r1 = min(a.m, r0 + a.rpb);
  const int wpg = a.gs / 64;       // waves per group
  for (int base = r0; base < r1; base += R) {
    const int i = base + g;
    const bool valid = i < r1;
    float v[NS * VEC];
    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int s = l + a.gs * k;
      if (valid && s < nv) {
        const float* gp = a.G + (size_t)i * a.n + (size_t)s * VEC;
        if constexpr (VEC == 4) {
          const float4 t = *reinterpret_cast<const float4*>(gp);
          v[k * 4] = t.x; v[k * 4 + 1] = t.y; v[k * 4 + 2] = t.z; v[k * 4 + 3] = t.w;
        } else {
          v[k * VEC] = gp[0];
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) dot += (double)v[k * VEC + e] * sx[s * VEC + e];
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[k * VEC + e] = 0.0f;
      }
    }
    dot = wave_sum(dot);
    if ((tid & 63) == 0) wsum[tid >> 6] = dot;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < wpg; ++w) t += wsum[g * wpg + w];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS * VEC; ++k) acc[k] += t * (double)v[k];
  }
  // combine the R groups in the block (fixed order), then store the block's partial
  double* sy = sx + a.n;
  for (int j = tid; j < a.n; j += kFT) sy[j] = 0.0;
  __syncthreads();
  for (int gg = 0; gg < R; ++gg) {
    if (g == gg) {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int s = l + a.gs * k;
        if (s < nv)
#pragma unroll
          for (int e = 0; e < VEC; ++e) sy[s * VEC + e] += acc[k * VEC + e];
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < a.n; j += kFT) a.partial[(size_t)blockIdx.x * a.n + j] = sy[j];
}

// y_j = sum over blocks of partial[b][j]; per-block sums of y_j^2
__global__ void __launch_bounds__(kFT) k_fw_power_cols(PowArgs a, int nb) {
  if (!a.st->pow_active) return;
  __shared__ double red[kFT / 64];
  double sq = 0.0;
  const int j = blockIdx.x * kFT + threadIdx.x;
  if (j < a.n) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += a.partial[(size_t)b * a.n + j];
    a.y[j] = s;
    sq = s * s;
  }
  double v[1] = {sq};
  block_sums<1>(v, red);
  if (threadIdx.x == 0) a.ypart[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kFT) k_fw_power_fin(PowArgs a, int nbc) {
  if (!a.st->pow_active) return;
  __shared__ double red[kFT / 64];
  __shared__ double snorm;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nbc; ++b) s += a.ypart[b];
    snorm = sqrt(s);
  }
  __syncthreads();
  const double nrm = snorm;
  double d2 = 0.0;
  for (int j = threadIdx.x; j < a.n; j += kFT) {
    const double vn = nrm > 0.0 ? a.y[j] / nrm : a.x[j];
    const double df = vn - a.x[j];
    d2 += df * df;
    a.x[j] = vn;
  }
  double v[1] = {d2};
  block_sums<1>(v, red);
  if (threadIdx.x == 0) {
    FwState* st = a.st;
    st->pow_steps += 1;
    st->pow_delta = sqrt(v[0]);
    if (st->pow_delta <= kPowEps || !(nrm > 0.0) || st->pow_steps >= kPowMax) st->pow_active = 0;
  }
}

__global__ void k_fw_power_start(FwState* st) {
  st->pow_active = 1;
  st->pow_steps = 0;
}

__global__ void k_fw_fill(double* x, int n, double v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) x[j] = v;
}

__global__ void k_fw_init_state(FwState* st) {
  FwState z{};
  *st = z;
}

// ---------------------------------------------------------------------------------
// Precomputed per-row coarse tables of the mask (multilevel): A_ic = sum_j Q_ij P_jc^2,
// B_ic = sum_j Q_ij P_jc P_j,c+1, QDP_ic = sum_j Q_ij D_ij P_jc.  One thread per (i, c).
__global__ void __launch_bounds__(kFT) k_fw_mask_tables(int m, int n, int nH, int levels, const float* __restrict__ D,
                                                       int ldd, const uint32_t* __restrict__ bits, int nw,
                                                       const uint32_t* __restrict__ taps, const int* __restrict__ first,
                                                       float* __restrict__ Aq, float* __restrict__ Bq,
                                                       float* __restrict__ QDP, int ld) {
  const float scale = ldexpf(1.0f, -levels);
  const unsigned total = (unsigned)m * nH;
  for (unsigned t = blockIdx.x * kFT + threadIdx.x; t < total; t += gridDim.x * kFT) {
    const int i = (int)(t / (unsigned)nH), c = (int)(t - (unsigned)i * nH);
    const float* drow = D + (size_t)i * ldd;
    double A = 0.0, B = 0.0, QD = 0.0;
    for (int j = first[c]; j < first[c + 1]; ++j) {
      if (bits && !mask_bit(bits, nw, i, j)) continue;
      const double w0 = (double)((float)(taps[j] & 0xFFFFu) * scale);
      A += w0 * w0;
      B += w0 * (1.0 - w0);
      QD += w0 * (double)drow[j];
    }
    if (c > 0)
      for (int j = first[c - 1]; j < first[c]; ++j) {
        if (bits && !mask_bit(bits, nw, i, j)) continue;
        const double w1 = 1.0 - (double)((float)(taps[j] & 0xFFFFu) * scale);
        A += w1 * w1;
        QD += w1 * (double)drow[j];
      }
    Aq[(size_t)i * ld + c] = (float)A;
    Bq[(size_t)i * ld + c] = (float)B;
    QDP[(size_t)i * ld + c] = (float)QD;
  }
}

// Returned iterate: L (multilevel: Z P^T; plain: already in L) and S = P_Q S_{lam_S}[D - L]
// (zero before the first threshold step).
template <bool ML>
__global__ void __launch_bounds__(kFT) k_fw_output(int m, int n, int nH, int levels, const float* __restrict__ D,
                                                  int ldd, const uint32_t* __restrict__ bits, int nw,
                                                  const float* __restrict__ Z, int ldz,
                                                  const uint32_t* __restrict__ taps, float lamS, int thr,
                                                  float* __restrict__ L, int ldl, float* __restrict__ S, int lds) {
  const float scale = ldexpf(1.0f, -levels);
  const unsigned total = (unsigned)m * n;
  for (unsigned t = blockIdx.x * kFT + threadIdx.x; t < total; t += gridDim.x * kFT) {
    const int i = (int)(t / (unsigned)n), j = (int)(t - (unsigned)i * n);
    float l;
    if (ML) {
      int c;
      float w0;
      unpack_tap(taps[j], scale, c, w0);
      l = lift(Z + (size_t)i * ldz, c, w0, nH);
      L[(size_t)i * ldl + j] = l;
    } else {
      l = L[(size_t)i * ldl + j];
    }
    const bool q = bits ? mask_bit(bits, nw, i, j) : true;
    float sv, gv;
    if (thr)
      entry<true>(D[(size_t)i * ldd + j], l, q, lamS, sv, gv);
    else
      entry<false>(D[(size_t)i * ldd + j], l, q, lamS, sv, gv);
    S[(size_t)i * lds + j] = sv;
  }
}

__global__ void k_fw_pack_mask(int m, int n, const uint8_t* __restrict__ Q, int nw, uint32_t* __restrict__ bits) {
  const size_t total = (size_t)m * nw;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / nw;
    const int w = (int)(idx % nw);
    uint32_t v = 0;
    const int j0 = w * 32;
    const int jn = min(32, n - j0);
    for (int b = 0; b < jn; ++b) v |= (Q[i * n + j0 + b] != 0 ? 1u : 0u) << b;
    bits[idx] = v;
  }
}

// ---------------------------------------------------------------------------------
// host side
int cus() {
  int dev = 0, c = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) return 256;
  return c;
}

unsigned grid_of(size_t work, unsigned cap) {
  size_t b = (work + kFT - 1) / kFT;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

struct FwPlan {
  int m, n, nH, levels, nw, VEC, R, ldz;
  bool ml, masked;
  unsigned grid_pass, grid_terms;
  size_t lds_pass;
  // plain power iteration
  int gs, rpb, NS;
  unsigned grid_pow, grid_cols;
  size_t lds_pow;
  size_t off_bits, off_state, off_part, off_pmax, off_pidx, off_tpart, off_gz, off_taps, off_first;
  size_t off_Z, off_GP, off_Aq, off_Bq, off_QDP, off_gram, off_gws, off_V, off_lam, off_perm, off_sw, off_T, off_Tt,
      off_ist;
  size_t off_G, off_w, off_powp, off_y, off_ypart;
  size_t total;
};

int make_fw_plan(int m, int n, int levels, bool masked, bool vec_ok, FwPlan& p) {
  p = FwPlan{};
  p.m = m;
  p.n = n;
  p.levels = levels;
  p.ml = levels > 0;
  p.masked = masked;
  p.nH = coarse_dim_checked(n, levels);
  if (p.nH < 1) return MLPCP_E_LEVELS;
  p.nw = (n + 31) / 32;
  p.VEC = (vec_ok && n % 4 == 0) ? 4 : 1;
  const int C = cus();
  if (p.ml) {
    if (p.nH > kEigInner || levels > 15 || p.nH >= 65535) return MLPCP_E_UNSUPPORTED;
    const int nv = n / p.VEC;
    p.R = std::max(1, std::min(8, (2 * kFT) / std::max(1, nv)));
    p.ldz = kPad;   // Z, GP, tables share the Gram's padded width
    p.lds_pass = (size_t)n * 4 + (size_t)(p.nH + 1) * 4 + (size_t)p.nH * 4 + (size_t)p.R * p.nH * 4 +
                 (size_t)p.R * n * 4;
    if (p.lds_pass > 150 * 1024) return MLPCP_E_UNSUPPORTED;
    const int per_cu = std::max(1, std::min(8, (int)((160 * 1024) / (p.lds_pass + 2048))));
    const int nbatch = (m + p.R - 1) / p.R;
    p.grid_pass = (unsigned)std::max(1, std::min(nbatch, per_cu * C));
  } else {
    const size_t slots = (size_t)m * (n / p.VEC);
    p.grid_pass = grid_of(slots, 4u * C);
    // power iteration layout
    const int nv = n / p.VEC;
    p.gs = std::min(kFT, (nv + 63) / 64 * 64);
    const int per = (nv + p.gs - 1) / p.gs;
    p.NS = per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : per <= 8 ? 8 : 0;
    if (p.NS == 0) return MLPCP_E_UNSUPPORTED;
    p.lds_pow = (size_t)2 * n * 8;
    if (p.lds_pow > 150 * 1024) return MLPCP_E_UNSUPPORTED;
    const int Rg = kFT / p.gs;
    const int blocks = std::max(1, std::min(C, (m + Rg - 1) / Rg));
    p.rpb = (m + blocks - 1) / blocks;
    p.grid_pow = (unsigned)((m + p.rpb - 1) / p.rpb);
    p.grid_cols = (unsigned)((n + kFT - 1) / kFT);
  }
  p.grid_terms = (unsigned)std::max(1, std::min((m + 3) / 4, 4 * C));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 1));
    return o;
  };
  const unsigned nbp = std::max(p.grid_pass, 1u);
  p.off_bits = take(masked ? (size_t)m * p.nw * 4 : 0);
  p.off_state = take(sizeof(FwState));
  p.off_part = take((size_t)nbp * kNSums * 8);
  p.off_pmax = take((size_t)nbp * 4);
  p.off_pidx = take((size_t)nbp * 8);
  p.off_tpart = take((size_t)p.grid_terms * kNTerms * 8);
  p.off_gz = take((size_t)m * 8);
  if (p.ml) {
    p.off_taps = take((size_t)n * 4);
    p.off_first = take((size_t)(p.nH + 1) * 4);
    const size_t mat = (size_t)m * p.ldz * 4;
    p.off_Z = take(mat);
    p.off_GP = take(mat);
    p.off_Aq = take(mat);
    p.off_Bq = take(mat);
    p.off_QDP = take(mat);
    const size_t sq = (size_t)kEigInner * kEigInner * 8;
    p.off_gram = take(sq);
    p.off_gws = take(gram_workspace_bytes(m, kPad));
    p.off_V = take(sq);
    p.off_lam = take((size_t)kEigInner * 8);
    p.off_perm = take((size_t)kEigInner * 4);
    p.off_sw = take((size_t)kEigInner * 8);
    p.off_T = take(sq);
    p.off_Tt = take(sq);
    p.off_ist = take(sizeof(IterStats));
  } else {
    p.off_G = take((size_t)m * n * 4);
    p.off_w = take((size_t)n * 8);
    p.off_powp = take((size_t)p.grid_pow * n * 8);
    p.off_y = take((size_t)n * 8);
    p.off_ypart = take((size_t)p.grid_cols * 8);
  }
  p.total = off + 256;
  return MLPCP_OK;
}

struct FwWS {
  char* base = nullptr;
  void* owned = nullptr;
  ~FwWS() {
    if (owned) (void)hipFree(owned);
  }
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(base + off);
  }
};

template <bool MASKED, int VEC>
int launch_pass_ml(const FwPlan& p, const PassML& a, bool thr, hipStream_t s) {
  auto k = thr ? k_fw_pass_ml<MASKED, VEC, true> : k_fw_pass_ml<MASKED, VEC, false>;
  MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)p.lds_pass));
  hipLaunchKernelGGL(k, dim3(p.grid_pass), dim3(kFT), p.lds_pass, s, a);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

template <bool MASKED, int VEC>
int launch_pass_plain(const FwPlan& p, const PassPlain& a, bool thr, hipStream_t s) {
  if (thr)
    hipLaunchKernelGGL((k_fw_pass_plain<MASKED, VEC, true>), dim3(p.grid_pass), dim3(kFT), 0, s, a);
  else
    hipLaunchKernelGGL((k_fw_pass_plain<MASKED, VEC, false>), dim3(p.grid_pass), dim3(kFT), 0, s, a);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

template <int VEC>
int launch_power_step(const FwPlan& p, const PowArgs& a, hipStream_t s) {
  void (*k)(PowArgs) = nullptr;
  switch (p.NS) {
    case 1: k = k_fw_power<VEC, 1>; break;
    case 2: k = k_fw_power<VEC, 2>; break;
    case 4: k = k_fw_power<VEC, 4>; break;
    default: k = k_fw_power<VEC, 8>; break;
  }
  MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)p.lds_pow));
  hipLaunchKernelGGL(k, dim3(p.grid_pow), dim3(kFT), p.lds_pow, s, a);
  hipLaunchKernelGGL(k_fw_power_cols, dim3(p.grid_cols), dim3(kFT), 0, s, a, (int)p.grid_pow);
  hipLaunchKernelGGL(k_fw_power_fin, dim3(1), dim3(kFT), 0, s, a, (int)p.grid_cols);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int fwt_solve(int m, int n, const float* D, int ldd, const uint8_t* Q, float lamL, float lamS, int levels,
              double tol, int max_iter, float* L, float* S, void* ws, size_t ws_bytes, mlpcp_fwt_info* info,
              void* stream) {
  if (m < 1 || n < 1 || m < n || ldd < n) return MLPCP_E_SHAPE;
  if (!D || !L || !S || L == S || (const float*)L == D || (const float*)S == D) return MLPCP_E_INVALID_ARG;
  if (!(lamL > 0.0f) || !(lamS > 0.0f) || !std::isfinite(lamL) || !std::isfinite(lamS)) return MLPCP_E_INVALID_ARG;
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 1) return MLPCP_E_INVALID_ARG;
  if ((long long)m * n >= (1LL << 31)) return MLPCP_E_UNSUPPORTED;   // 32-bit flat indices
  if (coarse_dim_checked(n, levels) < 1) return MLPCP_E_LEVELS;
  const bool vec_ok = (reinterpret_cast<uintptr_t>(D) % 16 == 0) && (ldd % 4 == 0) &&
                      (reinterpret_cast<uintptr_t>(L) % 16 == 0);
  FwPlan p;
  MLPCP_TRY(make_fw_plan(m, n, levels, Q != nullptr, vec_ok, p));
  if (ws && ws_bytes < p.total) return MLPCP_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, levels, s, &op));
  FwWS w;
  if (ws) {
    w.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  } else {
    MLPCP_HIP(hipMalloc(&w.owned, p.total));
    w.base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(w.owned) + 255) & ~uintptr_t(255));
  }
  uint32_t* bits = p.masked ? w.at<uint32_t>(p.off_bits) : nullptr;
  FwState* st = w.at<FwState>(p.off_state);
  double* part = w.at<double>(p.off_part);
  float* pmax = w.at<float>(p.off_pmax);
  long long* pidx = w.at<long long>(p.off_pidx);
  double* tpart = w.at<double>(p.off_tpart);
  double* gz = w.at<double>(p.off_gz);
  hipLaunchKernelGGL(k_fw_init_state, dim3(1), dim3(1), 0, s, st);
  if (p.masked) {
    const size_t words = (size_t)m * p.nw;
    hipLaunchKernelGGL(k_fw_pack_mask, dim3(grid_of(words, 65536)), dim3(kFT), 0, s, m, n, Q, p.nw, bits);
  }
  MLPCP_HIP(hipMemsetAsync(gz, 0, (size_t)m * 8, s));

  // operator tables (multilevel)
  uint32_t* taps = nullptr;
  int* first = nullptr;
  std::vector<uint32_t> htaps;
  std::vector<int> hfirst;
  if (p.ml) {
    std::vector<int> ri, cp, cr;
    std::vector<float> rw, cw;
    build_stencil_host(n, levels, ri, rw, cp, cr, cw, nullptr);
    htaps.resize(n);
    hfirst.assign(p.nH + 1, n);
    const double den = std::ldexp(1.0, levels);
    int prev = -1;
    for (int j = 0; j < n; ++j) {
      int c0 = ri[(size_t)j * kMaxStencil];
      double w0 = rw[(size_t)j * kMaxStencil];
      const double w1 = rw[(size_t)j * kMaxStencil + 1];
      const int c1 = ri[(size_t)j * kMaxStencil + 1];
      if (w1 != 0.0 && c1 != c0 + 1) return MLPCP_E_UNSUPPORTED;     // taps are adjacent pairs
      if (std::fabs(w0 + w1 - 1.0) > 1e-12) return MLPCP_E_UNSUPPORTED;
      if (c0 < prev) return MLPCP_E_UNSUPPORTED;                      // first taps non-decreasing
      const double num = w0 * den;
      if (num != std::floor(num) || num < 0 || num > 65535.0) return MLPCP_E_UNSUPPORTED;
      htaps[j] = ((uint32_t)c0 << 16) | (uint32_t)num;
      prev = c0;
    }
    for (int c = 0; c <= p.nH; ++c) {
      int j = 0;
      while (j < n && (int)(htaps[j] >> 16) < c) ++j;
      hfirst[c] = j;
    }
    taps = w.at<uint32_t>(p.off_taps);
    first = w.at<int>(p.off_first);
    MLPCP_HIP(hipMemcpyAsync(taps, htaps.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    MLPCP_HIP(hipMemcpyAsync(first, hfirst.data(), (size_t)(p.nH + 1) * 4, hipMemcpyHostToDevice, s));
    const size_t mat = (size_t)m * p.ldz * 4;
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_Z), 0, mat, s));
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_GP), 0, mat, s));
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_T), 0, (size_t)kEigInner * kEigInner * 8, s));
    hipLaunchKernelGGL(k_fw_mask_tables, dim3(grid_of((size_t)m * p.nH, 8192)), dim3(kFT), 0, s, m, n, p.nH, levels,
                       D, ldd, bits, p.nw, taps, first, w.at<float>(p.off_Aq), w.at<float>(p.off_Bq),
                       w.at<float>(p.off_QDP), p.ldz);
    MLPCP_HIP(hipGetLastError());
  } else {
    hipLaunchKernelGGL(k_fw_fill, dim3((n + 255) / 256), dim3(256), 0, s, w.at<double>(p.off_w), n,
                       1.0 / std::sqrt((double)n));
    MLPCP_HIP(hipGetLastError());
  }

  PassML pm{};
  PassPlain pp{};
  if (p.ml) {
    pm.m = m; pm.n = n; pm.nH = p.nH; pm.R = p.R; pm.nw = p.nw; pm.levels = levels;
    pm.D = D; pm.ldd = ldd; pm.bits = bits;
    pm.Z = w.at<float>(p.off_Z); pm.ldz = p.ldz;
    pm.GP = w.at<float>(p.off_GP); pm.ldg = p.ldz;
    pm.taps = taps; pm.first = first;
    pm.T = w.at<double>(p.off_T); pm.ldT = kEigInner;
    pm.gz = gz; pm.st = st; pm.lamS = lamS;
    pm.partial = part; pm.pmax = pmax; pm.pidx = pidx;
  } else {
    pp.m = m; pp.n = n; pp.nw = p.nw; pp.D = D; pp.ldd = ldd; pp.bits = bits;
    pp.L = L; pp.G = w.at<float>(p.off_G); pp.w = w.at<double>(p.off_w); pp.gz = gz; pp.st = st;
    pp.lamS = lamS; pp.partial = part; pp.pmax = pmax; pp.pidx = pidx;
  }
  auto pass = [&](bool thr) -> int {
    ProfScope ps(KC_FW_PASS, s);
    if (p.ml) {
      if (p.masked)
        return p.VEC == 4 ? launch_pass_ml<true, 4>(p, pm, thr, s) : launch_pass_ml<true, 1>(p, pm, thr, s);
      return p.VEC == 4 ? launch_pass_ml<false, 4>(p, pm, thr, s) : launch_pass_ml<false, 1>(p, pm, thr, s);
    }
    if (p.masked)
      return p.VEC == 4 ? launch_pass_plain<true, 4>(p, pp, thr, s) : launch_pass_plain<true, 1>(p, pp, thr, s);
    return p.VEC == 4 ? launch_pass_plain<false, 4>(p, pp, thr, s) : launch_pass_plain<false, 1>(p, pp, thr, s);
  };
  auto finalize = [&](bool thr) -> int {
    ProfScope ps(KC_FW_SMALL, s);
    hipLaunchKernelGGL(k_fw_finalize, dim3(1), dim3(64), 0, s, part, pmax, pidx, (int)p.grid_pass, (double)lamL,
                       (double)lamS, thr ? 1 : 0, st);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  };

  // iterate 0: L = S = 0
  MLPCP_TRY(pass(false));
  MLPCP_TRY(finalize(false));
  FwState hs;
  MLPCP_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  prof_drain();
  double f_prev = hs.f;
  int k = 0;
  bool converged = false, thr = false;
  int status = MLPCP_OK;
  long long pow_total = 0;
  int pow_batch = 4;
  double rel = 0.0;
  if (!(hs.f > 0.0)) converged = hs.f == 0.0;
  if (!std::isfinite(hs.f)) status = MLPCP_E_NONFINITE;
  bool warm = false;
  while (!converged && status == MLPCP_OK && k < max_iter) {
    // the nuclear direction
    if (p.ml) {
      {
        ProfScope ps(KC_GRAM, s);
        MLPCP_TRY(gram_f64(m, p.nH, kPad, w.at<float>(p.off_GP), p.ldz, w.at<double>(p.off_gram),
                           w.at<void>(p.off_gws), s, 0));
      }
      // top eigenpair of C (GP^T GP) C: the one-workgroup Jacobi; with a vanishing
      // threshold the first column of T = C V_sorted diag(1) is z = C v_top
      MLPCP_TRY(coarse_svt_small(p.nH, kEigInner, w.at<double>(p.off_gram), op->C, w.at<double>(p.off_V), warm,
                                 1e-300, w.at<double>(p.off_lam), w.at<int>(p.off_perm), w.at<double>(p.off_sw),
                                 w.at<double>(p.off_T), w.at<double>(p.off_Tt), nullptr,
                                 w.at<IterStats>(p.off_ist), s));
      warm = true;
      TermsML ta{};
      ta.m = m; ta.nH = p.nH; ta.Z = w.at<float>(p.off_Z); ta.GP = w.at<float>(p.off_GP);
      ta.Aq = w.at<float>(p.off_Aq); ta.Bq = w.at<float>(p.off_Bq); ta.QDP = w.at<float>(p.off_QDP);
      ta.ld = p.ldz; ta.T = w.at<double>(p.off_T); ta.ldT = kEigInner; ta.gz = gz; ta.partial = tpart;
      ProfScope ps(KC_FW_SMALL, s);
      hipLaunchKernelGGL(k_fw_terms_ml, dim3(p.grid_terms), dim3(kFT), (size_t)p.nH * 8, s, ta);
      MLPCP_HIP(hipGetLastError());
    } else {
      PowArgs pa{};
      pa.m = m; pa.n = n; pa.gs = p.gs; pa.rpb = p.rpb; pa.G = w.at<float>(p.off_G); pa.x = w.at<double>(p.off_w);
      pa.partial = w.at<double>(p.off_powp); pa.y = w.at<double>(p.off_y); pa.ypart = w.at<double>(p.off_ypart);
      pa.st = st;
      hipLaunchKernelGGL(k_fw_power_start, dim3(1), dim3(1), 0, s, st);
      int done_steps = 0;
      for (;;) {
        {
          ProfScope ps(KC_FW_POWER, s);
          for (int b = 0; b < pow_batch; ++b)
            MLPCP_TRY(p.VEC == 4 ? launch_power_step<4>(p, pa, s) : launch_power_step<1>(p, pa, s));
        }
        MLPCP_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        MLPCP_HIP(hipStreamSynchronize(s));
        prof_drain();
        done_steps = hs.pow_steps;
        if (!hs.pow_active) break;
      }
      pow_total += done_steps;
      pow_batch = std::max(1, std::min(64, done_steps));
      TermsPlain ta{};
      ta.m = m; ta.n = n; ta.nw = p.nw; ta.D = D; ta.ldd = ldd; ta.bits = bits; ta.L = L;
      ta.w = w.at<double>(p.off_w); ta.lamS = lamS; ta.thr = thr; ta.gz = gz; ta.partial = tpart;
      ProfScope ps(KC_FW_SMALL, s);
      const size_t lds = (size_t)n * 8;
      if (lds > 64 * 1024) {
        auto kk = p.masked ? (thr ? k_fw_terms_plain<true, true> : k_fw_terms_plain<true, false>)
                           : (thr ? k_fw_terms_plain<false, true> : k_fw_terms_plain<false, false>);
        MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kk), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
      }
      if (p.masked) {
        if (thr)
          hipLaunchKernelGGL((k_fw_terms_plain<true, true>), dim3(p.grid_terms), dim3(kFT), lds, s, ta);
        else
          hipLaunchKernelGGL((k_fw_terms_plain<true, false>), dim3(p.grid_terms), dim3(kFT), lds, s, ta);
      } else {
        if (thr)
          hipLaunchKernelGGL((k_fw_terms_plain<false, true>), dim3(p.grid_terms), dim3(kFT), lds, s, ta);
        else
          hipLaunchKernelGGL((k_fw_terms_plain<false, false>), dim3(p.grid_terms), dim3(kFT), lds, s, ta);
      }
      MLPCP_HIP(hipGetLastError());
    }
    {
      SolveArgs sa{};
      sa.m = m; sa.n = n; sa.nH = p.nH; sa.levels = levels; sa.partial = tpart; sa.nb = (int)p.grid_terms;
      sa.D = D; sa.ldd = ldd; sa.L = L; sa.Z = p.ml ? w.at<float>(p.off_Z) : nullptr; sa.ldz = p.ldz;
      sa.taps = taps;
      sa.T = p.ml ? w.at<double>(p.off_T) : nullptr; sa.ldT = kEigInner;
      sa.w = p.ml ? nullptr : w.at<double>(p.off_w); sa.gz = gz; sa.lamL = lamL; sa.lamS = lamS; sa.st = st;
      ProfScope ps(KC_FW_SMALL, s);
      hipLaunchKernelGGL(k_fw_solve, dim3(1), dim3(64), 0, s, sa);
      MLPCP_HIP(hipGetLastError());
    }
    MLPCP_TRY(pass(true));
    MLPCP_TRY(finalize(true));
    thr = true;
    MLPCP_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipStreamSynchronize(s));
    prof_drain();
    ++k;
    rel = f_prev > 0.0 ? std::fabs(f_prev - hs.f) / f_prev : 0.0;
    if (info && k <= info->history_len) {
      const int h = k - 1;
      if (info->f_history) info->f_history[h] = hs.f;
      if (info->alpha_history) info->alpha_history[h] = hs.alpha;
      if (info->beta_history) info->beta_history[h] = hs.beta;
      if (info->sigma_history) info->sigma_history[h] = hs.sigma;
    }
    if (!std::isfinite(hs.f)) {
      status = MLPCP_E_NONFINITE;
      break;
    }
    f_prev = hs.f;
    if (rel <= tol) converged = true;
  }
  if (status == MLPCP_OK) {
    ProfScope ps(KC_FINAL, s);
    const unsigned g = grid_of((size_t)m * n, 8192);
    if (p.ml)
      hipLaunchKernelGGL(k_fw_output<true>, dim3(g), dim3(kFT), 0, s, m, n, p.nH, levels, D, ldd, bits, p.nw,
                         w.at<float>(p.off_Z), p.ldz, taps, lamS, thr ? 1 : 0, L, n, S, n);
    else
      hipLaunchKernelGGL(k_fw_output<false>, dim3(g), dim3(kFT), 0, s, m, n, p.nH, levels, D, ldd, bits, p.nw,
                         nullptr, 0, nullptr, lamS, thr ? 1 : 0, L, n, S, n);
    MLPCP_HIP(hipGetLastError());
    MLPCP_HIP(hipStreamSynchronize(s));
    prof_drain();
    if (!converged) status = MLPCP_NOT_CONVERGED;
  }
  if (info) {
    info->iters = k;
    info->f = hs.f;
    info->t_L = hs.t_L;
    info->t_S = hs.t_S;
    info->rel_change = rel;
    info->gap = hs.gap;
    info->power_steps = pow_total;
    info->converged = converged ? 1 : 0;
  }
  return status;
}

}  // namespace
}  // namespace mlpcp

using namespace mlpcp;

extern "C" {

size_t mlpcp_fwt_workspace_bytes(int m, int n, int levels, int masked) {
  if (m < 1 || n < 1 || m < n || coarse_dim_checked(n, levels) < 1) return 0;
  // the larger of the vector and scalar layouts (the call picks one from its pointers)
  size_t best = 0;
  for (int v = 0; v < 2; ++v) {
    FwPlan p;
    if (make_fw_plan(m, n, levels, masked != 0, v == 0, p) == MLPCP_OK) best = std::max(best, p.total);
  }
  return best ? best + 256 : 0;
}

int mlpcp_cpcp_fwt(int m, int n, const float* D, int ldd, const uint8_t* Q, float lam_L, float lam_S, int levels,
                   double tol, int max_iter, float* L, float* S, void* ws, size_t ws_bytes, mlpcp_fwt_info* info,
                   void* stream) {
  return fwt_solve(m, n, D, ldd, Q, lam_L, lam_S, levels, tol, max_iter, L, S, ws, ws_bytes, info, stream);
}

}  // extern "C"
