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
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"
#include "profile.h"

namespace mlpcp {
namespace {

constexpr int kFT = 256;          // threads per block of the streaming kernels
constexpr int kNSums = 8;         // E2, ES, T5..T9, (pad) per block
constexpr int kNTerms = 7;        // S1..S4, and (multilevel) T5..T7 per block
constexpr int kPowMax = 500;      // power-iteration steps per FW iteration (cap)
constexpr double kPowEps = 1e-6;  // ||v_new - v_old|| that ends the power iteration

// Device state of one solve, read by the kernels and brought to the host once per
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

// The state as the host reads it, with the sequence number of the request written last.
struct FwRecord {
  FwState st;
  unsigned long long seq;
};

// Copies the state to pinned, host-mapped memory, then, behind a system-scope fence, the
// sequence number: the host reads the state as soon as it sees the number, without a copy
// or a stream synchronisation.
__global__ void k_fw_publish(const FwState* __restrict__ st, FwRecord* rec, unsigned long long seq) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    rec->st = *st;
    __threadfence_system();
    *reinterpret_cast<volatile unsigned long long*>(&rec->seq) = seq;
  }
}

// One pinned, host-mapped record per host thread (allocated on the thread's first solve,
// kept until the process ends; a solve runs to completion on its calling thread, so the
// record is never shared).  Null when the allocation fails: the state then comes back by
// a copy and a stream synchronisation.
struct FwSlot {
  FwRecord* host = nullptr;   // host address
  FwRecord* dev = nullptr;    // the same memory as the device addresses it
  unsigned long long next = 0;
};

FwSlot* fw_slot() {
  thread_local FwSlot slot;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, sizeof(FwRecord), hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable) ==
        hipSuccess) {
      static_cast<FwRecord*>(h)->seq = 0;
      if (hipHostGetDevicePointer(&d, h, 0) == hipSuccess) {
        slot.host = static_cast<FwRecord*>(h);
        slot.dev = static_cast<FwRecord*>(d);
      }
    }
    (void)hipGetLastError();
  }
  return slot.host ? &slot : nullptr;
}

// The device state st (after the work queued on s) into hs: published when a slot is
// there, else copied.
int read_state(FwSlot* sl, const FwState* st, FwState* hs, hipStream_t s) {
  if (sl) {
    const unsigned long long want = ++sl->next;
    hipLaunchKernelGGL(k_fw_publish, dim3(1), dim3(64), 0, s, st, sl->dev, want);
    MLPCP_HIP(hipGetLastError());
    MLPCP_TRY(wait_seq(&sl->host->seq, want, s));
    std::memcpy(hs, const_cast<const FwState*>(&sl->host->st), sizeof(FwState));
    return MLPCP_OK;
  }
  MLPCP_HIP(hipMemcpyAsync(hs, st, sizeof(FwState), hipMemcpyDeviceToHost, s));
  MLPCP_HIP(hipStreamSynchronize(s));
  return MLPCP_OK;
}

__device__ __forceinline__ float shrinkf(float x, float t) {
  const float a = fabsf(x) - t;
  return a > 0.0f ? copysignf(a, x) : 0.0f;
}
__device__ __forceinline__ float clampf(float x, float t) { return __builtin_amdgcn_fmed3f(x, -t, t); }

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

// sums of one short run of entries in float32 (a chunk of at most a few dozen
// entries), folded into the float64 Sums once per run: sum G^2, sum |S|, sum S^2 and,
// when ARGMAX, the first entry of largest |G| (by column).  The multilevel path gets
// the sums involving L from coarse quantities and sum G S = -lam_S sum |S| (G =
// -lam_S sign(S) wherever S != 0).
template <bool ARGMAX>
struct RunSums {
  float E2 = 0, ES = 0, T8 = 0;
  float best = -1.0f;
  int bj = 0;
  __device__ __forceinline__ void add(float s, float g, int j) {
    E2 = fmaf(g, g, E2);
    ES += fabsf(s);
    T8 = fmaf(s, s, T8);
    if (ARGMAX) {
      const float a = fabsf(g);
      if (a > best) {          // runs are visited in increasing j: the first maximum stays
        best = a;
        bj = j;
      }
    }
  }
  __device__ __forceinline__ void fold(Sums& sm, long long row_base) const {
    sm.E2 += E2;
    sm.ES += ES;
    sm.T8 += T8;
    if (ARGMAX) {
      const long long idx = row_base + bj;
      if (best > sm.best || (best == sm.best && best >= 0.0f && idx < sm.bidx)) {
        sm.best = best;
        sm.bidx = idx;
      }
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
// Multilevel pass.  A block takes R rows at a time.  All threads stage the rows of D
// and of the mask bits in LDS with coalesced loads (the next batch is fetched into
// registers while the current one is processed).  Each row's fine columns are cut into
// K contiguous chunks that lie inside one interval [first_c, first_{c+1}) of fine
// columns whose first stencil tap is the coarse column c, so a chunk only needs Z_c and
// Z_{c+1}; one (row, chunk) task per thread computes the entries (S, G) from LDS, the
// sums and the argmax, and the chunk's two partial restriction sums (sum w0 G for c,
// sum (1 - w0) G for c + 1), which are added per coarse column in chunk order: GP = G P.
// The new coarse rows (1 - alpha) Z - alpha U_L u_i z^T are formed at staging time.
constexpr int kChunkMin = 16;      // shortest chunk (unless its interval is shorter)

// a run of fine columns j0 <= j < j1 whose first tap is c; when `affine`, the first-tap
// weight is w0(j) = fmaf(ws, j - j0, wb) exactly (checked on the host), else the table
struct Chunk {
  int c, j0, j1, affine;
  float wb, ws, pad0, pad1;
};

__device__ __forceinline__ float chunk_w0(const Chunk& ch, int j, const float* __restrict__ w0tab) {
  return ch.affine ? fmaf(ch.ws, (float)(j - ch.j0), ch.wb) : w0tab[j];
}

struct PassML {
  int m, n, nH, R, K, nw, levels, maxlen;   // maxlen: the longest chunk
  const float* D;
  int ldd;
  const uint32_t* bits;
  const float* Zin;
  float* Zout;
  int ldz;
  float* GP;
  int ldg;
  const float* w0;        // [n] weight of the first tap of each fine column
  const Chunk* chunks;    // [K]
  const int* kfirst;      // [nH + 1]: first chunk of interval c
  const uint32_t* taps;   // [n] packed (output and step kernels)
  const double* T;        // direction z = T[c * ldT]
  int ldT;
  const double* gz;       // [m]: G w of the previous iterate (u = gz / sigma)
  const FwState* st;
  float lamS;
  double* partial;
  float* pmax;
  long long* pidx;
};

__device__ __forceinline__ float lift2(float z0, float z1, float w0, bool has_next) {
  const float a = w0 * z0;
  return (w0 < 1.0f && has_next) ? fmaf(1.0f - w0, z1, a) : a;
}

// LDS layout of the multilevel kernels (bytes), shared by the host sizing: partial
// sums (nsums per task, float or double), the coarse rows, the interval -> first chunk
// table, the staged rows of D and of the mask words
struct MlLds {
  size_t tz, sp, z, kf, d, q, total;
};
__host__ __device__ inline MlLds ml_lds(int n, int nH, int R, int K, int nw, int nsums, int bytes) {
  MlLds L{};
  size_t o = 0;
  L.tz = o;  o += (size_t)nH * 8;
  L.sp = o;  o += (size_t)nsums * R * K * bytes;
  L.z = o;   o += (size_t)R * nH * 4;
  L.kf = o;  o += (size_t)(nH + 1) * 4;
  o = (o + 15) & ~size_t(15);
  L.d = o;   o += (size_t)R * n * 4;
  L.q = o;   o += (size_t)R * nw * 4;
  L.total = o;
  return L;
}

// stage rows i0 .. i0+rows-1 of D and of the mask words: each thread holds 4 PF floats
// (PF float4 slots when VEC == 4, single floats otherwise)
template <int VEC, int PF, bool MASKED>
__device__ __forceinline__ void stage_load(const PassML& a, int i0, int rows, float (&rd)[4 * PF], uint32_t& rq) {
  const int nv = a.n / VEC;
#pragma unroll
  for (int k = 0; k < 4 * PF / VEC; ++k) {
    const int f = threadIdx.x + kFT * k;
    if (f < rows * nv) {
      const int r = f / nv, s = f - r * nv;
      const float* src = a.D + (size_t)(i0 + r) * a.ldd + (size_t)s * VEC;
      if constexpr (VEC == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        rd[4 * k] = v.x;
        rd[4 * k + 1] = v.y;
        rd[4 * k + 2] = v.z;
        rd[4 * k + 3] = v.w;
      } else {
        rd[k] = *src;
      }
    }
  }
  if (MASKED && (int)threadIdx.x < rows * a.nw) {
    const int r = threadIdx.x / a.nw, w = threadIdx.x - r * a.nw;
    rq = a.bits[(size_t)(i0 + r) * a.nw + w];
  }
}

template <int VEC, int PF, bool MASKED>
__device__ __forceinline__ void stage_store(const PassML& a, int rows, const float (&rd)[4 * PF], uint32_t rq,
                                            float* sD, uint32_t* sQ) {
  const int nv = a.n / VEC;
#pragma unroll
  for (int k = 0; k < 4 * PF / VEC; ++k) {
    const int f = threadIdx.x + kFT * k;
    if (f < rows * nv) {
      const int r = f / nv, s = f - r * nv;
      float* dst = sD + (size_t)r * a.n + (size_t)s * VEC;
      if constexpr (VEC == 4) *reinterpret_cast<float4*>(dst) = make_float4(rd[4 * k], rd[4 * k + 1], rd[4 * k + 2], rd[4 * k + 3]);
      else *dst = rd[k];
    }
  }
  if (MASKED && (int)threadIdx.x < rows * a.nw) sQ[threadIdx.x] = rq;
}

template <bool MASKED, int VEC, int PF, bool THR>
__global__ void __launch_bounds__(kFT) k_fw_pass_ml(PassML a) {
  extern __shared__ __align__(16) char smem_raw[];
  const MlLds lay = ml_lds(a.n, a.nH, a.R, a.K, a.nw, 2, 4);
  float* sp0 = reinterpret_cast<float*>(smem_raw + lay.sp);                // [R][K]
  float* sp1 = sp0 + (size_t)a.R * a.K;                                    // [R][K]
  float* sZ = reinterpret_cast<float*>(smem_raw + lay.z);                  // [R][nH]
  int* sKf = reinterpret_cast<int*>(smem_raw + lay.kf);                    // [nH + 1]
  float* sD = reinterpret_cast<float*>(smem_raw + lay.d);                  // [R][n]
  uint32_t* sQ = reinterpret_cast<uint32_t*>(smem_raw + lay.q);            // [R][nw]
  __shared__ double red[8 * (kFT / 64)];
  __shared__ float rv[kFT / 64];
  __shared__ long long ri[kFT / 64];
  const int tid = threadIdx.x;
  for (int c = tid; c <= a.nH; c += kFT) sKf[c] = a.kfirst[c];
  const double alpha = THR ? a.st->alpha : 0.0;
  const double coefL = THR ? a.st->coefL : 0.0;   // alpha U_L / sigma if the atom is taken
  // this thread's (row, chunk) task, the same for every batch
  const int tr = tid / a.K, tk = tid - tr * a.K;
  Chunk ch{};
  if (tr < a.R) ch = a.chunks[tk];
  const bool has_next = ch.c + 1 < a.nH;
  // the coarse direction z, once per block
  double* sTz = reinterpret_cast<double*>(smem_raw + lay.tz);             // [nH]
  for (int c = tid; c < a.nH; c += kFT) sTz[c] = THR ? a.T[(size_t)c * a.ldT] : 0.0;
  Sums sm;
  const int nbatch = (a.m + a.R - 1) / a.R;
  float rd[4 * PF];
  uint32_t rq = 0xFFFFFFFFu;
  // the coarse rows of the next batch (up to two entries per thread) and their gz
  float zq[2] = {0.0f, 0.0f};
  double gq[2] = {0.0, 0.0};
  auto coarse_load = [&](int i0n, int rows_n) {
    if (!THR) return;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = tid + kFT * u;
      if (t < rows_n * a.nH) {
        const int r = t / a.nH, c = t - r * a.nH;
        zq[u] = a.Zin[(size_t)(i0n + r) * a.ldz + c];
        gq[u] = a.gz[i0n + r];
      }
    }
  };
  int b = blockIdx.x;
  if (b < nbatch) {
    stage_load<VEC, PF, MASKED>(a, b * a.R, min(a.R, a.m - b * a.R), rd, rq);
    coarse_load(b * a.R, min(a.R, a.m - b * a.R));
  }
  __syncthreads();
  for (; b < nbatch; b += gridDim.x) {
    const int i0 = b * a.R;
    const int rows = min(a.R, a.m - i0);
    stage_store<VEC, PF, MASKED>(a, rows, rd, rq, sD, sQ);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = tid + kFT * u;
      if (t < rows * a.nH) {
        const int r = t / a.nH, c = t - r * a.nH;
        float zv = 0.0f;
        if (THR) {
          zv = (float)((1.0 - alpha) * (double)zq[u] - coefL * gq[u] * sTz[c]);
          a.Zout[(size_t)(i0 + r) * a.ldz + c] = zv;
        }
        sZ[r * a.nH + c] = zv;
      }
    }
    __syncthreads();
    const int bn = b + gridDim.x;
    if (bn < nbatch) {
      stage_load<VEC, PF, MASKED>(a, bn * a.R, min(a.R, a.m - bn * a.R), rd, rq);
      coarse_load(bn * a.R, min(a.R, a.m - bn * a.R));
    }
    if (tr < rows) {
      const int i = i0 + tr;
      const float z0 = sZ[tr * a.nH + ch.c];
      const float z1 = has_next ? sZ[tr * a.nH + ch.c + 1] : 0.0f;
      const float* drow = sD + (size_t)tr * a.n;
      const uint32_t* qrow = sQ + (size_t)tr * a.nw;
      const int len = ch.j1 - ch.j0;
      // within the chunk w0(t) = wb + ws t, so L(t) = l0 + t dl is affine too, and
      // sum w0 G = wb sum G + ws sum t G
      const float dz = z0 - z1;
      const float l0 = fmaf(ch.wb, dz, z1), dl = ch.ws * dz;
      // the chunk's mask bits (chunks are at most 32 long): bit t = entry j0 + t
      uint32_t qb = 0xFFFFFFFFu;
      if (MASKED) {
        const int w = ch.j0 >> 5;
        const uint32_t lo = qrow[w], hi = w + 1 < a.nw ? qrow[w + 1] : 0u;
        qb = (uint32_t)((((uint64_t)hi << 32) | lo) >> (ch.j0 & 31));
      }
      if (len < 32) qb &= (1u << len) - 1u;
      float ps = 0.0f, ptg = 0.0f;
      RunSums<!THR> rs;     // after the first step |G| <= lam_S: the l1 gate is closed
      // a uniform trip count (the longest chunk), predicated in groups of four
      for (int t0 = 0; t0 < a.maxlen; t0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = t0 + u;
          const float tf = (float)t;
          const bool q = (qb >> t) & 1u;                       // 0 past the chunk's end
          const int j = ch.j0 + min(t, len - 1);               // a column of the chunk
          const float d = drow[j];
          const float l = fmaf(tf, dl, l0);
          float sv, gv;
          entry<THR>(d, l, q, a.lamS, sv, gv);
          rs.add(sv, gv, j);
          ps += gv;
          ptg = fmaf(tf, gv, ptg);
        }
      }
      const float p0 = fmaf(ch.wb, ps, ch.ws * ptg);
      rs.fold(sm, (long long)i * a.n);
      sp0[tr * a.K + tk] = p0;
      sp1[tr * a.K + tk] = ps - p0;
    }
    __syncthreads();
    for (int t = tid; t < rows * a.nH; t += kFT) {
      const int r = t / a.nH, c = t - r * a.nH;
      double acc = 0.0;
      for (int k = sKf[c]; k < sKf[c + 1]; ++k) acc += sp0[r * a.K + k];
      if (c > 0)
        for (int k = sKf[c - 1]; k < sKf[c]; ++k) acc += sp1[r * a.K + k];
      a.GP[(size_t)(i0 + r) * a.ldg + c] = (float)acc;
    }
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
__global__ void __launch_bounds__(kFT) k_fw_finalize(const double* __restrict__ partial,
                                                     const float* __restrict__ pmax,
                                                     const long long* __restrict__ pidx, int nb, double lamL,
                                                     double lamS, int thr, FwState* st) {
  __shared__ double red[8 * (kFT / 64)];
  __shared__ float rv[kFT / 64];
  __shared__ long long ri[kFT / 64];
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  float best = -1.0f;
  long long bi = 0;
  for (int b = threadIdx.x; b < nb; b += kFT) {
    for (int k = 0; k < 7; ++k) v[k] += partial[(size_t)b * kNSums + k];
    if (pmax[b] > best || (pmax[b] == best && pidx[b] < bi)) {
      best = pmax[b];
      bi = pidx[b];
    }
  }
  block_sums<7>(v, red);
  block_argmax(best, bi, rv, ri);
  if (threadIdx.x == 0) {
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
  const double* T;        // direction z = T[c * ldT]
  int ldT;
  double* gz;
  double* partial;
};

__global__ void __launch_bounds__(kFT) k_fw_terms_ml(TermsML a) {
  extern __shared__ double sz[];   // [nH]
  __shared__ double red[7 * (kFT / 64)];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < a.nH; c += kFT) sz[c] = a.T[(size_t)c * a.ldT];
  __syncthreads();
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = blockIdx.x * (kFT / 64) + wid; i < a.m; i += gridDim.x * (kFT / 64)) {
    const size_t o = (size_t)i * a.ld;
    double g = 0, l = 0, d = 0, q = 0, t5 = 0, t6 = 0, zd = 0;
    for (int c = lane; c < a.nH; c += 64) {
      const double zc = sz[c];
      const double A = a.Aq[o + c], B = a.Bq[o + c];
      const double zn = c + 1 < a.nH ? sz[c + 1] : 0.0;
      const double Zc = a.Z[o + c];
      const double Zn = c + 1 < a.nH ? (double)a.Z[o + c + 1] : 0.0;
      const double Zp = c > 0 ? (double)a.Z[o + c - 1] : 0.0;
      const double Bp = c > 0 ? (double)a.Bq[o + c - 1] : 0.0;
      const double GPc = a.GP[o + c], QDc = a.QDP[o + c];
      g += zc * GPc;
      d += zc * QDc;
      l += zc * (A * Zc + B * Zn + Bp * Zp);
      q += A * zc * zc + 2.0 * B * zc * zn;
      // the iterate's own sums, L = Z P^T: sum_Q L^2, sum G L, sum Z (Q o D) P
      t5 += A * Zc * Zc + 2.0 * B * Zc * Zn;
      t6 += Zc * GPc;
      zd += Zc * QDc;
    }
    g = wave_sum(g);
    l = wave_sum(l);
    d = wave_sum(d);
    q = wave_sum(q);
    t5 = wave_sum(t5);
    t6 = wave_sum(t6);
    zd = wave_sum(zd);
    if (lane == 0) {
      a.gz[i] = g;
      acc[0] += g * g;
      acc[1] += g * g * q;
      acc[2] += g * l;
      acc[3] += g * d;
      acc[4] += t5;
      acc[5] += t6;
      acc[6] += t6 - t5 + zd;     // sum_Q L S: (Q o S) P = GP - (Q o L) P + (Q o D) P
    }
  }
  block_sums<7>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) a.partial[(size_t)blockIdx.x * kNTerms + k] = acc[k];
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
    for (int k = 0; k < kNTerms; ++k) a.partial[(size_t)blockIdx.x * kNTerms + k] = k < 4 ? acc[k] : 0.0;
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
  const double* T;        // ML direction z = T[c * ldT]
  int ldT;
  const double* w;        // plain direction
  const double* gz;
  double lamL, lamS;
  FwState* st;
};

__global__ void __launch_bounds__(kFT) k_fw_solve(SolveArgs a) {
  __shared__ double red[kNTerms * (kFT / 64)];
  double v[kNTerms] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < a.nb; b += kFT)
    for (int k = 0; k < kNTerms; ++k) v[k] += a.partial[(size_t)b * kNTerms + k];
  block_sums<kNTerms>(v, red);
  if (threadIdx.x != 0) return;
  FwState* st = a.st;
  if (a.levels > 0) {
    // the multilevel pass leaves the sums that involve L to the coarse terms
    st->T5 = v[4];
    st->T6 = v[5];
    st->T7 = v[6];
    st->T9 = -a.lamS * st->t_S;
  }
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
// gradient, warm-started from the previous direction.  Each step: t = G x (one wave per
// row), partial sums of G^T t over kPowRanges row ranges (fixed order), the column
// reduction over the ranges, then the
// normalisation and the convergence test.  Every kernel returns at once when the
// iteration has converged (device-gated steps, queued in batches by the host).
constexpr int kPowRanges = 32;   // row ranges of the G^T t partial sums

struct PowArgs {
  int m, n, nchunk;       // row ranges of the G^T t partial sums
  const float* G;
  double* x;              // [n] current direction (unit)
  double* t;              // [m] G x
  double* partial;        // [nchunk][n]
  double* y;              // [n]
  double* ypart;          // [ncolblocks]
  FwState* st;
};

template <int VEC>
__global__ void __launch_bounds__(kFT) k_fw_gx(PowArgs a) {
  if (!a.st->pow_active) return;
  extern __shared__ double sx[];   // [n]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < a.n; j += kFT) sx[j] = a.x[j];
  __syncthreads();
  const int nv = a.n / VEC;
  for (int i = blockIdx.x * (kFT / 64) + wid; i < a.m; i += gridDim.x * (kFT / 64)) {
    const float* g = a.G + (size_t)i * a.n;
    double d = 0.0;
    for (int s = lane; s < nv; s += 64) {
      if constexpr (VEC == 4) {
        const float4 v = *reinterpret_cast<const float4*>(g + s * 4);
        d += (double)v.x * sx[s * 4] + (double)v.y * sx[s * 4 + 1] + (double)v.z * sx[s * 4 + 2] +
             (double)v.w * sx[s * 4 + 3];
      } else {
        d += (double)g[s] * sx[s];
      }
    }
    d = wave_sum(d);
    if (lane == 0) a.t[i] = d;
  }
}

// partial[rc][j] = sum over the rows of range rc of t_i G_ij: a block covers 64 columns
// of one row range; 16 row groups of 16 threads walk the rows (each thread 4 columns),
// then the 16 group sums are added in a fixed order
constexpr int kGtyCols = 64;

template <int VEC>
__global__ void __launch_bounds__(kFT) k_fw_gty(PowArgs a) {
  if (!a.st->pow_active) return;
  __shared__ double red[16][kGtyCols + 1];
  const int cq = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const int c0 = blockIdx.x * kGtyCols;
  const int rc = blockIdx.y;
  const int per = (a.m + a.nchunk - 1) / a.nchunk;
  const int i0 = rc * per, i1 = min(a.m, i0 + per);
  int col[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) col[e] = VEC == 4 ? c0 + cq * 4 + e : c0 + cq + 16 * e;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (VEC == 4 ? col[0] < a.n : true) {
#pragma unroll 4
    for (int i = i0 + rg; i < i1; i += 16) {
      const double ti = a.t[i];
      const float* g = a.G + (size_t)i * a.n;
      if constexpr (VEC == 4) {
        const float4 v = *reinterpret_cast<const float4*>(g + col[0]);
        acc[0] += ti * v.x;
        acc[1] += ti * v.y;
        acc[2] += ti * v.z;
        acc[3] += ti * v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col[e] < a.n) acc[e] += ti * g[col[e]];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) red[rg][col[e] - c0] = acc[e];
  __syncthreads();
  if (threadIdx.x < kGtyCols) {
    const int j = c0 + threadIdx.x;
    double sum = 0.0;
    for (int r = 0; r < 16; ++r) sum += red[r][threadIdx.x];
    if (j < a.n) a.partial[(size_t)rc * a.n + j] = sum;
  }
}

// y_j = sum over blocks of partial[b][j]; per-block sums of y_j^2
__global__ void __launch_bounds__(kFT) k_fw_power_cols(PowArgs a, int nb) {
  if (!a.st->pow_active) return;
  __shared__ double red[kFT / 64];
  double sq = 0.0;
  const int j = blockIdx.x * kFT + threadIdx.x;
  if (j < a.n) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += a.partial[(size_t)b * a.n + j];   // fixed order
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
// B_ic = sum_j Q_ij P_jc P_j,c+1, QDP_ic = sum_j Q_ij D_ij P_jc; the pass's layout, five
// partial sums per chunk, added per coarse column in chunk order.
template <bool MASKED, int VEC, int PF>
__global__ void __launch_bounds__(kFT) k_fw_mask_tables(PassML a, float* __restrict__ Aq, float* __restrict__ Bq,
                                                       float* __restrict__ QDP) {
  extern __shared__ __align__(16) char smem_raw[];
  const MlLds lay = ml_lds(a.n, a.nH, a.R, a.K, a.nw, 5, 8);
  double* sp = reinterpret_cast<double*>(smem_raw + lay.sp);               // [5][R][K]
  int* sKf = reinterpret_cast<int*>(smem_raw + lay.kf);
  float* sD = reinterpret_cast<float*>(smem_raw + lay.d);
  uint32_t* sQ = reinterpret_cast<uint32_t*>(smem_raw + lay.q);
  const int tid = threadIdx.x;
  for (int c = tid; c <= a.nH; c += kFT) sKf[c] = a.kfirst[c];
  const int tr = tid / a.K, tk = tid - tr * a.K;
  Chunk ch{};
  if (tr < a.R) ch = a.chunks[tk];
  const size_t RK = (size_t)a.R * a.K;
  const int nbatch = (a.m + a.R - 1) / a.R;
  float rd[4 * PF];
  uint32_t rq = 0xFFFFFFFFu;
  for (int b = blockIdx.x; b < nbatch; b += gridDim.x) {
    const int i0 = b * a.R;
    const int rows = min(a.R, a.m - i0);
    stage_load<VEC, PF, MASKED>(a, i0, rows, rd, rq);
    stage_store<VEC, PF, MASKED>(a, rows, rd, rq, sD, sQ);
    __syncthreads();
    if (tr < rows) {
      const float* drow = sD + (size_t)tr * a.n;
      const uint32_t* qrow = sQ + (size_t)tr * a.nw;
      double A0 = 0, A1 = 0, B = 0, Q0 = 0, Q1 = 0;
      for (int j = ch.j0; j < ch.j1; ++j) {
        if (MASKED && !((qrow[j >> 5] >> (j & 31)) & 1u)) continue;
        const float wf = chunk_w0(ch, j, a.w0);
        const double w0 = wf, w1 = (double)(1.0f - wf);
        const double d = drow[j];
        A0 += w0 * w0;
        A1 += w1 * w1;
        B += w0 * w1;
        Q0 += w0 * d;
        Q1 += w1 * d;
      }
      const size_t o = (size_t)tr * a.K + tk;
      sp[o] = A0;
      sp[RK + o] = A1;
      sp[2 * RK + o] = B;
      sp[3 * RK + o] = Q0;
      sp[4 * RK + o] = Q1;
    }
    __syncthreads();
    for (int t = tid; t < rows * a.nH; t += kFT) {
      const int r = t / a.nH, c = t - r * a.nH;
      double A = 0, B = 0, QD = 0;
      for (int k = sKf[c]; k < sKf[c + 1]; ++k) {
        const size_t o = (size_t)r * a.K + k;
        A += sp[o];
        B += sp[2 * RK + o];
        QD += sp[3 * RK + o];
      }
      if (c > 0)
        for (int k = sKf[c - 1]; k < sKf[c]; ++k) {
          const size_t o = (size_t)r * a.K + k;
          A += sp[RK + o];
          QD += sp[4 * RK + o];
        }
      const size_t o = (size_t)(i0 + r) * a.ldz + c;
      Aq[o] = (float)A;
      Bq[o] = (float)B;
      QDP[o] = (float)QD;
    }
    __syncthreads();
  }
}

// Returned iterate: L (multilevel: Z P^T; plain: already in L) and S = P_Q S_{lam_S}[D - L]
// (zero before the first threshold step).  A block walks rows; multilevel stages the
// stencil taps once and each row of Z in LDS.
template <bool ML, int VEC>
__global__ void __launch_bounds__(kFT) k_fw_output(int m, int n, int nH, int levels, const float* __restrict__ D,
                                                  int ldd, const uint32_t* __restrict__ bits, int nw,
                                                  const float* __restrict__ Z, int ldz,
                                                  const uint32_t* __restrict__ taps, float lamS, int thr,
                                                  float* __restrict__ L, int ldl, float* __restrict__ S, int lds) {
  extern __shared__ char smem_raw[];
  uint32_t* sTap = reinterpret_cast<uint32_t*>(smem_raw);   // [n] (multilevel)
  float* sZr = reinterpret_cast<float*>(sTap + (ML ? n : 0)); // [nH]
  const float scale = ldexpf(1.0f, -levels);
  if (ML)
    for (int j = threadIdx.x; j < n; j += kFT) sTap[j] = taps[j];
  const int nv = n / VEC;
  for (int i = blockIdx.x; i < m; i += gridDim.x) {
    if (ML) {
      __syncthreads();
      for (int c = threadIdx.x; c < nH; c += kFT) sZr[c] = Z[(size_t)i * ldz + c];
      __syncthreads();
    }
    const float* drow = D + (size_t)i * ldd;
    float* lrow = L + (size_t)i * ldl;
    float* srow = S + (size_t)i * lds;
    for (int sv4 = threadIdx.x; sv4 < nv; sv4 += kFT) {
      const int j = sv4 * VEC;
      float d[VEC], l[VEC], sv[VEC];
      if constexpr (VEC == 4) {
        const float4 v = *reinterpret_cast<const float4*>(drow + j);
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        if (!ML) {
          const float4 x = *reinterpret_cast<const float4*>(lrow + j);
          l[0] = x.x; l[1] = x.y; l[2] = x.z; l[3] = x.w;
        }
      } else {
        d[0] = drow[j];
        if (!ML) l[0] = lrow[j];
      }
      const uint32_t word = bits ? bits[(size_t)i * nw + (j >> 5)] : 0xFFFFFFFFu;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        if (ML) {
          int c;
          float w0;
          unpack_tap(sTap[j + e], scale, c, w0);
          l[e] = lift(sZr, c, w0, nH);
        }
        const bool q = (word >> ((j + e) & 31)) & 1u;
        float gv;
        if (thr)
          entry<true>(d[e], l[e], q, lamS, sv[e], gv);
        else
          entry<false>(d[e], l[e], q, lamS, sv[e], gv);
      }
      if constexpr (VEC == 4) {
        if (ML) *reinterpret_cast<float4*>(lrow + j) = make_float4(l[0], l[1], l[2], l[3]);
        *reinterpret_cast<float4*>(srow + j) = make_float4(sv[0], sv[1], sv[2], sv[3]);
      } else {
        if (ML) lrow[j] = l[0];
        srow[j] = sv[0];
      }
    }
  }
}

// bits[i][w] bit b = (Q[i][32 w + b] != 0): one wave per 64 columns of a row, one byte
// per lane (coalesced), the words from a wave ballot
__global__ void __launch_bounds__(kFT) k_fw_pack_mask(int m, int n, const uint8_t* __restrict__ Q, int nw,
                                                     uint32_t* __restrict__ bits) {
  const int lane = threadIdx.x & 63;
  const int segs = (n + 63) / 64;
  const size_t total = (size_t)m * segs;
  for (size_t t = (size_t)blockIdx.x * (kFT / 64) + (threadIdx.x >> 6); t < total; t += (size_t)gridDim.x * (kFT / 64)) {
    const int i = (int)(t / segs), sg = (int)(t - (size_t)i * segs);
    const int j = sg * 64 + lane;
    const bool q = j < n && Q[(size_t)i * n + j] != 0;
    const unsigned long long b = __ballot(q);
    const int w = sg * 2;
    if (lane == 0) bits[(size_t)i * nw + w] = (uint32_t)b;
    if (lane == 1 && w + 1 < nw) bits[(size_t)i * nw + w + 1] = (uint32_t)(b >> 32);
  }
}

// The same packing for rows of a multiple of 8 bytes (8-byte aligned): each lane
// loads 8 mask bytes at once and makes 8 bits, four lanes make one 32-bit word (lane 0
// of the four gathers the others' bytes by shuffle and stores it), so a wave moves
// 512 mask bytes per load instead of 64.  Work item: one (row, word); 16 per wave.
__global__ void __launch_bounds__(kFT) k_fw_pack_mask8(int m, int n, const uint8_t* __restrict__ Q, int nw,
                                                      uint32_t* __restrict__ bits) {
  const int lane = threadIdx.x & 63, k = lane & 3;
  const int chunks = n / 8;   // 8-byte chunks per row
  const size_t total = (size_t)m * nw;
  const size_t wave = (size_t)blockIdx.x * (kFT / 64) + (threadIdx.x >> 6);
  for (size_t t0 = wave * 16; t0 < total; t0 += (size_t)gridDim.x * (kFT / 64) * 16) {
    const size_t t = t0 + (lane >> 2);   // this lane's (row, word)
    uint32_t b = 0;
    if (t < total) {
      const int i = (int)(t / nw), wd = (int)(t - (size_t)i * nw);
      const int c = 4 * wd + k;
      if (c < chunks) {
        const unsigned long long x = *reinterpret_cast<const unsigned long long*>(Q + (size_t)i * n + 8 * (size_t)c);
#pragma unroll
        for (int u = 0; u < 8; ++u) b |= (((x >> (8 * u)) & 0xFFull) != 0 ? 1u : 0u) << u;
      }
    }
    const uint32_t b1 = __shfl_down(b, 1), b2 = __shfl_down(b, 2), b3 = __shfl_down(b, 3);
    if (k == 0 && t < total) bits[t] = b | (b1 << 8) | (b2 << 16) | (b3 << 24);
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

// Host tables of the multilevel pass: each fine column's packed first stencil tap and
// weight, checked against the structure the kernels rely on (adjacent taps summing to
// one, first taps non-decreasing in j, dyadic weights), and the chunking of a row
// (contiguous fine columns inside one interval of equal first tap, at least kChunkMin
// long unless the interval is shorter, at most kFT chunks) with each interval's first
// chunk.  Built once per (n, levels) and kept.
struct FwTables {
  std::vector<uint32_t> taps;
  std::vector<float> w0;
  std::vector<Chunk> chunks;
  std::vector<int> kfirst;
  int maxlen = 0;
};

int fw_tables(int n, int levels, int nH, FwTables& t) {
  std::vector<int> ri, cp, cr;
  std::vector<float> rw, cw;
  build_stencil_host(n, levels, ri, rw, cp, cr, cw, nullptr);
  t.taps.assign(n, 0);
  t.w0.assign(n, 0.0f);
  const double den = std::ldexp(1.0, levels);
  int prev = -1;
  for (int j = 0; j < n; ++j) {
    const int c0 = ri[(size_t)j * kMaxStencil], c1 = ri[(size_t)j * kMaxStencil + 1];
    const double w0 = rw[(size_t)j * kMaxStencil], w1 = rw[(size_t)j * kMaxStencil + 1];
    if (w1 != 0.0 && c1 != c0 + 1) return MLPCP_E_UNSUPPORTED;      // taps are adjacent pairs
    if (std::fabs(w0 + w1 - 1.0) > 1e-12) return MLPCP_E_UNSUPPORTED;
    if (c0 < prev || c0 >= nH) return MLPCP_E_UNSUPPORTED;         // first taps non-decreasing
    const double num = w0 * den;
    if (num != std::floor(num) || num < 0 || num > 65535.0) return MLPCP_E_UNSUPPORTED;
    t.taps[j] = ((uint32_t)c0 << 16) | (uint32_t)num;
    t.w0[j] = (float)w0;
    prev = c0;
  }
  std::vector<int> first(nH + 1, n);
  {
    int j = 0;
    for (int c = 0; c <= nH; ++c) {
      while (j < n && (int)(t.taps[j] >> 16) < c) ++j;
      first[c] = j;
    }
  }
  // the shortest L (>= kChunkMin) whose chunking, with cuts where the weight stops being
  // affine, gives at most kFT chunks
  auto count = [&](int L) {
    long long cnt = 0;
    for (int c = 0; c < nH; ++c)
      for (int j = first[c]; j < first[c + 1];) {
        int j1 = std::min(first[c + 1], j + L);
        const float wb = t.w0[j], ws = j1 - j > 1 ? t.w0[j + 1] - t.w0[j] : 0.0f;
        for (int jj = j + 1; jj < j1; ++jj)
          if (std::fmaf(ws, (float)(jj - j), wb) != t.w0[jj]) {
            j1 = jj;
            break;
          }
        ++cnt;
        j = j1;
      }
    return cnt;
  };
  int L = kChunkMin;
  while (count(L) > kFT && L < 32) ++L;
  if (count(L) > kFT) return MLPCP_E_UNSUPPORTED;   // rows wider than 256 chunks of 32
  t.chunks.clear();
  t.maxlen = 0;
  t.kfirst.assign(nH + 1, 0);
  for (int c = 0; c < nH; ++c) {
    t.kfirst[c] = (int)t.chunks.size();
    for (int j = first[c]; j < first[c + 1];) {
      // at most L columns, cut where w0 stops being affine in j (exactly, in float)
      Chunk ch{c, j, std::min(first[c + 1], j + L), 1, t.w0[j], 0.0f, 0.0f, 0.0f};
      ch.ws = ch.j1 - ch.j0 > 1 ? t.w0[j + 1] - t.w0[j] : 0.0f;
      for (int jj = ch.j0 + 1; jj < ch.j1; ++jj)
        if (std::fmaf(ch.ws, (float)(jj - ch.j0), ch.wb) != t.w0[jj]) {
          ch.j1 = jj;
          break;
        }
      t.chunks.push_back(ch);
      t.maxlen = std::max(t.maxlen, ch.j1 - ch.j0);
      j = ch.j1;
    }
  }
  t.kfirst[nH] = (int)t.chunks.size();
  return MLPCP_OK;
}

std::mutex g_tab_mutex;
std::map<std::pair<int, int>, std::shared_ptr<const FwTables>> g_tabs;

int fw_tables_cached(int n, int levels, int nH, std::shared_ptr<const FwTables>& out) {
  std::lock_guard<std::mutex> lock(g_tab_mutex);
  auto it = g_tabs.find({n, levels});
  if (it != g_tabs.end()) {
    out = it->second;
    return MLPCP_OK;
  }
  auto t = std::make_shared<FwTables>();
  MLPCP_TRY(fw_tables(n, levels, nH, *t));
  g_tabs.emplace(std::make_pair(n, levels), t);
  out = t;
  return MLPCP_OK;
}

struct FwPlan {
  int m, n, nH, levels, nw, VEC, R, K, PF, ldz;
  bool ml, masked;
  unsigned grid_pass, grid_terms;
  size_t lds_pass, lds_tables;
  // plain power iteration
  int nchunk;
  unsigned grid_gx, grid_cols;
  size_t lds_pow;
  size_t off_bits, off_state, off_part, off_pmax, off_pidx, off_tpart, off_gz, off_taps, off_w0, off_chunks,
      off_kfirst;
  size_t off_Z, off_Z2, off_GP, off_Aq, off_Bq, off_QDP, off_gram, off_gws, off_lam, off_T;
  size_t off_G, off_w, off_powp, off_t, off_y, off_ypart;
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
    std::shared_ptr<const FwTables> t;
    MLPCP_TRY(fw_tables_cached(n, levels, p.nH, t));
    p.ldz = kPad;   // Z, GP, tables share the Gram's padded width
    p.K = (int)t->chunks.size();
    const int nv = n / p.VEC;
    // rows per batch: fill the tasks (R K <= kFT) within 8 float4 of staging per thread
    p.R = std::max(1, std::min(8, kFT / std::max(1, p.K)));
    auto pf_for = [&](int R) { return ((R * nv + kFT - 1) / kFT * p.VEC + 3) / 4; };   // float4s per thread
    while (p.R > 1 && (pf_for(p.R) > 8 || p.R * p.nw > kFT || p.R * p.nH > 2 * kFT)) --p.R;
    if (pf_for(p.R) > 8 || p.nw > kFT) return MLPCP_E_UNSUPPORTED;
    const int pf = pf_for(p.R);
    p.PF = pf <= 2 ? 2 : pf <= 4 ? 4 : pf <= 6 ? 6 : 8;
    p.lds_pass = ml_lds(n, p.nH, p.R, p.K, p.nw, 2, 4).total;
    p.lds_tables = ml_lds(n, p.nH, p.R, p.K, p.nw, 5, 8).total;
    if (p.lds_pass > 150 * 1024 || p.lds_tables > 150 * 1024) return MLPCP_E_UNSUPPORTED;
    const int per_cu = std::max(1, std::min(8, (int)((160 * 1024) / (p.lds_pass + 2048))));
    const int nbatch = (m + p.R - 1) / p.R;
    p.grid_pass = (unsigned)std::max(1, std::min(nbatch, per_cu * C));
  } else {
    const size_t slots = (size_t)m * (n / p.VEC);
    p.grid_pass = grid_of(slots, 4u * C);
    // power iteration layout
    if (n > 8192 || (p.VEC == 1 && n > 2048)) return MLPCP_E_UNSUPPORTED;
    p.lds_pow = (size_t)n * 8;
    p.nchunk = std::max(1, std::min(kPowRanges, (m + 15) / 16));
    p.grid_gx = (unsigned)std::max(1, std::min((m + 3) / 4, 8 * C));
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
    p.off_w0 = take((size_t)n * 4);
    p.off_chunks = take((size_t)p.K * sizeof(Chunk));
    p.off_kfirst = take((size_t)(p.nH + 1) * 4);
    const size_t mat = (size_t)m * p.ldz * 4;
    p.off_Z = take(mat);
    p.off_Z2 = take(mat);
    p.off_GP = take(mat);
    p.off_Aq = take(mat);
    p.off_Bq = take(mat);
    p.off_QDP = take(mat);
    const size_t sq = (size_t)kEigInner * kEigInner * 8;
    p.off_gram = take(sq);
    p.off_gws = take(gram_workspace_bytes(m, kPad));
    p.off_lam = take(8);
    p.off_T = take((size_t)kEigInner * 8);   // the coarse direction z
  } else {
    p.off_G = take((size_t)m * n * 4);
    p.off_w = take((size_t)n * 8);
    p.off_powp = take((size_t)p.nchunk * n * 8);
    p.off_t = take((size_t)m * 8);
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

template <bool MASKED, int VEC, int PF>
int launch_pass_ml_pf(const FwPlan& p, const PassML& a, bool thr, hipStream_t s) {
  auto k = thr ? k_fw_pass_ml<MASKED, VEC, PF, true> : k_fw_pass_ml<MASKED, VEC, PF, false>;
  if (p.lds_pass > 64 * 1024)
    MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_pass));
  hipLaunchKernelGGL(k, dim3(p.grid_pass), dim3(kFT), p.lds_pass, s, a);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

template <bool MASKED, int VEC>
int launch_pass_ml(const FwPlan& p, const PassML& a, bool thr, hipStream_t s) {
  switch (p.PF) {
    case 2: return launch_pass_ml_pf<MASKED, VEC, 2>(p, a, thr, s);
    case 4: return launch_pass_ml_pf<MASKED, VEC, 4>(p, a, thr, s);
    case 6: return launch_pass_ml_pf<MASKED, VEC, 6>(p, a, thr, s);
    default: return launch_pass_ml_pf<MASKED, VEC, 8>(p, a, thr, s);
  }
}

template <bool MASKED, int VEC, int PF>
int launch_tables_pf(const FwPlan& p, const PassML& a, float* Aq, float* Bq, float* QDP, hipStream_t s) {
  auto kt = k_fw_mask_tables<MASKED, VEC, PF>;
  if (p.lds_tables > 64 * 1024)
    MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kt), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_tables));
  hipLaunchKernelGGL(kt, dim3(p.grid_pass), dim3(kFT), p.lds_tables, s, a, Aq, Bq, QDP);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

template <bool MASKED, int VEC>
int launch_tables(const FwPlan& p, const PassML& a, float* Aq, float* Bq, float* QDP, hipStream_t s) {
  switch (p.PF) {
    case 2: return launch_tables_pf<MASKED, VEC, 2>(p, a, Aq, Bq, QDP, s);
    case 4: return launch_tables_pf<MASKED, VEC, 4>(p, a, Aq, Bq, QDP, s);
    case 6: return launch_tables_pf<MASKED, VEC, 6>(p, a, Aq, Bq, QDP, s);
    default: return launch_tables_pf<MASKED, VEC, 8>(p, a, Aq, Bq, QDP, s);
  }
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
  if (p.lds_pow > 64 * 1024)
    MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_fw_gx<VEC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_pow));
  hipLaunchKernelGGL(k_fw_gx<VEC>, dim3(p.grid_gx), dim3(kFT), p.lds_pow, s, a);
  const unsigned coltiles = (unsigned)((p.n + kGtyCols - 1) / kGtyCols);
  hipLaunchKernelGGL(k_fw_gty<VEC>, dim3(coltiles, (unsigned)p.nchunk), dim3(kFT), 0, s, a);
  hipLaunchKernelGGL(k_fw_power_cols, dim3(p.grid_cols), dim3(kFT), 0, s, a, p.nchunk);
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
    if (n % 8 == 0 && (reinterpret_cast<uintptr_t>(Q) & 7) == 0) {
      const size_t items = (size_t)m * p.nw;   // (row, word) pairs, 16 per wave, 4 waves per block
      hipLaunchKernelGGL(k_fw_pack_mask8, dim3((unsigned)std::min<size_t>((items + 63) / 64, 8u * cus())), dim3(kFT),
                         0, s, m, n, Q, p.nw, bits);
    } else {
      const size_t segs = (size_t)m * ((n + 63) / 64);
      hipLaunchKernelGGL(k_fw_pack_mask, dim3((unsigned)std::min<size_t>((segs + 3) / 4, 8u * cus())), dim3(kFT), 0,
                         s, m, n, Q, p.nw, bits);
    }
  }
  MLPCP_HIP(hipMemsetAsync(gz, 0, (size_t)m * 8, s));

  // operator tables (multilevel)
  uint32_t* taps = nullptr;
  std::shared_ptr<const FwTables> tbp;
  PassML pm{};
  if (p.ml) {
    MLPCP_TRY(fw_tables_cached(n, levels, p.nH, tbp));
    const FwTables& tb = *tbp;
    taps = w.at<uint32_t>(p.off_taps);
    MLPCP_HIP(hipMemcpyAsync(taps, tb.taps.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    if ((int)tb.chunks.size() != p.K) return MLPCP_E_UNSUPPORTED;
    MLPCP_HIP(hipMemcpyAsync(w.at<void>(p.off_w0), tb.w0.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    MLPCP_HIP(hipMemcpyAsync(w.at<void>(p.off_chunks), tb.chunks.data(), (size_t)p.K * sizeof(Chunk),
                             hipMemcpyHostToDevice, s));
    MLPCP_HIP(hipMemcpyAsync(w.at<void>(p.off_kfirst), tb.kfirst.data(), (size_t)(p.nH + 1) * 4,
                             hipMemcpyHostToDevice, s));
    const size_t mat = (size_t)m * p.ldz * 4;
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_Z), 0, mat, s));
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_Z2), 0, mat, s));
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_GP), 0, mat, s));
    MLPCP_HIP(hipMemsetAsync(w.at<void>(p.off_T), 0, (size_t)kEigInner * 8, s));
    pm.m = m; pm.n = n; pm.nH = p.nH; pm.R = p.R; pm.K = p.K; pm.nw = p.nw; pm.levels = levels;
    pm.maxlen = tb.maxlen;
    pm.D = D; pm.ldd = ldd; pm.bits = bits;
    pm.Zin = w.at<float>(p.off_Z); pm.Zout = w.at<float>(p.off_Z2); pm.ldz = p.ldz;
    pm.GP = w.at<float>(p.off_GP); pm.ldg = p.ldz;
    pm.taps = taps;
    pm.w0 = w.at<float>(p.off_w0); pm.chunks = w.at<Chunk>(p.off_chunks); pm.kfirst = w.at<int>(p.off_kfirst);
    pm.T = w.at<double>(p.off_T); pm.ldT = 1;
    pm.gz = gz; pm.st = st; pm.lamS = lamS;
    pm.partial = part; pm.pmax = pmax; pm.pidx = pidx;
    {
      float *Aq = w.at<float>(p.off_Aq), *Bq = w.at<float>(p.off_Bq), *QDP = w.at<float>(p.off_QDP);
      int st_tab;
      if (p.masked)
        st_tab = p.VEC == 4 ? launch_tables<true, 4>(p, pm, Aq, Bq, QDP, s) : launch_tables<true, 1>(p, pm, Aq, Bq, QDP, s);
      else
        st_tab = p.VEC == 4 ? launch_tables<false, 4>(p, pm, Aq, Bq, QDP, s)
                            : launch_tables<false, 1>(p, pm, Aq, Bq, QDP, s);
      MLPCP_TRY(st_tab);
    }
  } else {
    hipLaunchKernelGGL(k_fw_fill, dim3((n + 255) / 256), dim3(256), 0, s, w.at<double>(p.off_w), n,
                       1.0 / std::sqrt((double)n));
    MLPCP_HIP(hipGetLastError());
  }

  PassPlain pp{};
  if (!p.ml) {
    pp.m = m; pp.n = n; pp.nw = p.nw; pp.D = D; pp.ldd = ldd; pp.bits = bits;
    pp.L = L; pp.G = w.at<float>(p.off_G); pp.w = w.at<double>(p.off_w); pp.gz = gz; pp.st = st;
    pp.lamS = lamS; pp.partial = part; pp.pmax = pmax; pp.pidx = pidx;
  }
  // the current coarse state: Z (zeros) until the first step; each multilevel pass
  // reads it and writes the other buffer
  float* zbuf[2] = {p.ml ? w.at<float>(p.off_Z) : nullptr, p.ml ? w.at<float>(p.off_Z2) : nullptr};
  int zcur = 0;
  auto pass = [&](bool thr) -> int {
    ProfScope ps(KC_FW_PASS, s);
    if (p.ml) {
      pm.Zin = zbuf[zcur];
      pm.Zout = zbuf[1 - zcur];
      if (thr) zcur = 1 - zcur;
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
    hipLaunchKernelGGL(k_fw_finalize, dim3(1), dim3(kFT), 0, s, part, pmax, pidx, (int)p.grid_pass, (double)lamL,
                       (double)lamS, thr ? 1 : 0, st);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  };

  // iterate 0: L = S = 0
  MLPCP_TRY(pass(false));
  MLPCP_TRY(finalize(false));
  FwState hs;
  FwSlot* slot = fw_slot();
  MLPCP_TRY(read_state(slot, st, &hs, s));
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
  while (!converged && status == MLPCP_OK && k < max_iter) {
    // the nuclear direction
    if (p.ml) {
      {
        ProfScope ps(KC_GRAM, s);
        MLPCP_TRY(gram_f64(m, p.nH, kPad, w.at<float>(p.off_GP), p.ldz, w.at<double>(p.off_gram),
                           w.at<void>(p.off_gws), s, 0));
      }
      // the top eigenpair of C (GP^T GP) C gives z = C v_top: the coarse direction
      {
        ProfScope pt(KC_FW_TOP, s);
        MLPCP_TRY(coarse_top_small(p.nH, w.at<double>(p.off_gram), op->C, w.at<double>(p.off_T),
                                   w.at<double>(p.off_lam), s));
      }
      TermsML ta{};
      ta.m = m; ta.nH = p.nH; ta.Z = zbuf[zcur]; ta.GP = w.at<float>(p.off_GP);
      ta.Aq = w.at<float>(p.off_Aq); ta.Bq = w.at<float>(p.off_Bq); ta.QDP = w.at<float>(p.off_QDP);
      ta.ld = p.ldz; ta.T = w.at<double>(p.off_T); ta.ldT = 1; ta.gz = gz; ta.partial = tpart;
      ProfScope ps(KC_FW_SMALL, s);
      hipLaunchKernelGGL(k_fw_terms_ml, dim3(p.grid_terms), dim3(kFT), (size_t)p.nH * 8, s, ta);
      MLPCP_HIP(hipGetLastError());
    } else {
      PowArgs pa{};
      pa.m = m; pa.n = n; pa.nchunk = p.nchunk; pa.G = w.at<float>(p.off_G); pa.x = w.at<double>(p.off_w);
      pa.t = w.at<double>(p.off_t); pa.partial = w.at<double>(p.off_powp); pa.y = w.at<double>(p.off_y);
      pa.ypart = w.at<double>(p.off_ypart);
      pa.st = st;
      hipLaunchKernelGGL(k_fw_power_start, dim3(1), dim3(1), 0, s, st);
      int done_steps = 0;
      for (;;) {
        {
          ProfScope ps(KC_FW_POWER, s);
          for (int b = 0; b < pow_batch; ++b)
            MLPCP_TRY(p.VEC == 4 ? launch_power_step<4>(p, pa, s) : launch_power_step<1>(p, pa, s));
        }
        MLPCP_TRY(read_state(slot, st, &hs, s));
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
      sa.D = D; sa.ldd = ldd; sa.L = L; sa.Z = p.ml ? zbuf[zcur] : nullptr; sa.ldz = p.ldz;
      sa.taps = taps;
      sa.T = p.ml ? w.at<double>(p.off_T) : nullptr; sa.ldT = 1;
      sa.w = p.ml ? nullptr : w.at<double>(p.off_w); sa.gz = gz; sa.lamL = lamL; sa.lamS = lamS; sa.st = st;
      ProfScope ps(KC_FW_SMALL, s);
      hipLaunchKernelGGL(k_fw_solve, dim3(1), dim3(kFT), 0, s, sa);
      MLPCP_HIP(hipGetLastError());
    }
    MLPCP_TRY(pass(true));
    MLPCP_TRY(finalize(true));
    thr = true;
    MLPCP_TRY(read_state(slot, st, &hs, s));
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
    const unsigned g = (unsigned)std::min(m, 8 * cus());
    const size_t lds = p.ml ? (size_t)n * 4 + (size_t)p.nH * 4 : 0;
    const bool v4 = p.VEC == 4 && reinterpret_cast<uintptr_t>(S) % 16 == 0;
    float* zc = p.ml ? zbuf[zcur] : nullptr;
    auto ko = p.ml ? (v4 ? k_fw_output<true, 4> : k_fw_output<true, 1>) : (v4 ? k_fw_output<false, 4> : k_fw_output<false, 1>);
    if (lds > 64 * 1024)
      MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(ko), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
    hipLaunchKernelGGL(ko, dim3(g), dim3(kFT), lds, s, m, n, p.nH, levels, D, ldd, bits, p.nw, zc, p.ldz, taps, lamS,
                       thr ? 1 : 0, L, n, S, n);
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
