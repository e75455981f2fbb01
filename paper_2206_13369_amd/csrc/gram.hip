// Gram matrix G = A^T A of the (coarse) data, float64 accumulation on MFMA.
//
// The singular values of the coarse data (Alg. 4) are taken as square roots of the
// eigenvalues of its Gram matrix.  Products of float32 operands are exact in float64,
// so accumulating in float64 keeps the singular values as accurate as the float32
// data itself (absolute error ~ eps32 * sigma_max) instead of squaring the condition
// number; this matters for the values just above the threshold 1/mu.
//
// Tiling: one 256-thread block computes a 32 x 32 output tile for a slice of rows
// ("split"), as 2 x 2 wave tiles of v_mfma_f64_16x16x4f64.  Only tiles on or above the
// diagonal are computed.  Partial tiles of the splits are summed in a fixed order
// (deterministic), and the lower triangle is mirrored from the upper one so G is
// exactly symmetric.
#include "common.h"
#include "profile.h"

#include <algorithm>

namespace mlpcp {

namespace {

constexpr int GT = 32;   // output tile
constexpr int KC = 16;   // rows per LDS chunk

typedef double d4_t __attribute__((ext_vector_type(4)));

// Blocks are dealt to the eight XCDs in turn (block L to XCD L mod 8), and each XCD has
// its own L2.  With at least 8 splits a 1-D grid of 8 pairs ceil(splits / 8) blocks is
// decoded so that every block of split s runs on XCD s mod 8: the rows of a split are
// then fetched from HBM into one L2 only, however many output tiles read them (blocks
// with s >= splits exit).  With fewer splits the grid is pairs x splits, split-major.
__device__ __forceinline__ void xcd_decode(int L, int pairs, int splits, int& pair, int& s) {
  if (splits < 8) {
    pair = L % pairs;
    s = L / pairs;
    return;
  }
  const int xcd = L & 7, j = L >> 3;
  pair = j % pairs;
  s = (j / pairs) * 8 + xcd;
}

unsigned xcd_grid(int pairs, int splits) {
  return splits < 8 ? (unsigned)(pairs * splits) : (unsigned)(8 * pairs * ((splits + 7) / 8));
}

__device__ __forceinline__ void tri_decode(int p, int nt, int& ti, int& tj) {
  // p enumerates pairs (ti <= tj) row by row
  ti = 0;
  int rem = p;
  while (rem >= nt - ti) {
    rem -= nt - ti;
    ++ti;
  }
  tj = ti + rem;
}

// CROSS = false: G = A^T A, tiles on/above the diagonal; CROSS = true: G = A^T B, all tiles
template <bool CROSS>
__global__ void __launch_bounds__(256) k_gram_partial(const float* __restrict__ A, int m, int k, int lda, int kp,
                                                      int rows_per_split, int ntile, int splits,
                                                      double* __restrict__ part, const float* __restrict__ B,
                                                      int ldb) {
  __shared__ double sI[KC][GT + 1];
  __shared__ double sJ[KC][GT + 1];
  int ti, tj, pair, s;
  xcd_decode(blockIdx.x, CROSS ? ntile * ntile : ntile * (ntile + 1) / 2, splits, pair, s);
  if (s >= splits) return;
  if (CROSS) {
    ti = pair / ntile;
    tj = pair % ntile;
  } else {
    tri_decode(pair, ntile, ti, tj);
  }
  const int r0 = s * rows_per_split;
  const int r1 = min(m, r0 + rows_per_split);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int bi = wave >> 1, bj = wave & 1;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  const int ci0 = ti * GT, cj0 = tj * GT;
  for (int k0 = r0; k0 < r1; k0 += KC) {
#pragma unroll
    for (int x = 0; x < (KC * GT) / 256; ++x) {
      const int e = tid + 256 * x;
      const int row = e / GT, col = e % GT;
      const int gr = k0 + row;
      const bool rok = gr < r1;
      const int gi = ci0 + col, gj = cj0 + col;
      sI[row][col] = (rok && gi < k) ? (double)A[(size_t)gr * lda + gi] : 0.0;
      if (CROSS)
        sJ[row][col] = (rok && gj < k) ? (double)B[(size_t)gr * ldb + gj] : 0.0;
      else
        sJ[row][col] = (rok && gj < k) ? (double)A[(size_t)gr * lda + gj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const double a = sI[kk * 4 + (lane >> 4)][bi * 16 + (lane & 15)];
      const double b = sJ[kk * 4 + (lane >> 4)][bj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  double* P = part + (size_t)s * kp * kp;
  const int col = cj0 + bj * 16 + (lane & 15);
  // v_mfma_f64_16x16x4f64 output: register v of lane l holds row 4v + l/16, column l%16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = ci0 + bi * 16 + 4 * v + (lane >> 4);
    P[(size_t)row * kp + col] = acc[v];
  }
}

// Precision form of the Gram: operands rounded to bfloat16 (PREC 1) or split into
// bfloat16 hi + lo parts with three products hi*hi + hi*lo + lo*hi (PREC 2), on
// v_mfma_f32_16x16x32_bf16 with float32 accumulation over one 32-row chunk; the
// chunk sums are added in float64 (the Gram's smallest eigenvalues are what a long
// float32 running sum would lose), and the split partials by k_gram_reduce.  Operand layout of the
// instruction: lane l holds A[l%16][8(l/16)+q] and B[8(l/16)+q][l%16], q < 8; the
// output register v of lane l is row 4(l/16)+v, column l%16.
constexpr int KB = 32;  // rows per LDS chunk (one MFMA k-step)

template <int PREC>
__global__ void __launch_bounds__(256) k_gram_partial_bf16(const float* __restrict__ A, int m, int k, int lda, int kp,
                                                           int rows_per_split, int ntile, int splits,
                                                           double* __restrict__ part) {
  __shared__ float sI[KB][GT + 1];
  __shared__ float sJ[KB][GT + 1];
  int ti, tj, pair, s;
  xcd_decode(blockIdx.x, ntile * (ntile + 1) / 2, splits, pair, s);
  if (s >= splits) return;
  tri_decode(pair, ntile, ti, tj);
  const int r0 = s * rows_per_split;
  const int r1 = min(m, r0 + rows_per_split);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int bi = wave >> 1, bj = wave & 1;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  const int ci0 = ti * GT, cj0 = tj * GT;
  for (int k0 = r0; k0 < r1; k0 += KB) {
#pragma unroll
    for (int x = 0; x < (KB * GT) / 256; ++x) {
      const int e = tid + 256 * x;
      const int row = e / GT, col = e % GT;
      const int gr = k0 + row;
      const bool rok = gr < r1;
      const int gi = ci0 + col, gj = cj0 + col;
      sI[row][col] = (rok && gi < k) ? A[(size_t)gr * lda + gi] : 0.0f;
      sJ[row][col] = (rok && gj < k) ? A[(size_t)gr * lda + gj] : 0.0f;
    }
    __syncthreads();
    bf16x8_t ah, bh, al, bl;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kk = 8 * (lane >> 4) + q;
      const float xa = sI[kk][bi * 16 + (lane & 15)];
      const float xb = sJ[kk][bj * 16 + (lane & 15)];
      const unsigned short ha = f2bf(xa), hb = f2bf(xb);
      ah[q] = __builtin_bit_cast(__bf16, ha);
      bh[q] = __builtin_bit_cast(__bf16, hb);
      if (PREC == 2) {
        al[q] = __builtin_bit_cast(__bf16, f2bf(xa - bf2f(ha)));
        bl[q] = __builtin_bit_cast(__bf16, f2bf(xb - bf2f(hb)));
      }
    }
    f32x4_t c = {0.0f, 0.0f, 0.0f, 0.0f};
    if (PREC == 2) {
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    }
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += (double)c[v];
    __syncthreads();
  }
  double* P = part + (size_t)s * kp * kp;
  const int col = cj0 + bj * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = ci0 + bi * 16 + 4 * (lane >> 4) + v;
    P[(size_t)row * kp + col] = acc[v];
  }
}

// G[i][j] = sum over splits of the upper-triangle partial (i<=j mirrored), in a fixed
// order: 64 outputs per block, 4 thread groups each summing every 4th split, then the
// 4 group sums added in order.
template <bool CROSS>
__global__ void __launch_bounds__(256) k_gram_reduce(const double* __restrict__ part, int splits, int kp,
                                                     double* __restrict__ G) {
  __shared__ double red[4][64];
  const int e = threadIdx.x & 63, g = threadIdx.x >> 6;
  const size_t idx = (size_t)blockIdx.x * 64 + e;
  const size_t total = (size_t)kp * kp;
  double s = 0.0;
  if (idx < total) {
    const int i = (int)(idx / kp), j = (int)(idx % kp);
    const size_t off = CROSS ? idx : (size_t)min(i, j) * kp + max(i, j);
    for (int q = g; q < splits; q += 4) s += part[(size_t)q * total + off];
  }
  red[g][e] = s;
  __syncthreads();
  if (g == 0 && idx < total) G[idx] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// ---------------------------------------------------------------------------------
// Tall-skinny Gram for coarse widths k <= 64 (kp == 64): each block owns a row range
// and computes every upper 16 x 16 tile of the (k rounded up to 16)-wide Gram from
// 64-row chunks staged in LDS, the next chunk's loads in flight while the current one
// is multiplied.  Wave w owns tiles w, w + 4, w + 8.  PREC 0: float32 operands
// widened to float64 on v_mfma_f64_16x16x4f64 (exact products, float64 sums);
// PREC 1 / 2: bfloat16 / split bfloat16 on v_mfma_f32_16x16x32_bf16, chunk sums in
// float32 added in float64.  Partials: per split, tile u, 16 x 16 row-major.
constexpr int TALL_ROWS = 64;
constexpr int TALL_LD = 64 + 4;

// upper tile u of an nt x nt tile grid, row by row -> (ti, tj), ti <= tj
__device__ __forceinline__ void tall_tile(int u, int nt, int& ti, int& tj) {
  ti = 0;
  while (u >= nt - ti) {
    u -= nt - ti;
    ++ti;
  }
  tj = ti + u;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_gram_tall(const float* __restrict__ A, int m, int k, int lda,
                                                   int rows_per_split, int nt, double* __restrict__ part) {
  __shared__ float sX[TALL_ROWS][TALL_LD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int U = nt * (nt + 1) / 2;
  const int r0 = blockIdx.x * rows_per_split;
  const int r1 = min(m, r0 + rows_per_split);
  int ti[3], tj[3];
  bool own[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const int u = wave + 4 * x;
    own[x] = u < U;
    tall_tile(own[x] ? u : 0, nt, ti[x], tj[x]);
  }
  d4_t acc[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) acc[x] = (d4_t){0.0, 0.0, 0.0, 0.0};
  constexpr int PER = TALL_ROWS * 64 / 256;
  const int kc = nt * 16;
  float pre[PER];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int e = tid + 256 * x;
      const int row = e >> 6, col = e & 63;
      const int gr = c0 + row;
      pre[x] = (gr < r1 && col < k) ? A[(size_t)gr * lda + col] : 0.0f;
    }
  };
  fetch(r0);
  for (int c0 = r0; c0 < r1; c0 += TALL_ROWS) {
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int e = tid + 256 * x;
      const int col = e & 63;
      if (col < kc) sX[e >> 6][col] = pre[x];
    }
    __syncthreads();
    if (c0 + TALL_ROWS < r1) fetch(c0 + TALL_ROWS);
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      if (!own[x]) continue;
      const int ci = ti[x] * 16 + (lane & 15), cj = tj[x] * 16 + (lane & 15);
      if (PREC == 0) {
#pragma unroll
        for (int s = 0; s < TALL_ROWS / 4; ++s) {
          const int kk = 4 * s + (lane >> 4);
          acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)sX[kk][ci], (double)sX[kk][cj], acc[x], 0, 0, 0);
        }
      } else {
        constexpr int KS = TALL_ROWS / 32;
        bf16x8_t ah[KS], bh[KS], al[KS], bl[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int kk = 32 * s + 8 * (lane >> 4) + q;
            const float xa = sX[kk][ci], xb = sX[kk][cj];
            const unsigned short ha = f2bf(xa), hb = f2bf(xb);
            ah[s][q] = __builtin_bit_cast(__bf16, ha);
            bh[s][q] = __builtin_bit_cast(__bf16, hb);
            al[s][q] = __builtin_bit_cast(__bf16, f2bf(xa - bf2f(ha)));
            bl[s][q] = __builtin_bit_cast(__bf16, f2bf(xb - bf2f(hb)));
          }
        f32x4_t c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          if (PREC == 2) {
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s], bh[s], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], bl[s], c, 0, 0, 0);
          }
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], bh[s], c, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[x][v] += (double)c[v];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    if (!own[x]) continue;
    double* P = part + ((size_t)blockIdx.x * U + (wave + 4 * x)) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // f64 output: register v of lane l is row 4v + l/16; bf16: row 4(l/16) + v
      const int row = PREC == 0 ? 4 * v + (lane >> 4) : 4 * (lane >> 4) + v;
      P[row * 16 + (lane & 15)] = acc[x][v];
    }
  }
}

// Gram of coarse data at most 16 wide (the finest restrictions of the tall workloads),
// k <= 16: wave w of block b takes 64-row chunks of rows [r0 + w R, r0 + (w + 1) R),
// the next chunk's loads in flight while the current one is multiplied.  For
// v_mfma_f64_16x16x4f64 lane l reads A[row + l/16][l%16], which is both operands at once
// (A^T[l%16][l/16] and A[l/16][l%16]); with a leading dimension of 16 the four rows of a
// step are 256 contiguous bytes.  Precision forms (PREC 1 / 2) take 32 rows per
// v_mfma_f32_16x16x32_bf16 (lane l holds rows 8(l/16) + q, q < 8, of column l%16, again
// both operands), float32 sums over each 64-row chunk added in float64 as in
// k_gram_tall.  The four waves' 16 x 16 sums are added in a fixed order into the
// block's partial (split b, tile 0 of the tall partial layout).
template <int PREC>
__global__ void __launch_bounds__(256) k_gram16(const float* __restrict__ A, int m, int k, int lda,
                                                int rows_per_split, double* __restrict__ part) {
  __shared__ double red[4][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rw = rows_per_split / 4;   // rows per wave (a multiple of 64)
  const int r0 = blockIdx.x * rows_per_split + wave * rw;
  const int r1 = min(m, r0 + rw);
  const int c = lane & 15, g = lane >> 4;
  const bool cok = c < k;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  float cur[16], nxt[16];
  // element u of a chunk: PREC 0 row 4u + g; PREC 1/2 row 32(u / 8) + 8g + u % 8
  auto fetch = [&](int c0, float (&x)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int row = PREC == 0 ? c0 + 4 * u + g : c0 + 32 * (u >> 3) + 8 * g + (u & 7);
      x[u] = (cok && row < r1) ? A[(size_t)row * lda + c] : 0.0f;
    }
  };
  if (r0 < r1) fetch(r0, cur);
  for (int c0 = r0; c0 < r1; c0 += 64) {
    if (c0 + 64 < r1) fetch(c0 + 64, nxt);
    if (PREC == 0) {
#pragma unroll
      for (int u = 0; u < 16; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)cur[u], (double)cur[u], acc, 0, 0, 0);
    } else {
      f32x4_t cs = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        bf16x8_t h, lo;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float x = cur[8 * s2 + q];
          const unsigned short hb = f2bf(x);
          h[q] = __builtin_bit_cast(__bf16, hb);
          lo[q] = __builtin_bit_cast(__bf16, f2bf(x - bf2f(hb)));
        }
        if (PREC == 2) {
          cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, h, cs, 0, 0, 0);
          cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, lo, cs, 0, 0, 0);
        }
        cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, h, cs, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] += (double)cs[v];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) cur[u] = nxt[u];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // f64 output: register v of lane l is row 4v + l/16; bf16: row 4(l/16) + v
    const int row = PREC == 0 ? 4 * v + g : 4 * g + v;
    red[wave][row * 16 + c] = acc[v];
  }
  __syncthreads();
  part[(size_t)blockIdx.x * 256 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// G from the tall partials: 16 tile entries per block, 16 thread groups each summing
// every 16th split, then the group sums in order; each entry written to both halves.
// In a diagonal tile only the upper triangle is used: the split product sums (i, j)
// and (j, i) in different orders, so the two can differ in the last bits.
__global__ void __launch_bounds__(256) k_gram_tall_reduce(const double* __restrict__ part, int splits, int nt,
                                                          double* __restrict__ G, int ldg) {
  __shared__ double red[16][17];
  const int U = nt * (nt + 1) / 2;
  const int e = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int idx = blockIdx.x * 16 + e;
  const int total = U * 256;
  double s = 0.0;
  if (idx < total)
    for (int q = g; q < splits; q += 16) s += part[(size_t)q * total + idx];
  red[g][e] = s;
  __syncthreads();
  if (g == 0 && idx < total) {
    int a, b;
    tall_tile(idx >> 8, nt, a, b);
    const int r = (idx & 255) >> 4, c = idx & 15;
    if (a == b && r > c) return;
    const int i = a * 16 + r, j = b * 16 + c;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) v += red[k][e];
    G[(size_t)i * ldg + j] = v;
    G[(size_t)j * ldg + i] = v;
  }
}

void gram_tall_plan(int m, int nt, int& splits, int& rows_per_split) {
  const int U = nt * (nt + 1) / 2;
  const int target = U > 3 ? 512 : 1024;
  int rps = round_up((m + target - 1) / target, TALL_ROWS);
  splits = (m + rps - 1) / rps;
  rows_per_split = rps;
}

void gram_plan(int m, int kp, int& splits, int& rows_per_split, bool cross = false) {
  const int nt = kp / GT;
  const int pairs = cross ? nt * nt : nt * (nt + 1) / 2;
  int sp = (768 + pairs - 1) / pairs;
  const int max_by_rows = (m + 127) / 128;   // at least 128 rows per split
  if (sp > max_by_rows) sp = max_by_rows;
  const size_t cap = (size_t)64 << 20;
  const size_t per = (size_t)kp * kp * sizeof(double);
  if ((size_t)sp * per > cap) sp = (int)(cap / per);
  if (sp < 1) sp = 1;
  int rps = (m + sp - 1) / sp;
  rps = round_up(rps, KC);
  sp = (m + rps - 1) / rps;
  if (sp < 1) sp = 1;
  splits = sp;
  rows_per_split = rps;
}

}  // namespace

size_t gram_workspace_bytes(int m, int kp) {
  int sp, rps;
  gram_plan(m, kp, sp, rps);
  size_t b = (size_t)sp * kp * kp * sizeof(double);
  if (kp == 64)
    for (int nt = 1; nt <= 4; ++nt) {
      gram_tall_plan(m, nt, sp, rps);
      b = std::max(b, (size_t)sp * (nt * (nt + 1) / 2) * 256 * sizeof(double));
    }
  return align256(b);
}

// G = A^T A for few rows (m <= kGramDirectRows, a wide coarse model) in one launch: one
// upper 16 x 16 tile of G per block, the m rows split over the sixteen waves (float32
// operands converted exactly, v_mfma_f64_16x16x4f64 with two accumulator chains, the
// next 64 rows' operands loaded while the current ones are multiplied), the sixteen
// partial tiles summed in a fixed order and the tile written to both triangles (G exactly
// symmetric).  No partial Grams go through memory and there is no second launch: at
// 2000 x 250 the split form wrote and re-read 4.6 MB of partials per Gram.
constexpr int kGramDirectRows = 4096;
constexpr int kGdWaves = 16;
__global__ void __launch_bounds__(1024) k_gram_direct(const float* __restrict__ A, int m, int k, int lda, int kp,
                                                      double* __restrict__ G) {
  __shared__ double red[kGdWaves][256];
  const int nt = kp / 16;
  int tile = blockIdx.x, ti = 0;
  while (tile >= nt - ti) {
    tile -= nt - ti;
    ++ti;
  }
  const int tj = ti + tile;
  const int i0 = ti * 16, j0 = tj * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rpw = ((m + kGdWaves - 1) / kGdWaves + 3) & ~3;   // rows per wave, a multiple of 4
  const int r0 = wave * rpw, r1 = min(m, r0 + rpw);
  const int ci = i0 + li, cj = j0 + li;
  const bool vi = ci < k, vj = cj < k;
  d4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  constexpr int S = 16;   // MFMA steps (4 rows each) per batch
  float ca[S], cb[S], na[S], nb[S];
  auto load = [&](int r, float* a, float* b) {
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int row = r + 4 * q + lk;
      const bool in = row < r1;
      a[q] = (in && vi) ? A[(size_t)row * lda + ci] : 0.0f;
      b[q] = (in && vj) ? A[(size_t)row * lda + cj] : 0.0f;
    }
  };
  if (r0 < r1) load(r0, ca, cb);
  for (int r = r0; r < r1; r += 4 * S) {
    if (r + 4 * S < r1) load(r + 4 * S, na, nb);
#pragma unroll
    for (int q = 0; q < S; q += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ca[q], (double)cb[q], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ca[q + 1], (double)cb[q + 1], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
      ca[q] = na[q];
      cb[q] = nb[q];
    }
  }
  // output register v of lane l: row 4 v + l / 16, column l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][(4 * v + lk) * 16 + li] = acc0[v] + acc1[v];
  __syncthreads();
  if (tid >= 256) return;
  const int r = tid / 16, c = tid % 16;
  if (ti == tj && r > c) return;
  double g = 0.0;
#pragma unroll
  for (int w = 0; w < kGdWaves; ++w) g += red[w][tid];
  G[(size_t)(i0 + r) * kp + j0 + c] = g;
  G[(size_t)(j0 + c) * kp + i0 + r] = g;
}

int gram_f64(int m, int k, int kp, const float* A, int lda, double* G, void* ws, hipStream_t stream, int prec) {
  if (kp % GT != 0 || k > kp) return MLPCP_E_INVALID_ARG;
  int sp, rps;
  gram_plan(m, kp, sp, rps);
  const int nt = kp / GT;
  const int pairs = nt * (nt + 1) / 2;
  double* part = static_cast<double*>(ws);
  ProfScope ps(KC_GRAM, stream);
  if (kp == 64 && k <= 16) {
    // 256 rows per wave at most, at most 256 splits (blocks)
    rps = round_up((m + 255) / 256, 256);
    sp = (m + rps - 1) / rps;
    if (prec == MLPCP_BF16)
      hipLaunchKernelGGL(k_gram16<1>, dim3(sp), dim3(256), 0, stream, A, m, k, lda, rps, part);
    else if (prec == MLPCP_BF16X3)
      hipLaunchKernelGGL(k_gram16<2>, dim3(sp), dim3(256), 0, stream, A, m, k, lda, rps, part);
    else
      hipLaunchKernelGGL(k_gram16<0>, dim3(sp), dim3(256), 0, stream, A, m, k, lda, rps, part);
    hipLaunchKernelGGL(k_gram_tall_reduce, dim3(256 / 16), dim3(256), 0, stream, part, sp, 1, G, kp);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  if (kp == 64) {
    const int nt = (k + 15) / 16;
    gram_tall_plan(m, nt, sp, rps);
    if (prec == MLPCP_BF16)
      hipLaunchKernelGGL(k_gram_tall<1>, dim3(sp), dim3(256), 0, stream, A, m, k, lda, rps, nt, part);
    else if (prec == MLPCP_BF16X3)
      hipLaunchKernelGGL(k_gram_tall<2>, dim3(sp), dim3(256), 0, stream, A, m, k, lda, rps, nt, part);
    else
      hipLaunchKernelGGL(k_gram_tall<0>, dim3(sp), dim3(256), 0, stream, A, m, k, lda, rps, nt, part);
    const int total = nt * (nt + 1) / 2 * 256;
    hipLaunchKernelGGL(k_gram_tall_reduce, dim3((total + 15) / 16), dim3(256), 0, stream, part, sp, nt, G, kp);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  if (prec == 0 && m <= kGramDirectRows && kp <= 512) {
    const int nt16 = kp / 16;
    hipLaunchKernelGGL(k_gram_direct, dim3(nt16 * (nt16 + 1) / 2), dim3(1024), 0, stream, A, m, k, lda, kp, G);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  const dim3 grid(xcd_grid(pairs, sp));
  if (prec == MLPCP_BF16)
    hipLaunchKernelGGL(k_gram_partial_bf16<1>, grid, dim3(256), 0, stream, A, m, k, lda, kp, rps, nt, sp, part);
  else if (prec == MLPCP_BF16X3)
    hipLaunchKernelGGL(k_gram_partial_bf16<2>, grid, dim3(256), 0, stream, A, m, k, lda, kp, rps, nt, sp, part);
  else
    hipLaunchKernelGGL(k_gram_partial<false>, grid, dim3(256), 0, stream, A, m, k, lda, kp, rps, nt, sp, part,
                       nullptr, 0);
  const size_t nn = (size_t)kp * kp;
  hipLaunchKernelGGL(k_gram_reduce<false>, dim3((unsigned)((nn + 63) / 64)), dim3(256), 0, stream, part, sp, kp, G);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int cross_f64(int m, int k, int kp, const float* A, int lda, const float* B, int ldb, double* G, void* ws,
              hipStream_t stream) {
  if (kp % GT != 0 || k > kp) return MLPCP_E_INVALID_ARG;
  int sp, rps;
  gram_plan(m, kp, sp, rps, true);
  const int nt = kp / GT;
  double* part = static_cast<double*>(ws);
  ProfScope ps(KC_OTHER, stream);
  hipLaunchKernelGGL(k_gram_partial<true>, dim3(xcd_grid(nt * nt, sp)), dim3(256), 0, stream, A, m, k, lda, kp,
                     rps, nt, sp, part, B, ldb);
  const size_t nn = (size_t)kp * kp;
  hipLaunchKernelGGL(k_gram_reduce<true>, dim3((unsigned)((nn + 63) / 64)), dim3(256), 0, stream, part, sp, kp, G);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

}  // namespace mlpcp
