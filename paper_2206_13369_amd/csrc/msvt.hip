// Matrix-function form of the coarse singular value threshold.  The SVT step of Alg. 1
// and Alg. 4 maps the coarse data M (Gram G = M^T M, float64) to M f(G), with
// f(l) = (1 - tau / sqrt(l))_+ applied to the eigenvalues of G: only the singular values
// above tau enter (the paper remarks after Alg. 1 that only those need computing), and
// f is continuous, so f(G) can be formed from matrix products alone, without the
// eigenvectors:
//
//  1. sign phase: S = sign(A), A = G - tau^2 I, by the scaled Newton-Schulz iteration
//     X <- (a/2) X (3 I - a^2 X^2) from X = A / alpha (alpha >= ||A||_2), with the
//     coefficient a of each step chosen for the interval [l, 1] that holds the moduli
//     of X's eigenvalues (a = sqrt(3 / (1 + l + l^2)), after which the interval is
//     [a l (3 - a^2 l^2) / 2, 1]; Chen and Chow's scaling of the Newton-Schulz
//     iteration for the sign of a Hermitian matrix);
//  2. Gt = tau^2 I + (A + S A) / 2: the eigenvalues of G with those below tau^2
//     raised to tau^2, where f vanishes;
//  3. inverse square root phase: Z = (Gt / beta)^{-1/2} (beta >= ||Gt||_2) by the
//     coupled Newton-Schulz iteration T = (a/2)(3 I - a^2 Z Y), Y <- Y T, Z <- T Z from
//     Y = Gt / beta, Z = I (the sign iteration of [[0, Y], [I, 0]], scaled the same way
//     on [sqrt(tau^2 / beta), 1]);
//  4. f(G) = I - tau beta^{-1/2} Z, and the product operator K = C f(G) C of the
//     reconstruction L = M_P K P^T (C = (P^T P)^{-1/2}; C = I for the plain method).
//
// The iteration counts and coefficients are fixed on the host before the launches, from
// bounds carried over from the previous iteration (the device checks them and flags a
// violation).  An eigenvalue within l_0 alpha of tau^2 is left partly resolved by the
// sign phase; f is continuous with slope 1/(2 tau^2) there, so such an eigenvalue moves
// the result by at most about l_0 alpha / (2 tau^2) in its direction, where M has a
// singular value of about tau: l_0 is chosen so that this stays below kMsvtTarget
// relative to ||M||_2, and so that l_0 alpha is at most kMsvtRankRes tau^2.  The rank
// reported is the number of eigenvalues above tau^2, (N + trace S) / 2 rounded: exact
// for every eigenvalue farther than l_0 alpha from tau^2.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "profile.h"

namespace mlpcp {

namespace {

constexpr double kMsvtTarget = 1.0e-6;   // bound on the relative error of M f(G) (see above)
constexpr double kMsvtRankRes = 1.0e-3;  // every eigenvalue farther than this times tau^2 from
                                         // tau^2 is resolved (so the rank is exact there)
constexpr double kMsvtSignTail = 1.0e-8;  // the sign phase stops when 1 - l is below this
constexpr double kMsvtInvTail = 1.0e-10;  // the inverse square root phase likewise
constexpr double kMsvtKappa = 8.0;       // assumed ratio of the norm bound alpha to lambda_max
constexpr int kMsvtMaxSteps = 64;

typedef double d4_t __attribute__((ext_vector_type(4)));

// Scalars kept on the device (doubles in the workspace).
enum { SC_ALPHA = 0, SC_TRACE, SC_BETA, SC_CF, SC_COUNT };

// Coefficients of the scaled Newton-Schulz steps for moduli in [l0, 1], until 1 - l < tail.
int ns_schedule(double l0, double tail, double* a, int cap) {
  double l = std::min(std::max(l0, 1e-300), 1.0);
  int k = 0;
  while (k < cap) {
    const double ak = std::sqrt(3.0 / (1.0 + l + l * l));
    a[k++] = ak;
    l = 0.5 * ak * l * (3.0 - ak * ak * l * l);
    if (1.0 - l < tail) break;
  }
  return k;
}

// One product term of a launch: C = ca * s * (A B) + ce * E + ci * I, with s = *sp when sp
// is non-null (a scale computed on the device), N x N row-major, ld N.
struct MmOp {
  const double* A;
  const double* B;
  double* C;
  const double* E;
  const double* sp;
  double ca, ce, ci;
  int sym;   // the result is symmetric: upper tiles only, each written to both triangles
  int at;    // A is exactly symmetric: read as A[k][i] (coalesced like B)
};

// Output tiles of one product: all nt^2, or the nt (nt + 1) / 2 upper ones when the
// result is symmetric.
__host__ __device__ inline int ms_tiles(int nt, int sym) { return sym ? nt * (nt + 1) / 2 : nt * nt; }

// Blocks [0, tiles(o0)) compute o0, the next tiles(o1) blocks o1 (when two products are
// independent they share one launch).  One 16 x 16 output tile per block; the four waves
// take a quarter of K each with their MFMA operands loaded straight into registers
// (v_mfma_f64_16x16x4f64: lane l holds A[l % 16][k + l / 16] and B[k + l / 16][l % 16]),
// two accumulator chains each; partial tiles are summed in LDS.  An exactly symmetric A
// (a product written with sym set, or a symmetrised input) is read as A[k][i], each load
// then covering four 128-byte rows as B's do.  The sign phase's results, symmetric in
// exact arithmetic, are computed on the upper tiles and written to both triangles, which
// keeps them exactly symmetric for the next product.  The coupled inverse square root
// iteration must not be symmetrised that way (forcing Y T and T Z symmetric breaks the
// relation between its two sequences, and the iteration then diverges on Grams of
// condition number above about 1e5), so its products are computed in full.  The
// products are N <= 512 wide and one dependent chain: load latency, not MFMA
// throughput, bounds them.
__global__ void __launch_bounds__(256) k_ms_mm(int N, MmOp o0, MmOp o1) {
  __shared__ double red[4][256];
  const int nt = N / 16;
  const int t0 = ms_tiles(nt, o0.sym);
  const int b = blockIdx.x;
  const MmOp& o = b < t0 ? o0 : o1;
  int tile = b < t0 ? b : b - t0;
  int ti, tj;
  if (o.sym) {   // upper tile number -> (ti, tj), ti <= tj, row by row
    ti = 0;
    while (tile >= nt - ti) {
      tile -= nt - ti;
      ++ti;
    }
    tj = ti + tile;
  } else {
    ti = tile / nt;
    tj = tile % nt;
  }
  const int i0 = ti * 16, j0 = tj * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int kw = N / 4, kb = wave * kw;   // kw is a multiple of 16 (N % 64 == 0)
  d4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  // A[i][k] at Ar[k] (rows), or A[k][i] at Ac[k N] (exactly symmetric A)
  const double* Ar = o.A + (size_t)(i0 + li) * N + kb + lk;
  const double* Ac = o.A + (size_t)(kb + lk) * N + i0 + li;
  const double* Bc = o.B + (size_t)(kb + lk) * N + j0 + li;
  const size_t astride = o.at ? (size_t)N : 1;
  const double* Ap = o.at ? Ac : Ar;
  for (int k0 = 0; k0 < kw; k0 += 64) {
    double a[16], bb[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = k0 + 4 * s;
      const bool in = k < kw;
      a[s] = in ? Ap[(size_t)k * astride] : 0.0;
      bb[s] = in ? Bc[(size_t)k * N] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 16; s += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bb[s], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s + 1], bb[s + 1], acc1, 0, 0, 0);
    }
  }
  // output register v of lane l: row 4 v + l / 16, column l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][(4 * v + lk) * 16 + li] = acc0[v] + acc1[v];
  __syncthreads();
  const int r = tid / 16, c = tid % 16;
  const int gi = i0 + r, gj = j0 + c;
  if (o.sym && ti == tj && r > c) return;   // the diagonal tile's upper triangle is written twice
  const size_t off = (size_t)gi * N + gj;
  const double scale = o.sp ? *o.sp : 1.0;
  double v = o.ca * scale * ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]));
  if (o.E) v = fma(o.ce, o.E[off], v);
  if (gi == gj) v += o.ci;
  o.C[off] = v;
  if (o.sym) o.C[(size_t)gj * N + gi] = v;
}

// Row statistics of A = G - t I over the padded N x N matrix (G zero beyond n_H, and
// A_ii = -t there): rs[3 i] = sum_j |A_ij|, rs[3 i + 1] = sum_j A_ij^2, rs[3 i + 2] = G_ii.
// Called with t = 0 and n_H = N on Gt: the statistics of Gt.  One wave per row.
__global__ void __launch_bounds__(256) k_ms_rowstats(int N, int nH, const double* __restrict__ G, int ldg, double t,
                                                     double* __restrict__ rs) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  double sa = 0.0, sq = 0.0, gd = 0.0;
  for (int j = lane; j < N; j += 64) {
    const double g = (i < nH && j < nH) ? G[(size_t)i * ldg + j] : 0.0;
    const double x = g - (i == j ? t : 0.0);
    sa += fabs(x);
    sq += x * x;
    if (i == j) gd = g;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sa += __shfl_xor(sa, o);
    sq += __shfl_xor(sq, o);
    gd += __shfl_xor(gd, o);
  }
  if (lane == 0) {
    rs[3 * i] = sa;
    rs[3 * i + 1] = sq;
    rs[3 * i + 2] = gd;
  }
}

// Norm bound min(max_i sum_j |A_ij|, ||A||_F) >= ||A||_2 (A symmetric) and trace of G
// from the row statistics, by every block (N <= 1024 values); block 0 stores them.
__device__ void ms_bounds(int N, const double* __restrict__ rs, double* red, double& bound, double& trace) {
  const int tid = threadIdx.x;
  double mx = 0.0, fr = 0.0, tr = 0.0;
  for (int i = tid; i < N; i += blockDim.x) {
    mx = fmax(mx, rs[3 * i]);
    fr += rs[3 * i + 1];
    tr += rs[3 * i + 2];
  }
  red[tid] = mx;
  red[256 + tid] = fr;
  red[512 + tid] = tr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[tid] = fmax(red[tid], red[tid + w]);
      red[256 + tid] += red[256 + tid + w];
      red[512 + tid] += red[512 + tid + w];
    }
    __syncthreads();
  }
  bound = fmin(red[0], sqrt(red[256]));
  trace = red[512];
}

// A (N x N) = G - t I (padded), X = A / alpha, alpha = the norm bound (at least t, so a
// zero G still scales to -I); block 0 stores alpha and trace(G), and sets flag to 1 when
// alpha exceeds alpha_cap (the bound the host's step count assumed), else to 0.
__global__ void __launch_bounds__(256) k_ms_scale(int N, int nH, const double* __restrict__ G, int ldg, double t,
                                                  const double* __restrict__ rs, double alpha_cap,
                                                  double* __restrict__ A, double* __restrict__ X,
                                                  double* __restrict__ sc, int* __restrict__ flag) {
  __shared__ double red[768];
  double bound, trace;
  ms_bounds(N, rs, red, bound, trace);
  const double alpha = fmax(bound, t) * (1.0 + 1e-12);   // above rounding in the bound
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[SC_ALPHA] = alpha;
    sc[SC_TRACE] = trace;
    *flag = alpha > alpha_cap ? 1 : 0;   // first writer of the SVT's flag
  }
  const double inv = 1.0 / alpha;
  const size_t total = (size_t)N * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    // symmetrised: the Gram of the coarse data is symmetric up to the rounding of C G C
    const double g = (i < nH && j < nH) ? 0.5 * (G[(size_t)i * ldg + j] + G[(size_t)j * ldg + i]) : 0.0;
    const double x = g - (i == j ? t : 0.0);
    A[e] = x;
    X[e] = x * inv;
  }
}

// Y = (Gt + Gt^T) / (2 beta), T = c1 I + c2 Y (the first coupled step, Z = I), beta = the
// norm bound of Gt (at least t); block 0 stores beta and beta^{-1/2}.  flag |= 2 when beta
// exceeds beta_cap.
__global__ void __launch_bounds__(256) k_ms_ystart(int N, const double* __restrict__ Gt, const double* __restrict__ rs,
                                                   double t, double beta_cap, double c1, double c2,
                                                   double* __restrict__ Y, double* __restrict__ T,
                                                   double* __restrict__ sc, int* __restrict__ flag) {
  __shared__ double red[768];
  double bound, trace;
  ms_bounds(N, rs, red, bound, trace);
  const double beta = fmax(bound, t) * (1.0 + 1e-12);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[SC_BETA] = beta;
    sc[SC_CF] = 1.0 / sqrt(beta);
    if (beta > beta_cap) *flag |= 2;
  }
  const double inv = 0.5 / beta;
  const size_t total = (size_t)N * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    const double y = (Gt[e] + Gt[(size_t)j * N + i]) * inv;
    Y[e] = y;
    T[e] = c2 * y + (i == j ? c1 : 0.0);
  }
}

// K (ld ldk, n_H x n_H block, zero beyond) = I - tau beta^{-1/2} Z (the plain method).
__global__ void k_ms_plain_K(int N, int nH, const double* __restrict__ Z, const double* __restrict__ sc, double tau,
                             double* __restrict__ K, int ldk) {
  const double cf = tau * sc[SC_CF];
  const size_t total = (size_t)N * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    double v = 0.0;
    if (i < nH && j < nH) v = (i == j ? 1.0 : 0.0) - cf * Z[e];
    K[(size_t)i * ldk + j] = v;
  }
}

// Cp (N x N) = C zero-padded and symmetrised (C: n_H x n_H, ld n_H, symmetric up to the
// rounding of its construction).
__global__ void k_ms_padC(int N, int nH, const double* __restrict__ C, double* __restrict__ Cp) {
  const size_t total = (size_t)N * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    Cp[e] = (i < nH && j < nH) ? 0.5 * (C[(size_t)i * nH + j] + C[(size_t)j * nH + i]) : 0.0;
  }
}

// Statistics of the result: rank = (N + trace S) / 2 rounded, the trace of G, the
// factor form flag, no margin (the path does not resolve individual values).
__global__ void k_ms_stats(int N, const double* __restrict__ S, const double* __restrict__ sc,
                           const int* __restrict__ flag, IterStats* __restrict__ st) {
  __shared__ double red[256];
  double tr = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) tr += S[(size_t)i * N + i];
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int r = (int)floor(0.5 * ((double)N + red[0]) + 0.5);
    st->rank = min(max(r, 0), N);
    st->margin = -1.0;
    st->trace = sc[SC_TRACE];
    st->lam_r = 0.0;
    st->lam_65 = 0.0;
    st->kform = 1;
    st->msvt_flag = *flag;
    st->msvt_alpha = sc[SC_ALPHA];
    st->msvt_beta = sc[SC_BETA];
  }
}

// Rank-0 certificate by Gershgorin discs: rs[3 i] = sum_j |G_ij| (row statistics with
// t = 0); every eigenvalue of G is below t when every such sum is (G_ii >= 0).  pr[0] =
// 1 when certified, pr[1] = the largest row sum, pr[2] = trace G; when certified, st
// takes rank 0 in factor form and the margin (tau - sqrt(max sum)) / tau.
__global__ void __launch_bounds__(256) k_ms_probe(int N, const double* __restrict__ rs, double t, double tau,
                                                  double* __restrict__ pr, IterStats* __restrict__ st,
                                                  ProbeRecord* pub, unsigned long long seq) {
  __shared__ double red[768];
  double bound, trace;
  ms_bounds(N, rs, red, bound, trace);   // bound = min(max row sum, ||G||_F)
  if (threadIdx.x == 0) {
    const double gmax = red[0];
    const bool cert = gmax < t;
    pr[0] = cert ? 1.0 : 0.0;
    pr[1] = gmax;
    pr[2] = trace;
    if (cert) {
      st->rank = 0;
      st->kform = 0;
      st->margin = (tau - sqrt(gmax)) / tau;
      st->trace = trace;
      st->lam_r = 0.0;
      st->lam_65 = 0.0;
      st->msvt_flag = 0;
    }
    if (pub) {   // the same three values for the host, the sequence number last
      pub->v[0] = pr[0];
      pub->v[1] = gmax;
      pub->v[2] = trace;
      __threadfence_system();
      *reinterpret_cast<volatile unsigned long long*>(&pub->seq) = seq;
    }
  }
}

struct MsLayout {
  size_t off_A, off_X0, off_X1, off_P, off_Y0, off_Y1, off_Z0, off_Z1, off_T, off_Cp, off_C2, off_rs, off_sc,
      off_flag, off_probe, total;
};

MsLayout ms_layout(int N) {
  MsLayout l;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += align256(b);
    return o;
  };
  const size_t sq = (size_t)N * N * sizeof(double);
  l.off_A = take(sq);
  l.off_X0 = take(sq);
  l.off_X1 = take(sq);
  l.off_P = take(sq);
  l.off_Y0 = take(sq);
  l.off_Y1 = take(sq);
  l.off_Z0 = take(sq);
  l.off_Z1 = take(sq);
  l.off_T = take(sq);
  l.off_Cp = take(sq);
  l.off_C2 = take(sq);
  l.off_rs = take((size_t)3 * N * sizeof(double));
  l.off_sc = take(SC_COUNT * sizeof(double));
  l.off_flag = take(sizeof(int));
  l.off_probe = take(4 * sizeof(double));
  l.total = off;
  return l;
}

// Product term; sym: symmetric result (upper tiles, mirrored), at: A exactly symmetric.
MmOp mm(int sym, int at, const double* A, const double* B, double* C, double ca = 1.0, const double* E = nullptr,
        double ce = 0.0, double ci = 0.0, const double* sp = nullptr) {
  MmOp o;
  o.sym = sym;
  o.at = at;
  o.A = A;
  o.B = B;
  o.C = C;
  o.E = E;
  o.sp = sp;
  o.ca = ca;
  o.ce = ce;
  o.ci = ci;
  return o;
}

int launch_mm(int N, const MmOp& o0, const MmOp* o1, hipStream_t s, int* count) {
  const int nt = N / 16;
  const int blocks = ms_tiles(nt, o0.sym) + (o1 ? ms_tiles(nt, o1->sym) : 0);
  ProfKernel pk(KC_MSVT);
  hipExtLaunchKernelGGL(k_ms_mm, dim3(blocks), dim3(256), 0, s, pk.start, pk.stop, 0, N, o0, o1 ? *o1 : o0);
  MLPCP_HIP(hipGetLastError());
  *count += o1 ? 2 : 1;
  return MLPCP_OK;
}

int elem_grid(int N) { return std::min(1024, std::max(1, N * N / 1024)); }

}  // namespace

bool msvt_eligible(int N) { return N % 64 == 0 && N >= 128 && N <= kMsvtMaxWidth; }

size_t msvt_workspace_bytes(int N) { return ms_layout(N).total; }

int msvt_plan(double tau, double alpha_est, double beta_est, MsvtPlan* mp) {
  const double t = tau * tau;
  if (!(t > 0.0) || !(alpha_est > 0.0) || !(beta_est > 0.0)) return MLPCP_E_INVALID_ARG;
  mp->alpha_cap = std::max(alpha_est, t);
  mp->beta_cap = std::max(beta_est, t);
  // resolution l0 alpha in eigenvalue units: the error bound of the file header (with
  // lambda_max >= alpha / kappa), and at most kMsvtRankRes tau^2
  const double l0 = std::min({0.1, 2.0 * kMsvtTarget * std::sqrt(t / (kMsvtKappa * mp->alpha_cap)),
                              kMsvtRankRes * t / mp->alpha_cap});
  mp->n_sign = ns_schedule(l0, kMsvtSignTail, mp->a_sign, kMsvtMaxSteps);
  // Gt >= tau^2 / 2: a partly resolved eigenvalue l < tau^2 keeps the sign of l - tau^2
  // (the iteration's polynomials are odd and positive on (0, 1]), so its value s in
  // (-1, 0] gives tau^2 + (1 + s)(l - tau^2) / 2 >= (tau^2 + l) / 2
  const double l1 = std::min(0.999, 0.999 * std::sqrt(0.5 * t / mp->beta_cap));
  mp->n_inv = ns_schedule(l1, kMsvtInvTail, mp->a_inv, kMsvtMaxSteps);
  return MLPCP_OK;
}

int msvt_cgc(int nH, int N, const double* G, const double* C, bool prep, double* GH, void* ws, hipStream_t s,
             int* products) {
  if (!msvt_eligible(N) || nH < 1 || nH > N || !C) return MLPCP_E_INVALID_ARG;
  const MsLayout l = ms_layout(N);
  char* base = static_cast<char*>(ws);
  auto at = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  double* Cp = at(l.off_Cp);
  double* C2 = at(l.off_C2);
  double* T = at(l.off_T);
  int np = 0;
  if (prep) {
    {
      ProfScope ps(KC_SVT, s);
      hipLaunchKernelGGL(k_ms_padC, dim3(elem_grid(N)), dim3(256), 0, s, N, nH, C, Cp);
    }
    MLPCP_TRY(launch_mm(N, mm(1, 1, Cp, Cp, C2), nullptr, s, &np));
  }
  // G is an exactly symmetric Gram (its lower triangle mirrored from the upper one)
  MLPCP_TRY(launch_mm(N, mm(0, 1, G, Cp, T), nullptr, s, &np));
  MLPCP_TRY(launch_mm(N, mm(1, 1, Cp, T, GH), nullptr, s, &np));
  if (products) *products += np;
  return MLPCP_OK;
}

int msvt_probe(int nH, int N, const double* G, int ldg, double tau, IterStats* st, void* ws, hipStream_t s,
               bool* certified, double* gmax, double* trace, ProbeRecord* pub_host, ProbeRecord* pub_dev,
               unsigned long long seq) {
  if (!msvt_eligible(N) || nH < 1 || nH > N || ldg < nH) return MLPCP_E_INVALID_ARG;
  const MsLayout l = ms_layout(N);
  char* base = static_cast<char*>(ws);
  double* rs = reinterpret_cast<double*>(base + l.off_rs);
  double* pr = reinterpret_cast<double*>(base + l.off_probe);
  {
    ProfScope ps(KC_SVT, s);
    hipLaunchKernelGGL(k_ms_rowstats, dim3((N + 3) / 4), dim3(256), 0, s, N, nH, G, ldg, 0.0, rs);
    hipLaunchKernelGGL(k_ms_probe, dim3(1), dim3(256), 0, s, N, rs, tau * tau, tau, pr, st,
                       pub_host ? pub_dev : nullptr, seq);
  }
  MLPCP_HIP(hipGetLastError());
  double h[3];
  if (pub_host) {   // published to host memory: no copy, no stream synchronisation
    MLPCP_TRY(wait_seq(&pub_host->seq, seq, s));
    for (int i = 0; i < 3; ++i) h[i] = pub_host->v[i];
  } else {
    MLPCP_HIP(hipMemcpyAsync(h, pr, sizeof(h), hipMemcpyDeviceToHost, s));
    MLPCP_HIP(hipStreamSynchronize(s));
  }
  *certified = h[0] != 0.0;
  *gmax = h[1];
  *trace = h[2];
  return MLPCP_OK;
}

int svt_msvt(int nH, int N, const double* G, int ldg, double tau, const double* C, bool prep, const MsvtPlan& mp,
             double* K, int ldk, IterStats* st, void* ws, hipStream_t s, int* products) {
  if (!msvt_eligible(N) || nH < 1 || nH > N || ldk != N || ldg < nH || mp.n_sign < 1 || mp.n_inv < 1 ||
      mp.n_sign > 64 || mp.n_inv > 64)
    return MLPCP_E_INVALID_ARG;
  const MsLayout l = ms_layout(N);
  char* base = static_cast<char*>(ws);
  auto at = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  double* A = at(l.off_A);
  double* X[2] = {at(l.off_X0), at(l.off_X1)};
  double* P = at(l.off_P);
  double* Y[2] = {at(l.off_Y0), at(l.off_Y1)};
  double* Z[2] = {at(l.off_Z0), at(l.off_Z1)};
  double* T = at(l.off_T);
  double* Cp = at(l.off_Cp);
  double* C2 = at(l.off_C2);
  double* rs = at(l.off_rs);
  double* sc = at(l.off_sc);
  int* flag = reinterpret_cast<int*>(base + l.off_flag);
  const double t = tau * tau;
  const int eg = elem_grid(N);
  int np = 0;
  int* cnt = &np;
  if (C && prep) {
    {
      ProfScope ps(KC_SVT, s);
      hipLaunchKernelGGL(k_ms_padC, dim3(eg), dim3(256), 0, s, N, nH, C, Cp);
    }
    MLPCP_TRY(launch_mm(N, mm(1, 1, Cp, Cp, C2), nullptr, s, cnt));
  }
  // 1. sign phase
  {
    ProfScope ps(KC_SVT, s);
    hipLaunchKernelGGL(k_ms_rowstats, dim3((N + 3) / 4), dim3(256), 0, s, N, nH, G, ldg, t, rs);
    hipLaunchKernelGGL(k_ms_scale, dim3(eg), dim3(256), 0, s, N, nH, G, ldg, t, rs, mp.alpha_cap, A, X[0], sc,
                       flag);
  }
  int cur = 0;
  for (int k = 0; k < mp.n_sign; ++k) {
    const double a = mp.a_sign[k];
    MLPCP_TRY(launch_mm(N, mm(1, 1, X[cur], X[cur], P), nullptr, s, cnt));
    MLPCP_TRY(launch_mm(N, mm(1, 1, X[cur], P, X[cur ^ 1], -0.5 * a * a * a, X[cur], 1.5 * a), nullptr, s, cnt));
    cur ^= 1;
  }
  const double* S = X[cur];
  // 2. Gt = t I + (A + S A) / 2  (into P)
  MLPCP_TRY(launch_mm(N, mm(1, 1, S, A, P, 0.5, A, 0.5, t), nullptr, s, cnt));
  // 3. inverse square root phase: Y = Gt / beta, Z = I; first step T = c1 I + c2 Y
  {
    ProfScope ps(KC_SVT, s);
    hipLaunchKernelGGL(k_ms_rowstats, dim3((N + 3) / 4), dim3(256), 0, s, N, N, P, N, 0.0, rs);
    const double a = mp.a_inv[0];
    hipLaunchKernelGGL(k_ms_ystart, dim3(eg), dim3(256), 0, s, N, P, rs, t, mp.beta_cap, 1.5 * a,
                       -0.5 * a * a * a, Y[0], Z[0], sc, flag);
  }
  // Z_1 = T (in Z[0]); Y_1 = Y_0 T
  int yc = 0, zc = 0;
  if (mp.n_inv > 1) {
    MLPCP_TRY(launch_mm(N, mm(0, 1, Y[0], Z[0], Y[1]), nullptr, s, cnt));
    yc = 1;
  }
  for (int k = 1; k < mp.n_inv; ++k) {
    const double a = mp.a_inv[k];
    // T = c1 I + c2 Z Y
    MLPCP_TRY(launch_mm(N, mm(0, 0, Z[zc], Y[yc], T, -0.5 * a * a * a, nullptr, 0.0, 1.5 * a), nullptr, s, cnt));
    const MmOp oz = mm(0, 0, T, Z[zc], Z[zc ^ 1]);
    if (k + 1 < mp.n_inv) {
      const MmOp oy = mm(0, 0, Y[yc], T, Y[yc ^ 1]);
      MLPCP_TRY(launch_mm(N, oz, &oy, s, cnt));
      yc ^= 1;
    } else {
      MLPCP_TRY(launch_mm(N, oz, nullptr, s, cnt));
    }
    zc ^= 1;
  }
  const double* Zf = Z[zc];
  // 4. K = C (I - tau beta^{-1/2} Z) C = C^2 - tau beta^{-1/2} C (Z C)
  if (C) {
    // Cp and C2 are zero beyond n_H, so K is too
    MLPCP_TRY(launch_mm(N, mm(0, 0, Zf, Cp, T), nullptr, s, cnt));
    MLPCP_TRY(launch_mm(N, mm(1, 1, Cp, T, K, -tau, C2, 1.0, 0.0, sc + SC_CF), nullptr, s, cnt));
  }
  {
    ProfScope ps(KC_SVT, s);
    if (!C) hipLaunchKernelGGL(k_ms_plain_K, dim3(eg), dim3(256), 0, s, N, nH, Zf, sc, tau, K, ldk);
    hipLaunchKernelGGL(k_ms_stats, dim3(1), dim3(256), 0, s, N, S, sc, flag, st);
  }
  MLPCP_HIP(hipGetLastError());
  if (products) *products += np;
  return MLPCP_OK;
}

}  // namespace mlpcp
