// Symmetric eigensolver in float64 for the coarse Gram matrix (the SVD of the
// coarse data in Alg. 4 is taken as the eigendecomposition of its Gram matrix).
//
// Method: parallel two-sided cyclic Jacobi (Golub & Van Loan, sec. 8.5), blocked.
//  * Indices are grouped into blocks of b = 32.  An outer sweep visits every pair of
//    blocks once, in round-robin order (circle method: block 0 fixed, the others
//    rotating), so each outer round holds nb/2 disjoint block pairs (I, J).
//  * For each pair the 2b x 2b principal submatrix is loaded into LDS and rotated by
//    the cross pairs (p in I, q in J) in b rounds of b disjoint rotations
//    (p_i, q_{(i+s) mod b}); in the first outer round of a sweep the pairs inside
//    I and inside J are rotated first (b-1 rounds).  So one sweep visits every
//    off-diagonal position once in N-1 sequential rounds.  The product of the
//    rotations is the pair's orthogonal factor Q (2b x 2b).
//  * The outer round's transformation J = diag(Q_pair) is then applied tile by tile
//    on MFMA: A[Pa,Pb] <- Q_a^T A[Pa,Pb] Q_b (tiles with a <= b, mirrored), and
//    V[:,Pb] <- V[:,Pb] Q_b.  Tiles are disjoint, so the update is in place.
//  * A sweep starts only if some pair passes the rotation test (a sweep in which no
//    pair passes it rotates nothing), and a block pair with nothing to rotate is
//    skipped, its factor marked as the identity.
//  * Optional warm start: with V0 given, the iteration starts from A = V0^T A V0,
//    V = V0 (the previous solver iteration's eigenvectors).
//  * Optional threshold certificate (for the SVT, where only eigenvalues above a
//    threshold tau^2 matter): at the start of every sweep the Gershgorin bound
//    g_i = sum_j |a_ij| of every row is formed, and row i is certified if g_i < tau^2.
//    - If every row is certified, every eigenvalue lies below tau^2, the SVT of the
//      matrix is zero whatever its eigenvectors, and the iteration stops there.
//    - Partial form (N >= kCertPartialMin): pairs of two certified indices are not
//      rotated in the sweep, and convergence is declared when no other pair passes
//      the rotation test, the certified set taken from the final matrix.  Then the
//      certified principal block has all its eigenvalues below tau^2 (Gershgorin on
//      that block) and its coupling to the rest is below the rotation threshold, so it
//      maps to zero under the SVT whatever its basis; its diagonal entries (each below
//      tau^2) are returned as they are.
//    The partial form leaves work to later solves of a warm-started sequence (whose
//    threshold falls, so indices leave the certified set); it pays where the outer
//    rounds are bound by the number of tiles to update, which certified block pairs
//    skip (wide matrices: more apply tiles than compute units), and not where they are
//    bound by latency, where only the number of sweeps counts.
//  Problems of width 64 are solved by one kernel directly.
//  Rotation threshold (relative, Demmel-Veselic style, with an absolute floor for
//  singular Grams and for the rounding the tile products leave): rotate (p,q) iff
//  a_pq^2 > (1e-12)^2 |a_pp a_qq| (kRelEps2) and |a_pq| > 1e-14 trace(A) (kAbsTol).
#include "common.h"
#include "profile.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

namespace mlpcp {

namespace {

constexpr int IB = kEigBlock;       // 32
constexpr int IN = kEigInner;       // 64
constexpr int LDS_LD = IN + 1;
// Relative rotation threshold (squared).  An entry left at eps sqrt(a_pp a_qq) moves
// the eigenvalues by O(eps^2) and the eigenvectors by eps over the relative gap; the
// reconstruction is float32, so eps = 1e-12 leaves far more accuracy than the result
// carries, and it saves the last sweep of the quadratic convergence (the one that
// takes the off-diagonal from ~1e-8 to ~1e-16).
constexpr double kRelEps2 = 1.0e-24;  // (1e-12)^2
// Absolute rotation floor, relative to trace(A): an off-diagonal entry below it moves
// an eigenvalue by less than that share of the trace and the reconstruction
// L = M_P C V diag(w) V^T C by a comparable share of its norm, far below float32
// resolution; it stops sweeps that would only refine eigenvectors of clusters of
// tiny eigenvalues to their own relative precision.
constexpr double kAbsTol = 1.0e-14;
// Perturbative path of the one-workgroup SVT: accepted when every off-diagonal entry of
// the warm-started H is below kDkMaxCoupling sqrt(h_ii h_jj) (the neglected third-order
// terms are then of relative size about kDkMaxCoupling^3); divided differences use the
// derivative form for centres closer than kDkClose relative.
constexpr double kDkMaxCoupling = 2.0e-3;
constexpr double kDkClose = 1.0e-6;
// Widths from which the threshold certificate takes its partial form: at N = 1024 an
// outer round updates 120 + 256 tiles, more than the 256 compute units take at once.
constexpr int kCertPartialMin = 1024;

typedef double d4_t __attribute__((ext_vector_type(4)));

// circle method: position i of `players` (even) in round r, player 0 fixed
__device__ __forceinline__ int rr_player(int i, int r, int players) {
  return i == 0 ? 0 : 1 + ((i - 1 + r) % (players - 1));
}

__device__ __forceinline__ void rr_pair(int k, int r, int players, int& a, int& b) {
  const int x = rr_player(k, r, players);
  const int y = rr_player(players - 1 - k, r, players);
  a = x < y ? x : y;
  b = x < y ? y : x;
}

// rotation i of inner round s.  phase 0: pairs inside each half (b-player round robin
// on each half, b-1 rounds); phase 1: cross pairs (i, b + (i+s) mod b), b rounds.
__device__ __forceinline__ void inner_pair(int phase, int s, int i, int& p, int& q) {
  if (phase == 0) {
    const int h = i / (IB / 2), k = i % (IB / 2);
    int x, y;
    rr_pair(k, s, IB, x, y);
    p = h * IB + x;
    q = h * IB + y;
  } else {
    p = i;
    q = IB + ((i + s) & (IB - 1));
  }
}

// Jacobi rotation annihilating a_pq of [[app, apq], [apq, aqq]]:
//   [c s; -s c]^T A [c s; -s c] diagonal, t = s/c the root of smaller magnitude of
//   t^2 + 2 theta t - 1 = 0, theta = (aqq - app)/(2 apq), written without theta:
//   t = sign(d) 2 apq / (|d| + r), r = sqrt(d^2 + 4 apq^2), d = aqq - app.
// With u = |d| + r, 1 + t^2 = 2 r / u, so c^2 = u / (2 r), and with y = 1/r and
// w = 1/c:  s = sign(d) apq y w,  t = sign(d) apq y w^2.  That takes two reciprocal
// square roots (of r^2 and of c^2) and no division.  Each is the hardware estimate
// (relative error ~2^-24 on gfx950) refined by one third-order step,
// y (1 + e/2 + 3 e^2 / 8) with e = 1 - x y^2, whose truncation error is O(e^3): the
// results stay within a few units of the last place, so c^2 + s^2 = 1 holds to that
// accuracy, which keeps the accumulated factor orthogonal.  The rounds of the Jacobi
// kernels are a dependent chain through this computation.
__device__ __forceinline__ double rsq_refined(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}
__device__ __forceinline__ bool rotation_fast(double app, double aqq, double apq, double floor_abs, double& c,
                                              double& s, double& t) {
  const double a2 = apq * apq;
  if (!(fabs(apq) > floor_abs && a2 > kRelEps2 * fabs(app * aqq))) {
    c = 1.0;
    s = 0.0;
    t = 0.0;
    return false;
  }
  const double d = aqq - app;
  const double r2 = fma(d, d, 4.0 * a2);
  const double y = rsq_refined(r2);                 // 1 / r
  const double u = fma(r2, y, fabs(d));             // |d| + r
  const double z = (0.5 * u) * y;                   // c^2, in [1/2, 1]
  const double w = rsq_refined(z);                  // 1 / c
  const double ay = (d < 0.0 ? -apq : apq) * y;
  c = z * w;
  s = ay * w;
  t = s * w;
  return true;
}

__device__ __forceinline__ bool rotates(double app, double aqq, double apq, double floor_abs) {
  return fabs(apq) > floor_abs && apq * apq > kRelEps2 * fabs(app * aqq);
}

struct RotShared {
  double2 cs[2][IB];         // (c, s) of each rotation of the round (two buffers, by round parity)
  double t[IB];
  unsigned long long cert;   // bit l: local index l certified (partial certificate)
  int any;
};

// One phase (rounds of IB rotations) on the IN x IN matrix in LDS, accumulating
// Q <- Q J.  256 threads.  Sets rs.any if something rotated.  A skipped rotation is
// the identity (c = 1, s = t = 0), so every update below is applied unconditionally
// (exact for skipped pairs); all loads of a thread's items are issued before any of
// its stores (the items are disjoint), which keeps the LDS latency off the critical
// path.
template <int THREADS>
__device__ __forceinline__ void inner_phase(double (*A)[LDS_LD], double (*Q)[LDS_LD], int phase, double floor_abs,
                                            RotShared& rs) {
  const int tid = threadIdx.x;
  const int rounds = phase == 0 ? IB - 1 : IB;
  constexpr int NT = (IB * IB) / THREADS;   // 2x2 tiles per thread
  constexpr int NQ = (IN * IB) / THREADS;   // (row, pair) items of Q per thread
  for (int s = 0; s < rounds; ++s) {
    if (tid < IB) {
      int p, q;
      inner_pair(phase, s, tid, p, q);
      double c, sn, t;
      // two certified indices: not rotated (an infinite floor fails the test)
      const bool both = ((rs.cert >> p) & (rs.cert >> q) & 1ull) != 0;
      const bool on = rotation_fast(A[p][p], A[q][q], A[p][q], both ? INFINITY : floor_abs, c, sn, t);
      rs.cs[0][tid] = make_double2(c, sn);
      rs.t[tid] = t;
      if (on) rs.any = 1;
    }
    __syncthreads();
    {
      // tiles: this thread's NT tiles share the row pair a (params loaded once)
      const int a = tid / (IB / NT);
      int pa, qa;
      inner_pair(phase, s, a, pa, qa);
      const double2 pa_ = rs.cs[0][a];
      const double ca = pa_.x, sa = pa_.y, ta = rs.t[a];
      int pb[NT], qb[NT];
      double cb[NT], sb[NT];
      double t00[NT], t01[NT], t10[NT], t11[NT];
#pragma unroll
      for (int x = 0; x < NT; ++x) {
        const int b = (tid % (IB / NT)) * NT + x;
        inner_pair(phase, s, b, pb[x], qb[x]);
        const double2 pb_ = rs.cs[0][b];
        cb[x] = pb_.x; sb[x] = pb_.y;
        t00[x] = A[pa][pb[x]]; t01[x] = A[pa][qb[x]];
        t10[x] = A[qa][pb[x]]; t11[x] = A[qa][qb[x]];
      }
      // Q items: this thread's NQ rows share the column pair b
      const int bq = tid % IB;
      int qp, qq;
      inner_pair(phase, s, bq, qp, qq);
      const double2 pq_ = rs.cs[0][bq];
      const double qc = pq_.x, qs = pq_.y;
      double qx[NQ], qy[NQ];
#pragma unroll
      for (int x = 0; x < NQ; ++x) {
        const int i = x * (THREADS / IB) + tid / IB;
        qx[x] = Q[i][qp]; qy[x] = Q[i][qq];
      }
#pragma unroll
      for (int x = 0; x < NT; ++x) {
        const double u00 = ca * t00[x] - sa * t10[x], u01 = ca * t01[x] - sa * t11[x];
        const double u10 = sa * t00[x] + ca * t10[x], u11 = sa * t01[x] + ca * t11[x];
        double n00 = u00 * cb[x] - u01 * sb[x];
        double n01 = u00 * sb[x] + u01 * cb[x];
        double n10 = u10 * cb[x] - u11 * sb[x];
        double n11 = u10 * sb[x] + u11 * cb[x];
        if (pa == pb[x]) {   // diagonal 2x2 tile: exact form of the annihilation
          n00 = t00[x] - ta * t01[x];
          n11 = t11[x] + ta * t01[x];
          n01 = ta != 0.0 ? 0.0 : t01[x];
          n10 = n01;
        }
        A[pa][pb[x]] = n00; A[pa][qb[x]] = n01;
        A[qa][pb[x]] = n10; A[qa][qb[x]] = n11;
      }
#pragma unroll
      for (int x = 0; x < NQ; ++x) {
        const int i = x * (THREADS / IB) + tid / IB;
        Q[i][qp] = qc * qx[x] - qs * qy[x];
        Q[i][qq] = qs * qx[x] + qc * qy[x];
      }
    }
    __syncthreads();
  }
}

// Phase 1 (the cross pairs (i, b + (i+s) mod b), b rounds) with the 2x2 tiles and the
// factor items in registers, for IB * IB threads.  Thread (d, c) = (tid / IB, tid % IB)
// holds, in round s, the tile of rows (a, IB + (a+s) mod IB) x columns
// (c, IB + (c+s) mod IB) of A, a = (d + c) mod IB (a skewed layout: the diagonal tiles
// a = c are the first 32 lanes of wave 0, the subdiagonal tiles (c+1, c) its other 32
// lanes), and, for the rows i in {d, IB + d}, the factor entries Q[i][c] and
// Q[i][IB + (c+s) mod IB].  From one round to the next only the J-side indices move,
// by one position: the tile's J x J entry comes from tile (a+1, c+1) = thread (d, c+1)
// and the factor's J column from (d, c+1) (the same wave: lane shuffles); the tile's J
// column comes from tile (a, c+1) = thread (d-1, c+1) and its J row from tile
// (a+1, c) = thread (d+1, c) (through LDS).
// One barrier per round: wave 0 computes the next round's rotations as soon as its own
// tiles are updated, because everything they need is in wave 0 -- a_pp and a_qq of the
// diagonal tile (its own n00 and the n11 of thread (0, c+1)) and a_pq = a_{p_c, q_c(s+1)},
// which by symmetry is the n10 of the subdiagonal tile (c+1, c), thread (1, c).  The
// other waves meanwhile apply the current round, so the rotation chain overlaps their
// updates; rotation parameters and exchanged entries alternate between two buffers by
// round parity.  The arithmetic per tile is that of inner_phase; A and Q enter and leave
// in LDS (A serves as the exchange buffer in between).
__device__ __forceinline__ void cross_phase_regs(double (*A)[LDS_LD], double (*Q)[LDS_LD], double floor_abs,
                                                 RotShared& rs) {
  static_assert(IB == 32 && IN == 64, "lane arithmetic assumes 32 pairs, two tile rows per wave");
  static_assert(4 * IB * IB <= IN * LDS_LD, "two parities of two exchange arrays fit in the A buffer");
  const int tid = threadIdx.x, d = tid / IB, c = tid % IB;
  const int a = (d + c) & (IB - 1);
  const int lane = tid & 63;
  const int src = (lane & IB) | ((lane + 1) & (IB - 1));   // thread (d, c+1), same wave
  const int sub = IB | (lane & (IB - 1));                  // wave 0: thread (1, c)
  const bool diag = d == 0;                                 // wave 0, lanes 0..31
  const bool wave0 = tid < 64;                              // wave-uniform
  double t00 = A[a][c], t01 = A[a][IB + c], t10 = A[IB + a][c], t11 = A[IB + a][IB + c];
  double qx0 = Q[d][c], qy0 = Q[d][IB + c], qx1 = Q[IB + d][c], qy1 = Q[IB + d][IB + c];
  const unsigned long long cm = rs.cert;
  __syncthreads();   // A now serves as the exchange buffer
  double* x01 = &A[0][0];            // [parity][IB x IB by thread]: the tiles' J-column entries
  double* x10 = x01 + 2 * IB * IB;   // [parity][IB x IB by thread]: the tiles' J-row entries
  const int from01 = ((d + IB - 1) & (IB - 1)) * IB + ((c + 1) & (IB - 1));
  const int from10 = ((d + 1) & (IB - 1)) * IB + c;
  double tt = 0.0;
  auto rotate = [&](int s, int par) {   // diagonal threads: rotation c of round s
    double cc, sn;
    const int q = IB + ((c + s) & (IB - 1));
    // two certified indices: not rotated (an infinite floor fails the test)
    const bool both = ((cm >> c) & (cm >> q) & 1ull) != 0;
    if (rotation_fast(t00, t11, t01, both ? INFINITY : floor_abs, cc, sn, tt)) rs.any = 1;
    rs.cs[par][c] = make_double2(cc, sn);
  };
  if (diag) rotate(0, 0);
  __syncthreads();
  for (int s = 0;; ++s) {
    const int par = s & 1;
    const double2 pa = rs.cs[par][a], pb = rs.cs[par][c];
    const double ca = pa.x, sa = pa.y, cb = pb.x, sb = pb.y;
    const double u00 = ca * t00 - sa * t10, u01 = ca * t01 - sa * t11;
    const double u10 = sa * t00 + ca * t10, u11 = sa * t01 + ca * t11;
    double n00 = u00 * cb - u01 * sb, n01 = u00 * sb + u01 * cb;
    double n10 = u10 * cb - u11 * sb, n11 = u10 * sb + u11 * cb;
    if (diag) {   // diagonal 2x2 tile: exact form of the annihilation
      n00 = t00 - tt * t01;
      n11 = t11 + tt * t01;
      n01 = tt != 0.0 ? 0.0 : t01;
      n10 = n01;
    }
    const double m0 = cb * qx0 - sb * qy0, w0 = sb * qx0 + cb * qy0;
    const double m1 = cb * qx1 - sb * qy1, w1 = sb * qx1 + cb * qy1;
    t00 = n00;
    qx0 = m0;
    qx1 = m1;
    if (s == IB - 1) {
      t01 = n01; t10 = n10; t11 = n11;
      qy0 = w0; qy1 = w1;
      break;
    }
    double* xo01 = x01 + par * IB * IB;
    double* xo10 = x10 + par * IB * IB;
    xo01[tid] = n01;
    xo10[tid] = n10;
    t11 = __shfl(n11, src);
    qy0 = __shfl(w0, src);
    qy1 = __shfl(w1, src);
    if (wave0) {
      const double sub10 = __shfl(n10, sub);
      if (diag) {
        t01 = sub10;
        rotate(s + 1, par ^ 1);
      }
    }
    __syncthreads();
    if (!diag) t01 = xo01[from01];
    t10 = xo10[from10];
  }
  __syncthreads();   // exchange reads done: A and Q take the result (positions of round IB - 1)
  const int qa = IB + ((a + IB - 1) & (IB - 1)), qc = IB + ((c + IB - 1) & (IB - 1));
  A[a][c] = t00; A[a][qc] = t01;
  A[qa][c] = t10; A[qa][qc] = t11;
  Q[d][c] = qx0; Q[d][qc] = qy0;
  Q[IB + d][c] = qx1; Q[IB + d][qc] = qy1;
  __syncthreads();
}

// trace(A) -> floor = kAbsTol * |trace| (one block)
__global__ void k_floor(const double* __restrict__ A, int N, double* __restrict__ floor_out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) s += fabs(A[(size_t)i * N + i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) floor_out[0] = kAbsTol * red[0] + 1.0e-300;
}

// Whole problem (N == IN) in one block: full sweeps until nothing rotates.
__global__ void __launch_bounds__(256) k_jacobi_direct(double* __restrict__ A, double* __restrict__ V, int N,
                                                       const double* __restrict__ floor_p, int warm, int max_sweeps,
                                                       int* __restrict__ sweeps_out) {
  __shared__ double sA[IN][LDS_LD];
  __shared__ double sQ[IN][LDS_LD];
  __shared__ RotShared rs;
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) {
    const int i = it / IN, j = it % IN;
    sA[i][j] = A[(size_t)i * N + j];
    sQ[i][j] = warm ? V[(size_t)i * N + j] : (i == j ? 1.0 : 0.0);
  }
  const double fl = floor_p[0];
  if (threadIdx.x == 0) rs.cert = 0;
  int sweeps = 0;
  bool conv = false;
  for (; sweeps < max_sweeps; ++sweeps) {
    if (threadIdx.x == 0) rs.any = 0;
    __syncthreads();
    inner_phase<256>(sA, sQ, 0, fl, rs);
    inner_phase<256>(sA, sQ, 1, fl, rs);
    const int any = rs.any;
    __syncthreads();
    if (!any) {
      conv = true;
      break;
    }
  }
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) {
    const int i = it / IN, j = it % IN;
    A[(size_t)i * N + j] = sA[i][j];
    V[(size_t)i * N + j] = sQ[i][j];
  }
  if (threadIdx.x == 0) sweeps_out[0] = conv ? sweeps + 1 : -1;
}

__device__ __forceinline__ int pair_global(int l, int I, int J) { return l < IB ? I * IB + l : J * IB + (l - IB); }

// Outer round, step 1: one block per block pair: rotate the cross pairs (and, in the
// first round of a sweep, the pairs inside each block), write Q_pair.
// kPairThreads threads: a round is bound by LDS latency, which sixteen waves hide
// better than four (one 2x2 tile and two factor items per thread).
constexpr int kPairThreads = 1024;
static_assert(kPairThreads == IB * IB, "the cross phase keeps one 2x2 tile per thread");
// A and Aout: the matrix before and after the round (the same buffer, or, with the
// split apply step, the two buffers it alternates between; then this kernel writes
// the pair blocks of Aout, and on a round the pre-test disabled it copies all of A).
__global__ void __launch_bounds__(kPairThreads) k_jacobi_pairs(const double* A, double* Aout, int N, int nb,
                                                      int round, double* __restrict__ Qblk,
                                                      const double* __restrict__ floor_p,
                                                      const int* __restrict__ active, const double* __restrict__ gb) {
  __shared__ double sA[IN][LDS_LD];
  __shared__ double sQ[IN][LDS_LD];
  __shared__ RotShared rs;
  if (!*active) {   // the sweep's pre-test found nothing to rotate
    if (Aout != A) {
      const size_t nn = (size_t)N * N;
      for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x)
        Aout[e] = A[e];
    }
    return;
  }
  int I, J;
  rr_pair(blockIdx.x, round, nb, I, J);
  constexpr int PER = IN * IN / kPairThreads;
  double ra[PER];
#pragma unroll
  for (int x = 0; x < PER; ++x) {
    const int it = threadIdx.x + kPairThreads * x;
    ra[x] = A[(size_t)pair_global(it / IN, I, J) * N + pair_global(it % IN, I, J)];
  }
#pragma unroll
  for (int x = 0; x < PER; ++x) {
    const int it = threadIdx.x + kPairThreads * x;
    const int i = it / IN, j = it % IN;
    sA[i][j] = ra[x];
    sQ[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (threadIdx.x < 64) {   // wave 0: certified local indices (partial certificate)
    const bool c = gb != nullptr && gb[pair_global(threadIdx.x, I, J)] >= 0.0;
    const unsigned long long m = __ballot(c);
    if (threadIdx.x == 0) {
      rs.cert = m;
      rs.any = 0;
    }
  }
  __syncthreads();
  const double fl = floor_p[0];
  const unsigned long long cm = rs.cert;
  // nothing to rotate in this block pair (round 0: any pair; later rounds: the cross
  // pairs): leave A as it is and mark the factor as the identity, which the apply
  // step then neither reads nor applies
  int want = 0;
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) {
    const int i = it / IN, j = it % IN;
    const bool cand = (round == 0 ? i < j : (i < IB && j >= IB)) && !((cm >> i) & (cm >> j) & 1ull);
    if (cand && rotates(sA[i][i], sA[j][j], sA[i][j], fl)) want = 1;
  }
  if (!__syncthreads_or(want)) {
    if (threadIdx.x == 0) Qblk[(size_t)blockIdx.x * (IN * IN + 1) + IN * IN] = 0.0;
    if (Aout != A) {
#pragma unroll
      for (int x = 0; x < PER; ++x) {
        const int it = threadIdx.x + kPairThreads * x;
        Aout[(size_t)pair_global(it / IN, I, J) * N + pair_global(it % IN, I, J)] = ra[x];
      }
    }
    return;
  }
  if (round == 0) inner_phase<kPairThreads>(sA, sQ, 0, fl, rs);
  cross_phase_regs(sA, sQ, fl, rs);
  // the rotated 2b x 2b block goes straight back (annihilated entries stay exactly 0;
  // the apply step skips these diagonal tiles), and Q_pair to the workspace
  double* Qo = Qblk + (size_t)blockIdx.x * (IN * IN + 1);
#pragma unroll
  for (int x = 0; x < PER; ++x) {
    const int it = threadIdx.x + kPairThreads * x;
    const int i = it / IN, j = it % IN;
    Qo[it] = sQ[i][j];
    Aout[(size_t)pair_global(i, I, J) * N + pair_global(j, I, J)] = sA[i][j];
  }
  if (threadIdx.x == 0) Qo[IN * IN] = rs.any ? 1.0 : 0.0;   // per-pair "rotated" marker
}

// 64x64x64 product on MFMA f64 by 4 waves (each a 32x32 quadrant of 2x2 16x16 blocks):
//   out = opA(X) * Y   with opA(X)[i][k] = TRANS ? X[k][i] : X[i][k]   (X, Y in LDS)
// kmax (a multiple of 16, at most IN): rows and columns of X and Y from kmax on are zero
// (or, for the identity-padded basis, contribute nothing to the products formed here),
// so the contraction stops at kmax and output tiles from kmax on stay zero without MFMAs.
template <bool TRANS>
__device__ __forceinline__ void mm64(const double (*X)[LDS_LD], const double (*Y)[LDS_LD], d4_t acc[2][2],
                                     int kmax = IN) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = (d4_t){0.0, 0.0, 0.0, 0.0};
  if (kmax >= IN) {
#pragma unroll 4
    for (int k0 = 0; k0 < IN; k0 += 4) {
      double a[2], b[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int i = wi + bi * 16 + li;
        a[bi] = TRANS ? X[k0 + lk][i] : X[i][k0 + lk];
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) b[bj] = Y[k0 + lk][wj + bj * 16 + li];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    return;
  }
  if (wi >= kmax || wj >= kmax) return;
  for (int k0 = 0; k0 < kmax; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int i = wi + bi * 16 + li;
      a[bi] = TRANS ? X[k0 + lk][i] : X[i][k0 + lk];
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) b[bj] = Y[k0 + lk][wj + bj * 16 + li];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        if (wi + bi * 16 < kmax && wj + bj * 16 < kmax)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
}

// writes the accumulators (output layout: register v of lane l = row 4v + l/16, col l%16)
template <typename F>
__device__ __forceinline__ void mm64_store(const d4_t acc[2][2], F&& put) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) put(wi + bi * 16 + 4 * v + (lane >> 4), wj + bj * 16 + (lane & 15), acc[bi][bj][v]);
}

// Outer round, step 2: apply J.  Blocks [0, ntri) update A tiles (a < b, mirrored;
// the diagonal tiles a == b were written by the pair step); blocks
// [ntri, ntri + (N/IN)*npairs) update V tiles (IN-row chunk x pair b cols).
// Tiles whose two factors are both the identity are skipped.
__global__ void __launch_bounds__(256) k_jacobi_apply(double* __restrict__ A, double* __restrict__ V, int N, int nb,
                                                      int round, const double* __restrict__ Qblk,
                                                      const int* __restrict__ active) {
  __shared__ double sT[IN][LDS_LD];
  __shared__ double sQ[IN][LDS_LD];
  if (!*active) return;
  const int npairs = nb / 2;
  const int ntri = npairs * (npairs - 1) / 2;
  const int tid = threadIdx.x;
  int bid = blockIdx.x;
  d4_t acc[2][2];
  if (bid < ntri) {
    int a = 0, rem = bid;   // strictly upper pairs (a < b), row by row
    while (rem >= npairs - 1 - a) {
      rem -= npairs - 1 - a;
      ++a;
    }
    const int b = a + 1 + rem;
    const double* Qa = Qblk + (size_t)a * (IN * IN + 1);
    const double* Qb = Qblk + (size_t)b * (IN * IN + 1);
    const bool rot_a = Qa[IN * IN] != 0.0, rot_b = Qb[IN * IN] != 0.0;
    if (!rot_a && !rot_b) return;
    int Ia, Ja, Ib, Jb;
    rr_pair(a, round, nb, Ia, Ja);
    rr_pair(b, round, nb, Ib, Jb);
    // all global loads of the block are issued up front (tile, both factors)
    constexpr int PER = IN * IN / 256;
    double ra[PER], rqa[PER], rqb[PER];
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + 256 * x;
      const int i = it / IN, j = it % IN;
      ra[x] = A[(size_t)pair_global(i, Ia, Ja) * N + pair_global(j, Ib, Jb)];
      rqa[x] = rot_a ? Qa[it] : (i == j ? 1.0 : 0.0);
      rqb[x] = rot_b ? Qb[it] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + 256 * x;
      sT[it / IN][it % IN] = ra[x];
      sQ[it / IN][it % IN] = rqa[x];
    }
    __syncthreads();
    mm64<true>(sQ, sT, acc);   // U = Qa^T T
    __syncthreads();
    mm64_store(acc, [&](int i, int j, double v) { sT[i][j] = v; });
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + 256 * x;
      sQ[it / IN][it % IN] = rqb[x];
    }
    __syncthreads();
    mm64<false>(sT, sQ, acc);                      // T' = U Qb
    mm64_store(acc, [&](int i, int j, double v) {
      A[(size_t)pair_global(i, Ia, Ja) * N + pair_global(j, Ib, Jb)] = v;
      A[(size_t)pair_global(j, Ib, Jb) * N + pair_global(i, Ia, Ja)] = v;
    });
  } else {
    bid -= ntri;
    const int rb = bid / npairs, b = bid % npairs;
    const double* Qb = Qblk + (size_t)b * (IN * IN + 1);
    if (Qb[IN * IN] == 0.0) return;
    int Ib, Jb;
    rr_pair(b, round, nb, Ib, Jb);
    constexpr int PER = IN * IN / 256;
    double rv[PER], rq[PER];
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + 256 * x;
      rv[x] = V[(size_t)(rb * IN + it / IN) * N + pair_global(it % IN, Ib, Jb)];
      rq[x] = Qb[it];
    }
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + 256 * x;
      sT[it / IN][it % IN] = rv[x];
      sQ[it / IN][it % IN] = rq[x];
    }
    __syncthreads();
    mm64<false>(sT, sQ, acc);
    mm64_store(acc, [&](int i, int j, double v) { V[(size_t)(rb * IN + i) * N + pair_global(j, Ib, Jb)] = v; });
  }
}

// Outer round, step 2, for few tiles (N <= kSplitApplyMax): the same transformation
// spread over four blocks per tile, A out of place (A -> Aout), V in place.
//  * Off-diagonal tile pair (a < b), quadrant (hi, hj) of 32 x 32:
//      T'[hi, hj] = (Qa[:, hi]^T T) Qb[:, hj]   (T the whole 64 x 64 tile of A),
//    written to Aout at the tile's and at the mirrored position; a tile whose two
//    factors are the identity is copied.  Reading A and writing Aout keeps the four
//    blocks of a tile free of races.
//  * V tile (64-row chunk rb, pair b), quarter of 16 rows: V[rows, Pb] <- V[rows, Pb] Qb
//    (rows are independent, so in place).
// Each block does 0.75 (tile) or 0.25 (V) of a 64^3 product instead of 2 or 1: these
// rounds are few tiles on a 256-CU chip, bound by one CU's MFMA time per tile.
constexpr int kSplitApplyMax = 512;
__global__ void __launch_bounds__(256) k_jacobi_apply_split(const double* __restrict__ A, double* __restrict__ Aout,
                                                            double* __restrict__ V, int N, int nb, int round,
                                                            const double* __restrict__ Qblk,
                                                            const int* __restrict__ active) {
  __shared__ double sT[IN][LDS_LD];        // A tile, or the 16 V rows
  __shared__ double sQ[IN][LDS_LD];        // V: Qb; A tile: Qa[:, hi] in columns 0..31, Qb[:, hj] in 32..63
  __shared__ double sU[IB][LDS_LD];        // Qa[:, hi]^T T
  if (!*active) return;                    // the pair kernel copied A to Aout
  const int npairs = nb / 2;
  const int ntri = npairs * (npairs - 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int bid = blockIdx.x;
  if (bid < 4 * ntri) {
    const int quad = bid & 3, hi = quad >> 1, hj = quad & 1;
    int a = 0, rem = bid >> 2;   // strictly upper pairs (a < b), row by row
    while (rem >= npairs - 1 - a) {
      rem -= npairs - 1 - a;
      ++a;
    }
    const int b = a + 1 + rem;
    const double* Qa = Qblk + (size_t)a * (IN * IN + 1);
    const double* Qb = Qblk + (size_t)b * (IN * IN + 1);
    int Ia, Ja, Ib, Jb;
    rr_pair(a, round, nb, Ia, Ja);
    rr_pair(b, round, nb, Ib, Jb);
    // all global loads up front: the tile, both factor halves and the markers
    constexpr int PT = IN * IN / 256, PQ = IN * IB / 256;
    double rt[PT], rqa[PQ], rqb[PQ];
#pragma unroll
    for (int x = 0; x < PT; ++x) {
      const int it = tid + 256 * x;
      rt[x] = A[(size_t)pair_global(it / IN, Ia, Ja) * N + pair_global(it % IN, Ib, Jb)];
    }
#pragma unroll
    for (int x = 0; x < PQ; ++x) {
      const int it = tid + 256 * x, k = it / IB, c = it % IB;
      rqa[x] = Qa[k * IN + hi * IB + c];
      rqb[x] = Qb[k * IN + hj * IB + c];
    }
    const bool rot_a = Qa[IN * IN] != 0.0, rot_b = Qb[IN * IN] != 0.0;
    if (!rot_a && !rot_b) {   // copy the quadrant
#pragma unroll
      for (int x = 0; x < PT; ++x) {
        const int it = tid + 256 * x, i = it / IN, j = it % IN;
        if ((i >> 5) == hi && (j >> 5) == hj) {
          const int gi = pair_global(i, Ia, Ja), gj = pair_global(j, Ib, Jb);
          Aout[(size_t)gi * N + gj] = rt[x];
          Aout[(size_t)gj * N + gi] = rt[x];
        }
      }
      return;
    }
#pragma unroll
    for (int x = 0; x < PT; ++x) {
      const int it = tid + 256 * x;
      sT[it / IN][it % IN] = rt[x];
    }
#pragma unroll
    for (int x = 0; x < PQ; ++x) {
      const int it = tid + 256 * x, k = it / IB, c = it % IB;
      sQ[k][c] = rot_a ? rqa[x] : (k == hi * IB + c ? 1.0 : 0.0);
      sQ[k][IB + c] = rot_b ? rqb[x] : (k == hj * IB + c ? 1.0 : 0.0);
    }
    __syncthreads();
    // U = Qa[:, hi]^T T (32 x 64): wave w takes columns [16 w, 16 w + 16), both row blocks
    d4_t u[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll 4
    for (int k0 = 0; k0 < IN; k0 += 4) {
      const double bv = sT[k0 + lk][16 * wave + li];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
        u[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(sQ[k0 + lk][bi * 16 + li], bv, u[bi], 0, 0, 0);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) sU[bi * 16 + 4 * v + lk][16 * wave + li] = u[bi][v];
    __syncthreads();
    // T'[hi, hj] = U Qb[:, hj] (32 x 32): wave w takes the 16 x 16 block (w / 2, w % 2)
    const int bi = wave >> 1, bj = wave & 1;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < IN; k0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sU[bi * 16 + li][k0 + lk], sQ[k0 + lk][IB + bj * 16 + li], acc, 0,
                                                 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = pair_global(hi * IB + bi * 16 + 4 * v + lk, Ia, Ja);
      const int gj = pair_global(hj * IB + bj * 16 + li, Ib, Jb);
      Aout[(size_t)gi * N + gj] = acc[v];
      Aout[(size_t)gj * N + gi] = acc[v];
    }
  } else {
    bid -= 4 * ntri;
    const int qr = bid & 3;
    bid >>= 2;
    const int rb = bid / npairs, b = bid % npairs;
    const double* Qb = Qblk + (size_t)b * (IN * IN + 1);
    if (Qb[IN * IN] == 0.0) return;
    int Ib, Jb;
    rr_pair(b, round, nb, Ib, Jb);
    const int r0 = rb * IN + qr * 16;
    constexpr int PV = 16 * IN / 256, PQ = IN * IN / 256;
    double rv[PV], rq[PQ];
#pragma unroll
    for (int x = 0; x < PV; ++x) {
      const int it = tid + 256 * x;
      rv[x] = V[(size_t)(r0 + it / IN) * N + pair_global(it % IN, Ib, Jb)];
    }
#pragma unroll
    for (int x = 0; x < PQ; ++x) rq[x] = Qb[tid + 256 * x];
#pragma unroll
    for (int x = 0; x < PV; ++x) {
      const int it = tid + 256 * x;
      sT[it / IN][it % IN] = rv[x];
    }
#pragma unroll
    for (int x = 0; x < PQ; ++x) {
      const int it = tid + 256 * x;
      sQ[it / IN][it % IN] = rq[x];
    }
    __syncthreads();
    // V[r0 + 0..15, Pb] Qb: wave w takes output columns [16 w, 16 w + 16)
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < IN; k0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[li][k0 + lk], sQ[k0 + lk][16 * wave + li], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      V[(size_t)(r0 + 4 * v + lk) * N + pair_global(16 * wave + li, Ib, Jb)] = acc[v];
  }
}

// ---------------------------------------------------------------------------------
// The coarse SVT of a width-<=64 coarse model in one workgroup (the tall workloads):
// every step from the Gram to the reconstruction factors stays in LDS, and the
// Jacobi iteration runs over the n_e = n_H rounded up to even indices only (circle
// method, n_e - 1 rounds of n_e / 2 disjoint rotations per sweep).  Before each sweep
// the rotation test is evaluated on every pair; a sweep starts only if some pair
// passes it (a sweep in which no pair passes rotates nothing), so the final sweep of
// the plain iteration, which only confirms convergence, is replaced by that test.
typedef double LdsRow[LDS_LD];
// threads of the one-workgroup solver: a round of a 64-wide problem is bound by LDS
// latency, and sixteen waves hide it better than four (one 2x2 tile and two factor
// items per thread)
constexpr int kSmallThreads = 1024;


// pair k of round r of the circle method on ne players (player 0 fixed), p < q
__device__ __forceinline__ void pair_at(int ne, int k, int r, int& p, int& q) {
  const int m1 = ne - 1;
  int x = k - 1 + r;
  x = x >= m1 ? x - m1 : x;
  const int px = k == 0 ? 0 : 1 + x;
  int y = ne - 2 - k + r;
  y = y >= m1 ? y - m1 : y;
  const int py = 1 + y;
  p = min(px, py);
  q = max(px, py);
}

// Jacobi sweeps on the leading ne x ne block of A (LDS), Q <- Q J, until the rotation
// test passes for no pair (returns true) or max_sweeps sweeps ran.  cert_tau2 > 0: the
// threshold certificate of the blocked solver (at the start of each sweep; when every
// row's Gershgorin bound lies below cert_tau2 the sweeps stop with gbs[i] = the bound
// of row i, otherwise gbs[i] = -1).  ACTIVE threads
// take part in the rounds, each owning MT 2x2 tiles (pair a rows, pair b columns) and
// MQ (row, pair) items of Q for the whole iteration; the pairs' indices per round
// follow from the circle method arithmetically, so all loads of a round are issued
// at once, without branches.  Slots beyond the item counts point at the padding
// column IN of the thread's own lane row, which no result ever reads.
// WAVE: problems of width ne <= 16 run on wave 0 alone (ACTIVE = 64), synchronised at
// wavefront scope instead of by workgroup barriers (a wave's LDS accesses complete in
// issue order, so the fences only keep the compiler from reordering them); the caller
// synchronises the workgroup afterwards.
template <bool WAVE>
__device__ __forceinline__ void sweep_sync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Gate of the perturbative SVT finish on H (sA, n_H x n_H): every Gershgorin disc
// [h_i - r_i, h_i + r_i] lies above or below t2 = tau^2 and every coupling |h_ij| is below
// kDkMaxCoupling sqrt(h_i h_j).  Writes each index's class (1: disc above t2, 0: below,
// -1: straddles, or a centre not positive) to cls_out, the number above to rank, and this
// thread's term of the margin (the relative distance of its disc from tau) to mg.  Every
// thread of the block calls it.
__device__ __forceinline__ bool dk_gate(int nH, double tau, LdsRow* sA, double* cls_out, double* red, int* redi,
                                        double& mg, int& rank) {
  const int tid = threadIdx.x;
  const double t2 = tau * tau;
  double cmax = 0.0;
  int cls = 1;
  mg = 1.0e300;
  if (tid < nH) {
    const double hi = sA[tid][tid];
    double r = 0.0;
    for (int j = 0; j < nH; ++j)
      if (j != tid) {
        const double o = fabs(sA[tid][j]);
        r += o;
        const double hj = sA[j][j];
        cmax = (hi > 0.0 && hj > 0.0) ? fmax(cmax, o / sqrt(hi * hj)) : 1.0e300;
      }
    if (hi - r > t2 * (1.0 + 1.0e-12)) {
      cls = 1;
      mg = (sqrt(hi - r) - tau) / tau;
    } else if (hi + r < t2 * (1.0 - 1.0e-12) && hi > 0.0) {
      cls = 0;
      mg = (tau - sqrt(hi + r)) / tau;
    } else {
      cls = -1;
    }
    cls_out[tid] = cls;
  }
  red[tid] = (cls < 0) ? 1.0e300 : cmax;
  redi[tid] = (tid < nH && cls == 1) ? 1 : 0;
  __syncthreads();
  for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[tid] = fmax(red[tid], red[tid + w]);
      redi[tid] += redi[tid + w];
    }
    __syncthreads();
  }
  const double cm = red[0];
  rank = redi[0];
  __syncthreads();
  return cm < kDkMaxCoupling;
}

template <int ACTIVE, int MT, int MQ, bool WAVE = false>
__device__ bool small_sweeps(LdsRow* sA, LdsRow* sQ, int ne, double fl, double cert_tau2, int max_sweeps, double* pc,
                             double* ps, double* pt, double* gbs, int& sweeps, int gate_n = 0, double gate_tau = 0.0,
                             bool gate_first = false, double* gcls = nullptr, double* gred = nullptr,
                             int* gredi = nullptr, bool* gate_hit = nullptr) {
  static_assert(!WAVE || ACTIVE == 64, "the wave form runs on one wave");
  constexpr int kPadCol = IN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int np = ne / 2;
  int ta_[MT], tb_[MT], qi_[MQ], qb_[MQ];
  bool tv_[MT], qv_[MQ];
#pragma unroll
  for (int x = 0; x < MT; ++x) {
    const int e = tid + ACTIVE * x;
    tv_[x] = e < np * np;
    ta_[x] = tv_[x] ? e / np : 0;
    tb_[x] = tv_[x] ? e % np : 0;
  }
#pragma unroll
  for (int x = 0; x < MQ; ++x) {
    const int e = tid + ACTIVE * x;
    qv_[x] = e < ne * np;
    qi_[x] = qv_[x] ? e / np : lane;
    qb_[x] = qv_[x] ? e % np : 0;
  }
  for (sweeps = 0;; ++sweeps) {
    // the perturbative finish's gate (gate_n > 0; block form only), before the first
    // sweep only when gate_first: the sweeps converge quadratically, so its coupling
    // bound is met a sweep or more before the rotation test below stops them
    if (!WAVE && gate_n > 0 && (sweeps > 0 || gate_first)) {
      double mg;
      int rk;
      if (dk_gate(gate_n, gate_tau, sA, gcls, gred, gredi, mg, rk)) {
        *gate_hit = true;
        return false;
      }
    }
    if (cert_tau2 > 0.0) {
      // Gershgorin bound of each row: 16 threads per row (blockDim = 1024 covers 64 rows);
      // the wave form: 4 lanes per row (16 rows)
      constexpr int SUB = WAVE ? 4 : 16;
      const int row = tid / SUB, sub = tid % SUB;
      double g = 0.0;
      if (row < ne)
        for (int c = sub; c < ne; c += SUB) g += fabs(sA[row][c]);
      if (!WAVE) {
        g += __shfl_xor(g, 8);
        g += __shfl_xor(g, 4);
      }
      g += __shfl_xor(g, 2);
      g += __shfl_xor(g, 1);
      const bool cert = g < cert_tau2 * (1.0 - 1.0e-12);   // padding rows (zero) pass
      const bool all = WAVE ? (__all(cert) != 0) : __syncthreads_and(cert);
      if (sub == 0) gbs[row] = (all && row < ne) ? g : -1.0;
      if (all) {
        sweep_sync<WAVE>();
        return true;
      }
    }
    int want = 0;
    for (int it = tid; it < ne * ne; it += (WAVE ? 64 : (int)blockDim.x)) {
      const int i = it / ne, j = it % ne;
      if (i < j && rotates(sA[i][i], sA[j][j], sA[i][j], fl)) want = 1;
    }
    if (!(WAVE ? (__any(want) != 0) : __syncthreads_or(want))) return true;
    if (sweeps == max_sweeps) return false;
    for (int r = 0; r < ne - 1; ++r) {
      if (tid < np) {
        int p, q;
        pair_at(ne, tid, r, p, q);
        double c, sn, t;
        rotation_fast(sA[p][p], sA[q][q], sA[p][q], fl, c, sn, t);
        pc[tid] = c; ps[tid] = sn; pt[tid] = t;
      }
      sweep_sync<WAVE>();
      if (tid < ACTIVE) {
        double t00[MT], t01[MT], t10[MT], t11[MT], qx[MQ], qy[MQ];
        int rp[MT], rq[MT], cp[MT], cq[MT], qp[MQ], qq[MQ];
#pragma unroll
        for (int x = 0; x < MT; ++x) {
          pair_at(ne, ta_[x], r, rp[x], rq[x]);
          pair_at(ne, tb_[x], r, cp[x], cq[x]);
          if (!tv_[x]) {
            rp[x] = lane; rq[x] = lane;
            cp[x] = kPadCol; cq[x] = kPadCol;
          }
          t00[x] = sA[rp[x]][cp[x]]; t01[x] = sA[rp[x]][cq[x]];
          t10[x] = sA[rq[x]][cp[x]]; t11[x] = sA[rq[x]][cq[x]];
        }
#pragma unroll
        for (int x = 0; x < MQ; ++x) {
          pair_at(ne, qb_[x], r, qp[x], qq[x]);
          if (!qv_[x]) {
            qp[x] = kPadCol; qq[x] = kPadCol;
          }
          qx[x] = sQ[qi_[x]][qp[x]]; qy[x] = sQ[qi_[x]][qq[x]];
        }
#pragma unroll
        for (int x = 0; x < MT; ++x) {
          const int a = ta_[x], b = tb_[x];
          const double ca = pc[a], sa = ps[a], cb = pc[b], sb = ps[b], ta = pt[a];
          const double u00 = ca * t00[x] - sa * t10[x], u01 = ca * t01[x] - sa * t11[x];
          const double u10 = sa * t00[x] + ca * t10[x], u11 = sa * t01[x] + ca * t11[x];
          double n00 = u00 * cb - u01 * sb;
          double n01 = u00 * sb + u01 * cb;
          double n10 = u10 * cb - u11 * sb;
          double n11 = u10 * sb + u11 * cb;
          if (a == b) {   // diagonal 2x2 tile: exact form of the annihilation
            n00 = t00[x] - ta * t01[x];
            n11 = t11[x] + ta * t01[x];
            n01 = ta != 0.0 ? 0.0 : t01[x];
            n10 = n01;
          }
          sA[rp[x]][cp[x]] = n00; sA[rp[x]][cq[x]] = n01;
          sA[rq[x]][cp[x]] = n10; sA[rq[x]][cq[x]] = n11;
        }
#pragma unroll
        for (int x = 0; x < MQ; ++x) {
          const double c = pc[qb_[x]], sn = ps[qb_[x]];
          sQ[qi_[x]][qp[x]] = c * qx[x] - sn * qy[x];
          sQ[qi_[x]][qq[x]] = sn * qx[x] + c * qy[x];
        }
      }
      sweep_sync<WAVE>();
    }
  }
}

// The SVT's spectral function on one class of eigenvalues: f(x) = 1 - tau / sqrt(x) above
// tau^2, 0 below (the classes are separated by the Gershgorin test), and its first two
// derivatives.
struct SvtFn {
  double tau;
  __device__ double f(double x, bool up) const { return up ? 1.0 - tau / sqrt(x) : 0.0; }
  __device__ double d1(double x, bool up) const { return up ? 0.5 * tau / (x * sqrt(x)) : 0.0; }
  __device__ double d2(double x, bool up) const { return up ? -0.75 * tau / (x * x * sqrt(x)) : 0.0; }
  // first divided difference f[a, b] (a, b in classes ua, ub)
  __device__ double dd1(double a, bool ua, double b, bool ub) const {
    if (ua == ub && fabs(a - b) <= kDkClose * fmax(fabs(a), fabs(b))) return d1(0.5 * (a + b), ua);
    return (f(a, ua) - f(b, ub)) / (a - b);
  }
  // d/da f[a, b]
  __device__ double dd1_da(double a, bool ua, double b, bool ub) const {
    if (ua == ub && fabs(a - b) <= kDkClose * fmax(fabs(a), fabs(b))) return 0.5 * d2(a, ua);
    const double h = a - b;
    return (d1(a, ua) * h - (f(a, ua) - f(b, ub))) / (h * h);
  }
};

__global__ void __launch_bounds__(kSmallThreads) k_coarse_small(int nH, int ld, const double* __restrict__ G,
                                                      const double* __restrict__ C, double* __restrict__ V,
                                                      int warm, double tau, int certify, int max_sweeps,
                                                      double* __restrict__ lam, int* __restrict__ perm,
                                                      double* __restrict__ sw, double* __restrict__ T,
                                                      double* __restrict__ Tt, double* __restrict__ K,
                                                      IterStats* __restrict__ st) {
  extern __shared__ double dsm[];
  LdsRow* sA = reinterpret_cast<LdsRow*>(dsm);
  LdsRow* sQ = sA + IN;
  LdsRow* sC = sQ + IN;
  LdsRow* sW = sC + IN;
  __shared__ double pc[IB], ps[IB], pt[IB], swv[IN], gbs[IN], red[kSmallThreads];
  __shared__ int prm[IN], redi[kSmallThreads];
  const int tid = threadIdx.x;
  const bool mm_on = tid < 256;   // the 64^3 products run on the first four waves
  const int km = min(IN, (nH + 15) / 16 * 16);   // beyond it the operands are zero (identity in V)
  // With certify the basis kept in Q (and in V between calls) is S' = C V rather than V:
  // H = V^T (C G C) V = S'^T G S', rotations act on S' as on V, T = C V_r diag(w) =
  // S'_r diag(w) and K = S' F S'^T, so C G C and the products by C are not formed.
  const bool cb = certify != 0;
  d4_t acc[2][2];
  {
    constexpr int PER = IN * IN / kSmallThreads;
    double rg[PER], rc[PER], rv[PER];
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + kSmallThreads * x;
      const int i = it / IN, j = it % IN;
      const bool in = i < nH && j < nH;
      const double eye = i == j ? 1.0 : 0.0;
      rg[x] = in ? G[(size_t)i * ld + j] : 0.0;
      rc[x] = (C && in) ? C[(size_t)i * nH + j] : 0.0;
      if (warm)
        rv[x] = in ? V[(size_t)i * ld + j] : eye;
      else
        rv[x] = (cb && C && in) ? C[(size_t)i * nH + j] : eye;   // the C V basis starts at C
    }
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int it = tid + kSmallThreads * x;
      const int i = it / IN, j = it % IN;
      sA[i][j] = rg[x];
      sC[i][j] = rc[x];
      sQ[i][j] = rv[x];
    }
  }
  __syncthreads();
  if (C && !cb) {                            // G_H = C G C
    if (mm_on) {
      mm64<false>(sA, sC, acc, km);
      mm64_store(acc, [&](int i, int j, double v) { sW[i][j] = v; });
    }
    __syncthreads();
    if (mm_on) mm64<false>(sC, sW, acc, km);
    __syncthreads();
    if (mm_on) mm64_store(acc, [&](int i, int j, double v) { sA[i][j] = v; });
    __syncthreads();
  }
  if (warm || (cb && C)) {                   // A <- Q^T A Q (Q = V0, or S' = C V0)
    if (mm_on) {
      mm64<true>(sQ, sA, acc, km);
      mm64_store(acc, [&](int i, int j, double v) { sW[i][j] = v; });
    }
    __syncthreads();
    if (mm_on) mm64<false>(sW, sQ, acc, km);
    __syncthreads();
    if (mm_on) mm64_store(acc, [&](int i, int j, double v) { sA[i][j] = v; });
    __syncthreads();
  }
  // exact symmetry (the products above round each triangle separately)
  for (int it = tid; it < IN * IN; it += kSmallThreads) {
    const int i = it / IN, j = it % IN;
    if (i < j) {
      const double v = 0.5 * (sA[i][j] + sA[j][i]);
      sA[i][j] = v;
      sA[j][i] = v;
    }
  }
  // absolute floor of the rotation test: kAbsTol trace
  red[tid] = tid < nH ? fabs(sA[tid][tid]) : 0.0;
  if (tid < IN) gbs[tid] = -1.0;   // nothing certified unless the sweeps certify it
  __syncthreads();
  for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double fl = kAbsTol * red[0] + 1.0e-300;
  const double trace_h = red[0];
  // Perturbative path (warm start, K requested, SVT operator only).  In the previous
  // basis H = V^T G_H V is close to its diagonal D = diag(h_i): when every Gershgorin disc
  // [h_i - r_i, h_i + r_i] lies either above or below tau^2 (the rank is then the number
  // above, each class holding that many eigenvalues) and every coupling |o_ij| is below
  // kDkMaxCoupling sqrt(h_i h_j), the SVT operator f(H) (f(x) = 1 - tau / sqrt(x) above
  // tau^2, 0 below) is taken from its second-order expansion around D (Daleckii and
  // Krein's divided-difference series):
  //   f(H)_ij ~ f(h_i) [i = j] + o_ij f[h_i, h_j] + sum_k o_ik o_kj f[h_i, h_k, h_j],
  // the last term as ((A O - O A)_ij / (h_i - h_j)), A = O o f[.,.] (elementwise), and by
  // its derivative form for centres within kDkClose.  Then K = C V f(H) V^T C; T, Tt, lam,
  // perm, sw are not formed.  It is tried on the warm start and after each Jacobi sweep
  // (nsw: the sweeps run before it; their rotated basis V is the next warm start).
  auto dk_try = [&](int nsw) -> bool {
    double mg;
    int rank_dk;
    if (!dk_gate(nH, tau, sA, swv, red, redi, mg, rank_dk)) return false;
    red[tid] = mg;
    __syncthreads();
    for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] = fmin(red[tid], red[tid + w]);
      __syncthreads();
    }
    const double margin_dk = red[0];
    const SvtFn fn{tau};
    // the diagonal in gbs; O in sA (zero diagonal); A = O o f[h_i, h_j] in sC and
    // B = O o d/dh_i f[h_i, h_j] in sW (elementwise)
    if (tid < IN) gbs[tid] = tid < nH ? sA[tid][tid] : 0.0;
    __syncthreads();
    for (int it = tid; it < IN * IN; it += kSmallThreads) {
      const int i = it / IN, j = it % IN;
      double a = 0.0, b = 0.0;
      if (i < nH && j < nH && i != j) {
        const double o = sA[i][j];
        const bool ui = swv[i] > 0.5, uj = swv[j] > 0.5;
        a = o * fn.dd1(gbs[i], ui, gbs[j], uj);
        b = o * fn.dd1_da(gbs[i], ui, gbs[j], uj);
      }
      sC[i][j] = a;
      sW[i][j] = b;
    }
    __syncthreads();
    if (tid < nH) sA[tid][tid] = 0.0;
    __syncthreads();
    // P3 = B O: the second-order term in derivative form, sum_k o_ik o_kj f[h_i, h_k, h_i]
    // (the diagonal, and pairs of centres within kDkClose)
    if (mm_on) mm64<false>(sW, sA, acc, km);
    __syncthreads();
    if (mm_on) mm64_store(acc, [&](int i, int j, double v) { sW[i][j] = v; });
    __syncthreads();
    // P1 = A O (O A = P1^T: both symmetric); the second-order term elsewhere is
    // (P1 - P1^T)_ij / (h_i - h_j); P1 replaces A in sC (a_ij is recomputed from o_ij)
    if (mm_on) mm64<false>(sC, sA, acc, km);
    __syncthreads();
    if (mm_on) mm64_store(acc, [&](int i, int j, double v) { sC[i][j] = v; });
    __syncthreads();
    // F (in sW): f(h_i) [i = j] + a_ij + the second-order term
    for (int it = tid; it < IN * IN; it += kSmallThreads) {
      const int i = it / IN, j = it % IN;
      double x = 0.0;
      if (i < nH && j < nH) {
        const double hi = gbs[i], hj = gbs[j];
        const bool ui = swv[i] > 0.5, uj = swv[j] > 0.5;
        if (i == j)
          x = fn.f(hi, ui) + sW[i][j];
        else if (ui == uj && fabs(hi - hj) <= kDkClose * fmax(fabs(hi), fabs(hj)))
          x = sA[i][j] * fn.dd1(hi, ui, hj, uj) + sW[i][j];
        else
          x = sA[i][j] * fn.dd1(hi, ui, hj, uj) + (sC[i][j] - sC[j][i]) / (hi - hj);
      }
      sW[i][j] = x;   // each entry read and written by one thread
    }
    __syncthreads();
    // K = R^T (F R), R = S'^T = V^T C (Q holds S' here: the finish runs with certify)
    for (int it = tid; it < IN * IN; it += kSmallThreads) {
      const int i = it / IN, j = it % IN;
      sA[i][j] = sQ[j][i];
    }
    __syncthreads();
    if (mm_on) mm64<false>(sW, sA, acc, km);
    __syncthreads();
    if (mm_on) mm64_store(acc, [&](int i, int j, double v) { sC[i][j] = v; });
    __syncthreads();
    if (mm_on) {
      mm64<true>(sA, sC, acc, km);
      mm64_store(acc, [&](int i, int j, double v) { K[(size_t)i * IN + j] = v; });
    }
    if (nsw > 0)   // the rotated basis is the next warm start
      for (int it = tid; it < IN * IN; it += kSmallThreads) {
        const int i = it / IN, j = it % IN;
        V[(size_t)i * ld + j] = sQ[i][j];
      }
    if (tid == 0) {
      st->rank = rank_dk;
      st->kform = 0;
      st->margin = margin_dk;
      st->trace = trace_h;
      st->sweeps = nsw;
    }
    return true;
  };
  const int ne = nH + (nH & 1);
  int sweeps = 0;
  bool conv = false;
  const double ct2 = certify ? tau * tau : 0.0;
  // the perturbative finish: tried on the warm start, and in the block forms after each
  // sweep
  const bool dk_on = certify && K;
  const int gate_n = dk_on ? nH : 0;
  bool hit = false;
  if (ne <= 16) {
    if (dk_on && warm) {
      double mg;
      int rk;
      hit = dk_gate(nH, tau, sA, swv, red, redi, mg, rk);
    }
    if (!hit) {
      __shared__ int wave_res[2];
      if (tid < 64) {
        const bool c = small_sweeps<64, 1, 2, true>(sA, sQ, ne, fl, ct2, max_sweeps, pc, ps, pt, gbs, sweeps);
        if (tid == 0) {
          wave_res[0] = c ? 1 : 0;
          wave_res[1] = sweeps;
        }
      }
      __syncthreads();
      conv = wave_res[0] != 0;
      sweeps = wave_res[1];
    }
  } else if (ne <= 32)
    conv = small_sweeps<256, 1, 2>(sA, sQ, ne, fl, ct2, max_sweeps, pc, ps, pt, gbs, sweeps, gate_n, tau, warm, swv,
                                   red, redi, &hit);
  else
    conv = small_sweeps<kSmallThreads, 1, 2>(sA, sQ, ne, fl, ct2, max_sweeps, pc, ps, pt, gbs, sweeps, gate_n, tau,
                                             warm, swv, red, redi, &hit);
  if (hit) {
    if (dk_try(sweeps)) return;
    conv = false;   // not reached: the finish applies the same gate to the same matrix
  }
  // eigenvalues, descending order (ties by index), weights, rank, margin, trace
  double li = 0.0;
  if (tid < IN) {
    li = sA[tid][tid];
    lam[tid] = tid < nH ? li : 0.0;
  }
  if (tid < nH) {
    int rk = 0;
    for (int j = 0; j < nH; ++j) {
      const double lj = sA[j][j];
      rk += (lj > li) || (lj == li && j < tid);
    }
    prm[rk] = tid;
  } else if (tid < IN) {
    prm[tid] = tid;
  }
  __syncthreads();
  int kept = 0;
  double mg = 1.0e300, trc = 0.0;
  if (tid < nH) {
    const double lk = fmax(sA[prm[tid]][prm[tid]], 0.0);
    const double sg = sqrt(lk);
    double wk = 0.0;
    if (sg > tau) {
      kept = 1;
      wk = sqrt((sg - tau) / sg);
    }
    swv[tid] = wk;
    sw[tid] = wk;
    // a certified index enters through its bound: a lower bound on the distance
    const double g = gbs[prm[tid]];
    mg = g >= 0.0 ? (tau - sqrt(g)) / tau : fabs(sg - tau) / tau;
    trc = lk;
  } else if (tid < IN) {
    swv[tid] = 0.0;
  }
  if (tid < IN) perm[tid] = prm[tid];
  red[tid] = trc;
  redi[tid] = kept;
  __syncthreads();
  for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[tid] += red[tid + w];
      redi[tid] += redi[tid + w];
    }
    __syncthreads();
  }
  const double trace = red[0];
  const int rank = redi[0];
  __syncthreads();
  red[tid] = mg;
  __syncthreads();
  for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmin(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) {
    st->rank = rank;
    st->kform = 0;
    st->margin = red[0];
    st->trace = trace;
    st->sweeps = conv ? sweeps : -1;
  }
  // W = Q_sorted diag(sw) (columns k < rank), T = C W (with the C V basis, W is T), Tt,
  // K = T T^T
  for (int it = tid; it < IN * IN; it += kSmallThreads) {
    const int j = it / IN, k = it % IN;
    sW[j][k] = k < rank ? sQ[j][prm[k]] * swv[k] : 0.0;
  }
  __syncthreads();
  LdsRow* sT = sW;
  if (C && !cb) {
    if (mm_on) {
      mm64<false>(sC, sW, acc, km);
      mm64_store(acc, [&](int i, int j, double v) { sA[i][j] = v; });
    }
    __syncthreads();
    sT = sA;
  }
  for (int it = tid; it < IN * IN; it += kSmallThreads) {
    const int i = it / IN, j = it % IN;
    T[(size_t)i * ld + j] = sT[i][j];
    Tt[(size_t)j * ld + i] = sT[i][j];
    V[(size_t)i * ld + j] = sQ[i][j];
  }
  if (K) {
    // K = T T^T = X^T X with X = T^T staged in the Q buffer (V is already written)
    __syncthreads();
    for (int it = tid; it < IN * IN; it += kSmallThreads) {
      const int i = it / IN, j = it % IN;
      sQ[j][i] = sT[i][j];
    }
    __syncthreads();
    if (mm_on) {
      mm64<true>(sQ, sQ, acc, km);
      mm64_store(acc, [&](int i, int j, double v) { K[(size_t)i * IN + j] = v; });
    }
  }
}

// Threshold certificate of the sweep: gb[i] = sum_j |a_ij| (an upper bound on the
// Gershgorin interval of row i, as a_ii <= |a_ii|) if that lies below tau2 (less a
// relative 1e-12, so that rounding of the bound cannot reach tau2), else -1, and
// *uncert = 1 if some row is not certified.  One wave per row.
__global__ void __launch_bounds__(256) k_certify(const double* __restrict__ A, int N, double tau2,
                                                 double* __restrict__ gb, int* __restrict__ uncert) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= N) return;
  const double* a = A + (size_t)row * N;
  double s = 0.0;
  for (int j = lane; j < N; j += 64) s += fabs(a[j]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) {
    const bool c = s < tau2 * (1.0 - 1.0e-12);
    gb[row] = c ? s : -1.0;
    if (!c) atomicOr(uncert, 1);
  }
}

// after the sweeps (all-or-nothing form): a certificate that did not cover every row
// is void
__global__ void k_cert_finish(int N, const int* __restrict__ uncert, double* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && *uncert) gb[i] = -1.0;
}

// flag = 1 if any pair (p < q) of A passes the rotation test, unless the threshold
// certificate covers every row (uncert non-null and zero); with gb non-null (partial
// certificate) pairs of two certified indices are not counted
__global__ void __launch_bounds__(256) k_any_rotation(const double* __restrict__ A, int N,
                                                      const double* __restrict__ floor_p,
                                                      const int* __restrict__ uncert, const double* __restrict__ gb,
                                                      int* __restrict__ flag) {
  if (uncert != nullptr && *uncert == 0) return;
  const double fl = floor_p[0];
  int want = 0;
  const size_t total = (size_t)N * N;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / N), j = (int)(idx % N);
    if (i < j && !(gb != nullptr && gb[i] >= 0.0 && gb[j] >= 0.0) &&
        rotates(A[(size_t)i * N + i], A[(size_t)j * N + j], A[idx], fl))
      want = 1;
  }
  if (__syncthreads_or(want) && threadIdx.x == 0) atomicOr(flag, 1);
}

// The pre-test of a sweep in one launch, for widths below kCertPartialMin (so the
// certificate is all or nothing): each block forms the Gershgorin bounds of its rows
// (one wave per row; gb non-null) and the rotation test over its share of the pairs,
// and ORs both into scratch flags; the last block to finish (an atomic ticket, taken
// after a fence, so every block's flags are in; nothing waits) sets
// active = (some pair rotates) and (not every row certified), keeps the certificate's
// outcome for k_cert_finish, counts the sweep and clears the scratch for the next one.
// flags: [0] active, [1] some row not certified (kept), [2], [3] scratch ORs, [4] ticket.
__global__ void __launch_bounds__(256) k_pretest(const double* __restrict__ A, int N,
                                                 const double* __restrict__ floor_p, double tau2,
                                                 double* __restrict__ gb, int* __restrict__ flags,
                                                 int* __restrict__ count) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int unc = 0, want = 0;
  if (gb != nullptr) {
    for (int row = blockIdx.x * 4 + wv; row < N; row += gridDim.x * 4) {
      const double* a = A + (size_t)row * N;
      double sum = 0.0;
      for (int j = lane; j < N; j += 64) sum += fabs(a[j]);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
      if (lane == 0) {
        const bool c = sum < tau2 * (1.0 - 1.0e-12);
        gb[row] = c ? sum : -1.0;
        unc |= c ? 0 : 1;
      }
    }
  }
  const double fl = floor_p[0];
  const size_t total = (size_t)N * N;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / N), j = (int)(idx % N);
    if (i < j && rotates(A[(size_t)i * N + i], A[(size_t)j * N + j], A[idx], fl)) want = 1;
  }
  unc = __syncthreads_or(unc);
  want = __syncthreads_or(want);
  if (threadIdx.x == 0) {
    if (unc) atomicOr(&flags[2], 1);
    if (want) atomicOr(&flags[3], 1);
    __threadfence();
    if (atomicAdd(&flags[4], 1) == (int)gridDim.x - 1) {   // the last block
      const int u = atomicOr(&flags[2], 0), w = atomicOr(&flags[3], 0);
      const int act = (w && (gb == nullptr || u)) ? 1 : 0;
      flags[0] = act;
      flags[1] = u;
      if (act) count[0] += 1;
      flags[2] = 0;
      flags[3] = 0;
      flags[4] = 0;
    }
  }
}

// counts the sweeps whose pre-test found something to rotate
__global__ void k_count_sweep(const int* __restrict__ active, int* __restrict__ count) {
  if (threadIdx.x == 0 && *active) count[0] += 1;
}

__global__ void k_identity(double* __restrict__ V, int N) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)N * N) V[idx] = ((idx / N) == (idx % N)) ? 1.0 : 0.0;
}

// lam[i] = A_ii (all N)
__global__ void k_diag(const double* __restrict__ A, int N, double* __restrict__ lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) lam[i] = A[(size_t)i * N + i];
}

// perm[k] = i for the k-th largest lam among the first n (ties by index); n..N-1 map
// to themselves.  One thread per element, the n values staged in LDS.
__global__ void __launch_bounds__(256) k_rank(const double* __restrict__ lam, int N, int n, int* __restrict__ perm) {
  extern __shared__ double sl[];
  for (int j = threadIdx.x; j < n; j += blockDim.x) sl[j] = lam[j];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double li = sl[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = sl[j];
      rank += (lj > li) || (lj == li && j < i);
    }
    perm[rank] = i;
  } else if (i < N) {
    perm[i] = i;
  }
}

}  // namespace

int coarse_svt_small(int nH, int ld, const double* G, const double* C, double* V, bool warm, double tau,
                     bool certify, double* lam, int* perm, double* sw, double* T, double* Tt, double* K,
                     IterStats* st, hipStream_t stream) {
  if (nH < 1 || nH > IN || ld != IN) return MLPCP_E_INVALID_ARG;
  const size_t lds = (size_t)4 * IN * LDS_LD * sizeof(double);
  MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_coarse_small),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  ProfKernel pk(KC_COARSE_SMALL);
  hipExtLaunchKernelGGL(k_coarse_small, dim3(1), dim3(kSmallThreads), lds, stream, pk.start, pk.stop, 0, nH, ld, G,
                        C, V, warm ? 1 : 0, tau, certify ? 1 : 0, kMaxEigSweeps, lam, perm, sw, T, Tt, K, st);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

// Top eigenpair of H = C G C (n_H <= 64, one workgroup of four waves), for the nuclear
// linear oracle of multilevel Frank-Wolfe: repeated squaring P <- P P / trace(P P) from
// P = H / trace(H) until P is rank one to rounding (1 - ||P||_F^2 <= 1e-13; the
// top-eigenvalue share of P grows as (lambda_2 / lambda_1)^(2^s) shrinks), the column of
// P with the largest diagonal entry as the start, three power steps with H to polish,
// then z = C x and lam = x^T H x.  With a repeated top eigenvalue the result is a unit
// vector of the top eigenspace.  H = 0 gives z = 0, lam = 0.
constexpr int kTopThreads = 256;
constexpr int kTopSquarings = 24;

__global__ void __launch_bounds__(kTopThreads) k_coarse_top(int nH, const double* __restrict__ G,
                                                            const double* __restrict__ C, double* __restrict__ z,
                                                            double* __restrict__ lam_out) {
  extern __shared__ double dsm[];
  LdsRow* sC = reinterpret_cast<LdsRow*>(dsm);
  LdsRow* sH = sC + IN;
  LdsRow* sP = sH + IN;
  LdsRow* sQ = sP + IN;
  __shared__ double red[kTopThreads];
  __shared__ double sx[IN], sy[IN];
  const int tid = threadIdx.x;
  for (int it = tid; it < IN * IN; it += kTopThreads) {
    const int i = it / IN, j = it % IN;
    const bool in = i < nH && j < nH;
    sP[i][j] = in ? G[(size_t)i * IN + j] : 0.0;
    sC[i][j] = (C && in) ? C[(size_t)i * nH + j] : (C ? 0.0 : (i == j && i < nH ? 1.0 : 0.0));
  }
  __syncthreads();
  d4_t acc[2][2];
  mm64<false>(sP, sC, acc);                                  // G C
  mm64_store(acc, [&](int i, int j, double v) { sQ[i][j] = v; });
  __syncthreads();
  mm64<false>(sC, sQ, acc);                                  // C (G C)
  mm64_store(acc, [&](int i, int j, double v) { sP[i][j] = v; });
  __syncthreads();
  // H = sym(C G C), its trace
  double tr = 0.0;
  for (int it = tid; it < IN * IN; it += kTopThreads) {
    const int i = it / IN, j = it % IN;
    const double v = 0.5 * (sP[i][j] + sP[j][i]);
    sH[i][j] = v;
    if (i == j) tr += v;
  }
  red[tid] = tr;
  __syncthreads();
  for (int w = kTopThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double trace = red[0];
  __syncthreads();
  if (!(trace > 0.0)) {
    if (tid < IN) z[tid] = 0.0;
    if (tid == 0) *lam_out = 0.0;
    return;
  }
  for (int it = tid; it < IN * IN; it += kTopThreads) {
    const int i = it / IN, j = it % IN;
    sP[i][j] = sH[i][j] / trace;
  }
  __syncthreads();
  // two wave sums folded through LDS together: two barriers per reduction
  __shared__ double red2[2][kTopThreads / 64];
  auto block_total2 = [&](double& v0, double& v1) {
    for (int o = 32; o > 0; o >>= 1) {
      v0 += __shfl_xor(v0, o, 64);
      v1 += __shfl_xor(v1, o, 64);
    }
    __syncthreads();
    if ((tid & 63) == 0) {
      red2[0][tid >> 6] = v0;
      red2[1][tid >> 6] = v1;
    }
    __syncthreads();
    v0 = v1 = 0.0;
    for (int w = 0; w < kTopThreads / 64; ++w) {
      v0 += red2[0][w];
      v1 += red2[1][w];
    }
  };
  // P holds H / trace(H) (trace 1).  Each squaring stores P P / t^2, t = trace(P), so the
  // stored matrix is (P / t)^2 with trace in [1 / n_H, 1]; its trace and squared
  // Frobenius norm come from the accumulators.  Rank one to rounding when
  // ||P||_F^2 / trace(P)^2 >= 1 - 1e-13.
  double t_cur = 1.0;
  for (int sq = 0; sq < kTopSquarings; ++sq) {
    mm64<false>(sP, sP, acc);
    __syncthreads();                       // every wave has read P before it is overwritten
    const double inv = 1.0 / (t_cur * t_cur);
    double tr = 0.0, f2 = 0.0;
    mm64_store(acc, [&](int i, int j, double v) {
      const double x = v * inv;
      sP[i][j] = x;
      f2 += x * x;
      if (i == j) tr += x;
    });
    block_total2(tr, f2);
    if (!(tr > 0.0)) break;
    t_cur = tr;
    if (1.0 - f2 / (tr * tr) <= 1e-13) break;
  }
  __syncthreads();
  // start: the column with the largest diagonal entry (ties: smallest index)
  if (tid == 0) {
    int jb = 0;
    for (int j = 1; j < nH; ++j)
      if (sP[j][j] > sP[jb][jb]) jb = j;
    double nn = 0.0;
    for (int i = 0; i < IN; ++i) nn += sP[i][jb] * sP[i][jb];
    nn = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int i = 0; i < IN; ++i) sx[i] = nn > 0.0 ? sP[i][jb] * nn : (i == jb ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int step = 0; step < 3; ++step) {
    if (tid < IN) {
      double y = 0.0;
      for (int k = 0; k < IN; ++k) y += sH[tid][k] * sx[k];
      sy[tid] = y;
    }
    __syncthreads();
    if (tid == 0) {
      double nn = 0.0;
      for (int i = 0; i < IN; ++i) nn += sy[i] * sy[i];
      red[0] = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    }
    __syncthreads();
    const double inv = red[0];
    __syncthreads();
    if (tid < IN && inv > 0.0) sx[tid] = sy[tid] * inv;
    __syncthreads();
  }
  if (tid < IN) {
    double y = 0.0, zc = 0.0;
    for (int k = 0; k < IN; ++k) {
      y += sH[tid][k] * sx[k];
      zc += sC[tid][k] * sx[k];
    }
    sy[tid] = y * sx[tid];
    z[tid] = tid < nH ? zc : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double l = 0.0;
    for (int i = 0; i < IN; ++i) l += sy[i];
    *lam_out = l;
  }
}

int coarse_top_small(int nH, const double* G, const double* C, double* z, double* lam, hipStream_t stream) {
  if (nH < 1 || nH > IN) return MLPCP_E_INVALID_ARG;
  const size_t lds = (size_t)4 * IN * LDS_LD * sizeof(double);
  MLPCP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_coarse_top),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_coarse_top, dim3(1), dim3(kTopThreads), lds, stream, nH, G, C, z, lam);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

size_t eig_workspace_bytes(int N) {
  const size_t npairs = (size_t)(N / IB) / 2;
  return align256(std::max<size_t>(npairs, 1) * (IN * IN + 1) * sizeof(double)) +
         align256((size_t)N * N * sizeof(double)) + 256 + 256;
}

int eig_sym(int n, int N, double* A, double* V, double* lam, int* perm, void* ws, hipStream_t stream,
            int* sweeps_out, bool warm, int sweep_hint, double cert_tau2, double* gb) {
  if (cert_tau2 > 0.0 && gb == nullptr) return MLPCP_E_INVALID_ARG;
  if (!(cert_tau2 > 0.0)) gb = nullptr;
  const bool partial = gb != nullptr && N >= kCertPartialMin;
  if (N % IN != 0 || n > N || n < 1) return MLPCP_E_INVALID_ARG;
  char* w = static_cast<char*>(ws);
  const int nb = N / IB;
  const int npairs = nb / 2;
  double* Qblk = reinterpret_cast<double*>(w);
  w += align256((size_t)std::max(npairs, 1) * (IN * IN + 1) * sizeof(double));
  double* tmp = reinterpret_cast<double*>(w);
  w += align256((size_t)N * N * sizeof(double));
  double* floor_p = reinterpret_cast<double*>(w);
  int* flag = reinterpret_cast<int*>(w + 128);
  int* uncert = reinterpret_cast<int*>(w + 132);   // cleared with flag (one 8-byte memset)
  int* dsweeps = reinterpret_cast<int*>(w + 192);

  {
    ProfScope ps(KC_JACOBI_MISC, stream);
    hipLaunchKernelGGL(k_floor, dim3(1), dim3(256), 0, stream, A, N, floor_p);
    if (warm) {
      // A <- V0^T A V0 (V holds V0 and keeps it as the starting eigenvector basis)
      MLPCP_TRY(gemm_f64(true, false, N, N, N, 1.0, V, N, A, N, tmp, N, stream));
      MLPCP_TRY(gemm_f64(false, false, N, N, N, 1.0, tmp, N, V, N, A, N, stream));
    } else if (N != IN) {
      const size_t nn = (size_t)N * N;
      hipLaunchKernelGGL(k_identity, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, stream, V, N);
    }
  }
  int sweeps = 0;
  if (N == IN) {
    if (gb) return MLPCP_E_UNSUPPORTED;   // the certificate is not part of the direct solver
    {
      ProfScope ps(KC_JACOBI_PAIRS, stream);
      hipLaunchKernelGGL(k_jacobi_direct, dim3(1), dim3(256), 0, stream, A, V, N, floor_p, warm ? 1 : 0,
                         kMaxEigSweeps, dsweeps);
    }
    MLPCP_HIP(hipGetLastError());
    MLPCP_HIP(hipMemcpyAsync(&sweeps, dsweeps, sizeof(int), hipMemcpyDeviceToHost, stream));
    MLPCP_HIP(hipStreamSynchronize(stream));
    if (sweeps < 0) return MLPCP_E_EIG;
  } else {
    const int ntri = npairs * (npairs - 1) / 2;
    // few tiles: the split apply step, with A alternating between the caller's buffer
    // and tmp (free after the warm start) from round to round
    const bool split = N <= kSplitApplyMax;
    const int apply_blocks = split ? 4 * (ntri + (N / IN) * npairs) : ntri + (N / IN) * npairs;
    double* cur = A;
    double* other = split ? tmp : A;
    bool converged = false;
    // Each sweep starts with a device-side test (any pair passing the rotation test?)
    // whose result gates every kernel of the sweep, so sweeps can be queued without a
    // host round trip: a sweep after convergence costs its empty launches only.
    int* active = flag;
    MLPCP_HIP(hipMemsetAsync(dsweeps, 0, sizeof(int), stream));
    // flag[0..4]: active, uncert, two scratch ORs and the ticket of k_pretest (zero
    // between its launches)
    MLPCP_HIP(hipMemsetAsync(flag, 0, 5 * sizeof(int), stream));
    // a sweep is its pre-test (which sets `active` and counts the sweep) and its rounds,
    // whose kernels do nothing when the pre-test found nothing to rotate
    auto pretest = [&]() -> int {
      if (!partial) {   // one launch
        ProfScope ps(KC_JACOBI_MISC, stream);
        hipLaunchKernelGGL(k_pretest, dim3(64), dim3(256), 0, stream, cur, N, floor_p, cert_tau2, gb, flag, dsweeps);
        return MLPCP_OK;
      }
      MLPCP_HIP(hipMemsetAsync(active, 0, 2 * sizeof(int), stream));   // active, uncert
      ProfScope ps(KC_JACOBI_MISC, stream);
      if (gb) hipLaunchKernelGGL(k_certify, dim3((N + 3) / 4), dim3(256), 0, stream, cur, N, cert_tau2, gb, uncert);
      hipLaunchKernelGGL(k_any_rotation, dim3(64), dim3(256), 0, stream, cur, N, floor_p, gb ? uncert : nullptr,
                         partial ? gb : nullptr, active);
      hipLaunchKernelGGL(k_count_sweep, dim3(1), dim3(64), 0, stream, active, dsweeps);
      return MLPCP_OK;
    };
    auto rounds = [&]() {
      for (int r = 0; r < nb - 1; ++r) {
        {
          ProfKernel pk(KC_JACOBI_PAIRS);
          hipExtLaunchKernelGGL(k_jacobi_pairs, dim3(npairs), dim3(kPairThreads), 0, stream, pk.start, pk.stop, 0,
                                cur, other, N, nb, r, Qblk, floor_p, active, partial ? gb : nullptr);
        }
        {
          ProfKernel pk(KC_JACOBI_APPLY);
          if (split)
            hipExtLaunchKernelGGL(k_jacobi_apply_split, dim3(apply_blocks), dim3(256), 0, stream, pk.start, pk.stop,
                                  0, cur, other, V, N, nb, r, Qblk, active);
          else
            hipExtLaunchKernelGGL(k_jacobi_apply, dim3(apply_blocks), dim3(256), 0, stream, pk.start, pk.stop, 0, A,
                                  V, N, nb, r, Qblk, active);
        }
        std::swap(cur, other);
      }
    };
    // The first batch is one sweep less than the caller's hint (the previous solve's
    // count), followed by the pre-test of the next sweep alone; each host check then
    // queues that sweep's rounds only if its pre-test found something, and the next
    // pre-test.  So the sweep that confirms convergence costs its pre-test, not rounds.
    const int batch = std::max(0, std::min(sweep_hint - 1, kMaxEigSweeps));
    for (int b = 0; b < batch; ++b) {
      MLPCP_TRY(pretest());
      rounds();
    }
    MLPCP_TRY(pretest());
    int queued = batch;
    int hstate[2] = {0, 0};
    for (;;) {
      MLPCP_HIP(hipGetLastError());
      // active and the sweep count are adjacent in the workspace
      MLPCP_HIP(hipMemcpyAsync(&hstate[0], active, sizeof(int), hipMemcpyDeviceToHost, stream));
      MLPCP_HIP(hipMemcpyAsync(&hstate[1], dsweeps, sizeof(int), hipMemcpyDeviceToHost, stream));
      MLPCP_HIP(hipStreamSynchronize(stream));
      sweeps = hstate[1];
      if (!hstate[0]) {   // the last pre-test found nothing: converged
        converged = true;
        break;
      }
      if (sweeps >= kMaxEigSweeps || queued > 2 * kMaxEigSweeps) break;
      rounds();           // the sweep whose pre-test passed
      MLPCP_TRY(pretest());
      ++queued;
    }
    if (cur != A) MLPCP_HIP(hipMemcpyAsync(A, cur, (size_t)N * N * sizeof(double), hipMemcpyDeviceToDevice, stream));
    if (!converged) return MLPCP_E_EIG;
    if (gb && !partial) {
      ProfScope ps(KC_JACOBI_MISC, stream);
      hipLaunchKernelGGL(k_cert_finish, dim3((N + 255) / 256), dim3(256), 0, stream, N, uncert, gb);
    }
  }
  {
    ProfScope ps(KC_JACOBI_MISC, stream);
    hipLaunchKernelGGL(k_diag, dim3((N + 255) / 256), dim3(256), 0, stream, A, N, lam);
    hipLaunchKernelGGL(k_rank, dim3((N + 255) / 256), dim3(256), (size_t)n * sizeof(double), stream, lam, N, n,
                       perm);
  }
  MLPCP_HIP(hipGetLastError());
  if (sweeps_out) *sweeps_out = sweeps;
  return MLPCP_OK;
}

}  // namespace mlpcp
