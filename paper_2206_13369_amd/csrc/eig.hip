// Symmetric eigensolver in float64 for the coarse Gram matrix (the SVD of the
// coarse data in Alg. 4 is taken as the eigendecomposition of its Gram matrix).
//
// Method: parallel two-sided cyclic Jacobi (Golub & Van Loan, sec. 8.5), blocked.
//  * Indices are grouped into blocks of b = kEigBlock.  One outer sweep visits every
//    pair of blocks once, in round-robin order (the circle method: one block fixed,
//    the others rotating), so each round holds nb/2 disjoint block pairs.
//  * For each pair the 2b x 2b principal submatrix is diagonalised in LDS by an inner
//    cyclic Jacobi (itself in round-robin order: b disjoint 2x2 rotations at a time),
//    accumulating the orthogonal factor Q_pair.
//  * The round's transformation J = diag(Q_pair) is then applied tile by tile:
//    A[Pa,Pb] <- Q_a^T A[Pa,Pb] Q_b for every pair of pairs, V[:,Pb] <- V[:,Pb] Q_b.
//    Tiles are disjoint, so the update is in place.
//  * A sweep in which no inner problem rotated anything (every off-diagonal entry
//    below threshold) ends the iteration.
//  Problems of width <= 2b are solved by one inner solve directly.
//  Rotation threshold (Demmel-Veselic style, with an absolute floor for singular
//  Grams): rotate (p,q) iff |a_pq| > eps * sqrt(|a_pp a_qq|) and |a_pq| > floor,
//  floor = 1e-17 * trace(A).
#include "common.h"
#include "profile.h"

#include <cmath>

namespace mlpcp {

namespace {

constexpr int IB = kEigBlock;       // 16
constexpr int IN = kEigInner;       // 32
constexpr int LDS_LD = IN + 1;
constexpr double kRelEps = 2.0e-16;

// circle method: position i of 2p players in round r (player 0 fixed)
__device__ __forceinline__ int rr_player(int i, int r, int players) {
  return i == 0 ? 0 : 1 + ((i - 1 + r) % (players - 1));
}

__device__ __forceinline__ void rr_pair(int k, int r, int players, int& a, int& b) {
  int x = rr_player(k, r, players);
  int y = rr_player(players - 1 - k, r, players);
  a = x < y ? x : y;
  b = x < y ? y : x;
}

// Jacobi rotation annihilating a_pq of [[app, apq], [apq, aqq]]:
//   [c s; -s c]^T A [c s; -s c] diagonal, t = s / c the smaller root of
//   t^2 + 2 theta t - 1 = 0, theta = (aqq - app) / (2 apq).
__device__ __forceinline__ void rotation(double app, double aqq, double apq, double& c, double& s,
                                         double& t) {
  double theta = (aqq - app) / (2.0 * apq);
  double at = fabs(theta);
  if (at > 1.0e150) {
    t = 0.5 / theta;
  } else {
    t = (theta >= 0.0 ? 1.0 : -1.0) / (at + sqrt(1.0 + theta * theta));
  }
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// One inner sweep set on the IN x IN matrix in LDS, accumulating Q <- Q * J.
// Runs up to max_sweeps sweeps, stops early after a sweep with no rotation.
// Returns (in lds flag) whether any rotation happened.  256 threads.
__device__ void inner_jacobi(double (*A)[LDS_LD], double (*Q)[LDS_LD], int max_sweeps, double floor_abs,
                             int* any_rot) {
  __shared__ double rc[IB], rs[IB], rt[IB];
  __shared__ int rp[IB], rq[IB], rot_on[IB];
  __shared__ int sweep_rot;
  const int tid = threadIdx.x;
  if (tid == 0) *any_rot = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (tid == 0) sweep_rot = 0;
    __syncthreads();
    for (int r = 0; r < IN - 1; ++r) {
      if (tid < IB) {
        int p, q;
        rr_pair(tid, r, IN, p, q);
        double app = A[p][p], aqq = A[q][q], apq = A[p][q];
        double c = 1.0, s = 0.0, t = 0.0;
        int on = 0;
        if (fabs(apq) > floor_abs && fabs(apq) > kRelEps * sqrt(fabs(app) * fabs(aqq))) {
          rotation(app, aqq, apq, c, s, t);
          on = 1;
          sweep_rot = 1;
        }
        rc[tid] = c; rs[tid] = s; rt[tid] = t; rp[tid] = p; rq[tid] = q; rot_on[tid] = on;
      }
      __syncthreads();
      {  // 2x2 tile update: tile (a, b), one per thread (IB*IB = 256 tiles)
        const int a = tid / IB, b = tid % IB;
        const int pa = rp[a], qa = rq[a], pb = rp[b], qb = rq[b];
        if (rot_on[a] | rot_on[b]) {
          if (a == b) {
            const double t = rt[a], apq = A[pa][qa];
            A[pa][pa] -= t * apq;
            A[qa][qa] += t * apq;
            A[pa][qa] = 0.0;
            A[qa][pa] = 0.0;
          } else {
            const double ca = rc[a], sa = rs[a], cb = rc[b], sb = rs[b];
            const double t00 = A[pa][pb], t01 = A[pa][qb], t10 = A[qa][pb], t11 = A[qa][qb];
            const double u00 = ca * t00 - sa * t10, u01 = ca * t01 - sa * t11;
            const double u10 = sa * t00 + ca * t10, u11 = sa * t01 + ca * t11;
            A[pa][pb] = u00 * cb - u01 * sb;
            A[pa][qb] = u00 * sb + u01 * cb;
            A[qa][pb] = u10 * cb - u11 * sb;
            A[qa][qb] = u10 * sb + u11 * cb;
          }
        }
      }
      for (int it = tid; it < IN * IB; it += blockDim.x) {  // Q <- Q * J (row i, pair b)
        const int i = it / IB, b = it % IB;
        if (rot_on[b]) {
          const int pb = rp[b], qb = rq[b];
          const double c = rc[b], s = rs[b];
          const double x = Q[i][pb], y = Q[i][qb];
          Q[i][pb] = c * x - s * y;
          Q[i][qb] = s * x + c * y;
        }
      }
      __syncthreads();
    }
    const int any = sweep_rot;
    __syncthreads();
    if (!any) break;
    if (tid == 0) *any_rot = 1;
  }
  __syncthreads();
}

// trace(A) -> floor = 1e-17 * |trace| (one block)
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
  if (threadIdx.x == 0) floor_out[0] = 1.0e-17 * red[0] + 1.0e-300;
}

// Whole problem fits one inner solve (N == IN).
__global__ void __launch_bounds__(256) k_jacobi_direct(double* __restrict__ A, double* __restrict__ V, int N,
                                                       const double* __restrict__ floor_p, int max_sweeps,
                                                       int* __restrict__ sweeps_out) {
  __shared__ double sA[IN][LDS_LD];
  __shared__ double sQ[IN][LDS_LD];
  __shared__ int any;
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) {
    const int i = it / IN, j = it % IN;
    sA[i][j] = A[(size_t)i * N + j];
    sQ[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // run sweeps one at a time to count them
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    inner_jacobi(sA, sQ, 1, floor_p[0], &any);
    if (!any) break;
  }
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) {
    const int i = it / IN, j = it % IN;
    A[(size_t)i * N + j] = sA[i][j];
    V[(size_t)i * N + j] = sQ[i][j];
  }
  if (threadIdx.x == 0) sweeps_out[0] = (sweeps < max_sweeps) ? sweeps + 1 : -1;
}

__device__ __forceinline__ int pair_global(int l, int I, int J) {
  return l < IB ? I * IB + l : J * IB + (l - IB);
}

// Outer round, step 1: one block per block pair; diagonalise the 2b x 2b
// submatrix, write Q_pair.
__global__ void __launch_bounds__(256) k_jacobi_pairs(const double* __restrict__ A, int N, int nb, int round,
                                                      double* __restrict__ Qblk, const double* __restrict__ floor_p,
                                                      int inner_sweeps, int* __restrict__ flag) {
  __shared__ double sA[IN][LDS_LD];
  __shared__ double sQ[IN][LDS_LD];
  __shared__ int any;
  int I, J;
  rr_pair(blockIdx.x, round, nb, I, J);
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) {
    const int i = it / IN, j = it % IN;
    sA[i][j] = A[(size_t)pair_global(i, I, J) * N + pair_global(j, I, J)];
    sQ[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  inner_jacobi(sA, sQ, inner_sweeps, floor_p[0], &any);
  double* Qo = Qblk + (size_t)blockIdx.x * IN * IN;
  for (int it = threadIdx.x; it < IN * IN; it += blockDim.x) Qo[it] = sQ[it / IN][it % IN];
  if (threadIdx.x == 0 && any) atomicOr(flag, 1);
}

// Outer round, step 2: apply J.  Blocks [0, npairs^2) update A tiles (pair a rows x
// pair b cols); blocks [npairs^2, npairs^2 + (N/IN)*npairs) update V tiles
// (32-row chunk x pair b cols).
__global__ void __launch_bounds__(256) k_jacobi_apply(double* __restrict__ A, double* __restrict__ V, int N, int nb,
                                                      int round, const double* __restrict__ Qblk,
                                                      const int* __restrict__ flag) {
  __shared__ double sT[IN][LDS_LD];
  __shared__ double sU[IN][LDS_LD];
  __shared__ double sQa[IN][LDS_LD];
  __shared__ double sQb[IN][LDS_LD];
  const int npairs = nb / 2;
  const int tid = threadIdx.x;
  int bid = blockIdx.x;
  if (bid < npairs * npairs) {
    const int a = bid / npairs, b = bid % npairs;
    int Ia, Ja, Ib, Jb;
    rr_pair(a, round, nb, Ia, Ja);
    rr_pair(b, round, nb, Ib, Jb);
    const double* Qa = Qblk + (size_t)a * IN * IN;
    const double* Qb = Qblk + (size_t)b * IN * IN;
    for (int it = tid; it < IN * IN; it += blockDim.x) {
      const int i = it / IN, j = it % IN;
      sT[i][j] = A[(size_t)pair_global(i, Ia, Ja) * N + pair_global(j, Ib, Jb)];
      sQa[i][j] = Qa[it];
      sQb[i][j] = Qb[it];
    }
    __syncthreads();
    // U = Qa^T T
    for (int it = tid; it < IN * IN; it += blockDim.x) {
      const int i = it / IN, j = it % IN;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < IN; ++k) acc += sQa[k][i] * sT[k][j];
      sU[i][j] = acc;
    }
    __syncthreads();
    // T' = U Qb
    for (int it = tid; it < IN * IN; it += blockDim.x) {
      const int i = it / IN, j = it % IN;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < IN; ++k) acc += sU[i][k] * sQb[k][j];
      A[(size_t)pair_global(i, Ia, Ja) * N + pair_global(j, Ib, Jb)] = acc;
    }
  } else {
    bid -= npairs * npairs;
    const int rb = bid / npairs, b = bid % npairs;
    int Ib, Jb;
    rr_pair(b, round, nb, Ib, Jb);
    const double* Qb = Qblk + (size_t)b * IN * IN;
    for (int it = tid; it < IN * IN; it += blockDim.x) {
      const int i = it / IN, j = it % IN;
      sT[i][j] = V[(size_t)(rb * IN + i) * N + pair_global(j, Ib, Jb)];
      sQb[i][j] = Qb[it];
    }
    __syncthreads();
    for (int it = tid; it < IN * IN; it += blockDim.x) {
      const int i = it / IN, j = it % IN;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < IN; ++k) acc += sT[i][k] * sQb[k][j];
      V[(size_t)(rb * IN + i) * N + pair_global(j, Ib, Jb)] = acc;
    }
  }
  (void)flag;
}

__global__ void k_identity(double* __restrict__ V, int N) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)N * N) V[idx] = ((idx / N) == (idx % N)) ? 1.0 : 0.0;
}

// lam[i] = A_ii; perm[k] = i for the k-th largest among the first n (ties by index).
__global__ void __launch_bounds__(1024) k_eig_sort(const double* __restrict__ A, int N, int n,
                                                   double* __restrict__ lam, int* __restrict__ perm) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) lam[i] = A[(size_t)i * N + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double li = lam[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = lam[j];
      rank += (lj > li) || (lj == li && j < i);
    }
    perm[rank] = i;
  }
  for (int i = n + threadIdx.x; i < N; i += blockDim.x) perm[i] = i;
}

}  // namespace

size_t eig_workspace_bytes(int N) {
  const int nb = N / IB;
  const size_t npairs = nb / 2;
  return align256(npairs * IN * IN * sizeof(double)) + 256 + 256;
}

int eig_sym(int n, int N, double* A, double* V, double* lam, int* perm, void* ws, hipStream_t stream,
            int* sweeps_out) {
  if (N % IN != 0 || n > N || n < 1) return MLPCP_E_INVALID_ARG;
  char* w = static_cast<char*>(ws);
  const int nb = N / IB;
  const int npairs = nb / 2;
  double* Qblk = reinterpret_cast<double*>(w);
  w += align256((size_t)npairs * IN * IN * sizeof(double));
  double* floor_p = reinterpret_cast<double*>(w);
  int* flag = reinterpret_cast<int*>(w + 128);
  int* dsweeps = reinterpret_cast<int*>(w + 192);

  {
    ProfScope ps(KC_JACOBI_MISC, stream);
    hipLaunchKernelGGL(k_floor, dim3(1), dim3(256), 0, stream, A, N, floor_p);
  }
  int sweeps = 0;
  if (N == IN) {
    {
      ProfScope ps(KC_JACOBI_PAIRS, stream);
      hipLaunchKernelGGL(k_jacobi_direct, dim3(1), dim3(256), 0, stream, A, V, N, floor_p, kMaxEigSweeps,
                         dsweeps);
    }
    MLPCP_HIP(hipGetLastError());
    MLPCP_HIP(hipMemcpyAsync(&sweeps, dsweeps, sizeof(int), hipMemcpyDeviceToHost, stream));
    MLPCP_HIP(hipStreamSynchronize(stream));
    if (sweeps < 0) return MLPCP_E_EIG;
  } else {
    const size_t nn = (size_t)N * N;
    {
      ProfScope ps(KC_JACOBI_MISC, stream);
      hipLaunchKernelGGL(k_identity, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, stream, V, N);
    }
    const int apply_blocks = npairs * npairs + (N / IN) * npairs;
    bool converged = false;
    int hflag = 0;
    for (sweeps = 1; sweeps <= kMaxEigSweeps; ++sweeps) {
      MLPCP_HIP(hipMemsetAsync(flag, 0, sizeof(int), stream));
      for (int r = 0; r < nb - 1; ++r) {
        {
          ProfScope ps(KC_JACOBI_PAIRS, stream);
          hipLaunchKernelGGL(k_jacobi_pairs, dim3(npairs), dim3(256), 0, stream, A, N, nb, r, Qblk, floor_p, 1,
                             flag);
        }
        {
          ProfScope ps(KC_JACOBI_APPLY, stream);
          hipLaunchKernelGGL(k_jacobi_apply, dim3(apply_blocks), dim3(256), 0, stream, A, V, N, nb, r, Qblk,
                             flag);
        }
      }
      MLPCP_HIP(hipGetLastError());
      MLPCP_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
      MLPCP_HIP(hipStreamSynchronize(stream));
      if (!hflag) {
        converged = true;
        break;
      }
    }
    if (!converged) return MLPCP_E_EIG;
  }
  {
    ProfScope ps(KC_JACOBI_MISC, stream);
    hipLaunchKernelGGL(k_eig_sort, dim3(1), dim3(1024), 0, stream, A, N, n, lam, perm);
  }
  MLPCP_HIP(hipGetLastError());
  if (sweeps_out) *sweeps_out = sweeps;
  return MLPCP_OK;
}

}  // namespace mlpcp
