// Coarse-model operators (Sec. 3.1) and the streaming entry points restrict, prolong
// and shrink.
//
// The interpolation operator P_n of eq. (Rx) is read through the worked n = 6 example:
// even n -> n/2 coarse points, fine row 0 and fine row 1 both take coarse point 0, odd
// fine rows 2k+1 take coarse point k, even fine rows 2k (k >= 1) average coarse points
// k-1 and k.  Odd n (not covered by the paper) uses vertex-centred interpolation:
// coarse points at even fine rows, midpoints at odd rows, n_H = (n+1)/2.  "levels"
// composes that many operators.  The composite is piecewise linear, so each fine row
// has at most two nonzero weights; weights are dyadic, hence exact in float.
//
// The coarse model uses R = P C with C = (P^T P)^{-1/2}: orthonormal columns spanning
// range(P) (the normalisation for which the nuclear-norm gap of Thm. LH-eps vanishes).
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <utility>

namespace mlpcp {

int coarse_dim_checked(int n, int levels) {
  if (levels < 0 || n < 1) return MLPCP_E_LEVELS;
  for (int l = 0; l < levels; ++l) {
    if (n < 2) return MLPCP_E_LEVELS;
    n = (n % 2 == 0) ? n / 2 : (n + 1) / 2;
  }
  return n;
}

namespace {

using SparseRow = std::vector<std::pair<int, double>>;

// single-level operator rows: fine j -> (coarse, weight)
std::vector<SparseRow> level_rows(int n) {
  std::vector<SparseRow> rows(n);
  if (n % 2 == 0) {
    const int nH = n / 2;
    rows[0] = {{0, 1.0}};
    for (int k = 0; k < nH; ++k) rows[2 * k + 1] = {{k, 1.0}};
    for (int k = 1; k < nH; ++k) rows[2 * k] = {{k - 1, 0.5}, {k, 0.5}};
  } else {
    const int nH = (n + 1) / 2;
    for (int k = 0; k < nH; ++k) rows[2 * k] = {{k, 1.0}};
    for (int k = 0; k + 1 < nH; ++k) rows[2 * k + 1] = {{k, 0.5}, {k + 1, 0.5}};
  }
  return rows;
}

}  // namespace

void build_stencil_host(int n, int levels, std::vector<int>& row_idx, std::vector<float>& row_w,
                        std::vector<int>& col_ptr, std::vector<int>& col_row, std::vector<float>& col_w,
                        std::vector<double>* dense_P) {
  // compose: fine row j of P_n P_{n1} ... as a sparse combination of coarsest points
  std::vector<SparseRow> cur(n);
  for (int j = 0; j < n; ++j) cur[j] = {{j, 1.0}};
  int width = n;
  for (int l = 0; l < levels; ++l) {
    const std::vector<SparseRow> lr = level_rows(width);
    for (int j = 0; j < n; ++j) {
      std::map<int, double> acc;
      for (const auto& cw : cur[j])
        for (const auto& dw : lr[cw.first]) acc[dw.first] += cw.second * dw.second;
      SparseRow nr;
      for (const auto& kv : acc)
        if (kv.second != 0.0) nr.push_back(kv);
      cur[j] = nr;
    }
    width = (width % 2 == 0) ? width / 2 : (width + 1) / 2;
  }
  const int nH = width;
  row_idx.assign((size_t)n * kMaxStencil, 0);
  row_w.assign((size_t)n * kMaxStencil, 0.0f);
  std::vector<std::vector<std::pair<int, float>>> cols(nH);
  for (int j = 0; j < n; ++j) {
    int s = 0;
    for (const auto& cw : cur[j]) {
      if (s < kMaxStencil) {
        row_idx[(size_t)j * kMaxStencil + s] = cw.first;
        row_w[(size_t)j * kMaxStencil + s] = (float)cw.second;
      }
      ++s;
      cols[cw.first].push_back({j, (float)cw.second});
    }
  }
  col_ptr.assign(nH + 1, 0);
  col_row.clear();
  col_w.clear();
  for (int c = 0; c < nH; ++c) {
    col_ptr[c + 1] = col_ptr[c] + (int)cols[c].size();
    for (const auto& jw : cols[c]) {
      col_row.push_back(jw.first);
      col_w.push_back(jw.second);
    }
  }
  if (dense_P) {
    dense_P->assign((size_t)n * nH, 0.0);
    for (int j = 0; j < n; ++j)
      for (const auto& cw : cur[j]) (*dense_P)[(size_t)j * nH + cw.first] = cw.second;
  }
}

namespace {

// W[i][k] = V[i][k] / sqrt(lam[k]) for k < nH (i < nH)
__global__ void k_scale_cols_invsqrt(const double* __restrict__ V, const double* __restrict__ lam, int N, int nH,
                                     double* __restrict__ W) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nH * nH) return;
  const int i = (int)(idx / nH), k = (int)(idx % nH);
  W[(size_t)i * N + k] = V[(size_t)i * N + k] / sqrt(lam[k]);
}

struct OpDeleter {
  void operator()(Operator* op) const {
    if (!op) return;
    (void)hipFree(op->mem);
    delete op;
  }
};

std::mutex g_op_mutex;
std::map<std::tuple<int, int, int>, std::unique_ptr<Operator, OpDeleter>> g_ops;

// QfT = (P C)^T in float32 (kQfWidth x n, zero rows beyond n_H): row j of P has at most
// two taps, so column j of QfT is w0 C[c0, :] + w1 C[c1, :], formed in float64 and
// rounded once.
__global__ void k_build_Qf(int n, int nH, const int* __restrict__ row_idx, const float* __restrict__ row_w,
                           const double* __restrict__ C, float* __restrict__ Qf) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * kQfWidth; e += gridDim.x * blockDim.x) {
    const int j = e / kQfWidth, c = e % kQfWidth;
    double v = 0.0;
    if (c < nH)
      for (int t = 0; t < kMaxStencil; ++t)
        v = fma((double)row_w[j * kMaxStencil + t], C[(size_t)row_idx[j * kMaxStencil + t] * nH + c], v);
    Qf[(size_t)c * n + j] = (float)v;
  }
}

// Device memory of one operator, carved from two blocks: `kept` (stencil tables and C,
// alive as long as the operator) and `tmp` (the eigensolve that forms C).
struct OpLayout {
  size_t off_row_idx, off_row_w, off_col_ptr, off_col_row, off_col_w, off_C, off_Qf, kept;
  size_t off_A, off_V, off_W, off_lam, off_perm, off_ews, tmp;
};

OpLayout op_layout(int n, int levels) {
  OpLayout l{};
  const int nH = coarse_dim_checked(n, levels);
  const size_t nnz = (size_t)kMaxStencil * n;   // upper bound on the nonzeros of P
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += align256(std::max<size_t>(b, 1));
    return o;
  };
  l.off_row_idx = take((size_t)n * kMaxStencil * sizeof(int));
  l.off_row_w = take((size_t)n * kMaxStencil * sizeof(float));
  l.off_col_ptr = take((size_t)(nH + 1) * sizeof(int));
  l.off_col_row = take(nnz * sizeof(int));
  l.off_col_w = take(nnz * sizeof(float));
  l.off_C = take(levels > 0 ? (size_t)nH * nH * sizeof(double) : 0);
  l.off_Qf = take(levels > 0 && nH <= kQfWidth ? (size_t)n * kQfWidth * sizeof(float) : 0);
  l.kept = off;
  off = 0;
  if (levels > 0) {
    const int N = round_up(nH, kPad);
    const size_t nn = (size_t)N * N * sizeof(double);
    l.off_A = take(nn);
    l.off_V = take(nn);
    l.off_W = take(nn);
    l.off_lam = take((size_t)N * sizeof(double));
    l.off_perm = take((size_t)N * sizeof(int));
    l.off_ews = take(eig_workspace_bytes(N));
  }
  l.tmp = off;
  return l;
}

template <typename T>
int upload(const std::vector<T>& h, T* d, hipStream_t s) {
  if (!h.empty()) MLPCP_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return MLPCP_OK;
}

}  // namespace

size_t operator_bytes(int n, int levels) { return coarse_dim_checked(n, levels) < 1 ? 0 : op_layout(n, levels).kept; }
size_t operator_tmp_bytes(int n, int levels) {
  return coarse_dim_checked(n, levels) < 1 ? 0 : op_layout(n, levels).tmp;
}

int build_operator_at(int n, int levels, int r_norm, hipStream_t stream, Operator* op, void* mem, void* tmpmem) {
  const int nH = coarse_dim_checked(n, levels);
  if (nH < 1) return MLPCP_E_LEVELS;
  const OpLayout l = op_layout(n, levels);
  char* base = static_cast<char*>(mem);
  char* tb = static_cast<char*>(tmpmem);
  op->n = n;
  op->levels = levels;
  op->nH = nH;
  std::vector<int> ri, cp, cr;
  std::vector<float> rw, cw;
  build_stencil_host(n, levels, ri, rw, cp, cr, cw, nullptr);
  int mx = 0;
  for (int c = 0; c < nH; ++c) mx = std::max(mx, cp[c + 1] - cp[c]);
  op->max_col_nnz = mx;
  op->nnz = cp[nH];
  op->contig = true;
  for (int c = 0; c < nH; ++c)
    for (int t = cp[c] + 1; t < cp[c + 1]; ++t) op->contig = op->contig && cr[t] == cr[t - 1] + 1;
  {  // the kernels read exactly kMaxStencil weights per fine row
    std::vector<int> row_cnt(n, 0);
    for (int t = 0; t < op->nnz; ++t) ++row_cnt[cr[t]];
    for (int j = 0; j < n; ++j)
      if (row_cnt[j] > kMaxStencil) return MLPCP_E_UNSUPPORTED;
  }
  op->row_idx = reinterpret_cast<int*>(base + l.off_row_idx);
  op->row_w = reinterpret_cast<float*>(base + l.off_row_w);
  op->col_ptr = reinterpret_cast<int*>(base + l.off_col_ptr);
  op->col_row = reinterpret_cast<int*>(base + l.off_col_row);
  op->col_w = reinterpret_cast<float*>(base + l.off_col_w);
  op->C = levels > 0 ? reinterpret_cast<double*>(base + l.off_C) : nullptr;
  MLPCP_TRY(upload(ri, op->row_idx, stream));
  MLPCP_TRY(upload(rw, op->row_w, stream));
  MLPCP_TRY(upload(cp, op->col_ptr, stream));
  MLPCP_TRY(upload(cr, op->col_row, stream));
  MLPCP_TRY(upload(cw, op->col_w, stream));
  if (levels == 0) {
    MLPCP_HIP(hipStreamSynchronize(stream));   // the host tables go out of scope
    return MLPCP_OK;
  }
  // P^T P from the column lists (exact: dyadic weights), then C = (P^T P)^{-1/2}
  const int N = round_up(nH, kPad);
  std::vector<double> PtP((size_t)N * N, 0.0);
  {
    std::vector<std::vector<std::pair<int, double>>> rowsP(n);
    for (int c = 0; c < nH; ++c)
      for (int t = cp[c]; t < cp[c + 1]; ++t) rowsP[cr[t]].push_back({c, (double)cw[t]});
    for (int j = 0; j < n; ++j)
      for (const auto& a : rowsP[j])
        for (const auto& b : rowsP[j]) PtP[(size_t)a.first * N + b.first] += a.second * b.second;
  }
  double* dA = reinterpret_cast<double*>(tb + l.off_A);
  double* dV = reinterpret_cast<double*>(tb + l.off_V);
  double* dW = reinterpret_cast<double*>(tb + l.off_W);
  double* dlam = reinterpret_cast<double*>(tb + l.off_lam);
  int* dperm = reinterpret_cast<int*>(tb + l.off_perm);
  void* ews = tb + l.off_ews;
  const size_t nn = (size_t)N * N;
  MLPCP_HIP(hipMemcpyAsync(dA, PtP.data(), nn * 8, hipMemcpyHostToDevice, stream));
  int sweeps = 0;
  MLPCP_TRY(eig_sym(nH, N, dA, dV, dlam, dperm, ews, stream, &sweeps, false));
  if (r_norm == 0) {
    const size_t cnt = (size_t)nH * nH;
    hipLaunchKernelGGL(k_scale_cols_invsqrt, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, dV, dlam,
                       N, nH, dW);
    MLPCP_TRY(gemm_f64(false, true, nH, nH, nH, 1.0, dW, N, dV, N, op->C, nH, stream));
  } else {
    // the literal interpolation operator: C = I / ||P||_2 (r_norm 1) or C = I (r_norm 2);
    // ||P||_2^2 is the largest eigenvalue of P^T P
    std::vector<double> hl(N, 0.0);
    MLPCP_HIP(hipMemcpyAsync(hl.data(), dlam, (size_t)N * 8, hipMemcpyDeviceToHost, stream));
    MLPCP_HIP(hipStreamSynchronize(stream));
    double lmax = 0.0;
    for (int i = 0; i < nH; ++i) lmax = std::max(lmax, hl[i]);
    const double sc = r_norm == 1 ? 1.0 / std::sqrt(lmax) : 1.0;
    std::vector<double> hc((size_t)nH * nH, 0.0);
    for (int i = 0; i < nH; ++i) hc[(size_t)i * nH + i] = sc;
    MLPCP_HIP(hipMemcpyAsync(op->C, hc.data(), hc.size() * 8, hipMemcpyHostToDevice, stream));
  }
  if (nH <= kQfWidth) {
    op->Qf = reinterpret_cast<float*>(base + l.off_Qf);
    const int cnt = n * kQfWidth;
    hipLaunchKernelGGL(k_build_Qf, dim3((cnt + 255) / 256), dim3(256), 0, stream, n, nH, op->row_idx, op->row_w,
                       op->C, op->Qf);
    MLPCP_HIP(hipGetLastError());
  }
  MLPCP_HIP(hipStreamSynchronize(stream));
  return MLPCP_OK;
}

namespace {

int build_operator(int n, int levels, int r_norm, hipStream_t stream, Operator* op) {
  const OpLayout l = op_layout(n, levels);
  MLPCP_HIP(hipMalloc(&op->mem, l.kept));
  void* tmp = nullptr;
  if (l.tmp) MLPCP_HIP(hipMalloc(&tmp, l.tmp));
  const int st = build_operator_at(n, levels, r_norm, stream, op, op->mem, tmp);
  if (tmp) (void)hipFree(tmp);
  return st;
}

}  // namespace

int get_operator(int n, int levels, hipStream_t stream, const Operator** out, int r_norm) {
  if (r_norm < 0 || r_norm > 2) return MLPCP_E_UNSUPPORTED;
  int dev = 0;
  MLPCP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_op_mutex);
  auto key = std::make_tuple(dev, n, levels * 4 + r_norm);
  auto it = g_ops.find(key);
  if (it != g_ops.end()) {
    *out = it->second.get();
    return MLPCP_OK;
  }
  std::unique_ptr<Operator, OpDeleter> op(new Operator());
  const int st = build_operator(n, levels, r_norm, stream, op.get());
  if (st != MLPCP_OK) return st;
  *out = op.get();
  g_ops.emplace(key, std::move(op));
  return MLPCP_OK;
}

namespace {

__global__ void k_apply_P(int m, int n, int nH, const float* __restrict__ X, int ldx, float* __restrict__ XP,
                          int ldp, const int* __restrict__ col_ptr, const int* __restrict__ col_row,
                          const float* __restrict__ col_w) {
  const size_t total = (size_t)m * nH;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / nH;
    const int c = (int)(idx % nH);
    const float* x = X + i * ldx;
    float acc = 0.0f;
    for (int t = col_ptr[c]; t < col_ptr[c + 1]; ++t) acc = fmaf(col_w[t], x[col_row[t]], acc);
    XP[i * ldp + c] = acc;
  }
}

__global__ void k_apply_Pt(int m, int n, const float* __restrict__ Nm, int ldn, float* __restrict__ X, int ldx,
                           const int* __restrict__ row_idx, const float* __restrict__ row_w) {
  const size_t total = (size_t)m * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / n;
    const int j = (int)(idx % n);
    const float* y = Nm + i * ldn;
    float acc = 0.0f;
#pragma unroll
    for (int s = 0; s < kMaxStencil; ++s) acc = fmaf(row_w[j * kMaxStencil + s], y[row_idx[j * kMaxStencil + s]], acc);
    X[i * ldx + j] = acc;
  }
}

unsigned stream_grid(size_t total) {
  size_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

static_assert(kMaxStencil == 2, "the streaming prolongation reads two weights per fine row");

// Fallback for coarse widths whose float64 tiles do not fit the streaming kernels' LDS:
// XH rows = (X rows P) C for RROWS rows per block, accumulated in float64.
constexpr int RROWS = 8;
__global__ void __launch_bounds__(256) k_restrict_full(int m, int n, int nH, const float* __restrict__ X, int ldx,
                                                       float* __restrict__ XH, int ldh,
                                                       const int* __restrict__ col_ptr,
                                                       const int* __restrict__ col_row,
                                                       const float* __restrict__ col_w,
                                                       const double* __restrict__ C) {
  extern __shared__ double smem[];  // [RROWS][nH]
  const int i0 = blockIdx.x * RROWS;
  const int rows = min(RROWS, m - i0);
  for (int e = threadIdx.x; e < rows * nH; e += blockDim.x) {
    const int r = e / nH, c = e % nH;
    const float* x = X + (size_t)(i0 + r) * ldx;
    double acc = 0.0;
    for (int t = col_ptr[c]; t < col_ptr[c + 1]; ++t) acc += (double)col_w[t] * (double)x[col_row[t]];
    smem[r * nH + c] = acc;
  }
  __syncthreads();
  for (int c2 = threadIdx.x; c2 < nH; c2 += blockDim.x) {
    double acc[RROWS];
#pragma unroll
    for (int r = 0; r < RROWS; ++r) acc[r] = 0.0;
    for (int c1 = 0; c1 < nH; ++c1) {
      const double w = C[(size_t)c1 * nH + c2];
#pragma unroll
      for (int r = 0; r < RROWS; ++r) acc[r] += smem[(r < rows ? r : 0) * nH + c1] * w;
    }
    for (int r = 0; r < rows; ++r) XH[(size_t)(i0 + r) * ldh + c2] = (float)acc[r];
  }
}

// X rows = (XH rows C) P^T
__global__ void __launch_bounds__(256) k_prolong_full(int m, int n, int nH, const float* __restrict__ XH, int ldh,
                                                      float* __restrict__ X, int ldx,
                                                      const int* __restrict__ row_idx,
                                                      const float* __restrict__ row_w,
                                                      const double* __restrict__ C) {
  extern __shared__ double smem[];  // [2][RROWS][nH]
  double* sx = smem;
  double* sn = smem + RROWS * nH;
  const int i0 = blockIdx.x * RROWS;
  const int rows = min(RROWS, m - i0);
  for (int e = threadIdx.x; e < rows * nH; e += blockDim.x) {
    const int r = e / nH, c = e % nH;
    sx[r * nH + c] = (double)XH[(size_t)(i0 + r) * ldh + c];
  }
  __syncthreads();
  for (int c2 = threadIdx.x; c2 < nH; c2 += blockDim.x) {
    double acc[RROWS];
#pragma unroll
    for (int r = 0; r < RROWS; ++r) acc[r] = 0.0;
    for (int c1 = 0; c1 < nH; ++c1) {
      const double w = C[(size_t)c1 * nH + c2];  // C symmetric
#pragma unroll
      for (int r = 0; r < RROWS; ++r) acc[r] += sx[(r < rows ? r : 0) * nH + c1] * w;
    }
    for (int r = 0; r < rows; ++r) sn[r * nH + c2] = acc[r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * n; e += blockDim.x) {
    const int r = e / n, j = e % n;
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < kMaxStencil; ++s)
      acc += (double)row_w[j * kMaxStencil + s] * sn[r * nH + row_idx[j * kMaxStencil + s]];
    X[(size_t)(i0 + r) * ldx + j] = (float)acc;
  }
}

// S_tau[x] = sign(x) max(|x| - tau, 0); NaN propagates.
__device__ __forceinline__ float shrink1(float x, float tau) {
  const float a = fabsf(x) - tau;
  return (a > 0.0f) ? copysignf(a, x) : ((a == a) ? 0.0f : a);
}

__global__ void k_shrink(size_t count, const float* __restrict__ X, float tau, float* __restrict__ Y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    Y[i] = shrink1(X[i], tau);
}

// the same on 16-byte groups (X and Y 16-byte aligned): one float4 load and store per
// thread and step, the grid sized to a few blocks per compute unit
__global__ void __launch_bounds__(256) k_shrink4(size_t n4, const float4* __restrict__ X, float tau,
                                                 float4* __restrict__ Y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
    const float4 x = X[i];
    Y[i] = make_float4(shrink1(x.x, tau), shrink1(x.y, tau), shrink1(x.z, tau), shrink1(x.w, tau));
  }
}

// ---- streaming restriction and prolongation (the standalone entry points) ----------
// A block takes a tile of R rows.  Restriction: the R rows of X are staged in LDS with
// coalesced (float4 where aligned) loads, Y = X_tile P is formed in float64 from the
// column stencil, and XH_tile = Y C on float64 MFMA (v_mfma_f64_16x16x4f64, 16 x 16 output
// tiles over the four waves; Y padded to 16-row multiples and 16-column multiples with
// zeros, C read from global memory, where it stays cached).  Prolongation: the XH tile is
// staged (as float64), W = XH_tile C on MFMA, and X_tile = W P^T through the two-tap row
// stencil, written with coalesced (float4 where aligned) stores.
typedef double sd4_t __attribute__((ext_vector_type(4)));

// Z = Y C for Y (R16 x nHp, LDS, ld ldy, zero beyond the valid rows and columns) and C
// (nH x nH, global, ld nH); out(row, col, value) for every row < R16 and col < nHp.
template <typename F>
__device__ __forceinline__ void tile_times_C(const double* sY, int ldy, int R16, int nH, int nHp,
                                             const double* __restrict__ C, F out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rt = R16 / 16, ct = nHp / 16;
  const int K4 = (nH + 3) & ~3;
  for (int t = wave; t < rt * ct; t += 4) {
    const int ti = t / ct, tj = t % ct;
    const int col = tj * 16 + (lane & 15);
    sd4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K4; k0 += 4) {
      const int k = k0 + (lane >> 4);
      const double a = sY[(ti * 16 + (lane & 15)) * ldy + k];
      const double b = (k < nH && col < nH) ? C[(size_t)k * nH + col] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    // output register v of lane l: row 4v + l/16, column l%16 of the tile
#pragma unroll
    for (int v = 0; v < 4; ++v) out(ti * 16 + 4 * v + (lane >> 4), col, acc[v]);
  }
}

struct StreamPlan {
  int R, R16, nHp, ldy;   // rows per tile, rows padded to 16, n_H padded to 16, LDS ld of the float64 tiles
  size_t off_tab;         // byte offset of the stencil tables in the dynamic LDS
  size_t lds;             // dynamic LDS bytes
};

// Rows per tile for the streaming kernels: as many (up to 64) as the LDS budget allows,
// with the stencil tables staged too.  Restriction: the float64 Y tile, the float32 row
// tile and the column stencil (col_ptr, col_row, col_w); prolongation: the float64 XH
// and W tiles and the row stencil (row_idx, row_w).
bool stream_plan(int n, int nH, bool prolong, StreamPlan& sp) {
  constexpr size_t kBudget = 64 * 1024;
  sp.nHp = (nH + 15) / 16 * 16;
  sp.ldy = sp.nHp + 1;   // odd stride in doubles: MFMA operand reads across rows hit distinct banks
  const size_t tab = prolong ? (size_t)kMaxStencil * n * (sizeof(int) + sizeof(float))
                             : (size_t)(nH + 1) * sizeof(int) + (size_t)kMaxStencil * n * (sizeof(int) + sizeof(float));
  // restriction: at most 32 rows (about 34 KB at n = 200, so four blocks share a compute
  // unit and their loads overlap the others' arithmetic); prolongation: up to 64
  for (int R = prolong ? 64 : 32; R >= 1; R /= 2) {
    const int R16 = (R + 15) / 16 * 16;
    const size_t tiles = (size_t)(prolong ? 2 : 1) * R16 * sp.ldy * sizeof(double);
    const size_t rows = prolong ? 0 : (size_t)R * (n | 1) * sizeof(float);
    const size_t off_tab = (tiles + rows + 15) & ~size_t(15);
    if (off_tab + tab <= kBudget) {
      sp.R = R;
      sp.R16 = R16;
      sp.off_tab = off_tab;
      sp.lds = off_tab + tab;
      return true;
    }
  }
  return false;
}

// XH (m x nH) = X (m x n) P C
template <bool VEC>
__global__ void __launch_bounds__(256) k_restrict_stream(int m, int n, int nH, int R, int R16, int nHp, int ldy,
                                                         int off_tab, int nnz, const float* __restrict__ X, int ldx,
                                                         float* __restrict__ XH, int ldh,
                                                         const int* __restrict__ col_ptr,
                                                         const int* __restrict__ col_row,
                                                         const float* __restrict__ col_w,
                                                         const double* __restrict__ C) {
  extern __shared__ double dsm[];
  double* sY = dsm;                                              // R16 x ldy
  float* sX = reinterpret_cast<float*>(dsm + (size_t)R16 * ldy);   // R x n
  char* tb = reinterpret_cast<char*>(dsm) + off_tab;
  int* sptr = reinterpret_cast<int*>(tb);                        // nH + 1
  int* srow = sptr + (nH + 1);                                   // nnz
  float* sw = reinterpret_cast<float*>(srow + nnz);              // nnz
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * R;
  const int rows = min(R, m - i0);
  // 1. stage the rows (all loads issued before the first use) and the column stencil;
  //    the LDS row stride ls = n | 1 is odd, so the lanes of step 2, one row each, read
  //    the same fine column of different rows from different banks
  const int ls = n | 1;
  if (VEC) {
    const int n4 = n / 4;
    for (int e = tid; e < rows * n4; e += 256) {
      const int r = e / n4, q = e % n4;
      const float4 v = *reinterpret_cast<const float4*>(X + (size_t)(i0 + r) * ldx + 4 * q);
      float* d = sX + (size_t)r * ls + 4 * q;
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    }
  } else {
    for (int e = tid; e < rows * n; e += 256) {
      const int r = e / n, j = e % n;
      sX[(size_t)r * ls + j] = X[(size_t)(i0 + r) * ldx + j];
    }
  }
  for (int e = tid; e <= nH; e += 256) sptr[e] = col_ptr[e];
  for (int e = tid; e < nnz; e += 256) {
    srow[e] = col_row[e];
    sw[e] = col_w[e];
  }
  __syncthreads();
  // 2. Y = X_tile P (float64), zero in the padding.  Lane l of a wave takes row l % 32;
  //    the wave's two halves and the four waves split the coarse columns (c = h + 2 w + 8 k),
  //    so the 32 lanes of a half read the same stencil entry (broadcast) and one fine
  //    column of 32 rows (distinct banks).  Rows r >= R16 (a 16-row tile) are skipped.
  {
    const int lane = tid & 63, w = tid >> 6;
    const int half = lane >> 5, rl = lane & 31;
    for (int rb = 0; rb < R16; rb += 32) {
      const int r = rb + rl;
      const bool live = r < rows;
      const float* x = sX + (size_t)(live ? r : 0) * ls;
      for (int c = half + 2 * w; r < R16 && c < nHp; c += 8) {
        double acc = 0.0;
        if (c < nH && live) {
          const int t1 = sptr[c + 1];
          for (int t = sptr[c]; t < t1; ++t) acc = fma((double)sw[t], (double)x[srow[t]], acc);
        }
        sY[(size_t)r * ldy + c] = acc;
      }
    }
  }
  __syncthreads();
  // 3. XH_tile = Y C on MFMA
  tile_times_C(sY, ldy, R16, nH, nHp, C, [&](int r, int c, double v) {
    if (r < rows && c < nH) XH[(size_t)(i0 + r) * ldh + c] = (float)v;
  });
}

// Persistent restriction for float4-aligned rows whose tile and C fit the LDS together,
// for stencils whose columns have contiguous supports (true of the composite linear
// interpolation: column c of P touches the fine rows lo_c .. lo_c + cnt_c - 1).
// Each block walks the tiles blockIdx.x, blockIdx.x + gridDim.x, ...; the rows of the
// next tile are loaded into registers (kPipeChunks float4 per thread) before the current
// tile's stencil and MFMA work, so every wave keeps several HBM reads in flight through
// the arithmetic.  C is staged once per block in LDS (K4 x ldc, zero padded), which keeps
// the MFMA operand reads off the in-order vector-memory counter that the prefetch holds.
// The column weights are staged as float64, zero padded to W8 (a multiple of 8) per
// column, so a lane reads eight row entries at constant offsets from one base address
// and eight broadcast weights per step.
constexpr int kPipeChunks = 8;

__global__ void __launch_bounds__(256) k_restrict_pipe(int m, int n, int nH, int R, int R16, int nHp, int ldy,
                                                       int ldc, int W8, int off_c, int off_tab,
                                                       const float* __restrict__ X, int ldx, float* __restrict__ XH,
                                                       int ldh, const int* __restrict__ col_ptr,
                                                       const int* __restrict__ col_row,
                                                       const float* __restrict__ col_w,
                                                       const double* __restrict__ C) {
  extern __shared__ double dsm[];
  double* sY = dsm;                                              // R16 x ldy
  float* sX = reinterpret_cast<float*>(dsm + (size_t)R16 * ldy);   // R x (n | 1), then W8 spare
  double* sC = reinterpret_cast<double*>(reinterpret_cast<char*>(dsm) + off_c);   // K4 x ldc
  double* sw = reinterpret_cast<double*>(reinterpret_cast<char*>(dsm) + off_tab);   // nH x W8
  int* slo = reinterpret_cast<int*>(sw + (size_t)nH * W8);                          // nH
  int* scnt = slo + nH;                                                             // nH
  const int tid = threadIdx.x;
  const int n4 = n >> 2, ls = n | 1;
  const int K4 = (nH + 3) & ~3;
  const int ntiles = (m + R - 1) / R;
  for (int c = tid; c < nH; c += 256) {
    const int t0 = col_ptr[c];
    slo[c] = col_row[t0];
    scnt[c] = col_ptr[c + 1] - t0;
  }
  for (int e = tid; e < nH * W8; e += 256) {
    const int c = e / W8, k = e % W8;
    const int t0 = col_ptr[c];
    sw[e] = k < col_ptr[c + 1] - t0 ? (double)col_w[t0 + k] : 0.0;
  }
  for (int e = tid; e < K4 * nHp; e += 256) {
    const int k = e / nHp, c = e % nHp;
    sC[(size_t)k * ldc + c] = (k < nH && c < nH) ? C[(size_t)k * nH + c] : 0.0;
  }
  float4 buf[kPipeChunks];
  auto load = [&](int tile) {
    const int i0 = tile * R, cnt = min(R, m - i0) * n4;
#pragma unroll
    for (int k = 0; k < kPipeChunks; ++k) {
      const int e = tid + 256 * k;
      if (e < cnt) buf[k] = *reinterpret_cast<const float4*>(X + (size_t)(i0 + e / n4) * ldx + 4 * (e % n4));
    }
  };
  int tile = blockIdx.x;
  if (tile < ntiles) load(tile);
  const int lane = tid & 63, w = tid >> 6;
  for (; tile < ntiles; tile += gridDim.x) {
    const int i0 = tile * R, rows = min(R, m - i0), cnt = rows * n4;
#pragma unroll
    for (int k = 0; k < kPipeChunks; ++k) {
      const int e = tid + 256 * k;
      if (e < cnt) {
        float* d = sX + (size_t)(e / n4) * ls + 4 * (e % n4);
        d[0] = buf[k].x;
        d[1] = buf[k].y;
        d[2] = buf[k].z;
        d[3] = buf[k].w;
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) load(tile + gridDim.x);
    // Y = X_tile P in float64 (lane layout as in k_restrict_stream): eight entries per
    // step; beyond cnt_c the weight is zero and the row value is replaced by zero, so
    // the spare reads past the support (inside the tile buffer) never reach the sum
    {
      const int half = lane >> 5, rl = lane & 31;
      for (int rb = 0; rb < R16; rb += 32) {
        const int r = rb + rl;
        const bool live = r < rows;
        for (int c = half + 2 * w; r < R16 && c < nHp; c += 8) {
          double acc = 0.0;
          if (c < nH && live) {
            const int cnt = scnt[c];
            const float* x = sX + (size_t)r * ls + slo[c];
            const double* wc = sw + (size_t)c * W8;
            for (int k = 0; k < cnt; k += 8) {
              float xv[8];
              double wv[8];
#pragma unroll
              for (int i = 0; i < 8; ++i) {
                xv[i] = x[k + i];
                wv[i] = wc[k + i];
              }
#pragma unroll
              for (int i = 0; i < 8; ++i) acc = fma(wv[i], k + i < cnt ? (double)xv[i] : 0.0, acc);
            }
          }
          sY[(size_t)r * ldy + c] = acc;
        }
      }
    }
    __syncthreads();
    // XH_tile = Y C on float64 MFMA, both operands from LDS
    {
      const int rt = R16 / 16, ct = nHp / 16;
      for (int t = w; t < rt * ct; t += 4) {
        const int ti = t / ct, tj = t % ct;
        const int col = tj * 16 + (lane & 15);
        const double* a = sY + (size_t)(ti * 16 + (lane & 15)) * ldy + (lane >> 4);
        const double* b = sC + (size_t)(lane >> 4) * ldc + col;
        sd4_t acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < K4; k0 += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k0], b[(size_t)k0 * ldc], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = ti * 16 + 4 * v + (lane >> 4);
          if (r < rows && col < nH) XH[(size_t)(i0 + r) * ldh + col] = (float)acc[v];
        }
      }
    }
    __syncthreads();
  }
}

// LDS plan of k_restrict_pipe: R rows with R * n / 4 <= 256 * kPipeChunks (the tile
// plus W8 spare floats), C (K4 x (nHp + 1) doubles) and the tables (nH x W8 float64
// weights, lo_c and cnt_c).  False if nothing fits.
struct PipePlan {
  int R, R16, nHp, ldy, ldc, W8;
  size_t off_c, off_tab, lds;
};

bool pipe_plan(int n, int nH, int max_col_nnz, PipePlan& pp) {
  constexpr size_t kBudget = 64 * 1024;
  if (n % 4) return false;
  pp.nHp = (nH + 15) / 16 * 16;
  pp.ldy = pp.nHp + 1;
  pp.ldc = pp.nHp + 1;
  pp.W8 = (max_col_nnz + 7) / 8 * 8;
  const int K4 = (nH + 3) & ~3;
  const size_t tab = (size_t)nH * pp.W8 * sizeof(double) + (size_t)2 * nH * sizeof(int);
  const size_t cbytes = (size_t)K4 * pp.ldc * sizeof(double);
  int R = (256 * kPipeChunks) / (n / 4);
  if (R > 32) R = 32;
  for (; R >= 16; R /= 2) {
    const int R16 = (R + 15) / 16 * 16;
    const size_t xs = ((size_t)R * (n | 1) + pp.W8) * sizeof(float);
    const size_t off_c = (size_t)R16 * pp.ldy * sizeof(double) + ((xs + 15) & ~size_t(15));
    const size_t off_tab = off_c + cbytes;
    if (off_tab + tab <= kBudget) {
      pp.R = R;
      pp.R16 = R16;
      pp.off_c = off_c;
      pp.off_tab = off_tab;
      pp.lds = off_tab + tab;
      return true;
    }
  }
  return false;
}

// ---- restriction at coarse widths up to 16: the dense operator P C on float32 MFMA ----
// The restriction is then a product with an n x 16 matrix, which each wave keeps in
// registers as MFMA operand fragments for the whole launch; the data rows go from HBM
// straight to registers, with no LDS and no barrier, so a wave's whole tile is in flight
// at once, and the waves loop over 16-row tiles.  v_mfma_f32_16x16x4f32: lane l supplies
// A[l%16][k] and B[k][l%16] for its k of the step, and receives D[4(l/16) + v][l%16],
// v < 4.  Float32 accumulation (the output is float32): relative error about 1e-7
// against the float64 products at n = 200.  (The prolongation keeps the LDS-staged
// kernel: from registers its stores cover 64 bytes of each of 16 rows per instruction,
// which measured slower, 4.9 against 5.6 TB/s with the operand cache-resident, than
// whole staged rows.)
typedef float f4_t __attribute__((ext_vector_type(4)));

// XH (m x nH) = X (m x n) Qf: D = XH^T tile (coarse c x 16 rows) = Qf^T X^T.  Step (s, t)
// of lane group g = l/16 contracts the fine index k = 16 s + 4 g + t, so one float4 load
// per s gives a lane its four B operands; the A fragments qa[s][t] = Qf[k][l%16] follow
// the same order.
__global__ void __launch_bounds__(256) k_restrict_mfma(int m, int n, int nH, const float* __restrict__ X, int ldx,
                                                       float* __restrict__ XH, int ldh, const float* __restrict__ Qf) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int S = (n + 15) >> 4;   // at most 16 (n <= 256)
  // qa[s][t] = (P C)[16 s + 4 g + t][c] = QfT[c][16 s + 4 g + t]: one float4
  const float* QfT = Qf;
  float4 qa[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int k0 = 16 * s + 4 * g;
    qa[s] = (s < S && k0 < n) ? *reinterpret_cast<const float4*>(QfT + (size_t)c * n + k0)
                              : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  const int tiles = (m + 15) >> 4;
  const int nw = gridDim.x * 4;
  for (int tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles; tile += nw) {
    const int row = tile * 16 + c;
    float4 xv[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k0 = 16 * s + 4 * g;
      xv[s] = (s < S && k0 < n && row < m) ? *reinterpret_cast<const float4*>(X + (size_t)row * ldx + k0)
                                           : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    f4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (s < S) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[s].x, xv[s].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[s].y, xv[s].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[s].z, xv[s].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[s].w, xv[s].w, acc, 0, 0, 0);
      }
    }
    // lane l holds XH[row][4g + v]
    if (row < m) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (4 * g + v < nH) XH[(size_t)row * ldh + 4 * g + v] = acc[v];
    }
  }
}

// X (m x n) = XH (m x nH) C P^T
template <bool VEC>
__global__ void __launch_bounds__(256) k_prolong_stream(int m, int n, int nH, int R, int R16, int nHp, int ldy,
                                                        int off_tab, const float* __restrict__ XH, int ldh,
                                                        float* __restrict__ X, int ldx,
                                                        const int* __restrict__ row_idx,
                                                        const float* __restrict__ row_w,
                                                        const double* __restrict__ C) {
  extern __shared__ double dsm[];
  double* sW = dsm;                        // R16 x ldy: the XH tile
  double* sN = dsm + (size_t)R16 * ldy;    // R16 x ldy: W = XH_tile C
  char* tb = reinterpret_cast<char*>(dsm) + off_tab;
  int* sri = reinterpret_cast<int*>(tb);                  // 2 n
  float* srw = reinterpret_cast<float*>(sri + 2 * n);     // 2 n
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * R;
  const int rows = min(R, m - i0);
  for (int e = tid; e < R16 * nHp; e += 256) {
    const int r = e / nHp, c = e % nHp;
    sW[(size_t)r * ldy + c] = (r < rows && c < nH) ? (double)XH[(size_t)(i0 + r) * ldh + c] : 0.0;
  }
  for (int e = tid; e < 2 * n; e += 256) {
    sri[e] = row_idx[e];
    srw[e] = row_w[e];
  }
  __syncthreads();
  tile_times_C(sW, ldy, R16, nH, nHp, C, [&](int r, int c, double v) { sN[(size_t)r * ldy + c] = v; });
  __syncthreads();
  if (VEC) {
    const int n4 = n / 4;
    for (int e = tid; e < rows * n4; e += 256) {
      const int r = e / n4, j0 = 4 * (e % n4);
      const double* w = sN + (size_t)r * ldy;
      // the eight stencil entries of the four columns with two 16-byte LDS reads each
      // (consecutive lanes read consecutive 32-byte runs)
      const int4 ia = *reinterpret_cast<const int4*>(sri + 2 * j0), ib = *reinterpret_cast<const int4*>(sri + 2 * j0 + 4);
      const float4 wa = *reinterpret_cast<const float4*>(srw + 2 * j0),
                   wb = *reinterpret_cast<const float4*>(srw + 2 * j0 + 4);
      float o[4];
      o[0] = (float)fma((double)wa.y, w[ia.y], (double)wa.x * w[ia.x]);
      o[1] = (float)fma((double)wa.w, w[ia.w], (double)wa.z * w[ia.z]);
      o[2] = (float)fma((double)wb.y, w[ib.y], (double)wb.x * w[ib.x]);
      o[3] = (float)fma((double)wb.w, w[ib.w], (double)wb.z * w[ib.z]);
      *reinterpret_cast<float4*>(X + (size_t)(i0 + r) * ldx + j0) = make_float4(o[0], o[1], o[2], o[3]);
    }
  } else {
    for (int e = tid; e < rows * n; e += 256) {
      const int r = e / n, j = e % n;
      const double* w = sN + (size_t)r * ldy;
      X[(size_t)(i0 + r) * ldx + j] =
          (float)fma((double)srw[2 * j + 1], w[sri[2 * j + 1]], (double)srw[2 * j] * w[sri[2 * j]]);
    }
  }
}

// blocks of four waves for the register-operator kernels: one wave per 16-row tile up to
// a few waves per SIMD on every compute unit, the waves then looping over the tiles (the
// operator fragments are loaded once per wave)
unsigned mfma_grid(int tiles) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 256;
  const int blocks = (tiles + 3) / 4;
  return (unsigned)std::max(1, std::min(blocks, 8 * cus));
}

__global__ void k_copy_rows(int m, int n, const float* __restrict__ X, int ldx, float* __restrict__ Y, int ldy) {
  const size_t total = (size_t)m * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t i = idx / n;
    const int j = (int)(idx % n);
    Y[i * ldy + j] = X[i * ldx + j];
  }
}

}  // namespace

int apply_P(const Operator& op, int m, const float* X, int ldx, float* XP, int ldp, hipStream_t s) {
  const size_t total = (size_t)m * op.nH;
  if (total == 0) return MLPCP_OK;
  hipLaunchKernelGGL(k_apply_P, dim3(stream_grid(total)), dim3(256), 0, s, m, op.n, op.nH, X, ldx, XP, ldp,
                     op.col_ptr, op.col_row, op.col_w);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int apply_Pt(const Operator& op, int m, const float* Nm, int ldn, float* X, int ldx, hipStream_t s) {
  const size_t total = (size_t)m * op.n;
  if (total == 0) return MLPCP_OK;
  hipLaunchKernelGGL(k_apply_Pt, dim3(stream_grid(total)), dim3(256), 0, s, m, op.n, Nm, ldn, X, ldx, op.row_idx,
                     op.row_w);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

}  // namespace mlpcp

using namespace mlpcp;

extern "C" {

void mlpcp_default_opts(mlpcp_opts* o) {
  if (!o) return;
  o->levels = 0;
  o->tol = 1e-6;
  o->max_iter = 500;
  o->rho = 1.5;
  o->mu_max_factor = 1e7;
  o->prec = MLPCP_FP32;
  o->check_every = 1;
  o->r_norm = 0;
  o->svt_method = 0;
}

int mlpcp_coarse_dim(int n, int levels) { return coarse_dim_checked(n, levels); }

const char* mlpcp_status_string(int s) {
  switch (s) {
    case MLPCP_OK: return "ok";
    case MLPCP_NOT_CONVERGED: return "not converged: max_iter reached (outputs valid)";
    case MLPCP_E_INVALID_ARG: return "invalid argument";
    case MLPCP_E_SHAPE: return "invalid shape or leading dimension";
    case MLPCP_E_LEVELS: return "invalid number of levels for this width";
    case MLPCP_E_NONFINITE: return "feasibility gap became non-finite";
    case MLPCP_E_EIG: return "eigensolver did not converge within its sweep cap";
    case MLPCP_E_WORKSPACE: return "workspace too small";
    case MLPCP_E_HIP: return "HIP runtime error";
    case MLPCP_E_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

int mlpcp_shrink(size_t count, const float* X, float tau, float* Y, void* stream) {
  if ((count > 0 && (!X || !Y)) || !(tau >= 0.0f) || std::isinf(tau)) return MLPCP_E_INVALID_ARG;
  if (count == 0) return MLPCP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool vec = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15u) == 0;
  const size_t n4 = vec ? count / 4 : 0;
  if (n4) {
    const unsigned grid = (unsigned)std::min<size_t>((n4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_shrink4, dim3(grid), dim3(256), 0, s, n4, reinterpret_cast<const float4*>(X), tau,
                       reinterpret_cast<float4*>(Y));
  }
  if (count > 4 * n4)
    hipLaunchKernelGGL(k_shrink, dim3(stream_grid(count - 4 * n4)), dim3(256), 0, s, count - 4 * n4, X + 4 * n4, tau,
                       Y + 4 * n4);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int mlpcp_restrict(int m, int n, const float* X, int ldx, int levels, float* XH, int ldh, void* stream) {
  if (m < 0 || n < 1) return MLPCP_E_SHAPE;
  const int nH = coarse_dim_checked(n, levels);
  if (nH < 1) return MLPCP_E_LEVELS;
  if (ldx < n || ldh < nH) return MLPCP_E_SHAPE;
  if (m > 0 && (!X || !XH)) return MLPCP_E_INVALID_ARG;
  if (m == 0) return MLPCP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (levels == 0) {
    hipLaunchKernelGGL(k_copy_rows, dim3(stream_grid((size_t)m * n)), dim3(256), 0, s, m, n, X, ldx, XH, ldh);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, levels, s, &op));
  const bool vec = n % 4 == 0 && ldx % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  if (vec && op->Qf && n <= 256) {
    const int tiles = (m + 15) / 16;
    hipLaunchKernelGGL(k_restrict_mfma, dim3(mfma_grid(tiles)), dim3(256), 0, s, m, n, nH, X, ldx, XH, ldh, op->Qf);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  PipePlan pp;
  if (vec && op->contig && pipe_plan(n, nH, op->max_col_nnz, pp)) {
    const int ntiles = (m + pp.R - 1) / pp.R;
    int per_cu = 0, cus = 0, dev = 0;
    MLPCP_HIP(hipGetDevice(&dev));
    MLPCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MLPCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_restrict_pipe, 256, pp.lds));
    const int grid = std::max(1, std::min(ntiles, std::max(per_cu, 1) * std::max(cus, 1)));
    hipLaunchKernelGGL(k_restrict_pipe, dim3(grid), dim3(256), pp.lds, s, m, n, nH, pp.R, pp.R16, pp.nHp, pp.ldy,
                       pp.ldc, pp.W8, (int)pp.off_c, (int)pp.off_tab, X, ldx, XH, ldh, op->col_ptr, op->col_row,
                       op->col_w, op->C);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  StreamPlan sp;
  if (stream_plan(n, nH, false, sp)) {
    auto fn = vec ? k_restrict_stream<true> : k_restrict_stream<false>;
    hipLaunchKernelGGL(fn, dim3((m + sp.R - 1) / sp.R), dim3(256), sp.lds, s, m, n, nH, sp.R, sp.R16, sp.nHp, sp.ldy,
                       (int)sp.off_tab, op->nnz, X, ldx, XH, ldh, op->col_ptr, op->col_row, op->col_w, op->C);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  const size_t sm = (size_t)RROWS * nH * sizeof(double);
  if (sm > 64 * 1024) return MLPCP_E_UNSUPPORTED;
  hipLaunchKernelGGL(k_restrict_full, dim3((m + RROWS - 1) / RROWS), dim3(256), sm, s, m, n, nH, X, ldx, XH, ldh,
                     op->col_ptr, op->col_row, op->col_w, op->C);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

int mlpcp_prolong(int m, int n, const float* XH, int ldh, int levels, float* X, int ldx, void* stream) {
  if (m < 0 || n < 1) return MLPCP_E_SHAPE;
  const int nH = coarse_dim_checked(n, levels);
  if (nH < 1) return MLPCP_E_LEVELS;
  if (ldx < n || ldh < nH) return MLPCP_E_SHAPE;
  if (m > 0 && (!X || !XH)) return MLPCP_E_INVALID_ARG;
  if (m == 0) return MLPCP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (levels == 0) {
    hipLaunchKernelGGL(k_copy_rows, dim3(stream_grid((size_t)m * n)), dim3(256), 0, s, m, n, XH, ldh, X, ldx);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  const Operator* op = nullptr;
  MLPCP_TRY(get_operator(n, levels, s, &op));
  StreamPlan sp;
  if (stream_plan(n, nH, true, sp)) {
    const bool vec = n % 4 == 0 && ldx % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
    auto fn = vec ? k_prolong_stream<true> : k_prolong_stream<false>;
    hipLaunchKernelGGL(fn, dim3((m + sp.R - 1) / sp.R), dim3(256), sp.lds, s, m, n, nH, sp.R, sp.R16, sp.nHp, sp.ldy,
                       (int)sp.off_tab, XH, ldh, X, ldx, op->row_idx, op->row_w, op->C);
    MLPCP_HIP(hipGetLastError());
    return MLPCP_OK;
  }
  const size_t sm = (size_t)2 * RROWS * nH * sizeof(double);
  if (sm > 64 * 1024) return MLPCP_E_UNSUPPORTED;
  hipLaunchKernelGGL(k_prolong_full, dim3((m + RROWS - 1) / RROWS), dim3(256), sm, s, m, n, nH, XH, ldh, X, ldx,
                     op->row_idx, op->row_w, op->C);
  MLPCP_HIP(hipGetLastError());
  return MLPCP_OK;
}

}  // extern "C"
