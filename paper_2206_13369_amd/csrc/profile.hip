// Optional kernel timing: HIP events recorded on the launching stream around the
// kernels of the selected classes, accumulated per class.  Off by default; when off
// the hooks cost one relaxed atomic load.
#include "profile.h"

#include <atomic>
#include <mutex>
#include <vector>

namespace mlpcp {

namespace {

const char* kNames[KC_COUNT] = {"init_restrict", "gram", "coarse_CGC", "jacobi_pairs", "jacobi_apply",
                                "jacobi_misc", "svt_prep", "epilogue", "reduce", "finalize", "coarse_svt_small",
                                "fw_pass", "fw_power", "fw_small", "fw_top", "msvt_mm", "recon_gemm", "other"};

struct Pending {
  int cls;
  hipEvent_t a, b;
};

std::atomic<int> g_mask{0};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
long long g_launches[KC_COUNT];
double g_ms[KC_COUNT];
thread_local int t_cls = -1;
thread_local hipEvent_t t_start = nullptr;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

void prof_begin(int cls, hipStream_t s) {
  if (!((g_mask.load(std::memory_order_relaxed) >> cls) & 1)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = get_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  t_cls = cls;
  t_start = e;
}

void prof_end(int cls, hipStream_t s) {
  if (!((g_mask.load(std::memory_order_relaxed) >> cls) & 1) || t_start == nullptr || t_cls != cls) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = get_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_pending.push_back({cls, t_start, e});
  t_start = nullptr;
  t_cls = -1;
}

ProfKernel::ProfKernel(int c) : cls(c) {
  if (!((g_mask.load(std::memory_order_relaxed) >> cls) & 1)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  start = get_event();
  stop = get_event();
  if (!start || !stop) {
    if (start) g_pool.push_back(start);
    if (stop) g_pool.push_back(stop);
    start = stop = nullptr;
  }
}

ProfKernel::~ProfKernel() {
  if (!start) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({cls, start, stop});
}

void prof_drain() {
  if (!g_mask.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Pending& p : g_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_ms[p.cls] += ms;
      g_launches[p.cls] += 1;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}

}  // namespace mlpcp

using namespace mlpcp;

extern "C" {

int mlpcp_profile_enable(int mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < KC_COUNT; ++i) {
    g_launches[i] = 0;
    g_ms[i] = 0.0;
  }
  for (const Pending& p : g_pending) {
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
  g_mask.store(mask);
  return MLPCP_OK;
}

int mlpcp_profile_read(mlpcp_kernel_time* out, int cap) {
  prof_drain();
  std::lock_guard<std::mutex> lk(g_mu);
  const int k = cap < KC_COUNT ? cap : KC_COUNT;
  for (int i = 0; i < k && out; ++i) {
    out[i].name = kNames[i];
    out[i].launches = g_launches[i];
    out[i].total_ms = g_ms[i];
  }
  return KC_COUNT;
}

}  // extern "C"
