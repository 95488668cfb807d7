// Event-based per-kernel-class timing (negf_profile_enable / negf_profile_read)
// and the small host/device runtime helpers the orchestration uses.
#include "../../include/negf.h"
#include "internal.h"

#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

using namespace negf;

namespace {


struct ProfRec {
  hipEvent_t a, b;
  int cls;
  double flops, bytes;
};
std::mutex g_prof_mu;
// read on every launch without the lock (atomics: another thread may switch profiling meanwhile)
std::atomic<bool> g_prof_on{false};
std::atomic<unsigned> g_prof_mask{~0u}; // kernel classes whose launches get timing events
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
negf_kernel_stats g_prof_acc[KC_COUNT];
thread_local hipEvent_t t_open = nullptr;
thread_local bool g_capturing = false;   // no timing events inside a captured graph

hipEvent_t pool_get() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Executed flops per kernel class, counted by the kernels themselves while
// profiling is on (a launch's work depends on device data: the active masks of
// the decimation and the zero-slab maps), striped over PROF_SLOTS counters per
// class so that concurrent waves rarely add to the same address.
__device__ unsigned long long g_prof_flops[KC_COUNT * PROF_SLOTS];
std::atomic<unsigned long long*> g_prof_flops_ptr{nullptr};   // published before g_prof_on

}  // namespace

namespace negf {

unsigned long long* prof_flop_slots(int cls) {
  if (!g_prof_on.load() || g_capturing || cls < 0 || cls >= KC_COUNT) return nullptr;
  unsigned long long* p = g_prof_flops_ptr.load();
  return p ? p + (long)cls * PROF_SLOTS : nullptr;
}

void prof_begin(int cls, hipStream_t s) {
  if (!g_prof_on.load() || g_capturing || cls < 0 || cls >= KC_COUNT || !((g_prof_mask.load() >> cls) & 1u)) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  t_open = pool_get();
  if (t_open) (void)hipEventRecord(t_open, s);   // a failed record shows up when the pair is read
}

void prof_end(int cls, hipStream_t s, double flops, double bytes) {
  if (!g_prof_on.load() || !t_open || g_capturing) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = pool_get();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_prof_pending.push_back(ProfRec{t_open, e, cls, flops, bytes});
  t_open = nullptr;
}

}  // namespace negf

namespace negf {

hipError_t rt_copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

hipError_t rt_stream_create(hipStream_t* s) { return hipStreamCreateWithFlags(s, hipStreamNonBlocking); }
hipError_t rt_stream_destroy(hipStream_t s) { return hipStreamDestroy(s); }
hipError_t rt_event_create(hipEvent_t* e) { return hipEventCreateWithFlags(e, hipEventDisableTiming); }
hipError_t rt_event_destroy(hipEvent_t e) { return hipEventDestroy(e); }

hipError_t rt_record_wait(hipEvent_t e, hipStream_t from, hipStream_t to) {
  hipError_t r = hipEventRecord(e, from);
  if (r != hipSuccess) return r;
  return hipStreamWaitEvent(to, e, 0);
}

hipError_t rt_capture_begin(hipStream_t s) {
  g_capturing = true;
  hipError_t r = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (r != hipSuccess) g_capturing = false;
  return r;
}

hipError_t rt_capture_end(hipStream_t s, void** exec) {
  g_capturing = false;
  *exec = nullptr;
  hipGraph_t g = nullptr;
  hipError_t r = hipStreamEndCapture(s, &g);
  if (r != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  hipGraphExec_t ex = nullptr;
  r = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (r != hipSuccess) return r;
  *exec = (void*)ex;
  return hipSuccess;
}

hipError_t rt_graph_launch(void* exec, hipStream_t s) { return hipGraphLaunch((hipGraphExec_t)exec, s); }
hipError_t rt_graph_destroy(void* exec) { return exec ? hipGraphExecDestroy((hipGraphExec_t)exec) : hipSuccess; }

double rt_wallclock_hz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0.0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0.0;
  return 1e3 * khz;
}

}  // namespace negf

extern "C" {

void negf_profile_time_classes(uint32_t mask) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_mask.store(mask);
}

void negf_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!on) g_prof_on.store(false);
  if (on) {
    // the counters of the current device, cleared (synchronous), published before profiling turns on
    void* p = nullptr;
    g_prof_flops_ptr.store(nullptr);
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_prof_flops)) == hipSuccess &&
        hipMemset(p, 0, sizeof(unsigned long long) * KC_COUNT * PROF_SLOTS) == hipSuccess &&
        hipDeviceSynchronize() == hipSuccess)
      g_prof_flops_ptr.store((unsigned long long*)p);
    g_prof_on.store(true);
  }
  if (on) {
    for (auto& r : g_prof_pending) {
      g_prof_pool.push_back(r.a);
      g_prof_pool.push_back(r.b);
    }
    g_prof_pending.clear();
    std::memset(g_prof_acc, 0, sizeof(g_prof_acc));
  }
}

negf_status negf_profile_read(negf_kernel_stats* stats) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  negf_status st = NEGF_OK;
  for (auto& r : g_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      st = NEGF_EHIP;
    } else {
      negf_kernel_stats& a = g_prof_acc[r.cls];
      a.launches += 1;
      a.total_ms += ms;
      a.flops += r.flops;
      a.bytes += r.bytes;
    }
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_pending.clear();
  if (unsigned long long* fp = g_prof_flops_ptr.load()) {
    std::vector<unsigned long long> c((size_t)KC_COUNT * PROF_SLOTS);
    if (hipMemcpy(c.data(), fp, c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) !=
        hipSuccess) {
      st = NEGF_EHIP;
    } else {
      for (int k = 0; k < KC_COUNT; ++k) {
        double f = 0.0;
        for (int j = 0; j < PROF_SLOTS; ++j) f += (double)c[(size_t)k * PROF_SLOTS + j];
        g_prof_acc[k].flops += f;
      }
      if (hipMemset(fp, 0, c.size() * sizeof(unsigned long long)) != hipSuccess) st = NEGF_EHIP;
    }
  }
  if (stats)
    for (int i = 0; i < NEGF_KC_COUNT; ++i) stats[i] = i < KC_COUNT ? g_prof_acc[i] : negf_kernel_stats{};
  return st;
}

}  // extern "C"
