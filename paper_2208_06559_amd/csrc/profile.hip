// Per-kernel timing: a pool of HIP events recorded around each launch while
// profiling is on; totals are summed per kernel name on request.
#include <string.h>

#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace bd {

struct Profiler {
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  bool open = false;  // the last launch's begin event was recorded
  // Instrumentation must never throw across the C ABI: a failed host
  // allocation just leaves that launch untimed.
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      try {
        pool.push_back(e);
      } catch (...) {
        (void)hipEventDestroy(e);
        return nullptr;
      }
    }
    return pool[used++];
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

thread_local Profiler* g_prof = nullptr;

void prof_mark_begin(hipStream_t s, const char* name) {
  Profiler* p = g_prof;
  p->open = false;
  hipEvent_t a = p->take(), b = p->take();
  if (!a || !b) return;
  try {
    p->recs.push_back({name, a, b});
  } catch (...) {
    return;
  }
  (void)hipEventRecord(a, s);
  p->open = true;
}

void prof_mark_end(hipStream_t s) {
  Profiler* p = g_prof;
  if (!p->open) return;
  (void)hipEventRecord(p->recs.back().b, s);
  p->open = false;
}

Profiler* profiler_new() { return new (std::nothrow) Profiler; }
void profiler_delete(Profiler* p) { delete p; }

// Synchronises `s`, sums the elapsed time per kernel name and resets.
int profiler_collect(Profiler* p, hipStream_t s, bd_kernel_stat_t* out, int max_out) {
  (void)hipStreamSynchronize(s);
  int n = 0;
  try {
    std::map<std::string, std::pair<int64_t, double>> agg;
    for (const auto& r : p->recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
      auto& e = agg[r.name];
      e.first += 1;
      e.second += ms;
    }
    for (const auto& kv : agg) {
      if (n < max_out && out) {
        memset(&out[n], 0, sizeof(bd_kernel_stat_t));
        strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
        out[n].launches = kv.second.first;
        out[n].total_ms = kv.second.second;
      }
      ++n;
    }
  } catch (...) {
    n = 0;
  }
  p->recs.clear();
  p->used = 0;
  p->open = false;
  return n;
}

}  // namespace bd
