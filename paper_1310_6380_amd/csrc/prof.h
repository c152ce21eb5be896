// Per-kernel timing with HIP events on the launching stream (diagnostics).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace mvpb {

enum KernelId {
  K_SF = 0,
  K_SCATTER,
  K_POTRF,
  K_GEMM,
  K_COMBINE,
  K_FORM,
  K_PANEL,
  K_HEMM,
  K_WFORM,
  K_HER2K,
  K_HB2ST,
  K_TRIDIAG,
  K_BACKTRANSFORM,
  K_RR,
  K_HB2ST_IO,
  K_COUNT
};

struct Profiler {
  bool on = false;
  unsigned long long mask = ~0ull;   // kernel ids timed while on
  struct Rec {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[K_COUNT] = {};
  long long launches[K_COUNT] = {};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // Fold finished event pairs into the totals (waits for them).
  void drain() {
    for (Rec &r : pending) {
      float ms = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        total_ms[r.kernel] += ms;
        launches[r.kernel] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    drain();
    for (int i = 0; i < K_COUNT; ++i) {
      total_ms[i] = 0.0;
      launches[i] = 0;
    }
  }
  ~Profiler() {
    drain();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// The profiler of the call in progress on this host thread (NULL = off).
extern thread_local Profiler *t_prof;

struct ProfScope {
  Profiler *p;
  hipStream_t st;
  int k;
  hipEvent_t a = nullptr;
  ProfScope(int kernel, hipStream_t s) : p(t_prof), st(s), k(kernel) {
    if (p && p->on && ((p->mask >> kernel) & 1ull)) {
      a = p->get();
      (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = p->get();
      (void)hipEventRecord(b, st);
      p->pending.push_back({k, a, b});
    }
  }
};

}  // namespace mvpb
