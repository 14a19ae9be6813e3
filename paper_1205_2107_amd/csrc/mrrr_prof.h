// Per-kernel timing shared by the solver and the backward (see mrrr_profile_*).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace mrrr {

bool prof_enabled();
void prof_add(int kernel, int64_t launches, double ms, double work, double bytes);
// message returned by mrrr_last_error for the calling thread
void set_last_error(const char* msg);

// HIP events around launches on one stream; elapsed times are read after the
// caller has synchronized the stream.
struct ProfEvents {
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  hipStream_t st;
  bool on;
  std::vector<Rec> recs;
  Rec cur{};
  explicit ProfEvents(hipStream_t s) : st(s), on(prof_enabled()) {}
  void begin(int kind) {
    if (!on) return;
    cur.kind = kind;
    if (hipEventCreate(&cur.a) != hipSuccess || hipEventCreate(&cur.b) != hipSuccess) {
      on = false;
      return;
    }
    (void)hipEventRecord(cur.a, st);
  }
  void end() {
    if (!on) return;
    (void)hipEventRecord(cur.b, st);
    recs.push_back(cur);
  }
  // the same around launches on another stream s
  void begin_on(int kind, hipStream_t s) {
    hipStream_t keep = st;
    st = s;
    begin(kind);
    st = keep;
  }
  void end_on(hipStream_t s) {
    hipStream_t keep = st;
    st = s;
    end();
    st = keep;
  }
  // total milliseconds and launches of one kind
  void total(int kind, double* ms, int64_t* launches) {
    *ms = 0.0;
    *launches = 0;
    for (auto& r : recs)
      if (r.kind == kind) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) *ms += t;
        ++*launches;
      }
  }
  ~ProfEvents() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  }
};

}  // namespace mrrr
