// Optional per-stage device timing: HIP events recorded on the caller's
// stream around each pipeline launch, read back (and reset) on demand.
#include <vector>

#include "mm_internal.h"

namespace mm {

struct Profiler {
  struct Pair {
    int stage;
    int64_t samples;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Pair> pending;
  double ms[kProfStages] = {};
  int64_t launches[kProfStages] = {};
  int64_t samples[kProfStages] = {};

  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void flush() {
    for (auto& p : pending) {
      if (hipEventSynchronize(p.b) != hipSuccess) continue;
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        ms[p.stage] += t;
        launches[p.stage] += 1;
        samples[p.stage] += p.samples;
      }
    }
    pending.clear();
    used = 0;
  }
};

void prof_begin(ScanImpl* s, hipStream_t st, hipEvent_t* tok, int stage) {
  *tok = nullptr;
  if (!s->prof || s->capturing) return;   // no timing inside a captured graph
  if (!((s->prof_mask >> stage) & 1u)) return;   // stage not selected: no events
  if (s->prof->used > 32768) s->prof->flush();
  hipEvent_t e = s->prof->take();
  if (e && hipEventRecord(e, st) == hipSuccess) *tok = e;
}

void prof_end(ScanImpl* s, hipStream_t st, hipEvent_t tok, int stage, int64_t samples) {
  if (!s->prof || !tok) return;
  hipEvent_t e = s->prof->take();
  if (e && hipEventRecord(e, st) == hipSuccess) s->prof->pending.push_back({stage, samples, tok, e});
}

mm_status profile_enable(ScanImpl* s, int enable) {
  if (enable && !s->prof) s->prof = new Profiler;
  if (!enable && s->prof) {
    delete s->prof;
    s->prof = nullptr;
  }
  return MM_OK;
}

mm_status profile_stages(ScanImpl* s, uint32_t mask) {
  s->prof_mask = mask;
  return MM_OK;
}

mm_status profile_read(ScanImpl* s, mm_profile* out) {
  for (int i = 0; i < kProfStages; ++i) {
    out->ms[i] = 0.0;
    out->launches[i] = 0;
    out->samples[i] = 0;
  }
  out->n_stages = kProfStages;
  if (!s->prof) return MM_OK;
  s->prof->flush();
  for (int i = 0; i < kProfStages; ++i) {
    out->ms[i] = s->prof->ms[i];
    out->launches[i] = s->prof->launches[i];
    out->samples[i] = s->prof->samples[i];
    s->prof->ms[i] = 0.0;
    s->prof->launches[i] = 0;
    s->prof->samples[i] = 0;
  }
  return MM_OK;
}

void profile_free(ScanImpl* s) {
  delete s->prof;
  s->prof = nullptr;
}

}  // namespace mm
