// Per-phase GPU timing with HIP events recorded on the library's stream.
// Off by default; when on, every traced phase brackets its launches with a
// pair of events and afq_trace_query sums the elapsed times.
#include <array>
#include "common.h"
#include "trace.h"

namespace {
struct Slot {
  hipEvent_t a = nullptr, b = nullptr;
  int phase = 0;
};
struct TraceState {
  bool on = false;
  std::vector<Slot> slots;
  size_t used = 0;
  double ms[AFQ_TRACE_NPHASE] = {};
  int64_t cnt[AFQ_TRACE_NPHASE] = {};
};
TraceState g;

int collect() {
  for (size_t i = 0; i < g.used; ++i) {
    Slot& s = g.slots[i];
    AFQ_TRY_HIP(hipEventSynchronize(s.b));
    float t = 0.f;
    AFQ_TRY_HIP(hipEventElapsedTime(&t, s.a, s.b));
    g.ms[s.phase] += t;
    g.cnt[s.phase] += 1;
  }
  g.used = 0;
  return AFQ_OK;
}
}  // namespace

TraceScope::TraceScope(int phase, hipStream_t st) : slot_(-1), st_(st) {
  if (!g.on || phase < 0 || phase >= AFQ_TRACE_NPHASE) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;   // not inside graphs
  if (g.used == g.slots.size()) {
    if (g.used >= 65536 && collect() != AFQ_OK) return;
    if (g.used == g.slots.size()) {
      Slot s;
      if (hipEventCreate(&s.a) != hipSuccess || hipEventCreate(&s.b) != hipSuccess) return;
      g.slots.push_back(s);
    }
  }
  slot_ = (long)g.used++;
  g.slots[slot_].phase = phase;
  (void)hipEventRecord(g.slots[slot_].a, st_);
}

TraceScope::~TraceScope() {
  if (slot_ >= 0) (void)hipEventRecord(g.slots[slot_].b, st_);
}

extern "C" {

int afq_trace_enable(int on) {
  g.on = on != 0;
  return AFQ_OK;
}

int afq_trace_reset(void) {
  for (size_t i = 0; i < g.used; ++i) (void)hipEventSynchronize(g.slots[i].b);
  g.used = 0;
  for (int p = 0; p < AFQ_TRACE_NPHASE; ++p) { g.ms[p] = 0.0; g.cnt[p] = 0; }
  return AFQ_OK;
}

int afq_trace_query(int phase, double* ms, int64_t* count) {
  AFQ_CHECK(phase >= 0 && phase < AFQ_TRACE_NPHASE, AFQ_E_INVALID, "afq_trace_query: unknown phase");
  AFQ_RET(collect());
  if (ms) *ms = g.ms[phase];
  if (count) *count = g.cnt[phase];
  return AFQ_OK;
}

}  // extern "C"
