// Dispatch of the fused exchange contraction (tr Omega, tr Omega^2 per
// Cholesky vector, walker and spin) and its autotuner.
//
// Shapes with 65..100 electrons per spin in split-BF16x3 use the specialised
// kernel of exchange_big.hip (fixed tiling). Every other shape uses the generic
// kernel of exchange_generic.h, which has several launch variants (waves per
// workgroup, accumulator budget). The autotuner times each variant on the
// walker set's own shapes with HIP events and keeps the fastest, per walker set
// and in a process-wide table keyed by the shape, so later walker sets of the
// same shape start from the tuned choice.
#include <map>
#include <mutex>
#include <tuple>
#include "common.h"
#include "exchange_big.h"
#include "exchange_generic.h"

namespace {

using Key = std::tuple<int, int, int, int, int, int>;   // prec, n, np, kp, X, nw
std::mutex& tune_mutex() {
  static std::mutex* m = new std::mutex();
  return *m;
}
std::map<Key, int>& tune_table() {
  static auto* t = new std::map<Key, int>();
  return *t;
}
Key key_of(afq_system s, afq_walkers w, int spin) {
  const PackShape& ps = s->ps[spin];
  return Key{s->prec, ps.n, ps.np, ps.kp, s->X, w->nw};
}

exch::ExchArgs generic_args(afq_system s, afq_walkers w, int spin, size_t boff) {
  const PackShape& ps = s->ps[spin];
  exch::ExchArgs g{};
  g.a_hi = s->apack[spin].p;
  g.a_lo = s->apack_lo[spin].p;
  g.b_hi = w->bpack.as<char>() + boff;
  g.b_lo = s->prec == AFQ_BF16X3 ? (const void*)(w->bpack_lo.as<char>() + boff) : nullptr;
  g.n = ps.n; g.np = ps.np; g.kp = ps.kp; g.X = s->X; g.nw = w->nw; g.spin = spin;
  g.PN = 0; g.PW = 0;
  g.tro = w->tro.as<double2>();
  g.troo = w->troo.as<double2>();
  return g;
}

size_t b_offset(afq_system s, afq_walkers w, int spin) {
  const size_t esz = s->prec == AFQ_FP64 ? 8 : s->prec == AFQ_CFP32 ? 4 : 2;
  return (size_t)spin * s->ps[0].rows_b(w->nw) * s->ps[0].kp * esz;
}

int launch_generic(afq_system s, const exch::ExchArgs& g, int variant, hipStream_t st) {
  if (s->prec == AFQ_FP64) return exchange_generic_f64(g, variant, st);
  if (s->prec == AFQ_CFP32) return exchange_generic_f32(g, variant, st);
  return exchange_generic_bf16(g, variant, st);
}

int variant_for(afq_system s, afq_walkers w, int spin) {
  if (w->exch_var[spin] >= 0) return w->exch_var[spin];
  std::lock_guard<std::mutex> lk(tune_mutex());
  auto it = tune_table().find(key_of(s, w, spin));
  return it == tune_table().end() ? 0 : it->second;
}

}  // namespace

int exch_kchunk(int prec) {
  return prec == AFQ_FP64 ? exch::PolF64::KC : prec == AFQ_CFP32 ? exch::PolF32::KC : exch::PolBF16x3::KC;
}

int exchange_launch(afq_system s, afq_walkers w, int spin, hipStream_t st) {
  const PackShape& ps = s->ps[spin];
  const size_t boff = b_offset(s, w, spin);
  if (ps.big) {
    ExchBigArgs b{};
    b.a[0] = s->apack[spin].p;
    b.a[1] = s->apack_lo[spin].p;
    b.b[0] = w->bpack.as<char>() + boff;
    b.b[1] = s->prec == AFQ_BF16X3 ? (const void*)(w->bpack_lo.as<char>() + boff) : nullptr;
    b.n = ps.n; b.kp = ps.kp; b.X = s->X; b.nw = w->nw; b.spin = spin;
    b.rows_a = (long)s->X * ps.np + ps.pad;
    b.rows_b = ps.rows_b(w->nw);
    b.tro = w->tro.as<double2>();
    b.troo = w->troo.as<double2>();
    return exchange_big_launch(b, s->prec, st);
  }
  return launch_generic(s, generic_args(s, w, spin, boff), variant_for(s, w, spin), st);
}

// Times every launch variant of both spins on the current walkers (Theta is
// recomputed and packed first; only per-step scratch is written) and keeps the
// fastest. choice[spin] = the variant, or -1 where the shape has a single
// kernel (the specialised split-BF16x3 kernel).
int exchange_autotune(afq_system s, afq_walkers w, int reps, int* choice) {
  hipStream_t st = s->stream;
  AFQ_RET(system_prepare_pack(s, s->prec));
  if (s->kp_nk > 0 || s->msd_n > 0 || s->eri_ready) {   // no Cholesky-form exchange kernel in use
    choice[0] = choice[1] = -1;
    return AFQ_OK;
  }
  AFQ_RET(walkers_alloc_scratch(w));
  AFQ_RET(compute_overlap_theta(s, w, w->W.as<double2>(), true, w->logdet.as<double2>()));
  AFQ_RET(pack_theta(s, w, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  AFQ_TRY_HIP(hipEventCreate(&e0));
  AFQ_TRY_HIP(hipEventCreate(&e1));
  int rc = AFQ_OK;
  for (int spin = 0; spin < 2 && rc == AFQ_OK; ++spin) {
    choice[spin] = -1;
    if (s->ps[spin].big) continue;
    const exch::ExchArgs g = generic_args(s, w, spin, b_offset(s, w, spin));
    float best = 0.f;
    int best_v = -1;
    for (int v = 0; v < exch::kNumExchVariants && rc == AFQ_OK; ++v) {
      if (launch_generic(s, g, v, st) != AFQ_OK) continue;   // does not fit this shape (LDS)
      if ((rc = hip_status(hipEventRecord(e0, st), "hipEventRecord")) != AFQ_OK) break;
      for (int r = 0; r < reps && rc == AFQ_OK; ++r) rc = launch_generic(s, g, v, st);
      if (rc != AFQ_OK) break;
      if ((rc = hip_status(hipEventRecord(e1, st), "hipEventRecord")) != AFQ_OK) break;
      if ((rc = hip_status(hipEventSynchronize(e1), "hipEventSynchronize")) != AFQ_OK) break;
      float ms = 0.f;
      if ((rc = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) != AFQ_OK) break;
      if (best_v < 0 || ms < best) {
        best = ms;
        best_v = v;
      }
    }
    if (rc != AFQ_OK) break;
    if (best_v < 0) {
      afq_set_error("exchange autotune: no launch variant fits this shape");
      rc = AFQ_E_UNSUPPORTED;
      break;
    }
    choice[spin] = best_v;
    w->exch_var[spin] = best_v;
    std::lock_guard<std::mutex> lk(tune_mutex());
    tune_table()[key_of(s, w, spin)] = best_v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
