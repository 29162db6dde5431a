// Many uneven systems stepped together. Every step runs in three stages that
// end where overlap inverses are needed; each stage runs as concurrent
// branches (one stream per system, forked from and joined back to a root
// stream), and between the stages the overlaps T^H W, their Gauss-Jordan
// inverses and the Theta products of every system run as grouped launches on
// the root stream: one launch per kernel shape walks a work table of
// per-system tasks, so a step of 24 systems takes a handful of these launches
// instead of a hundred small ones.
// After eager warm-up steps that size every buffer, one cycle of `qr_every`
// steps (one step when QR is off) is captured into a HIP graph and replayed,
// so a whole cycle of all systems is one graph launch. Step counters live in
// device memory, so replays advance the Philox fields.
#include <algorithm>
#include "common.h"
#include "step_kernels.h"

struct afq_batch_s {
  std::vector<afq_system> sys;
  std::vector<afq_walkers> wk;
  hipStream_t origin = nullptr;   // the systems' common stream (may be the null stream)
  hipStream_t cap = nullptr;      // batch-owned stream the graph is captured on
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> fork, join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // parameters baked into the captured graph
  double dt = 0.0;
  uint64_t seed = 0;
  int qr_every = -1, order = 0, cycle = 0, prec = -1;
  bool tuned = false;
  std::vector<double> e_shift;
  std::vector<double> caps;   // (fb_cap, w_cap) of every walker set, baked into the graph
  std::vector<unsigned> versions;   // the systems' kernel-sequence versions at capture
  std::vector<char> carried_after;  // each walker set's carried-inverse flag after the captured cycle
  DevBuf emix_cycle;   // n x cycle, written by the graph
  ~afq_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : fork) (void)hipEventDestroy(e);
    for (auto e : join) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto st : streams) {
      if (!st) continue;
      gemm_release_workspace(st);
      (void)hipStreamDestroy(st);
    }
  }
};

namespace {

// out[i * n_steps + base + k] = cyc[i * cycle + k]
__global__ void scatter_emix(const double* __restrict__ cyc, int n, int cycle, int n_steps, int base,
                             double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * cycle) {
    const int i = t / cycle, k = t - i * cycle;
    out[(long)i * n_steps + base + k] = cyc[t];
  }
}

// Enqueue `steps` steps of every system; step k of the sequence uses Philox
// step (*counter + k) and writes E_mix to emix[i][k0 + k]. Per step and stage:
// fork from the root stream, the stage of every system on its branch (its
// overlap inverses deferred), join, the grouped inverses on the root stream.
int enqueue_steps(afq_batch b, hipStream_t root, int steps, bool capture_layout, double* emix_user,
                  int n_steps_user, int base) {
  const int n = (int)b->sys.size();
  std::vector<GjTask> tasks;
  std::vector<OvlTask> otasks;
  std::vector<ThetaTask> ttasks;
  for (int k = 0; k < steps; ++k) {
    for (int stage = 0; stage < 3; ++stage) {
      tasks.clear();
      otasks.clear();
      if (stage == 1) {   // Theta of every system (after the inverses) as grouped launches
        ttasks.clear();
        for (int i = 0; i < n; ++i) ttasks.push_back(theta_task_of(b->sys[i], b->wk[i]));
        AFQ_RET(theta_grouped(ttasks, root));
        for (auto w : b->wk) w->theta_pre = true;
      }
      AFQ_TRY_HIP(hipEventRecord(b->fork[0], root));
      for (int i = 0; i < n; ++i) {
        afq_system s = b->sys[i];
        afq_walkers w = b->wk[i];
        const uint64_t idx = w->counter + k;
        const bool do_qr = b->qr_every > 0 && (idx + 1) % (uint64_t)b->qr_every == 0;
        double* em = capture_layout ? b->emix_cycle.as<double>() + (long)i * b->cycle + k
                                    : (emix_user ? emix_user + (long)i * n_steps_user + base + k : nullptr);
        hipStream_t saved = s->stream;
        s->stream = b->streams[i];
        int rc = hip_status(hipStreamWaitEvent(b->streams[i], b->fork[0], 0), "afq_batch_step: fork");
        lu_defer(&tasks);
        if (stage < 2) overlap_defer(&otasks);
        if (rc == AFQ_OK)
          rc = step_stage(stage, s, w, b->dt, nullptr, b->seed, (uint32_t)i, k, do_qr, b->e_shift[i], b->order, em,
                          nullptr, nullptr, nullptr);
        overlap_defer(nullptr);
        lu_defer(nullptr);
        if (rc == AFQ_OK && stage == 2 && k == steps - 1)
          rc = counter_add(w->d_counter.as<uint64_t>(), (uint64_t)steps, b->streams[i]);
        s->stream = saved;
        AFQ_RET(rc);
        AFQ_TRY_HIP(hipEventRecord(b->join[i], b->streams[i]));
        AFQ_TRY_HIP(hipStreamWaitEvent(root, b->join[i], 0));
      }
      // the overlaps the stage requested, then their inverses
      if (!otasks.empty()) AFQ_RET(overlap_grouped(otasks, root));
      if (!tasks.empty()) AFQ_RET(lu_inverse_grouped(tasks, root));
    }
  }
  return AFQ_OK;
}

void advance_counters(afq_batch b, int steps) {
  for (auto w : b->wk) w->counter += steps;
}

int build_graph(afq_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  // the captured cycle starts from a full overlap inverse, whatever the state
  // of the walkers when it is replayed
  for (auto w : b->wk) w->s_carried = false;
  AFQ_TRY_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  const int rc = enqueue_steps(b, b->cap, b->cycle, true, nullptr, 0, 0);
  b->carried_after.clear();
  for (auto w : b->wk) b->carried_after.push_back(w->s_carried);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  AFQ_RET(rc);
  AFQ_TRY_HIP(e);
  b->graph = g;
  AFQ_TRY_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return AFQ_OK;
}

}  // namespace

int batch_create_impl(afq_batch* out, int n, const afq_system* systems, const afq_walkers* walkers) {
  AFQ_CHECK(out, AFQ_E_INVALID, "afq_batch_create: out is NULL");
  *out = nullptr;
  AFQ_CHECK(n >= 1 && n <= 4096 && systems && walkers, AFQ_E_INVALID, "afq_batch_create: need 1..4096 systems");
  for (int i = 0; i < n; ++i) {
    AFQ_CHECK(systems[i] && walkers[i], AFQ_E_INVALID, "afq_batch_create: NULL handle");
    AFQ_CHECK(walkers[i]->sys == systems[i], AFQ_E_STATE, "afq_batch_create: walkers belong to another system");
    AFQ_CHECK(systems[i]->stream == systems[0]->stream && systems[i]->device == systems[0]->device, AFQ_E_STATE,
              "afq_batch_create: systems must share one stream and device");
    AFQ_CHECK(systems[i]->prec == systems[0]->prec, AFQ_E_STATE, "afq_batch_create: systems must share a precision");
    for (int j = 0; j < i; ++j)
      AFQ_CHECK(walkers[j] != walkers[i], AFQ_E_INVALID, "afq_batch_create: a walker set appears twice");
  }
  afq_batch b = new afq_batch_s();
  b->sys.assign(systems, systems + n);
  b->wk.assign(walkers, walkers + n);
  b->origin = systems[0]->stream;
  b->streams.resize(n, nullptr);
  b->join.resize(n, nullptr);
  b->fork.resize(1, nullptr);
  int rc = [&]() -> int {
    for (int i = 0; i < n; ++i) {
      AFQ_TRY_HIP(hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking));
      AFQ_TRY_HIP(hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming));
    }
    AFQ_TRY_HIP(hipEventCreateWithFlags(&b->fork[0], hipEventDisableTiming));
    AFQ_TRY_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    return AFQ_OK;
  }();
  if (rc != AFQ_OK) {
    delete b;
    return rc;
  }
  for (auto w : b->wk) ++w->in_batch;   // their steps keep W and S^-1 where the graph expects them
  *out = b;
  return AFQ_OK;
}

int batch_step_impl(afq_batch b, int n_steps, double dt, uint64_t seed, int qr_every, const double* e_shift,
                    int order, double* emix_out) {
  AFQ_CHECK(b, AFQ_E_INVALID, "afq_batch_step: batch is NULL");
  AFQ_CHECK(n_steps >= 0 && qr_every >= 0 && order >= 1 && order <= 32 && dt >= 0.0, AFQ_E_INVALID,
            "afq_batch_step: bad argument");
  AFQ_CHECK(e_shift, AFQ_E_INVALID, "afq_batch_step: e_shift is NULL");
  const int n = (int)b->sys.size();
  for (int i = 1; i < n; ++i)
    AFQ_CHECK(b->wk[i]->counter == b->wk[0]->counter, AFQ_E_STATE,
              "afq_batch_step: the walker sets' step counters differ");
  for (int i = 0; i < n; ++i)
    AFQ_CHECK(n_steps == 0 || b->wk[i]->bp_n < 0 || b->wk[i]->bp_rec >= b->wk[i]->bp_n, AFQ_E_STATE,
              "afq_batch_step: a walker set has a back-propagation window that still records (use afq_step)");
  std::vector<double> es(e_shift, e_shift + n);
  std::vector<double> caps;
  for (int i = 0; i < n; ++i) {
    caps.push_back(b->wk[i]->fb_cap);
    caps.push_back(b->wk[i]->w_cap);
  }
  const int prec = b->sys[0]->prec;
  for (int i = 1; i < n; ++i)
    AFQ_CHECK(b->sys[i]->prec == prec, AFQ_E_STATE, "afq_batch_step: systems must share a precision");
  // settle every system's set-up first: it may change the kernel sequence
  for (int i = 0; i < n; ++i) {
    AFQ_RET(system_prepare_dt(b->sys[i], dt));
    AFQ_RET(system_prepare_pack(b->sys[i], b->sys[i]->prec));
    AFQ_RET(walkers_alloc_scratch(b->wk[i]));
  }
  std::vector<unsigned> versions;
  for (int i = 0; i < n; ++i) versions.push_back(b->sys[i]->version);
  if (!b->exec || b->prec != prec || b->dt != dt || b->seed != seed || b->qr_every != qr_every || b->order != order || b->e_shift != es ||
      b->caps != caps || b->versions != versions) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (b->prec != prec || b->versions != versions) b->tuned = false;
    b->prec = prec;
    b->dt = dt;
    b->seed = seed;
    b->qr_every = qr_every;
    b->order = order;
    b->e_shift = es;
    b->caps = caps;
    b->versions = versions;
    b->cycle = qr_every > 0 ? qr_every : 1;
    AFQ_RET(b->emix_cycle.alloc((size_t)n * b->cycle * sizeof(double)));
  }
  int done = 0;
  bool warmed = b->exec != nullptr;
  while (done < n_steps) {
    const uint64_t c = b->wk[0]->counter;
    const int left = n_steps - done;
    if (warmed && c % b->cycle == 0 && left >= b->cycle) {
      if (!b->exec) {
        if (!b->tuned) {   // exchange launch variants per system, before they are baked into the graph
          int c[2];
          for (int i = 0; i < n; ++i) AFQ_RET(exchange_autotune(b->sys[i], b->wk[i], 3, c));
          b->tuned = true;
        }
        AFQ_TRY_HIP(hipStreamSynchronize(b->origin));
        AFQ_RET(build_graph(b));
      }
      AFQ_TRY_HIP(hipGraphLaunch(b->exec, b->origin));
      for (size_t i = 0; i < b->wk.size(); ++i) b->wk[i]->s_carried = b->carried_after[i];
      if (emix_out) {
        const int tot = n * b->cycle;
        hipLaunchKernelGGL(scatter_emix, dim3(ceil_div(tot, 256)), dim3(256), 0, b->origin,
                           b->emix_cycle.as<double>(), n, b->cycle, n_steps, done, emix_out);
        AFQ_TRY_HIP(hipGetLastError());
      }
      advance_counters(b, b->cycle);
      done += b->cycle;
    } else {
      AFQ_RET(enqueue_steps(b, b->origin, 1, false, emix_out, n_steps, done));
      advance_counters(b, 1);
      done += 1;
      warmed = true;
    }
  }
  return AFQ_OK;
}

int batch_destroy_impl(afq_batch b) {
  if (!b) return AFQ_OK;
  (void)hipStreamSynchronize(b->origin);
  for (auto w : b->wk) --w->in_batch;
  delete b;
  return AFQ_OK;
}
