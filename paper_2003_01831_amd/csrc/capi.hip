// The extern "C" boundary: argument validation, status codes and the
// thread-local error message; everything else is delegated to the runtime.
#include <cmath>
#include "common.h"
#include "step_kernels.h"

static thread_local std::string g_last_error;
void afq_set_error(const std::string& msg) { g_last_error = msg; }

int system_create_impl(afq_system* out, int M, int n_up, int n_dn, int X, const double* h1, const double* chol,
                       const double* phi_t, double e_core, int prec, void* stream, unsigned flags);
int walkers_create_impl(afq_walkers* out, afq_system s, int nw, const double* w0, const double* wt0);
int energy_call(afq_system s, afq_walkers w, double* eloc_out, double* parts_out, double* vbar_out,
                double* emix_out);
int batch_create_impl(afq_batch* out, int n, const afq_system* systems, const afq_walkers* walkers);
int batch_step_impl(afq_batch b, int n_steps, double dt, uint64_t seed, int qr_every, const double* e_shift,
                    int order, double* emix_out);
int batch_destroy_impl(afq_batch b);

#define AFQ_GUARD(...)                                      \
  try {                                                     \
    __VA_ARGS__                                             \
  } catch (const std::exception& e) {                       \
    afq_set_error(std::string("internal error: ") + e.what()); \
    return AFQ_E_HIP;                                       \
  } catch (...) {                                           \
    afq_set_error("internal error");                        \
    return AFQ_E_HIP;                                       \
  }

static int check_device(afq_system s) {
  int dev = -1;
  AFQ_TRY_HIP(hipGetDevice(&dev));
  AFQ_CHECK(dev == s->device, AFQ_E_STATE, "the current HIP device differs from the system's device");
  return AFQ_OK;
}

extern "C" {

const char* afq_last_error(void) { return g_last_error.c_str(); }
int afq_version(void) { return (1 << 16) | 0; }

int afq_system_create(afq_system* out, int M, int n_up, int n_dn, int n_chol, const double* h1, const double* chol,
                      const double* phi_t, double e_core, int precision, void* stream, unsigned flags) {
  AFQ_GUARD(return system_create_impl(out, M, n_up, n_dn, n_chol, h1, chol, phi_t, e_core, precision, stream,
                                      flags);)
}

int afq_system_set_precision(afq_system s, int precision) {
  AFQ_CHECK(s, AFQ_E_INVALID, "afq_system_set_precision: system is NULL");
  AFQ_CHECK(precision >= AFQ_FP64 && precision <= AFQ_BF16X3, AFQ_E_INVALID, "unknown precision");
  AFQ_CHECK(s->msd_n == 0 || precision == AFQ_FP64, AFQ_E_UNSUPPORTED,
            "afq_system_set_precision: a multi-determinant trial runs in FP64 mode");
  AFQ_GUARD(AFQ_RET(check_device(s)); return system_prepare_pack(s, precision);)
}

int afq_system_set_exchange_form(afq_system s, int form) {
  AFQ_CHECK(s, AFQ_E_INVALID, "afq_system_set_exchange_form: system is NULL");
  AFQ_CHECK(form >= AFQ_EXCH_AUTO && form <= AFQ_EXCH_FOUR_INDEX, AFQ_E_INVALID,
            "afq_system_set_exchange_form: unknown form");
  AFQ_GUARD({
    AFQ_RET(check_device(s));
    if (form != s->eri_form) {
      s->eri_form = form;
      s->eri_declined = false;
    }
    return eri_sync(s);
  })
}

int afq_system_set_propagator_tile(afq_system s, int tile) {
  AFQ_CHECK(s, AFQ_E_INVALID, "afq_system_set_propagator_tile: system is NULL");
  AFQ_CHECK(tile >= -1 && tile < b3_num_tiles(), AFQ_E_INVALID, "afq_system_set_propagator_tile: tile must be -1..2");
  AFQ_GUARD(AFQ_RET(check_device(s)); return system_set_b3_tile(s, tile);)
}

int afq_system_propagator_tile(afq_system s, int* tile) {
  AFQ_CHECK(s && tile, AFQ_E_INVALID, "afq_system_propagator_tile: NULL argument");
  *tile = b3_tile_of(s);
  return AFQ_OK;
}

int afq_system_exchange_form(afq_system s, int* in_use, uint64_t* tensor_bytes) {
  AFQ_CHECK(s && in_use, AFQ_E_INVALID, "afq_system_exchange_form: NULL argument");
  *in_use = s->eri_ready ? AFQ_EXCH_FOUR_INDEX : AFQ_EXCH_CHOLESKY;
  if (tensor_bytes) *tensor_bytes = eri_tensor_bytes(s);
  return AFQ_OK;
}

int afq_kp_system_create(afq_system* out, int nk, const int32_t* kq, int m, int n_up, int n_dn, int xq,
                         const double* hk, const double* Lk, const double* phik, double e_core, int precision,
                         void* stream) {
  AFQ_GUARD(return kp_system_create_impl(out, nk, kq, m, n_up, n_dn, xq, hk, Lk, phik, e_core, precision, stream);)
}

int afq_system_set_msd(afq_system s, const double* C, int n_det, const double* coeffs, const int32_t* exc) {
  AFQ_CHECK(s, AFQ_E_INVALID, "afq_system_set_msd: system is NULL");
  AFQ_CHECK(s->kp_nk == 0, AFQ_E_UNSUPPORTED, "afq_system_set_msd: not available for k-point systems");
  AFQ_GUARD(AFQ_RET(check_device(s)); return msd_set(s, C, n_det, coeffs, exc);)
}

int afq_system_set_background(afq_system s, int on, const double* background) {
  AFQ_CHECK(s, AFQ_E_INVALID, "afq_system_set_background: system is NULL");
  AFQ_CHECK(on == 0 || on == 1, AFQ_E_INVALID, "afq_system_set_background: on must be 0 or 1");
  AFQ_CHECK(s->kp_nk == 0, AFQ_E_UNSUPPORTED,
            "afq_system_set_background: not available for k-point systems (complex vectors)");
  AFQ_GUARD(AFQ_RET(check_device(s)); return system_set_background(s, on, on ? background : nullptr);)
}

int afq_system_background(afq_system s, int* on, double* background) {
  AFQ_CHECK(s && on, AFQ_E_INVALID, "afq_system_background: NULL argument");
  *on = s->mf_on ? 1 : 0;
  if (background && s->mf_on)
    AFQ_GUARD({
      AFQ_RET(check_device(s));
      AFQ_TRY_HIP(hipMemcpyAsync(background, s->vmf.p, (size_t)s->X * sizeof(double), hipMemcpyDeviceToDevice,
                                 s->stream));
      return AFQ_OK;
    })
  return AFQ_OK;
}

int afq_system_destroy(afq_system s) {
  if (!s) return AFQ_OK;
  AFQ_GUARD((void)hipStreamSynchronize(s->stream); delete s; return AFQ_OK;)
}

int afq_walkers_create(afq_walkers* out, afq_system s, int n_walkers, const double* w0, const double* weights0) {
  AFQ_GUARD(if (s) AFQ_RET(check_device(s)); return walkers_create_impl(out, s, n_walkers, w0, weights0);)
}

int afq_walkers_destroy(afq_walkers w) {
  if (!w) return AFQ_OK;
  AFQ_GUARD((void)hipStreamSynchronize(w->sys->stream); delete w; return AFQ_OK;)
}

int afq_walkers_get(afq_walkers w, double* W, double* weights, double* logovlp, int32_t* alive, uint64_t* counter) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_walkers_get: walkers is NULL");
  AFQ_GUARD({
    afq_system s = w->sys;
    AFQ_RET(check_device(s));
    hipStream_t st = s->stream;
    const size_t per = (size_t)s->M * s->ntot;
    if (W) AFQ_TRY_HIP(hipMemcpyAsync(W, w->W.p, w->nw * per * 16, hipMemcpyDeviceToDevice, st));
    if (weights) AFQ_TRY_HIP(hipMemcpyAsync(weights, w->weights.p, w->nw * 8, hipMemcpyDeviceToDevice, st));
    if (alive) AFQ_TRY_HIP(hipMemcpyAsync(alive, w->alive.p, w->nw * 4, hipMemcpyDeviceToDevice, st));
    if (logovlp) {
      AFQ_RET(walkers_alloc_scratch(w));
      AFQ_RET(compute_overlap_theta(s, w, w->W.as<double2>(), s->msd_n > 0, w->logdet.as<double2>()));
      if (s->msd_n > 0) AFQ_RET(msd_overlap(s, w, w->logdet.as<double2>(), st));
      AFQ_RET(launch_logovlp(w->logdet.as<double2>(), w->nw, reinterpret_cast<double2*>(logovlp), st));
    }
    if (counter) *counter = w->counter;
    return AFQ_OK;
  })
}

int afq_walkers_set(afq_walkers w, const double* W, const double* weights, const int32_t* alive, uint64_t counter) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_walkers_set: walkers is NULL");
  AFQ_GUARD({
    afq_system s = w->sys;
    AFQ_RET(check_device(s));
    hipStream_t st = s->stream;
    const size_t per = (size_t)s->M * s->ntot;
    if (W) AFQ_TRY_HIP(hipMemcpyAsync(w->W.p, W, w->nw * per * 16, hipMemcpyDeviceToDevice, st));
    w->s_carried = false;
    if (weights) AFQ_TRY_HIP(hipMemcpyAsync(w->weights.p, weights, w->nw * 8, hipMemcpyDeviceToDevice, st));
    if (alive) AFQ_TRY_HIP(hipMemcpyAsync(w->alive.p, alive, w->nw * 4, hipMemcpyDeviceToDevice, st));
    AFQ_RET(counter_set(w->d_counter.as<uint64_t>(), counter, st));
    w->counter = counter;
    w->bp_n = -1;   // the kets of an open back-propagation window no longer match
    return AFQ_OK;
  })
}

int afq_walkers_set_controls(afq_walkers w, double fb_cap, double w_cap) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_walkers_set_controls: walkers is NULL");
  AFQ_CHECK(std::isfinite(fb_cap) && fb_cap >= 0.0 && std::isfinite(w_cap) && w_cap >= 0.0, AFQ_E_INVALID,
            "afq_walkers_set_controls: caps must be finite and >= 0");
  w->fb_cap = fb_cap;
  w->w_cap = w_cap;
  return AFQ_OK;
}

int afq_walkers_comb(afq_walkers w, double xi, int32_t* src_out, double* total_out) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_walkers_comb: walkers is NULL");
  AFQ_CHECK(xi >= 0.0 && xi < 1.0, AFQ_E_INVALID, "afq_walkers_comb: xi must be in [0, 1)");
  AFQ_GUARD(AFQ_RET(check_device(w->sys)); return walkers_comb(w, xi, src_out, total_out);)
}

int afq_eshift_update(double e_est, double w_total, double w_target, double dt, double gain_steps,
                      double* e_shift_out) {
  AFQ_CHECK(e_shift_out, AFQ_E_INVALID, "afq_eshift_update: output is NULL");
  AFQ_CHECK(w_total > 0.0 && w_target > 0.0 && dt > 0.0 && gain_steps > 0.0 && std::isfinite(e_est), AFQ_E_INVALID,
            "afq_eshift_update: weights, dt and gain must be positive");
  *e_shift_out = e_est - std::log(w_total / w_target) / (gain_steps * dt);
  return AFQ_OK;
}

int afq_walkers_stats(afq_walkers w, int* n_alive, int64_t* n_killed) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_walkers_stats: walkers is NULL");
  AFQ_GUARD({
    afq_system s = w->sys;
    AFQ_RET(check_device(s));
    std::vector<int> al(w->nw);
    int64_t k = 0;
    AFQ_TRY_HIP(hipMemcpyAsync(al.data(), w->alive.p, w->nw * 4, hipMemcpyDeviceToHost, s->stream));
    AFQ_TRY_HIP(hipMemcpyAsync(&k, w->killed.p, 8, hipMemcpyDeviceToHost, s->stream));
    AFQ_TRY_HIP(hipStreamSynchronize(s->stream));
    int c = 0;
    for (int a : al) c += a != 0;
    if (n_alive) *n_alive = c;
    if (n_killed) *n_killed = k;
    return AFQ_OK;
  })
}

int afq_step(afq_system s, afq_walkers w, int n_steps, double dt, const double* fields, uint64_t seed, int qr_every,
             double e_shift, int taylor_order, double* emix_out, double* eloc_out, double* weights_out,
             double* ratio_out) {
  AFQ_CHECK(s && w, AFQ_E_INVALID, "afq_step: NULL handle");
  AFQ_CHECK(w->sys == s, AFQ_E_STATE, "afq_step: walkers belong to another system");
  AFQ_CHECK(n_steps >= 0, AFQ_E_INVALID, "afq_step: n_steps < 0");
  AFQ_CHECK(std::isfinite(dt) && dt >= 0.0, AFQ_E_INVALID, "afq_step: dt must be finite and >= 0");
  AFQ_CHECK(qr_every >= 0, AFQ_E_INVALID, "afq_step: qr_every < 0");
  AFQ_CHECK(taylor_order >= 1 && taylor_order <= 32, AFQ_E_INVALID, "afq_step: taylor_order must be in [1, 32]");
  AFQ_CHECK(std::isfinite(e_shift), AFQ_E_INVALID, "afq_step: e_shift is not finite");
  AFQ_GUARD({
    AFQ_RET(check_device(s));
    AFQ_RET(system_prepare_dt(s, dt));
    AFQ_RET(system_prepare_pack(s, s->prec));
    AFQ_RET(walkers_alloc_scratch(w));
    AFQ_RET(bp_check_step(w, n_steps, dt, taylor_order));
    const long nw = w->nw, X = s->X;
    for (int k = 0; k < n_steps; ++k) {
      const uint64_t idx = w->counter + k;
      const bool do_qr = qr_every > 0 && (idx + 1) % (uint64_t)qr_every == 0;
      AFQ_RET(step_once(s, w, dt, fields ? fields + (long)k * nw * X : nullptr, seed, 0, k, do_qr, e_shift,
                        taylor_order, emix_out ? emix_out + k : nullptr, eloc_out ? eloc_out + 2 * k * nw : nullptr,
                        weights_out ? weights_out + k * nw : nullptr, ratio_out ? ratio_out + 2 * k * nw : nullptr,
                        bp_record_slot(w)));
      bp_advance(w, 1);
    }
    if (n_steps > 0) AFQ_RET(counter_add(w->d_counter.as<uint64_t>(), (uint64_t)n_steps, s->stream));
    w->counter += n_steps;
    return AFQ_OK;
  })
}

int afq_bp_begin(afq_walkers w, int n_bp) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_bp_begin: walkers is NULL");
  AFQ_CHECK(n_bp >= 0 && n_bp <= (1 << 20), AFQ_E_INVALID, "afq_bp_begin: n_bp must be in [0, 2^20]");
  AFQ_CHECK(w->sys->msd_n == 0, AFQ_E_UNSUPPORTED, "afq_bp_begin: back-propagation needs a single-determinant trial");
  AFQ_GUARD(AFQ_RET(check_device(w->sys)); return bp_begin(w, n_bp);)
}

int afq_bp_rdm1(afq_walkers w, int qr_every, double* rdm_out, double* wsum_out) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_bp_rdm1: walkers is NULL");
  AFQ_CHECK(rdm_out, AFQ_E_INVALID, "afq_bp_rdm1: rdm_out is NULL");
  AFQ_CHECK(qr_every >= 0, AFQ_E_INVALID, "afq_bp_rdm1: qr_every < 0");
  AFQ_GUARD(AFQ_RET(check_device(w->sys)); return bp_rdm1(w, qr_every, rdm_out, wsum_out);)
}

int afq_bp_end(afq_walkers w) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_bp_end: walkers is NULL");
  AFQ_GUARD(AFQ_RET(check_device(w->sys)); AFQ_TRY_HIP(hipStreamSynchronize(w->sys->stream)); bp_end(w);
            return AFQ_OK;)
}

int afq_energy(afq_system s, afq_walkers w, double* eloc_out, double* parts_out, double* vbar_out, double* emix_out) {
  AFQ_CHECK(s && w, AFQ_E_INVALID, "afq_energy: NULL handle");
  AFQ_CHECK(w->sys == s, AFQ_E_STATE, "afq_energy: walkers belong to another system");
  AFQ_GUARD(AFQ_RET(check_device(s)); return energy_call(s, w, eloc_out, parts_out, vbar_out, emix_out);)
}

int afq_autotune(afq_system s, afq_walkers w, int reps, int* choice_out) {
  AFQ_CHECK(s && w, AFQ_E_INVALID, "afq_autotune: NULL handle");
  AFQ_CHECK(w->sys == s, AFQ_E_STATE, "afq_autotune: walkers belong to another system");
  AFQ_CHECK(reps >= 1 && reps <= 1000, AFQ_E_INVALID, "afq_autotune: reps must be in 1..1000");
  AFQ_GUARD(AFQ_RET(check_device(s)); int c[2] = {-1, -1}; AFQ_RET(exchange_autotune(s, w, reps, c));
            int tile = -1; AFQ_RET(r32_autotune(s, w, reps, &tile));
            if (choice_out) { choice_out[0] = c[0]; choice_out[1] = c[1]; } return AFQ_OK;)
}

int afq_exchange_variant(afq_walkers w, int spin, int variant) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_exchange_variant: NULL handle");
  AFQ_CHECK(spin == 0 || spin == 1, AFQ_E_INVALID, "afq_exchange_variant: spin must be 0 or 1");
  AFQ_CHECK(variant >= -1 && variant < 3, AFQ_E_INVALID, "afq_exchange_variant: variant must be -1..2");
  w->exch_var[spin] = variant;
  return AFQ_OK;
}

int afq_energy_backward(afq_system s, afq_walkers w, double scale, double* d_h1, double* d_chol, double* d_walkers) {
  AFQ_CHECK(s && w, AFQ_E_INVALID, "afq_energy_backward: NULL handle");
  AFQ_CHECK(w->sys == s, AFQ_E_STATE, "afq_energy_backward: walkers belong to another system");
  AFQ_CHECK(std::isfinite(scale), AFQ_E_INVALID, "afq_energy_backward: scale is not finite");
  AFQ_CHECK(s->msd_n == 0, AFQ_E_UNSUPPORTED, "afq_energy_backward: needs a single-determinant trial");
  AFQ_CHECK(s->kp_nk == 0, AFQ_E_UNSUPPORTED, "afq_energy_backward: real Cholesky vectors only");
  AFQ_GUARD(AFQ_RET(check_device(s)); return energy_backward(s, w, scale, d_h1, d_chol, d_walkers);)
}

int afq_fields_generate(uint64_t seed, uint32_t sys_id, uint64_t step0, int n_steps, int n_walkers, int n_chol,
                        double* out, void* stream) {
  AFQ_CHECK(n_steps >= 0 && n_walkers >= 0 && n_chol >= 0, AFQ_E_INVALID, "afq_fields_generate: negative size");
  AFQ_CHECK(out || (long)n_steps * n_walkers * n_chol == 0, AFQ_E_INVALID, "afq_fields_generate: out is NULL");
  AFQ_GUARD(return launch_fields(seed, sys_id, step0, n_walkers, n_chol, out, (long)n_walkers * n_chol, n_steps,
                                 static_cast<hipStream_t>(stream));)
}

int afq_batch_create(afq_batch* out, int n, const afq_system* systems, const afq_walkers* walkers) {
  AFQ_GUARD(return batch_create_impl(out, n, systems, walkers);)
}

int afq_batch_step(afq_batch b, int n_steps, double dt, uint64_t seed, int qr_every, const double* e_shift,
                   int taylor_order, double* emix_out) {
  AFQ_GUARD(return batch_step_impl(b, n_steps, dt, seed, qr_every, e_shift, taylor_order, emix_out);)
}

int afq_batch_destroy(afq_batch b) { AFQ_GUARD(return batch_destroy_impl(b);) }

}  // extern "C"
