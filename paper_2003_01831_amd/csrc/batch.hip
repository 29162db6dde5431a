// Many uneven systems in one captured launch sequence (placeholder).
#include "common.h"

struct afq_batch_s { int n; };

int batch_create_impl(afq_batch* out, int n, const afq_system* systems, const afq_walkers* walkers) {
  (void)out; (void)n; (void)systems; (void)walkers;
  afq_set_error("afq_batch_create: not implemented yet");
  return AFQ_E_UNSUPPORTED;
}
int batch_step_impl(afq_batch b, int n_steps, double dt, uint64_t seed, int qr_every, const double* e_shift,
                    int order, double* emix_out) {
  (void)b; (void)n_steps; (void)dt; (void)seed; (void)qr_every; (void)e_shift; (void)order; (void)emix_out;
  afq_set_error("afq_batch_step: not implemented yet");
  return AFQ_E_UNSUPPORTED;
}
int batch_destroy_impl(afq_batch b) { (void)b; return AFQ_OK; }
