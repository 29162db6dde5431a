// Adjoint of the weighted mixed energy (placeholder until the kernels land).
#include "common.h"

int energy_backward(afq_system s, afq_walkers w, double scale, double* d_h1, double* d_chol, double* d_walkers) {
  (void)s; (void)w; (void)scale; (void)d_h1; (void)d_chol; (void)d_walkers;
  afq_set_error("afq_energy_backward: not implemented yet");
  return AFQ_E_UNSUPPORTED;
}
