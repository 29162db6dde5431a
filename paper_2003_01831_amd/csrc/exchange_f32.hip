// Instantiations of the generic exchange kernel for the F32 policy.
#include "exchange_generic.h"

int exchange_generic_f32(const exch::ExchArgs& g, int variant, hipStream_t st) {
  return exch::launch_policy<exch::PolF32>(g, variant, st);
}
