// Instantiations of the generic exchange kernel for the F64 policy.
#include "exchange_generic.h"

int exchange_generic_f64(const exch::ExchArgs& g, int variant, hipStream_t st) {
  return exch::launch_policy<exch::PolF64>(g, variant, st);
}
