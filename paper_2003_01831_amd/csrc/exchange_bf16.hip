// Instantiations of the generic exchange kernel for the BF16x3 policy.
#include "exchange_generic.h"

int exchange_generic_bf16(const exch::ExchArgs& g, int variant, hipStream_t st) {
  return exch::launch_policy<exch::PolBF16x3>(g, variant, st);
}
