// Kernel instantiations for one population format and lattice.
#include "fslbm_ops.h"

namespace fslbm_host {
Ops ops_f32_q27(int coll) {
  return coll == FSLBM_TRT ? Impl<ST_F32, 27, true>::ops() : Impl<ST_F32, 27, false>::ops();
}
}  // namespace fslbm_host
