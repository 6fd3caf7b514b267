// Kernel instantiations for one population format and lattice.
#include "fslbm_ops.h"

namespace fslbm_host {
Ops ops_f64_q19(int coll) {
  return coll == FSLBM_TRT ? Impl<ST_F64, 19, true>::ops() : Impl<ST_F64, 19, false>::ops();
}
}  // namespace fslbm_host
