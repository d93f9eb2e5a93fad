// mtpt_tiles_3d_tens.hip -- the row-sum and transfer passes of the MTPT step for 3-d
// simulations with a dispersion tensor (Mahalanobis distance, ellipsoidal cutoff), single and batched
// launches (one translation unit per dimension and metric, so that the
// build compiles them in parallel).
#include "mtpt_device.h"

namespace mtpt {
template hipError_t launch_tiles<3, true>(int, int, int, const SimArgs*, const Batch*, hipStream_t);
template hipError_t launch_tiles_export<3, true>(int, int, int, const SimArgs&, hipStream_t);
}  // namespace mtpt
