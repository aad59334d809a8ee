// 3-D fused rpADMM sweep.
#include "mf_kernels.h"

namespace mf {

hipError_t launch_fused3d(const SweepDesc&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace mf
