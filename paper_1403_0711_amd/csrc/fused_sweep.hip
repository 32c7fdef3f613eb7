// Fused red-black sweep: both colours of one sweep in one pass over the
// field (z-marching slabs).  Not enabled yet: fused_sweep_supported() is false.

#include "kernels.hpp"
#include "runtime_common.hpp"

namespace latcoul {

bool fused_sweep_supported(uint32_t, uint32_t) { return false; }

hipError_t launch_fused_sweep(const FusedArgs&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace latcoul
