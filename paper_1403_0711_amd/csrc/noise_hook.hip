// Test hook: the device's uniform -> Gaussian transform (heatbath_noise, the
// one every sweep kernel calls) evaluated at chosen points of the 24-bit
// uniform grid, so that it can be compared with an exact inverse normal CDF
// over the whole grid, both tails included.

#include "device_common.hpp"
#include "runtime_common.hpp"

#include "lattice_coulomb.h"

namespace latcoul {

__global__ __launch_bounds__(256) void noise_values(uint32_t k_first, uint32_t n, float* __restrict__ out) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = k_first + i;
    // the word's low 8 bits are not part of the grid point; they vary here
    // so that a transform that used them would show it
    out[i] = heatbath_noise((k << 8) | ((i * 37u) & 0xFFu));
}

}  // namespace latcoul

extern "C" int lattice_noise_values(int64_t k_first, int64_t n, float* dev_out, void* hip_stream) {
    using namespace latcoul;
    if (k_first < 0 || n < 0 || k_first + n > ((int64_t)1 << 24))
        return set_error(LAT_ERR_ARG, "grid points must lie in [0, 2^24)");
    if (n == 0) return LAT_OK;
    if (!dev_out) return set_error(LAT_ERR_ARG, "dev_out is NULL");
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(noise_values, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       (uint32_t)k_first, (uint32_t)n, dev_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LAT_OK : hip_fail(e, "noise hook launch");
}
