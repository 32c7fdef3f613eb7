// Per-sample estimator of the paper's Eq. (nsum2) on the device.
//
// X = sum_i q_i phi(n_i) and Y = sum_i q_i^2 phi(n_i)^2 are gathered from the
// site-aggregated charge list (Q_s = sum of q on site s, S_s = sum of q^2),
// which gives the same X and Y as the raw list.  Accumulation is FP64.  The
// reduction has a fixed shape: each thread sums a fixed strided subset, waves
// reduce by DPP, blocks write partials, and the last block to finish (integer
// ticket) adds the partials in block order.  So the result does not depend on
// scheduling.  The last block forms O = X^2 - Y and adds it to its bin with a
// compensated (Kahan) FP64 sum; this replaces the paper's global reduce.

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

constexpr int kMeasureThreads = 256;

uint32_t measure_blocks(uint32_t n) {
    // about 4 charged sites per thread, at most 2048 blocks
    uint32_t b = (n + kMeasureThreads * 4 - 1) / (kMeasureThreads * 4);
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return b;
}

template <class St>
__global__ __launch_bounds__(kMeasureThreads) void gather_measure(
    const typename St::T* __restrict__ field, const uint32_t* __restrict__ site,
    const double* __restrict__ Q, const double* __restrict__ S, uint32_t n,
    double* __restrict__ partials, uint32_t* ticket, double* bins, uint32_t bin, double* last_xy) {
    double x = 0.0, y = 0.0;
    const uint32_t stride = gridDim.x * kMeasureThreads;
    for (uint32_t i = blockIdx.x * kMeasureThreads + threadIdx.x; i < n; i += stride) {
        const double v = (double)St::ld(field, site[i]);
        x = fma(Q[i], v, x);
        y = fma(S[i], v * v, y);
    }
    block_sum2<kMeasureThreads>(x, y);

    __shared__ uint32_t s_last;
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = x;
        partials[2 * blockIdx.x + 1] = y;
        __threadfence();
        const uint32_t prev = atomicAdd(ticket, 1u);
        s_last = (prev == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;

    // last block: add the partials in block order
    __threadfence();
    double X = 0.0, Y = 0.0;
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += kMeasureThreads) {
        X += __hip_atomic_load(&partials[2 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Y += __hip_atomic_load(&partials[2 * b + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum2<kMeasureThreads>(X, Y);
    if (threadIdx.x == 0) {
        const double O = X * X - Y;
        // Kahan: bins[2b] running sum, bins[2b+1] compensation (lost low part, negated)
        double sum = bins[2 * bin];
        double comp = bins[2 * bin + 1];
        const double yk = O - comp;
        const double tk = sum + yk;
        comp = (tk - sum) - yk;
        sum = tk;
        bins[2 * bin] = sum;
        bins[2 * bin + 1] = comp;
        last_xy[0] = X;
        last_xy[1] = Y;
        *ticket = 0u;
    }
}

template <class St>
static hipError_t launch_measure_t(const MeasureArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(gather_measure<St>, dim3(a.blocks), dim3(kMeasureThreads), 0, stream,
                       static_cast<const typename St::T*>(a.field), a.site, a.Q, a.S, a.n,
                       a.partials, a.ticket, a.bins, a.bin, a.last_xy);
    return hipGetLastError();
}

hipError_t launch_measure(const MeasureArgs& a, hipStream_t stream) {
    switch (a.storage) {
        case 0: return launch_measure_t<StoreF32>(a, stream);
        case 1: return launch_measure_t<StoreBF16>(a, stream);
        case 2: return launch_measure_t<StoreF16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
