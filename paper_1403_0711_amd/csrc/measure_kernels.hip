// Per-sample estimator of the paper's Eq. (nsum2) on the device.
//
// X = sum_i q_i phi(n_i) and Y = sum_i q_i^2 phi(n_i)^2 are gathered from the
// site-aggregated charge list (Q_s = sum of q on site s, S_s = sum of q^2),
// which gives the same X and Y as the raw list.  Accumulation is FP64.  The
// reduction has a fixed shape, so the result does not depend on scheduling:
// each thread sums a fixed strided subset, waves reduce by DPP, and each block
// writes one partial (X_b, Y_b).  A second one-block launch adds the partials
// in block order, forms O = X^2 - Y and adds it to its bin with a compensated
// (Kahan) FP64 sum; this replaces the paper's global reduce.  The kernel
// boundary orders the two phases, so no device-scope fence or atomic is
// needed (a device-scope release on this multi-XCD chip writes back L2).
//
// Several charge sets can share one field chain (the paper's reuse of one set
// of samples for many charge configurations): their lists are concatenated,
// set k holding entries set_off[k] .. set_off[k+1]-1; grid row k gathers set
// k, and block k of the second launch forms set k's sample and bins it in its
// own bin array (stride bin_stride bins).

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

constexpr int kMeasureThreads = 256;
constexpr int kGatherUnroll = 4;

uint32_t measure_blocks(uint32_t n) {
    // kGatherUnroll charged sites per thread per pass, at most 2048 blocks
    uint32_t b = (n + kMeasureThreads * kGatherUnroll - 1) / (kMeasureThreads * kGatherUnroll);
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return b;
}

template <class St>
__device__ __forceinline__ float site_value(const typename St::T* f0, const typename St::T* f1, uint32_t vh,
                                            uint32_t s) {
    return s < vh ? St::ld(f0, s) : St::ld(f1, s - vh);
}

template <class St>
__global__ __launch_bounds__(kMeasureThreads) void gather_partials(const typename St::T* __restrict__ f0,
                                                                   const typename St::T* __restrict__ f1,
                                                                   uint32_t vh,
                                                                   const uint32_t* __restrict__ site,
                                                                   const double* __restrict__ Q,
                                                                   const double* __restrict__ S, uint32_t n,
                                                                   const uint32_t* __restrict__ set_off,
                                                                   double* __restrict__ partials) {
    double x = 0.0, y = 0.0;
    const uint32_t set = blockIdx.y;
    const uint32_t lo = set_off ? set_off[set] : 0u;
    n = set_off ? set_off[set + 1] : n;  // one past the set's last entry
    const uint32_t stride = gridDim.x * kMeasureThreads;
    uint32_t i = lo + blockIdx.x * kMeasureThreads + threadIdx.x;
    // kGatherUnroll independent loads in flight per thread
    for (; i + (kGatherUnroll - 1) * stride < n; i += kGatherUnroll * stride) {
        float v[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) v[u] = site_value<St>(f0, f1, vh, site[i + u * stride]);
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
            const double d = (double)v[u];
            x = fma(Q[i + u * stride], d, x);
            y = fma(S[i + u * stride], d * d, y);
        }
    }
    for (; i < n; i += stride) {
        const double d = (double)site_value<St>(f0, f1, vh, site[i]);
        x = fma(Q[i], d, x);
        y = fma(S[i], d * d, y);
    }
    block_sum2<kMeasureThreads>(x, y);
    if (threadIdx.x == 0) {
        const uint32_t b = set * gridDim.x + blockIdx.x;
        partials[2 * b] = x;
        partials[2 * b + 1] = y;
    }
}

constexpr int kFinalThreads = 1024;
constexpr int kFinalUnroll = 8;  // partial loads in flight per thread

// Sample m (counted from the device counter mdev when given: graph replays)
// goes to bin (m [+ *mdev]) / bin_size of the block's charge set.
__global__ __launch_bounds__(kFinalThreads) void finalize_measure(const double* __restrict__ partials,
                                                                  uint32_t blocks, double* bins, uint32_t m,
                                                                  uint32_t bin_size,
                                                                  const uint32_t* __restrict__ mdev,
                                                                  double* last_xy, uint32_t bin_stride) {
    const uint32_t bin = (m + (mdev ? mdev[0] : 0u)) / bin_size;
    const uint32_t set = blockIdx.x;
    const double2* p = reinterpret_cast<const double2*>(partials + 2 * (size_t)set * blocks);
    bins += 2 * (size_t)set * bin_stride;
    // kFinalUnroll independent chains per thread, summed in a fixed order
    double xs[kFinalUnroll], ys[kFinalUnroll];
#pragma unroll
    for (int u = 0; u < kFinalUnroll; ++u) xs[u] = ys[u] = 0.0;
    for (uint32_t b0 = 0; b0 < blocks; b0 += kFinalThreads * kFinalUnroll) {
        double2 v[kFinalUnroll];
#pragma unroll
        for (int u = 0; u < kFinalUnroll; ++u)  // unconditional loads (clamped index), all in flight
            v[u] = p[min(b0 + (uint32_t)u * kFinalThreads + threadIdx.x, blocks - 1u)];
#pragma unroll
        for (int u = 0; u < kFinalUnroll; ++u)
            if (b0 + (uint32_t)u * kFinalThreads + threadIdx.x < blocks) {
                xs[u] += v[u].x;
                ys[u] += v[u].y;
            }
    }
    double X = 0.0, Y = 0.0;
#pragma unroll
    for (int u = 0; u < kFinalUnroll; ++u) {
        X += xs[u];
        Y += ys[u];
    }
    block_sum2<kFinalThreads>(X, Y);
    if (threadIdx.x == 0) record_sample(X, Y, bins, bin, last_xy + 2 * set);
}

hipError_t launch_finalize_measure(const double* partials, uint32_t blocks, uint32_t n_sets, double* bins,
                                   uint32_t m, uint32_t bin_size, const uint32_t* mdev, double* last_xy,
                                   uint32_t bin_stride, hipStream_t stream) {
    hipLaunchKernelGGL(finalize_measure, dim3(n_sets), dim3(kFinalThreads), 0, stream, partials, blocks, bins, m,
                       bin_size, mdev, last_xy, bin_stride);
    return hipGetLastError();
}

template <class St>
static hipError_t launch_measure_t(const MeasureArgs& a, hipStream_t stream) {
    if (a.n_sets < 1 || (a.n_sets > 1 && !a.set_off)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_partials<St>, dim3(a.blocks, a.n_sets), dim3(kMeasureThreads), 0, stream,
                       static_cast<const typename St::T*>(a.field0), static_cast<const typename St::T*>(a.field1),
                       a.vh, a.site, a.Q, a.S, a.n, a.set_off, a.partials);
    hipLaunchKernelGGL(finalize_measure, dim3(a.n_sets), dim3(kFinalThreads), 0, stream, a.partials, a.blocks,
                       a.bins, a.m, a.bin_size, a.mdev, a.last_xy, a.bin_stride);
    return hipGetLastError();
}

hipError_t launch_measure(const MeasureArgs& a, hipStream_t stream) {
    switch (storage_grid(a.storage)) {
        case 0: return launch_measure_t<StoreF32>(a, stream);
        case 1: return launch_measure_t<StoreBF16>(a, stream);
        case 2: return launch_measure_t<StoreF16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
