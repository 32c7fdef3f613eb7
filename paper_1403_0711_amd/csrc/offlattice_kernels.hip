// Off-lattice charges: the paper's remark that a charge at an arbitrary
// position can be modelled by its nearest eight lattice sites, and forces
// evaluated by interpolation in the same way.
//
// Site (x, y, z) sits at position (x, y, z) in lattice units.  A charge at r
// (0 <= r_d <= L_d - 1, L_d >= 2) lies in the cell with origin
// b_d = min(floor(r_d), L_d - 2) and fraction f_d = r_d - b_d; corner b + e
// (e in {0,1}^3) has weight prod_d (e_d ? f_d : 1 - f_d).  The field at the
// charge is phi~ = sum_corners w phi(corner) and its gradient in r within the
// cell is sum_corners (+-1 on the axis, weights on the other two) phi(corner).
// A sample is O = X^2 - Y with X = sum_i q_i phi~_i, Y = sum_i (q_i phi~_i)^2;
// its mean is sum_{i != j} q_i q_j w_i^T G w_j (the interpolated lattice
// energy).  With forces on, each measured sweep also adds the sample
// dO/dr_i = 2 q_i grad phi~_i (X - q_i phi~_i) of dE/dr_i to per-charge FP64
// sums (E sums ordered pairs, so the physical force is -(1/2) dE/dr_i).
//
// Arithmetic on positions, weights and sums is FP64.  The partial sums have
// the fixed shape of the on-lattice gather (strided subsets, DPP wave sums,
// one partial per block), so results do not depend on scheduling.

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

constexpr int kOffThreads = 256;

template <class St>
__device__ __forceinline__ double corner_value(const typename St::T* f0, const typename St::T* f1, uint32_t lh,
                                               uint32_t ly, uint32_t x, uint32_t y, uint32_t z) {
    const uint32_t j = (x >> 1) + lh * (y + ly * z);
    return (double)(((x + y + z) & 1u) ? St::ld(f1, j) : St::ld(f0, j));
}

template <class St>
__global__ __launch_bounds__(kOffThreads) void gather_offlattice(const typename St::T* __restrict__ f0,
                                                                 const typename St::T* __restrict__ f1, uint32_t lx,
                                                                 uint32_t ly, uint32_t lz,
                                                                 const double* __restrict__ r,
                                                                 const double* __restrict__ q, uint32_t n,
                                                                 double* __restrict__ partials,
                                                                 double* __restrict__ phit) {
    const uint32_t lh = lx >> 1;
    const double top[3] = {(double)(lx - 2), (double)(ly - 2), (double)(lz - 2)};
    double x_acc = 0.0, y_acc = 0.0;
    for (uint32_t i = blockIdx.x * kOffThreads + threadIdx.x; i < n; i += gridDim.x * kOffThreads) {
        uint32_t b[3];
        double f[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double fl = fmin(floor(r[3 * i + d]), top[d]);
            b[d] = (uint32_t)fl;
            f[d] = r[3 * i + d] - fl;
        }
        double v = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
            const double wx = ex ? f[0] : 1.0 - f[0];
            const double wy = ey ? f[1] : 1.0 - f[1];
            const double wz = ez ? f[2] : 1.0 - f[2];
            const double p = corner_value<St>(f0, f1, lh, ly, b[0] + ex, b[1] + ey, b[2] + ez);
            v = fma(wx * wy * wz, p, v);
            g0 = fma((ex ? 1.0 : -1.0) * wy * wz, p, g0);
            g1 = fma(wx * (ey ? 1.0 : -1.0) * wz, p, g1);
            g2 = fma(wx * wy * (ez ? 1.0 : -1.0), p, g2);
        }
        const double qv = q[i] * v;
        x_acc += qv;
        y_acc = fma(qv, qv, y_acc);
        if (phit) {
            phit[4 * i] = v;
            phit[4 * i + 1] = g0;
            phit[4 * i + 2] = g1;
            phit[4 * i + 3] = g2;
        }
    }
    block_sum2<kOffThreads>(x_acc, y_acc);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = x_acc;
        partials[2 * blockIdx.x + 1] = y_acc;
    }
}

// After the sample's X is final (finalize_measure wrote it to xy[0]): add
// 2 q_i grad phi~_i (X - q_i phi~_i) and its square to charge i's sums.
__global__ __launch_bounds__(kOffThreads) void force_accumulate(const double* __restrict__ q,
                                                                const double* __restrict__ phit, uint32_t n,
                                                                const double* __restrict__ xy,
                                                                double* __restrict__ fsum,
                                                                double* __restrict__ fsq) {
    const uint32_t i = blockIdx.x * kOffThreads + threadIdx.x;
    if (i >= n) return;
    const double X = xy[0];
    const double c = 2.0 * q[i] * (X - q[i] * phit[4 * i]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double g = c * phit[4 * i + 1 + d];
        fsum[3 * i + d] += g;
        fsq[3 * i + d] = fma(g, g, fsq[3 * i + d]);
    }
}

template <class St>
static hipError_t launch_offlattice_t(const OffLatticeArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(gather_offlattice<St>, dim3(a.blocks), dim3(kOffThreads), 0, stream,
                       static_cast<const typename St::T*>(a.field0), static_cast<const typename St::T*>(a.field1),
                       a.lx, a.ly, a.lz, a.r, a.q, a.n, a.partials, a.fsum ? a.phit : nullptr);
    if (hipError_t e = launch_finalize_measure(a.partials, a.blocks, 1u, a.bins, a.m, a.bin_size, a.mdev,
                                               a.last_xy, a.bin_stride, stream))
        return e;
    if (a.fsum && a.n > 0)
        hipLaunchKernelGGL(force_accumulate, dim3((a.n + kOffThreads - 1) / kOffThreads), dim3(kOffThreads), 0,
                           stream, a.q, a.phit, a.n, a.last_xy, a.fsum, a.fsq);
    return hipGetLastError();
}

hipError_t launch_measure_offlattice(const OffLatticeArgs& a, hipStream_t stream) {
    if (a.lx < 2 || a.ly < 2 || a.lz < 2 || (a.lx & 1u)) return hipErrorInvalidValue;
    switch (storage_grid(a.storage)) {
        case 0: return launch_offlattice_t<StoreF32>(a, stream);
        case 1: return launch_offlattice_t<StoreBF16>(a, stream);
        case 2: return launch_offlattice_t<StoreF16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
