// Fused red-black sweep (temporal blocking of the two half-sweeps of one
// sweep): colour 0 is updated from the old colour 1 and colour 1 from the new
// colour 0 in one pass over HBM.
//
// A workgroup owns full-width x rows [y0, y0+TY) and planes [z0, z1) and
// walks z with a lag of one plane between the colours:
//   1. load old colour-1 plane zb = z - 1 + 2 rows of halo on each side into
//      an LDS ring of 3 planes (planes or rows outside the box read 0);
//   2. compute new colour-0 plane za = zb - 1 on rows y0-1 .. y0+TY from the
//      ring (the two halo rows are recomputed here; they draw the same Philox
//      numbers as in the workgroup that owns them, so the values agree) into
//      a second LDS ring; rows and planes the workgroup owns are also stored;
//   3. compute new colour-1 plane zc = za - 1 on its own rows from the
//      colour-0 ring and store it.
// Two barriers per plane.  Ring slots are overwritten only after a barrier
// that follows their last read (step 1 of plane z+1 overwrites the colour-1
// slot read by step 2 of plane z-1; step 2 of plane z+1 the colour-0 slot
// read by step 3 of plane z-1).
//
// Colour 1 is read from b_in and written to b_out, a different array:
// neighbouring workgroups still read old colour-1 halo rows while this one
// writes new values.  New colour-0 values are rounded to the storage format
// before colour 1 uses them, exactly as when they go through memory.
//
// HBM traffic per sweep: read colour 1, write colour 0 and colour 1 (6 bytes
// per site update in FP32 instead of 8), plus halo rows and planes.

#include "device_common.hpp"
#include "kernels.hpp"
#include "runtime_common.hpp"

namespace latcoul {

constexpr int kFusedRowLanes = 8;                // thread rows per workgroup (R)
constexpr size_t kFusedLdsBytes = 160 * 1024;   // LDS per CU on gfx950

// Largest TY whose two LDS rings fit: 3 planes x ((TY+4) + (TY+2)) rows x lh floats.
static uint32_t fused_rows(uint32_t lh) {
    const int64_t rows = (int64_t)(kFusedLdsBytes / (3u * 4u * (size_t)lh)) - 6;
    int64_t ty = rows / 2;
    if (ty > 2 * kFusedRowLanes - 2) ty = 2 * kFusedRowLanes - 2;  // A rows = TY + 2 = 2R: no idle lanes
    return ty < 2 ? 0u : (uint32_t)ty;
}

bool fused_sweep_supported(uint32_t lh, uint32_t ly) {
    (void)ly;
    const uint32_t nq = lh >> 2;
    return (lh & 3u) == 0 && nq >= 8 && nq * kFusedRowLanes <= 1024 && fused_rows(lh) >= 2;
}

template <class St>
__global__ __launch_bounds__(1024) void fused_sweep(typename St::T* __restrict__ c0,
                                                    const typename St::T* __restrict__ b_in,
                                                    typename St::T* __restrict__ b_out, uint32_t lh, uint32_t ly,
                                                    uint32_t lz, uint32_t ty_rows, uint32_t zc, uint32_t h0,
                                                    uint32_t k0, uint32_t k1, uint32_t chain, uint32_t xcd_order,
                                                    const uint32_t* __restrict__ tdev) {
    if (tdev) h0 += 2u * tdev[0];  // graph replays: sweep counter kept on the device
    extern __shared__ __align__(16) float lds[];
    const uint32_t TY = ty_rows, nq = lh >> 2;
    const uint32_t rowsB = TY + 4, rowsA = TY + 2;
    float* ringB = lds;                       // [3][rowsB][lh], row r <-> y0 - 2 + r
    float* ringA = lds + 3 * rowsB * lh;      // [3][rowsA][lh], row r <-> y0 - 1 + r
    const uint32_t nby = (ly + TY - 1) / TY;
    uint32_t b = blockIdx.x;
    if (xcd_order) {
        const uint32_t nb = gridDim.x, per = nb / 8u;
        if (b < 8u * per) b = (b % 8u) * per + b / 8u;
    }
    const uint32_t by = b % nby, bz = b / nby;
    const int y0 = (int)(by * TY);
    const int z0 = (int)(bz * zc);
    const int z1 = min(z0 + (int)zc, (int)lz);
    const uint32_t q = threadIdx.x % nq, r0 = threadIdx.x / nq;
    const uint32_t plane = ly * lh;
    const float sixth = 1.0f / 6.0f;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    auto slot = [](int z) { return (uint32_t)(((z % 3) + 3) % 3); };
    auto B4 = [&](uint32_t s, uint32_t r) -> float4& {
        return *reinterpret_cast<float4*>(&ringB[(s * rowsB + r) * lh + 4 * q]);
    };
    auto A4 = [&](uint32_t s, uint32_t r) -> float4& {
        return *reinterpret_cast<float4*>(&ringA[(s * rowsA + r) * lh + 4 * q]);
    };

    for (int i = 0;; ++i) {
        const int zb = z0 - 2 + i, za = zb - 1, zo = za - 1;
        if (zo >= z1) break;
        // 1. old colour 1, plane zb (needed up to plane z1 + 1)
        if (zb <= z1 + 1) {
            const uint32_t s = slot(zb);
            for (uint32_t r = r0; r < rowsB; r += kFusedRowLanes) {
                const int y = y0 - 2 + (int)r;
                float4 v = zero;
                if (zb >= 0 && zb < (int)lz && y >= 0 && y < (int)ly)
                    v = St::ld4(b_in, (uint32_t)zb * plane + (uint32_t)y * lh + 4 * q);
                B4(s, r) = v;
            }
        }
        __syncthreads();
        // 2. new colour 0, plane za, rows y0-1 .. y0+TY
        if (za >= z0 - 1 && za <= z1) {
            const uint32_t s = slot(za), sm = slot(za - 1), sp = slot(za + 1);
            for (uint32_t r = r0; r < rowsA; r += kFusedRowLanes) {
                const int y = y0 - 1 + (int)r;
                float4 out = zero;
                if (za >= 0 && za < (int)lz && y >= 0 && y < (int)ly) {
                    const uint32_t rb = r + 1;  // the same row in ringB
                    const float4 cen = B4(s, rb), ym = B4(s, rb - 1), yp = B4(s, rb + 1);
                    const float4 zm = B4(sm, rb), zp = B4(sp, rb);
                    const uint32_t p = ((uint32_t)y + (uint32_t)za) & 1u;  // colour 0
                    const float* rowp = &ringB[(s * rowsB + rb) * lh];
                    float a0, a1, a2, a3;
                    if (p == 0) {
                        const float e = q > 0 ? rowp[4 * q - 1] : 0.f;
                        a0 = e + cen.x;
                        a1 = cen.x + cen.y;
                        a2 = cen.y + cen.z;
                        a3 = cen.z + cen.w;
                    } else {
                        const float e = q + 1 < nq ? rowp[4 * q + 4] : 0.f;
                        a0 = cen.x + cen.y;
                        a1 = cen.y + cen.z;
                        a2 = cen.z + cen.w;
                        a3 = cen.w + e;
                    }
                    const uint32_t j0 = (uint32_t)za * plane + (uint32_t)y * lh + 4 * q;
                    const uint4 rr = philox4x32_10(j0 >> 2, h0, chain, 0u, k0, k1);
                    out.x = fmaf(a0 + ym.x + yp.x + zm.x + zp.x, sixth, heatbath_noise(rr.x));
                    out.y = fmaf(a1 + ym.y + yp.y + zm.y + zp.y, sixth, heatbath_noise(rr.y));
                    out.z = fmaf(a2 + ym.z + yp.z + zm.z + zp.z, sixth, heatbath_noise(rr.z));
                    out.w = fmaf(a3 + ym.w + yp.w + zm.w + zp.w, sixth, heatbath_noise(rr.w));
                    const float4 v = out;
                    out = St::round4(v, rr);
                    if (za >= z0 && za < z1 && y >= y0 && y < y0 + (int)TY) St::st4(c0, j0, v, rr);
                }
                A4(s, r) = out;
            }
        }
        __syncthreads();
        // 3. new colour 1, plane zo, own rows
        if (zo >= z0) {
            const uint32_t s = slot(zo), sm = slot(zo - 1), sp = slot(zo + 1);
            for (uint32_t r = r0; r < TY; r += kFusedRowLanes) {
                const int y = y0 + (int)r;
                if (y >= (int)ly) continue;
                const uint32_t ra = r + 1;  // the same row in ringA
                const float4 cen = A4(s, ra), ym = A4(s, ra - 1), yp = A4(s, ra + 1);
                const float4 zm = A4(sm, ra), zp = A4(sp, ra);
                const uint32_t p = (1u + (uint32_t)y + (uint32_t)zo) & 1u;  // colour 1
                const float* rowp = &ringA[(s * rowsA + ra) * lh];
                float a0, a1, a2, a3;
                if (p == 0) {
                    const float e = q > 0 ? rowp[4 * q - 1] : 0.f;
                    a0 = e + cen.x;
                    a1 = cen.x + cen.y;
                    a2 = cen.y + cen.z;
                    a3 = cen.z + cen.w;
                } else {
                    const float e = q + 1 < nq ? rowp[4 * q + 4] : 0.f;
                    a0 = cen.x + cen.y;
                    a1 = cen.y + cen.z;
                    a2 = cen.z + cen.w;
                    a3 = cen.w + e;
                }
                const uint32_t j0 = (uint32_t)zo * plane + (uint32_t)y * lh + 4 * q;
                const uint4 rr = philox4x32_10(j0 >> 2, h0 + 1u, chain, 0u, k0, k1);
                float4 out;
                out.x = fmaf(a0 + ym.x + yp.x + zm.x + zp.x, sixth, heatbath_noise(rr.x));
                out.y = fmaf(a1 + ym.y + yp.y + zm.y + zp.y, sixth, heatbath_noise(rr.y));
                out.z = fmaf(a2 + ym.z + yp.z + zm.z + zp.z, sixth, heatbath_noise(rr.z));
                out.w = fmaf(a3 + ym.w + yp.w + zm.w + zp.w, sixth, heatbath_noise(rr.w));
                St::st4(b_out, j0, out, rr);
            }
        }
    }
}

template <class St>
static hipError_t launch_fused_t(const FusedArgs& a, hipStream_t stream) {
    using T = typename St::T;
    const uint32_t ty = fused_rows(a.lh);
    const uint32_t nq = a.lh >> 2;
    const uint32_t zc = a.slab ? a.slab : 32u;
    const uint32_t nb = ((a.ly + ty - 1) / ty) * ((a.lz + zc - 1) / zc);
    const size_t lds = (size_t)3 * ((ty + 4) + (ty + 2)) * a.lh * sizeof(float);
    hipLaunchKernelGGL(fused_sweep<St>, dim3(nb), dim3(nq * kFusedRowLanes), lds, stream,
                       static_cast<T*>(a.c0), static_cast<const T*>(a.b_in), static_cast<T*>(a.b_out), a.lh, a.ly,
                       a.lz, ty, zc, a.h0, a.k0, a.k1, a.chain, a.xcd_order, a.tdev);
    return hipGetLastError();
}

// Allow the fused kernels the whole LDS of a CU (dynamic shared memory);
// called once before any fused launch, outside stream capture.
hipError_t prepare_fused_sweep() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_sweep<StoreF32>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_sweep<StoreBF16>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_sweep<StoreF16>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_sweep<StoreBF16SR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_sweep<StoreF16SR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes);
    return e;
}

hipError_t launch_fused_sweep(const FusedArgs& a, hipStream_t stream) {
    if (!fused_sweep_supported(a.lh, a.ly)) return hipErrorInvalidValue;
    switch (a.storage) {
        case 0: return launch_fused_t<StoreF32>(a, stream);
        case 1: return launch_fused_t<StoreBF16>(a, stream);
        case 2: return launch_fused_t<StoreF16>(a, stream);
        case 3: return launch_fused_t<StoreBF16SR>(a, stream);
        case 4: return launch_fused_t<StoreF16SR>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
