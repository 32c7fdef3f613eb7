// Red-black Gaussian heat-bath half-sweeps (the paper's Eq. phi on a Dirichlet
// box), one colour per launch.
//
// Layout: the field is two compact colour arrays of vh = V/2 elements in one
// allocation, colour c at offset c*vh.  Site (x, y, z) of colour
// c = (x+y+z) & 1 sits at compact index j = (x + lx (y + ly z)) >> 1 =
// (x >> 1) + lh (y + ly z), lh = lx/2.  In a row (y, z) the colour-c sites
// have x = 2hx + p with p = (c + y + z) & 1, so the x-neighbours of compact
// column hx are the other colour's columns hx - 1 + p and hx + p; the y- and
// z-neighbours are the other colour's column hx in rows y +- 1 and planes
// z +- 1.  Outside the box the field is 0 (Dirichlet ghosts).
//
// A half-sweep reads only the other colour and writes only its own (the heat
// bath never needs a site's old value): 2 * sizeof(storage) HBM bytes per
// site update.

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

// 4 consecutive compact sites of one row per thread (requires lh % 4 == 0,
// i.e. lx % 8 == 0): one Philox call gives the 4 words, loads and stores are
// 4-wide.  Block (kTX, kTY): kTX quads along x, kTY rows along y; grid.z = z.
template <class St>
__global__ __launch_bounds__(256) void halfsweep_quad(const typename St::T* __restrict__ other,
                                                      typename St::T* __restrict__ own, uint32_t lh,
                                                      uint32_t ly, uint32_t lz, uint32_t c,
                                                      uint32_t h, uint32_t k0, uint32_t k1,
                                                      uint32_t chain) {
    const uint32_t nq = lh >> 2;
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y * blockDim.y + threadIdx.y;
    const uint32_t z = blockIdx.z;
    if (q >= nq || y >= ly) return;
    const uint32_t p = (c + y + z) & 1u;
    const uint32_t plane = ly * lh;
    const uint32_t j0 = (z * ly + y) * lh + 4u * q;

    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 cen = St::ld4(other, j0);
    const float4 ym = y > 0 ? St::ld4(other, j0 - lh) : zero;
    const float4 yp = y + 1 < ly ? St::ld4(other, j0 + lh) : zero;
    const float4 zm = z > 0 ? St::ld4(other, j0 - plane) : zero;
    const float4 zp = z + 1 < lz ? St::ld4(other, j0 + plane) : zero;
    float edge;
    if (p == 0)
        edge = q > 0 ? St::ld(other, j0 - 1) : 0.f;
    else
        edge = q + 1 < nq ? St::ld(other, j0 + 4) : 0.f;

    float a0, a1, a2, a3;  // sum of the two x-neighbours of each site
    if (p == 0) {
        a0 = edge + cen.x;
        a1 = cen.x + cen.y;
        a2 = cen.y + cen.z;
        a3 = cen.z + cen.w;
    } else {
        a0 = cen.x + cen.y;
        a1 = cen.y + cen.z;
        a2 = cen.z + cen.w;
        a3 = cen.w + edge;
    }
    const uint4 r = philox4x32_10(j0 >> 2, h, chain, 0u, k0, k1);
    const float sixth = 1.0f / 6.0f;
    float4 out;
    out.x = fmaf(a0 + ym.x + yp.x + zm.x + zp.x, sixth, heatbath_noise(r.x));
    out.y = fmaf(a1 + ym.y + yp.y + zm.y + zp.y, sixth, heatbath_noise(r.y));
    out.z = fmaf(a2 + ym.z + yp.z + zm.z + zp.z, sixth, heatbath_noise(r.z));
    out.w = fmaf(a3 + ym.w + yp.w + zm.w + zp.w, sixth, heatbath_noise(r.w));
    St::st4(own, j0, out);
}

// One compact site per thread, any even lx.  Site j of colour c.
template <class St>
__global__ __launch_bounds__(256) void halfsweep_generic(const typename St::T* __restrict__ other,
                                                         typename St::T* __restrict__ own,
                                                         uint32_t lh, uint32_t ly, uint32_t lz,
                                                         uint32_t c, uint32_t h, uint32_t k0,
                                                         uint32_t k1, uint32_t chain) {
    const uint32_t vh = lh * ly * lz;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= vh) return;
    const uint32_t hx = j % lh;
    const uint32_t row = j / lh;
    const uint32_t y = row % ly;
    const uint32_t z = row / ly;
    const uint32_t p = (c + y + z) & 1u;
    const uint32_t plane = ly * lh;
    float s = 0.f;
    // x-neighbours: other-colour columns hx - 1 + p and hx + p of this row
    if (hx + p >= 1) s += St::ld(other, j - 1 + p);
    if (hx + p < lh) s += St::ld(other, j + p);
    if (y > 0) s += St::ld(other, j - lh);
    if (y + 1 < ly) s += St::ld(other, j + lh);
    if (z > 0) s += St::ld(other, j - plane);
    if (z + 1 < lz) s += St::ld(other, j + plane);
    const uint4 r = philox4x32_10(j >> 2, h, chain, 0u, k0, k1);
    const uint32_t w = (j & 3u) == 0 ? r.x : (j & 3u) == 1 ? r.y : (j & 3u) == 2 ? r.z : r.w;
    St::st(own, j, fmaf(s, 1.0f / 6.0f, heatbath_noise(w)));
}

// z-marching slab (2.5-D blocking): a workgroup owns a tile of kTX quads x
// kTY rows and walks `zc` planes along z.  Planes z-1 and z+1 of the other
// colour stay in registers (each plane is loaded once per tile); plane z is
// staged in double-buffered LDS with its two halo rows (y0-1, y0+kTY) and the
// two x-edge columns, which give the y- and x-neighbours.  One barrier per
// plane: with two buffers a thread can only overwrite buffer s-1 after every
// thread has passed the barrier of step s, i.e. finished its reads of s-1.
// Global loads per 4 sites: one float4 plus 2/kTY halo rows and 2/(4 kTX)
// edges.  Optional XCD-aware order: hardware block b runs on XCD b % 8, so
// b -> (b % 8) * (nb / 8) + b / 8 gives each XCD a contiguous run of tiles
// (neighbouring tiles share halo rows in that XCD's L2).
template <class St, int kTX, int kTY>
__global__ __launch_bounds__(kTX* kTY) void halfsweep_zslab(const typename St::T* __restrict__ other,
                                                           typename St::T* __restrict__ own, uint32_t lh,
                                                           uint32_t ly, uint32_t lz, uint32_t zc, uint32_t c,
                                                           uint32_t h, uint32_t k0, uint32_t k1,
                                                           uint32_t chain, uint32_t xcd_order) {
    static_assert(kTY >= 2, "halo rows are loaded by the first two thread rows");
    constexpr int kW = 4 * kTX + 2;  // LDS row: left edge, 4 kTX sites, right edge
    __shared__ float tile[2][kTY + 2][kW];

    const uint32_t nq = lh >> 2;
    const uint32_t nbx = (nq + kTX - 1) / kTX, nby = (ly + kTY - 1) / kTY;
    const uint32_t nb = gridDim.x;
    uint32_t b = blockIdx.x;
    if (xcd_order) {
        const uint32_t per = nb / 8u;
        if (b < 8u * per) b = (b % 8u) * per + b / 8u;
    }
    const uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const uint32_t q0 = bx * kTX, y0 = by * kTY;
    const uint32_t q = q0 + tx, y = y0 + ty;
    const uint32_t z0 = bz * zc;
    const uint32_t z1 = min(z0 + zc, lz);
    const bool active = q < nq && y < ly;
    const uint32_t plane = ly * lh;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);

    // halo row handled by this thread (first two thread rows only)
    const bool halo_thread = ty < 2 && q < nq;
    const uint32_t hy = ty == 0 ? y0 - 1u : y0 + kTY;  // wraps for y0 = 0: excluded below
    const bool halo_in = halo_thread && (ty == 0 ? y0 > 0 : y0 + kTY < ly);
    // x-edge column handled by this thread (first and last columns of the tile)
    const bool left_edge = tx == 0 && y < ly && q0 > 0;
    const bool right_edge = tx == kTX - 1 && y < ly && (q0 + kTX) < nq;

    const uint32_t rowj = y * lh + 4u * q;      // offset of the thread's quad within a plane
    const uint32_t haloj = hy * lh + 4u * q;
    const uint32_t edgej = y * lh + 4u * q0;    // first site of the tile row

    float4 bm = (active && z0 > 0) ? St::ld4(other, (z0 - 1) * plane + rowj) : zero;
    float4 bc = active ? St::ld4(other, z0 * plane + rowj) : zero;
    float4 hc = halo_in ? St::ld4(other, z0 * plane + haloj) : zero;
    float el = left_edge ? St::ld(other, z0 * plane + edgej - 1) : 0.f;
    float er = right_edge ? St::ld(other, z0 * plane + edgej + 4 * kTX) : 0.f;

    const float sixth = 1.0f / 6.0f;
    for (uint32_t z = z0; z < z1; ++z) {
        const int buf = (z - z0) & 1;
        float* row = &tile[buf][ty + 1][1 + 4 * tx];
        row[0] = bc.x;
        row[1] = bc.y;
        row[2] = bc.z;
        row[3] = bc.w;
        if (ty < 2) {
            float* hr = &tile[buf][ty == 0 ? 0 : kTY + 1][1 + 4 * tx];
            hr[0] = hc.x;
            hr[1] = hc.y;
            hr[2] = hc.z;
            hr[3] = hc.w;
        }
        if (tx == 0) tile[buf][ty + 1][0] = el;
        if (tx == kTX - 1) tile[buf][ty + 1][kW - 1] = er;
        // prefetch plane z + 1 (the z+1 neighbour now, the centre next step)
        const bool more = z + 1 < lz;
        const float4 bn = (active && more) ? St::ld4(other, (z + 1) * plane + rowj) : zero;
        const float4 hn = (halo_in && z + 1 < z1) ? St::ld4(other, (z + 1) * plane + haloj) : zero;
        const float eln = (left_edge && z + 1 < z1) ? St::ld(other, (z + 1) * plane + edgej - 1) : 0.f;
        const float ern = (right_edge && z + 1 < z1) ? St::ld(other, (z + 1) * plane + edgej + 4 * kTX) : 0.f;
        __syncthreads();
        if (active) {
            const float* up = &tile[buf][ty][1 + 4 * tx];
            const float* dn = &tile[buf][ty + 2][1 + 4 * tx];
            const float* mid = &tile[buf][ty + 1][1 + 4 * tx];
            const uint32_t p = (c + y + z) & 1u;
            // x-neighbours of site k: other columns h0+k-1+p and h0+k+p
            const float e = p == 0 ? mid[-1] : mid[4];
            float a0, a1, a2, a3;
            if (p == 0) {
                a0 = e + bc.x;
                a1 = bc.x + bc.y;
                a2 = bc.y + bc.z;
                a3 = bc.z + bc.w;
            } else {
                a0 = bc.x + bc.y;
                a1 = bc.y + bc.z;
                a2 = bc.z + bc.w;
                a3 = bc.w + e;
            }
            const uint32_t j0 = z * plane + rowj;
            const uint4 r = philox4x32_10(j0 >> 2, h, chain, 0u, k0, k1);
            float4 out;
            out.x = fmaf(a0 + up[0] + dn[0] + bm.x + bn.x, sixth, heatbath_noise(r.x));
            out.y = fmaf(a1 + up[1] + dn[1] + bm.y + bn.y, sixth, heatbath_noise(r.y));
            out.z = fmaf(a2 + up[2] + dn[2] + bm.z + bn.z, sixth, heatbath_noise(r.z));
            out.w = fmaf(a3 + up[3] + dn[3] + bm.w + bn.w, sixth, heatbath_noise(r.w));
            St::st4(own, j0, out);
        }
        bm = bc;
        bc = bn;
        hc = hn;
        el = eln;
        er = ern;
    }
}

template <class St>
static hipError_t launch_halfsweep_t(const SweepArgs& a, hipStream_t stream) {
    using T = typename St::T;
    const T* field = static_cast<const T*>(a.field);
    const T* other = field + (size_t)(a.c ^ 1u) * a.vh;
    T* own = const_cast<T*>(field) + (size_t)a.c * a.vh;
    if (a.variant == kVariantZslab) {
        constexpr int kTX = 32, kTY = 8;
        const uint32_t nq = a.lh >> 2;
        const uint32_t zc = a.zc ? a.zc : 32u;
        const uint32_t nb = ((nq + kTX - 1) / kTX) * ((a.ly + kTY - 1) / kTY) * ((a.lz + zc - 1) / zc);
        hipLaunchKernelGGL((halfsweep_zslab<St, kTX, kTY>), dim3(nb), dim3(kTX, kTY, 1), 0, stream, other, own,
                           a.lh, a.ly, a.lz, zc, a.c, a.h, a.k0, a.k1, a.chain, a.xcd_order);
    } else if (a.variant == kVariantQuad) {
        const uint32_t nq = a.lh >> 2;
        const uint32_t tx = nq >= 16 ? 16 : nq;
        const uint32_t ty = 256 / tx;
        dim3 block(tx, ty, 1);
        dim3 grid((nq + tx - 1) / tx, (a.ly + ty - 1) / ty, a.lz);
        hipLaunchKernelGGL(halfsweep_quad<St>, grid, block, 0, stream, other, own, a.lh, a.ly, a.lz,
                           a.c, a.h, a.k0, a.k1, a.chain);
    } else {
        dim3 block(256, 1, 1);
        dim3 grid((a.vh + 255) / 256, 1, 1);
        hipLaunchKernelGGL(halfsweep_generic<St>, grid, block, 0, stream, other, own, a.lh, a.ly,
                           a.lz, a.c, a.h, a.k0, a.k1, a.chain);
    }
    return hipGetLastError();
}

hipError_t launch_halfsweep(const SweepArgs& a, hipStream_t stream) {
    switch (a.storage) {
        case 0: return launch_halfsweep_t<StoreF32>(a, stream);
        case 1: return launch_halfsweep_t<StoreBF16>(a, stream);
        case 2: return launch_halfsweep_t<StoreF16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
