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
                                                      uint32_t chain, const uint32_t* __restrict__ tdev) {
    if (tdev) h += 2u * tdev[0];  // graph replays: sweep counter kept on the device
    const uint32_t nq = lh >> 2;
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y * blockDim.y + threadIdx.y;
    const uint32_t z = blockIdx.z;
    if (q >= nq || y >= ly) return;
    const uint32_t p = (c + y + z) & 1u;
    const uint32_t plane = ly * lh;
    const uint32_t j0 = (z * ly + y) * lh + 4u * q;

    const QuadOut out = quad_update_global<St>(other, j0, lh, plane, y > 0, y + 1 < ly, z > 0, z + 1 < lz,
                                               p == 0 ? q > 0 : q + 1 < nq, p, h, chain, k0, k1);
    St::st4(own, j0, out.v, out.w);
}

// One compact site per thread, any even lx.  Site j of colour c.
template <class St>
__global__ __launch_bounds__(256) void halfsweep_generic(const typename St::T* __restrict__ other,
                                                         typename St::T* __restrict__ own,
                                                         uint32_t lh, uint32_t ly, uint32_t lz,
                                                         uint32_t c, uint32_t h, uint32_t k0,
                                                         uint32_t k1, uint32_t chain,
                                                         const uint32_t* __restrict__ tdev) {
    if (tdev) h += 2u * tdev[0];
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
    St::st(own, j, fmaf(s, 1.0f / 6.0f, heatbath_noise(w)), w);
}

// z-marching slab (2.5-D blocking): a workgroup owns a tile of kTX quads x
// kTY rows and walks `zc` planes along z.  Planes z-1, z and z+1 of the other
// colour stay in registers (each plane is loaded once per tile); plane z is
// also staged in double-buffered LDS with its two halo rows (y0-1, y0+kTY)
// and the two x-edge columns, which give the y- and x-neighbours.  One
// barrier per plane: with two buffers a thread only overwrites buffer s-1
// after every thread has passed the barrier of step s, i.e. finished its
// reads of s-1.  Global loads per 4 sites: one 16-byte load plus 2/kTY halo
// rows and 2/(4 kTX) edges.
//
// The plane loop is unrolled 6-fold (lcm of the 3 register planes and the 2
// LDS buffers) so no register is copied between planes.  A wave holds
// R = 64 / kTX thread rows; thread rows are mapped to tile rows so that each
// wave gets R rows of one parity (within every group of 2R rows the first
// wave takes the even rows, the second the odd ones), so p = (c + y + z) & 1
// and the x-pair branch are uniform per wave.  Optional XCD-aware order: hardware block b
// runs on XCD b % 8, so b -> (b % 8) * (nb / 8) + b / 8 gives each XCD a
// contiguous run of tiles, whose halo rows then meet in that XCD's L2.
template <class St, int kTX, int kTY>
struct Zslab {
    static constexpr int kR = 64 / kTX;  // thread rows per wave
    static_assert(kTX * kR == 64 && kR >= 1, "a wave must hold whole thread rows");
    static_assert(kTY >= 2 && kTY % (2 * kR) == 0, "rows are permuted in groups of two waves");
    // thread row t -> tile row: t = g*2R + w*R + i  ->  g*2R + 2i + w
    static __device__ __forceinline__ int tile_row(int t) {
        const int g = t / (2 * kR), w = (t / kR) & 1, i = t % kR;
        return g * 2 * kR + 2 * i + w;
    }
    static constexpr int kW = 4 * kTX + 8;  // LDS row: 3 pad, left edge, 4 kTX sites, right edge, 3 pad
    static constexpr uint32_t kEsz = St::kBytes;
    using T = typename St::T;

    __amdgpu_buffer_rsrc_t src;  // the other colour; loads past its end read 0
    T* __restrict__ own;
    uint32_t plane, plane_b, c, h, k0, k1, chain;
    uint32_t y, z1, rowj;
    uint32_t rowb, halob, edgeb;  // byte offsets within a plane; kNoLoad for lanes with no load
    int tx, ty, row;
    bool active;
    float (*tile)[kTY + 2][kW];

    // plane z of the thread's quad (0 past the last plane or for inactive lanes)
    __device__ __forceinline__ float4 centre(uint32_t z) const { return St::bld4(src, z * plane_b + rowb); }
    __device__ __forceinline__ float4 halo(uint32_t z) const { return St::bld4(src, z * plane_b + halob); }
    __device__ __forceinline__ float edge(uint32_t z) const { return St::bld(src, z * plane_b + edgeb); }

    // stage plane z (centre row, halo rows, x-edges) in LDS buffer `buf`
    __device__ __forceinline__ void stage(int buf, const float4& bc, const float4& hc, float ec) const {
        *reinterpret_cast<float4*>(&tile[buf][row + 1][4 + 4 * tx]) = bc;
        if (ty < 2) *reinterpret_cast<float4*>(&tile[buf][ty == 0 ? 0 : kTY + 1][4 + 4 * tx]) = hc;
        if (tx == 0) tile[buf][row + 1][3] = ec;
        if (tx == kTX - 1) tile[buf][row + 1][kW - 4] = ec;
    }

    // update own colour at plane z from planes z-1, z, z+1 (registers) and
    // the y/x-neighbours of plane z (LDS buffer `buf`)
    __device__ __forceinline__ void update(uint32_t z, int buf, const float4& bm, const float4& bc,
                                           const float4& bn) const {
        if (!active) return;
        const float4 up = *reinterpret_cast<const float4*>(&tile[buf][row][4 + 4 * tx]);
        const float4 dn = *reinterpret_cast<const float4*>(&tile[buf][row + 2][4 + 4 * tx]);
        // uniform per wave (both rows of a wave have the same parity): say so,
        // so the branch below is a scalar branch
        const uint32_t p = __builtin_amdgcn_readfirstlane((c + y + z) & 1u);
        const float e = p == 0 ? tile[buf][row + 1][3 + 4 * tx] : tile[buf][row + 1][8 + 4 * tx];
        const uint32_t j0 = z * plane + rowj;
        const QuadOut out = heatbath_quad(bm, bc, bn, up, dn, e, p, j0, h, chain, k0, k1);
        St::st4(own, j0, out.v, out.w);
    }

    // one plane: stage bc (+ halo, edges) in LDS buffer kBuf, prefetch plane
    // z+1 into bn/hn/en, update own colour at plane z
    template <int kBuf>
    __device__ __forceinline__ void step(uint32_t z, const float4& bm, const float4& bc, float4& bn,
                                         const float4& hc, float4& hn, float ec, float& en) const {
        stage(kBuf, bc, hc, ec);
        bn = centre(z + 1);
        if (z + 1 < z1) {  // block-uniform
            if (ty < 2) hn = halo(z + 1);  // wave-uniform: the first wave loads the halo rows
            en = edge(z + 1);
        }
        __syncthreads();
        update(z, kBuf, bm, bc, bn);
    }
};

// Tile set-up shared by the slab kernels: block -> tile (optionally
// XCD-ordered), per-thread byte offsets of the centre, halo and edge loads.
// Returns the first plane of the block's slab.
template <class St, int kTX, int kTY>
__device__ __forceinline__ uint32_t zslab_setup(Zslab<St, kTX, kTY>& k, const typename St::T* other,
                                                typename St::T* own, uint32_t lh, uint32_t ly, uint32_t lz,
                                                uint32_t zc, uint32_t c, uint32_t h, uint32_t k0, uint32_t k1,
                                                uint32_t chain, uint32_t xcd_order,
                                                float (*tile)[kTY + 2][Zslab<St, kTX, kTY>::kW]) {
    using K = Zslab<St, kTX, kTY>;
    const uint32_t nq = lh >> 2;
    const uint32_t nbx = (nq + kTX - 1) / kTX, nby = (ly + kTY - 1) / kTY;
    const uint32_t nb = gridDim.x;
    uint32_t b = blockIdx.x;
    if (xcd_order) {
        const uint32_t per = nb / 8u;
        if (b < 8u * per) b = (b % 8u) * per + b / 8u;
    }
    const uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    constexpr uint32_t E = K::kEsz;
    k.plane = ly * lh;
    k.plane_b = k.plane * E;
    k.src = make_rsrc(other, k.plane_b * lz);
    k.own = own;
    k.c = c;
    k.h = h;
    k.k0 = k0;
    k.k1 = k1;
    k.chain = chain;
    k.tile = tile;
    k.tx = threadIdx.x;
    k.ty = threadIdx.y;
    k.row = K::tile_row(k.ty);
    const uint32_t q0 = bx * kTX, y0 = by * kTY;
    const uint32_t q = q0 + k.tx;
    k.y = y0 + k.row;
    const uint32_t z0 = bz * zc;
    k.z1 = min(z0 + zc, lz);
    k.active = q < nq && k.y < ly;
    k.rowj = k.y * lh + 4u * q;
    k.rowb = k.active ? k.rowj * E : kNoLoad;
    // halo rows: thread row 0 loads row y0-1, thread row 1 loads row y0+kTY
    const bool halo_in = k.ty < 2 && q < nq && (k.ty == 0 ? y0 > 0 : y0 + kTY < ly);
    const uint32_t hy = k.ty == 0 ? y0 - 1u : y0 + kTY;
    k.halob = halo_in ? (hy * lh + 4u * q) * E : kNoLoad;
    // x-edges: the first thread of a row loads the column left of the tile,
    // the last thread the column right of it
    const uint32_t edge_row = k.y * lh + 4u * q0;
    if (k.tx == 0 && k.y < ly && q0 > 0)
        k.edgeb = (edge_row - 1u) * E;
    else if (k.tx == kTX - 1 && k.y < ly && q0 + kTX < nq)
        k.edgeb = (edge_row + 4u * kTX) * E;
    else
        k.edgeb = kNoLoad;
    return z0;
}

// Requires vh * sizeof(storage) < 2^31 (kNoLoad must lie past the array).
// kWPE: minimum waves per SIMD the register allocation must allow.
template <class St, int kTX, int kTY, int kWPE>
__global__ __launch_bounds__(kTX* kTY) __attribute__((amdgpu_waves_per_eu(kWPE, 8))) void halfsweep_zslab(const typename St::T* __restrict__ other,
                                                           typename St::T* __restrict__ own, uint32_t lh,
                                                           uint32_t ly, uint32_t lz, uint32_t zc, uint32_t c,
                                                           uint32_t h, uint32_t k0, uint32_t k1,
                                                           uint32_t chain, uint32_t xcd_order,
                                                           const uint32_t* __restrict__ tdev) {
    if (tdev) h += 2u * tdev[0];
    using K = Zslab<St, kTX, kTY>;
    __shared__ __align__(16) float tile[2][kTY + 2][K::kW];
    K k;
    const uint32_t z0 = zslab_setup<St, kTX, kTY>(k, other, own, lh, ly, lz, zc, c, h, k0, k1, chain, xcd_order, tile);

    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 B0 = z0 > 0 ? k.centre(z0 - 1) : zero;
    float4 B1 = k.centre(z0), B2 = zero;
    float4 H0 = k.ty < 2 ? k.halo(z0) : zero, H1 = zero;
    float E0 = k.edge(z0), E1 = 0.f;
    const uint32_t z1 = k.z1;
    for (uint32_t z = z0; z < z1; z += 6) {
        k.template step<0>(z, B0, B1, B2, H0, H1, E0, E1);
        if (z + 1 >= z1) break;
        k.template step<1>(z + 1, B1, B2, B0, H1, H0, E1, E0);
        if (z + 2 >= z1) break;
        k.template step<0>(z + 2, B2, B0, B1, H0, H1, E0, E1);
        if (z + 3 >= z1) break;
        k.template step<1>(z + 3, B0, B1, B2, H1, H0, E1, E0);
        if (z + 4 >= z1) break;
        k.template step<0>(z + 4, B1, B2, B0, H0, H1, E0, E1);
        if (z + 5 >= z1) break;
        k.template step<1>(z + 5, B2, B0, B1, H1, H0, E1, E0);
    }
}

template <class St>
static hipError_t launch_halfsweep_t(const SweepArgs& a, hipStream_t stream) {
    using T = typename St::T;
    const T* field = static_cast<const T*>(a.field);
    const T* other = field + (size_t)(a.c ^ 1u) * a.vh;
    T* own = const_cast<T*>(field) + (size_t)a.c * a.vh;
    if (a.variant == kVariantZslab) {
        if ((uint64_t)a.vh * St::kBytes >= (1ull << 31)) return hipErrorInvalidValue;  // kNoLoad must be out of range
        const uint32_t zc = a.zc ? a.zc : 16u;
        const uint32_t nq = a.lh >> 2;
        auto launch = [&](auto kern, int tx, int ty) {
            const uint32_t nb = ((nq + tx - 1) / tx) * ((a.ly + ty - 1) / ty) * ((a.lz + zc - 1) / zc);
            hipLaunchKernelGGL(kern, dim3(nb), dim3(tx, ty, 1), 0, stream, other, own, a.lh, a.ly, a.lz, zc, a.c,
                               a.h, a.k0, a.k1, a.chain, a.xcd_order, a.tdev);
        };
        switch (a.tile) {  // tile quads x rows, minimum waves per SIMD
            case 0: launch(halfsweep_zslab<St, 32, 8, 1>, 32, 8); break;
            case 1: launch(halfsweep_zslab<St, 32, 8, 5>, 32, 8); break;
            case 2: launch(halfsweep_zslab<St, 32, 8, 6>, 32, 8); break;
            case 3: launch(halfsweep_zslab<St, 32, 8, 8>, 32, 8); break;
            case 4: launch(halfsweep_zslab<St, 16, 8, 6>, 16, 8); break;
            case 5: launch(halfsweep_zslab<St, 32, 4, 6>, 32, 4); break;
            case 6: launch(halfsweep_zslab<St, 64, 4, 4>, 64, 4); break;
            case 7: launch(halfsweep_zslab<St, 16, 16, 4>, 16, 16); break;
            default: return hipErrorInvalidValue;
        }
    } else if (a.variant == kVariantQuad) {
        const uint32_t nq = a.lh >> 2;
        const uint32_t tx = nq >= 16 ? 16 : nq;
        const uint32_t ty = 256 / tx;
        dim3 block(tx, ty, 1);
        dim3 grid((nq + tx - 1) / tx, (a.ly + ty - 1) / ty, a.lz);
        hipLaunchKernelGGL(halfsweep_quad<St>, grid, block, 0, stream, other, own, a.lh, a.ly, a.lz,
                           a.c, a.h, a.k0, a.k1, a.chain, a.tdev);
    } else {
        dim3 block(256, 1, 1);
        dim3 grid((a.vh + 255) / 256, 1, 1);
        hipLaunchKernelGGL(halfsweep_generic<St>, grid, block, 0, stream, other, own, a.lh, a.ly,
                           a.lz, a.c, a.h, a.k0, a.k1, a.chain, a.tdev);
    }
    return hipGetLastError();
}

// Sets / advances the device-side sweep and sample counters (graph replays).
__global__ void set_counters(uint32_t* ctr, uint32_t t, uint32_t m) {
    ctr[0] = t;
    ctr[1] = m;
}
__global__ void advance_counters(uint32_t* ctr, uint32_t dt, uint32_t dm) {
    ctr[0] += dt;
    ctr[1] += dm;
}
hipError_t launch_set_counters(uint32_t* ctr, uint32_t t, uint32_t m, hipStream_t stream) {
    hipLaunchKernelGGL(set_counters, dim3(1), dim3(1), 0, stream, ctr, t, m);
    return hipGetLastError();
}
hipError_t launch_advance_counters(uint32_t* ctr, uint32_t dt, uint32_t dm, hipStream_t stream) {
    hipLaunchKernelGGL(advance_counters, dim3(1), dim3(1), 0, stream, ctr, dt, dm);
    return hipGetLastError();
}

hipError_t launch_halfsweep(const SweepArgs& a, hipStream_t stream) {
    if (a.variant == kVariantStream) return launch_halfsweep_stream(a, stream);
    switch (a.storage) {
        case 0: return launch_halfsweep_t<StoreF32>(a, stream);
        case 1: return launch_halfsweep_t<StoreBF16>(a, stream);
        case 2: return launch_halfsweep_t<StoreF16>(a, stream);
        case 3: return launch_halfsweep_t<StoreBF16SR>(a, stream);
        case 4: return launch_halfsweep_t<StoreF16SR>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
