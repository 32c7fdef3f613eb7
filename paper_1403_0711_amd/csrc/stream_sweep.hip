// Streaming slab half-sweep: a producer wave feeds an LDS ring of planes
// with direct buffer-to-LDS loads, the compute waves update from LDS.
//
// A workgroup owns a tile of 32m quads (128m same-colour sites, m = 1..4) x
// kTY rows and walks `zc` planes along z, as the z-slab kernel does; what
// differs is who loads.  The workgroup is m kTY/2 compute waves plus one
// producer wave; a compute wave holds a 32-quad strip of two rows of the
// same parity, so the x-pairing of the update is uniform per wave.  A tile
// as wide as the box's rows makes every plane of the tile one contiguous run
// of memory.  The
// producer copies each plane of the other colour that the tile needs (its
// kTY rows, the halo rows y0-1 and y0+kTY, and the quads left and right of
// the tile) with `buffer_load ... lds`, which writes LDS without passing
// through registers, into a ring of R plane slots (R = 5..7), R-3 planes
// ahead of the plane being updated.  Its only memory operations are these
// loads, which complete in order, so a wait that leaves the newest planes in
// flight (vmcnt = their loads) is exact.  The compute waves read the 7-point
// neighbourhood from LDS and only store to HBM: they never wait for a load
// they issued, and never for their stores.
//
// Ring protocol (one workgroup barrier per plane; plane z0-1+l in slot l%R):
//   before barrier b_s the planes l = 0 .. s+2 (z0-1 .. z0+s+1) have landed;
//   step s (between b_s and b_{s+1}): the compute waves update plane z0+s
//   from slots s, s+1, s+2; the producer fills plane l = s+R-1 into slot
//   (s-1)%R, which held plane l = s-1, last read in step s-1 (before b_s),
//   then waits until plane l = s+3 has landed, leaving l = s+4 .. s+R-1 in
//   flight.
// Each load so has R-3 steps to land.  Lanes whose data lies outside the box
// (halo rows at y = -1 or ly, quads left of 0 or right of the row, ragged
// tiles) are masked off and never write: the ring is zeroed once, so they
// read 0, the Dirichlet ghost.  The plane past the last (z = lz) is zeroed
// by the producer with LDS stores.

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

template <class St, int kM, int kTY, int kRing_>
struct Stream {
    static constexpr int kTX = 32 * kM;                  // quads per tile row
    static constexpr int kRing = kRing_;                 // plane slots
    static constexpr uint32_t kEsz = St::kBytes;
    static constexpr uint32_t kQB = 4 * kEsz;            // bytes per quad
    static constexpr uint32_t kCS = kEsz == 4 ? 16 : 4;  // bytes one lane copies per load (whole quads only)
    static constexpr uint32_t kRB = (kTX + 2) * kQB;     // LDS row: left quad, kTX quads, right quad
    static constexpr uint32_t kRowChunks = kRB / kCS;
    static constexpr uint32_t kQuadChunks = kQB / kCS;
    static constexpr uint32_t kSlot = (kTY + 2) * kRB;   // rows y0-1 .. y0+kTY
    static constexpr uint32_t kChunks = kSlot / kCS;
    static constexpr int kNI = (int)((kChunks + 63) / 64);  // load instructions per plane
    static constexpr int kCompute = kTX * kTY;           // compute threads
    static constexpr int kThreads = kCompute + 64;
    static_assert(kTY % 4 == 0, "rows are permuted in groups of two waves");
    static_assert(kSlot % 16 == 0 && kRB % 16 == 0, "LDS rows must keep 16-byte alignment");
    static_assert(kRing >= 5 && kRing <= 7, "ring of 5..7 planes");
    static_assert(kM >= 1 && kM <= 4, "tile width 32 .. 128 quads");
    static_assert(kRing * kSlot <= 65536, "static LDS of one workgroup");
    static_assert((kRing - 4) * kNI < 64, "vmcnt (6 bits) must count the planes left in flight");

    // compute thread t -> (tile row, quad column): wave w takes 32-quad strip
    // w % m of the row pair w / m; pair g holds rows 4(g/2) + g%2 and the row
    // two below it (same parity), lanes 0..31 the first, 32..63 the second
    static __device__ __forceinline__ void place(uint32_t t, uint32_t& row, uint32_t& col) {
        const uint32_t w = t >> 6, lane = t & 63u;
        const uint32_t g = w / kM, strip = w % kM;
        row = 4u * (g >> 1) + (g & 1u) + 2u * (lane >> 5);
        col = 32u * strip + (lane & 31u);
    }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Direct buffer-to-LDS loads: each lane's `bytes` go to dst + lane * bytes.
// Non-template wrappers: the 16-byte form exists on gfx950 only, and a
// template kernel that names it directly is dropped by the host pass.
__device__ __forceinline__ void lds_load_b128(__amdgpu_buffer_rsrc_t r, lds_ptr_t dst, uint32_t voff,
                                              uint32_t soff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, soff, 0, 0);
}
__device__ __forceinline__ void lds_load_b32(__amdgpu_buffer_rsrc_t r, lds_ptr_t dst, uint32_t voff,
                                             uint32_t soff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 4, voff, soff, 0, 0);
}

// s_waitcnt immediates (gfx9 encoding): vmcnt in bits 3:0 and 15:14, expcnt
// 6:4, lgkmcnt 11:8; a field at its maximum does not wait.
template <int kVm>
__device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(kVm >= 0 && kVm < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((kVm & 15) | (7 << 4) | (0 << 8) | ((kVm >> 4) << 14));
}

// Workgroup barrier for the producer: its LDS writes were waited for above,
// and the asm statements keep the compiler from moving memory operations
// across the barrier.
__device__ __forceinline__ void producer_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// kNT: non-temporal stores of the updated colour.
template <class St, int kM, int kTY, int kRing, bool kNT>
__global__ __launch_bounds__((Stream<St, kM, kTY, kRing>::kThreads)) void halfsweep_stream(
    const typename St::T* __restrict__ other, typename St::T* __restrict__ own, uint32_t lh, uint32_t ly,
    uint32_t lz, uint32_t zc, uint32_t c, uint32_t h, uint32_t k0, uint32_t k1, uint32_t chain,
    uint32_t xcd_order, const uint32_t* __restrict__ tdev) {
    using S = Stream<St, kM, kTY, kRing>;
    using T = typename St::T;
    __shared__ __align__(16) unsigned char ring[S::kRing * S::kSlot];
    if (tdev) h += 2u * tdev[0];

    const uint32_t nq = lh >> 2;
    const uint32_t nbx = (nq + S::kTX - 1) / S::kTX, nby = (ly + kTY - 1) / kTY;
    uint32_t b = blockIdx.x;
    if (xcd_order) {
        const uint32_t per = gridDim.x / 8u;
        if (b < 8u * per) b = (b % 8u) * per + b / 8u;
    }
    const uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const uint32_t q0 = bx * S::kTX, y0 = by * kTY, z0 = bz * zc;
    const uint32_t z1 = min(z0 + zc, lz);
    const uint32_t n = z1 - z0;  // planes this workgroup updates (>= 1)
    const uint32_t plane = ly * lh, plane_b = plane * S::kEsz;

    for (uint32_t i = threadIdx.x; i < S::kRing * S::kSlot / 16; i += S::kThreads)
        reinterpret_cast<uint4*>(ring)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();

    if (threadIdx.x >= (uint32_t)S::kCompute) {
        // ---------------- producer wave ----------------
        const uint32_t lane = threadIdx.x - S::kCompute;
        const __amdgpu_buffer_rsrc_t src = make_rsrc(other, plane_b * lz);
        // byte offset within a plane of the chunk each lane copies per load
        // instruction (the same for every plane), kNoLoad if outside the box
        uint32_t off[S::kNI];
        bool every = true;  // every instruction has a lane to load (block-uniform)
#pragma unroll
        for (int i = 0; i < S::kNI; ++i) {
            const uint32_t ch = 64u * (uint32_t)i + lane;
            const uint32_t r = ch / S::kRowChunks, k = ch % S::kRowChunks;
            const int quad = (int)q0 - 1 + (int)(k / S::kQuadChunks);
            const int yr = (int)y0 - 1 + (int)r;
            const bool ok = ch < S::kChunks && quad >= 0 && quad < (int)nq && yr >= 0 && yr < (int)ly;
            off[i] = ok ? ((uint32_t)yr * lh + 4u * (uint32_t)quad) * S::kEsz + (k % S::kQuadChunks) * S::kCS
                        : kNoLoad;
            every = every && __builtin_amdgcn_ballot_w64(ok) != 0;
        }
        // whether plane l = z0-1+l is loaded (the ghost planes z0-1 = -1 and
        // lz are not; planes past z1 are not needed)
        auto loads = [&](uint32_t l) -> bool { return l <= n + 1u && !(l == 0 && z0 == 0) && z0 + l - 1u < lz; };
        // plane l into slot l % kRing
        auto produce = [&](uint32_t l) {
            unsigned char* dst = ring + (l % S::kRing) * S::kSlot;
            if (l > n + 1u || (l == 0 && z0 == 0)) return;  // not needed, or slot 0 still zero
            const uint32_t zp = z0 + l - 1u;
            if (zp >= lz) {  // the ghost plane past the box: only its kTY rows are read
                for (uint32_t i = lane; i < kTY * S::kRB / 16; i += 64)
                    reinterpret_cast<uint4*>(dst + S::kRB)[i] = make_uint4(0u, 0u, 0u, 0u);
                return;
            }
            const uint32_t soff = zp * plane_b;
#pragma unroll
            for (int i = 0; i < S::kNI; ++i)
                if (off[i] != kNoLoad) {
                    const lds_ptr_t d = (lds_ptr_t)(dst + 64u * S::kCS * i);
                    if constexpr (S::kCS == 16)
                        lds_load_b128(src, d, off[i], soff);
                    else
                        lds_load_b32(src, d, off[i], soff);
                }
        };
        // wait until only the loads of planes lo .. hi may be in flight (and
        // every LDS store of this wave is done); exact only if every plane
        // issues kNI loads, else wait for all
        auto wait_landed = [&](uint32_t lo, uint32_t hi) {
            uint32_t k = 0;
            for (uint32_t l = lo; l <= hi; ++l) k += loads(l) ? 1u : 0u;
            if (!every) k = 0;
            switch (k) {
                case 0: wait_vm_lgkm0<0>(); break;
                case 1: wait_vm_lgkm0<S::kNI>(); break;
                case 2: wait_vm_lgkm0<(S::kRing >= 6 ? 2 : 0) * S::kNI>(); break;
                default: wait_vm_lgkm0<(S::kRing >= 7 ? 3 : 0) * S::kNI>(); break;
            }
        };
        for (uint32_t l = 0; l + 1u < (uint32_t)S::kRing; ++l) produce(l);  // planes l = 0 .. R-2
        wait_landed(3u, S::kRing - 2u);
        producer_barrier();  // b_0
        for (uint32_t s = 0; s + 1u < n; ++s) {
            produce(s + S::kRing - 1u);
            wait_landed(s + 4u, s + S::kRing - 1u);
            producer_barrier();  // b_{s+1}
        }
    } else {
        // ---------------- compute waves ----------------
        uint32_t row, tx;
        S::place(threadIdx.x, row, tx);
        const uint32_t q = q0 + tx, y = y0 + row;
        const bool active = q < nq && y < ly;
        const uint32_t rowj = y * lh + 4u * q;
        const uint32_t qoff = (row + 1u) * S::kRB + (tx + 1u) * S::kQB;  // the thread's quad in a slot
        for (uint32_t s = 0; s < n; ++s) {
            __syncthreads();  // b_s
            if (!active) continue;
            const uint32_t z = z0 + s;
            const unsigned char* pm = ring + (s % S::kRing) * S::kSlot + qoff;
            const unsigned char* pc = ring + ((s + 1u) % S::kRing) * S::kSlot + qoff;
            const unsigned char* pn = ring + ((s + 2u) % S::kRing) * S::kSlot + qoff;
            const float4 bm = St::ld4(reinterpret_cast<const T*>(pm), 0);
            const float4 bc = St::ld4(reinterpret_cast<const T*>(pc), 0);
            const float4 bn = St::ld4(reinterpret_cast<const T*>(pn), 0);
            const float4 up = St::ld4(reinterpret_cast<const T*>(pc - S::kRB), 0);
            const float4 dn = St::ld4(reinterpret_cast<const T*>(pc + S::kRB), 0);
            const uint32_t p = __builtin_amdgcn_readfirstlane((c + y + z) & 1u);  // uniform per wave
            const float e = p == 0 ? St::ld(reinterpret_cast<const T*>(pc - S::kEsz), 0)
                                   : St::ld(reinterpret_cast<const T*>(pc + S::kQB), 0);
            const uint32_t j0 = z * plane + rowj;
            const float4 out = heatbath_quad(bm, bc, bn, up, dn, e, p, j0, h, chain, k0, k1);
            if constexpr (kNT)
                St::st4_nt(own, j0, out);
            else
                St::st4(own, j0, out);
        }
    }
}

// Tile 0: 8 rows (4 compute waves + producer, 27 KB LDS at FP32); tile 1:
// 16 rows (8 + 1 waves, 49 KB).  Requires lh % 4 == 0 and the other colour's
// array below 2 GiB (32-bit byte offsets).
template <class St, int kM, int kTY, int kRing, bool kNT>
static void launch_stream_cfg(const SweepArgs& a, const typename St::T* other, typename St::T* own,
                              uint32_t zc, hipStream_t stream) {
    using S = Stream<St, kM, kTY, kRing>;
    const uint32_t nq = a.lh >> 2;
    const uint32_t nb = ((nq + S::kTX - 1) / S::kTX) * ((a.ly + kTY - 1) / kTY) * ((a.lz + zc - 1) / zc);
    hipLaunchKernelGGL((halfsweep_stream<St, kM, kTY, kRing, kNT>), dim3(nb), dim3(S::kThreads), 0, stream, other,
                       own, a.lh, a.ly, a.lz, zc, a.c, a.h, a.k0, a.k1, a.chain, a.xcd_order, a.tdev);
}

// Tile configurations: tile width 32m quads, rows, ring slots, non-temporal
// stores.  LDS per workgroup at FP32 = slots * (rows + 2) * (32m + 2) * 16 bytes.
template <class St>
static hipError_t launch_stream_t(const SweepArgs& a, const typename St::T* other, typename St::T* own,
                                  hipStream_t stream) {
    const uint32_t zc = a.zc ? a.zc : 16u;
    switch (a.tile) {
        case 0: launch_stream_cfg<St, 1, 8, 6, true>(a, other, own, zc, stream); break;    // 33 KB
        case 1: launch_stream_cfg<St, 1, 8, 5, false>(a, other, own, zc, stream); break;   // 27 KB
        case 2: launch_stream_cfg<St, 1, 16, 5, false>(a, other, own, zc, stream); break;  // 49 KB
        case 3: launch_stream_cfg<St, 1, 8, 6, false>(a, other, own, zc, stream); break;   // 33 KB
        case 4: launch_stream_cfg<St, 2, 4, 5, false>(a, other, own, zc, stream); break;   // 32 KB
        case 5: launch_stream_cfg<St, 2, 8, 5, false>(a, other, own, zc, stream); break;   // 53 KB
        case 6: launch_stream_cfg<St, 3, 4, 5, false>(a, other, own, zc, stream); break;   // 47 KB
        case 7: launch_stream_cfg<St, 3, 4, 6, false>(a, other, own, zc, stream); break;   // 56 KB
        case 8: launch_stream_cfg<St, 4, 4, 5, false>(a, other, own, zc, stream); break;   // 62 KB
        case 9: launch_stream_cfg<St, 3, 4, 5, true>(a, other, own, zc, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_halfsweep_stream(const SweepArgs& a, hipStream_t stream) {
    if (a.lh % 4 != 0) return hipErrorInvalidValue;
    const uint32_t esz = a.storage == 0 ? 4u : 2u;
    if ((uint64_t)a.vh * esz >= (1ull << 31)) return hipErrorInvalidValue;
    switch (a.storage) {
        case 0: {
            float* f = static_cast<float*>(a.field);
            return launch_stream_t<StoreF32>(a, f + (size_t)(a.c ^ 1u) * a.vh, f + (size_t)a.c * a.vh, stream);
        }
        case 1: {
            uint16_t* f = static_cast<uint16_t*>(a.field);
            return launch_stream_t<StoreBF16>(a, f + (size_t)(a.c ^ 1u) * a.vh, f + (size_t)a.c * a.vh, stream);
        }
        case 2: {
            _Float16* f = static_cast<_Float16*>(a.field);
            return launch_stream_t<StoreF16>(a, f + (size_t)(a.c ^ 1u) * a.vh, f + (size_t)a.c * a.vh, stream);
        }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
