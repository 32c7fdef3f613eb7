// Streaming slab half-sweep: a producer wave feeds an LDS ring of planes
// with direct buffer-to-LDS loads, the compute waves update from LDS.
//
// A workgroup owns a tile of 32m quads (128m same-colour sites, m = 1..4),
// or of one 16-quad strip, x kTY rows and walks `zc` planes along z, as the
// z-slab kernel does; what differs is who loads.  The workgroup is
// (tile width) kTY / 64 compute waves plus one producer wave; a compute wave
// holds a 32-quad strip of two rows of the same parity (or a 16-quad strip
// of four), so the x-pairing of the update is uniform per wave.  A tile
// as wide as the box's rows makes every plane of the tile one contiguous run
// of memory.  The producer copies each plane of the other colour that the
// tile needs (its kTY rows, the halo rows y0-1 and y0+kTY, and the quads
// left and right of the tile) with `buffer_load ... lds`, which writes LDS
// without passing through registers, into a ring of R plane slots
// (R = 5..7), R-3 planes ahead of the plane being updated.  Its only memory operations are these
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
//
// Fused sample gather (g_key set): X = sum Q phi and Y = sum S phi^2 of a
// sample split by colour.  The sites of the colour that a launch does not
// update are final in the ring: the colour-1 half-sweep of a measured sweep
// gathers the charged colour-0 sites, the colour-0 half-sweep of the next
// sweep the charged colour-1 sites (whose values of the measured sweep it
// holds in its ring), so no value is read from memory twice or recomputed.
// The producer wave, idle between its loads, takes its tile's list plane by
// plane and writes one (X, Y) partial per tile.  The list (packed key, Q, S)
// is staged into dynamic LDS by the same direct loads, issued in step 0
// right after the first planes'; step 1 waits for it and moves the keys to
// registers.  Plane s is gathered in step s + 1, after that step's loads
// are requested; it touches only LDS, so it never waits on the plane loads
// in flight.  The colour-1 part of a run's last sample, with no next sweep,
// comes from gather_tail, whose lanes add the same entries in the same
// order from the field in memory: every partial is the same whichever
// kernel wrote it.  A sample completed by a colour-0 launch is finalized by
// workgroup 0 of the colour-1 launch that follows (fin set), while its first
// planes load; partials are kept in two buffers by sample parity, so that
// launch may open the next sample.

#include "device_common.hpp"
#include "kernels.hpp"
#include "lds_pipe.hpp"

#include <type_traits>

namespace latcoul {

template <class St, int kM, int kTY, int kRing_, int kQW = 32>
struct Stream {
    static constexpr int kTX = kQW * kM;                 // quads per tile row
    static constexpr int kRowsPerWave = 64 / kQW;        // rows of one parity a wave holds
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
    static_assert(kQW == 32 || kQW == 16, "strips of 32 or 16 quads");
    static_assert(kTY % (2 * kRowsPerWave) == 0, "rows are permuted in groups of two waves");
    static_assert(kSlot % 16 == 0 && kRB % 16 == 0, "LDS rows must keep 16-byte alignment");
    static_assert(kRing >= 5 && kRing <= 7, "ring of 5..7 planes");
    static_assert(kM >= 1 && kM <= 4, "tile width 1 .. 4 strips");
    static_assert(kRing * kSlot <= 65536, "static LDS of one workgroup");
    static_assert((kRing - 4) * kNI < 64, "vmcnt (6 bits) must count the planes left in flight");

    // compute thread t -> (tile row, quad column): wave w takes strip w % m
    // (kQW quads) of row group g = w / m, k = 64 / kQW rows of one parity:
    // rows 2k(g/2) + g%2, and the k - 1 rows two, four, .. below it, lanes
    // 0..kQW-1 the first (32-quad strips: two rows; 16-quad strips: four)
    static __device__ __forceinline__ void place(uint32_t t, uint32_t& row, uint32_t& col) {
        const uint32_t w = t >> 6, lane = t & 63u;
        const uint32_t g = w / kM, strip = w % kM;
        row = 2u * kRowsPerWave * (g >> 1) + (g & 1u) + 2u * (lane / kQW);
        col = kQW * strip + (lane % kQW);
    }
};

// Fused-gather list entries.  Staged key of entry i of a tile's list: the
// site's plane within the tile's slab (bits 16..31) and its byte offset in
// a ring slot (bits 0..15); entries are sorted by plane, and entry i always
// belongs to lane i % 64, which adds Q_i phi and S_i phi^2 in order of i.
// kGatherRegs keys per lane are held in registers (lists of up to 256).
constexpr int kGatherRegs = 4;
constexpr uint32_t kNoEntry = 0xFFFFFFFFu;  // plane field never matches

// kNT: non-temporal stores of the updated colour.
template <class St, int kM, int kTY, int kRing, bool kNT, int kQW = 32>
__global__ __launch_bounds__((Stream<St, kM, kTY, kRing, kQW>::kThreads)) void halfsweep_stream(
    const typename St::T* __restrict__ other, typename St::T* __restrict__ own, uint32_t lh, uint32_t ly,
    uint32_t lz, uint32_t zc, uint32_t c, uint32_t h, uint32_t k0, uint32_t k1, uint32_t chain,
    uint32_t xcd_order, const uint32_t* __restrict__ tdev, const uint32_t* __restrict__ g_off,
    const uint32_t* __restrict__ g_key, const double* __restrict__ g_Q, const double* __restrict__ g_S,
    double* __restrict__ g_part, uint32_t g_n, uint32_t g_cap, SampleFinalize fin, uint32_t zalt) {
    using S = Stream<St, kM, kTY, kRing, kQW>;
    using T = typename St::T;
    __shared__ __align__(16) unsigned char ring[S::kRing * S::kSlot];
    // fused gather: the tile's list offsets, then its keys, Q and S (g_cap
    // entries each)
    __shared__ __align__(16) uint32_t list_off[4];
    extern __shared__ __align__(16) unsigned char stage[];
    if (tdev) h += 2u * tdev[0];

    const uint32_t nq = lh >> 2;
    const uint32_t nbx = (nq + S::kTX - 1) / S::kTX, nby = (ly + kTY - 1) / kTY;
    // workgroup order over the 8 XCDs (the hardware deals blocks round-robin):
    // 0 as dealt; 1 each XCD a contiguous run of tiles; 2 each XCD a band of
    // the tiles of one slab, all XCDs moving through the slabs together
    uint32_t b = blockIdx.x;
    if (xcd_order == 1u) {
        const uint32_t per = gridDim.x / 8u;
        if (b < 8u * per) b = (b % 8u) * per + b / 8u;
    } else if (xcd_order == 2u) {
        const uint32_t t = nbx * nby, w = b % t, per = t / 8u;
        if (w < 8u * per) b = b - w + (w % 8u) * per + w / 8u;
    }
    const uint32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const uint32_t q0 = bx * S::kTX, y0 = by * kTY, z0 = bz * zc;
    const uint32_t z1 = min(z0 + zc, lz);
    const uint32_t n = z1 - z0;  // planes this workgroup updates (>= 1)
    // walk direction: odd slabs walk down (zalt), so that the two slabs on
    // either side of a slab boundary read the planes there at the same end of
    // their walks, close in time (one of the two reads then finds them in L2).
    // Walk index l (plane l in slot l % R) -> plane z0 - 1 + l going up,
    // z1 - l going down; step s updates the plane of walk index s + 1.
    const bool down = zalt && (bz & 1u);
    auto plane_of = [&](uint32_t l) -> int { return down ? (int)z1 - (int)l : (int)z0 - 1 + (int)l; };
    const uint32_t plane = ly * lh, plane_b = plane * S::kEsz;
    const uint32_t tile = bx + nbx * (by + nby * bz);
    const bool finalize = fin.part != nullptr && blockIdx.x == 0;  // the previous sample, in the first workgroup

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
        // whether walk plane l is loaded (the ghost planes -1 and lz are not;
        // planes past the slab's halo are not needed)
        auto loads = [&](uint32_t l) -> bool {
            const int zp = plane_of(l);
            return l <= n + 1u && zp >= 0 && zp < (int)lz;
        };
        // walk plane l into slot l % kRing
        auto produce = [&](uint32_t l) {
            unsigned char* dst = ring + (l % S::kRing) * S::kSlot;
            if (l > n + 1u) return;  // not needed
            const int zp = plane_of(l);
            if (zp < 0 || zp >= (int)lz) {  // a ghost plane beyond the box
                if (l == 0) return;         // slot 0 is still zero
                for (uint32_t i = lane; i < kTY * S::kRB / 16; i += 64)  // only its kTY rows are read
                    reinterpret_cast<uint4*>(dst + S::kRB)[i] = make_uint4(0u, 0u, 0u, 0u);
                return;
            }
            const uint32_t soff = (uint32_t)zp * plane_b;
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
            switch (k) {  // (a count beyond vmcnt's 6 bits waits for all)
                case 0: wait_vm_lgkm0<0>(); break;
                case 1: wait_vm_lgkm0<S::kNI>(); break;
                case 2: wait_vm_lgkm0<(2 * S::kNI < 64 ? 2 * S::kNI : 0)>(); break;
                case 3: wait_vm_lgkm0<(3 * S::kNI < 64 ? 3 * S::kNI : 0)>(); break;
                default: wait_vm_lgkm0<0>(); break;
            }
        };
        // fused gather: this tile's charged sites of the other colour, sorted
        // by plane.  The tile's two list offsets are loaded to LDS ahead of
        // the first planes and read after barrier b_0 (their latency hidden
        // by the plane loads).
        const bool gather = g_key != nullptr;
        uint32_t gbase = 0, ng = 0;
        uint32_t key[kGatherRegs];
        double gx = 0.0, gy = 0.0;
        const uint32_t a_key = lds_addr(stage), a_Q = a_key + 4u * g_cap, a_S = a_key + 12u * g_cap;
        const uint32_t a_ring = lds_addr(ring);
        auto stage_list = [&]() {
            const __amdgpu_buffer_rsrc_t rk = make_rsrc(g_key, 4u * g_n);
            const __amdgpu_buffer_rsrc_t rq = make_rsrc(g_Q, 8u * g_n);
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(g_S, 8u * g_n);
            for (uint32_t i = 0; 64u * i < ng; ++i)  // 64 keys per instruction
                if (64u * i + lane < ng)
                    lds_load_b32(rk, (lds_ptr_t)(stage + 256u * i), 4u * (64u * i + lane), 4u * gbase);
            for (uint32_t i = 0; 32u * i < ng; ++i)  // 32 doubles per instruction
                if (64u * i + lane < 2u * ng) {
                    lds_load_b32(rq, (lds_ptr_t)(stage + 4u * g_cap + 256u * i), 4u * (64u * i + lane), 8u * gbase);
                    lds_load_b32(rs, (lds_ptr_t)(stage + 12u * g_cap + 256u * i), 4u * (64u * i + lane),
                                 8u * gbase);
                }
        };
        auto load_keys = [&]() {
#pragma unroll
            for (int k = 0; k < kGatherRegs; ++k) {
                const uint32_t i = lane + 64u * (uint32_t)k;
                key[k] = i < ng ? lds_read_u32(a_key + 4u * i) : kNoEntry;
            }
        };
        // the plane of step s (walk plane s + 1, in ring slot s + 1): gathered
        // in step s + 1 (or after the last step), before step s + 2 refills
        // the slot; a key's plane field is that step s
        auto gather_plane = [&](uint32_t s) {
            const uint32_t slot = a_ring + ((s + 1u) % S::kRing) * S::kSlot;
#pragma unroll
            for (int k = 0; k < kGatherRegs; ++k) {
                const bool hit = (key[k] >> 16) == s;
                if (__builtin_amdgcn_ballot_w64(hit) == 0) continue;  // wave-uniform
                if (hit) {
                    const uint32_t i = lane + 64u * (uint32_t)k;
                    float v;
                    double Qi, Si;
                    lds_read_entry<St>(slot + (key[k] & 0xFFFFu), a_Q + 8u * i, a_S + 8u * i, v, Qi, Si);
                    const double d = (double)v;
                    gx = fma(Qi, d, gx);
                    gy = fma(Si, d * d, gy);
                }
            }
        };
        if (gather && lane < 2u)  // g_off[tile], g_off[tile + 1] into list_off
            lds_load_b32(make_rsrc(g_off, 4u * (gridDim.x + 1u)), (lds_ptr_t)list_off, 4u * lane, 4u * tile);
        for (uint32_t l = 0; l + 1u < (uint32_t)S::kRing; ++l) produce(l);  // planes l = 0 .. R-2
        if (finalize) finalize_in_workgroup<S::kThreads, S::kCompute>(fin);
        wait_landed(3u, S::kRing - 2u);  // (the offsets, loaded first, have landed)
        producer_barrier();  // b_0
        if (gather) {
            gbase = lds_read_u32(lds_addr(list_off));
            ng = lds_read_u32(lds_addr(list_off) + 4u) - gbase;  // <= g_cap
            stage_list();
        }
        for (uint32_t s = 0; s < n; ++s) {
            if (s + 1u < n) produce(s + S::kRing - 1u);
            if (gather && s >= 1u) {
                if (s == 1u) {  // the list, staged before plane R - 1
                    wait_landed(S::kRing - 1u, S::kRing);
                    load_keys();
                }
                gather_plane(s - 1u);
            }
            if (s + 1u < n) {
                wait_landed(s + 4u, s + S::kRing - 1u);
                producer_barrier();  // b_{s+1}
            }
        }
        if (gather) {
            if (n == 1u) {
                wait_vm_lgkm0<0>();
                load_keys();
            }
            gather_plane(n - 1u);
            gx = wave_sum(gx);
            gy = wave_sum(gy);
            if (lane == 0) {
                g_part[2 * tile] = gx;
                g_part[2 * tile + 1] = gy;
            }
        }
    } else {
        // ---------------- compute waves ----------------
        uint32_t row, tx;
        S::place(threadIdx.x, row, tx);
        const uint32_t q = q0 + tx, y = y0 + row;
        const bool active = q < nq && y < ly;
        const uint32_t rowj = y * lh + 4u * q;
        const uint32_t qoff = (row + 1u) * S::kRB + (tx + 1u) * S::kQB;  // the thread's quad in a slot
        if (finalize) finalize_in_workgroup<S::kThreads, S::kCompute>(fin);
        // The thread's quad of walk planes s and s + 1 is kept from the two
        // steps before (as FP32, or as raw halves for FP16, whose update adds
        // them in mixed-precision FMAs): a step reads (and widens) only the
        // quad of walk plane s + 2 besides plane z's rows y -+ 1 and its
        // x-neighbour.  Steps are unrolled by three, so that the three quads
        // rotate through registers without copies.
        using Q = typename QuadNeighbours<St>::Quad;
        auto ldq = [&](const unsigned char* pq) __attribute__((always_inline)) -> Q {
            if constexpr (kF16Grid<St>)
                return *reinterpret_cast<const u32x2*>(pq);
            else
                return St::ld4(reinterpret_cast<const T*>(pq), 0);
        };
        auto walk = [&](auto down_c) __attribute__((always_inline)) {
            constexpr bool kDown = decltype(down_c)::value;
            auto step = [&](uint32_t s, Q& wa, Q& wb, Q& wc, bool first) __attribute__((always_inline)) {
                __syncthreads();  // b_s
                if (!active) return;
                const uint32_t z = kDown ? z1 - 1u - s : z0 + s;
                const unsigned char* pc = ring + ((s + 1u) % S::kRing) * S::kSlot + qoff;
                if (first) {
                    wa = ldq(ring + (s % S::kRing) * S::kSlot + qoff);
                    wb = ldq(pc);
                }
                wc = ldq(ring + ((s + 2u) % S::kRing) * S::kSlot + qoff);
                const Q up = ldq(pc - S::kRB), dn = ldq(pc + S::kRB);
                const uint32_t p = __builtin_amdgcn_readfirstlane((c + y + z) & 1u);  // uniform per wave
                const unsigned char* pe = p == 0 ? pc - S::kEsz : pc + S::kQB;  // the x-neighbour beyond the quad
                const uint32_t j0 = z * plane + rowj;
                // walk planes s, s + 1, s + 2: planes z -+ 1, z, z +- 1
                QuadOut out;
                if constexpr (kF16Grid<St>) {
                    const uint32_t e = *reinterpret_cast<const uint16_t*>(pe);
                    out = kDown ? heatbath_quad_f16(wc, wb, wa, up, dn, e, p, j0, h, chain, k0, k1)
                                : heatbath_quad_f16(wa, wb, wc, up, dn, e, p, j0, h, chain, k0, k1);
                } else {
                    const float e = St::ld(reinterpret_cast<const T*>(pe), 0);
                    out = kDown ? heatbath_quad(wc, wb, wa, up, dn, e, p, j0, h, chain, k0, k1)
                                : heatbath_quad(wa, wb, wc, up, dn, e, p, j0, h, chain, k0, k1);
                }
                if constexpr (kNT)
                    St::st4_nt(own, j0, out.v, out.w);
                else
                    St::st4(own, j0, out.v, out.w);
            };
            Q qa = {}, qb = {}, qc = {};
            step(0u, qa, qb, qc, true);
            for (uint32_t s = 1; s < n; s += 3) {
                step(s, qb, qc, qa, false);
                if (s + 1u >= n) break;
                step(s + 1u, qc, qa, qb, false);
                if (s + 2u >= n) break;
                step(s + 2u, qa, qb, qc, false);
            }
        };
        if (down)
            walk(std::true_type());
        else
            walk(std::false_type());
    }
}

// One configuration: grid of tiles x slabs, dynamic LDS for a staged gather
// list.  Requires lh % 4 == 0 and the other colour's array below 2 GiB
// (32-bit byte offsets).
template <class St, int kM, int kTY, int kRing, bool kNT, int kQW = 32>
static void launch_stream_cfg(const SweepArgs& a, const typename St::T* other, typename St::T* own,
                              uint32_t zc, hipStream_t stream) {
    using S = Stream<St, kM, kTY, kRing, kQW>;
    const uint32_t nq = a.lh >> 2;
    const uint32_t nb = ((nq + S::kTX - 1) / S::kTX) * ((a.ly + kTY - 1) / kTY) * ((a.lz + zc - 1) / zc);
    const uint32_t dyn = a.g_key ? kGatherEntryBytes * a.g_cap : 0u;
    hipLaunchKernelGGL((halfsweep_stream<St, kM, kTY, kRing, kNT, kQW>), dim3(nb), dim3(S::kThreads), dyn, stream, other,
                       own, a.lh, a.ly, a.lz, zc, a.c, a.h, a.k0, a.k1, a.chain, a.xcd_order, a.tdev, a.g_off,
                       a.g_key, a.g_Q, a.g_S, a.g_part, a.g_n, a.g_cap, a.fin, kStreamAltZ ? 1u : 0u);
}

// Tile configurations: tile width 32m quads (tile 10: one 16-quad strip),
// rows, ring slots, non-temporal stores.  LDS per workgroup at FP32 =
// slots * (rows + 2) * (width + 2) * 16 bytes.
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
        case 10: launch_stream_cfg<St, 1, 16, 6, false, 16>(a, other, own, zc, stream); break;  // 31 KB
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Shape of each configuration: the layout of the per-tile charge lists of
// the fused gather and the LDS budget of their staging.
bool stream_tile_geometry(uint32_t tile, uint32_t esz, StreamTileShape* out) {
    static const uint32_t kShape[kStreamTiles][3] = {{32, 8, 6},  {32, 8, 5}, {32, 16, 5}, {32, 8, 6}, {64, 4, 5},
                                                     {64, 8, 5},  {96, 4, 5}, {96, 4, 6},  {128, 4, 5}, {96, 4, 5}, {16, 16, 6}};
    if (tile >= (uint32_t)kStreamTiles || (esz != 4 && esz != 2)) return false;
    const uint32_t q = kShape[tile][0], rows = kShape[tile][1], slots = kShape[tile][2];
    out->quads = q;
    out->rows = rows;
    out->waves = q * rows / 64u + 1u;
    // the plane ring, the list offsets (16 B, 16-byte aligned), the workgroup
    // sum of the in-kernel finalize (two doubles per wave): the compiler's
    // static LDS size of each instantiation
    out->lds = slots * (rows + 2u) * (q + 2u) * 4u * esz + 32u + 16u * out->waves;
    return true;
}

hipError_t launch_halfsweep_stream(const SweepArgs& a, hipStream_t stream) {
    if (a.lh % 4 != 0) return hipErrorInvalidValue;
    if (a.g_key && (!a.g_off || !a.g_Q || !a.g_S || !a.g_part || a.g_cap % 64u != 0 || a.g_cap > 64u * kGatherRegs ||
                    (uint64_t)a.g_n * 8u >= (1ull << 32)))
        return hipErrorInvalidValue;
    if (a.fin.part && (!a.fin.bins || !a.fin.last_xy || a.fin.n == 0 || a.fin.bin_size == 0))
        return hipErrorInvalidValue;
    if (a.g_key) {
        StreamTileShape sh;
        if (!stream_tile_geometry(a.tile, a.storage == 0 ? 4u : 2u, &sh) ||
            sh.lds + (uint64_t)kGatherEntryBytes * a.g_cap > 65536u)
            return hipErrorInvalidValue;
    }
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
        case 3: {
            uint16_t* f = static_cast<uint16_t*>(a.field);
            return launch_stream_t<StoreBF16SR>(a, f + (size_t)(a.c ^ 1u) * a.vh, f + (size_t)a.c * a.vh, stream);
        }
        case 4: {
            _Float16* f = static_cast<_Float16*>(a.field);
            return launch_stream_t<StoreF16SR>(a, f + (size_t)(a.c ^ 1u) * a.vh, f + (size_t)a.c * a.vh, stream);
        }
        default: return hipErrorInvalidValue;
    }
}

// The colour-1 part of a sample from the field in memory (a run's last
// sample): one wave per tile; lane i % 64 adds entry i of the tile's list in
// order of i, as in the streaming kernel, so the partial per tile is the
// same.
template <class St>
__global__ __launch_bounds__(64) void gather_tail(const typename St::T* __restrict__ f,
                                                 const uint32_t* __restrict__ g_off, const uint32_t* __restrict__ g_j,
                                                 const double* __restrict__ g_Q, const double* __restrict__ g_S,
                                                 double* __restrict__ g_part) {
    const uint32_t tile = blockIdx.x, lane = threadIdx.x;
    const uint32_t gbase = g_off[tile], ng = g_off[tile + 1] - gbase;
    double gx = 0.0, gy = 0.0;
    for (uint32_t i = lane; i < ng; i += 64u) {
        const double d = (double)St::ld(f, g_j[gbase + i]);
        gx = fma(g_Q[gbase + i], d, gx);
        gy = fma(g_S[gbase + i], d * d, gy);
    }
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    if (lane == 0) {
        g_part[2 * tile] = gx;
        g_part[2 * tile + 1] = gy;
    }
}

hipError_t launch_gather_tail(const GatherTailArgs& a, hipStream_t stream) {
    if (!a.field1 || !a.g_off || !a.g_j || !a.g_Q || !a.g_S || !a.g_part || a.tiles == 0) return hipErrorInvalidValue;
    switch (storage_grid(a.storage)) {
        case 0:
            hipLaunchKernelGGL(gather_tail<StoreF32>, dim3(a.tiles), dim3(64), 0, stream,
                               static_cast<const float*>(a.field1), a.g_off, a.g_j, a.g_Q, a.g_S, a.g_part);
            break;
        case 1:
            hipLaunchKernelGGL(gather_tail<StoreBF16>, dim3(a.tiles), dim3(64), 0, stream,
                               static_cast<const uint16_t*>(a.field1), a.g_off, a.g_j, a.g_Q, a.g_S, a.g_part);
            break;
        case 2:
            hipLaunchKernelGGL(gather_tail<StoreF16>, dim3(a.tiles), dim3(64), 0, stream,
                               static_cast<const _Float16*>(a.field1), a.g_off, a.g_j, a.g_Q, a.g_S, a.g_part);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace latcoul
