// Both half-sweeps of a sweep in one pass over memory (temporal blocking of
// the red-black heat bath, Eq. phi).
//
// The heat bath never reads a site's own old value, so colour 0 of sweep t
// is a function of colour 1 of sweep t - 1 alone, and colour 1 of sweep t a
// function of that colour 0.  One launch therefore reads colour 1 once and
// writes it once (4 B per site update at FP32, 2 B at 16-bit), keeping
// colour 0 in LDS; colour 0 is stored only when asked for (the last sweep of
// a call, samples that read it from memory).  Colour 1 is read from one
// array and written to another (a workgroup's halo rows and planes are other
// workgroups' interiors).
//
// A workgroup owns a tile of kty full rows (y0 .. y0+kty-1) and walks the
// planes z0 .. z1-1 of a slab.  Colour 0 is computed on kty + 2 rows (one
// halo row each side, recomputed by both neighbouring tiles with the same
// Philox draws) and on the planes z0-1 .. z1; colour 1 on the owned rows and
// planes.  Rows are whole, so there is no x halo: a row of LDS holds the
// row's quads between 16 bytes of zeros (the Dirichlet ghosts beyond x = 0
// and x = lx - 1).
//
// LDS (dynamic): a ring of kRing slots of old colour-1 planes (kty + 4 rows:
// y0-2 .. y0+kty+1), fed by a producer wave with direct buffer-to-LDS loads,
// and a ring of 3 slots of new colour-0 planes (kty + 2 rows).  Walk index
// l holds old plane o(l) = z0 - 2 + l in slot l % kRing; colour-0 walk index
// i holds plane z0 - 1 + i in slot i % 3.  Step s (s = 0 .. n+2, n = z1-z0;
// one workgroup barrier between steps):
//   * colour 0 of plane a = z0-1+s (s <= n+1) from old planes l = s+1 (the
//     window of x-neighbours and rows y-1, y+1) and l = s+2 (z+1); its z-1
//     neighbour (l = s) is the z+1 quad the same thread read two steps
//     earlier (registers), read from LDS only in step 0 for steps 0 and 1;
//     written to colour-0 slot s % 3 (a ghost plane a < 0 or a >= lz writes
//     zeros);
//   * colour 1 of plane b = z0-3+s (3 <= s <= n+2) from colour-0 planes
//     b (window, rows y-1, y+1) and b+1 (z+1); its z-1 neighbour is again the
//     quad read two steps earlier (colour-0 planes z0-1 and z0 are read into
//     those registers in steps 1 and 2); stored to memory;
//   * the producer requests old planes kRing, kRing+1 in step 1 and s+kRing
//     in step s >= 2 (into the slot of plane s, whose last LDS read was in
//     step s-1), then waits until plane s+3 has landed.
// Every LDS access of this protocol was checked against what each slot holds
// on a CPU model of the kernel before its first run.
//
// The work of a step is a list of wave-tasks of 64 quads: colour-0 tasks
// over (kty+2) x nq quads, then colour-1 tasks over kty x nq quads, row-major;
// compute wave w takes tasks w, w + kBlkCW, ... (with the hardware dealing a
// workgroup's waves over the 4 SIMDs in turn, task t runs on SIMD t % 4, so
// the SIMDs share a step's work evenly).  A lane's quad and its
// x-pairing p = (c + y + z) & 1 vary within a wave; p only moves the start of
// the 5-value window of x-neighbours, so every lane runs the same code.
// Sums are formed in the order of the other kernels (x-neighbours, y-1, y+1,
// z-1, z+1), so fields are bit for bit theirs.

#include "device_common.hpp"
#include "kernels.hpp"
#include "lds_pipe.hpp"

#include <mutex>
#include <type_traits>

namespace latcoul {

constexpr int kBlkCW = 12;                       // compute waves (three per SIMD)
constexpr int kBlkThreads = 64 * (kBlkCW + 1);   // and one producer wave
// load instructions the producer issues per plane: the plane's chunks, then
// loads past the array (no fetch) into a sink, so that the count is fixed and
// every wait has a compile-time count (at most two planes in flight: 48 < 64)
constexpr int kBlkNI = 24;
constexpr int kBlkTasks = 3;                     // wave-tasks per compute wave per step, at most
constexpr uint32_t kBlkGhost = 16;               // zero bytes at each end of an LDS row
// dynamic LDS of one workgroup: the CU's 160 KiB less 2 KiB for the
// kernel's static arrays (the padding loads' sink, list offsets, the
// finalize's wave sums)
constexpr uint32_t kBlkLdsMax = 160u * 1024u - 2048u;
// fused gather: a list's staged part is the keys (4 B), Q and S (8 B each)
// of its entries from the 16-byte boundaries below the part's start, each
// array in whole 16-byte chunks: g_cap entries plus 64 bytes per array
constexpr uint32_t kBlkStagePad = 3u * 64u;
__host__ __device__ constexpr uint32_t blk_stage_bytes(uint32_t cap) { return kGatherEntryBytes * cap + kBlkStagePad; }

// A quad of 4 same-colour values as loaded from LDS: FP32 values, or the raw
// halves of the 16-bit formats.
template <class St>
struct BlkTraits {
    using Q = typename St::Raw;
    static constexpr uint32_t kEsz = St::kBytes;
};

template <class St>
__device__ __forceinline__ typename BlkTraits<St>::Q blk_quad(const unsigned char* p) {
    return *reinterpret_cast<const typename BlkTraits<St>::Q*>(p);
}

// Loads from an LDS ring of one colour: a quad (FP32 and BF16 as FP32
// values, FP16 as raw halves for the mixed-precision adds of
// heatbath_quad_f16) and the single value beyond a quad.
template <class St>
__device__ __forceinline__ auto blk_ld4(const unsigned char* p) {
    if constexpr (kF16Grid<St>)
        return *reinterpret_cast<const u32x2*>(p);
    else
        return St::ld4(reinterpret_cast<const typename St::T*>(p), 0);
}
template <class St>
__device__ __forceinline__ auto blk_ld1(const unsigned char* p) {
    if constexpr (kF16Grid<St>)
        return (uint32_t) * reinterpret_cast<const uint16_t*>(p);
    else
        return St::ld(reinterpret_cast<const typename St::T*>(p), 0);
}

// The neighbours of the quad at byte offset qoff of ring slot `ring` (its
// own colour's other-colour neighbours: rows y-1, y+1 and the x-neighbour
// beyond the quad on the side p selects), z-1 and z+1 given.
template <class St>
__device__ __forceinline__ QuadNeighbours<St> blk_neighbours(const unsigned char* ring, uint32_t qoff, uint32_t rb,
                                                             uint32_t p, decltype(QuadNeighbours<St>::zm) zm,
                                                             decltype(QuadNeighbours<St>::zm) zp) {
    constexpr uint32_t kEsz = St::kBytes;
    QuadNeighbours<St> nb;
    nb.cen = blk_ld4<St>(ring + qoff);
    nb.ym = blk_ld4<St>(ring + qoff - rb);
    nb.yp = blk_ld4<St>(ring + qoff + rb);
    nb.zm = zm;
    nb.zp = zp;
    nb.e = blk_ld1<St>(ring + (p ? qoff + 4u * kEsz : qoff - kEsz));
    return nb;
}

// The stored form of an updated quad (rounded to the storage format with
// its Philox words) and its stores to LDS and memory.
template <class St>
__device__ __forceinline__ typename BlkTraits<St>::Q blk_round(const QuadOut& o) {
    return St::pack4(o.v, o.w);
}
template <class St, bool kNT>
__device__ __forceinline__ void blk_store(typename St::T* base, uint32_t j0, typename BlkTraits<St>::Q v) {
    using Q = typename BlkTraits<St>::Q;
    Q* p = &at<Q>(base, j0);
    if constexpr (kNT) {
        if constexpr (std::is_same<St, StoreF32>::value) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store(f4{v.x, v.y, v.z, v.w}, reinterpret_cast<f4*>(p));
        } else {
            __builtin_nontemporal_store(v, p);
        }
    } else {
        *p = v;
    }
}

template <class St, int kRing, int kTasks, bool kNT, bool kGather>
__global__ __launch_bounds__(kBlkThreads) void sweep_blocked(BlockedArgs a) {
    using T = typename St::T;
    using Q = typename BlkTraits<St>::Q;
    constexpr uint32_t kEsz = BlkTraits<St>::kEsz;
    constexpr uint32_t kQB = 4 * kEsz;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ __align__(16) uint32_t list_off[2 * (kBlockedMaxParts + 1)];  // fused gather: the tile's part bounds
    __shared__ __align__(16) unsigned char sink[1024];  // target of the producer's padding loads

    const uint32_t lh = a.lh, ly = a.ly, lz = a.lz, kty = a.kty, zc = a.zc;
    const uint32_t nq = lh >> 2;
    const uint32_t rb = 2u * kBlkGhost + nq * kQB;  // LDS row
    const uint32_t oslot = (kty + 4u) * rb, cslot = (kty + 2u) * rb;
    unsigned char* const oring = lds;
    unsigned char* const cring = lds + kRing * oslot;
    unsigned char* const stage = cring + 3u * cslot;  // fused gather: the two staged lists
    const uint32_t nby = (ly + kty - 1u) / kty;
    // workgroup order over the 8 XCDs (the hardware deals workgroups round
    // robin): 0 as dealt; 1 each XCD a contiguous run of tiles; 2 each XCD a
    // band of the tiles of one slab, all XCDs moving through the slabs
    // together (neighbouring tiles share halo rows in their XCD's L2)
    uint32_t b = blockIdx.x;
    if (a.xcd_order == 1u) {
        const uint32_t per = gridDim.x / 8u;
        if (b < 8u * per) b = (b % 8u) * per + b / 8u;
    } else if (a.xcd_order == 2u) {
        const uint32_t w = b % nby, per = nby / 8u;
        if (w < 8u * per) b = b - w + (w % 8u) * per + w / 8u;
    }
    const uint32_t by = b % nby, bz = b / nby;
    const uint32_t y0 = by * kty, z0 = bz * zc;
    const uint32_t z1 = min(z0 + zc, lz);
    const uint32_t n = z1 - z0;
    const uint32_t nsteps = n + 3u;
    const uint32_t plane = ly * lh;
    uint32_t h0 = a.h0;
    if (a.tdev) h0 += 2u * a.tdev[0];

    // zeros: the rows' ghost bytes, rows outside the box, both rings
    const uint32_t total16 = (kRing * oslot + 3u * cslot) / 16u;
    for (uint32_t i = threadIdx.x; i < total16; i += kBlkThreads)
        reinterpret_cast<uint4*>(lds)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();

    if (threadIdx.x >= 64u * kBlkCW) {
        // ---------------- producer wave ----------------
        const uint32_t lane = threadIdx.x & 63u;
        // the compute waves keep their SIMDs busy: without a raised priority
        // the producer's loads, waits and gather walks are issued late and
        // every step's barrier waits for them
        __builtin_amdgcn_s_setprio(2);
        const uint32_t plane_b = plane * kEsz;
        const __amdgpu_buffer_rsrc_t src = make_rsrc(a.c1_in, plane_b * lz);
        // fused gather: the tile's two list ranges (colour 0, colour 1) into
        // LDS ahead of the first planes, read after b_0
        const bool gather = kGather && a.g_key != nullptr && (a.part0 || a.part1);
        const uint32_t tiles = gridDim.x, tile = by + nby * bz;
        const uint32_t np1 = a.g_parts + 1u;  // part bounds per list
        if (gather && lane < 2u * np1)  // bounds of colour c: g_off[(c tiles + tile) np1 + p]
            lds_load_b32(make_rsrc(a.g_off, 4u * 2u * tiles * np1), (lds_ptr_t)list_off,
                         4u * ((lane / np1) * tiles * np1 + lane % np1), 4u * tile * np1);
        // 16-byte chunks of a slot: chunk k of row r holds bytes 16k .. 16k+15
        // of that row; the first and last chunks are the ghosts.  Lanes whose
        // chunk is a ghost or lies in a row outside the box load from an
        // offset past the array (the buffer returns zeros and fetches
        // nothing): every plane issues the same ni instructions.
        const uint32_t rbc = rb / 16u, chunks = oslot / 16u;
        const uint32_t ni = (chunks + 63u) / 64u;  // <= kBlkNI (checked on the host)
        uint32_t off[kBlkNI];
#pragma unroll
        for (int i = 0; i < kBlkNI; ++i) {
            const uint32_t ch = 64u * (uint32_t)i + lane;
            const uint32_t r = ch / rbc, k = ch - r * rbc;
            const int yr = (int)y0 - 2 + (int)r;
            const bool in = k >= 1u && k + 1u < rbc && yr >= 0 && yr < (int)ly;
            off[i] = ch >= chunks ? kNoLoad : in ? ((uint32_t)yr * lh) * kEsz + (k - 1u) * 16u : kNoLoad;
        }
        const bool last_in = 64u * (ni - 1u) + lane < chunks;  // this lane's chunk of the last instruction
        auto loads = [&](uint32_t l) -> bool {
            const int o = (int)z0 - 2 + (int)l;
            return l <= n + 3u && o >= 0 && o < (int)lz;
        };
        // old plane l into slot l % kRing: loads, or zeros for a ghost plane
        auto produce = [&](uint32_t l) {
            if (l > n + 3u) return;
            unsigned char* dst = oring + (l % kRing) * oslot;
            const int o = (int)z0 - 2 + (int)l;
            if (o < 0 || o >= (int)lz) {
                for (uint32_t i = lane; i < oslot / 16u; i += 64u)
                    reinterpret_cast<uint4*>(dst)[i] = make_uint4(0u, 0u, 0u, 0u);
                return;
            }
            const uint32_t soff = (uint32_t)o * plane_b;
            // every lane of instructions 0 .. ni-2 has a chunk of the slot;
            // only the last instruction's lanes past the slot are masked off
            // (one lane mask for the whole plane).  The tests of i against
            // ni are made afresh in each call (an opaque copy of ni): held
            // across the step loop they took 48 scalar registers, spilled
            uint32_t nl = ni;
            asm volatile("" : "+s"(nl));
#pragma unroll
            for (int i = 0; i < kBlkNI; ++i) {
                if ((uint32_t)i + 1u < nl) {
                    lds_load_b128(src, (lds_ptr_t)(dst + 1024u * (uint32_t)i), off[i], soff);
                } else if ((uint32_t)i + 1u == nl) {
                    if (last_in) lds_load_b128(src, (lds_ptr_t)(dst + 1024u * (uint32_t)i), off[i], soff);
                } else {
                    lds_load_b128(src, (lds_ptr_t)sink, kNoLoad, 0u);  // padding: zeros into the sink
                }
            }
        };
        // wait until every plane up to lmax has landed, planes lmax+1 ..
        // lhi (requested) left in flight: kBlkNI loads each
        auto wait_landed = [&](uint32_t lmax, uint32_t lhi) {
            uint32_t k = 0;
            for (uint32_t l = lmax + 1u; l <= lhi; ++l) k += loads(l) ? 1u : 0u;
            if (k == 0u)
                wait_vm_lgkm0<0>();
            else if (k == 1u)
                wait_vm_lgkm0<kBlkNI>();
            else
                wait_vm_lgkm0<2 * kBlkNI>();
        };
        for (uint32_t l = 0; l < (uint32_t)kRing; ++l) produce(l);
        if (kGather && a.fin.part && blockIdx.x == 0) finalize_in_workgroup<kBlkThreads, 64 * kBlkCW>(a.fin);
        wait_landed(2u, kRing - 1u);  // (the list offsets, requested first, have landed)
        producer_barrier();  // b_0
        // fused gather: each list (key, Q, S per entry) is staged into LDS in
        // parts of g_stride steps (part p: the entries of steps 1 + p stride
        // .. p stride + stride): part 0 after b_0, waited for in step 1; part
        // p in step p stride, once that step's walks are done with part p - 1,
        // waited for before the step's barrier.  Entry i of a list (counted
        // from the tile's list start) belongs to lane i % 64, which adds its
        // entries in order of i; a cursor walks each list step by step
        // (entries of a step are consecutive, the hits of a window a prefix of
        // it).  Bounds and cursors are kept in vector registers.
        uint32_t first[2] = {0u, 0u}, kbase[2] = {0u, 0u}, qbase[2] = {0u, 0u}, pend[2] = {0u, 0u}, cur[2];
        asm volatile("v_mov_b32 %0, 0\n\tv_mov_b32 %1, 0" : "=v"(cur[0]), "=v"(cur[1]));
        // per colour and charge set (the entry's set in bits 26-27 of its key)
        double gx[2][kBlockedMaxSets], gy[2][kBlockedMaxSets];
#pragma unroll
        for (uint32_t c = 0; c < 2u; ++c)
#pragma unroll
            for (uint32_t k = 0; k < kBlockedMaxSets; ++k) gx[c][k] = gy[c][k] = 0.0;
        const uint32_t a_stage = lds_addr(stage), sbytes = blk_stage_bytes(a.g_cap);
        const uint32_t kbytes = 4u * a.g_cap + 64u, qbytes = 8u * a.g_cap + 64u;  // per array
        auto stage_part = [&](uint32_t p) {
            const __amdgpu_buffer_rsrc_t rk = make_rsrc(a.g_key, 4u * a.g_n);
            const __amdgpu_buffer_rsrc_t rq = make_rsrc(a.g_Q, 8u * a.g_n);
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.g_S, 8u * a.g_n);
            for (uint32_t c = 0; c < 2u; ++c) {
                const uint32_t ps = lds_read_u32(lds_addr(list_off) + 4u * (c * np1 + p));
                pend[c] = lds_read_u32(lds_addr(list_off) + 4u * (c * np1 + p + 1u));
                kbase[c] = ps & ~3u;  // 16-byte boundaries: 4 keys, 2 doubles
                qbase[c] = ps & ~1u;
                unsigned char* st = stage + c * sbytes;
                const uint32_t kb = 4u * (pend[c] - kbase[c]), qb = 8u * (pend[c] - qbase[c]);  // < kbytes, qbytes
                for (uint32_t i = 0; 1024u * i < kb; ++i)  // 1 KiB per instruction
                    if (1024u * i + 16u * lane < kb)
                        lds_load_b128(rk, (lds_ptr_t)(st + 1024u * i), 1024u * i + 16u * lane, 4u * kbase[c]);
                for (uint32_t i = 0; 1024u * i < qb; ++i)
                    if (1024u * i + 16u * lane < qb) {
                        lds_load_b128(rq, (lds_ptr_t)(st + kbytes + 1024u * i), 1024u * i + 16u * lane,
                                      8u * qbase[c]);
                        lds_load_b128(rs, (lds_ptr_t)(st + kbytes + qbytes + 1024u * i), 1024u * i + 16u * lane,
                                      8u * qbase[c]);
                    }
            }
        };
        if (gather) {
            for (uint32_t c = 0; c < 2u; ++c) {
                first[c] = lds_read_u32(lds_addr(list_off) + 4u * c * np1);
                cur[c] += first[c];
            }
            stage_part(0u);
        }
        // the entries of list c gathered in step s, from ring slot `slot`
        // (the colour a compile-time constant: the accumulators stay in
        // registers, where a run-time index would put them in scratch)
        auto walk = [&](auto colour, uint32_t s, const unsigned char* slot) __attribute__((always_inline)) {
            constexpr uint32_t c = decltype(colour)::value;
            const uint32_t ak = a_stage + c * sbytes;
            const uint32_t aq = ak + kbytes, as = aq + qbytes;
            const uint32_t aslot = lds_addr(slot);
            for (;;) {
                const uint32_t rc = cur[c] - first[c];
                const uint32_t e = first[c] + rc + ((lane - rc) & 63u);  // this lane's entry of the window
                const uint32_t key = e < pend[c] ? lds_read_u32(ak + 4u * (e - kbase[c])) : 0xFFFFFFFFu;
                const bool hit = ((key >> 16) & kBlockedStepMask) == s;
                const uint32_t nhit = (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(hit));
                if (hit) {
                    float v;
                    double Qi, Si;
                    const uint32_t k = 8u * (e - qbase[c]);
                    lds_read_entry<St>(aslot + (key & 0xFFFFu), aq + k, as + k, v, Qi, Si);
                    const double d = (double)v;
                    if (a.g_sets == 1u) {
                        gx[c][0] = fma(Qi, d, gx[c][0]);
                        gy[c][0] = fma(Si, d * d, gy[c][0]);
                    } else {
                        // every set's pair takes the entry, with weights zero
                        // but for its own set (adding an exact zero): no index
                        // by the set, so the pairs stay in registers
                        const uint32_t set = key >> 26;
#pragma unroll
                        for (uint32_t k = 0; k < kBlockedMaxSets; ++k) {
                            const bool mine = set == k;
                            gx[c][k] = fma(mine ? Qi : 0.0, d, gx[c][k]);
                            gy[c][k] = fma(mine ? Si : 0.0, d * d, gy[c][k]);
                        }
                    }
                }
                cur[c] += nhit;
                if (nhit < 64u) break;
            }
        };
        uint32_t lhi = kRing - 1u;  // last plane requested
        for (uint32_t s = 0; s < nsteps; ++s) {
            bool restaged = false;
            if (gather && s >= 1u && s <= n + 1u) {
                // colour 1 of the previous sweep, plane z0-1+s (old walk index
                // s+1, landed, refilled only in step s+1); colour 0 of this
                // sweep, plane z0-2+s (colour-0 walk index s-1, written in
                // step s-1).  In step 1, before any new plane load, part 0
                // and every plane requested so far have landed.
                if (s == 1u) wait_vm_lgkm0<0>();
                if (a.part1) walk(std::integral_constant<uint32_t, 1u>(), s, oring + ((s + 1u) % kRing) * oslot);
                if (a.part0 && s >= 2u) walk(std::integral_constant<uint32_t, 0u>(), s, cring + ((s - 1u) % 3u) * cslot);
                if (s % a.g_stride == 0u && s <= n) {  // the walks' LDS reads have completed
                    stage_part(s / a.g_stride);
                    restaged = true;
                }
            }
            if (s == 1u) {
                produce(kRing);
                produce(kRing + 1u);
                lhi = kRing + 1u;
            } else if (s >= 2u) {
                produce(s + kRing);
                lhi = s + kRing;
            }
            if (s + 1u < nsteps) {
                // a part staged in this step lands before b_{s+1}: only this
                // step's planes, requested after it, stay in flight
                wait_landed(restaged ? (s == 1u ? kRing - 1u : s + kRing - 1u) : s + 3u, lhi);
                producer_barrier();  // b_{s+1}
            }
        }
        if (gather) {
#pragma unroll
            for (uint32_t c = 0; c < 2u; ++c) {
                double* part = c == 0u ? a.part0 : a.part1;
                if (!part) continue;
#pragma unroll
                for (uint32_t k = 0; k < kBlockedMaxSets; ++k) {
                    if (k >= a.g_sets) break;
                    const double x = wave_sum(gx[c][k]), y = wave_sum(gy[c][k]);
                    if (lane == 0) {
                        part[(size_t)k * a.g_set_stride + 2u * tile] = x;
                        part[(size_t)k * a.g_set_stride + 2u * tile + 1u] = y;
                    }
                }
            }
        }
    } else {
        // ---------------- compute waves ----------------
        // Tasks: colour-0 rows r = 0 .. kty+1 (y = y0-1+r), then colour-1 rows
        // r = 0 .. kty-1 (y = y0+r); within each, the rows of even r then those
        // of odd r, 64 quads per task, so that all lanes of a task have rows of
        // one parity and the x-pairing p is uniform over the wave.
        const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63u;
        auto group_tasks = [&](uint32_t rows, uint32_t g) { return (((rows + 1u - g) / 2u) * nq + 63u) / 64u; };
        const uint32_t ta0 = group_tasks(kty + 2u, 0u), t0 = ta0 + group_tasks(kty + 2u, 1u);
        const uint32_t ta1 = group_tasks(kty, 0u), t1 = ta1 + group_tasks(kty, 1u);
        using NbT = decltype(QuadNeighbours<St>::zm);
        // task i runs (bit i) and is a colour-0 task (bit 8 + i): wave-uniform,
        // one scalar register.  A lane with no quad in the box computes on
        // row 1 of the ring like the others (no branch around the update)
        // and drops its result: a colour-0 lane writes it to its own 16 bytes
        // of the sink, a colour-1 lane does not store it.
        uint32_t kinds = 0;
        uint32_t qoff[kTasks], woff[kTasks], rowoff[kTasks], py[kTasks], own0[kTasks], valid[kTasks];
#pragma unroll
        for (int i = 0; i < kTasks; ++i) {
            const uint32_t t = w + (uint32_t)(kBlkCW * i);
            const bool run = t < t0 + t1, c0 = t < t0;
            kinds |= (run ? 1u << i : 0u) | (c0 ? 1u << (8 + i) : 0u);
            const uint32_t tt = c0 ? t : t - t0;
            const uint32_t ta = c0 ? ta0 : ta1;
            const uint32_t g = tt < ta ? 0u : 1u;
            const uint32_t rows = c0 ? kty + 2u : kty;
            const uint32_t iq = (tt - g * ta) * 64u + lane;
            const uint32_t i2 = iq / nq, q = iq - i2 * nq;
            const uint32_t r = 2u * i2 + g;
            const int y = c0 ? (int)y0 - 1 + (int)r : (int)(y0 + r);
            const bool ok = run && r < rows && y >= 0 && y < (int)ly;
            const uint32_t yy = ok ? (uint32_t)y : 0u;
            valid[i] = ok ? 1u : 0u;
            qoff[i] = ok ? (r + 1u) * rb + kBlkGhost + q * kQB : rb + kBlkGhost;  // row r+1 of the ring holds y
            woff[i] = r * rb + kBlkGhost + q * kQB;  // colour-0 tasks: row r of the colour-0 ring
            rowoff[i] = yy * lh + 4u * q;
            // (c + y) & 1 from the group alone, uniform even where y is outside
            // the box: colour 0 with y = y0-1+r, colour 1 with y = y0+r, r = g mod 2
            py[i] = (y0 + g + 1u) & 1u;
            own0[i] = ok && c0 && r >= 1u && r <= kty ? 1u : 0u;  // an owned colour-0 row
        }
        kinds = __builtin_amdgcn_readfirstlane(kinds);
        unsigned char* const sinkp = sink + 16u * lane;  // a dropped colour-0 result
        NbT hist[kTasks][2];
        if (kGather && a.fin.part && blockIdx.x == 0) finalize_in_workgroup<kBlkThreads, 64 * kBlkCW>(a.fin);
        // Step s: colour 0 of plane z0-1+s (s <= n+1), colour 1 of plane
        // z0-3+s (3 <= s <= n+2), the history registers read in steps 0 (the
        // old planes z0-2, z0-1) and 1, 2 (colour 0 of planes z0-1, z0).
        // kSteady: 3 <= s <= n, where every task updates a plane inside the
        // box and none of those checks is needed.
        auto step = [&](uint32_t s, auto parity, auto steady) __attribute__((always_inline)) {
            constexpr uint32_t P = decltype(parity)::value;
            constexpr bool kSteady = decltype(steady)::value;
#pragma unroll
            for (int i = 0; i < kTasks; ++i) {
                if (!(kinds & (1u << i))) continue;
                if (kinds & (1u << (8 + i))) {
                    if (!kSteady && s > n + 1u) continue;
                    const unsigned char* lin = oring + ((s + 1u) % kRing) * oslot;
                    const unsigned char* lzp = oring + ((s + 2u) % kRing) * oslot;
                    if (!kSteady && s == 0u) {
                        hist[i][0] = blk_ld4<St>(oring + qoff[i]);
                        hist[i][1] = blk_ld4<St>(oring + oslot + qoff[i]);
                    }
                    const NbT zm = hist[i][P];
                    const NbT zp = blk_ld4<St>(lzp + qoff[i]);
                    hist[i][P] = zp;
                    unsigned char* wr = valid[i] ? cring + (s % 3u) * cslot + woff[i] : sinkp;
                    const int az = (int)z0 - 1 + (int)s;
                    if (!kSteady && (az < 0 || az >= (int)lz)) {
                        *reinterpret_cast<Q*>(wr) = blk_round<St>(QuadOut{make_float4(0.f, 0.f, 0.f, 0.f), uint4{}});
                        continue;
                    }
                    const uint32_t az_u = (uint32_t)az;
                    const uint32_t j0 = az_u * plane + rowoff[i];
                    const uint32_t pp = __builtin_amdgcn_readfirstlane(py[i] ^ (az_u & 1u));
                    const Q v = blk_round<St>(
                        quad_update_from<St>(blk_neighbours<St>(lin, qoff[i], rb, pp, zm, zp), pp, j0, h0, a.chain,
                                             a.k0, a.k1));
                    *reinterpret_cast<Q*>(wr) = v;
                    if (a.c0_out && own0[i] && az_u >= z0 && az_u < z1)
                        blk_store<St, false>(static_cast<T*>(a.c0_out), j0, v);
                } else {
                    if (!kSteady) {
                        if (s == 0u || s > n + 2u) continue;
                        if (s == 1u) {  // colour-0 walk index 0 (plane z0-1): z-1 of step 3
                            hist[i][1] = blk_ld4<St>(cring + qoff[i]);
                            continue;
                        }
                        if (s == 2u) {  // walk index 1 (plane z0): z-1 of step 4
                            hist[i][0] = blk_ld4<St>(cring + cslot + qoff[i]);
                            continue;
                        }
                    }
                    const uint32_t bi = s - 2u;  // colour-0 walk index of plane b
                    const unsigned char* cin = cring + (bi % 3u) * cslot;
                    const unsigned char* czp = cring + ((bi + 1u) % 3u) * cslot;
                    const NbT zm = hist[i][P];
                    const NbT zp = blk_ld4<St>(czp + qoff[i]);
                    hist[i][P] = zp;
                    const uint32_t bz_ = z0 + s - 3u;
                    const uint32_t j0 = bz_ * plane + rowoff[i];
                    const uint32_t pp = __builtin_amdgcn_readfirstlane(py[i] ^ (bz_ & 1u));
                    const Q v = blk_round<St>(quad_update_from<St>(blk_neighbours<St>(cin, qoff[i], rb, pp, zm, zp),
                                                                   pp, j0, h0 + 1u, a.chain, a.k0, a.k1));
                    if (valid[i]) blk_store<St, kNT>(static_cast<T*>(a.c1_out), j0, v);
                }
            }
        };
        using P0 = std::integral_constant<uint32_t, 0u>;
        using P1 = std::integral_constant<uint32_t, 1u>;
        using Edge = std::false_type;
        using Steady = std::true_type;
        auto edge_step = [&](uint32_t s) __attribute__((always_inline)) {
            if (s & 1u)
                step(s, P1(), Edge());
            else
                step(s, P0(), Edge());
        };
        __syncthreads();  // b_0
        uint32_t s = 0;
        for (; s < 3u; ++s) {  // nsteps >= 4
            edge_step(s);
            __syncthreads();  // b_{s+1}
        }
        for (; s + 1u <= n; s += 2u) {  // s odd
            step(s, P1(), Steady());
            __syncthreads();
            step(s + 1u, P0(), Steady());
            __syncthreads();
        }
        for (; s < nsteps; ++s) {
            edge_step(s);
            if (s + 1u < nsteps) __syncthreads();  // b_{s+1}
        }
    }
}

// Geometry of a launch: LDS bytes, load instructions per plane and
// wave-tasks per compute wave for kty rows per tile; false if the tile does
// not fit (LDS, loads or tasks).
bool blocked_geometry(uint32_t lh, uint32_t esz, uint32_t kty, uint32_t ring, BlockedShape* out, uint32_t g_cap) {
    if (lh % 4u != 0 || kty == 0 || (esz != 4 && esz != 2) || ring < 4 || ring > 5) return false;
    const uint32_t nq = lh / 4u;
    if ((nq * 4u * esz) % 16u != 0) return false;  // rows of whole 16-byte chunks
    const uint64_t rb = 2u * kBlkGhost + (uint64_t)nq * 4u * esz;
    const uint64_t oslot = (kty + 4u) * rb, cslot = (kty + 2u) * rb;
    const uint64_t lds = ring * oslot + 3u * cslot + (g_cap ? 2u * (uint64_t)blk_stage_bytes(g_cap) : 0u);
    const uint64_t ni = (oslot / 16u + 63u) / 64u;
    // tasks: the rows of each colour split by parity, 64 quads per task
    auto group = [&](uint64_t rows) { return ((rows + 1u) / 2u * nq + 63u) / 64u + (rows / 2u * nq + 63u) / 64u; };
    const uint64_t tasks = group(kty + 2u) + group(kty);
    const uint64_t per_wave = (tasks + kBlkCW - 1u) / kBlkCW;
    if (lds > kBlkLdsMax || ni > (uint64_t)kBlkNI || per_wave > (uint64_t)kBlkTasks) return false;
    out->lds = (uint32_t)lds;
    out->tasks_total = (uint32_t)tasks;
    out->tasks_per_wave = (uint32_t)per_wave;
    out->loads_per_plane = (uint32_t)ni;
    return true;
}

template <class St, int kRing, int kTasks, bool kNT, bool kGather>
static hipError_t set_lds_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&sweep_blocked<St, kRing, kTasks, kNT, kGather>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBlkLdsMax);
}

template <class St, bool kGather>
static hipError_t set_lds_attrs_g() {
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = set_lds_attr<St, 4, kBlkTasks, false, kGather>();
    if (e == hipSuccess) e = set_lds_attr<St, 4, kBlkTasks, true, kGather>();
    if (e == hipSuccess) e = set_lds_attr<St, 5, kBlkTasks, false, kGather>();
    if (e == hipSuccess) e = set_lds_attr<St, 5, kBlkTasks, true, kGather>();
    return e;
}
template <class St>
static hipError_t set_lds_attrs_t() {
    hipError_t e = set_lds_attrs_g<St, false>();
    if (e == hipSuccess) e = set_lds_attrs_g<St, true>();
    return e;
}

// Allow every instantiation the LDS of a whole CU (dynamic shared memory),
// once per process.
hipError_t prepare_blocked_sweep() {
    static std::once_flag once;
    static hipError_t result = hipSuccess;
    std::call_once(once, [] {
        result = set_lds_attrs_t<StoreF32>();
        if (result == hipSuccess) result = set_lds_attrs_t<StoreBF16>();
        if (result == hipSuccess) result = set_lds_attrs_t<StoreF16>();
        if (result == hipSuccess) result = set_lds_attrs_t<StoreBF16SR>();
        if (result == hipSuccess) result = set_lds_attrs_t<StoreF16SR>();
    });
    return result;
}

template <class St, int kRing, int kTasks>
static void launch_blocked_cfg(const BlockedArgs& a, uint32_t blocks, uint32_t lds, bool nt, hipStream_t stream) {
    // the sample gather and the finalize in their own instantiation: sweeps
    // without them keep the leaner register allocation
    const bool g = a.g_key != nullptr || a.fin.part != nullptr;
    if (nt && g)
        hipLaunchKernelGGL((sweep_blocked<St, kRing, kTasks, true, true>), dim3(blocks), dim3(kBlkThreads), lds,
                           stream, a);
    else if (nt)
        hipLaunchKernelGGL((sweep_blocked<St, kRing, kTasks, true, false>), dim3(blocks), dim3(kBlkThreads), lds,
                           stream, a);
    else if (g)
        hipLaunchKernelGGL((sweep_blocked<St, kRing, kTasks, false, true>), dim3(blocks), dim3(kBlkThreads), lds,
                           stream, a);
    else
        hipLaunchKernelGGL((sweep_blocked<St, kRing, kTasks, false, false>), dim3(blocks), dim3(kBlkThreads), lds,
                           stream, a);
}

template <class St>
static void launch_blocked_t(const BlockedArgs& a, const BlockedShape& sh, uint32_t blocks, hipStream_t stream) {  // sh.tasks_per_wave <= kBlkTasks
    const bool nt = a.nt != 0;
    if (a.ring == 4)
        launch_blocked_cfg<St, 4, kBlkTasks>(a, blocks, sh.lds, nt, stream);
    else
        launch_blocked_cfg<St, 5, kBlkTasks>(a, blocks, sh.lds, nt, stream);
}

hipError_t launch_blocked_sweep(const BlockedArgs& a, hipStream_t stream) {
    const uint32_t esz = a.storage == 0 ? 4u : 2u;
    BlockedShape sh;
    if (!a.c1_in || !a.c1_out || a.c1_in == a.c1_out || a.zc == 0 || a.ly == 0 || a.lz == 0 ||
        !blocked_geometry(a.lh, esz, a.kty, a.ring, &sh, a.g_key ? a.g_cap : 0u))
        return hipErrorInvalidValue;
    if (a.g_key && (!a.g_off || !a.g_Q || !a.g_S || a.g_cap == 0 || a.g_cap % 64u != 0 ||
                    (uint64_t)a.g_n * 8u >= (1ull << 32) || (a.zc + 2u) > kBlockedStepMask || a.g_parts == 0 ||
                    a.g_parts > kBlockedMaxParts || a.g_stride == 0 || (uint64_t)a.g_parts * a.g_stride < a.zc + 1u))
        return hipErrorInvalidValue;
    if ((a.part0 || a.part1) && !a.g_key) return hipErrorInvalidValue;
    if (a.g_key && (a.g_sets < 1 || a.g_sets > kBlockedMaxSets || (a.g_sets > 1 && a.g_set_stride == 0) ||
                    (a.g_sets > 1 && a.fin.part)))
        return hipErrorInvalidValue;
    if (a.fin.part && (!a.fin.bins || !a.fin.last_xy || a.fin.n == 0 || a.fin.bin_size == 0))
        return hipErrorInvalidValue;
    // 32-bit byte offsets: each colour array below 2 GiB
    if ((uint64_t)a.lh * a.ly * a.lz * esz >= (1ull << 31)) return hipErrorInvalidValue;
    if (hipError_t e = prepare_blocked_sweep()) return e;
    const uint64_t blocks = (uint64_t)((a.ly + a.kty - 1) / a.kty) * ((a.lz + a.zc - 1) / a.zc);
    if (blocks == 0 || blocks >= (1ull << 31)) return hipErrorInvalidValue;
    switch (a.storage) {
        case 0: launch_blocked_t<StoreF32>(a, sh, (uint32_t)blocks, stream); break;
        case 1: launch_blocked_t<StoreBF16>(a, sh, (uint32_t)blocks, stream); break;
        case 2: launch_blocked_t<StoreF16>(a, sh, (uint32_t)blocks, stream); break;
        case 3: launch_blocked_t<StoreBF16SR>(a, sh, (uint32_t)blocks, stream); break;
        case 4: launch_blocked_t<StoreF16SR>(a, sh, (uint32_t)blocks, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace latcoul
