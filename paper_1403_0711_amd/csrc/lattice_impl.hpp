// Internal state of a lattice handle and the functions the runtime's
// source files share: lattice_api.hip (the C ABI, sweep scheduling, graphs,
// bins), fused_gather.hip (the streaming kernel's sample lists) and
// autotune.hip.  Not part of the C ABI.

#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "lattice_coulomb.h"
#include "runtime_common.hpp"

using namespace latcoul;

// largest box that AUTO runs with the one-workgroup resident kernel
constexpr uint64_t kResidentMaxSites = 16384;
constexpr int64_t kMaxChargeSets = 65535;  // charge sets per lattice (a grid dimension of the gather)
constexpr uint32_t kTileDefault = 0xFFFFFFFFu;  // lattice_set_tuning(tile = -1): library default
constexpr uint32_t kStreamTileFullRow96 = 9;        // streaming kernel: 96-quad tiles, non-temporal stores
constexpr uint32_t kStreamTileFullRow96Cached = 6;  // 96-quad tiles, ordinary stores
constexpr uint32_t kStreamTileCached = 3;           // 32 quads x 8 rows, 6-slot ring, ordinary stores

// Planes per workgroup the slab kernels default to: 16 at FP32, where the
// sweep is bound by memory traffic and short slabs balance the chip best; 32
// at 16-bit storage, where arithmetic binds and longer slabs amortise each
// workgroup's start-up.
inline uint32_t default_slab(size_t esz) { return esz == 4 ? 16u : 32u; }
constexpr uint64_t kZslabAutoMinSites = (uint64_t)1 << 23;  // 8.4e6 sites: between 192^3 and 208^3
constexpr uint32_t kZslabTileAuto = 7;

struct lattice {
    int64_t lx = 0, ly = 0, lz = 0;
    uint32_t lh = 0, vh = 0;
    int storage = 0;
    size_t esz = 4;
    uint64_t seed = 0;
    uint32_t chain = 0;
    DeviceAllocator mem;
    int device = 0;  // the device current at creation (the field's)
    uint32_t cus = 256;  // its compute units
    hipStream_t stream = nullptr;
    void* field = nullptr;  // colour 0 then colour 1
    // second colour-1 array for the fused sweep, which reads colour 1 from one
    // array and writes the other; alt_current: the current colour 1 is there
    void* c1alt = nullptr;
    bool alt_current = false;
    // the second colour-1 array was allocated at creation for the library's
    // choice of the blocked sweep (FP32 boxes beyond the last-level cache)
    bool auto_blocked = false;
    // charges, aggregated per site
    int64_t n_raw = 0;
    uint32_t n_sites = 0;
    uint32_t* d_site = nullptr;
    double* d_Q = nullptr;
    double* d_S = nullptr;
    double* d_partials = nullptr;
    uint32_t meas_blocks = 1;
    // charge sets sharing the chain: set k is list entries set_off[k] ..
    // set_off[k+1]-1; bins of set k at d_bins + 2 * k * bin_cap
    uint32_t n_sets = 1;
    uint32_t* d_set_off = nullptr;
    double* d_lastxy = nullptr;  // X, Y of the last sample, per set
    // off-lattice charges (trilinear over the 8 corners of each cell)
    bool offl = false;
    uint32_t n_off = 0;
    double* d_r = nullptr;     // 3 n_off positions
    double* d_qo = nullptr;    // n_off charges
    double* d_phit = nullptr;  // 4 n_off scratch (forces only)
    double* d_fsum = nullptr;  // 3 n_off force sums (null: forces off)
    double* d_fsq = nullptr;
    int64_t force_base = 0;    // n_meas when the force sums were last cleared
    // off-lattice charges are stored sorted by cell (neighbouring charges then
    // share the cache lines of their corners); off_order[k] = the caller's
    // index of stored charge k
    std::shared_ptr<const std::vector<uint32_t>> off_order;
    // host copy of the aggregated list of a single on-lattice charge set
    // (shared: copies of the handle made by the autotuner do not copy it)
    struct HostCharges {
        std::vector<uint32_t> site;
        std::vector<double> Q, S;
        std::vector<uint32_t> set_off;  // n_sets + 1 offsets into site / Q / S
    };
    std::shared_ptr<const HostCharges> host_charges;
    // fused gather of the streaming kernel: the list split by colour and
    // regrouped per tile and by plane, for one tile shape and slab (d_off:
    // the colour-0 then the colour-1 offset tables, tiles + 1 each, into
    // d_key / d_Q / d_S; d_part: two buffers, by sample parity, each the
    // colour-0 then the colour-1 partials of one sample, 2 x tiles pairs)
    struct FusedGather {
        bool ready = false;
        bool tried = false;  // lists considered for (variant, tile, slab): ready, or the separate gather
        bool last = false;  // the samples of the last sweep_and_measure took this path
        int variant = 0;    // the kernel whose tiling the lists follow (streaming or blocked)
        uint32_t nbuf = 2;  // sample buffers of partials (2 streaming, 3 blocked)
        uint32_t tile = 0, slab = 0, blocks = 0;
        uint32_t n = 0, cap = 0;  // entries in all; LDS entries staged per workgroup (per list)
        // blocked: lists staged in `parts` parts of `stride` steps; their
        // bounds follow the cumulative offsets in d_off
        uint32_t parts = 1, stride = 0;
        uint32_t sets = 1;  // charge sets in the lists (blocked: up to kBlockedMaxSets)
        uint32_t* d_off = nullptr;
        uint32_t* d_key = nullptr;  // staged key: walk step << 16 | ring-slot byte offset
        uint32_t* d_j = nullptr;    // the site in its colour array (for gather_tail)
        double* d_Q = nullptr;
        double* d_S = nullptr;
        double* d_part = nullptr;
    } fg;
    // How the fused gather takes part in one sweep: its colour-0 launch
    // completes the open sample m (its colour-1 sites), which workgroup 0 of
    // the colour-1 launch records (sample m + *mdev when captured); the
    // colour-1 launch opens this sweep's sample m + 1 (its colour-0 sites;
    // m is the last sample number, modulo 2^32, when none is open).
    // The blocked sweep gathers a sample's colour-0 sites in its own launch
    // (open), its colour-1 sites in the next (finish) and records it in the
    // one after (record, sample m_rec).
    struct FusedStep {
        bool finish = false, open = false;
        uint32_t m = 0;
        const uint32_t* mdev = nullptr;
        bool record = false;
        uint32_t m_rec = 0;
    };
    // misc block: last X, Y (doubles at 64)
    void* d_misc = nullptr;
    // samples
    double* d_bins = nullptr;
    int64_t bin_cap = 0;
    int64_t bin_size = 0;
    int64_t n_meas = 0;
    int64_t t = 0;
    // captured chunks of sweeps (hipGraph) for boxes whose sweeps are short
    struct SweepGraph {
        hipGraphExec_t exec = nullptr;
        int64_t K = 0, every = 0, bin_size = 0;
        int variant = -1;
        uint32_t slab = 0, tile = 0;
        int xcd = 0;
        const void* bins = nullptr;
        const void* site = nullptr;
        const void* gather = nullptr;  // per-tile lists of a fused gather, else null
    };
    SweepGraph g_therm, g_meas;
    hipStream_t cap = nullptr;  // private capture stream
    int graph_mode = 1;         // 0 never, 1 boxes up to 2^24 sites, 2 always
    int variant = LAT_SWEEP_AUTO;
    uint32_t slab = 0;       // planes per workgroup for the slab kernels (0: library default)
    int xcd_order = -1;      // XCD-aware workgroup order for the slab kernels (-1: library default)
    uint32_t tile = kTileDefault;  // tile configuration of the slab kernels

    // the tile the slab kernel `v` runs: the set one, else the library's
    // default.  Streaming kernel: at FP32 (bound by memory traffic) a
    // full-row tile of 96 quads where it divides the row (every plane of a
    // tile is then one contiguous run of memory), else 32 quads x 8 rows with
    // a 6-slot ring; non-temporal stores only where one colour array alone
    // fills the 256 MiB last-level cache (smaller ones keep part of the
    // written colour there for the next half-sweep).
    uint32_t resolved_tile(int v) const {
        if (v == LAT_SWEEP_BLOCKED) return blocked_rows();
        if (tile != kTileDefault) return tile;
        if (v == LAT_SWEEP_ZSLAB && auto_zslab()) return kZslabTileAuto;
        if (v != LAT_SWEEP_STREAM) return 0u;
        const bool wide = esz == 4 && (lh / 4) % 96 == 0;
        const bool nt = (size_t)vh * esz >= ((size_t)256 << 20);
        return wide ? (nt ? kStreamTileFullRow96 : kStreamTileFullRow96Cached) : (nt ? 0u : kStreamTileCached);
    }
    // the planes per workgroup and the workgroup order the slab kernel `v`
    // runs: the set ones, else the library's defaults.  The streaming
    // kernel's full-row FP32 tile measured fastest with 24 planes and each
    // XCD taking a band of every slab's tiles, all XCDs moving through the
    // slabs together (order 2; at 768^3 338 us per half-sweep against 342 us
    // in the hardware's round-robin order and 354-361 us with a contiguous
    // run of tiles per XCD); everything else with 16 (FP32) or 32 (16-bit)
    // planes and a run of tiles per XCD (order 1).
    bool full_row_default(int v) const {
        return v == LAT_SWEEP_STREAM && esz == 4 && resolved_tile(v) == kStreamTileFullRow96;
    }
    uint32_t resolved_slab(int v) const {
        if (slab) return slab;
        if (v == LAT_SWEEP_BLOCKED) return blocked_choice().second;
        if (v == LAT_SWEEP_ZSLAB && auto_zslab()) return 8u;
        return full_row_default(v) ? 24u : default_slab(esz);
    }
    uint32_t resolved_xcd(int v) const {
        if (xcd_order >= 0) return (uint32_t)xcd_order;
        return full_row_default(v) || v == LAT_SWEEP_BLOCKED ? 2u : 1u;
    }
    // Blocked sweep: rows per tile (the set `tile`, else the most rows that
    // fit its LDS and give each compute wave at most three tasks per step),
    // and its old-plane ring (5 slots where the LDS holds them, else 4).
    // 0: the kernel cannot run this box.
    uint32_t blocked_rows() const {
        BlockedShape sh;
        if (tile != kTileDefault) return blocked_geometry(lh, (uint32_t)esz, tile, 4u, &sh) ? tile : 0u;
        return blocked_choice().first;
    }
    // The library's (rows per tile, planes per workgroup) for the blocked
    // sweep: the pair with the highest estimated rate, counting per step the
    // tasks of the busiest SIMD (task t runs on SIMD t % 4), per slab three
    // steps beyond its planes, and per launch whole rounds of workgroups over
    // the device's CUs.  One workgroup per CU: its 13 waves at 84-116 VGPRs
    // leave no SIMD room for the waves of a second.  (0, 0): the kernel
    // cannot run this box.
    std::pair<uint32_t, uint32_t> blocked_choice() const {
        static const uint32_t kSlabs[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
        double best = 0.0;
        std::pair<uint32_t, uint32_t> out(0u, 0u);
        const uint32_t ns = slab ? 1u : (uint32_t)(sizeof(kSlabs) / sizeof(kSlabs[0])) + 1u;
        for (uint32_t k = 1; k <= 16; ++k) {
            BlockedShape sh;
            if (!blocked_geometry(lh, (uint32_t)esz, k, 4u, &sh)) continue;
            const double per_cu = 1.0;
            for (uint32_t i = 0; i < ns; ++i) {
                const uint32_t zc = slab ? slab : (i < ns - 1u ? kSlabs[i] : (uint32_t)lz);
                if (zc > (uint32_t)lz) continue;
                const double wgs = std::ceil((double)ly / k) * std::ceil((double)lz / zc);
                const double slots = per_cu * (double)cus;
                const double rounds = std::ceil(wgs / slots);
                const double score = (double)k * zc / (std::ceil(sh.tasks_total / 4.0) * (zc + 3.0)) *
                                     (wgs / (slots * rounds));
                if (score > best * (1.0 + 1e-9)) {
                    best = score;
                    out = {k, zc};
                }
            }
        }
        return out;
    }
    uint32_t blocked_ring(uint32_t g_cap = 0) const {
        BlockedShape sh;
        return blocked_geometry(lh, (uint32_t)esz, blocked_rows(), 5u, &sh, g_cap) ? 5u : 4u;
    }
    double* last_xy() { return d_lastxy ? d_lastxy : reinterpret_cast<double*>(static_cast<char*>(d_misc) + 64); }
    uint32_t* counters() { return static_cast<uint32_t*>(d_misc); }  // [0] sweeps, [1] samples
    void* c1main() const { return static_cast<char*>(field) + (size_t)vh * esz; }
    void* c1cur() const { return alt_current ? c1alt : c1main(); }
    int effective_variant() const {
        if (variant != LAT_SWEEP_AUTO) return variant;
        // a box one workgroup sweeps in a few microseconds: launch overhead
        // would dominate, so run the whole call in one launch
        if ((uint64_t)vh * 2 <= kResidentMaxSites && n_sets == 1 && !offl) return LAT_SWEEP_RESIDENT;
        if (lh % 4 != 0) return LAT_SWEEP_GENERIC;
        // boxes that spill out of the 256 MB last-level cache: z-marching slabs
        // fed through LDS by a producer wave (colour arrays below 2 GiB)
        const size_t bytes = (size_t)vh * esz;
        if (2 * bytes >= ((size_t)256 << 20) && bytes < ((size_t)1 << 31)) {
            // FP32 with no tile or planes set (those name the streaming
            // kernel's): the blocked sweep, measured 5-22% faster per sweep
            // from 448^3 to 768^3.  Up to four on-lattice charge sets are
            // gathered in the kernel; more sets or off-lattice charges read
            // colour 0, which a measured sweep then stores, from memory
            // (768^3, four sets of 1.1e6 charges through the separate
            // gather: 0.780 against 0.803 ms per step on the streaming
            // sweep; off-lattice charges with forces: 0.862 against 0.906).
            // 16-bit storage keeps the streaming sweep
            // (24-32% faster than the blocked one at 512^3 and 768^3)
            if (auto_blocked && tile == kTileDefault && slab == 0 && blocked_rows() != 0) return LAT_SWEEP_BLOCKED;
            return LAT_SWEEP_STREAM;
        }
        // cache-resident boxes from about 200^3 sites: the z-slab kernel keeps
        // each plane in LDS (measured per sweep against the quad kernel, FP32:
        // -27% at 208^3, -36% at 240^3, equal at 256^3, -34% at 264^3 .. 304^3,
        // -18% at 320^3, -4% at 384^3; BF16: equal at 208^3 and 256^3, -9% to
        // -18% from 240^3 to 448^3).  FP16 storage, whose quad kernel adds
        // neighbours in mixed-precision FMAs, and smaller boxes (quad -20% at
        // 192^3, -55% at 128^3) stay with the quad kernel
        if (esz == 4 || storage == LAT_BF16 || storage == LAT_BF16_SR)
            if ((uint64_t)vh * 2 >= kZslabAutoMinSites) return LAT_SWEEP_ZSLAB;
        return LAT_SWEEP_QUAD;
    }
    // the library chose the z-slab kernel for a cache-resident box: its
    // tuning there is 16 x 16 tiles with 4 planes per step (tile 7), 8 planes
    // per workgroup
    bool auto_zslab() const { return variant == LAT_SWEEP_AUTO && effective_variant() == LAT_SWEEP_ZSLAB; }
};


namespace latcoul {

int check_lattice(const lattice* L);
void graphs_reset(lattice* L);
// fused gather (fused_gather.hip)
void fused_gather_release(lattice* L);
bool fused_gather_on(const lattice* L);
bool fused_gather_current(const lattice* L);  // lists considered for the current kernel and tiling
int fused_gather_prepare(lattice* L);
int enqueue_fused_tail(lattice* L, hipStream_t stream, uint32_t m, const uint32_t* mdev);
// blocked sweep: record sample m_prev (its colour-1 sites gathered by the
// call's last launch), then gather the last sample's colour-1 sites from
// memory and record it
int enqueue_blocked_tail(lattice* L, hipStream_t stream, bool rec_prev, uint32_t m_prev, bool open_last,
                         uint32_t m_last, const uint32_t* mdev);
// sweeps (lattice_api.hip)
// c0_needed: a sweep that keeps colour 0 on chip (LAT_SWEEP_BLOCKED) also
// stores it (for a sample read from memory, or a call's last sweep)
int enqueue_sweep_ex(lattice* L, hipStream_t stream, const uint32_t* tdev, uint32_t rel,
                     const lattice::FusedStep* fs = nullptr, bool c0_needed = true);
int enqueue_sweep(lattice* L, const lattice::FusedStep* fs = nullptr, bool c0_needed = true);
int enqueue_resident(lattice* L, int64_t n_therm, int64_t n_meas, int64_t every);
// n sweeps with a sample after every `every`-th (0: none); eager: launch by
// launch only, never capturing a graph (a capture creates a stream and
// instantiates a graph, which allocate)
int run_sweeps(lattice* L, int64_t n, int64_t every, bool eager = false);
// colour 1 back into field + vh if the blocked or fused sweep left it in the
// second array
int settle_colour1(lattice* L);
// sample bins with room for n_bins_needed bins per charge set (grown)
int ensure_bins(lattice* L, int64_t n_bins_needed);

}  // namespace latcoul
