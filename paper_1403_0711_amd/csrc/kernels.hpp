// Host-side launch interface of the library's kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace latcoul {

enum : int { kVariantQuad = 1, kVariantGeneric = 2, kVariantZslab = 3, kVariantFused = 4, kVariantStream = 6 };

// Storage codes: 0 FP32, 1 BF16, 2 FP16 (round to nearest even), 3 BF16 and
// 4 FP16 rounded stochastically.  The array format of a code (what readers
// of the field use): 3 is a BF16 array, 4 an FP16 one.
inline int storage_grid(int storage) { return storage == 3 ? 1 : storage == 4 ? 2 : storage; }

// One half-sweep of colour c = h & 1 on one lattice.
// Finalize of one sample inside a sweep launch (workgroup 0, overlapped with
// its first plane loads): the sum of n (X, Y) partial pairs at part is
// recorded as sample m (+ *mdev) in bin (m [+ *mdev]) / bin_size.
struct SampleFinalize {
    const double* part = nullptr;  // null: none
    uint32_t n = 0;
    double* bins = nullptr;
    uint32_t m = 0, bin_size = 1;
    const uint32_t* mdev = nullptr;
    double* last_xy = nullptr;
};

struct SweepArgs {
    void* field;      // 2 * vh elements: colour 0 then colour 1
    uint32_t lh, ly, lz, vh;
    uint32_t c, h;    // colour, half-sweep index (Philox counter word 1)
    uint32_t k0, k1;  // Philox key
    uint32_t chain;   // Philox counter word 2
    int storage;      // storage code (storage_grid)
    int variant;      // kVariantQuad / kVariantGeneric / kVariantZslab / kVariantStream
    uint32_t zc;      // slab kernels: planes per workgroup (0 = 16)
    uint32_t xcd_order;  // slab kernels: XCD-aware block order
    uint32_t tile;    // slab kernels: tile configuration (kZslabTiles / kStreamTiles of them)
    const uint32_t* tdev;  // if set, h += 2 * tdev[0] (sweep counter on the device)
    // streaming kernel: fused gather of the charged sites of the other
    // colour (1 - c) over per-tile lists (g_off: tiles + 1 absolute offsets;
    // g_key: the step of the tile's walk that updates the site's plane << 16
    // | its byte offset in a ring slot; g_Q, g_S; g_n entries in the arrays), one (X, Y)
    // partial per tile into g_part.  g_cap: LDS entries staged per workgroup
    // (a multiple of 64, at least the longest tile list, at most 256).
    // Null: no gather.
    const uint32_t* g_off = nullptr;
    const uint32_t* g_key = nullptr;
    const double* g_Q = nullptr;
    const double* g_S = nullptr;
    double* g_part = nullptr;
    uint32_t g_n = 0, g_cap = 0;
    // streaming kernel: finalize of the previous sample (see SampleFinalize)
    SampleFinalize fin;
};
constexpr uint32_t kGatherEntryBytes = 20;  // staged key (4 B), Q and S (8 B each)
constexpr int kZslabTiles = 8;
constexpr int kStreamTiles = 11;  // tile configurations of the streaming slab kernel
// streaming kernel: odd slabs walk down z (the fused gather's lists follow
// each tile's walk order)
constexpr bool kStreamAltZ = true;
hipError_t launch_halfsweep(const SweepArgs& a, hipStream_t stream);
hipError_t launch_halfsweep_stream(const SweepArgs& a, hipStream_t stream);  // tile 0 .. kStreamTiles-1
// Shape of a streaming-kernel tile configuration at element size esz: quads
// per tile row, rows, static LDS bytes (the plane ring and the kernel's small
// static arrays), waves per workgroup.
struct StreamTileShape {
    uint32_t quads, rows, lds, waves;
};
bool stream_tile_geometry(uint32_t tile, uint32_t esz, StreamTileShape* out);
// The colour-1 part of a fused-gather sample from the colour-1 array in
// memory, in the streaming kernel's order (one partial per tile).
struct GatherTailArgs {
    const void* field1;  // colour-1 array
    int storage;
    uint32_t tiles;
    const uint32_t* g_off;  // the colour-1 lists: tiles + 1 offsets into
    const uint32_t* g_j;    // site j in the colour-1 array, per entry
    const double* g_Q;
    const double* g_S;
    double* g_part;
};
hipError_t launch_gather_tail(const GatherTailArgs& a, hipStream_t stream);
// device-side sweep / sample counters (ctr[0], ctr[1]) for graph replays
hipError_t launch_set_counters(uint32_t* ctr, uint32_t t, uint32_t m, hipStream_t stream);
hipError_t launch_advance_counters(uint32_t* ctr, uint32_t dt, uint32_t dm, hipStream_t stream);

// Both half-sweeps of sweep t in one pass (temporal blocking), lh % 4 == 0.
struct FusedArgs {
    void* c0;          // colour 0 (written)
    const void* b_in;  // colour 1 before the sweep
    void* b_out;       // colour 1 after the sweep (a different array)
    uint32_t lh, ly, lz, vh;
    uint32_t h0;       // 2t: colour 0 uses h0, colour 1 uses h0 + 1
    uint32_t k0, k1, chain;
    int storage;
    uint32_t slab;     // planes per workgroup along z (0 = default)
    uint32_t xcd_order;
    const uint32_t* tdev;  // if set, h0 += 2 * tdev[0]
};
hipError_t launch_fused_sweep(const FusedArgs& a, hipStream_t stream);
hipError_t prepare_fused_sweep();  // once, before fused launches and outside capture

// Parts the blocked sweep's fused-gather lists are staged in, at most.
constexpr uint32_t kBlockedMaxParts = 8;
// Charge sets the blocked sweep's fused gather serves in one walk, at most
// (an entry's set in bits 26-27 of its key, the step in bits 16-25).
constexpr uint32_t kBlockedMaxSets = 4;
constexpr uint32_t kBlockedStepMask = 0x3FFu;

// Both half-sweeps of sweep t in one pass with colour 0 kept in LDS (the
// streaming temporally blocked sweep): colour 1 read from c1_in, written to
// c1_out (a different array), colour 0 stored to c0_out only if it is set.
// Full-row tiles of kty rows walking zc planes; lh % 4 == 0 and the rows a
// whole number of 16-byte chunks (16-bit storage: lx % 16 == 0).
struct BlockedArgs {
    const void* c1_in;
    void* c1_out;
    void* c0_out;      // null: colour 0 not stored
    uint32_t lh, ly, lz;
    uint32_t kty, zc;  // rows per tile, planes per workgroup
    uint32_t ring;     // old-plane slots: 4 or 5
    uint32_t nt;       // non-temporal stores of colour 1
    uint32_t h0;       // 2t: colour 0 uses h0, colour 1 h0 + 1
    uint32_t k0, k1, chain;
    uint32_t xcd_order;
    const uint32_t* tdev;  // if set, h0 += 2 * tdev[0]
    int storage;
    // fused gather (g_key set): per tile (by + nby bz) a list of its charged
    // colour-0 sites and one of its charged colour-1 sites (of all g_sets
    // charge sets), each sorted by the step that gathers it; entry key =
    // set << 26 | step << 16 | byte offset in a ring slot (colour 0: a
    // colour-0 slot; colour 1: an old-plane slot).  g_cap entries of each
    // list are staged in LDS (a multiple of 64).  part0: the (X, Y) pair per
    // tile of this sweep's colour-0 sites of set 0 (null: this sweep is not
    // sampled), set k's at part0 + k g_set_stride; part1: likewise the pairs
    // of the previous sweep's colour-1 sites (null: it was not sampled).
    // fin: the sample two sweeps back, recorded by workgroup 0 (one set).
    const uint32_t* g_off = nullptr;
    const uint32_t* g_key = nullptr;
    const double* g_Q = nullptr;
    const double* g_S = nullptr;
    uint32_t g_n = 0, g_cap = 0;
    // the lists are staged in g_parts parts of g_stride steps each (part p:
    // steps 1 + p g_stride .. (p + 1) g_stride); g_off holds, per colour c
    // and tile t, the g_parts + 1 part bounds at (c tiles + t)(g_parts + 1)
    uint32_t g_parts = 1, g_stride = 0;  // g_parts <= kBlockedMaxParts
    uint32_t g_sets = 1, g_set_stride = 0;  // g_sets <= kBlockedMaxSets; doubles between sets' partials
    double* part0 = nullptr;
    double* part1 = nullptr;
    SampleFinalize fin;
};
struct BlockedShape {
    uint32_t lds;              // dynamic LDS bytes per workgroup
    uint32_t tasks_total;      // wave-tasks of a step (both colours)
    uint32_t tasks_per_wave;   // wave-tasks of a compute wave per step
    uint32_t loads_per_plane;  // load instructions of the producer per plane
};
// g_cap: fused-gather entries staged per list (0: no fused gather)
bool blocked_geometry(uint32_t lh, uint32_t esz, uint32_t kty, uint32_t ring, BlockedShape* out,
                      uint32_t g_cap = 0);
hipError_t launch_blocked_sweep(const BlockedArgs& a, hipStream_t stream);
hipError_t prepare_blocked_sweep();  // once per process (also done by the first launch)

// Gather of the charge-weighted correlator after a sweep (Eq. nsum2):
// X = sum_s Q_s phi_s, Y = sum_s S_s phi_s^2 over the site-aggregated charge
// list, O = X^2 - Y compensated-added into bins[2*bin], bins[2*bin+1]; for
// several charge sets, per set (entries set_off[k] .. set_off[k+1]-1, bins at
// bins + 2 * k * bin_stride, X and Y at last_xy[2k], last_xy[2k+1]).
struct MeasureArgs {
    const void* field0;    // colour 0
    const void* field1;    // colour 1
    uint32_t vh;
    const uint32_t* site;  // c * vh + j, sorted ascending
    const double* Q;       // sum of q on the site
    const double* S;       // sum of q^2 on the site
    uint32_t n;            // number of charged sites
    double* partials;      // 2 * blocks * n_sets scratch
    double* bins;
    uint32_t m;            // sample index (relative to *mdev when mdev is set)
    uint32_t bin_size;
    const uint32_t* mdev;  // sample counter on the device, or null
    double* last_xy;       // X, Y of this sample, per set
    int storage;
    uint32_t blocks;       // blocks per set (fixed for given sets: fixes the sum order)
    const uint32_t* set_off;  // n_sets + 1 offsets into the list (null: one set of n entries)
    uint32_t n_sets;
    uint32_t bin_stride;   // bins per set in `bins`
};
hipError_t launch_measure(const MeasureArgs& a, hipStream_t stream);
uint32_t measure_blocks(uint32_t n);
// the second phase alone: per set, sum the partials, form O, bin it
hipError_t launch_finalize_measure(const double* partials, uint32_t blocks, uint32_t n_sets, double* bins,
                                   uint32_t m, uint32_t bin_size, const uint32_t* mdev, double* last_xy,
                                   uint32_t bin_stride, hipStream_t stream);

// Off-lattice charges (trilinear over the 8 corners of each charge's cell):
// one sample O = X^2 - Y into bins[2*bin], and with fsum set, the force
// sample 2 q_i grad phi~_i (X - q_i phi~_i) added to fsum / fsq (3 per charge).
struct OffLatticeArgs {
    const void* field0;
    const void* field1;
    uint32_t lx, ly, lz;
    const double* r;       // 3n positions, lattice units
    const double* q;       // n charges
    uint32_t n;
    double* partials;      // 2 * blocks scratch
    double* bins;
    uint32_t m;            // sample index (relative to *mdev when mdev is set)
    uint32_t bin_size;
    const uint32_t* mdev;
    double* last_xy;
    int storage;
    uint32_t blocks;
    uint32_t bin_stride;
    double* phit;          // 4n scratch: phi~ and its gradient per charge (forces only)
    double* fsum;          // 3n force sums, or null: no forces
    double* fsq;           // 3n sums of squares
};
hipError_t launch_measure_offlattice(const OffLatticeArgs& a, hipStream_t stream);

// Batched chains: one workgroup owns one chain and runs all its sweeps.
struct BatchChainDesc {
    uint64_t field_off;   // element offset of the chain's field (2 * vh elements)
    uint64_t bin_off;     // first bin slot of this chain (2 doubles each)
    uint32_t lh, ly, lz, vh;
    uint32_t chain_id;
    uint32_t site_off, n_sites;  // range in the concatenated charge arrays
    uint32_t meas0;              // samples this chain already holds
    uint32_t ring;               // 1: the LDS-ring half-sweep where the chain's planes allow it
};
// A chain the LDS-ring half-sweep can take (lh % 4 == 0, at most
// kBatchRingMaxPlaneQuads quads per plane) and that does not already keep its
// whole other colour in LDS (more than 1024 quads).
constexpr uint32_t kBatchRingMaxPlaneQuads = 3072;
inline bool batch_ring_applies(uint32_t lh, uint32_t ly, uint32_t vh) {
    return lh % 4u == 0 && (lh / 4u) * ly <= kBatchRingMaxPlaneQuads && vh > 4096u;
}
struct BatchArgs {
    void* field;
    const BatchChainDesc* desc;  // device table (batch) ...
    const uint32_t* order;       // ... chains in launch order (largest first)
    uint32_t n_chains;
    const uint32_t* site;
    const double* Q;
    const double* S;
    double* bins;
    uint32_t t0;        // sweep counter at the start of this run (same for all chains)
    uint32_t n_therm, n_meas, every, bin_size;
    uint32_t k0, k1;
    int storage;
    bool single;                 // one lattice: descriptor passed by value
    BatchChainDesc single_desc;
    double* last_xy;             // single: X, Y of the last sample (or null)
};
hipError_t launch_batch(const BatchArgs& a, hipStream_t stream);

}  // namespace latcoul
