// Host side of the sample gather fused into the streaming kernel: the
// charge list regrouped per colour, tile and walk step, uploaded once per
// tiling, and the tail that completes a run's last sample.

#include "lattice_impl.hpp"

#include <cstdlib>

namespace latcoul {

void fused_gather_release(lattice* L) {
    L->mem.release(L->fg.d_off);
    L->mem.release(L->fg.d_key);
    L->mem.release(L->fg.d_j);
    L->mem.release(L->fg.d_Q);
    L->mem.release(L->fg.d_S);
    L->mem.release(L->fg.d_part);
    L->fg = lattice::FusedGather();
}

// The sweep kernel whose tiling a fused gather follows (streaming or
// blocked) and that tiling (tile or rows per tile, planes per workgroup);
// variant 0 for kernels without a fused gather.
struct FusedTiling {
    int variant;
    uint32_t tile, slab;
};
static FusedTiling fused_tiling(const lattice* L) {
    const int v = L->effective_variant();
    if (v == LAT_SWEEP_STREAM) return {v, L->resolved_tile(v), L->resolved_slab(v)};
    if (v == LAT_SWEEP_BLOCKED) return {v, L->blocked_rows(), L->resolved_slab(v)};
    return {0, 0u, 0u};
}

bool fused_gather_current(const lattice* L) {
    const FusedTiling ft = fused_tiling(L);
    return L->fg.tried && L->fg.variant == ft.variant && L->fg.tile == ft.tile && L->fg.slab == ft.slab;
}

// Whether samples of this lattice are gathered inside the sweep kernel:
// on-lattice charges (one set; the blocked sweep up to kBlockedMaxSets) and
// the lists built for the current kernel, tiling and sets.
bool fused_gather_on(const lattice* L) {
    return L->fg.ready && L->fg.sets == L->n_sets && !L->offl && fused_gather_current(L) && L->fg.variant != 0;
}

// Lists of the blocked sweep's tiling: per tile (by + nby bz, kty rows, zc
// planes) the charged colour-0 sites, gathered by its producer wave in step
// z - z0 + 2 from a colour-0 slot (row y - y0 + 1), then the charged
// colour-1 sites, gathered in step z - z0 + 1 from an old-plane slot (row
// y - y0 + 2), each sorted by step, the entries of every charge set in one
// list (the set in the key's bits 26-27).  Three sample buffers of
// partials, each the colour-0 then the colour-1 pairs of set 0, then set 1's.
static int blocked_gather_prepare(lattice* L, uint32_t kty, uint32_t zc) {
    if (kty == 0 || zc == 0 || zc + 2u > kBlockedStepMask) return LAT_OK;
    const uint32_t nq = L->lh / 4, ly = (uint32_t)L->ly, lz = (uint32_t)L->lz;
    const uint32_t nby = (ly + kty - 1) / kty, nbz = (lz + zc - 1) / zc;
    const uint32_t tiles = nby * nbz;
    const uint32_t plane = ly * L->lh;
    const uint32_t rb = 32u + nq * 4u * (uint32_t)L->esz;
    if ((uint64_t)(kty + 4u) * rb > 0xFFFFu) return LAT_OK;  // slot offsets in 16 bits
    const lattice::HostCharges& hc = *L->host_charges;
    const size_t n = hc.site.size();
    const uint32_t sets = (uint32_t)hc.set_off.size() - 1u;
    std::vector<uint64_t> key_of(n);
    std::vector<uint32_t> tile_of(n), j_of(n), packed_of(n);
    size_t n0 = 0;
    uint32_t set = 0;
    for (size_t i = 0; i < n; ++i) {
        while (i >= hc.set_off[set + 1]) ++set;
        const uint32_t c = hc.site[i] >= L->vh ? 1u : 0u;
        const uint32_t j = hc.site[i] - c * L->vh;
        const uint32_t z = j / plane, rem = j - z * plane, y = rem / L->lh, jx = rem - y * L->lh;
        const uint32_t by = y / kty, bz = z / zc;
        tile_of[i] = by + nby * bz;
        j_of[i] = j;
        const uint32_t row = y - by * kty + 1u + c;
        const uint32_t step = z - bz * zc + 2u - c;
        packed_of[i] = (set << 26) | (step << 16) | (row * rb + 16u + jx * (uint32_t)L->esz);
        key_of[i] = ((uint64_t)c * tiles + tile_of[i]) * (zc + 2u) + step;
        n0 += c ? 0u : 1u;
    }
    std::vector<uint32_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key_of[a] < key_of[b]; });
    std::vector<uint32_t> off(2 * ((size_t)tiles + 1), 0u), key(n), jv(n);
    std::vector<double> Q(n), S(n);
    for (size_t k = 0; k < n; ++k) {
        const uint32_t i = order[k];
        const size_t c = k < n0 ? 0 : 1;
        off[c * (tiles + 1) + tile_of[i] + 1] += 1;
        key[k] = packed_of[i];
        jv[k] = j_of[i];
        Q[k] = hc.Q[i];
        S[k] = hc.S[i];
    }
    off[tiles + 1] = (uint32_t)n0;
    for (size_t c = 0; c < 2; ++c)
        for (size_t t = 0; t < tiles; ++t) off[c * (tiles + 1) + t + 1] += off[c * (tiles + 1) + t];
    // Each list is staged in parts of `stride` steps.  The fewest parts whose
    // longest part leaves room for the five-slot ring, else for four slots;
    // none: the separate gather.
    auto longest_part = [&](uint32_t parts, uint32_t stride) {
        uint32_t longest = 0;
        std::vector<uint32_t> cnt(parts);
        for (size_t ct = 0; ct < 2u * (size_t)tiles; ++ct) {
            const size_t c = ct / tiles, t = ct % tiles;
            std::fill(cnt.begin(), cnt.end(), 0u);
            for (uint32_t k = off[c * (tiles + 1) + t]; k < off[c * (tiles + 1) + t + 1]; ++k)
                ++cnt[(((key[k] >> 16) & kBlockedStepMask) - 1u) / stride];
            for (uint32_t x : cnt) longest = std::max(longest, x);
        }
        return std::max<uint32_t>(64u, (longest + 63u) / 64u * 64u);
    };
    // LATCOUL_GATHER_PART_CAP: a smaller bound on the entries of a part
    // (rounded up to 64), for tests of the multi-part staging
    uint32_t cap_limit = 0;
    if (const char* env = std::getenv("LATCOUL_GATHER_PART_CAP")) cap_limit = (uint32_t)std::strtoul(env, nullptr, 10);
    uint32_t parts = 0, stride = 0, cap = 0;
    BlockedShape sh;
    for (uint32_t ring = 5u; ring >= 4u && parts == 0; --ring)
        for (uint32_t p = 1; p <= kBlockedMaxParts && p <= zc + 1u; ++p) {
            const uint32_t st = (zc + 1u + p - 1u) / p, cp = longest_part(p, st);
            if (cap_limit && cp > std::max<uint32_t>(64u, (cap_limit + 63u) / 64u * 64u)) continue;
            if (blocked_geometry(L->lh, (uint32_t)L->esz, kty, ring, &sh, cp)) {
                parts = p;
                stride = st;
                cap = cp;
                break;
            }
        }
    if (parts == 0 || (uint64_t)n * 8u >= (1ull << 32)) return LAT_OK;  // the separate gather
    // part bounds per (colour, tile), after the cumulative table
    const size_t np1 = parts + 1u, pbase = off.size();
    off.resize(pbase + 2u * (size_t)tiles * np1);
    for (size_t ct = 0; ct < 2u * (size_t)tiles; ++ct) {
        const size_t c = ct / tiles, t = ct % tiles;
        const uint32_t b = off[c * (tiles + 1) + t], e = off[c * (tiles + 1) + t + 1];
        uint32_t k = b;
        for (uint32_t p = 0; p < parts; ++p) {
            while (k < e && (((key[k] >> 16) & kBlockedStepMask) - 1u) / stride < p) ++k;
            off[pbase + ct * np1 + p] = k;
        }
        off[pbase + ct * np1 + parts] = e;
    }
    lattice::FusedGather g = L->fg;
    g.d_off = static_cast<uint32_t*>(L->mem.alloc(off.size() * 4));
    g.d_key = static_cast<uint32_t*>(L->mem.alloc(std::max<size_t>(n, 1) * 4));
    g.d_j = static_cast<uint32_t*>(L->mem.alloc(std::max<size_t>(n, 1) * 4));
    g.d_Q = static_cast<double*>(L->mem.alloc(std::max<size_t>(n, 1) * 8));
    g.d_S = static_cast<double*>(L->mem.alloc(std::max<size_t>(n, 1) * 8));
    g.d_part = static_cast<double*>(L->mem.alloc((size_t)tiles * 96 * sets));
    L->fg = g;
    if (!g.d_off || !g.d_key || !g.d_j || !g.d_Q || !g.d_S || !g.d_part) {
        const lattice::FusedGather keep = L->fg;
        fused_gather_release(L);
        L->fg.tried = true;  // the separate gather for this tiling
        L->fg.variant = keep.variant;
        L->fg.tile = keep.tile;
        L->fg.slab = keep.slab;
        return LAT_OK;
    }
    hipError_t e = hipMemcpyAsync(g.d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_key, key.data(), n * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_j, jv.data(), n * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_Q, Q.data(), n * 8, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_S, S.data(), n * 8, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) {
        fused_gather_release(L);
        return hip_fail(e, "fused gather list upload");
    }
    L->fg.ready = true;
    L->fg.nbuf = 3;
    L->fg.sets = sets;
    L->fg.blocks = tiles;
    L->fg.n = (uint32_t)n;
    L->fg.cap = cap;
    L->fg.parts = parts;
    L->fg.stride = stride;
    return LAT_OK;
}

// Resident workgroups per CU of a kernel with `lds` bytes of LDS and `waves`
// waves per workgroup (160 KiB of LDS and 32 wave slots per CU).
static uint32_t workgroups_per_cu(uint32_t lds, uint32_t waves) {
    return std::min<uint32_t>(lds ? 163840u / lds : 32u, 32u / waves);
}

// Build the per-tile lists of the fused gather for the current tiling (host
// sort of the aggregated list, one upload); outside any capture.  Without
// them (other kernels, off-lattice charges, several sets on another kernel
// than the blocked sweep or more than it serves, a tile list too long to
// stage in LDS without costing the sweep kernel a resident workgroup,
// allocation failure) the samples go through the separate gather.
int fused_gather_prepare(lattice* L) {
    const FusedTiling ft = fused_tiling(L);
    if (ft.variant == 0 || L->offl || !L->host_charges || L->host_charges->site.size() != L->n_sites ||
        L->host_charges->set_off.size() != (size_t)L->n_sets + 1u ||
        (L->n_sets != 1 && ft.variant != LAT_SWEEP_BLOCKED) || L->n_sets > kBlockedMaxSets)
        return LAT_OK;
    if (fused_gather_current(L)) return LAT_OK;
    fused_gather_release(L);
    graphs_reset(L);
    L->fg.tried = true;
    L->fg.variant = ft.variant;
    L->fg.tile = ft.tile;
    L->fg.slab = ft.slab;
    if (ft.variant == LAT_SWEEP_BLOCKED) return blocked_gather_prepare(L, ft.tile, ft.slab);
    const uint32_t tile = ft.tile, slab = ft.slab;
    StreamTileShape sh;
    if (!stream_tile_geometry(tile, L->esz, &sh)) return LAT_OK;
    const uint32_t tq = sh.quads, ty = sh.rows;
    const uint32_t nq = L->lh / 4, ly = (uint32_t)L->ly, lz = (uint32_t)L->lz;
    const uint32_t nbx = (nq + tq - 1) / tq, nby = (ly + ty - 1) / ty, nbz = (lz + slab - 1) / slab;
    const uint32_t blocks = nbx * nby * nbz;
    const uint32_t plane = (uint32_t)L->ly * L->lh;
    const lattice::HostCharges& hc = *L->host_charges;
    const size_t n = hc.site.size();
    // sort key of every charged site: its colour, its tile, its plane
    // staged key: the step of the tile's walk that updates the site's plane
    // << 16 | byte offset of the site in a ring slot (rows y0-1 .. y0+ty of
    // tq + 2 quads: halo quad first); a tile's list is sorted by step
    if (slab > 0xFFFFu) return LAT_OK;
    const uint32_t row_bytes = (tq + 2u) * 4u * (uint32_t)L->esz;
    std::vector<uint64_t> key_of(n);
    std::vector<uint32_t> tile_of(n), j_of(n), packed_of(n);
    size_t n0 = 0;
    for (size_t i = 0; i < n; ++i) {
        const uint32_t c = hc.site[i] >= L->vh ? 1u : 0u;
        const uint32_t j = hc.site[i] - c * L->vh;
        const uint32_t z = j / plane, rem = j - z * plane, y = rem / L->lh, jx = rem - y * L->lh;
        const uint32_t bx = (jx / 4) / tq, by = y / ty, bz = z / slab;
        tile_of[i] = bx + nbx * (by + nby * bz);
        j_of[i] = j;
        const uint32_t off = (y - by * ty + 1u) * row_bytes + (jx - 4u * tq * bx + 4u) * (uint32_t)L->esz;
        // the step at which the tile's walk updates plane z (odd slabs walk down)
        const uint32_t z0 = bz * slab, z1 = std::min(z0 + slab, lz);
        const uint32_t step = kStreamAltZ && (bz & 1u) ? z1 - 1u - z : z - z0;
        packed_of[i] = (step << 16) | off;
        key_of[i] = ((uint64_t)c * blocks + tile_of[i]) * lz + step;
        n0 += c ? 0u : 1u;
    }
    std::vector<uint32_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key_of[a] < key_of[b]; });
    // offsets: colour 0 at [0, blocks], colour 1 at [blocks + 1, 2 blocks + 1]
    std::vector<uint32_t> off(2 * ((size_t)blocks + 1), 0u), key(n), jv(n);
    std::vector<double> Q(n), S(n);
    for (size_t k = 0; k < n; ++k) {
        const uint32_t i = order[k];
        const size_t c = k < n0 ? 0 : 1;
        off[c * (blocks + 1) + tile_of[i] + 1] += 1;
        key[k] = packed_of[i];
        jv[k] = j_of[i];
        Q[k] = hc.Q[i];
        S[k] = hc.S[i];
    }
    uint32_t longest = 0;
    for (size_t t = 0; t < 2 * ((size_t)blocks + 1); ++t) longest = std::max(longest, off[t]);
    const uint64_t cap = ((uint64_t)longest + 63u) / 64u * 64u;
    if (cap > 256u) return LAT_OK;  // the kernel holds up to 4 x 64 keys per tile in registers
    const uint64_t lds = sh.lds + (uint64_t)kGatherEntryBytes * cap;
    if (lds > 65536u || workgroups_per_cu((uint32_t)lds, sh.waves) < workgroups_per_cu(sh.lds, sh.waves) ||
        (uint64_t)n * 8u >= (1ull << 32))
        return LAT_OK;  // the separate gather
    off[blocks + 1] = (uint32_t)n0;
    for (size_t c = 0; c < 2; ++c)
        for (size_t t = 0; t < blocks; ++t) off[c * (blocks + 1) + t + 1] += off[c * (blocks + 1) + t];
    lattice::FusedGather g = L->fg;
    g.d_off = static_cast<uint32_t*>(L->mem.alloc(off.size() * 4));
    g.d_key = static_cast<uint32_t*>(L->mem.alloc(std::max<size_t>(n, 1) * 4));
    g.d_j = static_cast<uint32_t*>(L->mem.alloc(std::max<size_t>(n, 1) * 4));
    g.d_Q = static_cast<double*>(L->mem.alloc(std::max<size_t>(n, 1) * 8));
    g.d_S = static_cast<double*>(L->mem.alloc(std::max<size_t>(n, 1) * 8));
    g.d_part = static_cast<double*>(L->mem.alloc((size_t)blocks * 64));
    L->fg = g;  // released by fused_gather_release on any failure below
    if (!g.d_off || !g.d_key || !g.d_j || !g.d_Q || !g.d_S || !g.d_part) {
        fused_gather_release(L);
        L->fg.tried = true;  // the separate gather for this tiling
        L->fg.variant = LAT_SWEEP_STREAM;
        L->fg.tile = tile;
        L->fg.slab = slab;
        return LAT_OK;
    }
    hipError_t e = hipMemcpyAsync(g.d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_key, key.data(), n * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_j, jv.data(), n * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_Q, Q.data(), n * 8, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(g.d_S, S.data(), n * 8, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) {
        fused_gather_release(L);
        return hip_fail(e, "fused gather list upload");
    }
    L->fg.ready = true;
    L->fg.nbuf = 2;
    L->fg.blocks = blocks;
    L->fg.n = (uint32_t)n;
    L->fg.cap = (uint32_t)cap;
    return LAT_OK;
}


int enqueue_blocked_tail(lattice* L, hipStream_t stream, bool rec_prev, uint32_t m_prev, bool open_last,
                         uint32_t m_last, const uint32_t* mdev) {
    const lattice::FusedGather& g = L->fg;
    auto buf = [&](uint32_t k) { return g.d_part + (size_t)(k % 3u) * 4 * g.blocks * g.sets; };
    hipError_t e = hipSuccess;
    if (rec_prev)
        e = launch_finalize_measure(buf(m_prev), 2 * g.blocks, g.sets, L->d_bins, m_prev, (uint32_t)L->bin_size,
                                    mdev, L->last_xy(), (uint32_t)L->bin_cap, stream);
    if (e == hipSuccess && open_last && g.sets > 1) {
        // several sets: the last sample from memory by the separate gather
        // (the call's last sweep stored colour 0), into its own partials
        MeasureArgs a{L->field, L->c1cur(), L->vh, L->d_site, L->d_Q, L->d_S, L->n_sites, L->d_partials,
                      L->d_bins, m_last, (uint32_t)L->bin_size, mdev, L->last_xy(), L->storage, L->meas_blocks,
                      L->d_set_off, L->n_sets, (uint32_t)L->bin_cap};
        e = launch_measure(a, stream);
    } else if (e == hipSuccess && open_last) {
        GatherTailArgs a{L->c1cur(), L->storage, g.blocks, g.d_off + g.blocks + 1, g.d_j, g.d_Q, g.d_S,
                         buf(m_last) + 2 * (size_t)g.blocks};
        e = launch_gather_tail(a, stream);
        if (e == hipSuccess)
            e = launch_finalize_measure(buf(m_last), 2 * g.blocks, 1u, L->d_bins, m_last, (uint32_t)L->bin_size,
                                        mdev, L->last_xy(), (uint32_t)L->bin_cap, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "measure launch");
    return LAT_OK;
}

// The open sample's colour-1 sites from memory (no sweep follows it), then
// its finalize as sample m.
int enqueue_fused_tail(lattice* L, hipStream_t stream, uint32_t m, const uint32_t* mdev) {
    const lattice::FusedGather& g = L->fg;
    double* buf = g.d_part + (size_t)(m & 1u) * 4 * g.blocks;  // sample m's partials, colour 0 then 1
    GatherTailArgs a{L->c1cur(), L->storage, g.blocks, g.d_off + g.blocks + 1, g.d_j, g.d_Q, g.d_S,
                     buf + 2 * (size_t)g.blocks};
    hipError_t e = launch_gather_tail(a, stream);
    if (e == hipSuccess)
        e = launch_finalize_measure(buf, 2 * g.blocks, 1u, L->d_bins, m, (uint32_t)L->bin_size, mdev,
                                    L->last_xy(), (uint32_t)L->bin_cap, stream);
    if (e != hipSuccess) return hip_fail(e, "measure launch");
    return LAT_OK;
}

}  // namespace latcoul
