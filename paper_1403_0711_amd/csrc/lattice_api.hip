// C-ABI runtime of the heat-bath Coulomb-energy estimator: lattice objects,
// charge upload, sweep scheduling, graph capture, sample bins and the final
// estimate.  The kernels live in stream_sweep.hip, sweep_kernels.hip,
// fused_sweep.hip, measure_kernels.hip, offlattice_kernels.hip and
// batch_kernels.hip; the fused gather's host side in fused_gather.hip, the
// autotuner in autotune.hip.

#include "lattice_impl.hpp"

namespace latcoul {

int check_lattice(const lattice* L) {
    if (!L) return set_error(LAT_ERR_ARG, "null lattice handle");
    return LAT_OK;
}


// One sweep on `stream`.  Eager (tdev null): sweep index L->t, which is
// advanced.  Captured: index tdev[0] + rel, read on the device at run time.
// fs: the fused gather's part in this sweep (streaming kernel only).
int enqueue_sweep_ex(lattice* L, hipStream_t stream, const uint32_t* tdev, uint32_t rel,
                     const lattice::FusedStep* fs, bool c0_needed) {
    const uint32_t h0 = tdev ? 2u * rel : (uint32_t)(2 * L->t);
    const int v = L->effective_variant();
    hipError_t e;
    if (v == LAT_SWEEP_BLOCKED) {
        BlockedArgs a{};
        a.c1_in = L->c1cur();
        a.c1_out = L->alt_current ? L->c1main() : L->c1alt;
        a.c0_out = c0_needed ? L->field : nullptr;
        a.lh = L->lh;
        a.ly = (uint32_t)L->ly;
        a.lz = (uint32_t)L->lz;
        a.kty = L->blocked_rows();
        a.zc = L->resolved_slab(v);
        a.ring = L->blocked_ring();
        a.nt = (size_t)L->vh * L->esz >= ((size_t)256 << 20) ? 1u : 0u;
        a.h0 = h0;
        a.k0 = (uint32_t)L->seed;
        a.k1 = (uint32_t)(L->seed >> 32);
        a.chain = L->chain;
        a.xcd_order = L->resolved_xcd(v);
        a.tdev = tdev;
        a.storage = L->storage;
        bool record_after = false;  // several sets: the sample recorded by its own launch
        if (fs && (fs->open || fs->finish || fs->record)) {  // the fused gather's part in this sweep
            const lattice::FusedGather& g = L->fg;
            // sample k's buffer: per set, the colour-0 then the colour-1 pairs of every tile
            auto buf = [&](uint32_t k) { return g.d_part + (size_t)(k % 3u) * 4 * g.blocks * g.sets; };
            if (fs->open || fs->finish) {
                a.g_off = g.d_off + 2 * ((size_t)g.blocks + 1);  // the part bounds
                a.g_key = g.d_key;
                a.g_Q = g.d_Q;
                a.g_S = g.d_S;
                a.g_n = g.n;
                a.g_cap = g.cap;
                a.g_parts = g.parts;
                a.g_stride = g.stride;
                a.g_sets = g.sets;
                a.g_set_stride = 4 * g.blocks;
                a.ring = L->blocked_ring(g.cap);
            }
            if (fs->open) a.part0 = buf(fs->m + 1u);                               // colour-0 pairs
            if (fs->finish) a.part1 = buf(fs->m) + 2 * (size_t)g.blocks;           // colour-1 pairs
            record_after = fs->record && g.sets > 1;
            if (fs->record && g.sets == 1) {
                a.fin.part = buf(fs->m_rec);
                a.fin.n = 2 * g.blocks;
                a.fin.bins = L->d_bins;
                a.fin.m = fs->m_rec;
                a.fin.bin_size = (uint32_t)L->bin_size;
                a.fin.mdev = fs->mdev;
                a.fin.last_xy = L->last_xy();
            }
        }
        e = launch_blocked_sweep(a, stream);
        if (e == hipSuccess) L->alt_current = !L->alt_current;
        if (e == hipSuccess && record_after) {
            const lattice::FusedGather& g = L->fg;
            e = launch_finalize_measure(g.d_part + (size_t)(fs->m_rec % 3u) * 4 * g.blocks * g.sets, 2 * g.blocks,
                                        g.sets, L->d_bins, fs->m_rec, (uint32_t)L->bin_size, fs->mdev,
                                        L->last_xy(), (uint32_t)L->bin_cap, stream);
        }
    } else if (v == LAT_SWEEP_FUSED) {
        void* out = L->alt_current ? L->c1main() : L->c1alt;
        FusedArgs a{L->field, L->c1cur(), out, L->lh, (uint32_t)L->ly, (uint32_t)L->lz, L->vh, h0,
                    (uint32_t)L->seed, (uint32_t)(L->seed >> 32), L->chain, L->storage, L->resolved_slab(v),
                    L->resolved_xcd(v),
                    tdev};
        e = launch_fused_sweep(a, stream);
        if (e == hipSuccess) L->alt_current = !L->alt_current;
    } else {
        const int kv = v == LAT_SWEEP_QUAD     ? kVariantQuad
                       : v == LAT_SWEEP_ZSLAB  ? kVariantZslab
                       : v == LAT_SWEEP_STREAM ? kVariantStream
                                               : kVariantGeneric;
        SweepArgs a{L->field, L->lh, (uint32_t)L->ly, (uint32_t)L->lz, L->vh, 0u, h0,
                    (uint32_t)L->seed, (uint32_t)(L->seed >> 32), L->chain, L->storage, kv, L->resolved_slab(v),
                    L->resolved_xcd(v), L->resolved_tile(v), tdev};
        const lattice::FusedGather& g = L->fg;
        // sample k's partials: buffer k & 1, the colour-0 then the colour-1 pairs
        auto part = [&](uint32_t k, uint32_t colour) { return g.d_part + ((size_t)(k & 1u) * 2 + colour) * 2 * g.blocks; };
        auto gather_lists = [&](uint32_t colour, uint32_t k) {  // gather the charged sites of `colour` for sample k
            a.g_off = g.d_off + (size_t)colour * (g.blocks + 1);
            a.g_key = g.d_key;
            a.g_Q = g.d_Q;
            a.g_S = g.d_S;
            a.g_part = part(k, colour);
            a.g_n = g.n;
            a.g_cap = g.cap;
        };
        if (fs && fs->finish) gather_lists(1u, fs->m);
        e = launch_halfsweep(a, stream);
        if (e == hipSuccess) {
            a.c = 1u;
            a.h = h0 + 1u;
            a.g_off = a.g_key = nullptr;
            a.g_Q = a.g_S = nullptr;
            a.g_part = nullptr;
            if (fs && fs->finish) {
                a.fin.part = part(fs->m, 0u);
                a.fin.n = 2 * g.blocks;
                a.fin.bins = L->d_bins;
                a.fin.m = fs->m;
                a.fin.bin_size = (uint32_t)L->bin_size;
                a.fin.mdev = fs->mdev;
                a.fin.last_xy = L->last_xy();
            }
            if (fs && fs->open) gather_lists(0u, fs->m + 1u);  // the next sample
            e = launch_halfsweep(a, stream);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    if (!tdev) L->t += 1;
    return LAT_OK;
}

int enqueue_sweep(lattice* L, const lattice::FusedStep* fs, bool c0_needed) {
    if (L->t >= (int64_t)0x7FFFFFFF) return set_error(LAT_ERR_STATE, "sweep counter exhausted (2^31 sweeps)");
    return enqueue_sweep_ex(L, L->stream, nullptr, 0, fs, c0_needed);
}

// The resident path: n_therm unmeasured sweeps then n_meas sweeps with a
// sample after every `every`-th, all in one launch.
int enqueue_resident(lattice* L, int64_t n_therm, int64_t n_meas, int64_t every) {
    if (n_therm + n_meas == 0) return LAT_OK;
    if (int r = settle_colour1(L)) return r;
    BatchArgs a{};
    a.field = L->field;
    a.site = L->d_site;
    a.Q = L->d_Q;
    a.S = L->d_S;
    a.bins = L->d_bins;
    a.t0 = (uint32_t)L->t;
    a.n_therm = (uint32_t)n_therm;
    a.n_meas = (uint32_t)n_meas;
    a.every = (uint32_t)every;
    a.bin_size = (uint32_t)(L->bin_size > 0 ? L->bin_size : 1);
    a.k0 = (uint32_t)L->seed;
    a.k1 = (uint32_t)(L->seed >> 32);
    a.storage = L->storage;
    a.single = true;
    a.last_xy = L->last_xy();
    BatchChainDesc& d = a.single_desc;
    d.field_off = 0;
    d.lh = L->lh;
    d.ly = (uint32_t)L->ly;
    d.lz = (uint32_t)L->lz;
    d.vh = L->vh;
    d.chain_id = L->chain;
    d.site_off = 0;
    d.n_sites = L->n_sites;
    d.bin_off = 0;
    d.meas0 = (uint32_t)L->n_meas;
    hipError_t e = launch_batch(a, L->stream);
    if (e != hipSuccess) return hip_fail(e, "resident sweep launch");
    L->t += n_therm + n_meas;
    L->n_meas += n_meas / every;
    return LAT_OK;
}

// One sample on `stream`.  Eager (mdev null): sample index L->n_meas, which
// is advanced.  Captured: index mdev[0] + rel on the device.
static int enqueue_measure_ex(lattice* L, hipStream_t stream, const uint32_t* mdev, uint32_t rel) {
    if (L->offl) {
        OffLatticeArgs o{L->field, L->c1cur(), (uint32_t)L->lx, (uint32_t)L->ly, (uint32_t)L->lz, L->d_r, L->d_qo,
                         L->n_off, L->d_partials, L->d_bins, mdev ? rel : (uint32_t)L->n_meas,
                         (uint32_t)L->bin_size, mdev, L->last_xy(), L->storage, L->meas_blocks,
                         (uint32_t)L->bin_cap, L->d_phit, L->d_fsum, L->d_fsq};
        hipError_t e = launch_measure_offlattice(o, stream);
        if (e != hipSuccess) return hip_fail(e, "off-lattice measure launch");
        if (!mdev) L->n_meas += 1;
        return LAT_OK;
    }
    MeasureArgs a{L->field, L->c1cur(), L->vh, L->d_site, L->d_Q, L->d_S, L->n_sites, L->d_partials,
                  L->d_bins, mdev ? rel : (uint32_t)L->n_meas, (uint32_t)L->bin_size, mdev, L->last_xy(),
                  L->storage, L->meas_blocks, L->d_set_off, L->n_sets, (uint32_t)L->bin_cap};
    hipError_t e = launch_measure(a, stream);
    if (e != hipSuccess) return hip_fail(e, "measure launch");
    if (!mdev) L->n_meas += 1;
    return LAT_OK;
}

static int enqueue_measure(lattice* L) { return enqueue_measure_ex(L, L->stream, nullptr, 0); }

// After blocked or fused sweeps colour 1 may sit in the second array (the
// kernels that alternate the two read and write it there): copy it home
// before a kernel that reads colour 1 at field + vh, and before graph
// replays, which are captured with colour 1 at home.
int settle_colour1(lattice* L) {
    if (!L->alt_current) return LAT_OK;
    hipError_t e = hipMemcpyAsync(L->c1main(), L->c1alt, (size_t)L->vh * L->esz, hipMemcpyDeviceToDevice, L->stream);
    if (e != hipSuccess) return hip_fail(e, "colour-1 copy");
    L->alt_current = false;
    return LAT_OK;
}

static void graph_reset(lattice::SweepGraph& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = lattice::SweepGraph();
}

void graphs_reset(lattice* L) {
    graph_reset(L->g_therm);
    graph_reset(L->g_meas);
}

// Sweeps per captured chunk, or 0 to run eagerly: a multiple of
// measure_every (every > 0), even (the fused kernel alternates colour-1
// arrays, so a chunk must end where it starts).
static int64_t graph_chunk(const lattice* L, int64_t every) {
    if (L->graph_mode == 0) return 0;
    const int v = L->effective_variant();
    if (v == LAT_SWEEP_RESIDENT) return 0;
    if (L->graph_mode == 1 && (uint64_t)L->vh * 2 > ((uint64_t)1 << 24)) return 0;
    int64_t K = 32;
    if (every > 0) {
        if (every > 256) return 0;
        K = (32 + every - 1) / every * every;
    }
    if (K % 2) K *= 2;
    return K;
}

static const void* graph_gather_key(const lattice* L, int64_t every) {
    return every > 0 && fused_gather_on(L) ? L->fg.d_off : nullptr;
}

static bool graph_matches(const lattice* L, const lattice::SweepGraph& g, int64_t K, int64_t every) {
    return g.exec && g.gather == graph_gather_key(L, every) && g.K == K && g.every == every &&
           g.variant == L->effective_variant() && g.slab == L->slab && g.tile == L->tile &&
           g.xcd == L->xcd_order && g.site == L->d_site &&
           (every == 0 || (g.bins == L->d_bins && g.bin_size == L->bin_size));
}

// Record K sweeps (and their samples) relative to the device counters,
// followed by a one-thread kernel that advances the counters: the graph is
// then replayed unchanged.  Kernels only (no memset or copy nodes).
static int graph_capture(lattice* L, lattice::SweepGraph& g, int64_t K, int64_t every) {
    graph_reset(g);
    hipError_t e = hipSuccess;
    if (!L->cap) e = hipStreamCreateWithFlags(&L->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    const bool alt0 = L->alt_current;
    e = hipStreamBeginCapture(L->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    int rc = LAT_OK;
    uint32_t m = 0;
    const bool fused = graph_gather_key(L, every) != nullptr;
    const bool blocked = L->effective_variant() == LAT_SWEEP_BLOCKED;
    bool open = false;  // fused: sample m - 1 awaits its colour-1 sites
    bool mp2 = false;   // blocked: the sweep before the previous one was sampled (sample kp2)
    uint32_t kp2 = 0;
    for (int64_t s = 0; s < K && rc == LAT_OK; ++s) {
        const bool measured = every > 0 && (s + 1) % every == 0;
        if (fused && blocked) {
            lattice::FusedStep fs;
            fs.finish = open;
            fs.open = measured;
            fs.m = m - 1u;
            fs.mdev = L->counters() + 1;
            fs.record = mp2;
            fs.m_rec = kp2;
            rc = enqueue_sweep_ex(L, L->cap, L->counters(), (uint32_t)s, &fs, s + 1 == K);
            mp2 = open;
            kp2 = m - 1u;
            open = measured;
            m += measured ? 1u : 0u;
        } else if (fused) {
            lattice::FusedStep fs;
            fs.finish = open;
            fs.open = measured;
            fs.m = m - 1u;
            fs.mdev = L->counters() + 1;
            rc = enqueue_sweep_ex(L, L->cap, L->counters(), (uint32_t)s, &fs);
            open = measured;
            m += measured ? 1u : 0u;
        } else {
            rc = enqueue_sweep_ex(L, L->cap, L->counters(), (uint32_t)s, nullptr, measured || s + 1 == K);
            if (rc == LAT_OK && measured) rc = enqueue_measure_ex(L, L->cap, L->counters() + 1, m++);
        }
    }
    if (rc == LAT_OK && fused && blocked && (open || mp2))
        rc = enqueue_blocked_tail(L, L->cap, mp2, kp2, open, m - 1u, L->counters() + 1);
    else if (rc == LAT_OK && open)
        rc = enqueue_fused_tail(L, L->cap, m - 1u, L->counters() + 1);
    if (rc == LAT_OK) {
        e = launch_advance_counters(L->counters(), (uint32_t)K, m, L->cap);
        if (e != hipSuccess) rc = hip_fail(e, "capture");
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(L->cap, &graph);
    L->alt_current = alt0;
    if (rc != LAT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ee != hipSuccess) return hip_fail(ee, "end capture");
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g.exec = nullptr;
        return hip_fail(e, "graph instantiation");
    }
    g.K = K;
    g.every = every;
    g.bin_size = L->bin_size;
    g.variant = L->effective_variant();
    g.slab = L->slab;
    g.tile = L->tile;
    g.xcd = L->xcd_order;
    g.bins = L->d_bins;
    g.site = L->d_site;
    g.gather = graph_gather_key(L, every);
    return LAT_OK;
}

// n sweeps with a sample after every `every`-th (every = 0: no samples):
// whole chunks as graph replays where that pays (not when eager), the rest
// launch by launch.
int run_sweeps(lattice* L, int64_t n, int64_t every, bool eager) {
    int64_t done = 0;
    const int64_t K = eager ? 0 : graph_chunk(L, every);
    const int v = L->effective_variant();
    if (L->alt_current && ((K > 0 && n >= K) || (v != LAT_SWEEP_BLOCKED && v != LAT_SWEEP_FUSED)))
        if (int r = settle_colour1(L)) return r;
    if (K > 0 && n >= K) {
        lattice::SweepGraph& g = every > 0 ? L->g_meas : L->g_therm;
        if (!graph_matches(L, g, K, every))
            if (int r = graph_capture(L, g, K, every)) return r;
        hipError_t e = launch_set_counters(L->counters(), (uint32_t)L->t, (uint32_t)L->n_meas, L->stream);
        const int64_t chunks = n / K;
        for (int64_t r = 0; r < chunks && e == hipSuccess; ++r) e = hipGraphLaunch(g.exec, L->stream);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
        done = chunks * K;
        L->t += done;
        if (every > 0) L->n_meas += done / every;
    }
    const bool fused = every > 0 && fused_gather_on(L);
    const bool blocked = L->effective_variant() == LAT_SWEEP_BLOCKED;
    bool open = false;  // fused: sample L->n_meas - 1 awaits its colour-1 sites
    bool mp2 = false;   // blocked: the sweep before the previous one was sampled (sample kp2)
    uint32_t kp2 = 0;
    for (int64_t s = done; s < n; ++s) {
        const bool measured = every > 0 && (s + 1) % every == 0;
        if (fused && blocked) {
            // colour-0 sites in this launch, colour-1 sites in the next, the
            // sample recorded in the one after; only the call's last sweep
            // stores colour 0
            lattice::FusedStep fs;
            fs.finish = open;
            fs.open = measured;
            fs.m = (uint32_t)(L->n_meas - 1);
            fs.record = mp2;
            fs.m_rec = kp2;
            if (int r = enqueue_sweep(L, &fs, s + 1 == n)) return r;
            mp2 = open;
            kp2 = (uint32_t)(L->n_meas - 1);
            open = measured;
            L->n_meas += measured ? 1 : 0;
        } else if (fused) {
            lattice::FusedStep fs;
            fs.finish = open;
            fs.open = measured;
            fs.m = (uint32_t)(L->n_meas - 1);
            if (int r = enqueue_sweep(L, &fs)) return r;
            open = measured;
            L->n_meas += measured ? 1 : 0;
        } else {
            // a sweep that keeps colour 0 on chip stores it for a sample read
            // from memory and at the end of the call
            if (int r = enqueue_sweep(L, nullptr, measured || s + 1 == n)) return r;
            if (measured)
                if (int r = enqueue_measure(L)) return r;
        }
    }
    if (fused && blocked) {
        if (open || mp2)
            if (int r = enqueue_blocked_tail(L, L->stream, mp2, kp2, open, (uint32_t)(L->n_meas - 1), nullptr))
                return r;
    } else if (open) {
        if (int r = enqueue_fused_tail(L, L->stream, (uint32_t)(L->n_meas - 1), nullptr)) return r;
    }
    return LAT_OK;
}

// Bin arrays of every charge set, each with room for n_bins_needed bins
// (grown geometrically; each set's bins keep their place in its array).
int ensure_bins(lattice* L, int64_t n_bins_needed) {
    if (n_bins_needed <= L->bin_cap) return LAT_OK;
    int64_t cap = std::max<int64_t>({n_bins_needed, 2 * L->bin_cap, 64});
    const size_t pitch = sizeof(double) * 2 * (size_t)cap;
    double* nb = static_cast<double*>(L->mem.alloc(pitch * L->n_sets));
    if (!nb) return set_error(LAT_ERR_ALLOC, "allocation of sample bins failed");
    hipError_t e = hipMemsetAsync(nb, 0, pitch * L->n_sets, L->stream);
    if (e == hipSuccess && L->d_bins && L->bin_cap > 0) {
        const size_t old_pitch = sizeof(double) * 2 * (size_t)L->bin_cap;
        e = hipMemcpy2DAsync(nb, pitch, L->d_bins, old_pitch, old_pitch, L->n_sets, hipMemcpyDeviceToDevice,
                             L->stream);
    }
    if (e != hipSuccess) {
        L->mem.release(nb);
        return hip_fail(e, "bin resize");
    }
    if (L->d_bins) L->mem.release(L->d_bins);
    L->d_bins = nb;
    L->bin_cap = cap;
    return LAT_OK;
}

}  // namespace latcoul

extern "C" {

int lattice_create(int64_t lx, int64_t ly, int64_t lz, int storage, uint64_t seed, uint32_t chain_id,
                   const lat_allocator* alloc, void* hip_stream, lattice_t** out) {
    if (!out) return set_error(LAT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (lx < 2 || (lx & 1)) return set_error(LAT_ERR_ARG, "lx must be even and >= 2");
    if (ly < 1 || lz < 1) return set_error(LAT_ERR_ARG, "ly and lz must be >= 1");
    if ((double)lx * (double)ly * (double)lz >= 2147483648.0)
        return set_error(LAT_ERR_ARG, "lattice must have fewer than 2^31 sites");
    if (storage < LAT_FP32 || storage > LAT_FP16_SR) return set_error(LAT_ERR_ARG, "unknown storage format");
    if (alloc && (!alloc->alloc || !alloc->release))
        return set_error(LAT_ERR_ARG, "allocator needs both alloc and release");
    lattice* L = new lattice();
    L->lx = lx;
    L->ly = ly;
    L->lz = lz;
    L->lh = (uint32_t)(lx / 2);
    L->vh = (uint32_t)(lx / 2 * ly * lz);
    L->storage = storage;
    L->esz = storage == LAT_FP32 ? 4 : 2;
    L->seed = seed;
    L->chain = chain_id;
    L->mem = DeviceAllocator(alloc);
    L->stream = static_cast<hipStream_t>(hip_stream);
    int ncu = 0;
    hipError_t de = hipGetDevice(&L->device);
    if (de == hipSuccess) de = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, L->device);
    if (de != hipSuccess) {
        delete L;
        return hip_fail(de, "current device");
    }
    if (ncu > 0) L->cus = (uint32_t)ncu;
    const size_t fbytes = round_up(2 * (size_t)L->vh * L->esz, 256);
    L->field = L->mem.alloc(fbytes);
    L->d_misc = L->mem.alloc(256);
    if (!L->field || !L->d_misc) {
        lattice_destroy(L);
        return set_error(LAT_ERR_ALLOC, "allocation of the field failed");
    }
    hipError_t e = hipMemsetAsync(L->field, 0, fbytes, L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L->d_misc, 0, 256, L->stream);
    if (e != hipSuccess) {
        lattice_destroy(L);
        return hip_fail(e, "field initialisation");
    }
    // FP32 boxes beyond the last-level cache: the library's choice is the
    // blocked sweep, which needs a second colour-1 array (without it, the
    // streaming sweep)
    const size_t cbytes = (size_t)L->vh * L->esz;
    if (L->esz == 4 && L->lh % 4 == 0 && 2 * cbytes >= ((size_t)256 << 20) && cbytes < ((size_t)1 << 31) &&
        L->blocked_rows() != 0) {
        L->c1alt = L->mem.alloc(round_up(cbytes, 256));
        if (L->c1alt && prepare_blocked_sweep() == hipSuccess) {
            L->auto_blocked = true;
        } else {
            (void)hipGetLastError();
            L->mem.release(L->c1alt);
            L->c1alt = nullptr;
        }
    }
    *out = L;
    return LAT_OK;
}

void lattice_destroy(lattice_t* L) {
    if (!L) return;
    (void)hipStreamSynchronize(L->stream);
    graphs_reset(L);
    if (L->cap) (void)hipStreamDestroy(L->cap);
    L->mem.release(L->field);
    L->mem.release(L->c1alt);
    L->mem.release(L->d_misc);
    L->mem.release(L->d_site);
    L->mem.release(L->d_Q);
    L->mem.release(L->d_S);
    L->mem.release(L->d_partials);
    L->mem.release(L->d_set_off);
    L->mem.release(L->d_lastxy);
    L->mem.release(L->d_r);
    L->mem.release(L->d_qo);
    L->mem.release(L->d_phit);
    L->mem.release(L->d_fsum);
    L->mem.release(L->d_fsq);
    fused_gather_release(L);
    L->mem.release(L->d_bins);
    delete L;
}

// Tile configurations the variant's kernel has; for the other variants (the
// library's choice among them included) a tile every slab kernel has.
static uint32_t tiles_of(int variant) {
    if (variant == LAT_SWEEP_BLOCKED) return 65;  // rows per tile, 1 .. 64
    if (variant == LAT_SWEEP_ZSLAB) return kZslabTiles;
    if (variant == LAT_SWEEP_STREAM) return kStreamTiles;
    return (uint32_t)std::min(kZslabTiles, kStreamTiles);
}

int lattice_sweep_count(const lattice_t* L, int64_t* sweeps) {
    if (int r = check_lattice(L)) return r;
    if (!sweeps) return set_error(LAT_ERR_ARG, "sweeps is NULL");
    *sweeps = L->t;
    return LAT_OK;
}

int lattice_set_variant(lattice_t* L, int variant) {
    if (int r = check_lattice(L)) return r;
    switch (variant) {
        case LAT_SWEEP_AUTO:  // may pick a slab kernel, which uses the tile
            if (L->tile != kTileDefault && L->tile >= tiles_of(variant))
                return set_error(LAT_ERR_ARG, "the selected tile configuration does not exist for every slab kernel");
            break;
        case LAT_SWEEP_GENERIC: break;
        case LAT_SWEEP_RESIDENT:
            if (L->n_sets > 1) return set_error(LAT_ERR_ARG, "the resident kernel measures one charge set");
            if (L->offl) return set_error(LAT_ERR_ARG, "the resident kernel measures on-lattice charges only");
            break;
        case LAT_SWEEP_QUAD:
            if (L->lh % 4) return set_error(LAT_ERR_ARG, "this sweep kernel needs lx % 8 == 0");
            break;
        case LAT_SWEEP_ZSLAB:
        case LAT_SWEEP_STREAM:
            if (L->lh % 4) return set_error(LAT_ERR_ARG, "this sweep kernel needs lx % 8 == 0");
            if ((size_t)L->vh * L->esz >= ((size_t)1 << 31))
                return set_error(LAT_ERR_ARG, "slab kernel needs each colour array below 2 GiB");
            if (L->tile != kTileDefault && L->tile >= tiles_of(variant))
                return set_error(LAT_ERR_ARG, "the selected tile configuration does not exist for this kernel");
            break;
        case LAT_SWEEP_BLOCKED: {
            if (L->lh % 4) return set_error(LAT_ERR_ARG, "this sweep kernel needs lx % 8 == 0");
            if ((size_t)L->vh * L->esz >= ((size_t)1 << 31))
                return set_error(LAT_ERR_ARG, "the blocked sweep needs each colour array below 2 GiB");
            const uint32_t keep = L->tile;
            if (L->tile == 0 || (L->tile != kTileDefault && L->tile > 64)) L->tile = kTileDefault;
            const bool fits = L->blocked_rows() != 0;
            L->tile = keep;
            if (!fits)
                return set_error(LAT_ERR_ARG, "the blocked sweep needs rows of whole 16-byte chunks that fit in LDS "
                                              "(16-bit storage: lx % 16 == 0)");
            if (!L->c1alt) {
                L->c1alt = L->mem.alloc(round_up((size_t)L->vh * L->esz, 256));
                if (!L->c1alt) return set_error(LAT_ERR_ALLOC, "allocation of the second colour-1 array failed");
            }
            if (hipError_t e = prepare_blocked_sweep()) return hip_fail(e, "blocked sweep set-up");
            break;
        }
        case LAT_SWEEP_FUSED:
            if (L->lh % 4) return set_error(LAT_ERR_ARG, "fused sweep needs lx % 8 == 0");
            if (!fused_sweep_supported(L->lh, (uint32_t)L->ly))
                return set_error(LAT_ERR_ARG, "fused sweep needs 64 <= lx <= 1024 (full rows staged in LDS)");
            if (!L->c1alt) {
                L->c1alt = L->mem.alloc(round_up((size_t)L->vh * L->esz, 256));
                if (!L->c1alt) return set_error(LAT_ERR_ALLOC, "allocation of the second colour-1 array failed");
            }
            if (hipError_t e = prepare_fused_sweep()) return hip_fail(e, "fused sweep set-up");
            break;
        default: return set_error(LAT_ERR_ARG, "unknown sweep variant");
    }
    L->variant = variant;
    graphs_reset(L);
    return LAT_OK;
}

int lattice_get_tuning(const lattice_t* L, int* variant, int64_t* planes, int* tile, int* xcd_order) {
    if (int r = check_lattice(L)) return r;
    const int v = L->effective_variant();
    if (variant) *variant = v;
    if (planes) *planes = L->resolved_slab(v);
    if (tile) *tile = (int)L->resolved_tile(v);
    if (xcd_order) *xcd_order = (int)L->resolved_xcd(v);
    return LAT_OK;
}

int lattice_get_sample_path(const lattice_t* L, int* fused) {
    if (int r = check_lattice(L)) return r;
    if (fused) *fused = L->fg.last ? 1 : 0;
    return LAT_OK;
}

int lattice_get_gather_parts(const lattice_t* L, int* parts, int* part_entries) {
    if (int r = check_lattice(L)) return r;
    const bool on = latcoul::fused_gather_on(L) && L->fg.variant == LAT_SWEEP_BLOCKED;
    if (parts) *parts = on ? (int)L->fg.parts : 0;
    if (part_entries) *part_entries = on ? (int)L->fg.cap : 0;
    return LAT_OK;
}

int lattice_use_graphs(lattice_t* L, int mode) {
    if (int r = check_lattice(L)) return r;
    if (mode < 0 || mode > 2) return set_error(LAT_ERR_ARG, "graph mode must be 0, 1 or 2");
    L->graph_mode = mode;
    graphs_reset(L);
    return LAT_OK;
}

int lattice_set_tuning(lattice_t* L, int64_t planes, int tile, int xcd_order) {
    if (int r = check_lattice(L)) return r;
    if (planes < 0 || planes > L->lz) return set_error(LAT_ERR_ARG, "planes must be in [0, lz]");
    if (xcd_order > 2) return set_error(LAT_ERR_ARG, "xcd_order must be -1, 0, 1 or 2");
    if (tile < -1 || (tile >= 0 && (uint32_t)tile >= tiles_of(L->variant)))
        return set_error(LAT_ERR_ARG, "unknown tile configuration for the selected sweep kernel");
    if (L->variant == LAT_SWEEP_BLOCKED && tile >= 0) {
        BlockedShape sh;
        if (!blocked_geometry(L->lh, (uint32_t)L->esz, (uint32_t)tile, 4u, &sh))
            return set_error(LAT_ERR_ARG, "these rows per tile do not fit the blocked sweep's LDS");
    }
    L->slab = (uint32_t)planes;
    L->tile = tile < 0 ? kTileDefault : (uint32_t)tile;
    L->xcd_order = xcd_order < 0 ? -1 : xcd_order;
    graphs_reset(L);
    return LAT_OK;
}

static void release_offlattice(lattice* L) {
    L->mem.release(L->d_r);
    L->mem.release(L->d_qo);
    L->mem.release(L->d_phit);
    L->mem.release(L->d_fsum);
    L->mem.release(L->d_fsq);
    L->d_r = L->d_qo = L->d_phit = L->d_fsum = L->d_fsq = nullptr;
    L->offl = false;
    L->n_off = 0;
    L->force_base = 0;
    L->off_order.reset();
}

int lattice_set_charge_sets(lattice_t* L, int64_t n_sets, const int64_t* counts, const int32_t* xyz,
                            const double* q) {
    TraceRange tr("set_charges");
    if (int r = check_lattice(L)) return r;
    if (n_sets < 1 || n_sets > kMaxChargeSets) return set_error(LAT_ERR_ARG, "n_sets must be in [1, 65535]");
    if (!counts) return set_error(LAT_ERR_ARG, "counts is NULL");
    if (n_sets > 1 && L->variant == LAT_SWEEP_RESIDENT)
        return set_error(LAT_ERR_ARG, "the resident kernel measures one charge set");
    int64_t n = 0;
    for (int64_t k = 0; k < n_sets; ++k) {
        if (counts[k] < 0) return set_error(LAT_ERR_ARG, "negative charge count");
        n += counts[k];
    }
    if (n > 0 && (!xyz || !q)) return set_error(LAT_ERR_ARG, "xyz or q is NULL");
    // aggregate each set, concatenate
    AggregatedCharges all;
    std::vector<uint32_t> off(1, 0u);
    uint32_t max_ns = 0;
    int64_t first = 0;
    for (int64_t k = 0; k < n_sets; ++k) {
        AggregatedCharges agg;
        if (int r = aggregate_charges(counts[k], xyz ? xyz + 3 * first : nullptr, q ? q + first : nullptr, L->lx,
                                      L->ly, L->lz, L->vh, &agg))
            return r;
        first += counts[k];
        if (all.site.size() + agg.site.size() >= (size_t)0xFFFFFFFFu)
            return set_error(LAT_ERR_ARG, "too many charged sites");
        all.site.insert(all.site.end(), agg.site.begin(), agg.site.end());
        all.Q.insert(all.Q.end(), agg.Q.begin(), agg.Q.end());
        all.S.insert(all.S.end(), agg.S.begin(), agg.S.end());
        off.push_back((uint32_t)all.site.size());
        max_ns = std::max(max_ns, (uint32_t)agg.site.size());
    }
    const uint32_t ns = (uint32_t)all.site.size();
    const uint32_t blocks = measure_blocks(max_ns);
    const size_t cap = std::max<size_t>(ns, 1);
    uint32_t* d_site = static_cast<uint32_t*>(L->mem.alloc(cap * 4));
    double* d_Q = static_cast<double*>(L->mem.alloc(cap * 8));
    double* d_S = static_cast<double*>(L->mem.alloc(cap * 8));
    double* d_part = static_cast<double*>(L->mem.alloc((size_t)blocks * n_sets * 16));
    uint32_t* d_off = static_cast<uint32_t*>(L->mem.alloc(off.size() * 4));
    double* d_xy = static_cast<double*>(L->mem.alloc((size_t)n_sets * 16));
    auto release_new = [&] {
        L->mem.release(d_site);
        L->mem.release(d_Q);
        L->mem.release(d_S);
        L->mem.release(d_part);
        L->mem.release(d_off);
        L->mem.release(d_xy);
    };
    if (!d_site || !d_Q || !d_S || !d_part || !d_off || !d_xy) {
        release_new();
        return set_error(LAT_ERR_ALLOC, "allocation of the charge list failed");
    }
    hipError_t e = hipSuccess;
    if (ns > 0) {
        e = hipMemcpyAsync(d_site, all.site.data(), (size_t)ns * 4, hipMemcpyHostToDevice, L->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_Q, all.Q.data(), (size_t)ns * 8, hipMemcpyHostToDevice, L->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_S, all.S.data(), (size_t)ns * 8, hipMemcpyHostToDevice, L->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_xy, 0, (size_t)n_sets * 16, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) {
        release_new();
        return hip_fail(e, "charge upload");
    }
    L->mem.release(L->d_site);
    L->mem.release(L->d_Q);
    L->mem.release(L->d_S);
    L->mem.release(L->d_partials);
    L->mem.release(L->d_set_off);
    L->mem.release(L->d_lastxy);
    graphs_reset(L);
    L->d_site = d_site;
    L->d_Q = d_Q;
    L->d_S = d_S;
    L->d_partials = d_part;
    L->d_set_off = d_off;
    L->d_lastxy = d_xy;
    release_offlattice(L);
    fused_gather_release(L);
    if (n_sets <= (int64_t)kBlockedMaxSets) {  // kept for the fused gather's lists
        auto hc = std::make_shared<lattice::HostCharges>();
        hc->site.swap(all.site);
        hc->Q.swap(all.Q);
        hc->S.swap(all.S);
        hc->set_off.swap(off);
        L->host_charges = std::move(hc);
    } else {
        L->host_charges.reset();
    }
    L->n_sites = ns;
    L->n_raw = n;
    L->meas_blocks = blocks;
    // new observables: start new sample series (bin arrays sized per set)
    L->n_meas = 0;
    L->bin_size = 0;
    if (L->n_sets != (uint32_t)n_sets) {
        L->mem.release(L->d_bins);
        L->d_bins = nullptr;
        L->bin_cap = 0;
        L->n_sets = (uint32_t)n_sets;
    } else if (L->d_bins) {
        e = hipMemsetAsync(L->d_bins, 0, sizeof(double) * 2 * (size_t)L->bin_cap * L->n_sets, L->stream);
        if (e != hipSuccess) return hip_fail(e, "bin reset");
    }
    // the fused gather's per-tile lists for the current tiling, built here
    // where the host waits anyway, so that later calls only enqueue (the
    // GPU then runs thermalisation and measured sweeps back to back); a
    // later change of kernel or tiling rebuilds them at the next measured call
    return fused_gather_prepare(L);
}

int set_charges(lattice_t* L, int64_t n, const int32_t* xyz, const double* q) {
    if (int r = check_lattice(L)) return r;
    if (n < 0) return set_error(LAT_ERR_ARG, "negative charge count");
    return lattice_set_charge_sets(L, 1, &n, xyz, q);
}

int thermalise(lattice_t* L, int64_t n_sweeps) {
    TraceRange tr("thermalise");
    if (int r = check_lattice(L)) return r;
    if (n_sweeps < 0) return set_error(LAT_ERR_ARG, "n_sweeps < 0");
    if (L->t + n_sweeps > (int64_t)0x7FFFFFFF) return set_error(LAT_ERR_ARG, "sweep counter would exceed 2^31");
    if (L->effective_variant() == LAT_SWEEP_RESIDENT) return enqueue_resident(L, n_sweeps, 0, 1);
    return run_sweeps(L, n_sweeps, 0);
}

int sweep_and_measure(lattice_t* L, int64_t n_sweeps, int64_t measure_every, int64_t bin_size) {
    TraceRange tr("sweep_and_measure");
    if (int r = check_lattice(L)) return r;
    if (n_sweeps < 0) return set_error(LAT_ERR_ARG, "n_sweeps < 0");
    if (measure_every < 1) return set_error(LAT_ERR_ARG, "measure_every < 1");
    if (bin_size < 1) return set_error(LAT_ERR_ARG, "bin_size < 1");
    if (L->bin_size != 0 && bin_size != L->bin_size)
        return set_error(LAT_ERR_ARG, "bin_size differs from the one of earlier samples");
    if (L->t + n_sweeps > (int64_t)0x7FFFFFFF) return set_error(LAT_ERR_ARG, "sweep counter would exceed 2^31");
    if (!L->d_partials) {
        // no set_charges yet: an empty charge list
        if (int r = set_charges(L, 0, nullptr, nullptr)) return r;
    }
    const int64_t m = n_sweeps / measure_every;
    const int64_t total = L->n_meas + m;
    if ((total + bin_size - 1) / bin_size >= (int64_t)0xFFFFFFFF)
        return set_error(LAT_ERR_ARG, "too many bins");
    if (int r = ensure_bins(L, (total + bin_size - 1) / bin_size)) return r;
    L->bin_size = bin_size;
    if (L->effective_variant() == LAT_SWEEP_RESIDENT) {
        L->fg.last = false;
        return enqueue_resident(L, 0, n_sweeps, measure_every);
    }
    if (int r = fused_gather_prepare(L)) return r;
    L->fg.last = fused_gather_on(L);
    return run_sweeps(L, n_sweeps, measure_every);
}

int lattice_energy_estimate_set(lattice_t* L, int64_t set, double* mean, double* stderr_binned,
                                int64_t* n_samples, int64_t* n_bins) {
    TraceRange tr("energy_estimate");
    if (int r = check_lattice(L)) return r;
    if (set < 0 || set >= (int64_t)L->n_sets) return set_error(LAT_ERR_ARG, "no such charge set");
    const int64_t M = L->n_meas;
    const int64_t B = L->bin_size > 0 ? L->bin_size : 1;
    const int64_t used = std::min<int64_t>((M + B - 1) / B, L->bin_cap);
    std::vector<double> h((size_t)std::max<int64_t>(used, 1) * 2, 0.0);
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess && used > 0)
        e = hipMemcpy(h.data(), L->d_bins + 2 * (size_t)set * L->bin_cap, sizeof(double) * 2 * (size_t)used,
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "bin readback");
    EstimateResult res = estimate_from_bins(h.data(), used, M, B);
    if (mean) *mean = res.mean;
    if (stderr_binned) *stderr_binned = res.stderr_binned;
    if (n_samples) *n_samples = M;
    if (n_bins) *n_bins = res.full_bins;
    if (!res.finite) return set_error(LAT_ERR_STATE, "non-finite sample found (field or charges not finite)");
    if (res.full_bins < 2) return set_error(LAT_ERR_STATE, "fewer than 2 full bins: no error estimate");
    return LAT_OK;
}

int energy_estimate(lattice_t* L, double* mean, double* stderr_binned, int64_t* n_samples, int64_t* n_bins) {
    return lattice_energy_estimate_set(L, 0, mean, stderr_binned, n_samples, n_bins);
}

int lattice_set_offlattice_charges(lattice_t* L, int64_t n, const double* r, const double* q, int forces) {
    TraceRange tr("set_offlattice_charges");
    if (int r_ = check_lattice(L)) return r_;
    if (n < 0 || n >= (int64_t)0xFFFFFFFF) return set_error(LAT_ERR_ARG, "bad charge count");
    if (n > 0 && (!r || !q)) return set_error(LAT_ERR_ARG, "r or q is NULL");
    if (L->lx < 2 || L->ly < 2 || L->lz < 2)
        return set_error(LAT_ERR_ARG, "off-lattice charges need every box edge >= 2");
    if (L->variant == LAT_SWEEP_RESIDENT)
        return set_error(LAT_ERR_ARG, "the resident kernel measures on-lattice charges only");
    const double hi[3] = {(double)(L->lx - 1), (double)(L->ly - 1), (double)(L->lz - 1)};
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(q[i])) return set_error(LAT_ERR_ARG, "non-finite charge");
        for (int d = 0; d < 3; ++d) {
            const double v = r[3 * i + d];
            if (!std::isfinite(v) || v < 0.0 || v > hi[d])
                return set_error(LAT_ERR_ARG, "position outside [0, L - 1] on some axis");
        }
    }
    // order by cell (z, then y, then x of the cell origin), ties by input order
    auto order = std::make_shared<std::vector<uint32_t>>((size_t)n);
    std::vector<uint64_t> cell((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t b[3];
        for (int d = 0; d < 3; ++d) b[d] = (uint64_t)std::min(std::floor(r[3 * i + d]), hi[d] - 1.0);
        cell[(size_t)i] = (b[2] * (uint64_t)L->ly + b[1]) * (uint64_t)L->lx + b[0];
        (*order)[(size_t)i] = (uint32_t)i;
    }
    std::stable_sort(order->begin(), order->end(), [&](uint32_t a, uint32_t b) { return cell[a] < cell[b]; });
    std::vector<double> rs((size_t)n * 3), qs((size_t)n);
    for (size_t k = 0; k < (size_t)n; ++k) {
        const uint32_t i = (*order)[k];
        for (int d = 0; d < 3; ++d) rs[3 * k + d] = r[3 * (size_t)i + d];
        qs[k] = q[i];
    }
    const size_t cap = (size_t)std::max<int64_t>(n, 1);
    const uint32_t blocks = measure_blocks((uint32_t)n);
    double* d_r = static_cast<double*>(L->mem.alloc(cap * 24));
    double* d_q = static_cast<double*>(L->mem.alloc(cap * 8));
    double* d_part = static_cast<double*>(L->mem.alloc((size_t)blocks * 16));
    double* d_xy = static_cast<double*>(L->mem.alloc(16));
    double *d_phit = nullptr, *d_fsum = nullptr, *d_fsq = nullptr;
    if (forces) {
        d_phit = static_cast<double*>(L->mem.alloc(cap * 32));
        d_fsum = static_cast<double*>(L->mem.alloc(cap * 24));
        d_fsq = static_cast<double*>(L->mem.alloc(cap * 24));
    }
    auto release_new = [&] {
        L->mem.release(d_r);
        L->mem.release(d_q);
        L->mem.release(d_part);
        L->mem.release(d_xy);
        L->mem.release(d_phit);
        L->mem.release(d_fsum);
        L->mem.release(d_fsq);
    };
    if (!d_r || !d_q || !d_part || !d_xy || (forces && (!d_phit || !d_fsum || !d_fsq))) {
        release_new();
        return set_error(LAT_ERR_ALLOC, "allocation of the off-lattice charge list failed");
    }
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = hipMemcpyAsync(d_r, rs.data(), (size_t)n * 24, hipMemcpyHostToDevice, L->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(d_q, qs.data(), (size_t)n * 8, hipMemcpyHostToDevice, L->stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(d_xy, 0, 16, L->stream);
    if (e == hipSuccess && forces) e = hipMemsetAsync(d_fsum, 0, cap * 24, L->stream);
    if (e == hipSuccess && forces) e = hipMemsetAsync(d_fsq, 0, cap * 24, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) {
        release_new();
        return hip_fail(e, "off-lattice charge upload");
    }
    // replace every charge set by this one off-lattice set
    L->mem.release(L->d_site);
    L->mem.release(L->d_Q);
    L->mem.release(L->d_S);
    L->mem.release(L->d_partials);
    L->mem.release(L->d_set_off);
    L->mem.release(L->d_lastxy);
    L->d_site = nullptr;
    L->d_Q = L->d_S = nullptr;
    L->d_set_off = nullptr;
    release_offlattice(L);
    fused_gather_release(L);
    L->host_charges.reset();
    graphs_reset(L);
    L->d_partials = d_part;
    L->d_lastxy = d_xy;
    L->d_r = d_r;
    L->d_qo = d_q;
    L->d_phit = d_phit;
    L->d_fsum = d_fsum;
    L->d_fsq = d_fsq;
    L->offl = true;
    L->n_off = (uint32_t)n;
    L->off_order = std::move(order);
    L->n_sites = 0;
    L->n_raw = n;
    L->meas_blocks = blocks;
    L->n_meas = 0;
    L->bin_size = 0;
    L->force_base = 0;
    if (L->n_sets != 1) {
        L->mem.release(L->d_bins);
        L->d_bins = nullptr;
        L->bin_cap = 0;
        L->n_sets = 1;
    } else if (L->d_bins) {
        e = hipMemsetAsync(L->d_bins, 0, sizeof(double) * 2 * (size_t)L->bin_cap, L->stream);
        if (e != hipSuccess) return hip_fail(e, "bin reset");
    }
    return LAT_OK;
}

int lattice_force_estimate(lattice_t* L, double* dE_dr, double* stderr_naive, int64_t* n_samples) {
    if (int r_ = check_lattice(L)) return r_;
    if (!L->offl || !L->d_fsum) return set_error(LAT_ERR_STATE, "no off-lattice charges with forces");
    const int64_t M = L->n_meas - L->force_base;
    if (n_samples) *n_samples = M;
    const size_t k = (size_t)L->n_off * 3;
    std::vector<double> s(std::max<size_t>(k, 1)), s2(std::max<size_t>(k, 1));
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess && k > 0) e = hipMemcpy(s.data(), L->d_fsum, k * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && k > 0) e = hipMemcpy(s2.data(), L->d_fsq, k * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "force readback");
    if (M < 2) return set_error(LAT_ERR_STATE, "fewer than 2 force samples");
    for (size_t i = 0; i < k; ++i) {
        const size_t o = 3 * (size_t)(*L->off_order)[i / 3] + i % 3;  // the caller's order
        const double mean = s[i] / (double)M;
        if (dE_dr) dE_dr[o] = mean;
        if (stderr_naive) {
            const double var = std::max(0.0, (s2[i] - (double)M * mean * mean) / (double)(M - 1));
            stderr_naive[o] = std::sqrt(var / (double)M);
        }
    }
    return LAT_OK;
}

int lattice_get_field(lattice_t* L, float* host_out) {
    if (int r = check_lattice(L)) return r;
    if (!host_out) return set_error(LAT_ERR_ARG, "host_out is NULL");
    const size_t half = (size_t)L->vh * L->esz;
    std::vector<unsigned char> buf(2 * half);
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess) e = hipMemcpy(buf.data(), L->field, half, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + half, L->c1cur(), half, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "field readback");
    compact_to_natural(buf.data(), L->storage, L->lx, L->ly, L->lz, L->vh, host_out);
    return LAT_OK;
}

int lattice_set_field(lattice_t* L, const float* host_in) {
    if (int r = check_lattice(L)) return r;
    if (!host_in) return set_error(LAT_ERR_ARG, "host_in is NULL");
    const size_t V = (size_t)L->lx * L->ly * L->lz;
    for (size_t i = 0; i < V; ++i)
        if (!std::isfinite(host_in[i])) return set_error(LAT_ERR_ARG, "non-finite field value");
    std::vector<unsigned char> buf(2 * (size_t)L->vh * L->esz);
    natural_to_compact(host_in, L->storage, L->lx, L->ly, L->lz, L->vh, buf.data());
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess) e = hipMemcpy(L->field, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "field upload");
    L->alt_current = false;  // both colours now at home
    return LAT_OK;
}

int lattice_last_measure(lattice_t* L, double* X, double* Y) {
    if (int r = check_lattice(L)) return r;
    double h[2] = {0, 0};
    hipError_t e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess) e = hipMemcpy(h, L->last_xy(), 16, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "readback");
    if (X) *X = h[0];
    if (Y) *Y = h[1];
    return LAT_OK;
}

int lattice_get_state(lattice_t* L, int64_t* sweep_counter, int64_t* n_samples, double* bins_host, int64_t cap,
                      int64_t* n_bins) {
    if (int r = check_lattice(L)) return r;
    const int64_t B = L->bin_size > 0 ? L->bin_size : 1;
    const int64_t used = (L->n_meas + B - 1) / B;
    if (sweep_counter) *sweep_counter = L->t;
    if (n_samples) *n_samples = L->n_meas;
    if (n_bins) *n_bins = used;
    hipError_t e = hipStreamSynchronize(L->stream);
    // set-major: the `used` bins of set 0, then of set 1, ...; at most cap pairs
    for (int64_t k = 0; k < (int64_t)L->n_sets && e == hipSuccess && bins_host; ++k) {
        const int64_t room = std::min(used, cap - k * used);
        if (room <= 0) break;
        e = hipMemcpy(bins_host + 2 * k * used, L->d_bins + 2 * (size_t)k * L->bin_cap,
                      sizeof(double) * 2 * (size_t)room, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return hip_fail(e, "state readback");
    return LAT_OK;
}

int lattice_set_state(lattice_t* L, int64_t sweep_counter, int64_t n_samples, int64_t bin_size,
                      const double* bins_host, int64_t n_bins) {
    if (int r = check_lattice(L)) return r;
    if (sweep_counter < 0 || sweep_counter > (int64_t)0x7FFFFFFF) return set_error(LAT_ERR_ARG, "bad sweep counter");
    if (n_samples < 0 || (n_samples > 0 && bin_size < 1)) return set_error(LAT_ERR_ARG, "bad sample count or bin size");
    const int64_t B = bin_size > 0 ? bin_size : 1;
    const int64_t used = (n_samples + B - 1) / B;
    if (n_bins != used || (used > 0 && !bins_host)) return set_error(LAT_ERR_ARG, "bins do not match n_samples/bin_size");
    if (!L->d_partials)
        if (int r = set_charges(L, 0, nullptr, nullptr)) return r;
    if (int r = ensure_bins(L, std::max<int64_t>(used, 1))) return r;
    hipError_t e = hipMemsetAsync(L->d_bins, 0, sizeof(double) * 2 * (size_t)L->bin_cap * L->n_sets, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    // set-major, as lattice_get_state writes them
    for (int64_t k = 0; k < (int64_t)L->n_sets && e == hipSuccess && used > 0; ++k)
        e = hipMemcpy(L->d_bins + 2 * (size_t)k * L->bin_cap, bins_host + 2 * k * used,
                      sizeof(double) * 2 * (size_t)used, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "state upload");
    L->t = sweep_counter;
    L->n_meas = n_samples;
    L->bin_size = n_samples > 0 ? bin_size : 0;
    if (L->d_fsum) {  // force sums are not part of a checkpoint: restart them
        e = hipMemsetAsync(L->d_fsum, 0, (size_t)L->n_off * 24, L->stream);
        if (e == hipSuccess) e = hipMemsetAsync(L->d_fsq, 0, (size_t)L->n_off * 24, L->stream);
        if (e != hipSuccess) return hip_fail(e, "force reset");
        L->force_base = n_samples;
    }
    return LAT_OK;
}

}  // extern "C"
