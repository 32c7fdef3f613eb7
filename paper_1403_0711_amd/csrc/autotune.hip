// The autotuner: times every sweep kernel and tuning that can handle a box
// on scratch memory and keeps the fastest.  Choices are cached per (device
// architecture, box, storage, whether the single-workgroup kernel may run)
// for the process, and, when LATCOUL_TUNE_CACHE names a file, in that file
// across processes (one line per choice, appended).

#include "lattice_impl.hpp"

#include <cstdio>
#include <cstdlib>

struct TuneChoice {
    int variant;
    uint32_t slab, tile, xcd;
    double ms;
};
using TuneKey = std::tuple<std::string, int64_t, int64_t, int64_t, int, int>;
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune_cache;
static bool g_tune_file_read = false;

// Whether a choice (from the file, so possibly from another build) names a
// kernel and tuning this library has for the box.
static bool choice_valid(const lattice* L, const TuneChoice& c, bool resident_ok) {
    StreamTileShape sh;
    if (c.xcd > 2 || c.slab > (uint64_t)L->lz || !(c.ms >= 0.0)) return false;
    switch (c.variant) {
        case LAT_SWEEP_GENERIC: return true;
        case LAT_SWEEP_QUAD: return L->lh % 4 == 0;
        case LAT_SWEEP_RESIDENT: return resident_ok && (uint64_t)L->vh * 2 <= ((uint64_t)1 << 18);
        case LAT_SWEEP_ZSLAB: return L->lh % 4 == 0 && c.tile < (uint32_t)kZslabTiles;
        case LAT_SWEEP_STREAM: return L->lh % 4 == 0 && stream_tile_geometry(c.tile, L->esz, &sh);
        case LAT_SWEEP_FUSED: return L->lh % 4 == 0 && fused_sweep_supported(L->lh, (uint32_t)L->ly);
        case LAT_SWEEP_BLOCKED: {
            BlockedShape bs;
            return L->lh % 4 == 0 && c.slab >= 1 && (size_t)L->vh * L->esz < ((size_t)1 << 31) &&
                   blocked_geometry(L->lh, (uint32_t)L->esz, c.tile, 4u, &bs);
        }
        default: return false;
    }
}

// Lines "arch lx ly lz storage resident_ok variant slab tile xcd ms"; lines
// that do not parse are skipped.  Called with g_tune_mu held.
static void read_tune_file(const char* path) {
    g_tune_file_read = true;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512], arch[128];
    long long lx, ly, lz;
    int storage, rok, variant;
    unsigned slab, tile, xcd;
    double ms;
    while (std::fgets(line, sizeof line, f))
        if (std::sscanf(line, "%127s %lld %lld %lld %d %d %d %u %u %u %lf", arch, &lx, &ly, &lz, &storage, &rok,
                        &variant, &slab, &tile, &xcd, &ms) == 11)
            g_tune_cache[TuneKey(arch, lx, ly, lz, storage, rok)] = TuneChoice{variant, slab, tile, xcd, ms};
    std::fclose(f);
}

static void append_tune_file(const char* path, const TuneKey& k, const TuneChoice& c) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // the cache file is an optimisation: an unwritable one is ignored
    std::fprintf(f, "%s %lld %lld %lld %d %d %d %u %u %u %.6f\n", std::get<0>(k).c_str(), (long long)std::get<1>(k),
                 (long long)std::get<2>(k), (long long)std::get<3>(k), std::get<4>(k), std::get<5>(k), c.variant,
                 c.slab, c.tile, c.xcd, c.ms);
    std::fclose(f);
}

// Candidates in order of preference: the first is the library default for
// the box; a later one replaces the current best only if it is more than 3%
// faster, so that choices do not flip on timing noise.
static std::vector<TuneChoice> tune_candidates(const lattice* L) {
    std::vector<TuneChoice> c;
    const uint64_t V = (uint64_t)L->vh * 2;
    const bool resident_ok = L->n_sets == 1 && !L->offl;  // the resident kernel measures one on-lattice set
    if (V <= kResidentMaxSites && resident_ok) c.push_back({LAT_SWEEP_RESIDENT, 0, 0, 1, 0});
    if (L->lh % 4 != 0) {
        if (V > kResidentMaxSites && V <= (uint64_t)1 << 18 && resident_ok)
            c.push_back({LAT_SWEEP_RESIDENT, 0, 0, 1, 0});
        c.push_back({LAT_SWEEP_GENERIC, 0, 0, 1, 0});
        return c;
    }
    const bool slab_ok = (size_t)L->vh * L->esz < ((size_t)1 << 31);
    if (slab_ok) {
        lattice d = *L;  // the library's own choice for the box, when it is a slab kernel
        d.variant = LAT_SWEEP_AUTO;
        d.slab = 0;
        d.tile = kTileDefault;
        d.xcd_order = -1;
        const int v = d.effective_variant();
        if (v == LAT_SWEEP_STREAM || v == LAT_SWEEP_ZSLAB || v == LAT_SWEEP_BLOCKED)
            c.push_back({v, d.resolved_slab(v), d.resolved_tile(v), d.resolved_xcd(v), 0});
    }
    c.push_back({LAT_SWEEP_QUAD, 0, 0, 1, 0});
    if (V > kResidentMaxSites && V <= (uint64_t)1 << 18 && resident_ok)
        c.push_back({LAT_SWEEP_RESIDENT, 0, 0, 1, 0});
    if (slab_ok)
        for (uint32_t tile = 0; tile < (uint32_t)kStreamTiles; ++tile)
            for (uint32_t slab : {16u, 24u, 32u, 48u})
                for (uint32_t xcd : {1u, 2u, 0u})
                    if (slab <= L->lz) c.push_back({LAT_SWEEP_STREAM, slab, tile, xcd, 0});
    if (slab_ok)
        for (uint32_t tile : {0u, 1u, 7u})
            for (uint32_t slab : {8u, 16u, 32u})
                if (slab <= L->lz) c.push_back({LAT_SWEEP_ZSLAB, slab, tile, 1, 0});
    if (fused_sweep_supported(L->lh, (uint32_t)L->ly))
        for (uint32_t slab : {16u, 32u})
            if (slab <= L->lz) c.push_back({LAT_SWEEP_FUSED, slab, 0, 1, 0});
    // the blocked sweep: the library's rows per tile and one fewer, over a
    // range of slab depths
    if (slab_ok) {
        lattice d = *L;
        d.slab = 0;
        d.tile = kTileDefault;
        const uint32_t rows = d.blocked_choice().first;
        for (uint32_t k : {rows, rows - 1u}) {
            BlockedShape bs;
            if (k == 0 || !blocked_geometry(L->lh, (uint32_t)L->esz, k, 4u, &bs)) continue;
            for (uint32_t slab : {32u, 48u, 64u, 96u, 128u})
                if (slab <= L->lz) c.push_back({LAT_SWEEP_BLOCKED, slab, k, 2, 0});
        }
    }
    return c;
}

static void apply_choice(lattice* L, const TuneChoice& ch) {
    L->variant = ch.variant;
    L->slab = ch.slab;
    L->tile = ch.tile;
    L->xcd_order = (int)ch.xcd;
}

static int autotune(lattice* L, int64_t reps, TuneChoice* out) {
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t pe = hipGetDevice(&dev);
    if (pe == hipSuccess) pe = hipGetDeviceProperties(&prop, dev);
    if (pe != hipSuccess) return hip_fail(pe, "device properties");
    std::string arch(prop.gcnArchName);
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    const bool resident_ok = L->n_sets == 1 && !L->offl;
    const TuneKey key(arch, L->lx, L->ly, L->lz, L->storage, resident_ok ? 1 : 0);
    const char* path = std::getenv("LATCOUL_TUNE_CACHE");
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        if (path && *path && !g_tune_file_read) read_tune_file(path);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && choice_valid(L, it->second, resident_ok)) {
            *out = it->second;
            return LAT_OK;
        }
    }
    const std::vector<TuneChoice> cands = tune_candidates(L);
    if (fused_sweep_supported(L->lh, (uint32_t)L->ly))
        if (hipError_t e = prepare_fused_sweep()) return hip_fail(e, "fused sweep set-up");
    for (const TuneChoice& ch : cands)
        if (ch.variant == LAT_SWEEP_BLOCKED) {
            if (hipError_t e = prepare_blocked_sweep()) return hip_fail(e, "blocked sweep set-up");
            break;
        }
    const size_t fbytes = round_up(2 * (size_t)L->vh * L->esz, 256);
    void* scratch = L->mem.alloc(fbytes);
    void* scratch_alt = L->mem.alloc(round_up((size_t)L->vh * L->esz, 256));
    if (!scratch || !scratch_alt) {
        L->mem.release(scratch);
        L->mem.release(scratch_alt);
        return set_error(LAT_ERR_ALLOC, "allocation of autotuning scratch failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemsetAsync(scratch, 0, fbytes, L->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    TuneChoice best{LAT_SWEEP_AUTO, 0, 0, 1, 1e30};
    int rc = LAT_OK;
    for (size_t i = 0; i < cands.size() && e == hipSuccess && rc == LAT_OK; ++i) {
        lattice tmp = *L;  // shallow copy: same sizes and streams, scratch field, no charges
        tmp.field = scratch;
        tmp.c1alt = scratch_alt;
        tmp.alt_current = false;
        tmp.t = 0;
        tmp.n_meas = 0;
        apply_choice(&tmp, cands[i]);
        auto run = [&](int64_t n) {
            if (tmp.variant == LAT_SWEEP_RESIDENT) return enqueue_resident(&tmp, n, 0, 1);
            for (int64_t k = 0; k < n; ++k)
                if (int r = enqueue_sweep(&tmp)) return r;
            return (int)LAT_OK;
        };
        rc = run(1);
        if (rc == LAT_OK) e = hipEventRecord(e0, L->stream);
        if (rc == LAT_OK && e == hipSuccess) rc = run(reps);
        if (rc == LAT_OK && e == hipSuccess) e = hipEventRecord(e1, L->stream);
        if (rc == LAT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (rc == LAT_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rc == LAT_OK && e == hipSuccess && ms / reps < 0.97 * best.ms) {
            best = cands[i];
            best.ms = ms / reps;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(L->stream);
    L->mem.release(scratch);
    L->mem.release(scratch_alt);
    if (rc != LAT_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotuning");
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = best;
        if (path && *path) append_tune_file(path, key, best);
    }
    *out = best;
    return LAT_OK;
}

extern "C" {

int lattice_autotune(lattice_t* L, int64_t reps, int* variant, int64_t* planes, int* tile, int* xcd_order,
                     double* ms_per_sweep) {
    TraceRange tr("autotune");
    if (int r = check_lattice(L)) return r;
    if (reps < 1 || reps > 1000) return set_error(LAT_ERR_ARG, "reps must be in [1, 1000]");
    TuneChoice ch;
    if (int r = autotune(L, reps, &ch)) return r;
    if (ch.variant == LAT_SWEEP_FUSED || ch.variant == LAT_SWEEP_BLOCKED)
        if (int r = lattice_set_variant(L, ch.variant)) return r;  // allocates the second colour-1 array
    apply_choice(L, ch);
    graphs_reset(L);
    if (variant) *variant = ch.variant;
    if (planes) *planes = ch.slab;
    if (tile) *tile = (int)ch.tile;
    if (xcd_order) *xcd_order = (int)ch.xcd;
    if (ms_per_sweep) *ms_per_sweep = ch.ms;
    return LAT_OK;
}

}  // extern "C"
