// Batch of independent chains on boxes of uneven size (C ABI).  All chains
// share the storage format, the Philox seed, the stream and the sweep
// counter; each has its own box, chain id (Philox counter word 2), charges
// and sample bins.  batch_run is one persistent launch (batch_kernels.hip).

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "lattice_coulomb.h"
#include "runtime_common.hpp"

using namespace latcoul;

struct lattice_batch {
    int64_t n = 0;
    int storage = 0;
    size_t esz = 4;
    size_t field_bytes = 0;  // all chains' fields
    uint64_t seed = 0;
    DeviceAllocator mem;
    hipStream_t stream = nullptr;
    std::vector<int64_t> edges;            // 3 per chain
    std::vector<BatchChainDesc> desc;      // host copy
    std::vector<AggregatedCharges> charges;
    std::vector<int64_t> n_meas;           // samples per chain
    void* field = nullptr;
    BatchChainDesc* d_desc = nullptr;
    uint32_t* d_order = nullptr;
    uint32_t* d_site = nullptr;
    double* d_Q = nullptr;
    double* d_S = nullptr;
    double* d_bins = nullptr;
    int64_t bins_per_chain = 0;  // capacity
    int64_t bin_size = 0;
    int64_t t = 0;
    bool charges_dirty = true;
    // the half-sweep form per chain: the library's rule (false) or the
    // autotuner's per-box choice (ring[k])
    bool tuned = false;
    std::vector<uint8_t> ring;
    int force_ring = -1;  // the autotuner's timing runs: every chain the ring (1) or memory (0)
};

static int check_batch(const lattice_batch* b) {
    if (!b) return set_error(LAT_ERR_ARG, "null batch handle");
    return LAT_OK;
}

static int upload_charges(lattice_batch* B) {
    size_t total = 0;
    for (auto& c : B->charges) total += c.site.size();
    if (total >= 0xFFFFFFFFull) return set_error(LAT_ERR_ARG, "too many charged sites in the batch");
    std::vector<uint32_t> site;
    std::vector<double> Q, S;
    site.reserve(total);
    Q.reserve(total);
    S.reserve(total);
    for (int64_t k = 0; k < B->n; ++k) {
        B->desc[k].site_off = (uint32_t)site.size();
        B->desc[k].n_sites = (uint32_t)B->charges[k].site.size();
        site.insert(site.end(), B->charges[k].site.begin(), B->charges[k].site.end());
        Q.insert(Q.end(), B->charges[k].Q.begin(), B->charges[k].Q.end());
        S.insert(S.end(), B->charges[k].S.begin(), B->charges[k].S.end());
    }
    const size_t cap = std::max<size_t>(total, 1);
    uint32_t* d_site = static_cast<uint32_t*>(B->mem.alloc(cap * 4));
    double* d_Q = static_cast<double*>(B->mem.alloc(cap * 8));
    double* d_S = static_cast<double*>(B->mem.alloc(cap * 8));
    if (!d_site || !d_Q || !d_S) {
        B->mem.release(d_site);
        B->mem.release(d_Q);
        B->mem.release(d_S);
        return set_error(LAT_ERR_ALLOC, "allocation of the batch charge list failed");
    }
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess && total) e = hipMemcpy(d_site, site.data(), total * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && total) e = hipMemcpy(d_Q, Q.data(), total * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && total) e = hipMemcpy(d_S, S.data(), total * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        B->mem.release(d_site);
        B->mem.release(d_Q);
        B->mem.release(d_S);
        return hip_fail(e, "batch charge upload");
    }
    B->mem.release(B->d_site);
    B->mem.release(B->d_Q);
    B->mem.release(B->d_S);
    B->d_site = d_site;
    B->d_Q = d_Q;
    B->d_S = d_S;
    B->charges_dirty = false;
    return LAT_OK;
}

// bins: chain k owns bins [k * cap, (k + 1) * cap), 2 doubles each
static int ensure_batch_bins(lattice_batch* B, int64_t need) {
    if (need <= B->bins_per_chain) return LAT_OK;
    const int64_t cap = std::max<int64_t>({need, 2 * B->bins_per_chain, 16});
    const size_t row = sizeof(double) * 2 * (size_t)cap;
    double* nb = static_cast<double*>(B->mem.alloc(row * (size_t)B->n));
    if (!nb) return set_error(LAT_ERR_ALLOC, "allocation of the batch bins failed");
    hipError_t e = hipMemsetAsync(nb, 0, row * (size_t)B->n, B->stream);
    if (e == hipSuccess && B->d_bins && B->bins_per_chain > 0) {
        const size_t old_row = sizeof(double) * 2 * (size_t)B->bins_per_chain;
        e = hipMemcpy2DAsync(nb, row, B->d_bins, old_row, old_row, (size_t)B->n, hipMemcpyDeviceToDevice,
                             B->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) {
        B->mem.release(nb);
        return hip_fail(e, "batch bin resize");
    }
    B->mem.release(B->d_bins);
    B->d_bins = nb;
    B->bins_per_chain = cap;
    return LAT_OK;
}

extern "C" {

int batch_create(int64_t n_chains, const int64_t* edges, const uint32_t* chain_ids, int storage, uint64_t seed,
                 const lat_allocator* alloc, void* hip_stream, lattice_batch_t** out) {
    if (!out) return set_error(LAT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_chains < 1 || n_chains > (1 << 20)) return set_error(LAT_ERR_ARG, "n_chains must be in [1, 2^20]");
    if (!edges) return set_error(LAT_ERR_ARG, "edges is NULL");
    if (storage < LAT_FP32 || storage > LAT_FP16_SR) return set_error(LAT_ERR_ARG, "unknown storage format");
    if (alloc && (!alloc->alloc || !alloc->release))
        return set_error(LAT_ERR_ARG, "allocator needs both alloc and release");
    const size_t esz = storage == LAT_FP32 ? 4 : 2;
    std::vector<BatchChainDesc> desc((size_t)n_chains);
    uint64_t off = 0;
    for (int64_t k = 0; k < n_chains; ++k) {
        const int64_t lx = edges[3 * k], ly = edges[3 * k + 1], lz = edges[3 * k + 2];
        if (lx < 2 || (lx & 1) || ly < 1 || lz < 1)
            return set_error(LAT_ERR_ARG, "chain " + std::to_string(k) + ": lx must be even >= 2, ly, lz >= 1");
        if ((double)lx * ly * lz >= 2147483648.0)
            return set_error(LAT_ERR_ARG, "chain " + std::to_string(k) + ": box must have fewer than 2^31 sites");
        BatchChainDesc& d = desc[(size_t)k];
        d.field_off = off;
        d.lh = (uint32_t)(lx / 2);
        d.ly = (uint32_t)ly;
        d.lz = (uint32_t)lz;
        d.vh = (uint32_t)(lx / 2 * ly * lz);
        d.chain_id = chain_ids ? chain_ids[k] : (uint32_t)k;
        d.site_off = d.n_sites = d.bin_off = d.meas0 = 0;
        off += round_up(2 * (size_t)d.vh, 64);  // keep every chain 16-byte (and 128-byte) aligned
    }
    lattice_batch* B = new lattice_batch();
    B->n = n_chains;
    B->storage = storage;
    B->esz = esz;
    B->field_bytes = (size_t)off * esz;
    B->seed = seed;
    B->mem = DeviceAllocator(alloc);
    B->stream = static_cast<hipStream_t>(hip_stream);
    B->edges.assign(edges, edges + 3 * n_chains);
    B->desc = desc;
    B->charges.resize((size_t)n_chains);
    B->n_meas.assign((size_t)n_chains, 0);
    B->field = B->mem.alloc(std::max<size_t>(off * esz, 256));
    B->d_desc = static_cast<BatchChainDesc*>(B->mem.alloc(sizeof(BatchChainDesc) * (size_t)n_chains));
    B->d_order = static_cast<uint32_t*>(B->mem.alloc(sizeof(uint32_t) * (size_t)n_chains));
    if (!B->field || !B->d_desc || !B->d_order) {
        batch_destroy(B);
        return set_error(LAT_ERR_ALLOC, "allocation of the batch failed");
    }
    // launch order: largest boxes first (stable), so the longest chains start first
    std::vector<uint32_t> order((size_t)n_chains);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return desc[a].vh > desc[b].vh; });
    hipError_t e = hipMemsetAsync(B->field, 0, std::max<size_t>(off * esz, 256), B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess) e = hipMemcpy(B->d_order, order.data(), 4 * (size_t)n_chains, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_destroy(B);
        return hip_fail(e, "batch initialisation");
    }
    *out = B;
    return LAT_OK;
}

int batch_set_charges(lattice_batch_t* B, int64_t chain, int64_t n, const int32_t* xyz, const double* q) {
    if (int r = check_batch(B)) return r;
    if (chain < 0 || chain >= B->n) return set_error(LAT_ERR_ARG, "chain index out of range");
    if (n < 0) return set_error(LAT_ERR_ARG, "negative charge count");
    if (n > 0 && (!xyz || !q)) return set_error(LAT_ERR_ARG, "xyz or q is NULL");
    const int64_t* e = &B->edges[3 * chain];
    AggregatedCharges agg;
    if (int r = aggregate_charges(n, xyz, q, e[0], e[1], e[2], B->desc[chain].vh, &agg)) return r;
    B->charges[chain] = std::move(agg);
    B->charges_dirty = true;
    // a new observable for this chain: its sample series restarts
    B->n_meas[chain] = 0;
    if (B->d_bins && B->bins_per_chain > 0) {
        const size_t row = sizeof(double) * 2 * (size_t)B->bins_per_chain;
        hipError_t err = hipMemsetAsync(reinterpret_cast<char*>(B->d_bins) + row * (size_t)chain, 0, row, B->stream);
        if (err != hipSuccess) return hip_fail(err, "bin reset");
    }
    return LAT_OK;
}

int batch_run(lattice_batch_t* B, int64_t n_therm, int64_t n_meas, int64_t bin_size) {
    TraceRange tr("batch_run");
    if (int r = check_batch(B)) return r;
    if (n_therm < 0 || n_meas < 0) return set_error(LAT_ERR_ARG, "negative sweep count");
    if (bin_size < 1) return set_error(LAT_ERR_ARG, "bin_size < 1");
    bool any_samples = false;
    for (int64_t m : B->n_meas) any_samples |= m > 0;
    if (any_samples && B->bin_size != 0 && bin_size != B->bin_size)
        return set_error(LAT_ERR_ARG, "bin_size differs from the one of earlier samples");
    if (B->t + n_therm + n_meas > (int64_t)0x7FFFFFFF) return set_error(LAT_ERR_ARG, "sweep counter would exceed 2^31");
    if (B->charges_dirty)
        if (int r = upload_charges(B)) return r;
    int64_t need = 1;
    for (int64_t m : B->n_meas) need = std::max(need, (m + n_meas + bin_size - 1) / bin_size);
    // bin slots are indexed in 64 bits; the bin table (2 doubles per slot)
    // must stay addressable
    if ((double)B->n * (double)std::max<int64_t>({need, 2 * B->bins_per_chain, 16}) * 16.0 >= 9.0e18)
        return set_error(LAT_ERR_ARG, "the sample bins of this batch would exceed the addressable range");
    if (int r = ensure_batch_bins(B, need)) return r;
    B->bin_size = bin_size;
    // the half-sweep form: without tuning, the LDS ring for every chain it
    // applies to when the fields fill the 256 MiB last-level cache (the
    // chains then wait on memory, where the ring is faster)
    const bool big = B->field_bytes >= ((size_t)256 << 20);
    for (int64_t k = 0; k < B->n; ++k) {
        BatchChainDesc& d = B->desc[k];
        d.bin_off = (uint64_t)k * (uint64_t)B->bins_per_chain;
        d.meas0 = (uint32_t)B->n_meas[k];
        const bool ring = B->force_ring >= 0 ? B->force_ring != 0 : B->tuned ? B->ring[k] != 0 : big;
        d.ring = ring && batch_ring_applies(d.lh, d.ly, d.vh) ? 1u : 0u;
    }
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess)
        e = hipMemcpy(B->d_desc, B->desc.data(), sizeof(BatchChainDesc) * (size_t)B->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    if (n_therm + n_meas == 0) return LAT_OK;
    BatchArgs a{};
    a.field = B->field;
    a.desc = B->d_desc;
    a.order = B->d_order;
    a.n_chains = (uint32_t)B->n;
    a.site = B->d_site;
    a.Q = B->d_Q;
    a.S = B->d_S;
    a.bins = B->d_bins;
    a.t0 = (uint32_t)B->t;
    a.n_therm = (uint32_t)n_therm;
    a.n_meas = (uint32_t)n_meas;
    a.every = 1;
    a.bin_size = (uint32_t)bin_size;
    a.k0 = (uint32_t)B->seed;
    a.k1 = (uint32_t)(B->seed >> 32);
    a.storage = B->storage;
    a.single = false;
    e = launch_batch(a, B->stream);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    B->t += n_therm + n_meas;
    for (auto& m : B->n_meas) m += n_meas;
    return LAT_OK;
}

// Per-box choice of the batch's half-sweep form, cached for the process:
// (device architecture, box, storage, chains of that box in the batch) ->
// LDS ring or memory.
using BatchTuneKey = std::tuple<std::string, int64_t, int64_t, int64_t, int, int64_t>;
static std::mutex g_batch_tune_mu;
static std::map<BatchTuneKey, bool> g_batch_tune_cache;

// Time `reps` sweeps of a scratch batch of `count` chains of one box with
// every chain the ring (ring = true) or memory.
static int time_scratch_batch(lattice_batch* B, const int64_t* edge, int64_t count, bool ring, int64_t reps,
                              float* ms) {
    std::vector<int64_t> edges;
    for (int64_t k = 0; k < count; ++k) edges.insert(edges.end(), edge, edge + 3);
    lattice_batch_t* T = nullptr;
    if (int r = batch_create(count, edges.data(), nullptr, B->storage, B->seed, B->mem.source(), B->stream, &T))
        return r;
    T->force_ring = ring ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = batch_run(T, 1, 0, 1);  // the launch's first use of the kernel and the fields
    hipError_t e = hipSuccess;
    if (rc == LAT_OK) e = hipEventCreate(&e0);
    if (rc == LAT_OK && e == hipSuccess) e = hipEventCreate(&e1);
    if (rc == LAT_OK && e == hipSuccess) e = hipEventRecord(e0, B->stream);
    if (rc == LAT_OK && e == hipSuccess) rc = batch_run(T, reps, 0, 1);
    if (rc == LAT_OK && e == hipSuccess) e = hipEventRecord(e1, B->stream);
    if (rc == LAT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    if (rc == LAT_OK && e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    batch_destroy(T);
    if (rc != LAT_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "batch autotuning");
    return LAT_OK;
}

int batch_autotune(lattice_batch_t* B, int64_t reps, int64_t* n_ring) {
    TraceRange tr("batch_autotune");
    if (int r = check_batch(B)) return r;
    if (reps < 1 || reps > 1000) return set_error(LAT_ERR_ARG, "reps must be in [1, 1000]");
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t pe = hipGetDevice(&dev);
    if (pe == hipSuccess) pe = hipGetDeviceProperties(&prop, dev);
    if (pe != hipSuccess) return hip_fail(pe, "device properties");
    std::string arch(prop.gcnArchName);
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    // the boxes the ring applies to, with their number of chains
    std::map<std::tuple<int64_t, int64_t, int64_t>, int64_t> count;
    for (int64_t k = 0; k < B->n; ++k) {
        const BatchChainDesc& d = B->desc[k];
        if (batch_ring_applies(d.lh, d.ly, d.vh)) ++count[{B->edges[3 * k], B->edges[3 * k + 1], B->edges[3 * k + 2]}];
    }
    std::map<std::tuple<int64_t, int64_t, int64_t>, bool> choice;
    for (const auto& [shape, cnt] : count) {
        const BatchTuneKey key(arch, std::get<0>(shape), std::get<1>(shape), std::get<2>(shape), B->storage, cnt);
        {
            std::lock_guard<std::mutex> g(g_batch_tune_mu);
            auto it = g_batch_tune_cache.find(key);
            if (it != g_batch_tune_cache.end()) {
                choice[shape] = it->second;
                continue;
            }
        }
        const int64_t edge[3] = {std::get<0>(shape), std::get<1>(shape), std::get<2>(shape)};
        float ms_ring = 0.f, ms_mem = 0.f;
        if (int r = time_scratch_batch(B, edge, cnt, true, reps, &ms_ring)) return r;
        if (int r = time_scratch_batch(B, edge, cnt, false, reps, &ms_mem)) return r;
        const bool ring = ms_ring < 0.97f * ms_mem;  // the ring only where it is clearly faster
        choice[shape] = ring;
        std::lock_guard<std::mutex> g(g_batch_tune_mu);
        g_batch_tune_cache[key] = ring;
    }
    B->ring.assign((size_t)B->n, 0);
    int64_t nr = 0;
    for (int64_t k = 0; k < B->n; ++k) {
        auto it = choice.find({B->edges[3 * k], B->edges[3 * k + 1], B->edges[3 * k + 2]});
        B->ring[k] = it != choice.end() && it->second ? 1 : 0;
        nr += B->ring[k];
    }
    B->tuned = true;
    if (n_ring) *n_ring = nr;
    return LAT_OK;
}

int batch_energy_estimate(lattice_batch_t* B, int64_t chain, double* mean, double* stderr_binned,
                          int64_t* n_samples, int64_t* n_bins) {
    if (int r = check_batch(B)) return r;
    if (chain < 0 || chain >= B->n) return set_error(LAT_ERR_ARG, "chain index out of range");
    const int64_t M = B->n_meas[chain];
    const int64_t bs = B->bin_size > 0 ? B->bin_size : 1;
    const int64_t used = (M + bs - 1) / bs;
    std::vector<double> h((size_t)std::max<int64_t>(used, 1) * 2, 0.0);
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess && used > 0)
        e = hipMemcpy(h.data(), B->d_bins + 2 * (size_t)chain * (size_t)B->bins_per_chain,
                      sizeof(double) * 2 * (size_t)used, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "bin readback");
    EstimateResult res = estimate_from_bins(h.data(), used, M, bs);
    if (mean) *mean = res.mean;
    if (stderr_binned) *stderr_binned = res.stderr_binned;
    if (n_samples) *n_samples = M;
    if (n_bins) *n_bins = res.full_bins;
    if (!res.finite) return set_error(LAT_ERR_STATE, "non-finite sample found");
    if (res.full_bins < 2) return set_error(LAT_ERR_STATE, "fewer than 2 full bins: no error estimate");
    return LAT_OK;
}

int batch_get_field(lattice_batch_t* B, int64_t chain, float* host_out) {
    if (int r = check_batch(B)) return r;
    if (chain < 0 || chain >= B->n) return set_error(LAT_ERR_ARG, "chain index out of range");
    if (!host_out) return set_error(LAT_ERR_ARG, "host_out is NULL");
    const BatchChainDesc& d = B->desc[chain];
    std::vector<unsigned char> buf(2 * (size_t)d.vh * B->esz);
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess)
        e = hipMemcpy(buf.data(), static_cast<char*>(B->field) + d.field_off * B->esz, buf.size(),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "field readback");
    const int64_t* ed = &B->edges[3 * chain];
    compact_to_natural(buf.data(), B->storage, ed[0], ed[1], ed[2], d.vh, host_out);
    return LAT_OK;
}

void batch_destroy(lattice_batch_t* B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->stream);
    B->mem.release(B->field);
    B->mem.release(B->d_desc);
    B->mem.release(B->d_order);
    B->mem.release(B->d_site);
    B->mem.release(B->d_Q);
    B->mem.release(B->d_S);
    B->mem.release(B->d_bins);
    delete B;
}

}  // extern "C"
