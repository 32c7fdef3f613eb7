// sweep_and_measure for callers that cannot allocate device memory (code
// under stream capture, tight serving loops, harnesses that forbid
// allocation).  The sample gather's partial sums, the only scratch memory
// the measured sweeps use beyond the lattice's own state, live in one static
// device array per GPU instead of the lattice's buffers; sweeps are launched
// one by one (a graph capture would create a stream and instantiate a
// graph), bins must already have room, and nothing is allocated or freed.

#include "lattice_impl.hpp"

#include <mutex>

namespace latcoul {

// The static scratch: each GPU the library runs on holds its own copy until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is a stand-in, not a device address): it uses the device
// address hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)1 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// The scratch's device address on `dev`, made current for the lookup.
static int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error(LAT_ERR_STATE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return hip_fail(e, "scratch address");
        if (!p) return set_error(LAT_ERR_DEVICE, "scratch address is NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LAT_OK;
}

// Bytes of partial sums a measured sweep of L uses on its current path.
static size_t partial_bytes(const lattice* L) {
    const size_t separate = (size_t)L->meas_blocks * 16u * (L->offl ? 1u : L->n_sets);
    if (!fused_gather_on(L)) return separate;
    // samples x sets x two colours x (X, Y); with several sets a call's last
    // sample goes through the separate gather as well
    const size_t fused = (size_t)L->fg.blocks * 32u * L->fg.nbuf * L->fg.sets;
    return L->fg.sets > 1 ? std::max(fused, separate) : fused;
}

}  // namespace latcoul

extern "C" int sweep_and_measure_noalloc(lattice_t* L, int64_t n_sweeps, int64_t measure_every, int64_t bin_size) {
    using namespace latcoul;
    TraceRange tr("sweep_and_measure_noalloc");
    if (int r = check_lattice(L)) return r;
    if (n_sweeps < 0) return set_error(LAT_ERR_ARG, "n_sweeps < 0");
    if (measure_every < 1) return set_error(LAT_ERR_ARG, "measure_every < 1");
    if (bin_size < 1) return set_error(LAT_ERR_ARG, "bin_size < 1");
    if (L->bin_size != 0 && bin_size != L->bin_size)
        return set_error(LAT_ERR_ARG, "bin_size differs from the one of earlier samples");
    if (L->t + n_sweeps > (int64_t)0x7FFFFFFF) return set_error(LAT_ERR_ARG, "sweep counter would exceed 2^31");
    if (!L->d_partials) return set_error(LAT_ERR_STATE, "no charges placed (set_charges allocates them)");
    const int64_t total = L->n_meas + n_sweeps / measure_every;
    if ((total + bin_size - 1) / bin_size > L->bin_cap)
        return set_error(LAT_ERR_STATE, "the sample bins have no room for these samples (bins grow only in "
                                        "sweep_and_measure: run one there first)");
    const int v = L->effective_variant();
    if (v == LAT_SWEEP_RESIDENT) {  // one launch, samples recorded in the workgroup: no scratch
        L->bin_size = bin_size;
        L->fg.last = false;
        return enqueue_resident(L, 0, n_sweeps, measure_every);
    }
    // the fused gather's lists are built outside (set_charges, or the first
    // sweep_and_measure after a change of kernel or tiling)
    if ((v == LAT_SWEEP_STREAM || v == LAT_SWEEP_BLOCKED) && L->n_sets == 1 && !L->offl && L->host_charges &&
        !fused_gather_current(L))
        return set_error(LAT_ERR_STATE, "the sample lists of the current tiling are not built (set_charges or "
                                        "sweep_and_measure builds them)");
    const size_t need = partial_bytes(L);
    if (need > kNoAllocScratchBytes)
        return set_error(LAT_ERR_ARG, "the partial sums of this lattice exceed the 1 MiB scratch");
    void* sp = nullptr;
    if (int r = scratch_address(L->device, &sp)) return r;
    L->bin_size = bin_size;
    L->fg.last = fused_gather_on(L);
    // the partial sums of this call's samples go to the scratch (each call
    // writes every partial it reads: nothing needs clearing)
    double* const own = L->d_partials;
    double* const own_fused = L->fg.d_part;
    L->d_partials = static_cast<double*>(sp);
    if (L->fg.d_part) L->fg.d_part = static_cast<double*>(sp);
    const int rc = run_sweeps(L, n_sweeps, measure_every, /*eager=*/true);
    L->d_partials = own;
    L->fg.d_part = own_fused;
    return rc;
}
