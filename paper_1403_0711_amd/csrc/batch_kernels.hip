// Batched chains: many independent heat-bath chains on boxes of uneven size
// in one persistent launch.  Workgroup b runs chain order[b] (chains sorted
// largest first, so the longest chains start first) through all its sweeps:
// colour-0 half-sweep, workgroup barrier, colour-1 half-sweep, barrier, and
// after each measured sweep the gather of X = sum Q phi, Y = sum S phi^2 over
// the chain's charges, O = X^2 - Y and its compensated add into the chain's
// bin.  Only one workgroup touches a chain, so workgroup barriers (which
// order the workgroup's global stores before its later loads, and its LDS
// writes before its later LDS reads) are the only synchronisation.  Each site draws exactly the random numbers of a single
// lattice with the chain's id (same Philox counter layout).

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

constexpr int kBatchThreads = 1024;
// LDS ring of the other colour's quads, indexed by quad number modulo its
// size: a chunk of kBatchThreads quads reads one plane (qpp quads) on either
// side of it while the next chunk's new quads are written, so 2 * 1024 + 2 *
// qpp <= 8192 holds every chain with at most 3072 quads per plane.  128 KiB
// at FP32, within gfx950's 160 KiB per workgroup; the kernel's registers
// allow one 1024-thread workgroup per CU in any case.
constexpr uint32_t kRingQuads = 8192;
constexpr uint32_t kRingMaxPlaneQuads = (kRingQuads - 2u * kBatchThreads) / 2u;
static_assert(kRingMaxPlaneQuads == kBatchRingMaxPlaneQuads && 4u * kBatchThreads == 4096u,
              "the host's test of which chains the ring takes");

// One raw quad (4 elements) of a storage format
template <class St>
using RawQuad = typename St::Raw;

// The neighbours of quad qi (element 4 qi) read from the ring; the same
// values and face flags as quad_load_global reads from the colour array.
template <class St>
__device__ __forceinline__ QuadNeighbours<St> quad_load_ring(const typename St::T* ring, uint32_t qi, uint32_t nq,
                                                            uint32_t qpp, bool ym_in, bool yp_in, bool zm_in,
                                                            bool zp_in, bool e_in, uint32_t p) {
    auto el = [](uint32_t k) { return (k & (kRingQuads - 1u)) << 2; };
    const uint32_t ie = p == 0 ? el(qi - 1u) + 3u : el(qi + 1u);  // the x-neighbour beyond the quad
    QuadNeighbours<St> nb;
    if constexpr (kF16Grid<St>) {
        const u32x2 zero = {0u, 0u};
        nb.cen = at<u32x2>(ring, el(qi));
        nb.ym = ym_in ? at<u32x2>(ring, el(qi - nq)) : zero;
        nb.yp = yp_in ? at<u32x2>(ring, el(qi + nq)) : zero;
        nb.zm = zm_in ? at<u32x2>(ring, el(qi - qpp)) : zero;
        nb.zp = zp_in ? at<u32x2>(ring, el(qi + qpp)) : zero;
        nb.e = e_in ? (uint32_t)at<uint16_t>(ring, ie) : 0u;
    } else {
        const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
        nb.cen = St::ld4(ring, el(qi));
        nb.ym = ym_in ? St::ld4(ring, el(qi - nq)) : zero;
        nb.yp = yp_in ? St::ld4(ring, el(qi + nq)) : zero;
        nb.zm = zm_in ? St::ld4(ring, el(qi - qpp)) : zero;
        nb.zp = zp_in ? St::ld4(ring, el(qi + qpp)) : zero;
        nb.e = e_in ? St::ld(ring, ie) : 0.f;
    }
    return nb;
}

// One half-sweep of colour c over a whole chain by one workgroup, in one of
// four forms.  use_ring, lh % 4 == 0 and at most 3072 quads (4 compact sites
// of a row each) per plane: chunks of 1024 consecutive quads, one per thread, whose
// neighbours are read from an LDS ring of the other colour (each quad loaded
// from memory once per half-sweep); the load of the thread's quad of the next
// chunk is in flight while it updates this one, and a workgroup barrier ends
// each chunk.  The quads chunk 0 reads (the first 1024 + qpp) are, up to
// 2048 of them, the ones chunks 0 and 1 of the previous half-sweep updated:
// each thread keeps its two results and writes them into the ring after its
// last chunk, so that only the first half-sweep of a launch (seeded false)
// loads them from memory (planes over 1024 quads load the rest each time).
// The ring pays where the chains wait on memory (fields that fill the
// last-level cache: 256 chains of 64^3 sweep 12% faster); a chain bound by
// its CU's arithmetic runs 10% slower with it (the ring's address arithmetic
// and a barrier per chunk), so the host asks for it only for such batches.
// A chain of at most 1024 quads keeps its whole other colour in the ring in
// any batch: one chunk, nothing loaded after the first half-sweep.
// Otherwise, lh % 4 == 0: two quads per thread and
// iteration read from memory, whose loads are all issued before either
// update (a lane whose second quad lies past the end loads quad 0's centre,
// in range, with every face load switched off, and stores nothing).  Else
// one site per thread and iteration.
template <class St>
__device__ __forceinline__ void chain_halfsweep(typename St::T* field, const BatchChainDesc& d, uint32_t c,
                                                uint32_t h, uint32_t k0, uint32_t k1, bool use_ring,
                                                typename St::T* ring, bool seeded, typename St::Raw& keep0,
                                                typename St::Raw& keep1) {
    using T = typename St::T;
    const T* other = field + (size_t)(c ^ 1u) * d.vh;
    T* own = field + (size_t)c * d.vh;
    const uint32_t lh = d.lh, ly = d.ly, lz = d.lz, plane = ly * lh;
    const float sixth = 1.0f / 6.0f;
    if ((lh & 3u) == 0 && d.vh <= 4u * kBatchThreads) {
        // a chain of at most 1024 quads: the whole other colour is in the
        // ring (after the first half-sweep of a launch: the threads' own
        // results of the previous half-sweep), one quad per thread, no load
        const uint32_t nq = lh >> 2, qpp = nq * ly, nquads = d.vh >> 2, t = threadIdx.x;
        auto el = [](uint32_t k) { return (k & (kRingQuads - 1u)) << 2; };
        if (!seeded) {
            if (t < nquads) at<RawQuad<St>>(ring, el(t)) = at<RawQuad<St>>(other, t << 2);
            __syncthreads();
        }
        if (t < nquads) {
            const uint32_t r = t / nq, q = t - r * nq, y = r % ly, z = r / ly;
            const uint32_t p = (c + y + z) & 1u;
            const QuadNeighbours<St> nb = quad_load_ring<St>(ring, t, nq, qpp, y > 0, y + 1 < ly, z > 0, z + 1 < lz,
                                                             p == 0 ? q > 0 : q + 1 < nq, p);
            const QuadOut o = quad_update_from<St>(nb, p, t << 2, h, d.chain_id, k0, k1);
            keep0 = St::pack4(o.v, o.w);
            at<RawQuad<St>>(own, t << 2) = keep0;
        }
        __syncthreads();  // every ring read done before the ring takes this colour
        if (t < nquads) at<RawQuad<St>>(ring, el(t)) = keep0;
    } else if (use_ring && (lh & 3u) == 0 && (lh >> 2) * ly <= kRingMaxPlaneQuads) {
        using Raw = RawQuad<St>;
        const uint32_t nq = lh >> 2, qpp = nq * ly, nquads = d.vh >> 2;
        auto el = [](uint32_t k) { return (k & (kRingQuads - 1u)) << 2; };
        // the quads chunk 0 reads: [0, 1024 + qpp) within the box (at most
        // four per thread); a seeded ring already holds the first 2048
        const uint32_t pro = min((uint32_t)kBatchThreads + qpp, nquads);
        const uint32_t from = seeded ? min(2u * (uint32_t)kBatchThreads, pro) : 0u;
        if (from < pro) {
            for (uint32_t g = from + threadIdx.x; g < pro; g += kBatchThreads)
                at<Raw>(ring, el(g)) = at<Raw>(other, g << 2);
            __syncthreads();
        }
        const uint32_t t = threadIdx.x, r0 = t / nq;
        uint32_t qi = t, q = t - r0 * nq, y = r0 % ly, z = r0 / ly;
        const uint32_t drow = kBatchThreads / nq, dq = kBatchThreads - drow * nq;
        const uint32_t dz = drow / ly, dy = drow - dz * ly;
        for (uint32_t base = 0; base < nquads; base += kBatchThreads) {
            // this thread's quad of the next chunk's new ones: past the window
            // this chunk reads, so the slot it fills is not read before the barrier
            // (a lane past the box loads the last quad, in range, into a slot
            // that is never read: every read of a quad past the box is
            // switched off by its face flag).  Unconditional, and the update
            // is stored after the ring write, so that the wait for the
            // prefetched quad waits for nothing else.
            const uint32_t g = base + (uint32_t)kBatchThreads + qpp + t;
            const Raw nxt = at<Raw>(other, min(g, nquads - 1u) << 2);
            // a lane past the box (last chunk) computes from ring slots
            // (in range: indices are taken modulo the ring) and stores nothing
            const uint32_t p = (c + y + z) & 1u;
            const QuadNeighbours<St> nb = quad_load_ring<St>(ring, qi, nq, qpp, y > 0, y + 1 < ly, z > 0, z + 1 < lz,
                                                             p == 0 ? q > 0 : q + 1 < nq, p);
            const QuadOut o = quad_update_from<St>(nb, p, qi << 2, h, d.chain_id, k0, k1);
            const Raw v = St::pack4(o.v, o.w);
            at<Raw>(ring, el(g)) = nxt;
            if (qi < nquads) at<Raw>(own, qi << 2) = v;
            if (base == 0) keep0 = v;
            if (base == (uint32_t)kBatchThreads) keep1 = v;
            qi += kBatchThreads;
            q += dq;
            const uint32_t cq = q >= nq ? 1u : 0u;
            q -= cq * nq;
            y += dy + cq;
            const uint32_t cy = y >= ly ? 1u : 0u;
            y -= cy * ly;
            z += dz + cy;
            __syncthreads();
        }
        // the next half-sweep's first window: this colour's quads [0, pro)
        // below 2048, stored in the ring in the storage format, as in memory
        // (the caller's barrier orders these writes before the next
        // half-sweep's reads)
        if (t < pro) at<Raw>(ring, el(t)) = keep0;
        if (t + (uint32_t)kBatchThreads < pro) at<Raw>(ring, el(t + (uint32_t)kBatchThreads)) = keep1;
    } else if ((lh & 3u) == 0) {
        const uint32_t nq = lh >> 2, nquads = d.vh >> 2;
        // the thread's quad (q, y, z), advanced kBatchThreads quads at a time
        // with carries: one division per half-sweep instead of two per quad
        const uint32_t t = threadIdx.x, r0 = t / nq;
        uint32_t qi = t, q = t - r0 * nq, y = r0 % ly, z = r0 / ly;
        const uint32_t drow = kBatchThreads / nq, dq = kBatchThreads - drow * nq;
        const uint32_t dz = drow / ly, dy = drow - dz * ly;
        auto advance = [&]() {
            qi += kBatchThreads;
            q += dq;
            const uint32_t cq = q >= nq ? 1u : 0u;
            q -= cq * nq;
            y += dy + cq;
            const uint32_t cy = y >= ly ? 1u : 0u;
            y -= cy * ly;
            z += dz + cy;
        };
        while (qi < nquads) {
            uint32_t j0[2], p[2];
            bool in[2];
            QuadNeighbours<St> nb[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                in[u] = qi < nquads;
                p[u] = (c + y + z) & 1u;
                j0[u] = (z * ly + y) * lh + 4u * q;
                // a lane past the end loads in-range quads again (its first), and stores nothing
                const uint32_t jl = in[u] ? j0[u] : 0u;
                nb[u] = quad_load_global<St>(other, jl, lh, plane, in[u] && y > 0, in[u] && y + 1 < ly,
                                             in[u] && z > 0, in[u] && z + 1 < lz,
                                             in[u] && (p[u] == 0 ? q > 0 : q + 1 < nq), p[u]);
                advance();
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (in[u]) {
                    const QuadOut o = quad_update_from<St>(nb[u], p[u], j0[u], h, d.chain_id, k0, k1);
                    St::st4(own, j0[u], o.v, o.w);
                }
        }
    } else {
        for (uint32_t j = threadIdx.x; j < d.vh; j += kBatchThreads) {
            const uint32_t hx = j % lh, rowi = j / lh;
            const uint32_t y = rowi % ly, z = rowi / ly;
            const uint32_t p = (c + y + z) & 1u;
            float s = 0.f;
            if (hx + p >= 1) s += St::ld(other, j - 1 + p);
            if (hx + p < lh) s += St::ld(other, j + p);
            if (y > 0) s += St::ld(other, j - lh);
            if (y + 1 < ly) s += St::ld(other, j + lh);
            if (z > 0) s += St::ld(other, j - plane);
            if (z + 1 < lz) s += St::ld(other, j + plane);
            const uint4 r = philox4x32_10(j >> 2, h, d.chain_id, 0u, k0, k1);
            const uint32_t w = (j & 3u) == 0 ? r.x : (j & 3u) == 1 ? r.y : (j & 3u) == 2 ? r.z : r.w;
            St::st(own, j, fmaf(s, sixth, heatbath_noise(w)), w);
        }
    }
}

// All sweeps of one chain by one workgroup: n_therm unmeasured sweeps, then
// n_meas sweeps with a sample after every `every`-th one.
template <class St>
__device__ __forceinline__ void run_chain(typename St::T* fields, const BatchChainDesc& d,
                                          const uint32_t* __restrict__ site, const double* __restrict__ Q,
                                          const double* __restrict__ S, double* bins, uint32_t t0, uint32_t n_therm,
                                          uint32_t n_meas, uint32_t every, uint32_t bin_size, uint32_t k0,
                                          uint32_t k1, double* last_xy, bool use_ring) {
    typename St::T* field = fields + d.field_off;
    const typename St::T* cfield = field;
    __shared__ __align__(16) typename St::T ring[kRingQuads * 4];
    const uint32_t n_sweeps = n_therm + n_meas;
    typename St::Raw keep0{}, keep1{};
    for (uint32_t s = 0; s < n_sweeps; ++s) {
        const uint32_t t = t0 + s;
        chain_halfsweep<St>(field, d, 0u, 2u * t, k0, k1, use_ring, ring, s > 0, keep0, keep1);
        __syncthreads();
        chain_halfsweep<St>(field, d, 1u, 2u * t + 1u, k0, k1, use_ring, ring, true, keep0, keep1);
        __syncthreads();
        if (s >= n_therm && (s - n_therm + 1) % every == 0) {
            double x = 0.0, y = 0.0;
            for (uint32_t i = d.site_off + threadIdx.x; i < d.site_off + d.n_sites; i += kBatchThreads) {
                const double v = (double)St::ld(cfield, site[i]);
                x = fma(Q[i], v, x);
                y = fma(S[i], v * v, y);
            }
            block_sum2<kBatchThreads>(x, y);  // ends with a barrier
            if (threadIdx.x == 0) {
                const uint32_t m = (s - n_therm + 1) / every - 1;  // sample index within this run
                const uint64_t b = d.bin_off + (d.meas0 + m) / bin_size;
                const double O = x * x - y;
                double sum = bins[2 * b], comp = bins[2 * b + 1];
                const double yk = O - comp;
                const double tk = sum + yk;
                comp = (tk - sum) - yk;
                bins[2 * b] = tk;
                bins[2 * b + 1] = comp;
                if (last_xy) {
                    last_xy[0] = x;
                    last_xy[1] = y;
                }
            }
        }
    }
}

template <class St>
__global__ __launch_bounds__(kBatchThreads) void batch_chains(typename St::T* __restrict__ fields,
                                                              const BatchChainDesc* __restrict__ desc,
                                                              const uint32_t* __restrict__ order,
                                                              const uint32_t* __restrict__ site,
                                                              const double* __restrict__ Q,
                                                              const double* __restrict__ S, double* bins,
                                                              uint32_t t0, uint32_t n_therm, uint32_t n_meas,
                                                              uint32_t every, uint32_t bin_size, uint32_t k0,
                                                              uint32_t k1) {
    const BatchChainDesc d = desc[order[blockIdx.x]];
    run_chain<St>(fields, d, site, Q, S, bins, t0, n_therm, n_meas, every, bin_size, k0, k1, nullptr,
                  d.ring != 0);
}

// One lattice small enough for one workgroup: the whole run in one launch.
template <class St>
__global__ __launch_bounds__(kBatchThreads) void resident_chain(typename St::T* __restrict__ field,
                                                                BatchChainDesc d,
                                                                const uint32_t* __restrict__ site,
                                                                const double* __restrict__ Q,
                                                                const double* __restrict__ S, double* bins,
                                                                uint32_t t0, uint32_t n_therm, uint32_t n_meas,
                                                                uint32_t every, uint32_t bin_size, uint32_t k0,
                                                                uint32_t k1, double* last_xy) {
    run_chain<St>(field, d, site, Q, S, bins, t0, n_therm, n_meas, every, bin_size, k0, k1, last_xy, false);
}

template <class St>
static hipError_t launch_batch_t(const BatchArgs& a, hipStream_t stream) {
    if (a.single) {
        hipLaunchKernelGGL(resident_chain<St>, dim3(1), dim3(kBatchThreads), 0, stream,
                           static_cast<typename St::T*>(a.field), a.single_desc, a.site, a.Q, a.S, a.bins, a.t0,
                           a.n_therm, a.n_meas, a.every, a.bin_size, a.k0, a.k1, a.last_xy);
    } else {
        hipLaunchKernelGGL(batch_chains<St>, dim3(a.n_chains), dim3(kBatchThreads), 0, stream,
                           static_cast<typename St::T*>(a.field), a.desc, a.order, a.site, a.Q, a.S, a.bins, a.t0,
                           a.n_therm, a.n_meas, a.every, a.bin_size, a.k0, a.k1);
    }
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, hipStream_t stream) {
    switch (a.storage) {
        case 0: return launch_batch_t<StoreF32>(a, stream);
        case 1: return launch_batch_t<StoreBF16>(a, stream);
        case 2: return launch_batch_t<StoreF16>(a, stream);
        case 3: return launch_batch_t<StoreBF16SR>(a, stream);
        case 4: return launch_batch_t<StoreF16SR>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace latcoul
