// Host-side helpers of the runtime (see runtime_common.hpp).

#include "runtime_common.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace latcoul {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    (void)hipGetLastError();  // clear a sticky launch error so later calls can run
    return set_error(LAT_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void* DeviceAllocator::alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (custom_) return a_.alloc(a_.ctx, bytes);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void DeviceAllocator::release(void* p) {
    if (!p) return;
    if (custom_)
        a_.release(a_.ctx, p);
    else
        (void)hipFree(p);
}

int aggregate_charges(int64_t n, const int32_t* xyz, const double* q, int64_t lx, int64_t ly, int64_t lz,
                      uint32_t vh, AggregatedCharges* out) {
    std::vector<uint32_t> key((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (x < 0 || x >= lx || y < 0 || y >= ly || z < 0 || z >= lz)
            return set_error(LAT_ERR_ARG, "charge " + std::to_string(i) + " lies outside the lattice");
        if (!std::isfinite(q[i])) return set_error(LAT_ERR_ARG, "charge " + std::to_string(i) + " is not finite");
        const int64_t lin = x + lx * (y + ly * z);
        const uint32_t c = (uint32_t)((x + y + z) & 1);
        key[(size_t)i] = c * vh + (uint32_t)(lin >> 1);
    }
    std::vector<uint32_t> order((size_t)n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
    out->site.clear();
    out->Q.clear();
    out->S.clear();
    for (size_t k = 0; k < order.size(); ++k) {
        const uint32_t i = order[k];
        const double qi = q[i];
        if (out->site.empty() || out->site.back() != key[i]) {
            out->site.push_back(key[i]);
            out->Q.push_back(qi);
            out->S.push_back(qi * qi);
        } else {
            out->Q.back() += qi;
            out->S.back() += qi * qi;
        }
    }
    return LAT_OK;
}

EstimateResult estimate_from_bins(const double* bins, int64_t used_bins, int64_t n_samples, int64_t bin_size) {
    EstimateResult r;
    std::vector<double> tot((size_t)used_bins);
    for (int64_t b = 0; b < used_bins; ++b) {
        tot[(size_t)b] = bins[2 * b] - bins[2 * b + 1];  // Kahan: value = sum - compensation
        if (!std::isfinite(tot[(size_t)b])) r.finite = false;
    }
    // mean over all samples (compensated sum over bins)
    double s = 0.0, c = 0.0;
    for (double v : tot) {
        const double y = v - c;
        const double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    r.mean = n_samples > 0 ? s / (double)n_samples : 0.0;
    const int64_t nf = std::min<int64_t>(n_samples / bin_size, used_bins);  // full bins that are present
    r.full_bins = nf;
    if (nf < 2) {
        r.stderr_binned = NAN;
        return r;
    }
    double m = 0.0;
    for (int64_t b = 0; b < nf; ++b) m += tot[(size_t)b] / (double)bin_size;
    m /= (double)nf;
    double ss = 0.0;
    for (int64_t b = 0; b < nf; ++b) {
        const double d = tot[(size_t)b] / (double)bin_size - m;
        ss += d * d;
    }
    r.stderr_binned = std::sqrt(ss / ((double)nf * (double)(nf - 1)));
    return r;
}

static inline float bf16_bits_to_float(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
static inline uint16_t float_to_bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

void compact_to_natural(const void* compact, int storage, int64_t lx, int64_t ly, int64_t lz, uint32_t vh,
                        float* out) {
    for (int64_t z = 0; z < lz; ++z)
        for (int64_t y = 0; y < ly; ++y)
            for (int64_t x = 0; x < lx; ++x) {
                const int64_t i = x + lx * (y + ly * z);
                const size_t k = (size_t)((x + y + z) & 1) * vh + (size_t)(i >> 1);
                float v;
                if (storage == LAT_FP32)
                    v = static_cast<const float*>(compact)[k];
                else if (storage == LAT_BF16 || storage == LAT_BF16_SR)
                    v = bf16_bits_to_float(static_cast<const uint16_t*>(compact)[k]);
                else
                    v = (float)static_cast<const _Float16*>(compact)[k];
                out[i] = v;
            }
}

void natural_to_compact(const float* in, int storage, int64_t lx, int64_t ly, int64_t lz, uint32_t vh,
                        void* compact) {
    for (int64_t z = 0; z < lz; ++z)
        for (int64_t y = 0; y < ly; ++y)
            for (int64_t x = 0; x < lx; ++x) {
                const int64_t i = x + lx * (y + ly * z);
                const size_t k = (size_t)((x + y + z) & 1) * vh + (size_t)(i >> 1);
                if (storage == LAT_FP32)
                    static_cast<float*>(compact)[k] = in[i];
                else if (storage == LAT_BF16 || storage == LAT_BF16_SR)
                    static_cast<uint16_t*>(compact)[k] = float_to_bf16_rne(in[i]);
                else
                    static_cast<_Float16*>(compact)[k] = (_Float16)in[i];
            }
}

}  // namespace latcoul

extern "C" const char* lattice_last_error(void) { return latcoul::g_last_error.c_str(); }
