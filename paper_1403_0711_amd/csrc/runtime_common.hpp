// Host-side helpers shared by the single-lattice and batch runtimes
// (internal): error reporting, device allocation, charge aggregation, the
// binned estimate and layout conversion.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lattice_coulomb.h"

namespace latcoul {

int set_error(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* where);

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// A named roctx range for the lifetime of the object (a runtime call as seen
// by rocprofv3 --marker-trace; nothing is recorded without a profiler).
class TraceRange {
  public:
    explicit TraceRange(const char* name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Device memory from the caller's provider, or hipMalloc/hipFree.
class DeviceAllocator {
  public:
    DeviceAllocator() = default;
    explicit DeviceAllocator(const lat_allocator* a) {
        if (a) {
            a_ = *a;
            custom_ = true;
        }
    }
    void* alloc(size_t bytes);
    void release(void* p);
    const lat_allocator* source() const { return custom_ ? &a_ : nullptr; }  // the caller's provider, if any

  private:
    lat_allocator a_{};
    bool custom_ = false;
};

// Charges summed per site.  site = c * vh + j (colour c, compact index j),
// sorted ascending; Q = sum of q, S = sum of q^2 on the site (summed in input
// order).  X = sum Q phi and Y = sum S phi^2 equal the raw-list sums of the
// paper's Eq. (nsum2).
struct AggregatedCharges {
    std::vector<uint32_t> site;
    std::vector<double> Q, S;
};
int aggregate_charges(int64_t n, const int32_t* xyz, const double* q, int64_t lx, int64_t ly, int64_t lz,
                      uint32_t vh, AggregatedCharges* out);

// Binned estimate from compensated bin sums (2 doubles per bin: sum, comp).
struct EstimateResult {
    double mean = 0.0;
    double stderr_binned = 0.0;
    int64_t full_bins = 0;
    bool finite = true;
};
EstimateResult estimate_from_bins(const double* bins, int64_t used_bins, int64_t n_samples, int64_t bin_size);

// Layout conversion between the two compact colour arrays (storage format)
// and natural order float (x fastest).
void compact_to_natural(const void* compact, int storage, int64_t lx, int64_t ly, int64_t lz, uint32_t vh,
                        float* out);
void natural_to_compact(const float* in, int storage, int64_t lx, int64_t ly, int64_t lz, uint32_t vh,
                        void* compact);

// Whether the fused (both colours per pass) sweep handles an lh x ly row shape.
bool fused_sweep_supported(uint32_t lh, uint32_t ly);

}  // namespace latcoul
