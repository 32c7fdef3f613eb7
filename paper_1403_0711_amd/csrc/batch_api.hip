// Batch of independent chains (C ABI).  Not built yet: every call reports
// LAT_ERR_STATE.

#include "lattice_coulomb.h"
#include "runtime_common.hpp"

using namespace latcoul;

extern "C" {

int batch_create(int64_t, const int64_t*, const uint32_t*, int, uint64_t, const lat_allocator*, void*,
                 lattice_batch_t** out) {
    if (out) *out = nullptr;
    return set_error(LAT_ERR_STATE, "batched chains are not available in this build");
}
int batch_set_charges(lattice_batch_t*, int64_t, int64_t, const int32_t*, const double*) {
    return set_error(LAT_ERR_STATE, "batched chains are not available in this build");
}
int batch_run(lattice_batch_t*, int64_t, int64_t, int64_t) {
    return set_error(LAT_ERR_STATE, "batched chains are not available in this build");
}
int batch_energy_estimate(lattice_batch_t*, int64_t, double*, double*, int64_t*, int64_t*) {
    return set_error(LAT_ERR_STATE, "batched chains are not available in this build");
}
int batch_get_field(lattice_batch_t*, int64_t, float*) {
    return set_error(LAT_ERR_STATE, "batched chains are not available in this build");
}
void batch_destroy(lattice_batch_t*) {}

}  // extern "C"
