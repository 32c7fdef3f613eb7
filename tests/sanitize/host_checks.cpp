// Host code of the library and the C oracle exercised under AddressSanitizer
// and UndefinedBehaviorSanitizer (a host-only build, no GPU code): charge
// aggregation (duplicates, bounds, non-finite), the binned estimate (partial
// bins, too few bins, more samples than bins present, non-finite), the
// layout conversion round trip for every storage format on ragged shapes,
// and a few oracle sweeps with a gather.  Prints "ok" and exits 0 on success.

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "runtime_common.hpp"

extern "C" int64_t orc_run(double* phi, int64_t lx, int64_t ly, int64_t lz, int storage, uint64_t seed,
                           uint32_t chain, int64_t t0, int64_t n_sweeps, int64_t measure_every, int64_t n,
                           const int32_t* xyz, const double* q, double* samples);

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

int main() {
    using namespace latcoul;
    // aggregation: duplicates summed per site, sorted by (colour, compact index)
    {
        const int64_t lx = 6, ly = 3, lz = 2;
        const uint32_t vh = (uint32_t)(lx * ly * lz / 2);
        const int32_t xyz[] = {1, 1, 1, 0, 0, 0, 1, 1, 1, 5, 2, 1};
        const double q[] = {1.0, -2.0, 0.5, 3.0};
        AggregatedCharges a;
        CHECK(aggregate_charges(4, xyz, q, lx, ly, lz, vh, &a) == LAT_OK);
        CHECK(a.site.size() == 3);
        for (size_t k = 1; k < a.site.size(); ++k) CHECK(a.site[k - 1] < a.site[k]);
        double sq = 0.0, ss = 0.0;
        for (size_t k = 0; k < a.site.size(); ++k) {
            sq += a.Q[k];
            ss += a.S[k];
        }
        CHECK(std::fabs(sq - 2.5) < 1e-15 && std::fabs(ss - 14.25) < 1e-15);
        const int32_t out_of_box[] = {6, 0, 0};
        CHECK(aggregate_charges(1, out_of_box, q, lx, ly, lz, vh, &a) == LAT_ERR_ARG);
        const int32_t negative[] = {0, -1, 0};
        CHECK(aggregate_charges(1, negative, q, lx, ly, lz, vh, &a) == LAT_ERR_ARG);
        const double nan_q[] = {NAN};
        CHECK(aggregate_charges(1, xyz, nan_q, lx, ly, lz, vh, &a) == LAT_ERR_ARG);
        CHECK(aggregate_charges(0, nullptr, nullptr, lx, ly, lz, vh, &a) == LAT_OK && a.site.empty());
    }
    // binned estimate
    {
        std::vector<double> bins = {4.0, 0.0, 6.0, 0.0, 5.0, 0.0, 1.0, 0.0};  // 3 full bins of 2, one partial
        EstimateResult r = estimate_from_bins(bins.data(), 4, 7, 2);
        CHECK(r.full_bins == 3 && r.finite);
        CHECK(std::fabs(r.mean - 16.0 / 7.0) < 1e-15);
        CHECK(std::fabs(r.stderr_binned - std::sqrt(0.25 / 3.0)) < 1e-15);  // bin means 2, 3, 2.5
        r = estimate_from_bins(bins.data(), 1, 2, 2);
        CHECK(r.full_bins == 1 && std::isnan(r.stderr_binned));
        r = estimate_from_bins(bins.data(), 2, 100, 1);  // more samples than bins present
        CHECK(r.full_bins == 2);
        std::vector<double> bad = {1.0, 0.0, INFINITY, 0.0};
        CHECK(!estimate_from_bins(bad.data(), 2, 4, 2).finite);
        CHECK(estimate_from_bins(nullptr, 0, 0, 1).full_bins == 0);
    }
    // layout round trip (values exact in every storage format)
    {
        const int64_t shapes[][3] = {{2, 1, 1}, {6, 3, 2}, {10, 7, 5}, {16, 16, 16}};
        for (const auto& sh : shapes)
            for (int storage : {LAT_FP32, LAT_BF16, LAT_FP16, LAT_BF16_SR, LAT_FP16_SR}) {
                const int64_t lx = sh[0], ly = sh[1], lz = sh[2], V = lx * ly * lz;
                const uint32_t vh = (uint32_t)(V / 2);
                std::vector<float> in((size_t)V), back((size_t)V, -1.0f);
                for (int64_t i = 0; i < V; ++i) in[(size_t)i] = (float)((i % 17) - 8) * 0.25f;
                std::vector<unsigned char> comp(2 * (size_t)vh * (storage == LAT_FP32 ? 4 : 2));
                natural_to_compact(in.data(), storage, lx, ly, lz, vh, comp.data());
                compact_to_natural(comp.data(), storage, lx, ly, lz, vh, back.data());
                CHECK(std::memcmp(in.data(), back.data(), in.size() * sizeof(float)) == 0);
            }
    }
    // oracle: a few sweeps and samples on a small box
    {
        const int64_t lx = 8, ly = 6, lz = 5;
        std::vector<double> phi((size_t)(lx * ly * lz), 0.0);
        const int32_t xyz[] = {1, 1, 1, 6, 4, 3, 3, 2, 2};
        const double q[] = {1.0, -1.0, 0.5};
        std::vector<double> samples(3 * 10);
        for (int storage : {LAT_FP32, LAT_BF16, LAT_FP16, LAT_BF16_SR, LAT_FP16_SR}) {
            const int64_t m = orc_run(phi.data(), lx, ly, lz, storage, 7, 3, 0, 10, 1, 3, xyz, q, samples.data());
            CHECK(m == 10);
            for (double v : samples) CHECK(std::isfinite(v));
        }
    }
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
