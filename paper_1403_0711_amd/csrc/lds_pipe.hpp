// LDS pipeline helpers of the slab kernels whose producer wave feeds LDS
// rings with direct buffer-to-LDS loads (gfx950).
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace latcoul {

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Direct buffer-to-LDS loads: each lane's `bytes` go to dst + lane * bytes.
// Non-template wrappers: the 16-byte form exists on gfx950 only, and a
// template kernel that names it directly is dropped by the host pass.
__device__ __forceinline__ void lds_load_b128(__amdgpu_buffer_rsrc_t r, lds_ptr_t dst, uint32_t voff,
                                              uint32_t soff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, soff, 0, 0);
}
__device__ __forceinline__ void lds_load_b32(__amdgpu_buffer_rsrc_t r, lds_ptr_t dst, uint32_t voff,
                                             uint32_t soff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 4, voff, soff, 0, 0);
}

// LDS reads of the producer wave.  The compiler makes any LDS access that
// follows a direct buffer-to-LDS load wait until all of them have landed
// (vmcnt 0), which would drain the plane ring at every step; these reads
// wait only for themselves (lgkmcnt 0), inside the asm statement that issues
// them, so no output register is left pending.  Addresses are LDS byte
// addresses.

__device__ __forceinline__ uint32_t lds_addr(const void* p) { return (uint32_t)(size_t)(lds_ptr_t)p; }

__device__ __forceinline__ uint32_t lds_read_u32(uint32_t a) {
    uint32_t r;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(r) : "v"(a) : "memory");
    return r;
}
// One entry's value (at a ring address) and its Q and S (LDS), one wait.
template <class St>
__device__ __forceinline__ void lds_read_entry(uint32_t av, uint32_t aq, uint32_t as, float& v, double& Qi,
                                               double& Si) {
    u32x2 q, sv;
    uint32_t r;
    if constexpr (St::kBytes == 4)
        asm volatile("ds_read_b32 %0, %3\n\tds_read_b64 %1, %4\n\tds_read_b64 %2, %5\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(r), "=&v"(q), "=&v"(sv)
                     : "v"(av), "v"(aq), "v"(as)
                     : "memory");
    else
        asm volatile("ds_read_u16 %0, %3\n\tds_read_b64 %1, %4\n\tds_read_b64 %2, %5\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(r), "=&v"(q), "=&v"(sv)
                     : "v"(av), "v"(aq), "v"(as)
                     : "memory");
    if constexpr (St::kBytes == 4)
        v = __uint_as_float(r);
    else if constexpr (std::is_same<typename St::Grid, StoreBF16>::value)
        v = __uint_as_float(r << 16);
    else
        v = (float)__builtin_bit_cast(_Float16, (uint16_t)r);
    Qi = __builtin_bit_cast(double, q);
    Si = __builtin_bit_cast(double, sv);
}

// s_waitcnt immediates (gfx9 encoding): vmcnt in bits 3:0 and 15:14, expcnt
// 6:4, lgkmcnt 11:8; a field at its maximum does not wait.
template <int kVm>
__device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(kVm >= 0 && kVm < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((kVm & 15) | (7 << 4) | (0 << 8) | ((kVm >> 4) << 14));
}

// The same wait with a count known only at run time (wave-uniform): one of
// the 64 immediate forms; a count beyond vmcnt's 6 bits waits for all loads.
__device__ __forceinline__ void wait_vm_lgkm0_n(uint32_t n) {
    switch (n) {
        case 0: wait_vm_lgkm0<0>(); break;
        case 1: wait_vm_lgkm0<1>(); break;
        case 2: wait_vm_lgkm0<2>(); break;
        case 3: wait_vm_lgkm0<3>(); break;
        case 4: wait_vm_lgkm0<4>(); break;
        case 5: wait_vm_lgkm0<5>(); break;
        case 6: wait_vm_lgkm0<6>(); break;
        case 7: wait_vm_lgkm0<7>(); break;
        case 8: wait_vm_lgkm0<8>(); break;
        case 9: wait_vm_lgkm0<9>(); break;
        case 10: wait_vm_lgkm0<10>(); break;
        case 11: wait_vm_lgkm0<11>(); break;
        case 12: wait_vm_lgkm0<12>(); break;
        case 13: wait_vm_lgkm0<13>(); break;
        case 14: wait_vm_lgkm0<14>(); break;
        case 15: wait_vm_lgkm0<15>(); break;
        case 16: wait_vm_lgkm0<16>(); break;
        case 17: wait_vm_lgkm0<17>(); break;
        case 18: wait_vm_lgkm0<18>(); break;
        case 19: wait_vm_lgkm0<19>(); break;
        case 20: wait_vm_lgkm0<20>(); break;
        case 21: wait_vm_lgkm0<21>(); break;
        case 22: wait_vm_lgkm0<22>(); break;
        case 23: wait_vm_lgkm0<23>(); break;
        case 24: wait_vm_lgkm0<24>(); break;
        case 25: wait_vm_lgkm0<25>(); break;
        case 26: wait_vm_lgkm0<26>(); break;
        case 27: wait_vm_lgkm0<27>(); break;
        case 28: wait_vm_lgkm0<28>(); break;
        case 29: wait_vm_lgkm0<29>(); break;
        case 30: wait_vm_lgkm0<30>(); break;
        case 31: wait_vm_lgkm0<31>(); break;
        case 32: wait_vm_lgkm0<32>(); break;
        case 33: wait_vm_lgkm0<33>(); break;
        case 34: wait_vm_lgkm0<34>(); break;
        case 35: wait_vm_lgkm0<35>(); break;
        case 36: wait_vm_lgkm0<36>(); break;
        case 37: wait_vm_lgkm0<37>(); break;
        case 38: wait_vm_lgkm0<38>(); break;
        case 39: wait_vm_lgkm0<39>(); break;
        case 40: wait_vm_lgkm0<40>(); break;
        case 41: wait_vm_lgkm0<41>(); break;
        case 42: wait_vm_lgkm0<42>(); break;
        case 43: wait_vm_lgkm0<43>(); break;
        case 44: wait_vm_lgkm0<44>(); break;
        case 45: wait_vm_lgkm0<45>(); break;
        case 46: wait_vm_lgkm0<46>(); break;
        case 47: wait_vm_lgkm0<47>(); break;
        case 48: wait_vm_lgkm0<48>(); break;
        case 49: wait_vm_lgkm0<49>(); break;
        case 50: wait_vm_lgkm0<50>(); break;
        case 51: wait_vm_lgkm0<51>(); break;
        case 52: wait_vm_lgkm0<52>(); break;
        case 53: wait_vm_lgkm0<53>(); break;
        case 54: wait_vm_lgkm0<54>(); break;
        case 55: wait_vm_lgkm0<55>(); break;
        case 56: wait_vm_lgkm0<56>(); break;
        case 57: wait_vm_lgkm0<57>(); break;
        case 58: wait_vm_lgkm0<58>(); break;
        case 59: wait_vm_lgkm0<59>(); break;
        case 60: wait_vm_lgkm0<60>(); break;
        case 61: wait_vm_lgkm0<61>(); break;
        case 62: wait_vm_lgkm0<62>(); break;
        case 63: wait_vm_lgkm0<63>(); break;
        default: wait_vm_lgkm0<0>(); break;
    }
}

// Workgroup barrier for the producer: its LDS writes were waited for above,
// and the asm statements keep the compiler from moving memory operations
// across the barrier.
__device__ __forceinline__ void producer_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Finalize of the previous sample by workgroup 0 of a launch: threads below
// kLoaders (the compute waves, which issue no direct-to-LDS loads) sum the
// partial pairs with several loads in flight each, every thread takes part in
// the workgroup sum, thread 0 records the sample.  It runs while the
// producer's first planes are in flight.
template <int kThreads, int kLoaders>
__device__ __forceinline__ void finalize_in_workgroup(const SampleFinalize& f) {
    constexpr int kUnroll = 4;  // few registers: this code shares the kernel's register budget
    const uint32_t t = threadIdx.x;
    double X = 0.0, Y = 0.0;
    if (t < (uint32_t)kLoaders) {
        const double2* p = reinterpret_cast<const double2*>(f.part);
        for (uint32_t b0 = 0; b0 < f.n; b0 += kLoaders * kUnroll) {
            double2 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) v[u] = p[min(b0 + (uint32_t)u * kLoaders + t, f.n - 1u)];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (b0 + (uint32_t)u * kLoaders + t < f.n) {
                    X += v[u].x;
                    Y += v[u].y;
                }
        }
    }
    block_sum2<kThreads>(X, Y);
    if (t == 0) record_sample(X, Y, f.bins, (f.m + (f.mdev ? f.mdev[0] : 0u)) / f.bin_size, f.last_xy);
}

}  // namespace latcoul
