// Device building blocks of the heat-bath sweep: counter-based random
// numbers, the uniform -> Gaussian transform, field storage formats and
// wavefront reductions.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

#include "erfinv_coeffs.h"

namespace latcoul {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64-bit products on words 0 and 2, high halves xor-ed into the other
// words with the round key, key bumped by the Weyl constants between rounds.
// Counter words 1..3 and the key are wave-uniform here, so the compiler keeps
// them (and the first rounds' uniform products) on the scalar unit.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// a ^ b ^ c in one v_bitop3_b32 (gfx950's three-input bitwise op, truth
// table 0x96 = odd parity)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product per word: a single v_mad_u64_u32 (issued at
        // the integer rate, half the FP32 FMA rate on gfx950) instead of
        // separate low and high multiplies
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Heat-bath noise.  A 32-bit word u gives k = u >> 8 and the exact FP32
// s = 2r - 1 = (2k + 1 - 2^24) 2^-24 of the midpoint grid r = (k + 1/2) 2^-24.
// The noise of the paper's Eq. (phi), -erfc^{-1}(2r)/sqrt(3), equals
// erfinv(s)/sqrt(3); it is evaluated in Giles' two-region form with
// w = -log(1 - s^2) and coefficients fitted for this library
// (erfinv_coeffs.h, max relative error 3.3e-7 on the grid).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float grid_s(uint32_t u) {
    // ((u & ~0xFF) | 0x80) = 2^7 (2k + 1); flipping bit 31 subtracts 2^31, so as
    // a signed integer it is 2^7 (2k + 1 - 2^24): |.| < 2^31 with 24 significant
    // bits, exact in FP32.  Two integer ops (v_and_or_b32, v_xor_b32).
    const uint32_t v = ((u & 0xFFFFFF00u) | 0x80u) ^ 0x80000000u;
    return (float)(int)v * 0x1p-31f;
}

// The central polynomial is evaluated in every lane (its value at a tail
// lane's w is finite and discarded); the tail polynomial only in waves where
// some lane needs it, which is one wave branch instead of an if/else that
// splits the wave's lanes (the same arithmetic, so the same bits).
__device__ __forceinline__ float heatbath_noise(uint32_t u) {
    const float s = grid_s(u);
    const float omx2 = fmaf(-s, s, 1.0f);  // 1 - s^2, one rounding
    // v_log_f32 is log2: w - 2.5 = -ln(1 - s^2) - 2.5 in one fma
    const float wm = fmaf(__builtin_amdgcn_logf(omx2), -0.69314718055994531f, -2.5f);
    float p = kErfinvP[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) p = fmaf(p, wm, kErfinvP[i]);
    const bool tail = !(wm < LATCOUL_ERFINV_W_SPLIT - 2.5f);
    if (__builtin_amdgcn_ballot_w64(tail) != 0) {  // wave-uniform: about one wave in five
        const float x = __builtin_amdgcn_sqrtf(wm + 2.5f) - 3.0f;
        float q = kErfinvQ[8];
#pragma unroll
        for (int i = 7; i >= 0; --i) q = fmaf(q, x, kErfinvQ[i]);
        p = tail ? q : p;
    }
    return p * s;
}

// Heat-bath update of the 4 consecutive same-colour sites j0 .. j0+3 of one
// row (j0 % 4 == 0): bm/bn are the quads at planes z-1/z+1, up/dn at rows
// y-1/y+1, bc the other-colour quad at the same columns, e the other-colour
// value beyond the quad on the side p selects (p = (c + y + z) & 1: the
// x-neighbours of site k are other-colour columns k-1+p and k+p).  One
// Philox4x32-10 call with counter (j0/4, h, chain, 0) gives the 4 words;
// they are returned with the update, since the stochastically rounding
// storage formats draw their random bits from the words' low bytes (the
// uniform uses only the top 24 bits of a word).
struct QuadOut {
    float4 v;
    uint4 w;
};
__device__ __forceinline__ QuadOut heatbath_quad(const float4& bm, const float4& bc, const float4& bn,
                                                const float4& up, const float4& dn, float e, uint32_t p,
                                                uint32_t j0, uint32_t h, uint32_t chain, uint32_t k0,
                                                uint32_t k1) {
    float a0, a1, a2, a3;
    if (p == 0) {
        a0 = e + bc.x;
        a1 = bc.x + bc.y;
        a2 = bc.y + bc.z;
        a3 = bc.z + bc.w;
    } else {
        a0 = bc.x + bc.y;
        a1 = bc.y + bc.z;
        a2 = bc.z + bc.w;
        a3 = bc.w + e;
    }
    const uint4 r = philox4x32_10(j0 >> 2, h, chain, 0u, k0, k1);
    const float sixth = 1.0f / 6.0f;
    float4 out;
    out.x = fmaf(a0 + up.x + dn.x + bm.x + bn.x, sixth, heatbath_noise(r.x));
    out.y = fmaf(a1 + up.y + dn.y + bm.y + bn.y, sixth, heatbath_noise(r.y));
    out.z = fmaf(a2 + up.z + dn.z + bm.z + bn.z, sixth, heatbath_noise(r.z));
    out.w = fmaf(a3 + up.w + dn.w + bm.w + bn.w, sixth, heatbath_noise(r.w));
    return QuadOut{out, r};
}

// ---------------------------------------------------------------------------
// Raw buffer loads.  A buffer resource carries the array's size; a load at a
// byte offset >= that size returns 0 and fetches nothing (gfx9-family range
// check of raw buffers).  Kernels use this for Dirichlet ghosts and for lanes
// with nothing to load: such lanes get offset kNoLoad, which is out of range
// whenever the array is below 2 GiB (checked on the host), so no lane needs
// a predicate or a zeroing move.
// ---------------------------------------------------------------------------
constexpr uint32_t kNoLoad = 0x80000000u;
constexpr int kRawBufferDword3 = 0x00020000;  // gfx9-family raw buffer: no format conversion

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawBufferDword3);
}

__device__ __forceinline__ float4 bload_f32x4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}
__device__ __forceinline__ float bload_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// ---------------------------------------------------------------------------
// Field storage formats.  Arithmetic is always FP32.  A stored value is the
// FP32 update rounded to FP32 (no change), to BF16 or FP16 to nearest even,
// or to BF16 or FP16 stochastically (the SR formats: the same arrays as the
// round-to-nearest ones, only the rounding of an update differs).
//
// Stochastic rounding takes the 8 low bits u8 of the site's Philox word.
// With f the value's distance beyond the grid point below its magnitude, in
// grid spacings, and t = 256 f + u8, the magnitude goes up to the next grid
// point when t > 255.5, or t = 255.5 and u8 is even: over the 256 values of
// u8 it goes up in the nearest whole number of cases to 256 f (ties by the
// parity of u8), so the mean stored value is the FP32 value up to 1/512 of
// a spacing, with no drift toward or away from zero.
// ---------------------------------------------------------------------------
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Element i of an array as a 32-bit byte offset from its base (every array
// here is below 4 GiB), so loads use an SGPR base plus a VGPR offset instead
// of a 64-bit address per lane.
template <class V, class T>
__device__ __forceinline__ const V& at(const T* p, uint32_t i) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(p) + i * (uint32_t)sizeof(T));
}
template <class V, class T>
__device__ __forceinline__ V& at(T* p, uint32_t i) {
    return *reinterpret_cast<V*>(reinterpret_cast<char*>(p) + i * (uint32_t)sizeof(T));
}

// The FP32 value v as a register: the rounding to the storage format that
// follows cannot be folded into the FMA that produced v (a mixed-precision
// FMA rounds once, from the exact result), so every kernel stores the FP32
// update rounded to the storage format, and a value recomputed elsewhere
// rounds the same way.
__device__ __forceinline__ float fp32_reg(float v) {
    asm("" : "+v"(v));
    return v;
}

// Every format provides: T (array element), Grid (the round-to-nearest
// format of the same array, which readers use), Raw (a stored quad),
// ld/ld4/bld/bld4 (loads as FP32), unpack4, pack4 and pack1 (an updated
// quad or value with its Philox words, as stored), and through StoreOps the
// stores of updates st4/st4_nt/st and round4 (the value a store followed by
// a load returns).
template <class D>
struct StoreOps {
    template <class T>
    __device__ static __forceinline__ void st4(T* p, uint32_t i, float4 v, uint4 w) {
        at<typename D::Raw>(p, i) = D::pack4(v, w);
    }
    template <class T>
    __device__ static __forceinline__ void st4_nt(T* p, uint32_t i, float4 v, uint4 w) {
        __builtin_nontemporal_store(D::pack4(v, w), &at<typename D::Raw>(p, i));
    }
    template <class T>
    __device__ static __forceinline__ void st(T* p, uint32_t i, float v, uint32_t w) {
        at<T>(p, i) = D::pack1(v, w);
    }
    __device__ static __forceinline__ float4 round4(float4 v, uint4 w) { return D::unpack4(D::pack4(v, w)); }
};

struct StoreF32 : StoreOps<StoreF32> {
    using T = float;
    using Grid = StoreF32;
    using Raw = float4;
    static constexpr int kBytes = 4;
    static constexpr bool kSR = false;
    __device__ static __forceinline__ float ld(const T* p, uint32_t i) { return at<float>(p, i); }
    __device__ static __forceinline__ float4 ld4(const T* p, uint32_t i) { return at<float4>(p, i); }
    __device__ static __forceinline__ float4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t off) { return bload_f32x4(r, off); }
    __device__ static __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t off) { return bload_f32(r, off); }
    __device__ static __forceinline__ float4 unpack4(Raw r) { return r; }
    __device__ static __forceinline__ Raw pack4(float4 v, uint4) { return v; }
    __device__ static __forceinline__ float pack1(float v, uint32_t) { return v; }
    __device__ static __forceinline__ void st4_nt(T* p, uint32_t i, float4 v, uint4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(f4{v.x, v.y, v.z, v.w}, &at<f4>(p, i));
    }
};

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }
// Two values rounded to nearest even to BF16 and packed (a in the low half):
// gfx950's v_cvt_pk_bf16_f32, one instruction per pair instead of an integer
// rounding sequence per value; finite inputs only.
__device__ __forceinline__ uint32_t bf16x2_rne(float a, float b) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const f32x2 v = {fp32_reg(a), fp32_reg(b)};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// Stochastic rounding in hardware: gfx950's v_cvt_sr_bf16_f32 and
// v_cvt_sr_f16_f32 round with a 32-bit random operand R.  For BF16, with d
// the FP32 word's low 16 bits, the magnitude goes up when d plus R's top 16
// bits reaches 2^16; for FP16, with d the 13 dropped bits, when d plus R's
// top 13 bits reaches 2^13 (on the subnormal grid below 2^-14 the dropped
// fraction, which then has more bits, is first truncated to 13: there the
// device rounds down where the rule rounds up for about 1/64 of values,
// those just above a tie with an odd u8).  The rule above, with t = 256 f + u8 and f = d / 2^16 (BF16) or
// d / 2^13, is up when t > 255.5, and at a tie t = 255.5 when u8 is even:
// top bits 256 u8 + 128 - (u8 & 1) (BF16) or 32 u8 + 16 - (u8 & 1) (FP16).
// A tie needs d to end in exactly half of a 1/256 step, which 1/256 (BF16)
// and 1/32 (FP16) of FP32 values do: sending every tie up would move
// magnitudes away from zero on average (by 2^-25 of the value, a negative
// mass term), so ties go by the parity of u8.  One operand serves both
// formats: u8 in the top byte and 0x80 - (u8 & 1) in the next (FP16 reads
// its top 5 bits, 16 - (u8 & 1)), built by one byte permute (the top byte
// from w, the next from the sign of w << 15, i.e. 0x00 or 0xFF by u8 & 1)
// and an xor.  Checked bit for bit against the rule on 2^20 values (normal
// values, values next to powers of two, exact ties, zeros; FP16 subnormals
// as stated).
__device__ __forceinline__ uint32_t sr_operand(uint32_t w) {
    return __builtin_amdgcn_perm(w, w << 15, 0x04080C0Cu) ^ 0x800000u;
}
// Each conversion writes one half of its destination and keeps the other, so
// the pair starts from a's own register (both halves are overwritten), which
// needs no zeroing move.
__device__ __forceinline__ uint32_t bf16x2_sr(float a, float b, uint32_t wa, uint32_t wb) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const float ra = fp32_reg(a);
    bf16x2 o = __builtin_bit_cast(bf16x2, ra);
    o = __builtin_amdgcn_cvt_sr_bf16_f32(o, ra, sr_operand(wa), false);
    o = __builtin_amdgcn_cvt_sr_bf16_f32(o, fp32_reg(b), sr_operand(wb), true);
    return __builtin_bit_cast(uint32_t, o);
}

struct Bf16Array {
    using T = uint16_t;
    using Raw = u32x2;
    static constexpr int kBytes = 2;
    __device__ static __forceinline__ float ld(const T* p, uint32_t i) { return bf16_to_f32(at<uint16_t>(p, i)); }
    __device__ static __forceinline__ float4 unpack4(Raw w) {
        return make_float4(__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xFFFF0000u),
                           __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xFFFF0000u));
    }
    __device__ static __forceinline__ float4 ld4(const T* p, uint32_t i) { return unpack4(at<Raw>(p, i)); }
    __device__ static __forceinline__ float4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return unpack4(Raw{w[0], w[1]});
    }
    __device__ static __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
    }
};
struct StoreBF16 : Bf16Array, StoreOps<StoreBF16> {
    using Grid = StoreBF16;
    static constexpr bool kSR = false;
    __device__ static __forceinline__ Raw pack4(float4 v, uint4) {
        return Raw{bf16x2_rne(v.x, v.y), bf16x2_rne(v.z, v.w)};
    }
    __device__ static __forceinline__ T pack1(float v, uint32_t) { return (T)(bf16x2_rne(v, 0.0f) & 0xFFFFu); }
};
struct StoreBF16SR : Bf16Array, StoreOps<StoreBF16SR> {
    using Grid = StoreBF16;
    static constexpr bool kSR = true;
    __device__ static __forceinline__ Raw pack4(float4 v, uint4 w) {
        return Raw{bf16x2_sr(v.x, v.y, w.x, w.y), bf16x2_sr(v.z, v.w, w.z, w.w)};
    }
    __device__ static __forceinline__ T pack1(float v, uint32_t w) { return (T)(bf16x2_sr(v, 0.0f, w, 0u) & 0xFFFFu); }
};

__device__ __forceinline__ _Float16 to_f16(float v) { return (_Float16)fp32_reg(v); }
// Two values stochastically rounded to FP16 and packed (a in the low half).
__device__ __forceinline__ uint32_t f16x2_sr(float a, float b, uint32_t wa, uint32_t wb) {
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    const float ra = fp32_reg(a);
    f16x2 o = __builtin_bit_cast(f16x2, ra);  // both halves are overwritten (as in bf16x2_sr)
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, ra, sr_operand(wa), false);
    o = __builtin_amdgcn_cvt_sr_f16_f32(o, fp32_reg(b), sr_operand(wb), true);
    return __builtin_bit_cast(uint32_t, o);
}

struct F16Array {
    using T = _Float16;
    using Raw = u32x2;
    static constexpr int kBytes = 2;
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    __device__ static __forceinline__ float ld(const T* p, uint32_t i) { return (float)at<_Float16>(p, i); }
    __device__ static __forceinline__ float4 unpack4(Raw w) {
        const h4 hv = __builtin_bit_cast(h4, w);
        return make_float4((float)hv[0], (float)hv[1], (float)hv[2], (float)hv[3]);
    }
    __device__ static __forceinline__ float4 ld4(const T* p, uint32_t i) { return unpack4(at<Raw>(p, i)); }
    __device__ static __forceinline__ float4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return unpack4(Raw{w[0], w[1]});
    }
    __device__ static __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
    }
    __device__ static __forceinline__ uint32_t pair(_Float16 a, _Float16 b) {
        return __builtin_bit_cast(uint32_t, h2{a, b});
    }
};
struct StoreF16 : F16Array, StoreOps<StoreF16> {
    using Grid = StoreF16;
    static constexpr bool kSR = false;
    __device__ static __forceinline__ Raw pack4(float4 v, uint4) {
        return Raw{pair(to_f16(v.x), to_f16(v.y)), pair(to_f16(v.z), to_f16(v.w))};
    }
    __device__ static __forceinline__ T pack1(float v, uint32_t) { return to_f16(v); }
};
struct StoreF16SR : F16Array, StoreOps<StoreF16SR> {
    using Grid = StoreF16;
    static constexpr bool kSR = true;
    __device__ static __forceinline__ Raw pack4(float4 v, uint4 w) {
        return Raw{f16x2_sr(v.x, v.y, w.x, w.y), f16x2_sr(v.z, v.w, w.z, w.w)};
    }
    __device__ static __forceinline__ T pack1(float v, uint32_t w) {
        return __builtin_bit_cast(T, (uint16_t)(f16x2_sr(v, 0.0f, w, 0u) & 0xFFFFu));
    }
};

// FP16 arrays (either rounding) hold raw halves that the FP16 update adds
// in mixed-precision FMAs.
template <class St>
constexpr bool kF16Grid = std::is_same<typename St::Grid, StoreF16>::value;

// FP16 storage: the update of heatbath_quad on raw halves (element k of a
// quad in half k & 1 of word k >> 1).  Each f16 term joins its FP32 sum in
// one mixed-precision FMA, value * 1 + sum: the exact conversion and the
// FP32 add of the float path, rounded once as that add is, in the same
// order, so the result is bit for bit heatbath_quad's.
template <bool kHi>
__device__ __forceinline__ float add_f16(uint32_t w, float acc) {  // half kHi of w, plus acc
    float r;
    if constexpr (kHi)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(acc));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(acc));
    return r;
}
template <bool kHiA, bool kHiB>
__device__ __forceinline__ float add_f16_pair(uint32_t a, uint32_t b) {  // half kHiA of a plus half kHiB of b
    float r;
    if constexpr (!kHiA && !kHiB)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else if constexpr (!kHiA && kHiB)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else if constexpr (kHiA && !kHiB)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ QuadOut heatbath_quad_f16(u32x2 bm, u32x2 bc, u32x2 bn, u32x2 up, u32x2 dn, uint32_t e,
                                                    uint32_t p, uint32_t j0, uint32_t h, uint32_t chain, uint32_t k0,
                                                    uint32_t k1) {
    float a0, a1, a2, a3;  // e + x, x + y, y + z, z + w (p = 0); x + y, y + z, z + w, w + e (p = 1)
    if (p == 0) {
        a0 = add_f16_pair<false, false>(e, bc[0]);
        a1 = add_f16_pair<false, true>(bc[0], bc[0]);
        a2 = add_f16_pair<true, false>(bc[0], bc[1]);
        a3 = add_f16_pair<false, true>(bc[1], bc[1]);
    } else {
        a0 = add_f16_pair<false, true>(bc[0], bc[0]);
        a1 = add_f16_pair<true, false>(bc[0], bc[1]);
        a2 = add_f16_pair<false, true>(bc[1], bc[1]);
        a3 = add_f16_pair<true, false>(bc[1], e);
    }
    const uint4 r = philox4x32_10(j0 >> 2, h, chain, 0u, k0, k1);
    const float sixth = 1.0f / 6.0f;
    float4 out;
    out.x = fmaf(add_f16<false>(bn[0], add_f16<false>(bm[0], add_f16<false>(dn[0], add_f16<false>(up[0], a0)))),
                 sixth, heatbath_noise(r.x));
    out.y = fmaf(add_f16<true>(bn[0], add_f16<true>(bm[0], add_f16<true>(dn[0], add_f16<true>(up[0], a1)))), sixth,
                 heatbath_noise(r.y));
    out.z = fmaf(add_f16<false>(bn[1], add_f16<false>(bm[1], add_f16<false>(dn[1], add_f16<false>(up[1], a2)))),
                 sixth, heatbath_noise(r.z));
    out.w = fmaf(add_f16<true>(bn[1], add_f16<true>(bm[1], add_f16<true>(dn[1], add_f16<true>(up[1], a3)))), sixth,
                 heatbath_noise(r.w));
    return QuadOut{out, r};
}

// The neighbours of the quad at compact index j0 of a row, read straight
// from the other colour's array (0 beyond the box faces; p and the quad's
// position decide which x-neighbour beyond the quad is read), and the
// update computed from them.  FP16 storage keeps the raw halves.  Split so
// that a thread can have the loads of several quads in flight.
template <class St, bool kF16 = kF16Grid<St>>
struct QuadNeighbours {
    using Quad = float4;
    Quad cen, ym, yp, zm, zp;
    float e;
};
template <class St>
struct QuadNeighbours<St, true> {
    using Quad = u32x2;
    Quad cen, ym, yp, zm, zp;
    uint32_t e;
};

template <class St>
__device__ __forceinline__ QuadNeighbours<St> quad_load_global(const typename St::T* other, uint32_t j0, uint32_t lh,
                                                              uint32_t plane, bool ym_in, bool yp_in, bool zm_in,
                                                              bool zp_in, bool e_in, uint32_t p) {
    const uint32_t je = p == 0 ? j0 - 1u : j0 + 4u;  // the x-neighbour beyond the quad
    QuadNeighbours<St> nb;
    if constexpr (kF16Grid<St>) {
        const u32x2 zero = {0u, 0u};
        nb.cen = at<u32x2>(other, j0);
        nb.ym = ym_in ? at<u32x2>(other, j0 - lh) : zero;
        nb.yp = yp_in ? at<u32x2>(other, j0 + lh) : zero;
        nb.zm = zm_in ? at<u32x2>(other, j0 - plane) : zero;
        nb.zp = zp_in ? at<u32x2>(other, j0 + plane) : zero;
        nb.e = e_in ? (uint32_t)at<uint16_t>(other, je) : 0u;
    } else {
        const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
        nb.cen = St::ld4(other, j0);
        nb.ym = ym_in ? St::ld4(other, j0 - lh) : zero;
        nb.yp = yp_in ? St::ld4(other, j0 + lh) : zero;
        nb.zm = zm_in ? St::ld4(other, j0 - plane) : zero;
        nb.zp = zp_in ? St::ld4(other, j0 + plane) : zero;
        nb.e = e_in ? St::ld(other, je) : 0.f;
    }
    return nb;
}

template <class St>
__device__ __forceinline__ QuadOut quad_update_from(const QuadNeighbours<St>& nb, uint32_t p, uint32_t j0, uint32_t h,
                                                   uint32_t chain, uint32_t k0, uint32_t k1) {
    if constexpr (kF16Grid<St>)
        return heatbath_quad_f16(nb.zm, nb.cen, nb.zp, nb.ym, nb.yp, nb.e, p, j0, h, chain, k0, k1);
    else
        return heatbath_quad(nb.zm, nb.cen, nb.zp, nb.ym, nb.yp, nb.e, p, j0, h, chain, k0, k1);
}

template <class St>
__device__ __forceinline__ QuadOut quad_update_global(const typename St::T* other, uint32_t j0, uint32_t lh,
                                                     uint32_t plane, bool ym_in, bool yp_in, bool zm_in, bool zp_in,
                                                     bool e_in, uint32_t p, uint32_t h, uint32_t chain, uint32_t k0,
                                                     uint32_t k1) {
    return quad_update_from<St>(quad_load_global<St>(other, j0, lh, plane, ym_in, yp_in, zm_in, zp_in, e_in, p), p,
                                j0, h, chain, k0, k1);
}

// ---------------------------------------------------------------------------
// Wave64 FP64 sum by DPP data movement (each 32-bit half moved separately,
// the add in FP64): xor-1 and xor-2 quad permutes, row half-mirror and row
// mirror leave every lane of a 16-lane row holding the row sum; row_bcast:15
// and row_bcast:31 then fold the four rows into lane 63.  Fixed order, so the
// result is deterministic.  Returns the total in every lane (readlane 63).
// ---------------------------------------------------------------------------
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, kRowMask, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl, kRowMask, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_move<0x140, 0xF>(v);  // row_mirror
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Block sum of two FP64 values over kThreads threads (multiple of 64); the
// result is valid in every thread.  Fixed order: waves reduced by wave_sum,
// then wave totals added in wave order.
template <int kThreads>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
    constexpr int kWaves = kThreads / 64;
    __shared__ double sa[kWaves], sb[kWaves];
    a = wave_sum(a);
    b = wave_sum(b);
    const int wid = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sa[wid] = a;
        sb[wid] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        ta += sa[w];
        tb += sb[w];
    }
    a = ta;
    b = tb;
    __syncthreads();
}

// Record one sample (X, Y): O = X^2 - Y added to bin `bin` (bins[2b] running
// sum, bins[2b+1] the Kahan compensation, the lost low part negated), and
// (X, Y) kept in last_xy.  One thread.
__device__ __forceinline__ void record_sample(double X, double Y, double* bins, uint32_t bin, double* last_xy) {
    const double O = X * X - Y;
    double sum = bins[2 * bin];
    double comp = bins[2 * bin + 1];
    const double yk = O - comp;
    const double tk = sum + yk;
    comp = (tk - sum) - yk;
    sum = tk;
    bins[2 * bin] = sum;
    bins[2 * bin + 1] = comp;
    last_xy[0] = X;
    last_xy[1] = Y;
}

}  // namespace latcoul
