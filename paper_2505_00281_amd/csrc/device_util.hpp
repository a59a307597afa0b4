// device_util.hpp -- device-side helpers: storage-type tags and conversions,
// wave64/workgroup reductions and a bounded grid barrier for cooperative
// (co-resident) launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace ofrr {

// 16-bit storage tags (bit patterns held in uint16_t).
struct bf16_t {
    uint16_t bits;
};
struct f16_t {
    uint16_t bits;
};

// The conversions below round an FP32 value that has already been rounded
// to FP32.  The empty asm hides the value's origin from the compiler, which
// would otherwise fuse an FP32 fma followed by the conversion into one
// mixed-precision fma (v_fma_mixlo_f16) that rounds the exact result to
// binary16 once; FP32 arithmetic on 16-bit data rounds twice (to FP32, then
// to the storage type), and the tests compare against exactly that.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
    __asm__("" : "+v"(x));
    __bf16 h = (__bf16)x;  // round to nearest even (hardware conversion on gfx950)
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_bits(float x) {
    __asm__("" : "+v"(x));
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
}

// OCP e4m3fn, nearest value with ties to the even code, saturating at 448.
__device__ __forceinline__ uint8_t f32_to_e4m3_bits(float x) {
    const uint8_t sign = signbit(x) ? 0x80 : 0x00;
    float a = fabsf(x);
    if (a != a) return 0x7F | sign;
    if (a >= 448.f) return 0x7E | sign;
    if (a < 0x1.0p-6f) {
        // multiples of the smallest subnormal 2^-9; 8 * 2^-9 is the min normal
        int m = (int)rintf(a * 512.f);
        return (uint8_t)m | sign;
    }
    int e;
    float f = frexpf(a, &e);  // a = f 2^e, f in [0.5, 1)
    e -= 1;                   // a = (2f) 2^e, 2f in [1, 2)
    int mm = (int)rintf((2.f * f - 1.f) * 8.f);
    if (mm == 8) {
        mm = 0;
        e += 1;
    }
    return (uint8_t)(((e + 7) << 3) | mm) | sign;
}

__device__ __forceinline__ float e4m3_bits_to_f32(uint8_t c) {
    const int e = (c >> 3) & 15, m = c & 7;
    float v = e == 0 ? (float)m * 0x1.0p-9f : ldexpf(1.f + (float)m * 0.125f, e - 7);
    return (c & 0x80) ? -v : v;
}

// Generic loads/stores through FP64.
__device__ __forceinline__ double load_as_f64(const double *p) { return *p; }
__device__ __forceinline__ double load_as_f64(const float *p) { return (double)*p; }
__device__ __forceinline__ double load_as_f64(const bf16_t *p) { return (double)bf16_bits_to_f32(p->bits); }
__device__ __forceinline__ double load_as_f64(const f16_t *p) { return (double)f16_bits_to_f32(p->bits); }

template <class T>
__device__ __forceinline__ void store_as(T *p, double v);
template <>
__device__ __forceinline__ void store_as<double>(double *p, double v) { *p = v; }
template <>
__device__ __forceinline__ void store_as<float>(float *p, double v) { *p = (float)v; }
template <>
__device__ __forceinline__ void store_as<bf16_t>(bf16_t *p, double v) { p->bits = f32_to_bf16_bits((float)v); }
template <>
__device__ __forceinline__ void store_as<f16_t>(f16_t *p, double v) { p->bits = f32_to_f16_bits((float)v); }

// Column maxima of a row-major block, as order-preserving 32-bit keys of
// the magnitudes: the FP32 bits for FP32 and narrower element types, the
// upper word of the FP64 bits for FP64 (sign cleared: exponent and leading
// mantissa bits, so the largest key has the largest exponent over FP64's
// whole range; a column whose entries are all FP64 subnormals below 2^-1022
// keys as zero).  NaN or infinity gives all ones.
template <class T>
__device__ __forceinline__ unsigned mag_key(double v) {
    if (!(v == v) || isinf(v)) return 0xFFFFFFFFu;
    if constexpr (sizeof(T) == 8)
        return (unsigned)((unsigned long long)__double_as_longlong(fabs(v)) >> 32);
    else
        return __float_as_uint((float)fabs(v));
}

// 2^-e for the column maximum m = f 2^e, f in [1/2, 1) (the scaled column has
// infinity-norm in (1/2, 1]); 1 for a zero column; NaN for a NaN/Inf key.
template <class T>
__device__ __forceinline__ double key_scale(unsigned key) {
    if (key == 0xFFFFFFFFu) return __builtin_nan("");
    if (key == 0u) return 1.0;
    int e;
    if constexpr (sizeof(T) == 8)
        (void)frexp(__hiloint2double((int)key, 0), &e);
    else
        (void)frexpf(__uint_as_float(key), &e);
    return ldexp(1.0, -e);
}

// column maxima are merged into CM_COPIES copies of a 512-entry key array
// (block index mod CM_COPIES), which spreads the atomics of many blocks
constexpr int CM_COPIES = 4;

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ float wave_max_f32(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide reductions for blockDim.x a multiple of 64 (<= 1024).
__device__ __forceinline__ float block_max_f32(float v) {
    __shared__ float s[16];
    v = wave_max_f32(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) s[w] = v;
    __syncthreads();
    float r = s[0];
    for (int i = 1; i < nw; ++i) r = fmaxf(r, s[i]);
    __syncthreads();
    return r;
}
__device__ __forceinline__ bool block_any(bool v) { return __syncthreads_or(v ? 1 : 0) != 0; }

__device__ __forceinline__ double block_sum_f64(double v) {
    __shared__ double s[16];
    v = wave_sum_f64(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (l == 0) s[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += s[i];  // fixed order: deterministic
    __syncthreads();
    return r;
}

// -------------------------------------------------------------- grid barrier
//
// Counter-based barrier for a cooperative launch (every workgroup is
// co-resident).  `counter` starts at 0 and only grows; barrier number e
// (1-based) completes when it reaches e * nblocks.  The wait is bounded: on
// timeout the error flag is raised and false is returned, so that every
// workgroup still runs to completion.
__device__ __forceinline__ bool grid_barrier(unsigned *counter, unsigned nblocks, unsigned &epoch,
                                             int *err) {
    __shared__ int s_ok;
    // every thread's earlier global writes are released at device scope
    // before the workgroup arrives; every thread acquires after it leaves
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += 1;
        const unsigned target = epoch * nblocks;
        int ok = 1;
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > (1ull << 25)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool ok = s_ok != 0;
    __syncthreads();
    return ok;
}

}  // namespace ofrr
