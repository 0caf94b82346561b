// Storage types of the filtered and decimated sinograms: FP32, FP16 and
// BF16.  Arithmetic is always FP32; these helpers convert on load and store
// (round to nearest even on store).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdkod {

template <int S> struct Store;

template <> struct Store<0> {
    using T = float;
    static __device__ __forceinline__ float cvt(T x) { return x; }
    static __device__ __forceinline__ float load(const T* p, size_t i) { return p[i]; }
    static __device__ __forceinline__ void put(T* p, size_t i, float v) { p[i] = v; }
    // load through a raw buffer resource at a byte offset (zero when out of range)
    static __device__ __forceinline__ float raw(__amdgpu_buffer_rsrc_t r, int off) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    // store through a raw buffer resource at a byte offset (dropped when out of range)
    static __device__ __forceinline__ void put_raw(__amdgpu_buffer_rsrc_t r, int off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
    }
    // the stored bits, unconverted (zero when out of range), and their value
    static __device__ __forceinline__ uint32_t raw_bits(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    }
    static __device__ __forceinline__ float from_bits(uint32_t b) { return __uint_as_float(b); }
};

template <> struct Store<1> {
    using T = _Float16;
    static __device__ __forceinline__ float cvt(T x) { return (float)x; }
    static __device__ __forceinline__ float load(const T* p, size_t i) { return (float)p[i]; }
    static __device__ __forceinline__ void put(T* p, size_t i, float v) { p[i] = (_Float16)v; }
    static __device__ __forceinline__ float raw(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return (float)__builtin_bit_cast(_Float16, h);
    }
    static __device__ __forceinline__ void put_raw(__amdgpu_buffer_rsrc_t r, int off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, off, 0, 0);
    }
    static __device__ __forceinline__ uint32_t raw_bits(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
    static __device__ __forceinline__ float from_bits(uint32_t b) {
        return (float)__builtin_bit_cast(_Float16, (unsigned short)b);
    }
};

template <> struct Store<2> {
    using T = uint16_t;  // bfloat16 bit pattern
    static __device__ __forceinline__ float cvt(T x) { return __uint_as_float(((uint32_t)x) << 16); }
    static __device__ __forceinline__ float load(const T* p, size_t i) {
        return __uint_as_float(((uint32_t)p[i]) << 16);
    }
    // round to nearest even; a NaN stays a (quiet) NaN.  Written as a select,
    // not a branch: a branch here splits the caller's arithmetic into blocks
    // and changes which of its multiplies and adds are fused
    static __device__ __forceinline__ uint16_t enc(float v) {
        const uint32_t b = __float_as_uint(v);
        const uint32_t rne = (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
        const uint32_t qnan = (b >> 16) | 0x40u;
        return (uint16_t)(v != v ? qnan : rne);
    }
    static __device__ __forceinline__ void put(T* p, size_t i, float v) { p[i] = enc(v); }
    static __device__ __forceinline__ float raw(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return __uint_as_float(((uint32_t)h) << 16);
    }
    static __device__ __forceinline__ void put_raw(__amdgpu_buffer_rsrc_t r, int off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)enc(v), r, off, 0, 0);
    }
    static __device__ __forceinline__ uint32_t raw_bits(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
    static __device__ __forceinline__ float from_bits(uint32_t b) { return __uint_as_float(b << 16); }
};

inline int store_bytes(int s) { return s == 0 ? 4 : 2; }

// A pointer that is the same in every lane, held in scalar registers.
template <class T>
__device__ __forceinline__ void* uniform_ptr(const T* p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// A structure read from global memory at a lane-uniform address, returned in
// scalar registers (every 32-bit word through readfirstlane).
template <class T>
__device__ __forceinline__ T uniform_load(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
    T out;
    const int* src = (const int*)uniform_ptr(p);
    int* dst = (int*)&out;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

// A table that no kernel writes while it runs, read at a lane-uniform
// address through the constant address space: scalar loads into scalar
// registers (through the generic address space the compiler cannot rule out
// a write, and issues vector loads that each wait on memory).
template <class T>
__device__ __forceinline__ T const_load(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
    typedef const __attribute__((address_space(4))) int* cword;
    const cword src = (cword)(p);
    T out;
    int* dst = (int*)&out;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return out;
}

// The volume v with start[v] <= b < start[v + 1] (start ascending, nvol >= 1,
// a read-only table; b lane-uniform): a binary search in scalar registers.
__device__ __forceinline__ int batch_volume(const int* start, int nvol, int b) {
    int lo = 0, hi = nvol - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (const_load(start + mid) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Wait for every outstanding vector memory access of the wave (s_waitcnt
// vmcnt(0) on gfx9 encodings; expcnt and lgkmcnt left at their maxima).  A
// kernel places it where every load it issued has been consumed, on every
// path: loads whose consumer sits in a branch that a wave skipped otherwise
// stay pending in the compiler's bookkeeping, and later code then waits on
// loads issued after them.
__device__ __forceinline__ void vmem_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Buffer resource over n elements of ES bytes at a lane-uniform address; raw
// loads through it return zero outside [0, n * ES).
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T* p, int n) {
    return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(p), (short)0, n * (int)sizeof(T), 0x00020000);
}

}  // namespace fdkod
