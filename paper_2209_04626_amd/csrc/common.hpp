// Device helpers shared by the gfx950 kernels: wavefront reductions, MFMA
// wrappers and small numeric traits.  Wavefront size is 64 throughout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#define MPJ_WAVE 64

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Butterfly sum over the 64 lanes of a wavefront; every lane gets the total.
// The summation tree is fixed, so results are bitwise reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, MPJ_WAVE);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, MPJ_WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, MPJ_WAVE));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, MPJ_WAVE));
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, MPJ_WAVE);
    return v;
}

// Sum over a whole workgroup of NT threads (NT a multiple of 64).  `red`
// must hold NT/64 entries of T in LDS.  All threads receive the result.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    v = wave_sum(v);
    const int w = threadIdx.x / MPJ_WAVE, l = threadIdx.x % MPJ_WAVE;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int i = 0; i < NT / MPJ_WAVE; ++i) s += red[i];
    return s;
}

template <int NT>
__device__ __forceinline__ int block_or(int v, int *red) {
    v = wave_or(v);
    const int w = threadIdx.x / MPJ_WAVE, l = threadIdx.x % MPJ_WAVE;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int i = 0; i < NT / MPJ_WAVE; ++i) s |= red[i];
    return s;
}

// Loads and stores that are coherent across the chip's L2 caches (relaxed
// atomics at device scope).  Workgroups of one launch exchange data through
// them: the writer stores with coh_store, waits for its stores to complete
// (publish_fence), then one thread raises a flag with coh_store after a
// barrier; the reader polls the flag with coh_load and reads the data with
// coh_load.  No cache-wide write-back or invalidate is involved.
template <typename U>
__device__ __forceinline__ void coh_store(U *p, U v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U>
__device__ __forceinline__ U coh_load(const U *p) {
    return __hip_atomic_load(const_cast<U *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every thread's coherent stores complete before the barrier that precedes
// the flag: s_waitcnt vmcnt(0).  (A workgroup-scope release fence emits no
// wait on gfx950, and stores to different addresses may complete out of
// order, so without it the flag could become visible before the data.)
__device__ __forceinline__ void publish_fence() {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unchanged
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

// 16-byte form of coh_load for FP32 data: a buffer load with the same cache
// policy (sc1) as a device-scope relaxed atomic load.  byte_off from base,
// 16-byte aligned.
__device__ __forceinline__ flt4 coh_load4(const float *base, int byte_off) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), 0, 0x7fffffff, 0x00020000);
    return __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off, 0, 16);
}

// 16x16x4 MFMA, FP64 and FP32.  Operand layout for lane l of the wavefront:
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): column l % 16; accumulator element r holds row
//                mfma_row<T>(l, r): 4 (l / 16) + r for FP32, but
//                l / 16 + 4 r for FP64 (rows interleaved across lane groups).
// (Both checked on gfx950 with a one-wavefront probe.)
__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma16(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int mfma_row(int lane, int r);
template <> __device__ __forceinline__ int mfma_row<double>(int lane, int r) { return lane / 16 + 4 * r; }
template <> __device__ __forceinline__ int mfma_row<float>(int lane, int r) { return 4 * (lane / 16) + r; }

template <typename T> struct acc4;
template <> struct acc4<double> { typedef dbl4 type; };
template <> struct acc4<float> { typedef flt4 type; };

template <typename T> __device__ __forceinline__ T tsqrt(T x);
template <> __device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline long long cdivl(long long a, long long b) { return (a + b - 1) / b; }

// Round-robin (circle method) tournament on nb players: in round r
// (0 <= r < nb - 1, nb even) slot 0 pairs r with nb - 1 and slot k pairs
// (r + k) mod (nb - 1) with (r - k) mod (nb - 1).  Returns lo < hi.
__host__ __device__ inline void rr_slot(int nb, int r, int k, int *lo, int *hi) {
    int a, b;
    if (k == 0) { a = r; b = nb - 1; }
    else {
        const int M = nb - 1;
        a = (r + k) % M;
        b = ((r - k) % M + M) % M;
    }
    *lo = a < b ? a : b;
    *hi = a < b ? b : a;
}
