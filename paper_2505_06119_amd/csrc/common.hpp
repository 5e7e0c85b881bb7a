// Device helpers shared by the gfx950 kernels: complex arithmetic on
// float2/double2 storage with FP64 math, wavefront (64 lanes) and block
// reductions, and HIP error plumbing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MPS_WAVE 64

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---- complex helpers (storage type T = float2 or double2; math in double2) ----

__device__ __forceinline__ double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 to_d(double2 v) { return v; }

template <typename T> __device__ __forceinline__ T from_d(double2 v);
template <> __device__ __forceinline__ float2 from_d<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ double2 from_d<double2>(double2 v) { return v; }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b)
{
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 czero() { return make_double2(0.0, 0.0); }

// ---- reductions ----

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, MPS_WAVE);
    return v;
}

__device__ __forceinline__ double2 wave_sum(double2 v)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    return v;
}

// Sum over a 256-thread block; every thread receives the total.  `scratch`
// must hold 4 doubles (one per wave) and is reused after a barrier.
__device__ __forceinline__ double block_sum256(double v, double* scratch)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    return scratch[0] + scratch[1] + scratch[2] + scratch[3];
}

// (value, key, slot) argmax: larger value wins; equal values go to the
// smaller key (the original column index).
struct ArgBest {
    double val;
    int32_t key;
    int32_t slot;
};

__device__ __forceinline__ bool arg_better(double v1, int32_t k1, double v2, int32_t k2)
{
    return v1 > v2 || (v1 == v2 && k1 < k2);
}

__device__ __forceinline__ ArgBest wave_argmax(ArgBest a)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double v = __shfl_xor(a.val, off, MPS_WAVE);
        int32_t k = __shfl_xor(a.key, off, MPS_WAVE);
        int32_t s = __shfl_xor(a.slot, off, MPS_WAVE);
        if (arg_better(v, k, a.val, a.key)) { a.val = v; a.key = k; a.slot = s; }
    }
    return a;
}

// Block (256 threads) argmax; result valid in every thread.
__device__ __forceinline__ ArgBest block_argmax256(ArgBest a, ArgBest* scratch)
{
    a = wave_argmax(a);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = a;
    __syncthreads();
    ArgBest b = scratch[0];
    for (int w = 1; w < 4; ++w)
        if (arg_better(scratch[w].val, scratch[w].key, b.val, b.key)) b = scratch[w];
    return b;
}

// "Last block done" ticket: every block calls it after publishing its partial
// results; exactly one block (the last to arrive) gets true and may then read
// all partials.  The counter is reset by the last block for the next launch.
__device__ __forceinline__ bool last_block_ticket(unsigned int* counter, unsigned int nblocks, int* flag_lds)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int t = atomicAdd(counter, 1u);
        *flag_lds = (t == nblocks - 1) ? 1 : 0;
    }
    __syncthreads();
    bool last = *flag_lds != 0;
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return last;
}

// Loads that must observe writes made by other blocks of the same launch
// (published before a last_block_ticket) go around the non-coherent caches.
__device__ __forceinline__ double ld_coherent(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_coherent(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
