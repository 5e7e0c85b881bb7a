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

// DPP row shift: lane l of each row of 16 lanes receives lane l - N of the
// same row; lanes without such a source receive `own` instead.  (Cross-lane
// data moves inside the VALU: no LDS round trip as with a shuffle.)
template <int N>
__device__ __forceinline__ int dpp_row_shr(int v, int own)
{
    return __builtin_amdgcn_update_dpp(own, v, 0x110 + N, 0xf, 0xf, false);
}
template <int N>
__device__ __forceinline__ double dpp_row_shr(double v, double own)
{
    const int lo = dpp_row_shr<N>(__double2loint(v), __double2loint(own));
    const int hi = dpp_row_shr<N>(__double2hiint(v), __double2hiint(own));
    return __hiloint2double(hi, lo);
}
// The value lane L holds (L a constant), in every lane.
__device__ __forceinline__ double lane_value(double v, int L)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), L),
                            __builtin_amdgcn_readlane(__double2loint(v), L));
}

// Wavefront sum, every lane receiving it: a scan inside each row of 16 lanes
// (row shifts 1, 2, 4, 8) leaves the row sums in lanes 15, 31, 47 and 63,
// which are then added in row order.  Called by all 64 lanes.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_row_shr<1>(v, 0.0);
    v += dpp_row_shr<2>(v, 0.0);
    v += dpp_row_shr<4>(v, 0.0);
    v += dpp_row_shr<8>(v, 0.0);
    return ((lane_value(v, 15) + lane_value(v, 31)) + lane_value(v, 47)) + lane_value(v, 63);
}

__device__ __forceinline__ double2 wave_sum(double2 v)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    return v;
}

// Wavefront reduce-scatter of NV doubles (NV a power of two, <= 64): at the
// level with exchange distance `off` every lane keeps one half of its values
// and receives its partner's copy of that half, so the values held per lane
// halve at each level (NV - 1 exchanges instead of 6 NV for NV all-reduces).
// On return lane L holds the wave total of value L / (64 / NV) (lanes that
// share that index hold the same total).
template <int NV>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[NV])
{
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
    const int lane = threadIdx.x & 63;
    if constexpr (NV > 1) {
        constexpr int H = NV / 2;
        constexpr int OFF = 32;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const double send = up ? v[q] : v[q + H];
            const double keep = up ? v[q + H] : v[q];
            v[q] = keep + __shfl_xor(send, OFF, MPS_WAVE);
        }
    }
    if constexpr (NV > 2) {
        constexpr int H = NV / 4;
        constexpr int OFF = 16;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const double send = up ? v[q] : v[q + H];
            const double keep = up ? v[q + H] : v[q];
            v[q] = keep + __shfl_xor(send, OFF, MPS_WAVE);
        }
    }
    if constexpr (NV > 4) {
        constexpr int H = NV / 8;
        constexpr int OFF = 8;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const double send = up ? v[q] : v[q + H];
            const double keep = up ? v[q + H] : v[q];
            v[q] = keep + __shfl_xor(send, OFF, MPS_WAVE);
        }
    }
    if constexpr (NV > 8) {
        constexpr int H = NV / 16;
        constexpr int OFF = 4;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const double send = up ? v[q] : v[q + H];
            const double keep = up ? v[q + H] : v[q];
            v[q] = keep + __shfl_xor(send, OFF, MPS_WAVE);
        }
    }
    if constexpr (NV > 16) {
        constexpr int H = NV / 32;
        constexpr int OFF = 2;
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const double send = up ? v[q] : v[q + H];
            const double keep = up ? v[q + H] : v[q];
            v[q] = keep + __shfl_xor(send, OFF, MPS_WAVE);
        }
    }
    if constexpr (NV > 32) {
        const bool up = (lane & 1) != 0;
        const double send = up ? v[0] : v[1];
        const double keep = up ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 1, MPS_WAVE);
    }
    double r = v[0];
#pragma unroll
    for (int off = 32 / NV; off > 0; off >>= 1) r += __shfl_xor(r, off, MPS_WAVE);
    return r;
}

// Block (256 threads) sum of NV doubles per thread into out[0..NV) (LDS),
// using lds[4 * NV] as staging; ends with a barrier, after which out[] is
// visible to every thread.  The per-wave totals are added in wave order.
template <int NV>
__device__ __forceinline__ void block_sum_rs(double (&v)[NV], double* lds, double* out)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double r = wave_reduce_scatter<NV>(v);
    constexpr int REP = 64 / NV;
    if (lane % REP == 0) lds[wid * NV + lane / REP] = r;
    __syncthreads();
    if (threadIdx.x < NV)
        out[threadIdx.x] = ((lds[threadIdx.x] + lds[NV + threadIdx.x]) + lds[2 * NV + threadIdx.x]) +
                           lds[3 * NV + threadIdx.x];
    __syncthreads();
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

// Pivot comparisons see a non-negative squared residual norm rounded to the
// nearest value with 40 significant mantissa bits (the low 12 bits rounded
// off): norms that agree to about 2^-41 relative count as equal and the
// smaller key wins.  A tie that is exact in exact arithmetic then resolves by
// key whatever last-bit rounding the evaluation of the two norms carried;
// rounding to nearest keeps simple values such as 1/2 or 1/4 in the middle of
// their interval, where a few ulps either way do not move them out of it.
__device__ __forceinline__ double pivot_key(double v)
{
    return __longlong_as_double((__double_as_longlong(v) + 0x800LL) & ~0xfffLL);
}

__device__ __forceinline__ bool arg_better(double v1, int32_t k1, double v2, int32_t k2)
{
    const double a = pivot_key(v1), b = pivot_key(v2);
    return a > b || (a == b && k1 < k2);
}

// The same order on the exact values (for maxima that are not pivot choices).
__device__ __forceinline__ bool arg_better_exact(double v1, int32_t k1, double v2, int32_t k2)
{
    return v1 > v2 || (v1 == v2 && k1 < k2);
}

template <bool EXACT, int N>
__device__ __forceinline__ void argmax_row_step(ArgBest& a)
{
    const double v = dpp_row_shr<N>(a.val, a.val);
    const int32_t k = dpp_row_shr<N>(a.key, a.key);
    const int32_t s = dpp_row_shr<N>(a.slot, a.slot);
    const bool better = EXACT ? arg_better_exact(v, k, a.val, a.key) : arg_better(v, k, a.val, a.key);
    if (better) { a.val = v; a.key = k; a.slot = s; }
}

template <bool EXACT>
__device__ __forceinline__ void argmax_take_lane(ArgBest& b, const ArgBest& a, int L)
{
    const double v = lane_value(a.val, L);
    const int32_t k = __builtin_amdgcn_readlane(a.key, L);
    const int32_t s = __builtin_amdgcn_readlane(a.slot, L);
    const bool better = EXACT ? arg_better_exact(v, k, b.val, b.key) : arg_better(v, k, b.val, b.key);
    if (better) { b.val = v; b.key = k; b.slot = s; }
}

// Wavefront argmax, every lane receiving it: a max-scan inside each row of
// 16 lanes, then the four row winners (lanes 15, 31, 47, 63).  The order is
// total (keys are distinct), so the winner does not depend on the grouping.
// Called by all 64 lanes.
template <bool EXACT = false>
__device__ __forceinline__ ArgBest wave_argmax(ArgBest a)
{
    argmax_row_step<EXACT, 1>(a);
    argmax_row_step<EXACT, 2>(a);
    argmax_row_step<EXACT, 4>(a);
    argmax_row_step<EXACT, 8>(a);
    ArgBest b;
    b.val = lane_value(a.val, 15);
    b.key = __builtin_amdgcn_readlane(a.key, 15);
    b.slot = __builtin_amdgcn_readlane(a.slot, 15);
    argmax_take_lane<EXACT>(b, a, 31);
    argmax_take_lane<EXACT>(b, a, 47);
    argmax_take_lane<EXACT>(b, a, 63);
    return b;
}

// Block (256 threads) argmax; result valid in every thread.  EXACT: on the
// exact values instead of the pivot comparison.
template <bool EXACT = false>
__device__ __forceinline__ ArgBest block_argmax256(ArgBest a, ArgBest* scratch)
{
    a = wave_argmax<EXACT>(a);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = a;
    __syncthreads();
    ArgBest b = scratch[0];
    for (int w = 1; w < 4; ++w) {
        const bool better = EXACT ? arg_better_exact(scratch[w].val, scratch[w].key, b.val, b.key)
                                  : arg_better(scratch[w].val, scratch[w].key, b.val, b.key);
        if (better) b = scratch[w];
    }
    return b;
}
