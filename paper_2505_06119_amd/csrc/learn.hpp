// Learned pivot proposal: a Gaussian sketch of theta, per-column sketch
// features, a small MLP that scores the columns, and the ranking that turns
// scores into a pivot order.  The pivoted QR then runs with that order fixed
// (no per-column pivot search); plain pivoted QR stays the fallback.
//
// Random numbers: the sketch matrix Omega (ell x m) is drawn from a
// counter-based generator -- the SplitMix64 output function (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
// applied to seed + (counter+1) * 0x9E3779B97F4A7C15 -- and the Box-Muller
// transform.  Entry (r, i) uses counters 2*(i*ell + r) and 2*(i*ell + r) + 1;
// it is a complex Gaussian with E|w|^2 = 1.
//
// Network: features phi (PN_F = 4 per column) -> tanh hidden layer (PN_H = 16)
// -> one linear score.  Parameters (float32, PN_P = 97):
//   W1[h*PN_F + f] (64), b1[h] (16), w2[h] (16), b2 (1).
#pragma once
#include "common.hpp"

#define PN_F 4
#define PN_H 16
#define PN_P (PN_H * PN_F + PN_H + PN_H + 1)

__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// uniform in (0, 1]: top 53 bits
__device__ __forceinline__ double u01(uint64_t x) { return ((double)(x >> 11) + 1.0) * (1.0 / 9007199254740992.0); }

template <typename T>
__global__ __launch_bounds__(256) void k_sketch_omega(T* Om, int64_t ell, int64_t m, uint64_t seed)
{
    const int64_t total = ell * m;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
        const int64_t r = q % ell, i = q / ell;     // column-major ell x m
        const uint64_t c0 = 2ull * (uint64_t)(i * ell + r);
        const double u1 = u01(splitmix64(seed, c0)), u2 = u01(splitmix64(seed, c0 + 1));
        const double rad = sqrt(-log(u1));           // |w|^2 ~ Exp(1): E|w|^2 = 1
        const double ang = 6.283185307179586 * u2;
        Om[q] = from_d<T>(make_double2(rad * cos(ang), rad * sin(ang)));
    }
}

// s[c] = ||Y[:, c]||^2 (FP64), one thread per column; Y is ell x n (ld ell).
template <typename T>
__global__ __launch_bounds__(256) void k_sketch_norms(const T* Y, int64_t ell, int64_t n, double* s)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    double acc = 0.0;
    for (int64_t r = 0; r < ell; ++r) acc += cabs2(to_d(Y[r + ell * c]));
    s[c] = acc;
}

// One block: mean and max of s and the index of the max (smallest index on ties).
__global__ __launch_bounds__(256) void k_sketch_stats(const double* s, int64_t n, double* stats)
{
    __shared__ double red[4];
    __shared__ ArgBest arg_lds[4];
    double sum = 0.0;
    ArgBest b;
    b.val = -1.0;
    b.key = 0x7fffffff;
    b.slot = -1;
    for (int64_t c = threadIdx.x; c < n; c += 256) {
        sum += s[c];
        if (arg_better_exact(s[c], (int32_t)c, b.val, b.key)) {
            b.val = s[c];
            b.key = (int32_t)c;
            b.slot = (int32_t)c;
        }
    }
    sum = block_sum256(sum, red);
    b = block_argmax256<true>(b, arg_lds);
    if (threadIdx.x == 0) {
        stats[0] = n > 0 ? sum / (double)n : 0.0;
        stats[1] = b.val;
        stats[2] = (double)b.slot;
    }
}

// phi[c] = (s_c/mean, log(s_c/mean + 1e-30), s_c/max, |<y_top, y_c>|^2 / (s_top s_c))
template <typename T>
__global__ __launch_bounds__(256) void k_sketch_features(const T* Y, int64_t ell, int64_t n, const double* s,
                                                         const double* stats, float* phi)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const double mean = stats[0] > 0.0 ? stats[0] : 1.0, mx = stats[1] > 0.0 ? stats[1] : 1.0;
    const int64_t top = (int64_t)stats[2];
    double2 dot = czero();
    for (int64_t r = 0; r < ell; ++r) dot = cadd(dot, cmulc(to_d(Y[r + ell * top]), to_d(Y[r + ell * c])));
    const double sc = s[c];
    const double st = s[top];
    const double rel = sc / mean;
    phi[c * PN_F + 0] = (float)rel;
    phi[c * PN_F + 1] = (float)log(rel + 1e-30);
    phi[c * PN_F + 2] = (float)(sc / mx);
    phi[c * PN_F + 3] = (float)(cabs2(dot) / (st * sc + 1e-300));
}

__device__ __forceinline__ float pn_forward_one(const float* p, const float* phi, float* a /* PN_H */)
{
    float out = p[PN_H * PN_F + 2 * PN_H];
#pragma unroll
    for (int h = 0; h < PN_H; ++h) {
        float z = p[PN_H * PN_F + h];
#pragma unroll
        for (int f = 0; f < PN_F; ++f) z += p[h * PN_F + f] * phi[f];
        a[h] = tanhf(z);
        out += p[PN_H * PN_F + PN_H + h] * a[h];
    }
    return out;
}

// scores[c] = MLP(phi[c])
__global__ __launch_bounds__(256) void k_pn_forward(const float* params, const float* phi, int64_t n, float* scores)
{
    __shared__ float p[PN_P];
    for (int q = threadIdx.x; q < PN_P; q += 256) p[q] = params[q];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    float a[PN_H];
    scores[c] = pn_forward_one(p, phi + c * PN_F, a);
}

// Per-block partial gradients of the mean binary cross-entropy with logits,
// L = (1/n) sum_c [softplus(s_c) - y_c s_c]; partial loss in slot PN_P.
// gpart: gridDim.x x (PN_P + 1) floats.
__global__ __launch_bounds__(256) void k_pn_grad(const float* params, const float* phi, const uint8_t* labels,
                                                 int64_t n, float* gpart)
{
    __shared__ float p[PN_P];
    __shared__ double red[4];
    for (int q = threadIdx.x; q < PN_P; q += 256) p[q] = params[q];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float g[PN_P + 1];
#pragma unroll
    for (int q = 0; q < PN_P + 1; ++q) g[q] = 0.f;
    if (c < n) {
        const float* x = phi + c * PN_F;
        float a[PN_H];
        const float s = pn_forward_one(p, x, a);
        const float y = labels[c] ? 1.f : 0.f;
        const float inv_n = 1.f / (float)n;
        const float sig = 1.f / (1.f + expf(-s));
        const float ds = (sig - y) * inv_n;
        g[PN_P] = (fmaxf(s, 0.f) - y * s + log1pf(expf(-fabsf(s)))) * inv_n;
        g[PN_H * PN_F + 2 * PN_H] = ds;                           // b2
#pragma unroll
        for (int h = 0; h < PN_H; ++h) {
            g[PN_H * PN_F + PN_H + h] = ds * a[h];                // w2
            const float dz = ds * p[PN_H * PN_F + PN_H + h] * (1.f - a[h] * a[h]);
            g[PN_H * PN_F + h] = dz;                              // b1
#pragma unroll
            for (int f = 0; f < PN_F; ++f) g[h * PN_F + f] = dz * x[f];   // W1
        }
    }
    for (int q = 0; q < PN_P + 1; ++q) {
        const double t = block_sum256((double)g[q], red);
        if (threadIdx.x == 0) gpart[(int64_t)blockIdx.x * (PN_P + 1) + q] = (float)t;
    }
}

// grad[q] = sum of the block partials in a fixed order (FP64); loss in grad[PN_P].
__global__ __launch_bounds__(128) void k_pn_grad_sum(const float* gpart, int nblocks, float* grad)
{
    const int q = threadIdx.x;
    if (q > PN_P) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += gpart[(int64_t)b * (PN_P + 1) + q];
    grad[q] = (float)s;
}

// Adam step (Kingma & Ba 2015) with bias correction; t >= 1.
__global__ __launch_bounds__(128) void k_pn_adam(float* params, const float* grad, float* m1, float* m2, int t,
                                                 float lr)
{
    const int q = threadIdx.x;
    if (q >= PN_P) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[q];
    m1[q] = b1 * m1[q] + (1.f - b1) * g;
    m2[q] = b2 * m2[q] + (1.f - b2) * g * g;
    const float mh = m1[q] / (1.f - powf(b1, (float)t));
    const float vh = m2[q] / (1.f - powf(b2, (float)t));
    params[q] -= lr * mh / (sqrtf(vh) + eps);
}

// order[rank(c)] = c, rank(c) = #{c' : score[c'] > score[c] or (== and c' < c)}.
// Exact ranking by counting, in LDS tiles of the score vector.  A NaN score
// counts as -infinity, so the ranks stay a permutation of 0..n-1 (every order
// slot is written) whatever the scores hold.
__device__ __forceinline__ float rank_key(float v) { return v != v ? -INFINITY : v; }

__global__ __launch_bounds__(256) void k_rank_desc(const float* scores, int64_t n, int32_t* order)
{
    __shared__ float tile[1024];
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float sc = c < n ? rank_key(scores[c]) : 0.f;
    int64_t rank = 0;
    for (int64_t t0 = 0; t0 < n; t0 += 1024) {
        __syncthreads();
        for (int q = threadIdx.x; q < 1024; q += 256)
            tile[q] = (t0 + q < n) ? rank_key(scores[t0 + q]) : -INFINITY;
        __syncthreads();
        const int64_t lim = (n - t0) < 1024 ? (n - t0) : 1024;
        for (int q = 0; q < lim; ++q) {
            const float o = tile[q];
            const int64_t c2 = t0 + q;
            rank += (o > sc || (o == sc && c2 < c)) ? 1 : 0;
        }
    }
    if (c < n) order[rank] = (int32_t)c;
}

// dst[:, j] = src[:, order[j]] (m rows), and perm[j] = order[j].  An entry
// outside [0, n) is clamped, so a corrupt order cannot read outside src.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_cols(const T* src, int64_t lds, T* dst, int64_t ldd, int64_t m,
                                                     const int32_t* order, int32_t* perm, int64_t n)
{
    const int64_t j = blockIdx.y;
    const int64_t o = order[j];
    const int64_t c = o < 0 ? 0 : (o >= n ? n - 1 : o);
    if (blockIdx.x == 0 && threadIdx.x == 0) perm[j] = (int32_t)c;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
        dst[i + ldd * j] = src[i + lds * c];
}

// One block: max over the per-block argmax partials (values) -> out[0];
// min over |diagR[0..k)| -> out[1].
__global__ __launch_bounds__(256) void k_certificate(const ArgBest* cpart, int nparts, const double* diagR,
                                                     int64_t k, double* out)
{
    __shared__ double red[4];
    __shared__ ArgBest arg_lds[4];
    ArgBest b;
    b.val = 0.0;
    b.key = 0x7fffffff;
    b.slot = -1;
    for (int q = threadIdx.x; q < nparts; q += 256)
        if (cpart[q].slot >= 0 && arg_better_exact(cpart[q].val, cpart[q].key, b.val, b.key)) b = cpart[q];
    b = block_argmax256<true>(b, arg_lds);
    double mn = 1e300;
    for (int64_t j = threadIdx.x; j < k; j += 256) mn = fmin(mn, fabs(diagR[j]));
    // block min via negated max of a sum-free reduction
    __shared__ double mins[256];
    mins[threadIdx.x] = mn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) mins[threadIdx.x] = fmin(mins[threadIdx.x], mins[threadIdx.x + s]);
        __syncthreads();
    }
    (void)red;
    if (threadIdx.x == 0) {
        out[0] = b.val;       // largest squared residual norm outside the selected set
        out[1] = mins[0];     // smallest |R_jj| inside it
    }
}
