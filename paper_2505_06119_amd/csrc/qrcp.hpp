// Column-pivoted Householder QR on the GPU, with the trailing-matrix update
// delayed over a panel of columns (the BLAS-3 formulation of pivoted QR by
// Quintana-Orti, Sun and Bischof, SIAM J. Sci. Comput. 19, 1998).
//
// theta (m x n, column-major, complex64 or complex128 storage) is factorised
// in place.  Inside a panel that starts at column p0 the trailing block keeps
// its panel-start values A_ps; the reflectors applied so far are carried as
//     A_current = A_ps - V F^H,
// with V the stored Householder vectors (unit lower trapezoidal, columns
// p0..j-1 of theta) and F (n x nb).  One pivot step j costs two launches:
//
//   step A  (rows split over blocks)  every block first reduces the argmax
//           partials of the previous launch to the pivot p; then the pivot
//           swap, the bring-up of the pivot column (x = A_ps[:, j] - V F[j, :]^H)
//           and per-block partial sums of ||x||^2 and V^H x.
//   step C  (columns split over blocks)  every block first reduces step A's
//           partials to the reflector (beta, tau, scale in FP64) and
//           aux = V^H v; then the GEMV w = A_ps^H v over the whole trailing
//           block (the HBM-bound part), the new F column
//           F[:, jj] = tau (w - F aux), the pivot row of R, the FP64 downdate
//           of the residual column norms and a per-block argmax partial.
//
// The redundant per-block reductions replace in-kernel cross-block
// synchronisation: partial results only cross a kernel boundary, so no block
// ever waits for or fences against another.
//
// At the end of a panel the host launches the MFMA update
// A[j:, j:] -= V F^H.  A residual norm whose downdated value has fallen below
// tol times its last exact value ends the panel early; all remaining norms are
// then recomputed exactly from the updated trailing block (robust downdating
// in the sense of Drmac and Bujanovic, 2008).
//
// Householder convention: beta = -sign(Re alpha) ||x||, tau = (beta-alpha)/beta,
// v = (1, x_rest/(alpha-beta)); H = I - tau v v^H and H^H x = beta e_1; a
// column with x_rest = 0 and real alpha gets tau = 0 (H = I).
#pragma once
#include "common.hpp"

#define QR_NBMAX 64
#define QR_CW 4            // columns per block in step C and the norm kernel

enum {
    CTL_PIV = 0,      // pivot position of the current step (written by step A)
    CTL_STOP = 1,     // panel must end: a norm needs recomputing
    CTL_JDONE = 2,    // number of completed steps
    CTL_TFAIL = 3,    // window panels: first step whose greedy replay fails
    CTL_TFLAG = 4,    // window panels: first step after which a norm needs recomputing, plus one
    CTL_COUNT = 16
};
enum { DSC_NORM2 = 0, DSC_EPS2 = 1, DSC_COUNT = 8 };

template <typename T>
struct QrcpDev {
    T* A;
    int64_t lda, m, n, k;
    double* nu;
    double* nuref;
    int32_t* perm;
    T* F;
    int64_t ldf;
    double2* tau;
    double* diagR;
    double2* xbuf;     // pivot column after bring-up, FP64
    T* xlo;            // the same in storage precision (vector GEMV operand)
    double* apart;     // step-A partials, (2 + 2*QR_NBMAX) doubles per block
    double2* hh;       // [0] alpha (written by the block holding row j)
    double2* fsave;    // QR_NBMAX
    double* pivval;    // QR_NBMAX: downdated norm of each step's pivot at its step
    int32_t* pivkey;   // QR_NBMAX: its key (original column index)
    ArgBest* cpart;    // argmax partials of the last producer (gate, norms, step C)
    int32_t* cflag;    // per-partial "a norm needs recomputing" flags
    double* npart;     // per-block partial sums of squares
    int32_t* ctl;      // CTL_COUNT ints
    double* dsc;       // DSC_COUNT doubles
    double tol;        // recompute threshold on nu / nuref
    int pivoting;      // 1: greedy pivoting, 0: columns in their given order
};

#define APART_STRIDE (2 + 2 * QR_NBMAX)

// Sum NV doubles over a 256-thread block; results land in out[0..NV) (LDS)
// and are valid after the function returns (it ends with a barrier).
template <int NV>
__device__ __forceinline__ void block_sum_vec(double (&v)[NV], double* lds /* 4*NV */, double* out)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = wave_sum(v[e]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < NV; ++e) lds[wid * NV + e] = v[e];
    }
    __syncthreads();
    if (threadIdx.x < NV)
        out[threadIdx.x] = lds[threadIdx.x] + lds[NV + threadIdx.x] + lds[2 * NV + threadIdx.x] +
                           lds[3 * NV + threadIdx.x];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// step A: pivot choice + swap + bring-up of the pivot column + partial sums.
// grid: ceil(m / 256) blocks, one row per thread.  nparts: number of argmax
// partials left by the previous launch.  JMAX bounds the panel position jj
// (16, 32 or 64): the row's panel reflectors V[i, p0:j] stay in registers
// from the bring-up to the partial sums.  Everything that does not depend on
// the pivot (the stop flag, the argmax partials, V[i, p0:j] and A[i, j]) is
// loaded in one round before the pivot is known, so a step costs two
// dependent memory round trips.
// ---------------------------------------------------------------------------
template <typename T, int JMAX>
__global__ __launch_bounds__(256) void k_step_a(QrcpDev<T> d, int64_t j, int64_t p0, int jj, int nparts)
{
    __shared__ double2 fp[JMAX];
    __shared__ double s_red[4 * 2 * JMAX];
    __shared__ double s_rest[4];
    __shared__ ArgBest arg_lds[4];
    __shared__ int s_fl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int32_t stop = d.ctl[CTL_STOP];
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    const bool in = i < d.m, below = in && i >= j;
    // loads are unconditional from clamped in-range addresses and masked
    // afterwards, so they issue back to back without branches
    const int64_t ic = in ? i : d.m - 1;
    const T* arow = d.A + ic;
    // the reflector row is held as two scalar arrays (real, imaginary parts)
    // so that it stays in registers
    using S = typename std::conditional<sizeof(T) == 8, float, double>::type;
    S vre[JMAX], vim[JMAX];
#pragma unroll
    for (int t = 0; t < JMAX; ++t) {
        // entries t >= jj and rows outside [j, m) are never used (the sums
        // below test t < jj, and x = 0 off those rows)
        const int64_t col = p0 + (t < jj ? t : 0);   // p0 <= j: always a valid column
        const T v = arow[d.lda * col];
        vre[t] = v.x;
        vim[t] = v.y;
    }
    const T aj = arow[d.lda * j];

    int64_t p = j;
    if (d.pivoting) {
        if (tid == 0) s_fl = 0;
        ArgBest b;
        b.val = -1.0;
        b.key = 0x7fffffff;
        b.slot = -1;
        int fl = 0;
        for (int q0 = 0; q0 < nparts; q0 += 256 * 8) {
            // up to 8 partial loads per thread in flight before using any
            ArgBest e[8];
            int32_t f[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + tid + 256 * u;
                const int qc = q < nparts ? q : 0;
                e[u] = d.cpart[qc];
                f[u] = d.cflag[qc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool ok = q0 + tid + 256 * u < nparts;
                if (ok && e[u].slot >= 0 && arg_better(e[u].val, e[u].key, b.val, b.key)) b = e[u];
                fl |= ok ? f[u] : 0;
            }
        }
        b = wave_argmax(b);
        __syncthreads();   // orders the s_fl reset before the flag stores
        if (fl) s_fl = 1;
        if (lane == 0) arg_lds[wid] = b;
        __syncthreads();
        ArgBest bb = arg_lds[0];
        for (int w = 1; w < 4; ++w)
            if (arg_better(arg_lds[w].val, arg_lds[w].key, bb.val, bb.key)) bb = arg_lds[w];
        if (stop) return;
        if (s_fl) {
            // a residual norm of the previous step became unreliable: end the panel
            if (blockIdx.x == 0 && tid == 0) d.ctl[CTL_STOP] = 1;
            return;
        }
        if (bb.slot >= j) p = bb.slot;
        if (blockIdx.x == 0 && tid == 0) {
            d.ctl[CTL_PIV] = (int32_t)p;
            d.pivval[jj] = bb.slot >= j ? bb.val : -1.0;
            d.pivkey[jj] = bb.key;
        }
    } else if (stop) {
        return;
    }
    if (tid < jj) fp[tid] = to_d(d.F[p + d.ldf * tid]);
    const T ap = arow[d.lda * p];
    if (blockIdx.x == 0 && p != j) {
        if (tid < jj) {
            const T fj = d.F[j + d.ldf * tid];
            d.fsave[tid] = to_d(fj);
            d.F[j + d.ldf * tid] = d.F[p + d.ldf * tid];
        }
        if (tid == 0) {
            double t0 = d.nu[j]; d.nu[j] = d.nu[p]; d.nu[p] = t0;
            double t1 = d.nuref[j]; d.nuref[j] = d.nuref[p]; d.nuref[p] = t1;
            int32_t t2 = d.perm[j]; d.perm[j] = d.perm[p]; d.perm[p] = t2;
        }
    }
    __syncthreads();

    if (in && p != j) {
        d.A[i + d.lda * j] = ap;
        d.A[i + d.lda * p] = aj;
    }
    double2 x = czero();
    if (below) {
        // four interleaved partial sums shorten the FP64 dependency chain
        double2 xs[4] = {to_d(ap), czero(), czero(), czero()};
#pragma unroll
        for (int t = 0; t < JMAX; ++t)
            if (t < jj) xs[t & 3] = csub(xs[t & 3], cmul(make_double2(vre[t], vim[t]), cconj(fp[t])));
        x = cadd(cadd(xs[0], xs[1]), cadd(xs[2], xs[3]));
        d.xbuf[i] = x;
        d.xlo[i] = from_d<T>(x);
        if (i == j) d.hh[0] = x;
    }

    // partials: rest = sum_{i>j} |x_i|^2 and W_t = sum_i conj(V[i, t]) x_i
    {
        const double r = wave_sum((below && i > j) ? cabs2(x) : 0.0);
        if (lane == 0) s_rest[wid] = r;
    }
#pragma unroll
    for (int c0 = 0; c0 < JMAX; c0 += 16) {
        if (c0 < jj) {
            double v[32];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const double2 w =
                    c0 + u < jj ? cmulc(make_double2(vre[c0 + u], vim[c0 + u]), x) : czero();
                v[2 * u] = w.x;
                v[2 * u + 1] = w.y;
            }
            const double r = wave_reduce_scatter<32>(v);   // lane L: value L / 2 of the chunk
            if ((lane & 1) == 0) s_red[wid * 2 * JMAX + 2 * c0 + (lane >> 1)] = r;
        }
    }
    __syncthreads();
    double* part = d.apart + (int64_t)blockIdx.x * APART_STRIDE;
    if (tid < 2 * jj)
        part[2 + tid] = ((s_red[tid] + s_red[2 * JMAX + tid]) + s_red[4 * JMAX + tid]) + s_red[6 * JMAX + tid];
    if (tid == 255) part[0] = ((s_rest[0] + s_rest[1]) + s_rest[2]) + s_rest[3];
}

// Launch step A with the register budget that covers panel position jj.
template <typename T>
static void launch_step_a(const QrcpDev<T>& d, unsigned nblocks, int64_t j, int64_t p0, int jj, int nparts,
                          hipStream_t st)
{
    if (jj <= 16)
        hipLaunchKernelGGL((k_step_a<T, 16>), dim3(nblocks), dim3(256), 0, st, d, j, p0, jj, nparts);
    else if (jj <= 32)
        hipLaunchKernelGGL((k_step_a<T, 32>), dim3(nblocks), dim3(256), 0, st, d, j, p0, jj, nparts);
    else
        hipLaunchKernelGGL((k_step_a<T, 64>), dim3(nblocks), dim3(256), 0, st, d, j, p0, jj, nparts);
}

// Partial GEMV of one thread: acc[2u], acc[2u+1] += sum over this thread's
// rows i > j of conj(A[i, cbase+u]) x_i, for the CW columns cbase.. (< cend).
// x is read in storage precision (xlo); every product is formed and
// accumulated in FP64 (for complex64 data the products are exact, so the sum
// is the FP64 sum of the exact terms).  Storage is read in 16-byte vectors
// (two complex64 rows or one complex128 row per load), RU row groups per
// column in flight per thread.  The leading dimension is even, so every column
// starts 16-byte aligned.
//
// complex64: an empty asm statement on each loaded vector keeps the FP32 ->
// FP64 conversions at the point of use.  Left free, the compiler converts
// every vector as soon as it arrives, which doubles the live registers,
// lowers occupancy and with it the loads in flight per CU (measured: 4.6 TB/s
// instead of 6.0 TB/s on an 8192 x 8192 complex64 block with RU = 1).
template <typename T, int CW, int RU = (sizeof(T) == 8 ? 1 : 4)>
__device__ __forceinline__ void gemv_cols(const QrcpDev<T>& d, int64_t j, int64_t cbase, int64_t cend,
                                          double (&acc)[2 * CW])
{
#pragma unroll
    for (int u = 0; u < 2 * CW; ++u) acc[u] = 0.0;
    const int tid = threadIdx.x;
    const int64_t ncols = cend - cbase;
    const int64_t m = d.m;
    if constexpr (sizeof(T) == 8) {
        // complex64: pairs of rows (r, r+1), r even, starting at the pair holding row j+1
        const int64_t r0 = (j + 1) & ~(int64_t)1;
        // loads are unconditional, from clamped rows and columns: a row past m
        // is masked by lo/hi below, and a column past cend only feeds an
        // accumulator nobody reads.  (Conditional loads compile to a branch
        // that waits for each load before the next one issues.)
        const int64_t rlast = (m - 1) & ~(int64_t)1;   // last pair start; m odd: rows m-1, m < lda
        for (int64_t rb = r0 + 2 * tid; rb < m; rb += 512 * RU) {
            float4 xv[RU], av[RU][CW];
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                const int64_t r = rb + 512 * q;
                const int64_t rc = r < m ? r : rlast;
                xv[q] = *(const float4*)(d.xlo + rc);
#pragma unroll
                for (int u = 0; u < CW; ++u) {
                    const int64_t cc = cbase + (u < ncols ? u : 0);
                    av[q][u] = *(const float4*)(d.A + d.lda * cc + rc);
                }
            }
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                const int64_t r = rb + 512 * q;
                // rows outside (j, m) contribute nothing (select, so no NaN leaks in)
                const bool lo = r > j && r < m, hi = r + 1 < m;
                float4 xq = xv[q];
                asm volatile("" : "+v"(xq.x), "+v"(xq.y), "+v"(xq.z), "+v"(xq.w));
                const double x0r = lo ? (double)xq.x : 0.0, x0i = lo ? (double)xq.y : 0.0;
                const double x1r = hi ? (double)xq.z : 0.0, x1i = hi ? (double)xq.w : 0.0;
#pragma unroll
                for (int u = 0; u < CW; ++u) {
                    float4 a = av[q][u];
                    asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
                    const double ar = a.x, ai = a.y, br = a.z, bi = a.w;
                    // conj(a0) x0 + conj(a1) x1
                    acc[2 * u] = fma(ar, x0r, fma(ai, x0i, fma(br, x1r, fma(bi, x1i, acc[2 * u]))));
                    acc[2 * u + 1] = fma(ar, x0i, fma(-ai, x0r, fma(br, x1i, fma(-bi, x1r, acc[2 * u + 1]))));
                }
            }
        }
    } else {
        // complex128: one row per 16-byte load
        for (int64_t rb = j + 1 + tid; rb < m; rb += 256 * RU) {
            double2 xv[RU], av[RU][CW];
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                const int64_t r = rb + 256 * q;
                const int64_t rc = r < m ? r : m - 1;
                xv[q] = to_d(d.xlo[rc]);
#pragma unroll
                for (int u = 0; u < CW; ++u) {
                    const int64_t cc = cbase + (u < ncols ? u : 0);
                    av[q][u] = to_d(d.A[d.lda * cc + rc]);
                }
            }
            // pin the loaded values here so that all loads issue before any is used
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                asm volatile("" : "+v"(xv[q].x), "+v"(xv[q].y));
#pragma unroll
                for (int u = 0; u < CW; ++u) asm volatile("" : "+v"(av[q][u].x), "+v"(av[q][u].y));
            }
#pragma unroll
            for (int q = 0; q < RU; ++q)
                if (rb + 256 * q >= m) xv[q] = czero();   // rows past m contribute nothing
#pragma unroll
            for (int q = 0; q < RU; ++q) {
#pragma unroll
                for (int u = 0; u < CW; ++u) {
                    const double2 p = cmulc(av[q][u], xv[q]);
                    acc[2 * u] += p.x;
                    acc[2 * u + 1] += p.y;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// step C: reflector from step A's partials, GEMV over the trailing block,
// new F column, pivot row of R, downdate + per-block argmax partial.
// grid: ceil((cend - j - 1) / CW) blocks (at least one); na = step A blocks.
// CW columns per block: 4 over a full trailing block, 1 over a narrow window
// (more blocks for the same columns).
// ---------------------------------------------------------------------------
template <typename T, int CW = QR_CW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CW == 1 ? 1 : (sizeof(T) == 8 ? 8 : 4))))
void k_step_c(QrcpDev<T> d, int64_t j, int64_t p0, int jj, int64_t cend, int na)
{
    __shared__ double2 s_aux[QR_NBMAX], s_vj[QR_NBMAX], s_w[QR_NBMAX];
    __shared__ double2 s_par[4];   // beta, tau, scale, alpha
    __shared__ double red_lds[4 * 2 * CW];
    __shared__ double red_out[2 * CW];
    __shared__ double s_red[256];
    __shared__ double s_tot[2 * QR_NBMAX + 1];
    __shared__ int s_flag;
    __shared__ double2 s_f[CW][QR_NBMAX];
    __shared__ double2 s_arow[CW];
    __shared__ double s_nu[CW], s_nuref[CW];
    __shared__ int32_t s_perm[CW];

    // Every load that does not depend on another is issued first: the stop
    // flag (tested before the first store), step A's partials, this block's
    // F rows and column scalars, then the GEMV stream.  Only then do the
    // reductions and the reflector arithmetic wait on them.
    const int32_t stop = d.ctl[CTL_STOP];
    const int tid = threadIdx.x;
    const int64_t p = d.pivoting ? (int64_t)d.ctl[CTL_PIV] : j;
    const int64_t cbase = j + 1 + (int64_t)blockIdx.x * CW;

    // step A's partials: the S = 1 + 2*jj values of each step-A block are
    // summed by G = 256/S thread groups (group g takes blocks g, g+G, ...)
    const int S = 1 + 2 * jj, G = 256 / S;
    const int slot = tid % S, grp = tid / S;
    const int off = slot == 0 ? 0 : slot + 1;    // rest at 0, W re/im from 2
    // (held in registers across the GEMV only by the one-column variant, whose
    // occupancy does not matter; the wide variant loads them after the GEMV)
    constexpr int NPV = CW == 1 ? 16 : 0;
    double pv[NPV > 0 ? NPV : 1];
    pv[0] = 0.0;
#pragma unroll
    for (int u = 0; u < NPV; ++u) {
        // unconditional loads from clamped indices, masked afterwards
        const int b = grp + u * G;
        const int bc = (grp < G && b < na) ? b : 0;
        pv[u] = d.apart[(int64_t)bc * APART_STRIDE + off];
    }
#pragma unroll
    for (int u = 0; u < NPV; ++u) pv[u] = (grp < G && grp + u * G < na) ? pv[u] : 0.0;
    const double2 alpha_st = CW == 1 ? d.hh[0] : czero();
    // staged operands of the per-column work (at most one F entry per thread)
    // (unconditional loads from clamped in-range indices; a conditional load
    // would wait for its data before the GEMV stream could be issued)
    const bool has_f = tid < CW * jj && cbase + tid % CW < cend;
    double2 f_st;
    {
        const int t = has_f ? tid / CW : 0;
        const int64_t c = has_f ? cbase + tid % CW : cbase;
        const double2 fs = d.fsave[t];
        const double2 fr = to_d(d.F[c + d.ldf * t]);
        f_st = (d.pivoting && c == p && p != j) ? fs : fr;
    }
    const int64_t cst = cbase + (tid < CW && cbase + tid < cend ? tid : 0);
    const double2 arow_st = to_d(d.A[j + d.lda * cst]);
    const double nu_st = d.nu[cst], nuref_st = d.nuref[cst];
    const int32_t perm_st = d.perm[cst];
    const double2 vj_st = to_d(d.A[j + d.lda * (p0 + (tid < jj ? tid : 0))]);
    // this block's share of the reflector column (stored at the end): rows
    // [vr0, vr1); the one-column variant fetches its first 256 rows now
    const int64_t vlen = d.m - j - 1;
    const int64_t vchunk = (vlen + gridDim.x - 1) / gridDim.x;
    const int64_t vr0 = j + 1 + (int64_t)blockIdx.x * vchunk;
    const int64_t vr1 = vr0 + vchunk < d.m ? vr0 + vchunk : d.m;
    double2 xv_st = czero();
    if constexpr (CW == 1) {
        const int64_t i = vr0 + tid < d.m ? vr0 + tid : d.m - 1;   // clamped, masked at the store
        xv_st = d.xbuf[i];
    }
    auto stage = [&]() {
        if (has_f) s_f[tid % CW][tid / CW] = f_st;
        if (tid < CW) {
            s_arow[tid] = arow_st;
            s_nu[tid] = nu_st;
            s_nuref[tid] = nuref_st;
            s_perm[tid] = perm_st;
        }
        if (tid < jj) s_vj[tid] = vj_st;
    };
    // the wide variant parks the staged values in LDS now (its occupancy
    // needs the registers during the GEMV); the one-column variant after it
    if constexpr (CW > 1) stage();

    // ---- GEMV: g_u = sum_{i>j} conj(A[i, c_u]) x_i (independent of the reflector scalars) ----
    double acc[2 * CW];
    // one column per block (window panels): many rows in flight per thread instead
    gemv_cols<T, CW, CW == 1 ? 16 : (sizeof(T) == 8 ? 1 : 4)>(d, j, cbase, cend, acc);

    // ---- reflector from step A's partials (identical in every block) ----
    {
        double sacc = 0.0;
#pragma unroll
        for (int u = 0; u < NPV; ++u) sacc += pv[u];
        if (grp < G) {
            for (int b0 = grp + NPV * G; b0 < na; b0 += 16 * G) {   // the partials not loaded above
                double v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int b = b0 + u * G;
                    v[u] = b < na ? d.apart[(int64_t)b * APART_STRIDE + off] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) sacc += v[u];
            }
        }
        s_red[tid] = grp < G ? sacc : 0.0;
        if constexpr (CW == 1) stage();
        if (tid == 0) s_flag = 0;
        __syncthreads();
        if (tid < S) {
            double s2 = 0.0;
            for (int g = 0; g < G; ++g) s2 += s_red[g * S + tid];
            s_tot[tid] = s2;
        }
        __syncthreads();
    }
    if (tid < jj) s_w[tid] = make_double2(s_tot[1 + 2 * tid], s_tot[2 + 2 * tid]);
    if (tid == 64) {
        const double rest = s_tot[0];
        const double2 alpha = CW == 1 ? alpha_st : d.hh[0];
        double2 tau, scale;
        double beta;
        if (rest == 0.0 && alpha.y == 0.0) {
            tau = czero();
            scale = czero();
            beta = alpha.x;
        } else {
            const double nrm = sqrt(cabs2(alpha) + rest);
            beta = alpha.x >= 0.0 ? -nrm : nrm;
            tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            scale = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
        }
        s_par[0] = make_double2(beta, 0.0);
        s_par[1] = tau;
        s_par[2] = scale;
        s_par[3] = alpha;
    }
    __syncthreads();
    if (tid < jj) {
        // aux_t = V[:, t]^H v with v = (1, scale * x_rest), V[j, t] = s_vj[t]
        const double2 vjt = cconj(s_vj[tid]);
        const double2 rest = csub(s_w[tid], cmul(vjt, s_par[3]));
        s_aux[tid] = cadd(vjt, cmul(s_par[2], rest));
    }
    // (the barrier that publishes s_aux is the GEMV reduction's)
    const double beta = s_par[0].x;
    const double2 tau = s_par[1], scale = s_par[2];
    block_sum_rs<2 * CW>(acc, red_lds, red_out);
    if (stop) return;

    // ---- per-column scalar work: wave 0, 16 lanes per column, each lane
    //      summing the panel terms t = lane % 16 (mod 16), then a 16-lane
    //      shuffle reduction; lane 0 of each group finishes its column ----
    __shared__ ArgBest s_best[CW];
    if (tid < 16 * CW) {
        const int u = tid >> 4, tq = tid & 15;
        const int64_t c = cbase + u;
        const bool valid = c < cend;
        const bool moved = valid && d.pivoting && c == p && p != j;
        double2 corr = czero(), rs = czero();   // sum_t F[c,t] aux_t, sum_t V[j,t] conj(F[c,t])
        if (valid) {
            for (int t = tq; t < jj; t += 16) {
                const double2 f = s_f[u][t];
                corr = cadd(corr, cmul(f, s_aux[t]));
                rs = cadd(rs, cmul(s_vj[t], cconj(f)));
                if (moved) d.F[c + d.ldf * t] = from_d<T>(f);
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            corr.x += __shfl_xor(corr.x, off, MPS_WAVE);
            corr.y += __shfl_xor(corr.y, off, MPS_WAVE);
            rs.x += __shfl_xor(rs.x, off, MPS_WAVE);
            rs.y += __shfl_xor(rs.y, off, MPS_WAVE);
        }
        if (tq == 0) {
            ArgBest best;
            best.val = -1.0;
            best.key = 0x7fffffff;
            best.slot = -1;
            if (valid) {
                const double2 g = make_double2(red_out[2 * u], red_out[2 * u + 1]);
                const double2 ajc = s_arow[u];
                const double2 w = cadd(cconj(ajc), cmul(scale, g));
                const T fnew_t = from_d<T>(cmul(tau, csub(w, corr)));
                const double2 fnew = to_d(fnew_t);
                d.F[c + d.ldf * jj] = fnew_t;
                const double2 rrow = csub(csub(ajc, rs), cconj(fnew));
                d.A[j + d.lda * c] = from_d<T>(rrow);
                if (d.pivoting) {
                    double nn = s_nu[u] - cabs2(rrow);
                    if (nn < 0.0) nn = 0.0;
                    const bool flag = nn <= d.tol * s_nuref[u];
                    d.nu[c] = nn;
                    if (flag) {
                        s_flag = 1;
                    } else {
                        best.val = nn;
                        best.key = s_perm[u];
                        best.slot = (int32_t)c;
                    }
                }
            }
            s_best[u] = best;
        }
    }

    // ---- the reflector column below the diagonal, split evenly over the
    //      blocks; block 0 also stores R_jj, tau and the progress counter ----
    {
        int64_t i = vr0 + tid;
        if constexpr (CW == 1) {
            if (i < vr1) d.A[i + d.lda * j] = from_d<T>(cmul(scale, xv_st));
            i += 256;
        }
        for (; i < vr1; i += 256) d.A[i + d.lda * j] = from_d<T>(cmul(scale, d.xbuf[i]));
    }
    if (blockIdx.x == 0 && tid == 0) {
        d.A[j + d.lda * j] = from_d<T>(make_double2(beta, 0.0));
        d.tau[j] = tau;
        d.diagR[j] = beta;
        d.ctl[CTL_JDONE] = (int32_t)(j + 1);
    }
    if (!d.pivoting) return;
    __syncthreads();   // publishes s_best and s_flag
    if (tid == 0) {
        ArgBest b = s_best[0];
        for (int u = 1; u < CW; ++u)
            if (arg_better(s_best[u].val, s_best[u].key, b.val, b.key)) b = s_best[u];
        d.cpart[blockIdx.x] = b;
        d.cflag[blockIdx.x] = s_flag;
        // the panel ends here and the norms are recomputed before the next
        // one, also when this was the panel's last step (no step A follows
        // in this panel to turn the flag into the stop)
        if (s_flag) d.ctl[CTL_STOP] = 1;
    }
}

// ---------------------------------------------------------------------------
// Exact squared norms of columns [c0, n) over rows [r0, m) (FP64); optionally
// (re)sets nu = nuref = norm and perm; per-block partial sums and argmax.
// grid: ceil((n - c0) / QR_CW) blocks.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_colnorms(QrcpDev<T> d, int64_t r0, int64_t c0, int write_nu,
                                                  int init_perm)
{
    __shared__ double red_lds[4 * QR_CW];
    __shared__ double red_out[QR_CW];
    __shared__ ArgBest arg_lds[4];
    const int tid = threadIdx.x;
    const int64_t cbase = c0 + (int64_t)blockIdx.x * QR_CW;
    double acc[QR_CW];
#pragma unroll
    for (int u = 0; u < QR_CW; ++u) acc[u] = 0.0;
    for (int64_t i = r0 + tid; i < d.m; i += 256) {
#pragma unroll
        for (int u = 0; u < QR_CW; ++u)
            if (cbase + u < d.n) acc[u] += cabs2(to_d(d.A[i + d.lda * (cbase + u)]));
    }
    block_sum_vec<QR_CW>(acc, red_lds, red_out);
    ArgBest best;
    best.val = -1.0;
    best.key = 0x7fffffff;
    best.slot = -1;
    if (tid < QR_CW && cbase + tid < d.n) {
        const int64_t c = cbase + tid;
        if (init_perm) d.perm[c] = (int32_t)c;
        if (write_nu) {
            d.nu[c] = red_out[tid];
            d.nuref[c] = red_out[tid];
            best.val = red_out[tid];
            best.key = init_perm ? (int32_t)c : d.perm[c];
            best.slot = (int32_t)c;
        }
    }
    best = block_argmax256(best, arg_lds);
    if (tid == 0) {
        d.cpart[blockIdx.x] = best;
        d.cflag[blockIdx.x] = 0;
        double s = 0.0;
        for (int u = 0; u < QR_CW; ++u) s += red_out[u];
        d.npart[blockIdx.x] = s;
    }
}

// One block: fixed-order FP64 sum of the per-block partial sums into dsc[dslot].
__global__ __launch_bounds__(256) void k_sum_partials(const double* npart, int nparts, double* dsc, int dslot)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += 256) s += npart[q];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) dsc[dslot] = s;
}

// Reset the per-factorisation control block.
__global__ void k_ctl_reset(int32_t* ctl, double* dsc)
{
    if (threadIdx.x < CTL_COUNT) ctl[threadIdx.x] = 0;
    if (threadIdx.x < DSC_COUNT) dsc[threadIdx.x] = 0.0;
}

__global__ void k_ctl_panel(int32_t* ctl, int32_t jdone)
{
    if (threadIdx.x == 0) {
        ctl[CTL_STOP] = 0;
        ctl[CTL_JDONE] = jdone;
        ctl[CTL_TFAIL] = 0x7fffffff;   // atomic minima of a window panel's replay
        ctl[CTL_TFLAG] = 0x7fffffff;
    }
}
