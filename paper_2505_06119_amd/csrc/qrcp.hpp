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
//   step A  (rows split over blocks)  pivot swap, bring the pivot column up to
//           date (x = A_ps[:, j] - V F[j, :]^H), partial sums of ||x||^2 and
//           V^H x; the last block to finish forms the reflector
//           (beta, tau, scale) in FP64 and aux = V^H v.
//   step C  (columns split over blocks)  the GEMV w = A_ps^H v over the whole
//           trailing block (the HBM-bound part), the new F column
//           F[:, jj] = tau (w - F aux), the pivot row of R, the FP64 downdate
//           of the residual column norms and a partial argmax; the last block
//           to finish picks the next pivot.
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
#define QR_CW 4            // columns per block in step C

enum {
    CTL_PIV = 0,      // pivot position for the next step
    CTL_STOP = 1,     // panel must end: a norm needs recomputing
    CTL_JDONE = 2,    // number of completed steps
    CTL_TICKET_A = 3,
    CTL_TICKET_C = 4,
    CTL_TICKET_M = 5,
    CTL_PEND = 6,     // a column was flagged during the current step C
    CTL_NREFRESH = 7, // number of norm refreshes (statistics)
    CTL_COUNT = 16
};
enum { DSC_NORM2 = 0, DSC_EPS2 = 1, DSC_RET2 = 2, DSC_COUNT = 8 };

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
    double2* xbuf;
    double* apart;     // step-A partials, (2 + 2*QR_NBMAX) doubles per block
    double2* hh;       // [0] alpha [1] beta [2] tau [3] scale [4..] aux
    double2* fsave;    // QR_NBMAX
    ArgBest* cpart;    // step-C / norm-kernel argmax partials
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
// step A: pivot swap + bring-up of the pivot column + reflector (last block)
// grid: ceil(m / 256) blocks, one row per thread.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_step_a(QrcpDev<T> d, int64_t j, int64_t p0, int jj)
{
    __shared__ double2 fp[QR_NBMAX];
    __shared__ double red_lds[4 * 16];
    __shared__ double red_out[16];
    __shared__ int last_flag;
    if (ld_coherent(&d.ctl[CTL_STOP])) return;

    const int tid = threadIdx.x;
    const int64_t p = d.pivoting ? (int64_t)d.ctl[CTL_PIV] : j;
    if (tid < jj) fp[tid] = to_d(d.F[p + d.ldf * tid]);
    if (blockIdx.x == 0 && p != j) {
        if (tid < jj) {
            T fj = d.F[j + d.ldf * tid];
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

    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    double2 x = czero();
    bool has = false;
    if (i < d.m) {
        T aj = d.A[i + d.lda * j];
        T ap = d.A[i + d.lda * p];
        if (p != j) {
            d.A[i + d.lda * j] = ap;
            d.A[i + d.lda * p] = aj;
        }
        if (i >= j) {
            x = to_d(ap);
            for (int t = 0; t < jj; ++t)
                x = csub(x, cmul(to_d(d.A[i + d.lda * (p0 + t)]), cconj(fp[t])));
            d.xbuf[i] = x;
            has = true;
            if (i == j) d.hh[0] = x;
        }
    }
    double* part = d.apart + (int64_t)blockIdx.x * APART_STRIDE;
    {
        double v[1] = {(has && i > j) ? cabs2(x) : 0.0};
        block_sum_vec<1>(v, red_lds, red_out);
        if (tid == 0) part[0] = red_out[0];
    }
    for (int t0 = 0; t0 < jj; t0 += 8) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + u;
            double2 w = czero();
            if (has && t < jj) w = cmulc(to_d(d.A[i + d.lda * (p0 + t)]), x);
            v[2 * u] = w.x;
            v[2 * u + 1] = w.y;
        }
        block_sum_vec<16>(v, red_lds, red_out);
        if (tid < 16 && t0 + tid / 2 < jj) part[2 + 2 * t0 + tid] = red_out[tid];
    }

    if (!last_block_ticket((unsigned int*)&d.ctl[CTL_TICKET_A], gridDim.x, &last_flag)) return;

    // ---- last block: reduce partials, form the reflector ----
    __shared__ double2 wsum[QR_NBMAX];
    __shared__ double2 s_alpha, s_scale;
    const int nb = gridDim.x;
    if (tid < jj) {
        double2 w = czero();
        for (int b = 0; b < nb; ++b) {
            w.x += ld_coherent(d.apart + (int64_t)b * APART_STRIDE + 2 + 2 * tid);
            w.y += ld_coherent(d.apart + (int64_t)b * APART_STRIDE + 3 + 2 * tid);
        }
        wsum[tid] = w;
    }
    if (tid == 0) {
        double rest = 0.0;
        for (int b = 0; b < nb; ++b) rest += ld_coherent(d.apart + (int64_t)b * APART_STRIDE);
        double2 alpha;
        alpha.x = ld_coherent(&d.hh[0].x);
        alpha.y = ld_coherent(&d.hh[0].y);
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
        d.hh[1] = make_double2(beta, 0.0);
        d.hh[2] = tau;
        d.hh[3] = scale;
        s_alpha = alpha;
        s_scale = scale;
    }
    __syncthreads();
    if (tid < jj) {
        // aux_t = V[:, t]^H v with v = (1, scale * x_rest)
        const double2 vjt = cconj(to_d(d.A[j + d.lda * (p0 + tid)]));
        const double2 rest = csub(wsum[tid], cmul(vjt, s_alpha));
        d.hh[4 + tid] = cadd(vjt, cmul(s_scale, rest));
    }
}

// ---------------------------------------------------------------------------
// step C: GEMV over the trailing block, new F column, pivot row of R,
// downdate + partial argmax; last block picks the next pivot.
// grid: ceil((cend - j - 1) / QR_CW) blocks (at least one).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_step_c(QrcpDev<T> d, int64_t j, int64_t p0, int jj, int64_t cend)
{
    __shared__ double2 s_aux[QR_NBMAX], s_vj[QR_NBMAX];
    __shared__ double2 s_par[4];   // beta, tau, scale
    __shared__ double red_lds[4 * 2 * QR_CW];
    __shared__ double red_out[2 * QR_CW];
    __shared__ ArgBest arg_lds[4];
    __shared__ int last_flag;
    if (ld_coherent(&d.ctl[CTL_STOP])) return;

    const int tid = threadIdx.x;
    if (tid < jj) {
        s_aux[tid] = d.hh[4 + tid];
        s_vj[tid] = to_d(d.A[j + d.lda * (p0 + tid)]);
    }
    if (tid < 3) s_par[tid] = d.hh[1 + tid];
    __syncthreads();
    const double beta = s_par[0].x;
    const double2 tau = s_par[1], scale = s_par[2];
    const int64_t p = d.pivoting ? (int64_t)d.ctl[CTL_PIV] : j;

    // ---- GEMV: g_u = sum_{i>j} conj(A[i, c_u]) x_i ----
    const int64_t cbase = j + 1 + (int64_t)blockIdx.x * QR_CW;
    double acc[2 * QR_CW];
#pragma unroll
    for (int u = 0; u < 2 * QR_CW; ++u) acc[u] = 0.0;
    for (int64_t i = j + 1 + tid; i < d.m; i += 256) {
        const double2 xi = d.xbuf[i];
#pragma unroll
        for (int u = 0; u < QR_CW; ++u) {
            const int64_t c = cbase + u;
            if (c < cend) {
                const double2 w = cmulc(to_d(d.A[i + d.lda * c]), xi);
                acc[2 * u] += w.x;
                acc[2 * u + 1] += w.y;
            }
        }
    }
    block_sum_vec<2 * QR_CW>(acc, red_lds, red_out);

    // ---- per-column scalar work (one thread per column) ----
    ArgBest best;
    best.val = -1.0;
    best.key = 0x7fffffff;
    best.slot = -1;
    if (tid < QR_CW) {
        const int64_t c = cbase + tid;
        if (c < cend) {
            const bool moved = d.pivoting && c == p && p != j;
            const double2 g = make_double2(red_out[2 * tid], red_out[2 * tid + 1]);
            const double2 ajc = to_d(d.A[j + d.lda * c]);
            double2 w = cadd(cconj(ajc), cmul(scale, g));
            double2 corr = czero(), rrow = ajc;
            for (int t = 0; t < jj; ++t) {
                const double2 f = moved ? d.fsave[t] : to_d(d.F[c + d.ldf * t]);
                corr = cadd(corr, cmul(f, s_aux[t]));
                rrow = csub(rrow, cmul(s_vj[t], cconj(f)));
                if (moved) d.F[c + d.ldf * t] = from_d<T>(f);
            }
            const T fnew_t = from_d<T>(cmul(tau, csub(w, corr)));
            const double2 fnew = to_d(fnew_t);
            d.F[c + d.ldf * jj] = fnew_t;
            rrow = csub(rrow, cconj(fnew));
            d.A[j + d.lda * c] = from_d<T>(rrow);
            if (d.pivoting) {
                double nn = d.nu[c] - cabs2(rrow);
                if (nn < 0.0) nn = 0.0;
                const bool flag = nn <= d.tol * d.nuref[c];
                d.nu[c] = nn;
                if (flag) atomicOr(&d.ctl[CTL_PEND], 1);
                else {
                    best.val = nn;
                    best.key = d.perm[c];
                    best.slot = (int32_t)c;
                }
            }
        }
    }

    // ---- block 0 stores the reflector and R_jj ----
    if (blockIdx.x == 0) {
        for (int64_t i = j + 1 + tid; i < d.m; i += 256)
            d.A[i + d.lda * j] = from_d<T>(cmul(scale, d.xbuf[i]));
        if (tid == 0) {
            d.A[j + d.lda * j] = from_d<T>(make_double2(beta, 0.0));
            d.tau[j] = tau;
            d.diagR[j] = beta;
            d.ctl[CTL_JDONE] = (int32_t)(j + 1);
        }
    }
    if (!d.pivoting) return;

    best = block_argmax256(best, arg_lds);
    if (tid == 0) d.cpart[blockIdx.x] = best;
    if (!last_block_ticket((unsigned int*)&d.ctl[CTL_TICKET_C], gridDim.x, &last_flag)) return;

    // ---- last block: next pivot ----
    ArgBest b;
    b.val = -1.0;
    b.key = 0x7fffffff;
    b.slot = -1;
    for (int q = tid; q < (int)gridDim.x; q += 256) {
        ArgBest e;
        e.val = ld_coherent(&d.cpart[q].val);
        e.key = ld_coherent(&d.cpart[q].key);
        e.slot = ld_coherent(&d.cpart[q].slot);
        if (e.slot >= 0 && arg_better(e.val, e.key, b.val, b.key)) b = e;
    }
    b = block_argmax256(b, arg_lds);
    if (tid == 0) {
        d.ctl[CTL_PIV] = b.slot >= 0 ? b.slot : (int32_t)(j + 1 < d.n ? j + 1 : j);
        if (ld_coherent(&d.ctl[CTL_PEND])) {
            d.ctl[CTL_PEND] = 0;
            d.ctl[CTL_STOP] = 1;
        }
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
        double s = 0.0;
        for (int u = 0; u < QR_CW; ++u) s += red_out[u];
        d.npart[blockIdx.x] = s;
    }
}

// One block: reduce the partials of k_colnorms (or of the gate kernel) into
// the next pivot and/or a scalar sum stored in dsc[dslot] (dslot < 0: none).
template <typename T>
__global__ __launch_bounds__(256) void k_partials_final(QrcpDev<T> d, int nparts, int do_piv, int dslot,
                                                        int64_t fallback_piv)
{
    __shared__ ArgBest arg_lds[4];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    ArgBest b;
    b.val = -1.0;
    b.key = 0x7fffffff;
    b.slot = -1;
    double s = 0.0;
    for (int q = tid; q < nparts; q += 256) {
        if (do_piv) {
            ArgBest e = d.cpart[q];
            if (e.slot >= 0 && arg_better(e.val, e.key, b.val, b.key)) b = e;
        }
        if (dslot >= 0) s += d.npart[q];
    }
    // fixed-order FP64 sum: per-thread strided partials, then a block sum
    s = block_sum256(s, red);
    b = block_argmax256(b, arg_lds);
    if (tid == 0) {
        if (do_piv) d.ctl[CTL_PIV] = b.slot >= 0 ? b.slot : (int32_t)fallback_piv;
        if (dslot >= 0) d.dsc[dslot] = s;
    }
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
        ctl[CTL_PEND] = 0;
        ctl[CTL_JDONE] = jdone;
    }
}
