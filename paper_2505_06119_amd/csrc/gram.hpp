// Candidate-window panels whose pivots come from the window's Gram matrix:
// a second way to run the truncated QR with column pivoting of Table III.
//
// Greedy column pivoting picks at each step the column of largest residual
// norm.  Those residual norms, and the R rows that downdate them, are fixed
// by the inner products of the columns: the pivots and R of pivoted
// Householder QR are those of pivoted Cholesky of G = A^H A (up to the signs
// of R's rows).  A panel over the W-column window therefore runs as
//
//   1. norms    exact FP64 norms of the window columns (the panel-start nu)
//               and G = A_w^H A_w over the rows from p0 (one GEMM);
//   2. pivots   pivoted Cholesky of G in one workgroup: at step t the live
//               column of largest d_c (the pivot comparison of the step
//               kernels, ties by key), R[t, c] = (G[p, c] - sum_{s<t}
//               conj(R[s, p]) R[s, c]) / sqrt(d_p), d_c -= |R[t, c]|^2;
//               the panel ends early when the pivot's d has cancelled below
//               GRAM_CANCEL of its panel-start value;
//   3. Q        CholeskyQR2 of the nbe chosen columns in FP64: Q1 = A_s R1^-1
//               (R1 the Cholesky rows of the pivots), R2 = chol(Q1^H Q1),
//               Q = Q1 R2^-1, R = R2 R1;
//   4. V, T     Householder reconstruction: the LU factorisation without
//               pivoting of Q diag(s) - [I; 0] = Y U, with s_j = -sign(Re w_j)
//               chosen when column j is reached (w_j its Schur-complement
//               diagonal), is the compact-WY form of the Householder QR of
//               the same columns with the xLARFG convention: Y the unit lower
//               reflectors, T = -U Y_1^-H (tau_j = T_jj), R_hh = diag(s) R,
//               beta_j = s_j R_jj.
//
// The panel then ends like a right-looking window panel: the pivots' final
// columns go through vbuf and the window reorder; every other column of the
// trailing block, inside the window or outside it, takes the block update
// and the greedy replay.  A replay miss or a failed Cholesky restores the
// window and runs the panel with the per-step kernels instead.
#pragma once
#include "window.hpp"

#define GRAM_W_MAX 256      // window columns (one thread each)
#define GRAM_NB_MAX 32      // pivots per panel
#define GRAM_CANCEL 1e-6    // relative cancellation of a pivot's norm that ends the panel
#define GRAM_ROWS_NT 64     // threads per block of the row-parallel kernels

// Small FP64 matrices of one Gram panel (ld GRAM_NB_MAX each, offsets in double2).
enum { GSM_R1 = 0, GSM_G2 = 1024, GSM_R2 = 2048, GSM_RF = 3072, GSM_Y1 = 4096, GSM_U = 5120, GSM_S = 6144,
       GSM_COUNT = 8192 };

// Step 1: exact FP64 norms of the window's columns over rows p0 .. m-1 into
// nu and nuref (block b = column p0 + b, 256 threads).
template <typename T>
__global__ __launch_bounds__(256) void k_win_norms(QrcpDev<T> d, int64_t p0)
{
    __shared__ double s_w[4];
    const int tid = threadIdx.x;
    const int64_t c = p0 + blockIdx.x;
    const T* col = d.A + d.lda * c;
    double acc = 0.0;
    for (int64_t i = p0 + tid; i < d.m; i += 256) acc += cabs2(to_d(col[i]));
    acc = wave_sum(acc);
    if ((tid & 63) == 0) s_w[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        const double v = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
        d.nu[c] = v;
        d.nuref[c] = v;
    }
}

// Step 2: one block of 256 threads, thread c = window column p0 + c (c < W).
// G (W x W, ld ldg) = A_w^H A_w; d.nu holds the window's exact norms.  Writes
// pivval/pivkey/wpiv per step, R1 = the pivots' Cholesky rows (upper
// triangular in step order, ld GRAM_NB_MAX) and ctl[CTL_JDONE] = p0 + nbe.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_pivots(QrcpDev<T> d, const T* G, int64_t ldg, int64_t p0, int W,
                                                     int nsteps, int32_t* wpiv, double2* R1)
{
    __shared__ ArgBest s_arg[4];
    __shared__ double2 s_rp[GRAM_NB_MAX];
    __shared__ double s_d0;
    const int c = threadIdx.x;
    const bool in = c < W;
    double dc = in ? d.nu[p0 + c] : 0.0;
    const double d0 = dc;
    const int32_t key = in ? d.perm[p0 + c] : 0x7fffffff;
    bool live = in;
    double2 rc[GRAM_NB_MAX];   // R[0:t, c], static indices only
#pragma unroll
    for (int s = 0; s < GRAM_NB_MAX; ++s) rc[s] = czero();
    int myq = -1, nbe = 0;
    for (int t = 0; t < nsteps; ++t) {
        ArgBest a;
        a.val = live ? (dc > 0.0 ? dc : 0.0) : -1.0;
        a.key = live ? key : 0x7fffffff;
        a.slot = live ? c : -1;
        const ArgBest b = block_argmax256(a, s_arg);
        if (b.slot < 0) break;   // uniform: no live column
        const int p = b.slot;
        // G[p, c] = a_p^H a_c = conj(G[c, p]), loaded before the broadcast
        const double2 gpc = live && c != p ? cconj(to_d(G[c + ldg * p])) : czero();
        if (c == p) {
#pragma unroll
            for (int s = 0; s < GRAM_NB_MAX; ++s)
                if (s < t) s_rp[s] = rc[s];
            s_d0 = d0;
        }
        __syncthreads();
        const double dp = b.val;
        if (!(dp > GRAM_CANCEL * s_d0)) break;   // uniform
        const double rtp = sqrt(dp), rinv = 1.0 / rtp;
        if (c == p) {
#pragma unroll
            for (int s = 0; s < GRAM_NB_MAX; ++s)
                if (s == t) rc[s] = make_double2(rtp, 0.0);
            live = false;
            myq = t;
        } else if (live) {
            // four independent partial sums keep the dependent chain short
            double2 g0 = gpc, g1 = czero(), g2 = czero(), g3 = czero();
#pragma unroll
            for (int s = 0; s < GRAM_NB_MAX; s += 4) {
                if (s < t) g0 = csub(g0, cmulc(s_rp[s], rc[s]));
                if (s + 1 < t) g1 = csub(g1, cmulc(s_rp[s + 1], rc[s + 1]));
                if (s + 2 < t) g2 = csub(g2, cmulc(s_rp[s + 2], rc[s + 2]));
                if (s + 3 < t) g3 = csub(g3, cmulc(s_rp[s + 3], rc[s + 3]));
            }
            const double2 r = cscale(cadd(cadd(g0, g1), cadd(g2, g3)), rinv);
#pragma unroll
            for (int s = 0; s < GRAM_NB_MAX; ++s)
                if (s == t) rc[s] = r;
            const double nd = dc - cabs2(r);
            dc = nd > 0.0 ? nd : 0.0;
        }
        if (c == 0) {
            d.pivval[t] = dp;
            d.pivkey[t] = b.key;
            wpiv[t] = (int32_t)(p0 + p);
        }
        nbe = t + 1;
        __syncthreads();
    }
    if (myq >= 0) {
#pragma unroll
        for (int s = 0; s < GRAM_NB_MAX; ++s) R1[s + GRAM_NB_MAX * myq] = s <= myq ? rc[s] : czero();
    }
    if (c == 0) d.ctl[CTL_JDONE] = (int32_t)(p0 + nbe);
}

// X = B R^-1 row by row (R upper triangular nbe x nbe with a positive real
// diagonal, ld GRAM_NB_MAX, FP64), rows p0 .. m-1 of the panel: B is the
// pivot columns of d.A (FROM_A, columns wpiv[0..nbe)) or X itself (in place).
// nbe = ctl[CTL_JDONE] - p0 (nothing to do when 0).  grid: rows / GRAM_ROWS_NT
// (one row per thread, small blocks so that the rows spread over the CUs).
template <typename T, bool FROM_A>
__global__ __launch_bounds__(GRAM_ROWS_NT) void k_cqr_trsm(QrcpDev<T> d, int64_t p0, const int32_t* wpiv,
                                                           const double2* R, double2* X, int64_t ldx)
{
    __shared__ double2 Rs[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double rinv[GRAM_NB_MAX];
    __shared__ int64_t s_col[GRAM_NB_MAX];
    const int nbe = d.ctl[CTL_JDONE] - (int)p0;
    const int tid = threadIdx.x;
    for (int q = tid; q < GRAM_NB_MAX * GRAM_NB_MAX; q += GRAM_ROWS_NT) Rs[q % GRAM_NB_MAX][q / GRAM_NB_MAX] = R[q];
    if (tid < GRAM_NB_MAX) {
        rinv[tid] = tid < nbe ? 1.0 / R[tid * (GRAM_NB_MAX + 1)].x : 0.0;
        s_col[tid] = FROM_A && tid < nbe ? (int64_t)wpiv[tid] : 0;
    }
    __syncthreads();
    const int64_t rows = d.m - p0, i = (int64_t)blockIdx.x * GRAM_ROWS_NT + tid;
    if (nbe <= 0 || i >= rows) return;
    double2 x[GRAM_NB_MAX];
#pragma unroll
    for (int q = 0; q < GRAM_NB_MAX; ++q)
        x[q] = FROM_A ? to_d(d.A[p0 + i + d.lda * s_col[q]]) : X[i + ldx * q];
#pragma unroll
    for (int q = 0; q < GRAM_NB_MAX; ++q) {
        double2 b0 = x[q], b1 = czero(), b2 = czero(), b3 = czero();
#pragma unroll
        for (int s = 0; s < q; s += 4) {
            b0 = csub(b0, cmul(x[s], Rs[s][q]));
            if (s + 1 < q) b1 = csub(b1, cmul(x[s + 1], Rs[s + 1][q]));
            if (s + 2 < q) b2 = csub(b2, cmul(x[s + 2], Rs[s + 2][q]));
            if (s + 3 < q) b3 = csub(b3, cmul(x[s + 3], Rs[s + 3][q]));
        }
        x[q] = q < nbe ? cscale(cadd(cadd(b0, b1), cadd(b2, b3)), rinv[q]) : czero();
    }
#pragma unroll
    for (int q = 0; q < GRAM_NB_MAX; ++q)
        if (q < nbe) X[i + ldx * q] = x[q];
}

// R2 = chol(G2) (upper, G2 = Q1^H Q1 at GSM_G2) and R = R2 R1, one block of
// 1024 threads (thread (r, c) = entry r, c).  A G2 that is not positive
// definite sets ctl[CTL_JDONE] = p0: the later kernels then do nothing and
// the host takes the per-step path for the panel.
__global__ __launch_bounds__(1024) void k_cqr_chol(int32_t* ctl, int64_t p0, double2* sm)
{
    __shared__ double2 A[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double2 R1[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ int s_bad;
    const int nbe = ctl[CTL_JDONE] - (int)p0;
    const int tid = threadIdx.x, r = tid % GRAM_NB_MAX, c = tid / GRAM_NB_MAX;
    const bool in = r < nbe && c < nbe;
    A[r][c] = in ? sm[GSM_G2 + r + GRAM_NB_MAX * c] : czero();
    R1[r][c] = in ? sm[GSM_R1 + r + GRAM_NB_MAX * c] : czero();
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int k = 0; k < nbe; ++k) {
        const double akk = A[k][k].x;
        const double ukk = akk > 0.0 ? sqrt(akk) : 1.0;
        __syncthreads();
        if (tid == 0) {
            if (!(akk > 0.0)) s_bad = 1;
            A[k][k] = make_double2(ukk, 0.0);
        }
        if (r == k && c > k && c < nbe) A[k][c] = cscale(A[k][c], 1.0 / ukk);
        __syncthreads();
        if (r > k && c >= r && c < nbe) A[r][c] = csub(A[r][c], cmulc(A[k][r], A[k][c]));
        __syncthreads();
    }
    const bool up = in && r <= c;
    sm[GSM_R2 + r + GRAM_NB_MAX * c] = up ? A[r][c] : czero();
    double2 f0 = czero(), f1 = czero();
    if (up) {
        int s2 = r;
        for (; s2 + 1 <= c; s2 += 2) {
            f0 = cadd(f0, cmul(A[r][s2], R1[s2][c]));
            f1 = cadd(f1, cmul(A[r][s2 + 1], R1[s2 + 1][c]));
        }
        if (s2 <= c) f0 = cadd(f0, cmul(A[r][s2], R1[s2][c]));
    }
    sm[GSM_RF + r + GRAM_NB_MAX * c] = cadd(f0, f1);
    if (tid == 0 && s_bad) ctl[CTL_JDONE] = (int32_t)p0;
}

// Householder reconstruction from the top nbe x nbe block of Q (rows p0 ..
// p0+nbe-1, FP64 at Q, ld ldq), one block of 1024 threads (thread (r, c) =
// entry r, c): the LU of Q diag(s) - [I; 0] with the signs chosen column by
// column, then T = -U Y_1^-H.  Writes Tout (ld ldt, the panel's T factor),
// tau and diagR of the panel's steps, and Y_1, the signed U and s into sm
// for k_recon_rows.
template <typename T>
__global__ __launch_bounds__(1024) void k_recon(QrcpDev<T> d, int64_t p0, const double2* Q, int64_t ldq,
                                                double2* sm, T* Tout, int ldt)
{
    __shared__ double2 Wm[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double2 Ys[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double2 Us[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double ss[GRAM_NB_MAX];
    const int nbe = d.ctl[CTL_JDONE] - (int)p0;
    const int tid = threadIdx.x, r = tid % GRAM_NB_MAX, c = tid / GRAM_NB_MAX;
    const bool in = r < nbe && c < nbe;
    Wm[r][c] = in ? Q[r + ldq * c] : czero();
    Ys[r][c] = czero();
    Us[r][c] = czero();
    if (tid < GRAM_NB_MAX) ss[tid] = 1.0;
    __syncthreads();
    for (int j = 0; j < nbe; ++j) {
        // every thread derives s_j and U_jj from the same Schur-complement entry
        const double2 w = Wm[j][j];
        const double s = w.x >= 0.0 ? -1.0 : 1.0;
        const double2 ujj = make_double2(s * w.x - 1.0, s * w.y);
        double2 l = czero(), wjc = czero();
        if (r > j && r < nbe) l = cdiv(cscale(Wm[r][j], s), ujj);
        if (c > j && c < nbe) wjc = Wm[j][c];
        __syncthreads();
        if (tid == 0) {
            ss[j] = s;
            Us[j][j] = ujj;
        }
        if (c == j && r > j && r < nbe) Ys[r][j] = l;
        if (r == j && c > j && c < nbe) Us[j][c] = wjc;
        if (r > j && r < nbe && c > j && c < nbe) Wm[r][c] = csub(Wm[r][c], cmul(l, wjc));
        __syncthreads();
    }
    if (r < c && c < nbe) Us[r][c] = cscale(Us[r][c], ss[c]);
    if (r == c && r < nbe) Ys[r][r] = make_double2(1.0, 0.0);
    __syncthreads();
    // T Y_1^H = -U, row by row (T upper triangular); Wm is reused for T
    if (tid < nbe) {
        const int i = tid;
        for (int k = 0; k < nbe; ++k) {
            double2 t0 = czero(), t1 = czero();
            if (k >= i) {
                t0 = cscale(Us[i][k], -1.0);
                int l2 = i;
                for (; l2 + 1 < k; l2 += 2) {
                    t0 = csub(t0, cmul(Wm[i][l2], cconj(Ys[k][l2])));
                    t1 = csub(t1, cmul(Wm[i][l2 + 1], cconj(Ys[k][l2 + 1])));
                }
                if (l2 < k) t0 = csub(t0, cmul(Wm[i][l2], cconj(Ys[k][l2])));
            }
            Wm[i][k] = cadd(t0, t1);
        }
    }
    __syncthreads();
    Tout[r + ldt * c] = from_d<T>(in && r <= c ? Wm[r][c] : czero());
    sm[GSM_Y1 + r + GRAM_NB_MAX * c] = Ys[r][c];
    sm[GSM_U + r + GRAM_NB_MAX * c] = Us[r][c];
    if (tid < nbe) {
        d.tau[p0 + tid] = Wm[tid][tid];
        d.diagR[p0 + tid] = ss[tid] * sm[GSM_RF + tid * (GRAM_NB_MAX + 1)].x;
        sm[GSM_S + tid] = make_double2(ss[tid], 0.0);
    }
}

// The pivots' final columns, rows p0 .. m-1: for step k, beta_k at row p0+k
// and the reflector below it into vbuf[:, k] (rows of Y_1 inside the top
// block, Y_2 = Q_2 diag(s) U^-1 below it), and R_hh[i, k] = s_i R[i, k] for
// i < k into the pivot column itself (the rows a window reorder keeps from
// d.A).  grid: rows / GRAM_ROWS_NT.
template <typename T>
__global__ __launch_bounds__(GRAM_ROWS_NT) void k_recon_rows(QrcpDev<T> d, int64_t p0, const int32_t* wpiv,
                                                             const double2* Q, int64_t ldq, const double2* sm, T* vbuf)
{
    __shared__ double2 Us[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double2 Y1[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double2 Rf[GRAM_NB_MAX][GRAM_NB_MAX + 1];
    __shared__ double ss[GRAM_NB_MAX];
    __shared__ int64_t s_col[GRAM_NB_MAX];
    const int nbe = d.ctl[CTL_JDONE] - (int)p0;
    const int tid = threadIdx.x;
    for (int q = tid; q < GRAM_NB_MAX * GRAM_NB_MAX; q += GRAM_ROWS_NT) {
        const int rr = q % GRAM_NB_MAX, cc = q / GRAM_NB_MAX;
        Us[rr][cc] = sm[GSM_U + q];
        Y1[rr][cc] = sm[GSM_Y1 + q];
        Rf[rr][cc] = sm[GSM_RF + q];
    }
    if (tid < GRAM_NB_MAX) {
        ss[tid] = sm[GSM_S + tid].x;
        s_col[tid] = tid < nbe ? (int64_t)wpiv[tid] : 0;
    }
    __syncthreads();
    const int64_t rows = d.m - p0, i = (int64_t)blockIdx.x * GRAM_ROWS_NT + tid;
    if (nbe <= 0 || i >= rows) return;
    const int64_t row = p0 + i;
    if (i < nbe) {
        const int ii = (int)i;
        for (int k = 0; k < nbe; ++k) {
            if (k < ii) vbuf[row + d.lda * k] = from_d<T>(Y1[ii][k]);
            else if (k == ii) vbuf[row + d.lda * k] = from_d<T>(make_double2(ss[ii] * Rf[ii][ii].x, 0.0));
            else d.A[row + d.lda * s_col[k]] = from_d<T>(cscale(Rf[ii][k], ss[ii]));
        }
        return;
    }
    double2 y[GRAM_NB_MAX];
#pragma unroll
    for (int k = 0; k < GRAM_NB_MAX; ++k) y[k] = Q[i + ldq * k];
#pragma unroll
    for (int k = 0; k < GRAM_NB_MAX; ++k) {
        double2 b0 = cscale(y[k], ss[k]), b1 = czero(), b2 = czero(), b3 = czero();
#pragma unroll
        for (int j = 0; j < k; j += 4) {
            b0 = csub(b0, cmul(y[j], Us[j][k]));
            if (j + 1 < k) b1 = csub(b1, cmul(y[j + 1], Us[j + 1][k]));
            if (j + 2 < k) b2 = csub(b2, cmul(y[j + 2], Us[j + 2][k]));
            if (j + 3 < k) b3 = csub(b3, cmul(y[j + 3], Us[j + 3][k]));
        }
        y[k] = k < nbe ? cdiv(cadd(cadd(b0, b1), cadd(b2, b3)), Us[k][k]) : czero();
    }
#pragma unroll
    for (int k = 0; k < GRAM_NB_MAX; ++k)
        if (k < nbe) vbuf[row + d.lda * k] = from_d<T>(y[k]);
}
