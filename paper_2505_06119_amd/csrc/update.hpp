// The two-site update (paper Sec. III-C.2 "tensor application" for a gate on
// neighbouring sites, with the truncated pivoted-QR decomposition of Table III):
//
//   a1  theta0 = A_i A_{i+1}                       (MFMA GEMM)
//   a2  theta  = G applied to the physical indices  (fused with a3)
//   a3  FP64 column norms of theta, ||theta||_F^2
//   a4-a9  pivoted QR with delayed panel updates   (qrcp.hpp + MFMA GEMM)
//   a10 eps^2 = ||R22||_F^2 from the final trailing block
//   a11 Q_k = H_0 ... H_{k-1} [I; 0] by blocked backward accumulation
//   a12 split: A_i' = Q_k, A_{i+1}' = R_k P^T (scaled)
//
// Site storage: A[l, s, r] at l + chi_l*(s + 2r) (column-major in (l, s, r)).
// Site i is then a column-major (2 chi_l) x chi_m matrix with row l + chi_l*s,
// site i+1 a column-major chi_m x (2 chi_r) matrix with column s + 2r, and
// theta is column-major (2 chi_l) x (2 chi_r); Q_k is the new site i and
// R_k P^T the new site i+1 without any transposition.
#pragma once
#include <mutex>
#include <vector>
#include "gemm.hpp"
#include "prof.hpp"
#include "qrcp.hpp"
#include "window.hpp"
#include "gram.hpp"
#include <stdarg.h>
#include <stdio.h>

// What the last failed pivoted QR of this host thread found inconsistent (the
// hipErrorUnknown returns of run_qrcp and window_panel below); empty when none.
static thread_local char g_qr_diag[320];

static void qr_diag(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
static void qr_diag(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_qr_diag, sizeof(g_qr_diag), fmt, ap);
    va_end(ap);
}

struct Gate4 {
    double2 g[16];   // row-major: g[4*(2a'+b') + (2a+b)]
};

// a2 + a3: apply the gate in place to column pair (b=0,b=1) of bond index r
// and row pair (a=0,a=1) of each l; FP64 norms of the two columns.
template <typename T>
__global__ __launch_bounds__(256) void k_gate_norms(QrcpDev<T> d, int64_t chi_l, Gate4 G)
{
    __shared__ double red_lds[4 * 2];
    __shared__ double red_out[2];
    __shared__ ArgBest arg_lds[4];
    const int64_t r = blockIdx.x;
    const int64_t c0 = 2 * r, c1 = 2 * r + 1;
    double n0 = 0.0, n1 = 0.0;
    for (int64_t l = threadIdx.x; l < chi_l; l += 256) {
        double2 t[4];
        t[0] = to_d(d.A[l + d.lda * c0]);            // a=0, b=0
        t[1] = to_d(d.A[l + d.lda * c1]);            // a=0, b=1
        t[2] = to_d(d.A[l + chi_l + d.lda * c0]);    // a=1, b=0
        t[3] = to_d(d.A[l + chi_l + d.lda * c1]);    // a=1, b=1
        double2 o[4];
#pragma unroll
        for (int row = 0; row < 4; ++row) {
            double2 s = czero();
#pragma unroll
            for (int col = 0; col < 4; ++col) s = cadd(s, cmul(G.g[4 * row + col], t[col]));
            o[row] = s;
        }
        T o0 = from_d<T>(o[0]), o1 = from_d<T>(o[1]), o2 = from_d<T>(o[2]), o3 = from_d<T>(o[3]);
        d.A[l + d.lda * c0] = o0;
        d.A[l + d.lda * c1] = o1;
        d.A[l + chi_l + d.lda * c0] = o2;
        d.A[l + chi_l + d.lda * c1] = o3;
        n0 += cabs2(to_d(o0)) + cabs2(to_d(o2));
        n1 += cabs2(to_d(o1)) + cabs2(to_d(o3));
    }
    double v[2] = {n0, n1};
    block_sum_vec<2>(v, red_lds, red_out);
    ArgBest best;
    best.val = -1.0;
    best.key = 0x7fffffff;
    best.slot = -1;
    if (threadIdx.x < 2) {
        const int64_t c = c0 + threadIdx.x;
        d.nu[c] = red_out[threadIdx.x];
        d.nuref[c] = red_out[threadIdx.x];
        d.perm[c] = (int32_t)c;
        best.val = red_out[threadIdx.x];
        best.key = (int32_t)c;
        best.slot = (int32_t)c;
    }
    best = block_argmax256(best, arg_lds);
    if (threadIdx.x == 0) {
        d.cpart[r] = best;
        d.cflag[r] = 0;
        d.npart[r] = red_out[0] + red_out[1];
    }
}

// a12: RPt[:, perm[c]] = column c of R (rows < k; R[t,c] = 0 for t > c),
// times the scale 1/sqrt(||theta||^2 - eps^2) when renormalising.
template <typename T>
__global__ __launch_bounds__(256) void k_rpt(const T* A, int64_t lda, const int32_t* perm, int64_t k, int64_t n,
                                             T* out, int64_t ldo, const double* dsc, int renorm)
{
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    double s = 1.0;
    if (renorm) {
        const double kept = dsc[DSC_NORM2] - dsc[DSC_EPS2];
        s = kept > 0.0 ? 1.0 / sqrt(kept) : 1.0;
    }
    const int64_t oc = perm[c];
    for (int64_t t = threadIdx.x; t < k; t += 256) {
        double2 v = t <= c ? to_d(A[t + lda * c]) : czero();
        out[t + ldo * oc] = from_d<T>(cscale(v, s));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_eye(T* Q, int64_t ldq, int64_t m, int64_t k)
{
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        T v;
        v.x = (i == c) ? 1 : 0;
        v.y = 0;
        Q[i + ldq * c] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_cols(const T* src, int64_t lds, T* dst, int64_t ldd, int64_t m)
{
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
        dst[i + ldd * c] = src[i + lds * c];
}

#define UNGQR_NB 64

// T factor of a block reflector (forward, columnwise): H_0..H_{nb-1} = I - V T V^H
// with T[t,t] = tau_t and T[0:t, t] = -tau_t T[0:t, 0:t] (V^H V)[0:t, t].
// Computed by blocks of 16 columns: the diagonal blocks by that recurrence
// (all four at once, 16 dependent steps), then block column J from the
// blocks left of it as T[0:J, J] = -T[0:J, 0:J] (V^H V)[0:J, J] T[J, J]
// (the product rule for two block reflectors).  One block of 256 threads;
// G = V^H V (nb x nb, ld UNGQR_NB) from a GEMM.  Writes T[0:nb, 0:nb] (ld UNGQR_NB).
#define LARFT_B 16
template <typename T>
__device__ void larft_block(const T* G, const double2* tau, int nb, T* Tout)
{
    __shared__ double2 Ts[UNGQR_NB][UNGQR_NB + 1];
    __shared__ double2 Gs[UNGQR_NB][UNGQR_NB + 1];
    __shared__ double2 Xs[UNGQR_NB][LARFT_B + 1];
    const int tid = threadIdx.x;
    for (int q = tid; q < nb * nb; q += 256) {
        const int r = q % nb, c = q / nb;
        Gs[r][c] = to_d(G[r + UNGQR_NB * c]);
        Ts[r][c] = czero();
    }
    __syncthreads();
    // diagonal blocks: thread (blk, row s of the block); step tt fills column
    // 16 blk + tt of every block at once
    const int nblk = (nb + LARFT_B - 1) / LARFT_B;
    {
        const int blk = tid / LARFT_B, sl = tid % LARFT_B;   // 16 blocks x 16 rows of capacity
        const int c0 = blk * LARFT_B;
        for (int tt = 0; tt < LARFT_B; ++tt) {
            const int t = c0 + tt, s = c0 + sl;
            if (blk < nblk && t < nb) {
                const double2 tau_t = tau[t];
                if (sl < tt) {
                    double2 v = czero();
                    for (int u = s; u < t; ++u) v = cadd(v, cmul(Ts[s][u], Gs[u][t]));
                    Ts[s][t] = cscale(cmul(tau_t, v), -1.0);
                } else if (sl == tt) {
                    Ts[s][t] = tau_t;
                }
            }
            __syncthreads();
        }
    }
    // block columns 1 .. nblk-1
    for (int J = 1; J < nblk; ++J) {
        const int c0 = J * LARFT_B, cw = nb - c0 < LARFT_B ? nb - c0 : LARFT_B;
        // X = G[0:c0, J] T[J, J]
        for (int q = tid; q < c0 * cw; q += 256) {
            const int r = q % c0, cc = q / c0;
            double2 x = czero();
            for (int u = 0; u <= cc; ++u) x = cadd(x, cmul(Gs[r][c0 + u], Ts[c0 + u][c0 + cc]));
            Xs[r][cc] = x;
        }
        __syncthreads();
        // T[0:c0, J] = -T[0:c0, 0:c0] X   (T upper triangular)
        for (int q = tid; q < c0 * cw; q += 256) {
            const int r = q % c0, cc = q / c0;
            double2 y = czero();
            for (int u = r; u < c0; ++u) y = cadd(y, cmul(Ts[r][u], Xs[u][cc]));
            Ts[r][c0 + cc] = cscale(y, -1.0);
        }
        __syncthreads();
    }
    for (int q = tid; q < nb * nb; q += 256) {
        const int r = q % nb, c = q / nb;
        Tout[r + UNGQR_NB * c] = from_d<T>(Ts[r][c]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_larft(const T* G, const double2* tau, int nb, T* Tout)
{
    larft_block<T>(G, tau, nb, Tout);
}

// The T factors of every UNGQR_NB-column block of k reflectors at once (block b
// of the launch: G and T at offset b * UNGQR_NB^2, reflectors b*UNGQR_NB ..).
template <typename T>
__global__ __launch_bounds__(256) void k_larft_all(const T* G, const double2* tau, int64_t k, T* Tout)
{
    const int64_t b0 = (int64_t)blockIdx.x * UNGQR_NB;
    const int nb = (int)(k - b0 < UNGQR_NB ? k - b0 : UNGQR_NB);
    const int64_t off = (int64_t)blockIdx.x * UNGQR_NB * UNGQR_NB;
    larft_block<T>(G + off, tau + b0, nb, Tout + off);
}

// The R rows of a panel for the columns outside its window, from the split-K
// partial products of W = V^H A_o (nz slices, slice z at P + z*zs, ld ldp):
//   w = sum_z P_z[:, c]            (FP64, fixed order)
//   W2[:, c] = T^H w               (T: the panel's T factor, ld UNGQR_NB)
//   R12[:, c] = A_o[0:nbe, c] - V_top W2[:, c]   (V_top unit lower triangular)
// W2 and R12 have leading dimension UNGQR_NB.  nbe <= 32.  Each half
// wavefront (lane r = row r) takes one column at a time; T and V_top sit in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_panel_rows(const T* P, int64_t ldp, int64_t zs, int nz, const T* Tm,
                                                    const T* V, int64_t lda, const T* Ao, int64_t nout, int nbe,
                                                    T* W2, T* R12)
{
    __shared__ double2 Ts[32][33], Vs[32][33];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int q = tid; q < 32 * 32; q += 256) {
        const int r = q % 32, c = q / 32;
        const bool in = r < nbe && c < nbe;
        Ts[r][c] = in ? to_d(Tm[r + UNGQR_NB * c]) : czero();
        // V_top: entries below the diagonal from storage, 1 on it, 0 above
        Vs[r][c] = in && r > c ? to_d(V[r + lda * c]) : (in && r == c ? make_double2(1.0, 0.0) : czero());
    }
    __syncthreads();
    const int r = lane & 31, hb = lane & 32;
    const bool live = r < nbe;
    for (int64_t c = ((int64_t)blockIdx.x * 4 + wid) * 2 + (lane >> 5); c < nout; c += (int64_t)gridDim.x * 8) {
        // the partials in slice order, eight loads in flight at a time
        double2 w = czero();
        const T* pc = P + (live ? r : 0) + ldp * c;
        int z = 0;
        for (; z + 8 <= nz; z += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = pc[(int64_t)(z + u) * zs];
#pragma unroll
            for (int u = 0; u < 8; ++u) w = cadd(w, to_d(v[u]));
        }
        for (; z < nz; ++z) w = cadd(w, to_d(pc[(int64_t)z * zs]));
        if (!live) w = czero();
        double2 w2 = czero();
        for (int rr = 0; rr < nbe; ++rr) {
            const double2 wr = make_double2(__shfl(w.x, hb + rr, MPS_WAVE), __shfl(w.y, hb + rr, MPS_WAVE));
            w2 = cadd(w2, cmulc(Ts[rr][r], wr));   // (T^H)[r, rr] = conj(T[rr, r])
        }
        double2 vw = czero();
        for (int rr = 0; rr < nbe; ++rr) {
            const double2 x = make_double2(__shfl(w2.x, hb + rr, MPS_WAVE), __shfl(w2.y, hb + rr, MPS_WAVE));
            vw = cadd(vw, cmul(Vs[r][rr], x));
        }
        if (live) {
            W2[r + UNGQR_NB * c] = from_d<T>(w2);
            R12[r + UNGQR_NB * c] = from_d<T>(csub(to_d(Ao[r + lda * c]), vw));
        }
    }
}

// Scratch carved from a caller-provided workspace.
struct Carver {
    char* base;
    int64_t cap, used;
    void* take(int64_t bytes)
    {
        int64_t off = (used + 255) & ~(int64_t)255;
        if (bytes < 0 || off + bytes > cap) return nullptr;
        used = off + bytes;
        return base ? (void*)(base + off) : (void*)(intptr_t)(off + 256);
    }
};

template <typename T>
struct UpdateWs {
    QrcpDev<T> d;
    T* Gbuf;       // UNGQR_NB^2
    T* Tbuf;       // UNGQR_NB^2
    T* Tbuf2;      // UNGQR_NB^2: the T of alternate panels of the unpivoted QR (its update of panel p runs beside panel p+1)
    T* Wsm;        // UNGQR_NB^2: W = V^H A_t of the next panel's columns only (the lookahead update)
    T* W2sm;       // UNGQR_NB^2: and T^H W
    void* gsplit2; // split-K scratch of the GEMMs on the panel's stream while the trailing update runs beside it
    int64_t gsplit2_bytes;
    T* Gall;       // Q formation: V^H V of every UNGQR_NB block (ceil(k / UNGQR_NB) x UNGQR_NB^2)
    T* Tall;       // and their T factors
    T* Wbuf;       // UNGQR_NB x k
    T* W2buf;      // UNGQR_NB x k
    void* gsplit;  // split-K scratch
    int64_t gsplit_bytes;
    int nb;        // QRCP panel width
    int win;       // candidate-window width of the pivoted panels (0: every panel reads the whole trailing block)
    int32_t* wplan;          // 1 + 2 * QR_WIN_MAX: swap plan of a window selection
    T* wsave;                // min(QR_WIN_MAX, n) columns of lda: the window state at the panel start
    double* wsnu;            // QR_WIN_MAX
    double* wsnuref;         // QR_WIN_MAX
    int32_t* wsperm;         // QR_WIN_MAX
    ArgBest* wcp;            // 2 * QR_WIN_MAX: argmax partials of the right-looking window steps (double buffer)
    int32_t* wpiv;           // QR_NBMAX: pivot positions of those steps
    int32_t* wstep;          // QR_WIN_MAX: step at which a window column became the pivot
    int32_t* worder;         // 1 + 3 QR_WIN_MAX: the panel-end column moves of the window
    T* wtmp;                 // like wsave: the window reordered at the panel end
    T* vbuf;                 // QR_NBMAX columns of lda: beta and v of those steps
    int32_t* wflag;          // QR_NBMAX: step flags of the one-launch unpivoted panels
    double2* wscale;         // QR_NBMAX: the FP64 scale of those panels' reflectors
    double* wtnu;            // QR_WIN_MAX
    double* wtnuref;         // QR_WIN_MAX
    int32_t* wtperm;         // QR_WIN_MAX
    T* gw;                   // GRAM_W_MAX^2: the Gram matrix of a window (Gram panels)
    double2* gq;             // GRAM_NB_MAX columns of lda: Q of the panel's pivots in FP64 (Gram panels)
    double2* gsm;            // GSM_COUNT: the panel's small FP64 factors (Gram panels)
};

static inline int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Lay out the workspace of one factorisation of an m x n matrix with k steps.
// theta_in_ws: whether theta itself lives in the workspace.  With base == null
// only sizes are computed; returns false when cap is too small.
template <typename T>
static bool carve_update_ws(Carver& cv, UpdateWs<T>& w, int64_t m, int64_t n, int64_t k, bool theta_in_ws)
{
    QrcpDev<T>& d = w.d;
    d.m = m; d.n = n; d.k = k; d.lda = m > 1 ? m + (m & 1) : 2;   // even: 16-byte aligned columns
    d.A = theta_in_ws ? (T*)cv.take((int64_t)sizeof(T) * d.lda * n) : nullptr;
    d.nu = (double*)cv.take(8 * (n + 1));
    d.nuref = (double*)cv.take(8 * (n + 1));
    d.perm = (int32_t*)cv.take(4 * (n + 1));
    d.ldf = n > 1 ? n : 1;
    d.F = (T*)cv.take((int64_t)sizeof(T) * d.ldf * QR_NBMAX);
    d.tau = (double2*)cv.take(16 * (k + 1));
    d.diagR = (double*)cv.take(8 * (k + 1));
    d.xbuf = (double2*)cv.take(16 * (m + 1));
    d.xlo = (T*)cv.take((int64_t)sizeof(T) * (d.lda + 2));
    d.apart = (double*)cv.take(8 * APART_STRIDE * (rup(m, 256) + 1));
    d.hh = (double2*)cv.take(16 * (4 + QR_NBMAX));
    d.fsave = (double2*)cv.take(16 * QR_NBMAX);
    d.pivval = (double*)cv.take(8 * QR_NBMAX);
    d.pivkey = (int32_t*)cv.take(4 * QR_NBMAX);
    const int64_t np = rup(n, QR_CW) + rup(n, 2) + 8;
    d.cpart = (ArgBest*)cv.take((int64_t)sizeof(ArgBest) * np);
    d.npart = (double*)cv.take(8 * np);
    d.cflag = (int32_t*)cv.take(4 * np);
    d.ctl = (int32_t*)cv.take(4 * CTL_COUNT);
    d.dsc = (double*)cv.take(8 * DSC_COUNT);
    w.Gbuf = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB);
    w.Tbuf = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB);
    w.Tbuf2 = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB);
    w.Wsm = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB);
    w.W2sm = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB);
    w.gsplit2_bytes = (int64_t)sizeof(T) * 16 * UNGQR_NB * UNGQR_NB;
    w.gsplit2 = cv.take(w.gsplit2_bytes);
    const int64_t qblocks = (k + UNGQR_NB - 1) / UNGQR_NB > 0 ? (k + UNGQR_NB - 1) / UNGQR_NB : 1;
    w.Gall = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB * qblocks);
    w.Tall = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * UNGQR_NB * qblocks);
    // W / W2 hold nb x (columns right of a panel): up to n (blocked QR) or k (UNGQR)
    const int64_t wcols = (n > k ? n : k) + 1;
    w.Wbuf = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * wcols);
    w.W2buf = (T*)cv.take((int64_t)sizeof(T) * UNGQR_NB * wcols);
    const int64_t sk = (int64_t)sizeof(T) * 16 * UNGQR_NB * (wcols > UNGQR_NB ? wcols : UNGQR_NB);
    w.gsplit = cv.take(sk);
    w.gsplit_bytes = sk;
    const int64_t wmax = n < QR_WIN_MAX ? n : QR_WIN_MAX;
    w.wplan = (int32_t*)cv.take(4 * (1 + 3 * QR_WIN_MAX));
    w.wsave = (T*)cv.take((int64_t)sizeof(T) * d.lda * (wmax > 0 ? wmax : 1));
    w.wsnu = (double*)cv.take(8 * QR_WIN_MAX);
    w.wsnuref = (double*)cv.take(8 * QR_WIN_MAX);
    w.wsperm = (int32_t*)cv.take(4 * QR_WIN_MAX);
    w.wcp = (ArgBest*)cv.take((int64_t)sizeof(ArgBest) * 2 * QR_WIN_MAX);
    w.wpiv = (int32_t*)cv.take(4 * QR_NBMAX);
    w.wstep = (int32_t*)cv.take(4 * QR_WIN_MAX);
    w.worder = (int32_t*)cv.take(4 * (1 + 3 * QR_WIN_MAX));
    w.wtmp = (T*)cv.take((int64_t)sizeof(T) * d.lda * (wmax > 0 ? wmax : 1));
    w.vbuf = (T*)cv.take((int64_t)sizeof(T) * d.lda * QR_NBMAX);
    w.wflag = (int32_t*)cv.take(4 * QR_NBMAX);
    w.wscale = (double2*)cv.take(16 * QR_NBMAX);
    w.wtnu = (double*)cv.take(8 * QR_WIN_MAX);
    w.wtnuref = (double*)cv.take(8 * QR_WIN_MAX);
    w.wtperm = (int32_t*)cv.take(4 * QR_WIN_MAX);
    w.gw = (T*)cv.take((int64_t)sizeof(T) * GRAM_W_MAX * GRAM_W_MAX);
    w.gq = (double2*)cv.take((int64_t)16 * d.lda * GRAM_NB_MAX);
    w.gsm = (double2*)cv.take((int64_t)16 * GSM_COUNT);
    w.win = 0;
    return d.nu && d.nuref && d.perm && d.F && d.tau && d.diagR && d.xbuf && d.xlo && d.apart && d.hh && d.fsave &&
           d.cpart && d.npart && d.cflag && d.ctl && d.dsc && w.Gbuf && w.Tbuf && w.Tbuf2 && w.Wsm && w.W2sm &&
           w.gsplit2 && w.Gall && w.Tall && w.Wbuf && w.W2buf && w.gsplit &&
           d.pivval && d.pivkey && w.wplan && w.wsave && w.wsnu && w.wsnuref && w.wsperm && w.wcp &&
           w.wpiv && w.wstep && w.worder && w.wtmp && w.vbuf && w.wflag && w.wscale && w.wtnu && w.wtnuref && w.wtperm &&
           w.gw && w.gq && w.gsm &&
           (!theta_in_ws || d.A);
}

static const double2 C_ONE = {1.0, 0.0};
static const double2 C_MONE = {-1.0, 0.0};
static const double2 C_ZERO = {0.0, 0.0};

struct QrcpStats {
    int panels = 0;
    int refreshes = 0;
    int window_misses = 0;   // window panels cut short by the greedy replay
};

template <typename T> static void run_window_steps(UpdateWs<T>& w, hipStream_t st, int64_t p0, int64_t nsteps, int W);
template <typename T> static void window_reorder(UpdateWs<T>& w, hipStream_t st, int64_t p0, int nbe, int W);
template <typename T> static void run_fixed_panel(UpdateWs<T>& w, hipStream_t st, int64_t p0, int64_t nsteps, int W);

// Set for the duration of a call that must not allocate: the control-block
// readback then uses its pinned mailbox only if an earlier call has already
// allocated it, and the unpivoted QR keeps to the caller's stream.
static thread_local bool g_no_alloc = false;

// How the pivoted window panels take their steps (mps_set_panel_mode):
// 0 one launch per pivot step, 1 pivots from the window's Gram matrix.
// Process-wide.
static int g_panel_mode = 0;

// A second stream per device and host thread (default priority, created on
// first use and kept for the life of the thread) with three events, for the
// trailing updates that run beside the next panel's factorisation.  Null when
// it cannot be created or when the caller must not allocate; the work then
// stays on the caller's stream.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, panel = nullptr, trail = nullptr;
    bool failed = false;
};
#define SIDE_MAX_DEVICES 16
static SideStream* side_stream()
{
    if (g_no_alloc) return nullptr;
    static thread_local SideStream per_dev[SIDE_MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SIDE_MAX_DEVICES) return nullptr;
    SideStream& ss = per_dev[dev];
    if (ss.failed) return nullptr;
    if (!ss.s) {
        if (hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ss.panel, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ss.trail, hipEventDisableTiming) != hipSuccess) {
            ss.failed = true;
            (void)hipGetLastError();
            return nullptr;
        }
    }
    return &ss;
}

// A_t -= V T^H... : the block reflector of one panel applied to the columns
// A_t (rows x cols, from row p0) as three MFMA GEMMs W = V^H A_t, W2 = T^H W,
// A_t -= V W2, on stream st with its own W, W2 and split-K scratch.
template <typename T>
static bool panel_update(hipStream_t st, const T* V, int64_t lda, const T* Tm, int nbe, int64_t rows, int64_t cols,
                         T* At, T* Wb, T* W2b, int64_t ldw, void* split, int64_t split_bytes)
{
    const double rc = (double)rows * (double)cols;
    hipEvent_t et = prof_begin(st);
    if (!zgemm<T>(st, OP_C, true, OP_N, false, nbe, cols, rows, C_ONE, V, lda, At, lda, C_ZERO, Wb, ldw, split,
                  split_bytes))
        return false;
    prof_end(et, st, PK_PANEL, (double)sizeof(T) * rc, 8.0 * nbe * rc);
    hipEvent_t e2 = prof_begin(st);
    if (!zgemm<T>(st, OP_C, false, OP_N, false, nbe, cols, nbe, C_ONE, Tm, UNGQR_NB, Wb, ldw, C_ZERO, W2b, ldw,
                  nullptr, 0))
        return false;
    prof_end(e2, st, PK_REFL, (double)sizeof(T) * 2.0 * nbe * cols, 8.0 * (double)nbe * nbe * cols);
    hipEvent_t eu = prof_begin(st);
    if (!zrank_update<T>(st, true, rows, cols, nbe, C_MONE, V, lda, W2b, ldw, At, lda) &&
        !zgemm<T>(st, OP_N, true, OP_N, false, rows, cols, nbe, C_MONE, V, lda, W2b, ldw, C_ONE, At, lda, nullptr, 0))
        return false;
    prof_end(eu, st, PK_TRAIL, 2.0 * (double)sizeof(T) * rc, 8.0 * nbe * rc);
    return true;
}

// Householder QR of d.A with the columns in their given order (a centre move,
// or QR with a column order known in advance).  Only the panel's own columns
// go through per-column steps; the trailing columns receive the panel's block
// reflector I - V T V^H at the panel end (panel_update).  With the order
// fixed, panel p + 1 depends only on its own columns, so the update is split
// (look-ahead): the next panel's columns are updated on the caller's stream,
// right before that panel is factorised, while the rest of the trailing
// block is updated on a second stream, beside the factorisation of panel
// p + 1.  Events keep the order per column: panel p's update of the far
// columns waits for panel p's factors, and the next-panel update of panel
// p + 1's columns waits for panel p - 1's far update, which covered them.
// T is double-buffered (panel p's far update may still read it while panel
// p + 1 forms its own), and each stream has its own GEMM scratch.
// While the rows left fit one window-step block (m - p0 <= 8192), a panel is
// a window of its own nb columns factorised by one k_fixed_panel launch
// (each column's block applies the panel's earlier reflectors as they are
// published); taller panels take the delayed-update steps (step A + step C,
// two launches per column).  Either way a GEMM forms V^H V for T.  Nothing
// depends on data on the host, so no synchronisation is needed; the caller's
// stream waits for the second stream before the final norm, so the call
// keeps stream semantics.
template <typename T>
static hipError_t run_blocked_fixed(UpdateWs<T>& w, hipStream_t st, QrcpStats* stats)
{
    QrcpDev<T>& d = w.d;
    const int64_t m = d.m, n = d.n, k = d.k;
    const int nb = w.nb < UNGQR_NB ? w.nb : UNGQR_NB;
    const unsigned na = (unsigned)rup(m, 256);
    SideStream* ss = n > nb ? side_stream() : nullptr;
    hipStream_t s2 = ss ? ss->s : st;
    if (ss) {
        if (hipEventRecord(ss->fork, st) != hipSuccess || hipStreamWaitEvent(s2, ss->fork, 0) != hipSuccess)
            return hipErrorInvalidValue;
    }
    bool far_pending = false;   // a far update has been issued on s2 (ss->trail marks its end)
    hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)0);
    hipLaunchKernelGGL(k_fixed_flags_reset, dim3(1), dim3(QR_NBMAX), 0, st, w.wflag, (int)QR_NBMAX);
    int parity = 0;
    for (int64_t p0 = 0; p0 < k; p0 += nb, parity ^= 1) {
        const int64_t pend = (p0 + nb < k) ? p0 + nb : k;
        const int nbe = (int)(pend - p0);
        const bool right = m - p0 <= (int64_t)WSTEP_NT * WSTEP_RPT;
        if (right) {
            hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)p0);
            run_fixed_panel<T>(w, st, p0, nbe, nbe);
            window_reorder<T>(w, st, p0, nbe, nbe);
        }
        for (int64_t jc = right ? pend : p0; jc < pend; ++jc) {
            const int jj = (int)(jc - p0);
            hipEvent_t ea = prof_begin(st);
            launch_step_a<T>(d, na, jc, p0, jj, 0, st);
            prof_end(ea, st, PK_STEP_A, (double)sizeof(T) * (double)(m - jc) * (jj + 1), 8.0 * (m - jc) * jj);
            const int64_t ncol = pend - jc - 1;
            const unsigned nc = (unsigned)(ncol > 0 ? rup(ncol, QR_CW) : 1);
            hipEvent_t ec = prof_begin(st, PK_STEP_C);
            hipLaunchKernelGGL((k_step_c<T>), dim3(nc), dim3(256), 0, st, d, jc, p0, jj, pend, (int)na);
            prof_end(ec, st, PK_STEP_C, (double)sizeof(T) * (double)(m - jc) * (double)(ncol > 0 ? ncol : 0),
                     8.0 * (double)(m - jc) * (double)(ncol > 0 ? ncol : 0));
        }
        if (stats) stats->panels++;
        if (pend >= n) continue;
        const T* V = d.A + p0 + d.lda * p0;
        const int64_t rows = m - p0;
        T* Tm = parity ? w.Tbuf2 : w.Tbuf;
        hipEvent_t eg = prof_begin(st);
        // G = V^H V, then T
        if (!zgemm<T>(st, OP_C, true, OP_N, true, nbe, nbe, rows, C_ONE, V, d.lda, V, d.lda, C_ZERO, w.Gbuf,
                      UNGQR_NB, w.gsplit2, w.gsplit2_bytes))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_larft<T>), dim3(1), dim3(256), 0, st, w.Gbuf, d.tau + p0, nbe, Tm);
        prof_end(eg, st, PK_REFL, (double)sizeof(T) * rows * nbe, 8.0 * (double)nbe * nbe * rows);
        // the next panel's columns [pend, pend + nb) on st, after the far
        // update of the previous panel (which covered them)
        const int64_t near_end = pend + nb < n ? pend + nb : n;
        const int64_t far_cols = n - near_end;
        if (far_pending && hipStreamWaitEvent(st, ss->trail, 0) != hipSuccess) return hipErrorInvalidValue;
        if (far_cols > 0 && ss && hipEventRecord(ss->panel, st) != hipSuccess) return hipErrorInvalidValue;
        if (!panel_update<T>(st, V, d.lda, Tm, nbe, rows, near_end - pend, d.A + p0 + d.lda * pend, w.Wsm, w.W2sm,
                             UNGQR_NB, w.gsplit2, w.gsplit2_bytes))
            return hipErrorInvalidValue;
        if (far_cols > 0) {
            // the rest of the trailing block beside the next panel
            if (ss && hipStreamWaitEvent(s2, ss->panel, 0) != hipSuccess) return hipErrorInvalidValue;
            if (!panel_update<T>(s2, V, d.lda, Tm, nbe, rows, far_cols, d.A + p0 + d.lda * near_end, w.Wbuf,
                                 w.W2buf, UNGQR_NB, w.gsplit, w.gsplit_bytes))
                return hipErrorInvalidValue;
            if (ss) {
                if (hipEventRecord(ss->trail, s2) != hipSuccess) return hipErrorInvalidValue;
                far_pending = true;
            }
        }
    }
    if (far_pending && hipStreamWaitEvent(st, ss->trail, 0) != hipSuccess) return hipErrorInvalidValue;
    // a10: ||R22||_F^2 over the final trailing block
    if (m > k && n > k) {
        const unsigned nblk = (unsigned)rup(n - k, QR_CW);
        hipLaunchKernelGGL((k_colnorms<T>), dim3(nblk), dim3(256), 0, st, d, k, k, 0, 0);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double*)d.npart, (int)nblk, d.dsc,
                           (int)DSC_EPS2);
    }
    return hipGetLastError();
}

// Pivot steps jc = p0 .. p0+nsteps-1 of one panel; step C covers the columns
// up to cend (the whole trailing block, or a candidate window with one column
// per block).  Returns the number of argmax partials of the last step C.
template <typename T>
static int run_panel_steps(QrcpDev<T>& d, hipStream_t st, int64_t p0, int64_t nsteps, int64_t cend, bool window,
                           int nparts)
{
    const int64_t m = d.m;
    const unsigned na = (unsigned)rup(m, 256);
    for (int64_t jc = p0; jc < p0 + nsteps; ++jc) {
        const int jj = (int)(jc - p0);
        hipEvent_t ea = prof_begin(st);
        launch_step_a<T>(d, na, jc, p0, jj, nparts, st);
        prof_end(ea, st, PK_STEP_A, (double)sizeof(T) * (double)(m - jc) * (jj + 1), 8.0 * (m - jc) * jj);
        const int64_t ncol = cend - jc - 1;
        const int cw = window ? 1 : QR_CW;
        const unsigned nc = (unsigned)(ncol > 0 ? rup(ncol, cw) : 1);
        hipEvent_t ec = prof_begin(st, PK_STEP_C);
        if (window)
            hipLaunchKernelGGL((k_step_c<T, 1>), dim3(nc), dim3(256), 0, st, d, jc, p0, jj, cend, (int)na);
        else
            hipLaunchKernelGGL((k_step_c<T, QR_CW>), dim3(nc), dim3(256), 0, st, d, jc, p0, jj, cend, (int)na);
        nparts = (int)nc;
        // algorithmic traffic of one step: one read of the columns it covers
        prof_end(ec, st, PK_STEP_C, (double)sizeof(T) * (double)(m - jc) * (double)(ncol > 0 ? ncol : 0),
                 8.0 * (double)(m - jc) * (double)(ncol > 0 ? ncol : 0));
    }
    return nparts;
}

// Host copy of the control block after a stream synchronisation.
// Host readback of the control block.  A one-block kernel copies it into
// coherent pinned host memory and then publishes a sequence number there; the
// host spins on that number instead of synchronising the stream and copying
// into pageable memory (about 7 us per readback instead of about 23).  The
// mailbox is process-global and is allocated on first use; a mutex makes each
// readback (export launch and spin) one critical section, so host threads
// that factorise on different streams never read each other's control blocks.
// Without the mailbox the readback is a copy and a stream synchronisation.
struct CtlMailbox {
    int32_t* buf = nullptr;   // CTL_COUNT values, then the sequence number
    int32_t seq = 0;
    bool tried = false;
    std::mutex mu;
};
static CtlMailbox g_ctl_mbox;

__global__ __launch_bounds__(64) void k_ctl_export(const int32_t* ctl, int32_t* hbuf, int32_t seq)
{
    const int t = threadIdx.x;
    if (t < CTL_COUNT) __hip_atomic_store(hbuf + t, ctl[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
    __syncthreads();
    if (t == 0) __hip_atomic_store(hbuf + CTL_COUNT, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
static hipError_t read_ctl(const QrcpDev<T>& d, hipStream_t st, int32_t* hctl)
{
    CtlMailbox& mb = g_ctl_mbox;
    std::lock_guard<std::mutex> lock(mb.mu);
    if (!mb.tried && !g_no_alloc) {
        mb.tried = true;
        void* p = nullptr;
        if (hipHostMalloc(&p, 64 * sizeof(int32_t), hipHostMallocCoherent | hipHostMallocPortable) == hipSuccess) {
            mb.buf = (int32_t*)p;
            for (int i = 0; i <= CTL_COUNT; ++i) mb.buf[i] = 0;
        } else {
            (void)hipGetLastError();
        }
    }
    if (!mb.buf) {
        hipError_t e = hipMemcpyAsync(hctl, d.ctl, sizeof(int32_t) * CTL_COUNT, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(st);
        prof_flush();
        return e;
    }
    mb.seq = mb.seq == 0x7fffffff ? 1 : mb.seq + 1;
    const int32_t seq = mb.seq;
    hipLaunchKernelGGL(k_ctl_export, dim3(1), dim3(64), 0, st, (const int32_t*)d.ctl, mb.buf, seq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // spin on the sequence number; every 1024 polls ask whether the stream
    // has drained or failed, so a failed launch cannot leave the host waiting
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(mb.buf + CTL_COUNT, __ATOMIC_ACQUIRE) == seq) break;
        if ((it & 1023) == 0) {
            e = hipStreamQuery(st);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return e;
            // drained: the number is in host memory once the kernel has completed
            bool seen = false;
            for (int r = 0; r < 4096 && !seen; ++r) seen = __atomic_load_n(mb.buf + CTL_COUNT, __ATOMIC_ACQUIRE) == seq;
            if (seen) break;
            qr_diag("control readback: the stream drained without publishing sequence %d", (int)seq);
            return hipErrorUnknown;
        }
    }
    for (int i = 0; i < CTL_COUNT; ++i) hctl[i] = __atomic_load_n(mb.buf + i, __ATOMIC_RELAXED);
    prof_flush();
    return hipSuccess;
}

// Select the window for a panel at p0, bring it to [p0, p0+W) and save that state.
template <typename T>
static void window_setup(UpdateWs<T>& w, hipStream_t st, int64_t p0, bool save)
{
    QrcpDev<T>& d = w.d;
    const int W = w.win;
    hipLaunchKernelGGL((k_window_select<T>), dim3(1), dim3(1024), 0, st, d, p0, W, w.wplan, w.wcp);
    hipLaunchKernelGGL((k_window_place<T>), dim3((unsigned)W), dim3(256), 0, st, d, p0, W, (const int32_t*)w.wplan,
                       w.wsave, d.lda, w.wsnu, w.wsnuref, w.wsperm, save ? 1 : 0);
}

// Right-looking pivot steps p0 .. p0+nsteps-1 inside the window (k_window_step),
// then the window's columns in their final order: pivots first, in step order.
template <typename T>
static void run_window_steps(UpdateWs<T>& w, hipStream_t st, int64_t p0, int64_t nsteps, int W)
{
    QrcpDev<T>& d = w.d;
    // sampled profiling times the whole run with one event pair
    hipEvent_t er = prof_begin_run(st);
    double rbytes = 0.0, rflops = 0.0;
    // the block shape follows the rows left: one wave of 8 rows per lane up to
    // 512 rows, four waves up to 2048, otherwise 512 threads of 16 rows
    const int64_t rows0 = d.m - p0;
    for (int64_t jj = 0; jj < nsteps; ++jj) {
        const int64_t j = p0 + jj;
        hipEvent_t ec = g_prof.stride > 1 ? nullptr : prof_begin(st, PK_STEP_C);
        const ArgBest* cin = w.wcp + (jj & 1) * QR_WIN_MAX;
        ArgBest* cout = w.wcp + ((jj + 1) & 1) * QR_WIN_MAX;
        if (rows0 <= 64 * 8)
            hipLaunchKernelGGL((k_window_step<T, 64, 8>), dim3((unsigned)W), dim3(64), 0, st, d, j, p0, (int)jj, cin,
                               cout, w.wpiv, w.vbuf, w.wstep, w.Gbuf, (int)UNGQR_NB);
        else if (rows0 <= 256 * 8)
            hipLaunchKernelGGL((k_window_step<T, 256, 8>), dim3((unsigned)W), dim3(256), 0, st, d, j, p0, (int)jj,
                               cin, cout, w.wpiv, w.vbuf, w.wstep, w.Gbuf, (int)UNGQR_NB);
        else
            hipLaunchKernelGGL((k_window_step<T>), dim3((unsigned)W), dim3(WSTEP_NT), 0, st, d, j, p0, (int)jj, cin,
                               cout, w.wpiv, w.vbuf, w.wstep, w.Gbuf, (int)UNGQR_NB);
        // algorithmic traffic of one step: the window right of the pivot read and written once
        const double cols = (double)(p0 + W - j - 1), rows = (double)(d.m - j);
        prof_end(ec, st, PK_STEP_C, 2.0 * sizeof(T) * rows * cols, 16.0 * rows * cols);
        rbytes += 2.0 * sizeof(T) * rows * cols;
        rflops += 16.0 * rows * cols;
    }
    prof_end(er, st, PK_STEP_C, rbytes, rflops, nsteps);
}

// Unpivoted steps p0 .. p0+nsteps-1 of a window of W columns in column
// order: one k_fixed_panel launch (the block shape follows the rows left, as
// in run_window_steps).  The flags must have been reset for this
// factorisation (k_fixed_flags_reset); the epoch p0 + 1 is then new to them.
template <typename T>
static void run_fixed_panel(UpdateWs<T>& w, hipStream_t st, int64_t p0, int64_t nsteps, int W)
{
    QrcpDev<T>& d = w.d;
    const int64_t rows0 = d.m - p0;
    const int32_t epoch = (int32_t)(p0 + 1);
    hipEvent_t ec = prof_begin(st, PK_STEP_C);
    if (rows0 <= 64 * 8)
        hipLaunchKernelGGL((k_fixed_panel<T, 64, 8>), dim3((unsigned)W), dim3(64), 0, st, d, p0, (int)nsteps, epoch,
                           w.wflag, w.wscale, w.wpiv, w.vbuf);
    else if (rows0 <= 256 * 8)
        hipLaunchKernelGGL((k_fixed_panel<T, 256, 8>), dim3((unsigned)W), dim3(256), 0, st, d, p0, (int)nsteps, epoch,
                           w.wflag, w.wscale, w.wpiv, w.vbuf);
    else
        hipLaunchKernelGGL((k_fixed_panel<T, WSTEP_NT, WSTEP_RPT>), dim3((unsigned)W), dim3(WSTEP_NT), 0, st, d, p0,
                           (int)nsteps, epoch, w.wflag, w.wscale, w.wpiv, w.vbuf);
    // algorithmic traffic: every column of the window read and written once,
    // each reflector's rows read once per column right of it
    double by = 2.0 * sizeof(T) * (double)rows0 * W, fl = 0.0;
    for (int64_t s = 0; s < nsteps; ++s) {
        by += sizeof(T) * (double)(rows0 - s) * (double)(W - s - 1);
        fl += 16.0 * (double)(rows0 - s) * (double)(W - s - 1);
    }
    prof_end(ec, st, PK_STEP_C, by, fl);
}

template <typename T>
static void window_reorder(UpdateWs<T>& w, hipStream_t st, int64_t p0, int nbe, int W)
{
    QrcpDev<T>& d = w.d;
    hipEvent_t ew = prof_begin(st);
    hipLaunchKernelGGL(k_window_order, dim3(1), dim3(1024), 0, st, (const int32_t*)w.wpiv, nbe, p0, W, w.worder);
    // at most 2 nbe columns move
    dim3 grid((unsigned)(rup(d.m, 256) < 64 ? rup(d.m, 256) : 64), (unsigned)(2 * nbe < W ? 2 * nbe : W));
    hipLaunchKernelGGL((k_window_gather<T>), grid, dim3(256), 0, st, d, (const int32_t*)w.worder, p0,
                       (const T*)w.vbuf, w.wtmp, w.wtnu, w.wtnuref, w.wtperm, 0);
    hipLaunchKernelGGL((k_window_gather<T>), grid, dim3(256), 0, st, d, (const int32_t*)w.worder, p0,
                       (const T*)w.vbuf, w.wtmp, w.wtnu, w.wtnuref, w.wtperm, 1);
    prof_end(ew, st, PK_WINDOW, (double)sizeof(T) * 8.0 * (double)d.m * nbe, 0.0);
}

// Unpivoted Householder QR with every column in one window (n <= WSTEP_NT,
// m <= WSTEP_NT * WSTEP_RPT): per panel of nb columns, one k_fixed_panel
// launch over every remaining column (each reflector reaches every column
// right of it, so no trailing update is left), then the panel's reflectors
// are written into place.  For the centre moves of bonds up to a few
// hundred.
template <typename T>
static hipError_t run_window_fixed(UpdateWs<T>& w, hipStream_t st, QrcpStats* stats)
{
    QrcpDev<T>& d = w.d;
    const int64_t n = d.n, k = d.k;
    const int nb = w.nb > 0 && w.nb < QR_NBMAX ? w.nb : 32;
    hipLaunchKernelGGL(k_fixed_flags_reset, dim3(1), dim3(QR_NBMAX), 0, st, w.wflag, (int)QR_NBMAX);
    for (int64_t p0 = 0; p0 < k; p0 += nb) {
        const int64_t nsteps = (p0 + nb < k ? p0 + nb : k) - p0;
        const int W = (int)(n - p0);
        hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)p0);
        run_fixed_panel<T>(w, st, p0, nsteps, W);
        window_reorder<T>(w, st, p0, (int)nsteps, W);
        if (stats) stats->panels++;
    }
    return hipGetLastError();
}

// The replay's outcome applied on the device, before the host has read it:
// t* = min(nbe, first failing step, first flag) as the host computes it, the
// rows t >= t* of W2 (UNGQR_NB x nout) set to zero, so that the rank-nbe
// update A_o -= V W2 that follows is exactly the rank-t* one, and, unless a
// norm refresh is due (stop flag or first flag <= t*, with p0 + t* < k), the
// outside columns' norms downdated by their R rows 0 .. t*-1 in R12 (the
// arithmetic of k_window_commit).  One thread per outside column c0 + q.
template <typename T>
__global__ __launch_bounds__(256) void k_replay_commit(QrcpDev<T> d, int64_t p0, int nbe, T* W2, const T* R12,
                                                       int64_t ldw, int64_t c0, int64_t nout)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nout) return;
    int tstar = nbe;
    if (d.ctl[CTL_TFAIL] < tstar) tstar = d.ctl[CTL_TFAIL];
    if (d.ctl[CTL_TFLAG] < tstar) tstar = d.ctl[CTL_TFLAG];
    if (tstar < 0) tstar = 0;
    const bool refresh = d.ctl[CTL_STOP] != 0 || d.ctl[CTL_TFLAG] <= tstar;
    for (int t = tstar; t < nbe; ++t) W2[t + ldw * q] = from_d<T>(czero());
    if (refresh && p0 + tstar < d.k) return;
    const int64_t c = c0 + q;
    const T* rq = R12 + ldw * q;
    double s = d.nu[c];
    for (int t = 0; t < tstar; ++t) {
        const double nn = s - cabs2(to_d(rq[t]));
        s = nn < 0.0 ? 0.0 : nn;
    }
    d.nu[c] = s;
}

// The window's columns and their norms and keys back from the state saved at
// the panel's set-up.
template <typename T>
static void window_restore(UpdateWs<T>& w, hipStream_t st, int64_t p0, int W)
{
    QrcpDev<T>& d = w.d;
    dim3 grid((unsigned)(rup(d.m, 256) < 64 ? rup(d.m, 256) : 64), (unsigned)W);
    hipLaunchKernelGGL((k_copy_cols<T>), grid, dim3(256), 0, st, (const T*)w.wsave, d.lda, d.A + d.lda * p0, d.lda,
                       d.m);
    hipLaunchKernelGGL((k_window_meta<T>), dim3((unsigned)rup(W, 256)), dim3(256), 0, st, d, p0, W, w.wsnu,
                       w.wsnuref, w.wsperm, 1);
}

// Up to nsteps pivot steps of the window at p0 from its Gram matrix
// (gram.hpp): exact norms and G, pivoted Cholesky, CholeskyQR2 of the chosen
// columns, Householder reconstruction.  Leaves what the right-looking steps
// leave for the window reorder (ctl JDONE, wpiv, vbuf, the R rows above the
// diagonal in the pivot columns, tau, diagR, pivval, pivkey) and the panel's
// T factor in w.Tbuf; the window's other columns keep their panel-start
// values.  ctl JDONE = p0 when no step could be taken.
template <typename T>
static hipError_t gram_panel_steps(UpdateWs<T>& w, hipStream_t st, int64_t p0, int nsteps, int W)
{
    QrcpDev<T>& d = w.d;
    const int64_t rows = d.m - p0;
    const unsigned rb = (unsigned)rup(rows, GRAM_ROWS_NT);
    hipEvent_t eg = prof_begin(st, PK_STEP_C);
    hipLaunchKernelGGL((k_win_norms<T>), dim3((unsigned)W), dim3(256), 0, st, d, p0);
    const T* Aw = d.A + p0 + d.lda * p0;
    if (!zgemm<T>(st, OP_C, false, OP_N, false, W, W, rows, C_ONE, Aw, d.lda, Aw, d.lda, C_ZERO, w.gw,
                  GRAM_W_MAX, w.gsplit, w.gsplit_bytes))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gram_pivots<T>), dim3(1), dim3(256), 0, st, d, (const T*)w.gw, (int64_t)GRAM_W_MAX, p0, W,
                       nsteps, w.wpiv, w.gsm + GSM_R1);
    hipLaunchKernelGGL((k_cqr_trsm<T, true>), dim3(rb), dim3(GRAM_ROWS_NT), 0, st, d, p0, (const int32_t*)w.wpiv,
                       (const double2*)(w.gsm + GSM_R1), w.gq, d.lda);
    if (!zgemm<double2>(st, OP_C, false, OP_N, false, nsteps, nsteps, rows, C_ONE, w.gq, d.lda, w.gq, d.lda, C_ZERO,
                        w.gsm + GSM_G2, GRAM_NB_MAX, w.gsplit, w.gsplit_bytes))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cqr_chol, dim3(1), dim3(1024), 0, st, d.ctl, p0, w.gsm);
    hipLaunchKernelGGL((k_cqr_trsm<T, false>), dim3(rb), dim3(GRAM_ROWS_NT), 0, st, d, p0, (const int32_t*)nullptr,
                       (const double2*)(w.gsm + GSM_R2), w.gq, d.lda);
    hipLaunchKernelGGL((k_recon<T>), dim3(1), dim3(1024), 0, st, d, p0, (const double2*)w.gq, d.lda, w.gsm, w.Tbuf,
                       (int)UNGQR_NB);
    hipLaunchKernelGGL((k_recon_rows<T>), dim3(rb), dim3(GRAM_ROWS_NT), 0, st, d, p0, (const int32_t*)w.wpiv,
                       (const double2*)w.gq, d.lda, (const double2*)w.gsm, w.vbuf);
    const double wr = (double)rows * W;
    prof_end(eg, st, PK_STEP_C, (double)sizeof(T) * (wr + 2.0 * rows * nsteps) + 16.0 * 6.0 * rows * nsteps,
             8.0 * wr * W + 16.0 * (double)rows * nsteps * nsteps);
    return hipGetLastError();
}

// One candidate-window panel at p0 (see window.hpp).  On return *jend is the
// first column of the next panel and *nparts the argmax partials for its
// first step (0 when there are none: the next panel then starts from nu).
template <typename T>
static hipError_t window_panel(UpdateWs<T>& w, hipStream_t st, QrcpStats* stats, int64_t p0, int64_t* jend_out,
                               int* nparts, bool allow_gram = true)
{
    QrcpDev<T>& d = w.d;
    const int64_t m = d.m, n = d.n, k = d.k;
    const int W = w.win;
    const int64_t cend = p0 + W;
    int64_t nout = n - cend;
    const int64_t nsteps = (p0 + w.nb < k ? p0 + w.nb : k) - p0;
    // right-looking steps keep the window current (one launch per step) while
    // the rows fit one 1024-thread block; otherwise delayed-update steps
    const bool right = m - p0 <= WSTEP_NT * WSTEP_RPT;
    // pivots from the window's Gram matrix (gram.hpp) instead of per-step launches
    const bool gram = allow_gram && g_panel_mode == 1 && right && W <= GRAM_W_MAX && nsteps <= GRAM_NB_MAX;

    hipEvent_t ew = prof_begin(st);
    window_setup<T>(w, st, p0, true);
    prof_end(ew, st, PK_WINDOW, (double)sizeof(T) * 4.0 * (double)m * W, 0.0);
    hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)p0);
    if (gram) {
        hipError_t eg = gram_panel_steps<T>(w, st, p0, (int)nsteps, W);
        if (eg != hipSuccess) return eg;
    } else if (right) {
        run_window_steps<T>(w, st, p0, nsteps, W);
    } else {
        run_panel_steps<T>(d, st, p0, nsteps, cend, true, 1);
    }
    int32_t hctl[CTL_COUNT];
    hipError_t e = hipSuccess;
    // The right-looking steps always take all nsteps steps (a 256-column
    // window cannot run out of live columns in 32 steps, and they never set
    // the stop flag), so the host goes on without reading the control block
    // here; the replay's read-back below checks the step count.
    const bool assume_full = right && !gram;
    int64_t jend = p0 + nsteps;
    hctl[CTL_STOP] = 0;
    if (!assume_full) {
        e = read_ctl<T>(d, st, hctl);
        if (e != hipSuccess) return e;
        jend = hctl[CTL_JDONE];
    }
    if (gram && jend == p0) {   // no pivot passed the Cholesky: the per-step path takes the panel
        window_restore<T>(w, st, p0, W);
        return window_panel<T>(w, st, stats, p0, jend_out, nparts, false);
    }
    if (jend <= p0 || jend > p0 + nsteps) {   // no progress: corrupt state
        qr_diag("window panel p0=%lld: %lld steps done of %lld (right-looking %d, m=%lld n=%lld k=%lld)",
                (long long)p0, (long long)(jend - p0), (long long)nsteps, (int)right, (long long)m, (long long)n,
                (long long)k);
        return hipErrorUnknown;
    }
    int nbe = (int)(jend - p0);
    bool refresh = hctl[CTL_STOP] != 0;
    if (right) window_reorder<T>(w, st, p0, nbe, W);
    // the columns the block update and the replay cover: those outside the
    // window, and with Gram pivots also the window's non-pivot columns
    const int64_t c_o = gram ? jend : cend;
    nout = n - c_o;

    // block reflector of the panel and the R rows of the outside columns
    const T* V = d.A + p0 + d.lda * p0;
    const int64_t rows = m - p0;
    T* Ao = d.A + p0 + d.lda * c_o;
    const double ro = (double)rows * (double)nout;
    hipEvent_t eg = prof_begin(st);
    // G = V^H V: the right-looking steps have formed its upper triangle (the
    // part the T recurrence reads); the delayed-update steps need the GEMM
    if (!right && !zgemm<T>(st, OP_C, true, OP_N, true, nbe, nbe, rows, C_ONE, V, d.lda, V, d.lda, C_ZERO, w.Gbuf,
                            UNGQR_NB, w.gsplit, w.gsplit_bytes))
        return hipErrorInvalidValue;
    if (!gram) hipLaunchKernelGGL((k_larft<T>), dim3(1), dim3(256), 0, st, w.Gbuf, d.tau + p0, nbe, w.Tbuf);
    prof_end(eg, st, PK_REFL, right ? 0.0 : (double)sizeof(T) * rows * nbe,
             right ? 0.0 : 8.0 * (double)nbe * nbe * rows);
    hipEvent_t et = prof_begin(st);
    // nbe <= 32: the split-K partials stay unreduced for k_panel_rows
    const bool fused = nbe <= 32;
    int nzw = 1;
    if (!zgemm<T>(st, OP_C, true, OP_N, false, nbe, nout, rows, C_ONE, V, d.lda, Ao, d.lda, C_ZERO, w.Wbuf,
                  UNGQR_NB, w.gsplit, w.gsplit_bytes, fused ? &nzw : nullptr))
        return hipErrorInvalidValue;
    prof_end(et, st, PK_PANEL, (double)sizeof(T) * ro, 8.0 * nbe * ro);
    // W2 = T^H W and R12 = A_o[p0:p0+nbe] - V_top W2
    hipEvent_t e2 = prof_begin(st);
    if (fused) {
        const bool split = nzw > 1;
        const T* P = split ? (const T*)w.gsplit : (const T*)w.Wbuf;
        const int64_t ldp = split ? nbe : UNGQR_NB, zs = (int64_t)nbe * nout;
        int64_t blocks = (nout + 7) / 8;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL((k_panel_rows<T>), dim3((unsigned)blocks), dim3(256), 0, st, P, ldp, zs, nzw,
                           (const T*)w.Tbuf, V, d.lda, (const T*)Ao, nout, nbe, w.W2buf, w.Wbuf);
    } else {
        if (!zgemm<T>(st, OP_C, false, OP_N, false, nbe, nout, nbe, C_ONE, w.Tbuf, UNGQR_NB, w.Wbuf, UNGQR_NB,
                      C_ZERO, w.W2buf, UNGQR_NB, nullptr, 0))
            return hipErrorInvalidValue;
        dim3 grid(1, (unsigned)nout);
        hipLaunchKernelGGL((k_copy_cols<T>), grid, dim3(256), 0, st, (const T*)Ao, d.lda, w.Wbuf, (int64_t)UNGQR_NB,
                           (int64_t)nbe);
        if (!zgemm<T>(st, OP_N, true, OP_N, false, nbe, nout, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, C_ONE,
                      w.Wbuf, UNGQR_NB, nullptr, 0))
            return hipErrorInvalidValue;
    }
    prof_end(e2, st, PK_REFL, (double)sizeof(T) * ((double)nzw + 3.0) * nbe * nout, 16.0 * (double)nbe * nbe * nout);

    // greedy replay of every step against the outside columns
    hipEvent_t ek = prof_begin(st);
    const unsigned nchk = (unsigned)rup(nout, 256);
    hipLaunchKernelGGL((k_window_check<T>), dim3(nchk), dim3(256), 0, st, d, (const T*)w.Wbuf, (int64_t)UNGQR_NB,
                       c_o, nout, nbe);
    prof_end(ek, st, PK_WINDOW, 8.0 * (double)nbe * nout, 0.0);
    // Right-looking panels enqueue the outside columns' update and norm
    // commit before the host reads the replay's outcome: they take it from the
    // control block (k_replay_commit), and a replay miss later redoes only the
    // window, whose first t* reflectors come out bit-identical.
    const bool spec = assume_full;
    if (spec) {
        hipLaunchKernelGGL((k_replay_commit<T>), dim3(nchk), dim3(256), 0, st, d, p0, nbe, w.W2buf,
                           (const T*)w.Wbuf, (int64_t)UNGQR_NB, c_o, nout);
        hipEvent_t eu = prof_begin(st);
        if (!zrank_update<T>(st, true, rows, nout, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, Ao, d.lda) &&
            !zgemm<T>(st, OP_N, true, OP_N, false, rows, nout, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, C_ONE, Ao,
                      d.lda, nullptr, 0))
            return hipErrorInvalidValue;
        prof_end(eu, st, PK_TRAIL, 2.0 * sizeof(T) * ro, 8.0 * ro * nbe);
    }
    e = read_ctl<T>(d, st, hctl);
    if (e != hipSuccess) return e;
    if (assume_full && hctl[CTL_JDONE] != jend) {
        qr_diag("window panel p0=%lld: the right-looking steps ended at %d of %lld (m=%lld n=%lld k=%lld)",
                (long long)p0, (int)(hctl[CTL_JDONE] - p0), (long long)nsteps, (long long)m, (long long)n,
                (long long)k);
        return hipErrorUnknown;
    }
    if (assume_full && hctl[CTL_STOP]) refresh = true;
    int tstar = nbe;
    if (hctl[CTL_TFAIL] < tstar) tstar = hctl[CTL_TFAIL];
    if (hctl[CTL_TFLAG] < tstar) tstar = hctl[CTL_TFLAG];
    if (tstar < 1) {   // the window always holds the first pivot
        qr_diag("window panel p0=%lld: replay accepts no step (nbe=%d, first fail %d, first flag %d; m=%lld n=%lld "
                "k=%lld)", (long long)p0, nbe, (int)hctl[CTL_TFAIL], (int)hctl[CTL_TFLAG], (long long)m,
                (long long)n, (long long)k);
        return hipErrorUnknown;
    }
    if (tstar < nbe && gram) {
        // a column outside the Gram pivots would have been chosen at step
        // tstar: the per-step path takes the panel from its saved state
        window_restore<T>(w, st, p0, W);
        if (stats) stats->window_misses++;
        return window_panel<T>(w, st, stats, p0, jend_out, nparts, false);
    }
    if (hctl[CTL_TFLAG] <= tstar) refresh = true;
    if (tstar < nbe) {
        // an outside column would have been chosen at step tstar (or the panel
        // would have ended there): redo exactly tstar steps from the saved state
        hipEvent_t er = prof_begin(st);
        dim3 grid((unsigned)(rup(m, 256) < 64 ? rup(m, 256) : 64), (unsigned)W);
        hipLaunchKernelGGL((k_copy_cols<T>), grid, dim3(256), 0, st, (const T*)w.wsave, d.lda, d.A + d.lda * p0,
                           d.lda, m);
        hipLaunchKernelGGL((k_window_meta<T>), dim3((unsigned)rup(W, 256)), dim3(256), 0, st, d, p0, W, w.wsnu,
                           w.wsnuref, w.wsperm, 1);
        window_setup<T>(w, st, p0, false);   // same window, no swaps left: restores the first partial
        prof_end(er, st, PK_WINDOW, (double)sizeof(T) * 2.0 * (double)m * W, 0.0);
        hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)p0);
        if (right) run_window_steps<T>(w, st, p0, tstar, W);
        else run_panel_steps<T>(d, st, p0, tstar, cend, true, 1);
        e = read_ctl<T>(d, st, hctl);
        if (e != hipSuccess) return e;
        if (hctl[CTL_JDONE] != p0 + tstar) {
            qr_diag("window panel p0=%lld: redo of %d steps ended at %d (m=%lld n=%lld k=%lld)", (long long)p0,
                    tstar, (int)(hctl[CTL_JDONE] - p0), (long long)m, (long long)n, (long long)k);
            return hipErrorUnknown;
        }
        if (right) window_reorder<T>(w, st, p0, tstar, W);
        nbe = tstar;
        jend = p0 + tstar;
        if (stats) stats->window_misses++;
    }

    if (spec) {   // the update and the commit are already on the stream
        if (stats) stats->panels++;
        if (refresh && jend < k) {
            const unsigned nblk = (unsigned)rup(n - jend, QR_CW);
            hipEvent_t en = prof_begin(st);
            hipLaunchKernelGGL((k_colnorms<T>), dim3(nblk), dim3(256), 0, st, d, jend, jend, 1, 0);
            prof_end(en, st, PK_NORMS, (double)sizeof(T) * (double)(m - jend) * (double)(n - jend), 0.0);
            *nparts = (int)nblk;
            if (stats) stats->refreshes++;
        } else {
            *nparts = 0;
        }
        *jend_out = jend;
        return hipSuccess;
    }

    // updates: the window's remaining columns from F (right-looking steps have
    // kept them current already), the outside columns from W2
    hipEvent_t eu = prof_begin(st);
    if (!right && m > jend && cend > jend) {
        if (!zgemm<T>(st, OP_N, false, OP_C, false, m - jend, cend - jend, nbe, C_MONE, d.A + jend + d.lda * p0,
                      d.lda, d.F + jend, d.ldf, C_ONE, d.A + jend + d.lda * jend, d.lda, nullptr, 0))
            return hipErrorInvalidValue;
    }
    if (!zrank_update<T>(st, true, rows, nout, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, Ao, d.lda) &&
        !zgemm<T>(st, OP_N, true, OP_N, false, rows, nout, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, C_ONE, Ao,
                  d.lda, nullptr, 0))
        return hipErrorInvalidValue;
    const double mn = (right ? 0.0 : (double)(m - jend) * (double)(cend - jend)) + ro;
    prof_end(eu, st, PK_TRAIL, 2.0 * sizeof(T) * mn, 8.0 * mn * nbe);
    if (stats) stats->panels++;
    if (refresh && jend < k) {
        const unsigned nblk = (unsigned)rup(n - jend, QR_CW);
        hipEvent_t en = prof_begin(st);
        hipLaunchKernelGGL((k_colnorms<T>), dim3(nblk), dim3(256), 0, st, d, jend, jend, 1, 0);
        prof_end(en, st, PK_NORMS, (double)sizeof(T) * (double)(m - jend) * (double)(n - jend), 0.0);
        *nparts = (int)nblk;
        if (stats) stats->refreshes++;
    } else {
        hipLaunchKernelGGL((k_window_commit<T>), dim3(nchk), dim3(256), 0, st, d, (const T*)w.Wbuf,
                           (int64_t)UNGQR_NB, c_o, nout, nbe);
        *nparts = 0;
    }
    *jend_out = jend;
    return hipSuccess;
}

// nparts: argmax partials left by the kernel that set up the norms (ignored
// without pivoting).
template <typename T>
static hipError_t run_qrcp(UpdateWs<T>& w, hipStream_t st, QrcpStats* stats, int nparts)
{
    QrcpDev<T>& d = w.d;
    g_qr_diag[0] = 0;
    if (!d.pivoting) {
        // the a10 trailing norm is only needed when the factorisation truncates
        const bool trunc = d.m > d.k && d.n > d.k;
        if (!trunc && d.n <= WSTEP_NT && d.m <= (int64_t)WSTEP_NT * WSTEP_RPT && d.n <= QR_WIN_MAX)
            return run_window_fixed<T>(w, st, stats);
        return run_blocked_fixed<T>(w, st, stats);
    }
    const int64_t m = d.m, n = d.n, k = d.k;
    const int nb = w.nb;
    int64_t j = 0;
    while (j < k) {
        const int64_t p0 = j;
        const int64_t pend = (p0 + nb < k) ? p0 + nb : k;
        if (w.win > 0 && n - p0 > w.win && n - p0 <= WIN_SORT_MAX) {
            int64_t jend = p0;
            hipError_t e = window_panel<T>(w, st, stats, p0, &jend, &nparts);
            if (e != hipSuccess) return e;
            j = jend;
            continue;
        }
        if (w.win > 0 && n - p0 <= WSTEP_NT && n - p0 <= QR_WIN_MAX && m - p0 <= (int64_t)WSTEP_NT * WSTEP_RPT) {
            // every remaining column fits one window: right-looking steps over
            // all of them keep every norm exact, so there is nothing outside to
            // replay against and every later panel fits as well
            for (int64_t q0 = p0; q0 < k; q0 += nb) {
                const int64_t nsteps = (q0 + nb < k ? q0 + nb : k) - q0;
                const int W = (int)(n - q0);
                hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)q0);
                hipLaunchKernelGGL((k_nu_partials<T>), dim3(1), dim3(1024), 0, st, d, w.wcp, q0, W);
                run_window_steps<T>(w, st, q0, nsteps, W);
                window_reorder<T>(w, st, q0, (int)nsteps, W);
                if (stats) stats->panels++;
            }
            int32_t hctl[CTL_COUNT];
            hipError_t e = read_ctl<T>(d, st, hctl);
            if (e != hipSuccess) return e;
            if (hctl[CTL_JDONE] != k) {
                qr_diag("all-column window panels from p0=%lld ended at step %d of %lld (m=%lld n=%lld)",
                        (long long)p0, (int)hctl[CTL_JDONE], (long long)k, (long long)m, (long long)n);
                return hipErrorUnknown;
            }
            j = k;
            break;
        }
        if (nparts == 0) {
            // the previous panel left no partials: take them from the norms
            const unsigned nb2 = (unsigned)rup(n - p0, 256);
            hipLaunchKernelGGL((k_nu_argmax<T>), dim3(nb2), dim3(256), 0, st, d, p0);
            nparts = (int)nb2;
        }
        hipLaunchKernelGGL(k_ctl_panel, dim3(1), dim3(64), 0, st, d.ctl, (int32_t)p0);
        nparts = run_panel_steps<T>(d, st, p0, pend - p0, n, false, nparts);
        int32_t hctl[CTL_COUNT];
        hipError_t e = read_ctl<T>(d, st, hctl);
        if (e != hipSuccess) return e;
        const int64_t jend = hctl[CTL_JDONE];
        if (jend <= p0 || jend > pend) {   // no progress: corrupt state
            qr_diag("panel p0=%lld: %lld steps done of %lld (m=%lld n=%lld k=%lld)", (long long)p0,
                    (long long)(jend - p0), (long long)(pend - p0), (long long)m, (long long)n, (long long)k);
            return hipErrorUnknown;
        }
        const int64_t nbe = jend - p0;
        // trailing update A[jend:, jend:] -= V[jend:, p0:jend] F[jend:, 0:nbe]^H
        if (m > jend && n > jend) {
            hipEvent_t et = prof_begin(st);
            if (!zgemm<T>(st, OP_N, false, OP_C, false, m - jend, n - jend, nbe, C_MONE,
                          d.A + jend + d.lda * p0, d.lda, d.F + jend, d.ldf, C_ONE,
                          d.A + jend + d.lda * jend, d.lda, nullptr, 0))
                return hipErrorInvalidValue;
            const double mn = (double)(m - jend) * (double)(n - jend);
            prof_end(et, st, PK_TRAIL, 2.0 * sizeof(T) * mn, 8.0 * mn * nbe);
        }
        if (stats) stats->panels++;
        if (hctl[CTL_STOP] && jend < k) {
            const unsigned nblk = (unsigned)rup(n - jend, QR_CW);
            hipEvent_t en = prof_begin(st);
            hipLaunchKernelGGL((k_colnorms<T>), dim3(nblk), dim3(256), 0, st, d, jend, jend, 1, 0);
            nparts = (int)nblk;
            prof_end(en, st, PK_NORMS, (double)sizeof(T) * (double)(m - jend) * (double)(n - jend), 0.0);
            if (stats) stats->refreshes++;
        }
        j = jend;
    }
    // a10: ||R22||_F^2 over the final trailing block
    if (m > k && n > k) {
        const unsigned nblk = (unsigned)rup(n - k, QR_CW);
        hipEvent_t en = prof_begin(st);
        hipLaunchKernelGGL((k_colnorms<T>), dim3(nblk), dim3(256), 0, st, d, k, k, 0, 0);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double*)d.npart, (int)nblk, d.dsc,
                           (int)DSC_EPS2);
        prof_end(en, st, PK_NORMS, (double)sizeof(T) * (double)(m - k) * (double)(n - k), 0.0);
    }
    return hipGetLastError();
}

// a11: Q (m x k, ldq) = H_0 ... H_{k-1} [I_k; 0] from the reflectors stored in
// d.A below the diagonal, by blocks of UNGQR_NB from the last block backwards.
template <typename T>
static hipError_t form_q(UpdateWs<T>& w, T* Q, int64_t ldq, hipStream_t st)
{
    QrcpDev<T>& d = w.d;
    const int64_t m = d.m, k = d.k;
    if (k <= 0) return hipSuccess;
    {
        dim3 grid((unsigned)(rup(m, 256) < 64 ? rup(m, 256) : 64), (unsigned)k);
        hipLaunchKernelGGL((k_eye<T>), grid, dim3(256), 0, st, Q, ldq, m, k);
    }
    const int64_t last = ((k - 1) / UNGQR_NB) * UNGQR_NB;
    hipEvent_t eq = prof_begin(st);
    double flops = 0.0, bytes = 0.0;
    // every block's G = V^H V, then all T factors in one launch: none of them
    // depends on Q, so they stay off the chain of dependent Q updates
    for (int64_t b0 = 0; b0 <= last; b0 += UNGQR_NB) {
        const int nbe = (int)((k - b0) < UNGQR_NB ? (k - b0) : UNGQR_NB);
        const T* V = d.A + b0 + d.lda * b0;
        if (!zgemm<T>(st, OP_C, true, OP_N, true, nbe, nbe, m - b0, C_ONE, V, d.lda, V, d.lda, C_ZERO,
                      w.Gall + (b0 / UNGQR_NB) * UNGQR_NB * UNGQR_NB, UNGQR_NB, w.gsplit, w.gsplit_bytes))
            return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_larft_all<T>), dim3((unsigned)(last / UNGQR_NB + 1)), dim3(256), 0, st, (const T*)w.Gall,
                       (const double2*)d.tau, k, w.Tall);
    for (int64_t b0 = last; b0 >= 0; b0 -= UNGQR_NB) {
        const int nbe = (int)((k - b0) < UNGQR_NB ? (k - b0) : UNGQR_NB);
        const T* V = d.A + b0 + d.lda * b0;
        const int64_t rows = m - b0, cols = k - b0;
        const T* Tb = w.Tall + (b0 / UNGQR_NB) * UNGQR_NB * UNGQR_NB;
        // W = V^H Q[b0:, b0:k]
        if (!zgemm<T>(st, OP_C, true, OP_N, false, nbe, cols, rows, C_ONE, V, d.lda, Q + b0 + ldq * b0, ldq,
                      C_ZERO, w.Wbuf, UNGQR_NB, w.gsplit, w.gsplit_bytes))
            return hipErrorInvalidValue;
        // W2 = T W
        if (!zgemm<T>(st, OP_N, false, OP_N, false, nbe, cols, nbe, C_ONE, Tb, UNGQR_NB, w.Wbuf, UNGQR_NB, C_ZERO,
                      w.W2buf, UNGQR_NB, nullptr, 0))
            return hipErrorInvalidValue;
        // Q[b0:, b0:k] -= V W2
        if (!zrank_update<T>(st, true, rows, cols, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, Q + b0 + ldq * b0, ldq) &&
            !zgemm<T>(st, OP_N, true, OP_N, false, rows, cols, nbe, C_MONE, V, d.lda, w.W2buf, UNGQR_NB, C_ONE,
                      Q + b0 + ldq * b0, ldq, nullptr, 0))
            return hipErrorInvalidValue;
        flops += 8.0 * nbe * ((double)rows * nbe + 2.0 * (double)rows * cols + (double)nbe * cols);
        bytes += (double)sizeof(T) * (3.0 * (double)rows * cols + 2.0 * (double)rows * nbe);
    }
    prof_end(eq, st, PK_UNGQR, bytes, flops);
    return hipGetLastError();
}

// Norms, perm and first-pivot partials of a matrix already in d.A (no gate);
// returns the number of argmax partials left for the first step.
template <typename T>
static int init_norms(UpdateWs<T>& w, hipStream_t st)
{
    QrcpDev<T>& d = w.d;
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, d.ctl, d.dsc);
    if (d.n <= 0) return 0;
    const unsigned nblk = (unsigned)rup(d.n, QR_CW);
    hipLaunchKernelGGL((k_colnorms<T>), dim3(nblk), dim3(256), 0, st, d, (int64_t)0, (int64_t)0, 1, 1);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double*)d.npart, (int)nblk, d.dsc,
                       (int)DSC_NORM2);
    return (int)nblk;
}
