// The two-site update (included by abi.hip after the error helpers):
// contraction + gate (a1-a3), factorisation by plain pivoted QR (a4-a10) or by
// a learned pivot order with certificate / verification and fallback
// (a15-a18), Q formation (a11) and split (a12); plus the entry points of the
// learned proposal's pieces.
#include "learn.hpp"

static bool gate_finite(const double* g)
{
    for (int q = 0; q < 32; ++q)
        if (!isfinite(g[q])) return false;
    return true;
}

static Gate4 make_gate(const double* g)
{
    Gate4 G;
    for (int q = 0; q < 16; ++q) G.g[q] = make_double2(g[2 * q], g[2 * q + 1]);
    return G;
}

#define PN_ELL_MAX 256

// Workspace of the learned path (carved after the main factorisation's).
template <typename T>
struct LearnWs {
    UpdateWs<T> w2;   // factorisation of the column-gathered copy of theta
    T* Om;
    T* Y;
    double* s;
    double* stats;
    float* phi;
    float* scores;
    int32_t* order;
    double* cert;
};

template <typename T>
static bool carve_learn_ws(Carver& cv, LearnWs<T>& L, int64_t m, int64_t n, int64_t k, int64_t ell)
{
    if (!carve_update_ws<T>(cv, L.w2, m, n, k, true)) return false;
    L.Om = (T*)cv.take((int64_t)sizeof(T) * ell * m);
    L.Y = (T*)cv.take((int64_t)sizeof(T) * ell * n);
    L.s = (double*)cv.take(8 * (n + 1));
    L.stats = (double*)cv.take(64);
    L.phi = (float*)cv.take(4 * PN_F * (n + 1));
    L.scores = (float*)cv.take(4 * (n + 1));
    L.order = (int32_t*)cv.take(4 * (n + 1));
    L.cert = (double*)cv.take(64);
    return L.Om && L.Y && L.s && L.stats && L.phi && L.scores && L.order && L.cert;
}

template <typename T>
static int64_t learn_ws_bytes(int64_t m, int64_t n, int64_t k, int64_t ell)
{
    Carver cv{nullptr, (int64_t)1 << 62, 0};
    LearnWs<T> L;
    carve_learn_ws<T>(cv, L, m, n, k, ell);
    return cv.used + 256;
}

// a15 + a16: sketch, features, scores and the proposed column order of the
// matrix in d.A.
template <typename T>
static hipError_t propose_order(const QrcpDev<T>& d, LearnWs<T>& L, const mps_learned_cfg* lc, void* gsplit,
                                int64_t gsb, hipStream_t st)
{
    const int64_t m = d.m, n = d.n, ell = lc->sketch_rows;
    const int64_t blocks = rup(ell * m, 256) < 4096 ? rup(ell * m, 256) : 4096;
    hipLaunchKernelGGL((k_sketch_omega<T>), dim3((unsigned)blocks), dim3(256), 0, st, L.Om, ell, m, lc->seed);
    if (!zgemm<T>(st, OP_N, false, OP_N, false, ell, n, m, C_ONE, L.Om, ell, d.A, d.lda, C_ZERO, L.Y, ell, gsplit,
                  gsb))
        return hipErrorInvalidValue;
    const unsigned nb = (unsigned)rup(n, 256);
    hipLaunchKernelGGL((k_sketch_norms<T>), dim3(nb), dim3(256), 0, st, (const T*)L.Y, ell, n, L.s);
    hipLaunchKernelGGL(k_sketch_stats, dim3(1), dim3(256), 0, st, (const double*)L.s, n, L.stats);
    hipLaunchKernelGGL((k_sketch_features<T>), dim3(nb), dim3(256), 0, st, (const T*)L.Y, ell, n,
                       (const double*)L.s, (const double*)L.stats, L.phi);
    hipLaunchKernelGGL(k_pn_forward, dim3(nb), dim3(256), 0, st, lc->params, (const float*)L.phi, n, L.scores);
    hipLaunchKernelGGL(k_rank_desc, dim3(nb), dim3(256), 0, st, (const float*)L.scores, n, L.order);
    return hipGetLastError();
}

__global__ void k_copy_norm2(const double* src, double* dst)
{
    if (threadIdx.x == 0) dst[DSC_NORM2] = src[DSC_NORM2];
}

// Result of the factorisation step: the workspace whose factors are kept
// (the plain or the learned one), the QR statistics and the acceptance data.
template <typename T>
struct FactorOut {
    UpdateWs<T>* use = nullptr;
    QrcpStats stats;
    int fallback = 0;
    double eps_s2 = -1.0, eps_q2 = -1.0;
};

// ||A||^2 of the matrix in d after its norm kernels: one readback, taken
// before the learned proposal so that a non-finite input is refused before
// anything depends on its ranking.
template <typename T>
static hipError_t read_norm2(const QrcpDev<T>& d, hipStream_t st, double* out)
{
    hipError_t e = hipMemcpyAsync(out, d.dsc + DSC_NORM2, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    prof_flush();
    return e;
}

// a4-a10 (plain pivoted QR) or a15-a18 (learned proposal, QR with the proposed
// order fixed, acceptance, fallback) on the matrix in w.d.A, whose column
// norms, argmax partials (nparts of them) and ||A||^2 are in place.  L and lc
// are null for plain pivoted QR.
template <typename T>
static mps_status factorise(UpdateWs<T>& w, LearnWs<T>* L, const mps_learned_cfg* lc, int nparts, hipStream_t st,
                            FactorOut<T>& out)
{
    QrcpDev<T>& d = w.d;
    const int64_t m = d.m, n = d.n, k = d.k;
    out.use = &w;
    if (!lc) {
        HIPCHK(run_qrcp<T>(w, st, &out.stats, nparts), "pivoted QR");
        return MPS_OK;
    }
    double n2 = 0.0;
    HIPCHK(read_norm2<T>(d, st, &n2), "norm readback");
    if (!isfinite(n2)) return fail(MPS_ENUMERIC, "learned pivots: non-finite input");
    // a15-a17: proposal, then QR with the proposed order fixed
    hipEvent_t ep = prof_begin(st);
    HIPCHK(propose_order<T>(d, *L, lc, w.gsplit, w.gsplit_bytes, st), "learned proposal");
    QrcpDev<T>& d2 = L->w2.d;
    dim3 ggrid((unsigned)(rup(m, 256) < 64 ? rup(m, 256) : 64), (unsigned)n);
    hipLaunchKernelGGL((k_gather_cols<T>), ggrid, dim3(256), 0, st, (const T*)d.A, d.lda, d2.A, d2.lda, m,
                       (const int32_t*)L->order, d2.perm, n);
    prof_end(ep, st, PK_PROPOSE, (double)sizeof(T) * 3.0 * (double)m * (double)n,
             8.0 * (double)lc->sketch_rows * (double)m * (double)n);
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, d2.ctl, d2.dsc);
    hipLaunchKernelGGL(k_copy_norm2, dim3(1), dim3(64), 0, st, (const double*)d.dsc, d2.dsc);
    L->w2.nb = w.nb;
    L->w2.win = w.win;
    d2.tol = 0.0;
    d2.pivoting = 0;
    QrcpStats s2;
    HIPCHK(run_qrcp<T>(L->w2, st, &s2, 0), "known-order QR");
    // a18: certificate = (largest squared residual norm of an unselected
    // column, smallest |R_jj| of a selected one)
    int nblk = 0;
    if (m > k && n > k) {
        nblk = (int)rup(n - k, QR_CW);
        hipLaunchKernelGGL((k_colnorms<T>), dim3((unsigned)nblk), dim3(256), 0, st, d2, k, k, 1, 0);
    }
    hipLaunchKernelGGL(k_certificate, dim3(1), dim3(256), 0, st, (const ArgBest*)d2.cpart, nblk,
                       (const double*)d2.diagR, k, L->cert);
    double cert[2], dsc2[DSC_COUNT];
    HIPCHK(hipMemcpyAsync(cert, L->cert, sizeof(cert), hipMemcpyDeviceToHost, st), "certificate readback");
    HIPCHK(hipMemcpyAsync(dsc2, d2.dsc, sizeof(dsc2), hipMemcpyDeviceToHost, st), "certificate readback");
    HIPCHK(hipStreamSynchronize(st), "certificate sync");
    prof_flush();
    out.eps_s2 = dsc2[DSC_EPS2];
    bool accept;
    if (lc->verify == 2) {
        accept = true;   // trusted: kept without a check (measures the proposal's own cost)
    } else if (lc->verify) {
        HIPCHK(run_qrcp<T>(w, st, &out.stats, nparts), "verification QRCP");
        double dq[DSC_COUNT];
        HIPCHK(hipMemcpyAsync(dq, d.dsc, sizeof(dq), hipMemcpyDeviceToHost, st), "verification readback");
        HIPCHK(hipStreamSynchronize(st), "verification sync");
        prof_flush();
        out.eps_q2 = dq[DSC_EPS2];
        const double r2 = lc->fallback_ratio * lc->fallback_ratio;
        accept = out.eps_s2 <= r2 * out.eps_q2 + 1e-300;
    } else {
        accept = cert[0] <= cert[1] * cert[1] * (1.0 + 1e-12);
    }
    if (accept) {
        out.use = &L->w2;
        out.stats = s2;
    } else {
        out.fallback = 1;
        if (lc->verify == 0) HIPCHK(run_qrcp<T>(w, st, &out.stats, nparts), "fallback QRCP");
    }
    return MPS_OK;
}

template <typename T>
static void fill_info(mps_update_info* info, int64_t k, const double* dsc, const FactorOut<T>& f, bool learned)
{
    if (!info) return;
    info->k = k;
    info->trunc_err_sq = dsc[DSC_EPS2];
    info->norm_sq = dsc[DSC_NORM2];
    info->retained = dsc[DSC_NORM2] > 0 ? 1.0 - dsc[DSC_EPS2] / dsc[DSC_NORM2] : 1.0;
    info->fallback = f.fallback;
    info->panels = f.stats.panels;
    info->refreshes = f.stats.refreshes;
    info->window_misses = f.stats.window_misses;
    info->learned_err_sq = f.eps_s2;
    // plain pivoted QR's error: measured by the verification, or the kept
    // result itself when plain pivoted QR produced it
    info->qrcp_err_sq = !learned || f.fallback ? dsc[DSC_EPS2] : f.eps_q2;
}

// theta is formed in the workspace before any output is written, so the
// outputs may alias the input sites.
template <typename T>
static mps_status update_core(int64_t chi_l, int64_t chi_m, int64_t chi_r, int64_t chi_cap, mps_precision prec,
                              const T* A, const T* B, const double* g, T* A_out, T* B_out, int renorm,
                              const mps_learned_cfg* lc, mps_update_info* info, void* work, int64_t work_bytes,
                              hipStream_t st)
{
    const int64_t m = 2 * chi_l, n = 2 * chi_r;
    int64_t k = chi_cap < m ? chi_cap : m;
    k = k < n ? k : n;
    Carver cv{(char*)work, work_bytes, 0};
    UpdateWs<T> w;
    if (!carve_update_ws<T>(cv, w, m, n, k, true)) return fail(MPS_ENOMEM, "update: workspace too small");
    LearnWs<T> L;
    if (lc && !carve_learn_ws<T>(cv, L, m, n, k, lc->sketch_rows))
        return fail(MPS_ENOMEM, "update: workspace too small for the learned path");
    w.nb = panel_width(m, n);
    w.win = qr_window(w.nb, n);
    w.d.tol = recompute_tol(prec);
    w.d.pivoting = 1;
    QrcpDev<T>& d = w.d;

    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, d.ctl, d.dsc);
    // a1: theta0 = A_mat (m x chi_m) * B_mat (chi_m x n)
    hipEvent_t e1 = prof_begin(st);
    if (!zgemm<T>(st, OP_N, false, OP_N, false, m, n, chi_m, C_ONE, A, m, B, chi_m, C_ZERO, d.A, d.lda, w.gsplit,
                  w.gsplit_bytes))
        return fail(MPS_EINVAL, "update: gemm form unavailable");
    prof_end(e1, st, PK_CONTRACT, (double)sizeof(T) * ((double)m * chi_m + (double)chi_m * n + (double)m * n),
             8.0 * (double)m * (double)n * (double)chi_m);
    // a2 + a3
    hipEvent_t e2 = prof_begin(st);
    hipLaunchKernelGGL((k_gate_norms<T>), dim3((unsigned)chi_r), dim3(256), 0, st, d, chi_l, make_gate(g));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double*)d.npart, (int)chi_r, d.dsc,
                       (int)DSC_NORM2);
    prof_end(e2, st, PK_GATE, 2.0 * sizeof(T) * (double)m * (double)n, 64.0 * (double)m * (double)n / 4.0);
    HIPCHK(hipGetLastError(), "update launch");

    FactorOut<T> f;
    mps_status s = factorise<T>(w, lc ? &L : nullptr, lc, (int)chi_r, st, f);
    if (s != MPS_OK) return s;
    QrcpDev<T>& du = f.use->d;
    HIPCHK(form_q<T>(*f.use, A_out, m, st), "update Q");
    hipEvent_t e3 = prof_begin(st);
    hipLaunchKernelGGL((k_rpt<T>), dim3((unsigned)n), dim3(256), 0, st, (const T*)du.A, du.lda,
                       (const int32_t*)du.perm, k, n, B_out, k, (const double*)du.dsc, renorm);
    prof_end(e3, st, PK_SPLIT, 2.0 * sizeof(T) * (double)k * (double)n, 0.0);
    double dsc[DSC_COUNT];
    HIPCHK(hipMemcpyAsync(dsc, du.dsc, sizeof(dsc), hipMemcpyDeviceToHost, st), "update readback");
    HIPCHK(hipStreamSynchronize(st), "update sync");
    prof_flush();
    if (!isfinite(dsc[DSC_NORM2]) || !isfinite(dsc[DSC_EPS2]))
        return fail(MPS_ENUMERIC, "update: non-finite theta");
    fill_info<T>(info, k, dsc, f, lc != nullptr);
    return MPS_OK;
}

static bool learned_cfg_valid(const mps_learned_cfg* lc)
{
    return lc && lc->params && lc->sketch_rows >= 1 && lc->sketch_rows <= PN_ELL_MAX &&
           (lc->verify >= 0 && lc->verify <= 2) && lc->fallback_ratio >= 1.0 && isfinite(lc->fallback_ratio);
}

extern "C" int64_t mps_update_work_bytes(int64_t chi_l, int64_t chi_m, int64_t chi_r, int64_t chi_cap,
                                         mps_precision prec, mps_pivot pivot)
{
    (void)chi_m;
    if (chi_l < 1 || chi_r < 1 || chi_cap < 1 || !valid_prec(prec)) return -1;
    if (pivot != MPS_PIVOT_QRCP && pivot != MPS_PIVOT_LEARNED) return -1;
    const int64_t m = 2 * chi_l, n = 2 * chi_r;
    int64_t k = chi_cap < m ? chi_cap : m;
    k = k < n ? k : n;
    int64_t b = prec == MPS_FP64 ? update_ws_bytes<double2>(m, n, k) : update_ws_bytes<float2>(m, n, k);
    if (pivot == MPS_PIVOT_LEARNED)
        b += prec == MPS_FP64 ? learn_ws_bytes<double2>(m, n, k, PN_ELL_MAX)
                              : learn_ws_bytes<float2>(m, n, k, PN_ELL_MAX);
    return b;
}

extern "C" mps_status mps_update_bond(int64_t chi_l, int64_t chi_m, int64_t chi_r, int64_t chi_cap,
                                      mps_precision prec, mps_pivot pivot, const void* A, const void* B,
                                      const double* g, void* A_out, void* B_out, int renormalize,
                                      const mps_learned_cfg* learned, mps_update_info* info, void* work,
                                      int64_t work_bytes, void* hip_stream)
{
    if (chi_l < 1 || chi_m < 1 || chi_r < 1 || chi_cap < 1)
        return fail(MPS_EINVAL, "mps_update_bond: dimensions must be >= 1");
    if (chi_l > (1 << 19) || chi_r > (1 << 19) || chi_m > (1 << 20))
        return fail(MPS_EINVAL, "mps_update_bond: dimension too large");
    if (!valid_prec(prec)) return fail(MPS_EINVAL, "mps_update_bond: bad precision %d", (int)prec);
    if (pivot != MPS_PIVOT_QRCP && pivot != MPS_PIVOT_LEARNED)
        return fail(MPS_EINVAL, "mps_update_bond: bad pivot mode %d", (int)pivot);
    if (pivot == MPS_PIVOT_LEARNED && !learned_cfg_valid(learned))
        return fail(MPS_EINVAL, "mps_update_bond: learned pivots need a valid mps_learned_cfg");
    if (!A || !B || !g || !A_out || !B_out || !work) return fail(MPS_EINVAL, "mps_update_bond: null pointer");
    if (!gate_finite(g)) return fail(MPS_ENUMERIC, "mps_update_bond: non-finite gate entry");
    const int64_t need = mps_update_work_bytes(chi_l, chi_m, chi_r, chi_cap, prec, pivot);
    if (work_bytes < need)
        return fail(MPS_ENOMEM, "mps_update_bond: need %lld work bytes, got %lld", (long long)need,
                    (long long)work_bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    const mps_learned_cfg* lc = pivot == MPS_PIVOT_LEARNED ? learned : nullptr;
    if (prec == MPS_FP64)
        return update_core<double2>(chi_l, chi_m, chi_r, chi_cap, prec, (const double2*)A, (const double2*)B, g,
                                    (double2*)A_out, (double2*)B_out, renormalize, lc, info, work, work_bytes, st);
    return update_core<float2>(chi_l, chi_m, chi_r, chi_cap, prec, (const float2*)A, (const float2*)B, g,
                               (float2*)A_out, (float2*)B_out, renormalize, lc, info, work, work_bytes, st);
}

template <typename T>
static mps_status theta_impl(int64_t chi_l, int64_t chi_m, int64_t chi_r, const T* A, const T* B, const double* g,
                             T* theta, int64_t ld, void* work, int64_t work_bytes, hipStream_t st)
{
    const int64_t m = 2 * chi_l, n = 2 * chi_r;
    Carver cv{(char*)work, work_bytes, 0};
    UpdateWs<T> w;
    if (!carve_update_ws<T>(cv, w, m, n, 1, false)) return fail(MPS_ENOMEM, "mps_theta: workspace too small");
    w.d.A = theta;
    w.d.lda = ld;
    if (!zgemm<T>(st, OP_N, false, OP_N, false, m, n, chi_m, C_ONE, A, m, B, chi_m, C_ZERO, theta, ld, w.gsplit,
                  w.gsplit_bytes))
        return fail(MPS_EINVAL, "mps_theta: gemm form unavailable");
    hipLaunchKernelGGL((k_gate_norms<T>), dim3((unsigned)chi_r), dim3(256), 0, st, w.d, chi_l, make_gate(g));
    HIPCHK(hipGetLastError(), "mps_theta launch");
    HIPCHK(hipStreamSynchronize(st), "mps_theta sync");
    return MPS_OK;
}

extern "C" mps_status mps_theta(int64_t chi_l, int64_t chi_m, int64_t chi_r, mps_precision prec, const void* A,
                                const void* B, const double* g, void* theta, int64_t ld, void* work,
                                int64_t work_bytes, void* hip_stream)
{
    if (chi_l < 1 || chi_m < 1 || chi_r < 1) return fail(MPS_EINVAL, "mps_theta: dimensions must be >= 1");
    if (!valid_prec(prec)) return fail(MPS_EINVAL, "mps_theta: bad precision");
    if (!A || !B || !g || !theta || !work) return fail(MPS_EINVAL, "mps_theta: null pointer");
    if (ld < 2 * chi_l) return fail(MPS_EINVAL, "mps_theta: leading dimension too small");
    if (!gate_finite(g)) return fail(MPS_ENUMERIC, "mps_theta: non-finite gate entry");
    if (work_bytes < mps_update_work_bytes(chi_l, chi_m, chi_r, 1, prec, MPS_PIVOT_QRCP))
        return fail(MPS_ENOMEM, "mps_theta: workspace too small");
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == MPS_FP64)
        return theta_impl<double2>(chi_l, chi_m, chi_r, (const double2*)A, (const double2*)B, g, (double2*)theta, ld,
                                   work, work_bytes, st);
    return theta_impl<float2>(chi_l, chi_m, chi_r, (const float2*)A, (const float2*)B, g, (float2*)theta, ld, work,
                              work_bytes, st);
}

// ---------------------------------------------------------------------------
// pivot-proposal network entry points
// ---------------------------------------------------------------------------
extern "C" int64_t pivnet_work_bytes(int64_t m, int64_t n, int32_t sketch_rows, mps_precision prec)
{
    if (m < 1 || n < 1 || sketch_rows < 1 || sketch_rows > PN_ELL_MAX || !valid_prec(prec)) return -1;
    const int64_t eb = elem_bytes(prec);
    const int64_t gsplit = 16 * eb * (int64_t)sketch_rows * n;   // split-K partials of the sketch GEMM
    const int64_t gpart = 4 * (PN_P + 1) * (rup(n, 256) + 1);
    return eb * (int64_t)sketch_rows * (m + n) + 8 * (n + 16) + gsplit + gpart + 8 * 256;
}

template <typename T>
static mps_status features_impl(int64_t m, int64_t n, const T* theta, int64_t ld, int32_t ell, uint64_t seed,
                                float* phi, void* work, int64_t work_bytes, hipStream_t st)
{
    Carver cv{(char*)work, work_bytes, 0};
    T* Om = (T*)cv.take((int64_t)sizeof(T) * ell * m);
    T* Y = (T*)cv.take((int64_t)sizeof(T) * ell * n);
    double* s = (double*)cv.take(8 * (n + 1));
    double* stats = (double*)cv.take(64);
    const int64_t gsb = 16 * (int64_t)sizeof(T) * ell * n;
    void* gsplit = cv.take(gsb);
    if (!Om || !Y || !s || !stats || !gsplit) return fail(MPS_ENOMEM, "pivnet_features: workspace too small");
    const int64_t blocks = rup((int64_t)ell * m, 256) < 4096 ? rup((int64_t)ell * m, 256) : 4096;
    hipLaunchKernelGGL((k_sketch_omega<T>), dim3((unsigned)blocks), dim3(256), 0, st, Om, (int64_t)ell, m, seed);
    if (!zgemm<T>(st, OP_N, false, OP_N, false, ell, n, m, C_ONE, Om, ell, theta, ld, C_ZERO, Y, ell, gsplit, gsb))
        return fail(MPS_EINVAL, "pivnet_features: gemm form unavailable");
    const unsigned nb = (unsigned)rup(n, 256);
    hipLaunchKernelGGL((k_sketch_norms<T>), dim3(nb), dim3(256), 0, st, (const T*)Y, (int64_t)ell, n, s);
    hipLaunchKernelGGL(k_sketch_stats, dim3(1), dim3(256), 0, st, (const double*)s, n, stats);
    hipLaunchKernelGGL((k_sketch_features<T>), dim3(nb), dim3(256), 0, st, (const T*)Y, (int64_t)ell, n,
                       (const double*)s, (const double*)stats, phi);
    HIPCHK(hipGetLastError(), "pivnet_features launch");
    return MPS_OK;
}

extern "C" mps_status pivnet_features(int64_t m, int64_t n, mps_precision prec, const void* theta, int64_t ld,
                                      int32_t sketch_rows, uint64_t seed, float* phi, void* work,
                                      int64_t work_bytes, void* hip_stream)
{
    if (m < 1 || n < 1 || !valid_prec(prec) || sketch_rows < 1 || sketch_rows > PN_ELL_MAX)
        return fail(MPS_EINVAL, "pivnet_features: bad sizes");
    if (!theta || !phi || !work) return fail(MPS_EINVAL, "pivnet_features: null pointer");
    if (ld < m) return fail(MPS_EINVAL, "pivnet_features: leading dimension too small");
    if (work_bytes < pivnet_work_bytes(m, n, sketch_rows, prec))
        return fail(MPS_ENOMEM, "pivnet_features: workspace too small");
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == MPS_FP64)
        return features_impl<double2>(m, n, (const double2*)theta, ld, sketch_rows, seed, phi, work, work_bytes, st);
    return features_impl<float2>(m, n, (const float2*)theta, ld, sketch_rows, seed, phi, work, work_bytes, st);
}

extern "C" mps_status pivnet_forward(const float* params, const float* phi, int64_t n, float* scores,
                                     void* hip_stream)
{
    if (!params || !phi || !scores || n < 1) return fail(MPS_EINVAL, "pivnet_forward: bad arguments");
    hipLaunchKernelGGL(k_pn_forward, dim3((unsigned)rup(n, 256)), dim3(256), 0, (hipStream_t)hip_stream, params,
                       phi, n, scores);
    HIPCHK(hipGetLastError(), "pivnet_forward launch");
    return MPS_OK;
}

extern "C" mps_status pivnet_grad(const float* params, const float* phi, const uint8_t* labels, int64_t n,
                                  float* grad, void* work, int64_t work_bytes, void* hip_stream)
{
    if (!params || !phi || !labels || !grad || !work || n < 1) return fail(MPS_EINVAL, "pivnet_grad: bad arguments");
    const int64_t nb = rup(n, 256);
    if (work_bytes < 4 * (PN_P + 1) * nb) return fail(MPS_ENOMEM, "pivnet_grad: workspace too small");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_pn_grad, dim3((unsigned)nb), dim3(256), 0, st, params, phi, labels, n, (float*)work);
    hipLaunchKernelGGL(k_pn_grad_sum, dim3(1), dim3(128), 0, st, (const float*)work, (int)nb, grad);
    HIPCHK(hipGetLastError(), "pivnet_grad launch");
    return MPS_OK;
}

extern "C" mps_status pivnet_adam(float* params, const float* grad, float* m1, float* m2, int32_t t, float lr,
                                  void* hip_stream)
{
    if (!params || !grad || !m1 || !m2 || t < 1 || !(lr > 0.f)) return fail(MPS_EINVAL, "pivnet_adam: bad arguments");
    hipLaunchKernelGGL(k_pn_adam, dim3(1), dim3(128), 0, (hipStream_t)hip_stream, params, grad, m1, m2, (int)t, lr);
    HIPCHK(hipGetLastError(), "pivnet_adam launch");
    return MPS_OK;
}

extern "C" mps_status pivnet_rank(const float* scores, int64_t n, int32_t* order, void* hip_stream)
{
    if (!scores || !order || n < 1) return fail(MPS_EINVAL, "pivnet_rank: bad arguments");
    hipLaunchKernelGGL(k_rank_desc, dim3((unsigned)rup(n, 256)), dim3(256), 0, (hipStream_t)hip_stream, scores, n,
                       order);
    HIPCHK(hipGetLastError(), "pivnet_rank launch");
    return MPS_OK;
}
