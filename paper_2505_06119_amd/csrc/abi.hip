// C-ABI of libmpsgpu.so (declared in include/mps_abi.h): argument checking on
// the host, workspace carving, and the host-side sequencing of the gfx950
// kernels for the two-site update, pivoted QR and the stateful MPS.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/mps_abi.h"
#include "chain.hpp"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static mps_status fail(mps_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static mps_status fail(mps_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

static mps_status hip_fail(hipError_t e, const char* where)
{
    if (e == hipErrorUnknown && g_qr_diag[0]) return fail(MPS_EDEVICE, "%s: %s", where, g_qr_diag);
    return fail(MPS_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

extern "C" const char* mps_last_error(void) { return g_err.c_str(); }

#define HIPCHK(expr, where)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(_e, where);     \
    } while (0)

static inline int64_t elem_bytes(mps_precision p) { return p == MPS_FP64 ? 16 : 8; }
static inline bool valid_prec(int p) { return p == MPS_FP64 || p == MPS_MIXED; }

// Tuning of the pivoted QR (mps_set_tuning): panel width (0: automatic) and
// candidate-window width (-1: automatic, 0: off).
static int g_panel_width = 0;
static int g_qr_window = -1;
#define QR_WIN_DEFAULT 256

// Tiles chosen by mps_autotune per bucket of column counts (sorted by n_max;
// empty: the built-in defaults).  Explicit values of mps_set_tuning win.
static std::vector<mps_tune_entry> g_tune;

static const mps_tune_entry* tuned_for(int64_t n)
{
    for (const mps_tune_entry& e : g_tune)
        if (n <= e.n_max) return &e;
    return nullptr;
}

// Panel width of the delayed-update QRCP: wider panels raise the arithmetic
// intensity of the rank-nb trailing update but lengthen every pivot step's
// F-correction.
static int panel_width(int64_t m, int64_t n)
{
    (void)m;
    if (g_panel_width > 0) return n <= 64 && g_panel_width > 16 ? 16 : g_panel_width;
    if (n <= 64) return 16;
    if (const mps_tune_entry* e = tuned_for(n)) return e->panel_width;
    return 32;
}

// Candidate-window width for a pivoted factorisation of n columns with panel
// width nb (0: no window panels).
static int qr_window(int nb, int64_t n)
{
    int w = g_qr_window;
    if (w < 0) {
        const mps_tune_entry* e = g_panel_width > 0 ? nullptr : tuned_for(n);
        w = e ? e->qr_window : QR_WIN_DEFAULT;
    }
    return w >= nb && w <= QR_WIN_MAX ? w : 0;
}

extern "C" mps_status mps_set_panel_mode(int32_t mode)
{
    if (mode != 0 && mode != 1) return fail(MPS_EINVAL, "mps_set_panel_mode: mode %d not 0 or 1", (int)mode);
    g_panel_mode = mode;
    return MPS_OK;
}

extern "C" mps_status mps_set_tuning(int32_t panel_width_, int32_t qr_window_)
{
    if (panel_width_ != 0 && panel_width_ != 16 && panel_width_ != 32 && panel_width_ != 64)
        return fail(MPS_EINVAL, "mps_set_tuning: panel width %d not in {0, 16, 32, 64}", (int)panel_width_);
    if (qr_window_ < -1 || qr_window_ > QR_WIN_MAX || (qr_window_ > 0 && qr_window_ < 64))
        return fail(MPS_EINVAL, "mps_set_tuning: window %d not -1, 0 or in [64, %d]", (int)qr_window_, QR_WIN_MAX);
    g_panel_width = panel_width_;
    g_qr_window = qr_window_;
    return MPS_OK;
}

static double recompute_tol(mps_precision p)
{
    // squared-norm ratio below which a downdated residual norm is recomputed:
    // sqrt of the storage precision's unit roundoff
    return p == MPS_FP64 ? 1.4901161193847656e-08 : 3.4526698300124393e-04;
}

template <typename T>
static int64_t update_ws_bytes(int64_t m, int64_t n, int64_t k)
{
    Carver cv{nullptr, (int64_t)1 << 62, 0};
    UpdateWs<T> w;
    carve_update_ws<T>(cv, w, m, n, k, true);
    return cv.used + 256;
}

// two-site update, learned proposal entry points
#include "bond.hpp"

// truncated-SVD updates beyond the small-bond chains
#include "svd.hpp"

// ---------------------------------------------------------------------------
// qrcp_truncate
// ---------------------------------------------------------------------------
extern "C" int64_t qrcp_work_bytes(int64_t m, int64_t n, int64_t k_max, mps_precision prec, mps_pivot mode)
{
    if (m < 0 || n < 0 || k_max < 0 || !valid_prec(prec)) return -1;
    if (mode != MPS_PIVOT_QRCP && mode != MPS_PIVOT_LEARNED) return -1;
    int64_t k = k_max < m ? k_max : m;
    k = k < n ? k : n;
    int64_t b = prec == MPS_FP64 ? update_ws_bytes<double2>(m, n, k) : update_ws_bytes<float2>(m, n, k);
    if (mode == MPS_PIVOT_LEARNED)
        b += prec == MPS_FP64 ? learn_ws_bytes<double2>(m, n, k, PN_ELL_MAX) : learn_ws_bytes<float2>(m, n, k, PN_ELL_MAX);
    return b;
}

template <typename T>
static mps_status qrcp_impl(int64_t m, int64_t n, int64_t k, mps_precision prec, const mps_learned_cfg* lc,
                            const void* A, int64_t lda, void* Q, int64_t ldq, void* RPt, int64_t ldr, int32_t* piv,
                            double* diagR, int64_t* k_out, double* err_fro, double* a_fro, mps_update_info* info,
                            void* work, int64_t work_bytes, hipStream_t st)
{
    Carver cv{(char*)work, work_bytes, 0};
    UpdateWs<T> w;
    if (!carve_update_ws<T>(cv, w, m, n, k, true))
        return fail(MPS_ENOMEM, "qrcp_truncate: work_bytes %lld too small", (long long)work_bytes);
    LearnWs<T> L;
    if (lc && !carve_learn_ws<T>(cv, L, m, n, k, lc->sketch_rows))
        return fail(MPS_ENOMEM, "qrcp_truncate: work_bytes %lld too small for learned pivots", (long long)work_bytes);
    w.nb = panel_width(m, n);
    w.win = qr_window(w.nb, n);
    w.d.tol = recompute_tol(prec);
    w.d.pivoting = 1;
    {
        dim3 grid((unsigned)(rup(m, 256) < 64 ? rup(m, 256) : 64), (unsigned)n);
        hipLaunchKernelGGL((k_copy_cols<T>), grid, dim3(256), 0, st, (const T*)A, lda, w.d.A, w.d.lda, m);
    }
    const int nparts = init_norms<T>(w, st);
    HIPCHK(hipGetLastError(), "qrcp_truncate launch");
    FactorOut<T> f;
    mps_status s = factorise<T>(w, lc ? &L : nullptr, lc, nparts, st, f);
    if (s != MPS_OK) return s;
    QrcpDev<T>& du = f.use->d;
    HIPCHK(form_q<T>(*f.use, (T*)Q, ldq, st), "qrcp_truncate Q");
    hipLaunchKernelGGL((k_rpt<T>), dim3((unsigned)n), dim3(256), 0, st, (const T*)du.A, du.lda,
                       (const int32_t*)du.perm, k, n, (T*)RPt, ldr, (const double*)du.dsc, 0);
    HIPCHK(hipMemcpyAsync(diagR, du.diagR, sizeof(double) * k, hipMemcpyDeviceToDevice, st), "diagR");
    HIPCHK(hipMemcpyAsync(piv, du.perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st), "piv");
    double dsc[DSC_COUNT];
    HIPCHK(hipMemcpyAsync(dsc, du.dsc, sizeof(dsc), hipMemcpyDeviceToHost, st), "qrcp_truncate readback");
    HIPCHK(hipStreamSynchronize(st), "qrcp_truncate sync");
    prof_flush();
    if (!isfinite(dsc[DSC_NORM2]) || !isfinite(dsc[DSC_EPS2])) return fail(MPS_ENUMERIC, "qrcp_truncate: non-finite input");
    if (k_out) *k_out = k;
    if (err_fro) *err_fro = sqrt(dsc[DSC_EPS2] > 0 ? dsc[DSC_EPS2] : 0.0);
    if (a_fro) *a_fro = sqrt(dsc[DSC_NORM2]);
    fill_info<T>(info, k, dsc, f, lc != nullptr);
    return MPS_OK;
}

// Host-side checks shared by qrcp_truncate and qrcp_truncate_noalloc.
static mps_status qrcp_check(const char* who, int64_t m, int64_t n, int64_t k_max, mps_precision prec,
                             mps_pivot mode, const mps_learned_cfg* learned, const void* A, int64_t lda,
                             const void* Q, int64_t ldq, const void* RPt, int64_t ldr, const int32_t* piv,
                             const double* diagR)
{
    if (m < 1 || n < 1 || k_max < 1) return fail(MPS_EINVAL, "%s: m, n, k_max must be >= 1", who);
    if (!valid_prec(prec)) return fail(MPS_EINVAL, "%s: bad precision %d", who, (int)prec);
    if (mode != MPS_PIVOT_QRCP && mode != MPS_PIVOT_LEARNED)
        return fail(MPS_EINVAL, "%s: bad pivot mode %d", who, (int)mode);
    if (mode == MPS_PIVOT_LEARNED && !learned_cfg_valid(learned))
        return fail(MPS_EINVAL, "%s: learned pivots need a valid mps_learned_cfg", who);
    if (m > (1 << 20) || n > (1 << 20)) return fail(MPS_EINVAL, "%s: dimension too large", who);
    int64_t k = k_max < m ? k_max : m;
    k = k < n ? k : n;
    if (!A || !Q || !RPt || !piv || !diagR) return fail(MPS_EINVAL, "%s: null device pointer", who);
    if (lda < m || ldq < m || ldr < k) return fail(MPS_EINVAL, "%s: leading dimension too small", who);
    return MPS_OK;
}

static mps_status qrcp_run(int64_t m, int64_t n, int64_t k_max, mps_precision prec, mps_pivot mode,
                           const mps_learned_cfg* learned, const void* A, int64_t lda, void* Q, int64_t ldq,
                           void* RPt, int64_t ldr, int32_t* piv, double* diagR, int64_t* k_out, double* err_fro,
                           double* a_fro, mps_update_info* info, void* work, int64_t work_bytes, hipStream_t st)
{
    int64_t k = k_max < m ? k_max : m;
    k = k < n ? k : n;
    const mps_learned_cfg* lc = mode == MPS_PIVOT_LEARNED ? learned : nullptr;
    if (prec == MPS_FP64)
        return qrcp_impl<double2>(m, n, k, prec, lc, A, lda, Q, ldq, RPt, ldr, piv, diagR, k_out, err_fro, a_fro,
                                  info, work, work_bytes, st);
    return qrcp_impl<float2>(m, n, k, prec, lc, A, lda, Q, ldq, RPt, ldr, piv, diagR, k_out, err_fro, a_fro, info,
                             work, work_bytes, st);
}

extern "C" mps_status qrcp_truncate(int64_t m, int64_t n, int64_t k_max, mps_precision prec, mps_pivot mode,
                                    const mps_learned_cfg* learned, const void* A, int64_t lda, void* Q, int64_t ldq,
                                    void* RPt, int64_t ldr, int32_t* piv, double* diagR, int64_t* k_out,
                                    double* err_fro, double* a_fro, mps_update_info* info, void* work,
                                    int64_t work_bytes, void* hip_stream)
{
    mps_status s = qrcp_check("qrcp_truncate", m, n, k_max, prec, mode, learned, A, lda, Q, ldq, RPt, ldr, piv,
                              diagR);
    if (s != MPS_OK) return s;
    if (!work) return fail(MPS_EINVAL, "qrcp_truncate: null device pointer");
    const int64_t need = qrcp_work_bytes(m, n, k_max, prec, mode);
    if (work_bytes < need)
        return fail(MPS_ENOMEM, "qrcp_truncate: need %lld work bytes, got %lld", (long long)need,
                    (long long)work_bytes);
    return qrcp_run(m, n, k_max, prec, mode, learned, A, lda, Q, ldq, RPt, ldr, piv, diagR, k_out, err_fro, a_fro,
                    info, work, work_bytes, (hipStream_t)hip_stream);
}

// ---------------------------------------------------------------------------
// qrcp_truncate_noalloc: qrcp_truncate with its scratch in a static device
// array instead of a workspace argument, for callers that cannot allocate.
// `scratch` is a host-side stand-in in host code: its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is passed on.  Each GPU holds its own copy until the
// process ends.  Nothing in it needs to start at zero: the factorisation
// writes every scratch word before reading it (the same holds for the
// uninitialised workspace qrcp_truncate accepts).
// ---------------------------------------------------------------------------
#define NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
#define NOALLOC_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static mps_status noalloc_scratch(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "qrcp_truncate_noalloc: hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(MPS_EINVAL, "qrcp_truncate_noalloc: device %d beyond the %d supported", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "qrcp_truncate_noalloc: hipGetSymbolAddress");
        if (!p) return fail(MPS_EDEVICE, "qrcp_truncate_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MPS_OK;
}

// Marks the calling thread as one that must not allocate for the scope.
struct NoAllocScope {
    bool prev;
    NoAllocScope() : prev(g_no_alloc) { g_no_alloc = true; }
    ~NoAllocScope() { g_no_alloc = prev; }
};

extern "C" int64_t qrcp_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" mps_status qrcp_truncate_noalloc(int64_t m, int64_t n, int64_t k_max, mps_precision prec,
                                            mps_pivot mode, const mps_learned_cfg* learned, const void* A,
                                            int64_t lda, void* Q, int64_t ldq, void* RPt, int64_t ldr, int32_t* piv,
                                            double* diagR, int64_t* k_out, double* err_fro, double* a_fro,
                                            mps_update_info* info, void* hip_stream)
{
    mps_status s = qrcp_check("qrcp_truncate_noalloc", m, n, k_max, prec, mode, learned, A, lda, Q, ldq, RPt, ldr,
                              piv, diagR);
    if (s != MPS_OK) return s;
    const int64_t need = qrcp_work_bytes(m, n, k_max, prec, mode);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(MPS_ENOMEM, "qrcp_truncate_noalloc: needs %lld bytes of scratch, the static array holds %lld",
                    (long long)need, (long long)NOALLOC_SCRATCH_BYTES);
    void* work = nullptr;
    s = noalloc_scratch(&work);
    if (s != MPS_OK) return s;
    NoAllocScope guard;
    return qrcp_run(m, n, k_max, prec, mode, learned, A, lda, Q, ldq, RPt, ldr, piv, diagR, k_out, err_fro, a_fro,
                    info, work, NOALLOC_SCRATCH_BYTES, (hipStream_t)hip_stream);
}

// stateful MPS context
#include "context.hpp"

// MPO application by zip-up, state loading
#include "mpo.hpp"

// autotuner of the pivoted-QR tiles
#include "autotune.hpp"

// ---------------------------------------------------------------------------
// per-kernel timing
// ---------------------------------------------------------------------------
extern "C" mps_status mps_profile(int mode)
{
    if (mode < 0) return fail(MPS_EINVAL, "mps_profile: mode %d < 0", mode);
    g_prof.on = mode != 0;
    g_prof.stride = mode > 1 ? mode : 1;
    g_prof.counter = 0;
    g_prof.runs = 0;
    for (auto& r : g_prof.pending) {
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.pending.clear();
    for (int c = 0; c < PK_COUNT; ++c) g_prof.acc[c] = ProfAcc{0, 0.0, 0.0, 0.0};
    return MPS_OK;
}

extern "C" mps_status mps_profile_read(mps_kernel_stats* out, int32_t n)
{
    if (!out || n < 1) return fail(MPS_EINVAL, "mps_profile_read: bad arguments");
    for (int c = 0; c < n && c < PK_COUNT; ++c) {
        out[c].launches = g_prof.acc[c].launches;
        out[c].total_ms = g_prof.acc[c].total_ms;
        out[c].alg_bytes = g_prof.acc[c].alg_bytes;
        out[c].alg_flops = g_prof.acc[c].alg_flops;
    }
    return MPS_OK;
}
