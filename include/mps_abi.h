/*
 * mps_abi.h -- C interface of libmpsgpu.so: the two-site gate update of
 * matrix-product-state circuit emulation with truncation by column-pivoted
 * Householder QR, on one AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2505.06119 (Adamski & Brown, "Tensor-Parallel Emulation of
 * Quantum Circuits with Block-Cyclic Distributed Matrix Product States").
 *   - MPS form of a state: Sec. II-B, Eq. (2).
 *   - tensor application of a gate on neighbouring sites: Sec. III-C.2 (the
 *     sites are contracted, the gate applied, and the result decomposed back
 *     by a truncating decomposition).
 *   - QR with pivoting, M = Q R P^T: Table III (Sec. III-B.2).
 *   - canonicalisation by QR / LQ: Sec. III-C.1.
 *   - norm fidelity <Psi_T|Psi_T>: Sec. III-E.
 *
 * Conventions shared by every call
 *   complex numbers   interleaved (re, im); complex64 storage for MPS_MIXED,
 *                     complex128 for MPS_FP64.  Scalars reported to the host
 *                     are always double.
 *   matrices          column-major with an explicit leading dimension.
 *   site tensors      A[l, s, r] (left bond l, physical s in {0,1}, right bond
 *                     r) stored at offset l + chi_l*(s + 2*r).
 *   gates             host array of 32 doubles: a 4x4 complex matrix, row-major,
 *                     row index 2a'+b', column index 2a+b, a = qubit on the
 *                     lower site.  Site 0 is the most significant bit.
 *   device pointers   "device" buffers are HIP device memory owned by the
 *                     caller; the library never allocates device memory.  All
 *                     work runs on the caller's HIP stream (hipStream_t passed
 *                     as void*; NULL = the null stream).  Host outputs are
 *                     written after the stream has been synchronised.
 *   errors            every call returns an mps_status; on failure
 *                     mps_last_error() gives a thread-local message.  Argument
 *                     errors (MPS_EINVAL) are detected on the host before any
 *                     device work and leave every output untouched.  After
 *                     MPS_ENUMERIC (a non-finite value in theta or A) the
 *                     device outputs of a stateless call are unspecified, and a
 *                     context is marked unusable (later calls: MPS_ESTATE).
 *   threads           the stateless calls (qrcp_truncate, mps_update_bond,
 *                     mps_theta, pivnet_*) may run concurrently from several
 *                     host threads, each on its own stream and workspace.  A
 *                     context serves one thread at a time.  mps_set_tuning,
 *                     mps_set_small_bond_limit and mps_profile change
 *                     process-wide settings and must not overlap other calls.
 */
#ifndef MPS_ABI_H
#define MPS_ABI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPS_OK = 0,
    MPS_EINVAL = 1,   /* bad argument: nothing was done */
    MPS_ENOMEM = 2,   /* workspace / arena too small: nothing was done */
    MPS_EDEVICE = 3,  /* a HIP call failed */
    MPS_ENUMERIC = 4, /* non-finite input or result */
    MPS_ESTATE = 5    /* context unusable after an earlier device failure or a
                         non-finite update result */
} mps_status;

typedef enum { MPS_FP64 = 0, MPS_MIXED = 1 } mps_precision;
typedef enum { MPS_PIVOT_QRCP = 0, MPS_PIVOT_LEARNED = 1 } mps_pivot;

/* Result of one truncating update (host struct). */
typedef struct {
    int64_t k;            /* new bond dimension = min(chi_cap, 2 chi_l, 2 chi_r) */
    double trunc_err_sq;  /* ||R22||_F^2, the discarded weight (Sec. III-E)       */
    double norm_sq;       /* ||theta||_F^2 before truncation                       */
    double retained;      /* 1 - trunc_err_sq / norm_sq: this update's factor of
                             the norm fidelity                                      */
    int32_t fallback;     /* learned pivots rejected, plain QRCP used (0/1)          */
    int32_t panels;       /* QR panels processed                                     */
    int32_t refreshes;    /* exact recomputations of the residual column norms       */
    int32_t window_misses;/* candidate-window panels the greedy replay cut short     */
    double learned_err_sq;/* learned pivots: ||R22||^2 of the proposed order (-1: n/a) */
    double qrcp_err_sq;   /* ||R22||^2 of plain pivoted QR when it ran (-1: n/a)      */
} mps_update_info;

/* Learned pivot proposal (an addition of this library, not in the paper): a Gaussian
 * sketch Y = Omega theta (sketch_rows x n, Omega from a SplitMix64 counter
 * generator seeded with `seed`), per-column sketch features, and a small
 * network (MPS_PIVNET_PARAMS float32 parameters: 4 features -> 16 tanh units
 * -> 1 score) rank the columns; the pivoted QR then runs with that column order
 * fixed.  Acceptance:
 *   verify = 0  certificate: every unselected column's residual norm is at most
 *               the smallest |R_jj| of the selected ones (what plain pivoted QR
 *               guarantees by construction);
 *   verify = 1  plain pivoted QR also runs and the proposal is kept only if
 *               its truncation error is at most fallback_ratio times QRCP's;
 *   verify = 2  trusted: the proposal is kept without a check (its error is
 *               still reported), to measure what the proposal path costs.
 * A rejected proposal falls back to plain pivoted QR of the same theta. */
#define MPS_PIVNET_PARAMS 97
#define MPS_PIVNET_FEATURES 4
typedef struct {
    const float* params;   /* device, MPS_PIVNET_PARAMS floats */
    int32_t sketch_rows;   /* 1..256 */
    int32_t verify;        /* 0, 1 or 2, see above */
    uint64_t seed;
    double fallback_ratio; /* >= 1, e.g. 1.01 */
} mps_learned_cfg;

const char* mps_last_error(void);

/* ------------------------------------------------------------------------
 * qrcp_truncate -- column-pivoted Householder QR of A (m x n), stopped after
 * k = min(k_max, m, n) steps (Table III, "QR with pivoting", M = Q R P^T,
 * truncated as in Sec. II-B).  Stateless.
 *
 *   mode  MPS_PIVOT_QRCP: greedy pivoting, the largest residual column norm
 *         at every step; exact ties go to the smaller original column index.
 *         MPS_PIVOT_LEARNED: the column order proposed by `learned` (see
 *         mps_learned_cfg above) is factorised without pivot search and kept
 *         if it passes the acceptance rule, else plain pivoted QR runs
 *         (info->fallback = 1).
 *   learned host, required for MPS_PIVOT_LEARNED (copied), else ignored.
 *   A     device, read-only, m x n (lda >= m), precision prec.
 *   Q     device, m x k (ldq >= m): orthonormal columns Q_k.
 *   RPt   device, k x n (ldr >= k): R_k P^T, i.e. column piv[j] of RPt holds
 *         column j of the upper-trapezoidal R_k.  Q RPt is the rank-k
 *         approximation of A.
 *   piv   device, n int32: piv[j] = original column placed at position j
 *         (0-based; all n entries).  For an accepted learned proposal this is
 *         the proposed order, so piv[0..k) is the selected column set S.
 *   diagR device, k doubles: R_jj (real; sign as produced by the reflector
 *         beta = -sign(Re alpha) ||x||).
 *   k_out, err_fro (= ||R22||_F), a_fro (= ||A||_F): host, may be NULL.
 *   info  host, may be NULL: k, ||R22||^2 (trunc_err_sq), ||A||^2 (norm_sq),
 *         fallback and the statistics of mps_update_info.
 *   work  device scratch of at least qrcp_work_bytes(m, n, k_max, prec, mode)
 *         bytes.
 * Errors: MPS_EINVAL (sizes, null pointers, leading dimensions, an invalid
 * learned configuration) and MPS_ENOMEM (work too small) before any device
 * work; MPS_ENUMERIC when A holds a non-finite value (outputs unspecified);
 * MPS_EDEVICE when a HIP call fails.
 * ------------------------------------------------------------------------ */
int64_t qrcp_work_bytes(int64_t m, int64_t n, int64_t k_max, mps_precision prec, mps_pivot mode);
mps_status qrcp_truncate(int64_t m, int64_t n, int64_t k_max, mps_precision prec, mps_pivot mode,
                         const mps_learned_cfg* learned, const void* A, int64_t lda, void* Q, int64_t ldq,
                         void* RPt, int64_t ldr, int32_t* piv, double* diagR, int64_t* k_out, double* err_fro,
                         double* a_fro, mps_update_info* info, void* work, int64_t work_bytes, void* hip_stream);

/* ------------------------------------------------------------------------
 * qrcp_truncate_noalloc -- for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * qrcp_truncate with the same arguments and results, minus work and
 * work_bytes.  Its scratch is a static device array of
 * qrcp_noalloc_scratch_bytes() = 64 MiB that every GPU the library runs on
 * holds until the process ends (its device address is looked up once per
 * device, with that device current); the call uses the array of the current
 * device, so hip_stream must belong to it.  It calls no hipMalloc, hipFree or
 * other allocating routine; the one pinned host word of the control readback
 * is used only if an earlier call of another entry point has created it,
 * else the readback copies and synchronises the stream.
 * Limit: qrcp_work_bytes(m, n, k_max, prec, mode) <= 64 MiB (for example
 * m = n = 1024 in FP64 with plain pivoting, or in complex64 with learned
 * pivots); larger problems return MPS_ENOMEM before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other host threads, or other streams before this call has returned)
 * race and corrupt each other's results.  The array keeps the last call's
 * contents; nothing in it needs to start at zero.
 * ------------------------------------------------------------------------ */
int64_t qrcp_noalloc_scratch_bytes(void);
mps_status qrcp_truncate_noalloc(int64_t m, int64_t n, int64_t k_max, mps_precision prec, mps_pivot mode,
                                 const mps_learned_cfg* learned, const void* A, int64_t lda, void* Q, int64_t ldq,
                                 void* RPt, int64_t ldr, int32_t* piv, double* diagR, int64_t* k_out,
                                 double* err_fro, double* a_fro, mps_update_info* info, void* hip_stream);

/* ------------------------------------------------------------------------
 * mps_update_bond -- one two-site update on explicit site tensors
 * (Sec. III-C.2): theta = G (A B) contracted over the shared bond chi_m,
 * truncated pivoted QR of theta as a (2 chi_l) x (2 chi_r) matrix, split into
 *   A_out = Q_k            (chi_l x 2 x k site, left-orthonormal)
 *   B_out = R_k P^T        (k x 2 x chi_r site)
 * with k = min(chi_cap, 2 chi_l, 2 chi_r).  When renormalize != 0, B_out is
 * scaled by 1/||Q_k R_k P^T||_F so that a state that was normalised stays
 * normalised; info->retained then carries the norm-fidelity factor.
 *
 *   A, B        device, read-only sites (chi_l x 2 x chi_m, chi_m x 2 x chi_r).
 *   g           host, 32 doubles (4x4 complex, see conventions).
 *   A_out       device, room for chi_l*2*k elements.
 *   B_out       device, room for k*2*chi_r elements; must not overlap A_out.
 *               theta is formed in the workspace first, so the outputs may
 *               alias the input sites.
 *   learned     host, required for pivot = MPS_PIVOT_LEARNED, else ignored.
 *   info        host, may be NULL.
 *   work        device scratch of at least mps_update_work_bytes(...) bytes.
 * ------------------------------------------------------------------------ */
int64_t mps_update_work_bytes(int64_t chi_l, int64_t chi_m, int64_t chi_r, int64_t chi_cap,
                              mps_precision prec, mps_pivot pivot);
mps_status mps_update_bond(int64_t chi_l, int64_t chi_m, int64_t chi_r, int64_t chi_cap,
                           mps_precision prec, mps_pivot pivot, const void* A, const void* B,
                           const double* g, void* A_out, void* B_out, int renormalize,
                           const mps_learned_cfg* learned, mps_update_info* info, void* work,
                           int64_t work_bytes, void* hip_stream);

/* ------------------------------------------------------------------------
 * mps_move_centre -- one move of the orthogonality centre on explicit sites
 * (Sec. III-C.1: canonicalisation by QR to the right, LQ to the left), the
 * operation a context performs before a two-site update away from the
 * centre.  Sites A (chi_l x 2 x chi_c) and B (chi_c x 2 x chi_r) share the
 * bond chi_c; layout as for mps_update_bond.
 *   direction +1: A is the centre.  A = Q R (unpivoted Householder QR of the
 *     (2 chi_l) x chi_c matrix, xLARFG convention), k = min(2 chi_l, chi_c);
 *     A_out = Q (chi_l x 2 x k, left-orthonormal), B_out = R B (k x 2 x chi_r).
 *   direction -1: B is the centre.  B = L Q' (LQ of the chi_c x (2 chi_r)
 *     matrix, as the QR of its conjugate transpose), k = min(chi_c, 2 chi_r);
 *     B_out = Q' (k x 2 x chi_r, right-orthonormal), A_out = A L
 *     (chi_l x 2 x k).
 * A, B: device, read-only.  A_out, B_out: device, must not overlap the inputs
 * or each other.  k_out: host, may be NULL.  work: device scratch of at least
 * mps_move_work_bytes(...) bytes.  Errors: MPS_EINVAL / MPS_ENOMEM before
 * any device work, MPS_EDEVICE when a HIP call fails.
 * ------------------------------------------------------------------------ */
int64_t mps_move_work_bytes(int64_t chi_l, int64_t chi_c, int64_t chi_r, mps_precision prec, int32_t direction);
mps_status mps_move_centre(int64_t chi_l, int64_t chi_c, int64_t chi_r, mps_precision prec, int32_t direction,
                           const void* A, const void* B, void* A_out, void* B_out, int64_t* k_out, void* work,
                           int64_t work_bytes, void* hip_stream);

/* theta = G (A B) of the two-site update (steps before the factorisation),
 * written column-major (2 chi_l) x (2 chi_r) into the device buffer theta
 * (ld >= 2 chi_l).  work: at least mps_update_work_bytes(chi_l, chi_m, chi_r,
 * 1, prec, MPS_PIVOT_QRCP) bytes. */
mps_status mps_theta(int64_t chi_l, int64_t chi_m, int64_t chi_r, mps_precision prec, const void* A,
                     const void* B, const double* g, void* theta, int64_t ld, void* work, int64_t work_bytes,
                     void* hip_stream);

/* ------------------------------------------------------------------------
 * Pivot-proposal network: the pieces of the learned path, exposed for
 * training and testing.  All arrays are device memory; phi is n x 4 float32
 * (row c = features of column c), scores n float32, labels n bytes (1 = the
 * column is among plain pivoted QR's first k pivots), grad MPS_PIVNET_PARAMS+1
 * float32 (gradient of the mean logistic loss, then the loss itself).
 * ------------------------------------------------------------------------ */
int64_t pivnet_work_bytes(int64_t m, int64_t n, int32_t sketch_rows, mps_precision prec);
mps_status pivnet_features(int64_t m, int64_t n, mps_precision prec, const void* theta, int64_t ld,
                           int32_t sketch_rows, uint64_t seed, float* phi, void* work, int64_t work_bytes,
                           void* hip_stream);
mps_status pivnet_forward(const float* params, const float* phi, int64_t n, float* scores, void* hip_stream);
mps_status pivnet_grad(const float* params, const float* phi, const uint8_t* labels, int64_t n, float* grad,
                       void* work, int64_t work_bytes, void* hip_stream);
/* Adam step on params with moment buffers m1, m2 (MPS_PIVNET_PARAMS each); t >= 1. */
mps_status pivnet_adam(float* params, const float* grad, float* m1, float* m2, int32_t t, float lr,
                       void* hip_stream);
/* order[r] = column with the r-th largest score (ties: smaller column first). */
mps_status pivnet_rank(const float* scores, int64_t n, int32_t* order, void* hip_stream);

/* ------------------------------------------------------------------------
 * Stateful MPS of n_sites qubits in the product state |0...0> (all bond
 * dimensions 1), stored in a caller-provided device arena.  Bond b (between
 * sites b-1 and b) never exceeds min(2^b, 2^(n-b), chi_max).  The stored state
 * is kept normalised with the orthogonality centre on one site; the norm
 * fidelity (Sec. III-E) is accumulated as log F in FP64.
 * ------------------------------------------------------------------------ */
typedef struct mps_ctx mps_ctx;

typedef struct {
    int32_t n_sites;       /* >= 2 */
    int32_t chi_max;       /* truncation cap chi, >= 1 */
    mps_precision prec;
    mps_pivot pivot;
    double fallback_ratio; /* learned pivots: accept if eps_S <= ratio * eps_QRCP (1.01) */
    int32_t sketch_rows;   /* learned pivots: rows of the Gaussian sketch */
    int32_t pad;
    uint64_t seed;
    /* learned pivots, optional: the proposal network's parameters (device,
     * MPS_PIVNET_PARAMS float32, must stay valid) and the acceptance rule
     * (learned_verify 0: certificate, 1: verification against plain pivoted
     * QR, 2: trusted).  NULL leaves the network unset until mps_set_pivot_network. */
    const float* mlp_weights;
    int32_t learned_verify;
    int32_t pad2;
} mps_config;

/* Device bytes the arena of mps_create must provide for this configuration:
 * one slot per site sized for its largest bond dimensions min(2^b, 2^(n-b),
 * chi_max) (the bond bound of the MPS form, Sec. II-B, Eq. (2)), then the
 * workspace of the largest two-site update (Sec. III-C.2).  -1 for an
 * invalid configuration. */
int64_t mps_arena_bytes(const mps_config* cfg);

/* A new MPS (Sec. II-B, Eq. (2)) in the product state |0...0> with every bond
 * dimension 1 and the orthogonality centre on site 0 (a product state is in
 * canonical form, Sec. III-C.1).  The arena (device, >= mps_arena_bytes)
 * stays owned by the caller and must outlive the context; the stream is used
 * by every later call on it.  Errors: MPS_EINVAL (configuration, null
 * pointers), MPS_ENOMEM (arena too small). */
mps_status mps_create(const mps_config* cfg, void* dev_arena, int64_t arena_bytes, void* hip_stream,
                      mps_ctx** out);
mps_status mps_destroy(mps_ctx* ctx);

/* For a context created with pivot = MPS_PIVOT_LEARNED: the proposal network
 * and acceptance policy used by every later update (cfg is copied; the
 * parameter buffer it points to must stay valid).  Updates fail with
 * MPS_EINVAL until it has been set. */
mps_status mps_set_pivot_network(mps_ctx* ctx, const mps_learned_cfg* cfg);

/* Apply the 4x4 gate g (host, 32 doubles) to sites (i, i+1), 0 <= i < n-1:
 * the orthogonality centre is first moved to site i (or to i+1 when it lies
 * right of i) by unpivoted QR / LQ (Sec. III-C.1), then the two-site update
 * runs and the centre ends on site i+1.  info (host) may be NULL. */
mps_status mps_apply_gate(mps_ctx* ctx, int32_t i, const double* g, mps_update_info* info);

/* Apply one layer of two-site gates (Sec. III-C.2, tensor application; a
 * circuit layer acts on disjoint neighbouring pairs, Sec. III-D) on pairwise
 * disjoint bonds (i[t] + 1 < i[t+1]), in array order, with the semantics of n
 * calls of mps_apply_gate.  g: n x 32 doubles; info: n entries or NULL.
 * Overlapping or unsorted bonds: MPS_EINVAL, no state change. */
mps_status mps_apply_layer(mps_ctx* ctx, int64_t n, const int32_t* i, const double* g,
                           mps_update_info* info);

/* Apply a matrix product operator (Sec. III-C.3, MPO application: long-range
 * operators of small bond m, contracted with the state by the zip-up
 * algorithm) to the sites first .. first + n_sites - 1.  mdims (host, n_sites
 * + 1 int32): the MPO bonds, mdims[0] = mdims[n_sites] = 1 and 1 <= mdims[t]
 * <= 2 (the bond of the inverse QFT's MPOs; it is what the context's bond
 * storage leaves room for during a sweep).  W (host, FP64 complex as (re, im) pairs): the site tensors in order,
 * site t holding 4 mdims[t] mdims[t+1] entries W_t[a, s', s, b] at index
 * a + mdims[t] (s' + 2 (s + 2 b)) (s the input, s' the output physical
 * index; e.g. the controlled-phase MPO of the inverse QFT, Sec. III-D.1, has
 * m = 2).  The centre moves to `first`; a carried matrix is swept from left
 * to right, each site's contraction truncated by pivoted QR to the bond cap
 * (Table III), leaving left-canonical sites and the centre on the last site.
 * The squared norm of the result there is the norm fidelity factor of the
 * application (Sec. III-E; exact for a unitary MPO such as the inverse QFT's):
 * its log goes to *log_retained (host, may be NULL) and into the log norm
 * fidelity, and the state is normalised.  MPS_EINVAL: sites out of range, bad mdims or NULL
 * arrays (no state change); MPS_ENUMERIC: non-finite entry (refused before
 * any change) or non-finite intermediate (the context is then poisoned). */
mps_status mps_apply_mpo(mps_ctx* ctx, int32_t first, int32_t n_sites, const int32_t* mdims, const double* W,
                         double* log_retained);

/* Replace the state: dims (host, n_sites + 1 int64, dims[0] = dims[n] = 1,
 * each within the context's bond cap) and data (host, FP64 complex pairs):
 * the sites in order, site j holding dims[j] x 2 x dims[j+1] entries at
 * l + dims[j] (s + 2 r).  The state is brought to right-canonical form by
 * LQ moves (Sec. III-C.1) with the centre on site 0, normalised, and the
 * norm fidelity restarts at 1 (the random-saturation input of the inverse
 * QFT experiment, Sec. III-D.1, is loaded this way).  MPS_EINVAL: bad dims
 * or NULL arrays; MPS_ENUMERIC: non-finite or zero state. */
mps_status mps_load_state(mps_ctx* ctx, const int64_t* dims, const double* data);

/* <x|Psi_T> for the bit string x (host, n_sites bytes of 0/1; site 0 first),
 * where Psi_T is the stored normalised state times sqrt(norm fidelity), i.e.
 * the paper's unnormalised truncated state.  out: host, 2 doubles. */
mps_status mps_amplitude(mps_ctx* ctx, const uint8_t* bits, double* out);

/* log of the norm fidelity accumulated so far (host double). */
mps_status mps_log_norm_fidelity(const mps_ctx* ctx, double* out);

/* Bond dimensions: dims[b] for b = 0..n_sites (dims[0] = dims[n] = 1). */
mps_status mps_bond_dims(const mps_ctx* ctx, int64_t* dims);

/* Orthogonality centre site index (host int32). */
mps_status mps_centre(const mps_ctx* ctx, int32_t* out);

/* Copy site j (chi_l x 2 x chi_r elements, site layout above, complex64 or
 * complex128 per the context) to the device buffer dst of dst_bytes. */
mps_status mps_get_site(mps_ctx* ctx, int32_t j, void* dst, int64_t dst_bytes);

/* ------------------------------------------------------------------------
 * Tuning of the pivoted QR, process-wide (not thread-safe; affects later
 * calls).  panel_width: 16, 32 or 64 pivot steps per delayed-update panel
 * (0: automatic, 16 for n <= 64 and 32 otherwise).  qr_window: width W of the
 * candidate window of the pivoted panels (-1: automatic, 256; 0: off, every
 * pivot step reads the whole trailing block; otherwise 64 <= W <= 512).  A
 * window panel factorises up to panel_width steps inside the W columns of
 * largest residual norm and accepts them only as far as a greedy replay
 * against all other columns confirms them, so the pivots are those of the
 * full search; a window narrower than the panel width is not used.  Returns
 * MPS_EINVAL for values outside these sets (nothing changes then).
 * ------------------------------------------------------------------------ */
mps_status mps_set_tuning(int32_t panel_width, int32_t qr_window);

/* ------------------------------------------------------------------------
 * How the pivoted window panels take their pivot steps, process-wide (not
 * thread-safe; affects later calls).  mode 0 (default): one launch per pivot
 * step (the right-looking window kernel).  mode 1: the pivots of a panel
 * from pivoted Cholesky of the window's Gram matrix A_w^H A_w (greedy
 * pivoting picks the column of largest residual norm, and those norms and
 * the R rows are fixed by the inner products: Table III's QR with pivoting),
 * then CholeskyQR2 of the chosen columns and a Householder reconstruction
 * with the xLARFG sign convention, so R, the reflectors and tau are those of
 * the Householder QR of the chosen columns.  Used for windows of at most 256
 * columns and panels of at most 32 steps while the rows fit one window-step
 * block; a replay miss or a failed Cholesky sends the panel back to mode 0.
 * Returns MPS_EINVAL for other modes.
 * ------------------------------------------------------------------------ */
mps_status mps_set_panel_mode(int32_t mode);

/* ------------------------------------------------------------------------
 * Autotuner of the pivoted-QR tiles, process-wide (not thread-safe; affects
 * later calls).  A circuit layer holds two-site updates of very different
 * bond dimensions (Sec. III-D: bonds grow from 2 up to the cap); the panel
 * width and candidate-window width that make the pivoted QR fastest differ
 * between them.  mps_autotune times, on the caller's stream, one synthetic
 * update per candidate (panel width 16/32/64 with window 0/128/256/512) for
 * each bond bucket chi = 128, 256, ... <= chi_max (chi_l = chi_m = chi_r =
 * chi, a Gaussian pair whose middle bond carries exp(-k / (150 chi / 1024)),
 * precision prec), keeps the fastest, and from then on every pivoted QR
 * with n columns uses the entry of the first bucket with n <= n_max.  The
 * pivots themselves do not depend on the tiles.  mps_set_tuning with
 * explicit values overrides the table; mps_clear_autotune drops it.
 *   work: device scratch of mps_autotune_work_bytes(chi_max, prec) bytes;
 *   table: host, max_entries entries; *n_entries receives the count.
 * chi_max must lie in [128, 8192].
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_max;        /* column counts this entry covers (above the previous entry's) */
    int32_t panel_width;  /* chosen panel width */
    int32_t qr_window;    /* chosen candidate-window width (0: no window) */
    double ms;            /* time of the tuning update with these tiles */
    double ms_default;    /* time with the built-in default (32, 256) */
} mps_tune_entry;
int64_t mps_autotune_work_bytes(int32_t chi_max, mps_precision prec);
mps_status mps_autotune(int32_t chi_max, mps_precision prec, void* work, int64_t work_bytes, void* hip_stream,
                        mps_tune_entry* table, int32_t max_entries, int32_t* n_entries);
mps_status mps_clear_autotune(void);

/* ------------------------------------------------------------------------
 * Small-bond chains, process-wide (not thread-safe; affects later calls).
 * mps_apply_gate / mps_apply_layer run a gate sequence as the ordered chain
 * of centre moves (unpivoted QR / LQ, Sec. III-C.1) and two-site updates
 * (Sec. III-C.2) that sequential application defines.  Every maximal run of
 * consecutive operations whose bond dimensions are all <= max_dim executes
 * as ONE kernel launch: a single workgroup performs the run's moves and
 * updates in order, in FP64 on workspace copies (contraction and gate,
 * Householder QR with greedy column pivoting on exactly recomputed residual
 * norms, truncation to k = min(chi_cap, 2 chi_l, 2 chi_r), Q, R P^T and the
 * renormalisation), reading and writing the sites in the context's storage
 * precision.  The remaining operations take the multi-kernel path in between.
 * The bookkept results (bond dimensions, norm fidelity, update info) are those
 * of the multi-kernel path; panels, refreshes and window_misses read 0 for a
 * chained update.  Contexts with learned pivots never chain.
 * max_dim: 0 (off) .. 64; the default is 64.  Other values: MPS_EINVAL.
 * ------------------------------------------------------------------------ */
mps_status mps_set_small_bond_limit(int32_t max_dim);

/* ------------------------------------------------------------------------
 * Truncation of a context's two-site updates (Table III: pivoted QR
 * M = Q R P^T, or SVD M = U S V^dagger; Sec. III-C.2 applies either).
 *   MPS_TRUNC_QRCP (default): truncated pivoted QR, site i <- Q_k,
 *                  site i+1 <- R_k P^T.
 *   MPS_TRUNC_SVD:  truncated SVD keeping the k = min(chi_cap, 2 chi_l,
 *                  2 chi_r) largest singular values (ties: the smaller
 *                  row of theta^H's Jacobi order), site i <- U_k,
 *                  site i+1 <- S_k V_k^dagger; eps^2 = the sum of the
 *                  discarded squared singular values.  Computed by one-sided
 *                  Jacobi in FP64: inside a small-bond chain when the bonds
 *                  are within the chain limit (mps_set_small_bond_limit),
 *                  otherwise by the multi-kernel Jacobi (a launch per round
 *                  of column pairs, a host check per sweep; meant for bonds
 *                  up to a few hundred).  Needs pivot = MPS_PIVOT_QRCP.
 * The renormalisation, norm-fidelity bookkeeping and update info are those
 * of the QR updates (qrcp_err_sq reads -1 for an SVD update).  Returns
 * MPS_EINVAL for a NULL context, an unknown mode or SVD with learned pivots.
 * ------------------------------------------------------------------------ */
typedef enum { MPS_TRUNC_QRCP = 0, MPS_TRUNC_SVD = 1 } mps_truncation;
mps_status mps_set_truncation(mps_ctx* ctx, int32_t mode);

/* ------------------------------------------------------------------------
 * Per-kernel timing.  mps_profile(mode) resets the counters and sets the
 * process-wide timing of the library's launches with HIP events recorded on
 * the caller's stream: mode 0 off; mode 1 every launch of every class; mode
 * s >= 2 only the pivot steps (MPS_K_STEP_C), sampled: one run of a panel's
 * back-to-back window-step launches in s is bracketed by a single event pair
 * and counted as that many launches (outside a window, one step launch in
 * s), which leaves the measured run nearly undisturbed (each event marker
 * costs a few microseconds of stream time).  A negative mode is MPS_EINVAL.
 * mps_profile_read fills up to n entries, indexed by mps_kernel_class, with
 * the timed launch count, their summed event time and their algorithmic
 * bytes and flops.  Not thread-safe.
 * ------------------------------------------------------------------------ */
typedef enum {
    MPS_K_CONTRACT = 0, /* theta0 = A_i A_{i+1} (MFMA GEMM)                   */
    MPS_K_GATE = 1,     /* gate + FP64 column norms                           */
    MPS_K_STEP_A = 2,   /* pivot swap, pivot-column bring-up, reflector       */
    MPS_K_STEP_C = 3,   /* pivot step: GEMV or window update, pivot row, norms*/
    MPS_K_TRAIL = 4,    /* panel-end updates A -= V F^H, A -= V W2 (MFMA)     */
    MPS_K_NORMS = 5,    /* exact norm recomputation and ||R22||_F             */
    MPS_K_UNGQR = 6,    /* Q_k formation (MFMA)                               */
    MPS_K_SPLIT = 7,    /* R_k P^T scatter into the right site                */
    MPS_K_PROPOSE = 8,  /* learned proposal: sketch, features, scores, order  */
    MPS_K_WINDOW = 9,   /* candidate-window selection, swaps, greedy replay   */
    MPS_K_PANEL = 10,   /* W = V^H A over the trailing columns (MFMA)         */
    MPS_K_REFL = 11,    /* V^H V, T, T^H W, R rows outside a window           */
    MPS_K_COUNT = 12
} mps_kernel_class;

typedef struct {
    int64_t launches;
    double total_ms;
    double alg_bytes;
    double alg_flops;
} mps_kernel_stats;

mps_status mps_profile(int mode);
mps_status mps_profile_read(mps_kernel_stats* out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* MPS_ABI_H */
