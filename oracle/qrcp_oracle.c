/*
 * Plain FP64 CPU oracle for the two-site update's factorisation step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path loads this file's
 * library; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (paper Sec. III-B.2, Table III "QR with pivoting",
 * M = Q R P^T, and Sec. II-B: pivoted QR allows truncation):
 *
 *   Greedy column-pivoted Householder QR, stopped after k = min(kmax, m, n)
 *   columns.  At every step j the pivot is the column whose residual (the
 *   part orthogonal to the columns already chosen) has the largest Euclidean
 *   norm.  The residual norms are recomputed exactly at every step from the
 *   current trailing block -- no norm downdating -- so the pivot rule is the
 *   greedy definition written out.  Equal norms go to the smallest original
 *   column index.  "Equal" is read at 40 significant bits: the squared norms
 *   are compared after rounding off the low 12 bits of their FP64 mantissa,
 *   so a tie that is exact in exact arithmetic resolves by index whatever
 *   last-bit rounding the summation left (see pivot_key).
 *
 *   Householder convention (LAPACK xLARFG): for x = (alpha, x_rest),
 *     if x_rest = 0 and Im(alpha) = 0:  tau = 0 (H = I), beta = alpha;
 *     else beta = -sign(Re alpha) * ||x||,  tau = (beta - alpha)/beta,
 *          v = (1, x_rest / (alpha - beta)).
 *   H = I - tau v v^H,  H^H x = (beta, 0, ..., 0),  Q = H_0 H_1 ... H_{k-1}.
 *
 * All matrices are column-major with explicit leading dimensions.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

static double abs2(cplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* A non-negative squared norm rounded to the nearest value with 40
 * significant mantissa bits (the low 12 bits rounded off): values within
 * about 2^-41 relative compare equal.  Rounding to nearest keeps simple
 * values such as 1/2 in the middle of their interval, so last-bit rounding
 * on either side of them does not separate them. */
static double pivot_key(double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    b = (b + (uint64_t)0x800) & ~(uint64_t)0xfff;
    memcpy(&v, &b, sizeof v);
    return v;
}

/* Generate the reflector for x[0..len-1] in place: x[0] <- beta, x[1:] <- v[1:].
 * Returns tau. */
static cplx householder(cplx* x, int64_t len)
{
    double rest = 0.0;
    for (int64_t i = 1; i < len; ++i) rest += abs2(x[i]);
    cplx alpha = x[0];
    if (rest == 0.0 && cimag(alpha) == 0.0) return 0.0;
    double nrm = sqrt(abs2(alpha) + rest);
    double beta = creal(alpha) >= 0.0 ? -nrm : nrm;
    cplx tau = (beta - alpha) / beta;
    cplx scale = 1.0 / (alpha - beta);
    for (int64_t i = 1; i < len; ++i) x[i] *= scale;
    x[0] = beta;
    return tau;
}

/*
 * orc_qrcp: factorise A (m x n) as A P = Q R, keep k = min(kmax, m, n) steps.
 *
 *   pivoting = 0 gives the unpivoted Householder QR (piv = identity).
 *   Q     : m x k, orthonormal columns (ldq >= m)
 *   R     : k x n upper trapezoidal, columns in pivot order (ldr >= k)
 *   piv   : piv[j] = original column placed at position j (all n entries)
 *   diagR : R[j, j] for j < k (real)
 *   err_fro : Frobenius norm of the trailing block left after k steps (||R22||_F)
 *   gaps  : optional (may be NULL), k doubles: at pivoting step j the relative
 *           margin (nu_1 - nu_2) / nu_1 between the largest and the second
 *           largest squared residual norm among the candidates (1 when only one
 *           candidate is left or nu_1 = 0).  A margin near the rounding level
 *           marks a step whose pivot another correct implementation may take
 *           differently.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int orc_qrcp(int64_t m, int64_t n, int64_t kmax, int pivoting,
             const cplx* A, int64_t lda,
             cplx* Q, int64_t ldq, cplx* R, int64_t ldr,
             int32_t* piv, double* diagR, double* err_fro, int64_t* k_out, double* gaps)
{
    if (m < 0 || n < 0 || kmax < 0 || lda < (m > 1 ? m : 1)) return -1;
    int64_t k = kmax;
    if (k > m) k = m;
    if (k > n) k = n;
    if (ldq < (m > 1 ? m : 1) || ldr < (k > 1 ? k : 1)) return -1;

    cplx* W = (cplx*)malloc(sizeof(cplx) * (size_t)(m > 0 ? m : 1) * (size_t)(n > 0 ? n : 1));
    cplx* tau = (cplx*)malloc(sizeof(cplx) * (size_t)(k > 0 ? k : 1));
    double* nrm = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!W || !tau || !nrm) { free(W); free(tau); free(nrm); return -1; }
    for (int64_t c = 0; c < n; ++c)
        memcpy(W + c * m, A + c * lda, sizeof(cplx) * (size_t)m);
    for (int64_t c = 0; c < n; ++c) piv[c] = (int32_t)c;

    for (int64_t j = 0; j < k; ++j) {
        if (pivoting) {
            /* exact residual norms of the trailing columns */
            #pragma omp parallel for schedule(static)
            for (int64_t c = j; c < n; ++c) {
                double s = 0.0;
                const cplx* col = W + c * m;
                for (int64_t i = j; i < m; ++i) s += abs2(col[i]);
                nrm[c] = s;
            }
            int64_t best = j;
            for (int64_t c = j + 1; c < n; ++c) {
                const double kc = pivot_key(nrm[c]), kb = pivot_key(nrm[best]);
                if (kc > kb || (kc == kb && piv[c] < piv[best]))
                    best = c;
            }
            if (gaps) {
                double second = -1.0;
                for (int64_t c = j; c < n; ++c)
                    if (c != best && nrm[c] > second) second = nrm[c];
                gaps[j] = (second < 0.0 || nrm[best] <= 0.0) ? 1.0 : (nrm[best] - second) / nrm[best];
            }
            if (best != j) {
                cplx* a = W + j * m;
                cplx* b = W + best * m;
                for (int64_t i = 0; i < m; ++i) { cplx t = a[i]; a[i] = b[i]; b[i] = t; }
                int32_t t = piv[j]; piv[j] = piv[best]; piv[best] = t;
            }
        } else if (gaps) {
            gaps[j] = 1.0;
        }
        cplx* x = W + j * m + j;
        tau[j] = householder(x, m - j);
        diagR[j] = creal(x[0]);
        /* apply H_j^H = I - conj(tau) v v^H to the trailing columns */
        const cplx ctau = conj(tau[j]);
        if (ctau != 0.0) {
            #pragma omp parallel for schedule(static)
            for (int64_t c = j + 1; c < n; ++c) {
                cplx* col = W + c * m + j;
                cplx w = col[0];                       /* v[0] = 1 */
                for (int64_t i = 1; i < m - j; ++i) w += conj(x[i]) * col[i];
                w *= ctau;
                col[0] -= w;
                for (int64_t i = 1; i < m - j; ++i) col[i] -= x[i] * w;
            }
        }
    }

    /* R: upper trapezoid of the first k rows */
    for (int64_t c = 0; c < n; ++c)
        for (int64_t t = 0; t < k; ++t)
            R[t + c * ldr] = (c < t) ? 0.0 : (c == t ? (cplx)diagR[t] : W[t + c * m]);

    /* truncation error: the block below row k right of column k */
    double e2 = 0.0;
    for (int64_t c = k; c < n; ++c)
        for (int64_t i = k; i < m; ++i) e2 += abs2(W[i + c * m]);
    *err_fro = sqrt(e2);

    /* Q = H_0 ... H_{k-1} [I_k; 0], accumulated backwards */
    for (int64_t c = 0; c < k; ++c)
        for (int64_t i = 0; i < m; ++i) Q[i + c * ldq] = (i == c) ? 1.0 : 0.0;
    for (int64_t j = k - 1; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        const cplx* v = W + j * m + j;   /* v[0] = 1 implicitly */
        const cplx tj = tau[j];
        #pragma omp parallel for schedule(static)
        for (int64_t c = j; c < k; ++c) {
            cplx* col = Q + c * ldq + j;
            cplx w = col[0];
            for (int64_t i = 1; i < m - j; ++i) w += conj(v[i]) * col[i];
            w *= tj;
            col[0] -= w;
            for (int64_t i = 1; i < m - j; ++i) col[i] -= v[i] * w;
        }
    }
    *k_out = k;
    free(W); free(tau); free(nrm);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
