// Small-bond chains: one launch for a run of a layer's operations.
//
// Under sequential-canonical semantics a layer is an ordered chain of
// operations: before each two-site update the orthogonality centre moves to
// the bond by unpivoted QR (to the right) or LQ (to the left) of the sites on
// the way, then the update contracts, pivots, truncates and splits (paper
// Sec. III-C.1 and III-C.2; the ordering reading is the sequential one).  Near
// the ends of the chain the bonds are small (2, 4, 8, ...), and on the
// multi-kernel path such an operation costs launch and host-synchronisation
// latency, not arithmetic.  Here one workgroup runs a whole run of
// consecutive small operations, in order, from a single launch:
//
//   * every matrix (theta at most 2*CH_DIM_MAX square) lives in the workspace
//     in FP64; sites are read and written in the context's storage precision;
//   * factorisations are unblocked Householder QR (LAPACK reflector
//     convention) with, for the update, greedy column pivoting on residual
//     column norms recomputed exactly after every step (ties: the smaller
//     original column index);
//   * Q is accumulated backwards from the reflectors; R P^T is scattered into
//     the right site and scaled by 1/sqrt(||theta||^2 - eps^2);
//   * with SVD truncation (Table III) the update instead runs one-sided
//     Jacobi on theta^H and keeps the k largest singular values (below).
//
// The bond dimension every operation produces follows from the shapes alone
// (k = min(chi_cap, m, n) for an update, min(rows, cols) for a centre move),
// so the host plans the run up front and reads the per-update norms back once.
#pragma once
#include "update.hpp"

#define CH_NT 256          // threads of the chain workgroup
#define CH_DIM_MAX 64      // largest bond dimension a chain operation may touch

enum { CH_RIGHT = 0, CH_LEFT = 1, CH_UPDATE = 2, CH_UPDATE_SVD = 3 };

// One operation of a chain (host-built, read by the kernel).
//   CH_RIGHT  centre s -> s+1.  s0 = site s (2 dl x dr), s1 = site s+1
//             (dr x 2 dx).  Site s <- Q (2 dl x k); site s+1 <- R (site s+1).
//   CH_LEFT   centre s -> s-1.  s0 = site s (dl x 2 dr as a matrix),
//             s1 = site s-1 (2 dx x dl).  With site^H = Q' R':
//             site s <- Q'^H (k x 2 dr); site s-1 <- (site s-1) R'^H.
//   CH_UPDATE bond (i, i+1).  s0 = site i (2 dl x dm), s1 = site i+1
//             (dm x 2 dr).  Site i <- Q (2 dl x k), site i+1 <- R P^T
//             renormalised; info[2 slot] = ||theta||^2, info[2 slot + 1] = eps^2.
//   CH_UPDATE_SVD  as CH_UPDATE with the truncated SVD instead of pivoted QR:
//             site i <- U_k, site i+1 <- S_k V_k^H renormalised.
struct ChainOp {
    int32_t kind;
    int32_t slot;
    int32_t dl, dm, dr, dx, k, pad;
    void* s0;
    void* s1;
    double2 g[16];   // gate, row (a' b'), column (a b), a on the left site
};

// FP64 scratch of the chain kernel (one workgroup): matrices of mat x mat.
struct ChainWs {
    double2* M;      // the matrix being factorised (ld = its row count)
    double2* Q;      // accumulated Q
    double2* P;      // product staging
    double2* tau;    // mat
    double* nu;      // mat
    int32_t* perm;   // mat
};

static inline int64_t chain_ws_bytes(int64_t mat)
{
    return 3 * (16 * mat * mat + 256) + (16 + 8 + 4) * mat + 3 * 256;
}

// Lanes that cooperate on one column when `ncols` columns share the block:
// the largest power of two with G * ncols <= CH_NT, at most a wavefront.
__device__ __forceinline__ int ch_group(int ncols)
{
    int G = 64;
    while (G > 1 && G * ncols > CH_NT) G >>= 1;
    return G;
}

__device__ __forceinline__ double ch_group_sum(double v, int G)
{
    for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, MPS_WAVE);
    return v;
}

// nu[c] = sum_{i >= r0} |X[i, c]|^2 for c < ncols (X ld ldx).
__device__ void ch_colnorms(const double2* X, int ldx, int rows, int r0, int ncols, double* nu)
{
    const int G = ch_group(ncols), gl = threadIdx.x % G, groups = CH_NT / G;
    for (int c = threadIdx.x / G; c < ncols; c += groups) {
        const double2* x = X + (int64_t)ldx * c;
        double s = 0.0;
        for (int i = r0 + gl; i < rows; i += G) s += cabs2(x[i]);
        s = ch_group_sum(s, G);
        if (gl == 0) nu[c] = s;
    }
}

// Apply I - coef v v^H to columns [0, ncols) of X (rows 0..len-1 of X are
// rows j.. of the matrix; v(0) = 1, v(i) = V[i] for i >= 1).  With nu, also
// nu[c] = sum_{i >= 1} |X[i, c]|^2 afterwards (the residual norm below the
// reflector's row).
__device__ void ch_reflect(const double2* V, int len, double2 coef, double2* X, int ldx, int ncols, double* nu)
{
    if (ncols <= 0) return;
    const int G = ch_group(ncols), gl = threadIdx.x % G, groups = CH_NT / G;
    for (int c = threadIdx.x / G; c < ncols; c += groups) {
        double2* x = X + (int64_t)ldx * c;
        double sr = 0.0, si = 0.0;
        for (int i = gl; i < len; i += G) {
            const double2 v = i == 0 ? make_double2(1.0, 0.0) : V[i];
            const double2 t = cmulc(v, x[i]);
            sr += t.x;
            si += t.y;
        }
        sr = ch_group_sum(sr, G);
        si = ch_group_sum(si, G);
        const double2 w = cmul(coef, make_double2(sr, si));
        double nn = 0.0;
        for (int i = gl; i < len; i += G) {
            const double2 v = i == 0 ? make_double2(1.0, 0.0) : V[i];
            const double2 xn = csub(x[i], cmul(w, v));
            x[i] = xn;
            if (i > 0) nn += cabs2(xn);
        }
        if (nu) {
            nn = ch_group_sum(nn, G);
            if (gl == 0) nu[c] = nn;
        }
    }
}

struct ChLds {
    double red[4];
    ArgBest arg[4];
    int flag;
};

// Householder QR of M (m x n, ld m) in place, k steps: R on and above the
// diagonal, reflector j below it (v(0) = 1 implicit), tau[j].  With pivot,
// step j first brings the column of largest residual norm (rows >= j) to
// position j; perm tracks the original indices.  Returns with a barrier.
__device__ void ch_qr(double2* M, int m, int n, int k, bool pivot, double2* tau, double* nu, int32_t* perm, ChLds& L)
{
    const int tid = threadIdx.x;
    if (pivot) {
        for (int c = tid; c < n; c += CH_NT) perm[c] = c;
        ch_colnorms(M, m, m, 0, n, nu);
    }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        double2* col = M + (int64_t)m * j;
        if (pivot) {
            ArgBest a;
            a.val = -1.0;
            a.key = 0x7fffffff;
            a.slot = -1;
            for (int c = j + tid; c < n; c += CH_NT)
                if (arg_better(nu[c], perm[c], a.val, a.key)) {
                    a.val = nu[c];
                    a.key = perm[c];
                    a.slot = c;
                }
            a = block_argmax256(a, L.arg);
            const int p = a.slot;
            if (p != j && p >= 0) {
                double2* cp = M + (int64_t)m * p;
                for (int i = tid; i < m; i += CH_NT) {
                    const double2 t = col[i];
                    col[i] = cp[i];
                    cp[i] = t;
                }
                if (tid == 0) {
                    const int32_t tp = perm[j];
                    perm[j] = perm[p];
                    perm[p] = tp;
                    const double tn = nu[j];
                    nu[j] = nu[p];
                    nu[p] = tn;
                }
            }
            __syncthreads();
        }
        double rest = 0.0;
        for (int i = j + 1 + tid; i < m; i += CH_NT) rest += cabs2(col[i]);
        rest = block_sum256(rest, L.red);
        const double2 alpha = col[j];
        double2 t, scale;
        double beta;
        if (rest == 0.0 && alpha.y == 0.0) {
            t = czero();
            scale = czero();
            beta = alpha.x;
        } else {
            const double nrm = sqrt(cabs2(alpha) + rest);
            beta = alpha.x >= 0.0 ? -nrm : nrm;
            t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
            scale = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
        }
        __syncthreads();   // alpha read everywhere before it is overwritten
        for (int i = j + 1 + tid; i < m; i += CH_NT) col[i] = cmul(scale, col[i]);
        if (tid == 0) {
            col[j] = make_double2(beta, 0.0);
            tau[j] = t;
        }
        __syncthreads();
        // the columns right of j: a <- (I - conj(tau) v v^H) a
        ch_reflect(col + j, m - j, cconj(t), M + j + (int64_t)m * (j + 1), m, n - j - 1, pivot ? nu + j + 1 : nullptr);
        __syncthreads();
    }
}

// Q (m x k, ld m) = H_0 ... H_{k-1} [I_k; 0] from the reflectors of ch_qr.
__device__ void ch_form_q(const double2* M, int m, int k, const double2* tau, double2* Q)
{
    for (int idx = threadIdx.x; idx < m * k; idx += CH_NT)
        Q[idx] = (idx % m == idx / m) ? make_double2(1.0, 0.0) : czero();
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {
        ch_reflect(M + j + (int64_t)m * j, m - j, tau[j], Q + j + (int64_t)m * j, m, k - j, nullptr);
        __syncthreads();
    }
}

// theta = G (A B): A = site (2 dl x dm), B = site (dm x 2 dr); theta row
// l + dl a', column b' + 2 r.
template <typename T>
__device__ void ch_theta(const T* A, const T* B, int dl, int dm, int dr, const double2* g, double2* th)
{
    const int m = 2 * dl;
    for (int pidx = threadIdx.x; pidx < dl * dr; pidx += CH_NT) {
        const int l = pidx % dl, r = pidx / dl;
        double2 t[4] = {czero(), czero(), czero(), czero()};   // (a, b) = 00, 01, 10, 11
        for (int q = 0; q < dm; ++q) {
            const double2 a0 = to_d(A[l + (int64_t)m * q]), a1 = to_d(A[l + dl + (int64_t)m * q]);
            const double2 b0 = to_d(B[q + (int64_t)dm * (2 * r)]), b1 = to_d(B[q + (int64_t)dm * (2 * r + 1)]);
            t[0] = cadd(t[0], cmul(a0, b0));
            t[1] = cadd(t[1], cmul(a0, b1));
            t[2] = cadd(t[2], cmul(a1, b0));
            t[3] = cadd(t[3], cmul(a1, b1));
        }
        double2 o[4];
#pragma unroll
        for (int row = 0; row < 4; ++row) {
            double2 s = czero();
#pragma unroll
            for (int c = 0; c < 4; ++c) s = cadd(s, cmul(g[4 * row + c], t[c]));
            o[row] = s;
        }
        th[l + (int64_t)m * (2 * r)] = o[0];
        th[l + (int64_t)m * (2 * r + 1)] = o[1];
        th[l + dl + (int64_t)m * (2 * r)] = o[2];
        th[l + dl + (int64_t)m * (2 * r + 1)] = o[3];
    }
}

template <typename T>
__device__ void ch_update(const ChainOp* op, const ChainWs& w, double* info, ChLds& L)
{
    const int dl = op->dl, dm = op->dm, dr = op->dr, k = op->k;
    const int m = 2 * dl, n = 2 * dr;
    T* A = (T*)op->s0;
    T* B = (T*)op->s1;
    ch_theta<T>(A, B, dl, dm, dr, op->g, w.M);
    __syncthreads();
    double s_all = 0.0;
    for (int idx = threadIdx.x; idx < m * n; idx += CH_NT) s_all += cabs2(w.M[idx]);
    s_all = block_sum256(s_all, L.red);
    ch_qr(w.M, m, n, k, true, w.tau, w.nu, w.perm, L);
    // eps^2 = ||R22||_F^2 over the trailing block, explicitly
    double s_eps = 0.0;
    for (int idx = threadIdx.x; idx < m * n; idx += CH_NT) {
        const int i = idx % m, c = idx / m;
        if (i >= k && c >= k) s_eps += cabs2(w.M[idx]);
    }
    s_eps = block_sum256(s_eps, L.red);
    ch_form_q(w.M, m, k, w.tau, w.Q);
    const double kept = s_all - s_eps;
    const double sc = kept > 0.0 ? 1.0 / sqrt(kept) : 1.0;
    for (int idx = threadIdx.x; idx < m * k; idx += CH_NT) A[idx] = from_d<T>(w.Q[idx]);
    for (int idx = threadIdx.x; idx < k * n; idx += CH_NT) {
        const int t = idx % k, c = idx / k;
        const double2 v = t <= c ? w.M[t + (int64_t)m * c] : czero();
        B[t + (int64_t)k * w.perm[c]] = from_d<T>(cscale(v, sc));
    }
    if (threadIdx.x == 0) {
        info[2 * op->slot] = s_all;
        info[2 * op->slot + 1] = s_eps;
    }
}

// One-sided (Hestenes) Jacobi on the columns of X (rx x cols, ld rx): pairs of
// columns are rotated until every pair is orthogonal to working precision,
// |x_p^H x_q| <= CH_JTOL ||x_p|| ||x_q||; the same unitary rotations are
// applied to the columns of V (rv x cols, ld rv).  A column with
// ||x||^2 <= floor2 counts as numerically zero and is not rotated (with more
// columns than rows, or a rank-deficient X, such columns hold only rounding
// noise, whose angles never settle).  A sweep visits every pair once in
// round-robin order (cols/2 disjoint pairs per round, one group of lanes per
// pair); at most CH_JSWEEPS sweeps.  Returns with a barrier.
#define CH_JTOL 1e-14
#define CH_JSWEEPS 60
__device__ void ch_jacobi(double2* X, int rx, int cols, double2* V, int rv, double floor2, ChLds& L)
{
    if (cols < 2) return;
    const int cp = cols + (cols & 1), npairs = cp / 2;
    const int G = ch_group(npairs), gl = threadIdx.x % G, pi = threadIdx.x / G;
    for (int sweep = 0; sweep < CH_JSWEEPS; ++sweep) {
        if (threadIdx.x == 0) L.flag = 0;
        __syncthreads();
        for (int r = 0; r < cp - 1; ++r) {
            int p = cp - 1, q = r;
            if (pi > 0) {
                p = (r + pi) % (cp - 1);
                q = (r - pi + cp - 1) % (cp - 1);
            }
            if (p > q) {
                const int t = p;
                p = q;
                q = t;
            }
            if (pi < npairs && q < cols) {
                double2* xp = X + (int64_t)rx * p;
                double2* xq = X + (int64_t)rx * q;
                double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
                for (int i = gl; i < rx; i += G) {
                    const double2 u = xp[i], v = xq[i];
                    a += cabs2(u);
                    b += cabs2(v);
                    const double2 t = cmulc(u, v);   // conj(u) v
                    gr += t.x;
                    gi += t.y;
                }
                a = ch_group_sum(a, G);
                b = ch_group_sum(b, G);
                gr = ch_group_sum(gr, G);
                gi = ch_group_sum(gi, G);
                const double g = sqrt(gr * gr + gi * gi);
                if (a > floor2 && b > floor2 && g > CH_JTOL * sqrt(a * b)) {
                    // [x_p, x_q] <- [x_p, x_q] J, J = [[c, s e], [-s conj(e), c]],
                    // e = gamma / |gamma|, t = s / c the smaller root of
                    // t^2 + 2 zeta t - 1 = 0, zeta = (b - a) / (2 |gamma|)
                    const double zeta = (b - a) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    const double2 e = make_double2(gr / g, gi / g);
                    const double2 se = cscale(e, sn), sec = cscale(cconj(e), sn);
                    for (int i = gl; i < rx; i += G) {
                        const double2 u = xp[i], v = xq[i];
                        xp[i] = csub(cscale(u, c), cmul(sec, v));
                        xq[i] = cadd(cmul(se, u), cscale(v, c));
                    }
                    double2* vp = V + (int64_t)rv * p;
                    double2* vq = V + (int64_t)rv * q;
                    for (int i = gl; i < rv; i += G) {
                        const double2 u = vp[i], v = vq[i];
                        vp[i] = csub(cscale(u, c), cmul(sec, v));
                        vq[i] = cadd(cmul(se, u), cscale(v, c));
                    }
                    if (gl == 0) L.flag = 1;
                }
            }
            __syncthreads();
        }
        const int rotated = L.flag;
        __syncthreads();   // every lane has read the flag before it is reset
        if (!rotated) break;
    }
}

// Truncated SVD update.  With X = theta^H (n x m) and V = I (m x m), Jacobi
// gives X V = W with orthogonal columns, so theta = V W^H and the singular
// values are the column norms of W.  The k largest (ties: the smaller
// column) are kept: site i <- their columns of V (orthonormal whatever the
// rank), site i+1 <- the matching rows of W^H scaled by 1/sqrt(kept);
// eps^2 = the sum of the discarded squared column norms.
template <typename T>
__device__ void ch_update_svd(const ChainOp* op, const ChainWs& w, double* info, ChLds& L)
{
    const int dl = op->dl, dm = op->dm, dr = op->dr, k = op->k;
    const int m = 2 * dl, n = 2 * dr;
    T* A = (T*)op->s0;
    T* B = (T*)op->s1;
    ch_theta<T>(A, B, dl, dm, dr, op->g, w.M);
    __syncthreads();
    double s_all = 0.0;
    for (int idx = threadIdx.x; idx < m * n; idx += CH_NT) s_all += cabs2(w.M[idx]);
    s_all = block_sum256(s_all, L.red);
    double2* X = w.P;   // n x m, ld n
    for (int idx = threadIdx.x; idx < n * m; idx += CH_NT) {
        const int i = idx % n, c = idx / n;
        X[idx] = cconj(w.M[c + (int64_t)m * i]);
    }
    for (int idx = threadIdx.x; idx < m * m; idx += CH_NT)
        w.Q[idx] = (idx % m == idx / m) ? make_double2(1.0, 0.0) : czero();
    __syncthreads();
    // columns below 1e-14 of ||theta||_F are numerically zero
    ch_jacobi(X, n, m, w.Q, m, 1e-28 * s_all, L);
    ch_colnorms(X, n, n, 0, m, w.nu);
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += CH_NT) {
        const double v = w.nu[j];
        int rank = 0;
        for (int i = 0; i < m; ++i) rank += (w.nu[i] > v || (w.nu[i] == v && i < j)) ? 1 : 0;
        w.perm[rank] = j;
    }
    __syncthreads();
    double s_eps = 0.0;
    for (int r = k + (int)threadIdx.x; r < m; r += CH_NT) s_eps += w.nu[w.perm[r]];
    s_eps = block_sum256(s_eps, L.red);
    const double kept = s_all - s_eps;
    const double sc = kept > 0.0 ? 1.0 / sqrt(kept) : 1.0;
    for (int idx = threadIdx.x; idx < m * k; idx += CH_NT) {
        const int i = idx % m, t = idx / m;
        A[idx] = from_d<T>(w.Q[i + (int64_t)m * w.perm[t]]);
    }
    for (int idx = threadIdx.x; idx < k * n; idx += CH_NT) {
        const int t = idx % k, c = idx / k;
        B[idx] = from_d<T>(cscale(cconj(X[c + (int64_t)n * w.perm[t]]), sc));
    }
    if (threadIdx.x == 0) {
        info[2 * op->slot] = s_all;
        info[2 * op->slot + 1] = s_eps;
    }
}

template <typename T>
__device__ void ch_move_right(const ChainOp* op, const ChainWs& w, ChLds& L)
{
    const int m = 2 * op->dl, n = op->dr, k = op->k, nx = 2 * op->dx;
    T* S = (T*)op->s0;
    T* B = (T*)op->s1;
    for (int idx = threadIdx.x; idx < m * n; idx += CH_NT) w.M[idx] = to_d(S[idx]);
    __syncthreads();
    ch_qr(w.M, m, n, k, false, w.tau, w.nu, w.perm, L);
    ch_form_q(w.M, m, k, w.tau, w.Q);
    // P (k x nx) = R (k x n) B (n x nx)
    for (int idx = threadIdx.x; idx < k * nx; idx += CH_NT) {
        const int t = idx % k, c = idx / k;
        double2 s = czero();
        for (int q = t; q < n; ++q) s = cadd(s, cmul(w.M[t + (int64_t)m * q], to_d(B[q + (int64_t)n * c])));
        w.P[idx] = s;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * k; idx += CH_NT) S[idx] = from_d<T>(w.Q[idx]);
    for (int idx = threadIdx.x; idx < k * nx; idx += CH_NT) B[idx] = from_d<T>(w.P[idx]);
}

template <typename T>
__device__ void ch_move_left(const ChainOp* op, const ChainWs& w, ChLds& L)
{
    const int dl = op->dl, m = 2 * op->dr, k = op->k, mx = 2 * op->dx;
    T* S = (T*)op->s0;   // dl x m matrix view (ld dl)
    T* P0 = (T*)op->s1;  // site s-1: mx x dl
    // M = S^H (m x dl)
    for (int idx = threadIdx.x; idx < m * dl; idx += CH_NT) {
        const int i = idx % m, c = idx / m;
        w.M[idx] = cconj(to_d(S[c + (int64_t)dl * i]));
    }
    __syncthreads();
    ch_qr(w.M, m, dl, k, false, w.tau, w.nu, w.perm, L);
    ch_form_q(w.M, m, k, w.tau, w.Q);
    // P (mx x k) = P0 (mx x dl) R'^H, R' = k x dl upper trapezoidal
    for (int idx = threadIdx.x; idx < mx * k; idx += CH_NT) {
        const int i = idx % mx, t = idx / mx;
        double2 s = czero();
        for (int c = t; c < dl; ++c) s = cadd(s, cmul(to_d(P0[i + (int64_t)mx * c]), cconj(w.M[t + (int64_t)m * c])));
        w.P[idx] = s;
    }
    __syncthreads();
    // site s <- Q'^H (k x m, ld k)
    for (int idx = threadIdx.x; idx < k * m; idx += CH_NT) {
        const int t = idx % k, i = idx / k;
        S[idx] = from_d<T>(cconj(w.Q[i + (int64_t)m * t]));
    }
    for (int idx = threadIdx.x; idx < mx * k; idx += CH_NT) P0[idx] = from_d<T>(w.P[idx]);
}

// One workgroup executes ops[0 .. nops) in order.
template <typename T>
__global__ __launch_bounds__(CH_NT) void k_chain(const ChainOp* ops, int nops, ChainWs w, double* info)
{
    __shared__ ChLds L;
    for (int o = 0; o < nops; ++o) {
        const ChainOp* op = ops + o;
        const int kind = op->kind;
        if (kind == CH_UPDATE) ch_update<T>(op, w, info, L);
        else if (kind == CH_UPDATE_SVD) ch_update_svd<T>(op, w, info, L);
        else if (kind == CH_RIGHT) ch_move_right<T>(op, w, L);
        else ch_move_left<T>(op, w, L);
        __syncthreads();
    }
}
