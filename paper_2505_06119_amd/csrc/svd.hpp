// Truncated SVD of a two-site update for bonds beyond the small-bond chains
// (Table III, M = U S V^dagger; Sec. III-C.2 applies it as the truncating
// decomposition).  Included by abi.hip after bond.hpp.
//
// The method is the chain kernel's one-sided (Hestenes) Jacobi, spread over
// the GPU: with X = theta^H (n x m, FP64) and V = I (m x m), each round of a
// sweep rotates the m/2 disjoint column pairs of the round-robin schedule,
// one block per pair (a block reduction of ||x_p||^2, ||x_q||^2 and
// x_p^H x_q, then the rotation of both columns of X and of V), so a sweep is
// m - 1 launches; sweeps repeat until one rotates nothing (the host reads a
// flag per sweep) or 60 have run.  Then X V = W has orthogonal columns,
// theta = V W^H, and the singular values are the column norms of W: the k
// largest (ties: the smaller column) give site i <- their columns of V and
// site i+1 <- the matching rows of W^H scaled to unit norm; eps^2 is the sum
// of the discarded squared norms.  The rotation, the tolerance and the
// treatment of numerically zero columns are the chain kernel's (chain.hpp).

#define SVD_NT 256

// X (n x m, ld n) = theta^H in FP64, V = I (m x m)
template <typename T>
__global__ __launch_bounds__(256) void k_svd_init(const T* th, int64_t ldt, int m, int n, double2* X, double2* V)
{
    const int64_t total = (int64_t)n * m;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, c = e / n;   // X[i, c] = conj(theta[c, i])
        X[e] = cconj(to_d(th[c + ldt * i]));
    }
    const int64_t tv = (int64_t)m * m;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tv; e += (int64_t)gridDim.x * 256)
        V[e] = (e % m == e / m) ? make_double2(1.0, 0.0) : czero();
}

__global__ void k_svd_flag_reset(int32_t* flag)
{
    if (threadIdx.x == 0) __hip_atomic_store(flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One round r of a sweep: block pi takes pair pi of the round-robin schedule
// over cp = m rounded up to even columns (the chain kernel's order); pairs
// that touch the padding column are skipped.  floor2 = 1e-28 ||theta||^2
// (dsc[DSC_NORM2]) marks numerically zero columns.
__global__ __launch_bounds__(SVD_NT) void k_jacobi_round(double2* X, int rx, int cols, double2* V, int rv, int r,
                                                         const double* dsc, int32_t* flag)
{
    __shared__ double red[4][SVD_NT / 64];
    const int cp = cols + (cols & 1);
    const int pi = blockIdx.x;
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
    if (q >= cols) return;   // uniform over the block
    double2* xp = X + (int64_t)rx * p;
    double2* xq = X + (int64_t)rx * q;
    double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
    for (int i = threadIdx.x; i < rx; i += SVD_NT) {
        const double2 u = xp[i], v = xq[i];
        a += cabs2(u);
        b += cabs2(v);
        const double2 t = cmulc(u, v);   // conj(u) v
        gr += t.x;
        gi += t.y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    gr = wave_sum(gr);
    gi = wave_sum(gi);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
        red[2][wid] = gr;
        red[3][wid] = gi;
    }
    __syncthreads();
    a = b = gr = gi = 0.0;
    for (int w = 0; w < SVD_NT / 64; ++w) {
        a += red[0][w];
        b += red[1][w];
        gr += red[2][w];
        gi += red[3][w];
    }
    const double floor2 = 1e-28 * dsc[DSC_NORM2];
    const double g = sqrt(gr * gr + gi * gi);
    if (!(a > floor2 && b > floor2 && g > CH_JTOL * sqrt(a * b))) return;   // uniform
    // [x_p, x_q] <- [x_p, x_q] J, J = [[c, s e], [-s conj(e), c]], e = gamma / |gamma|,
    // t = s / c the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (b - a) / (2 |gamma|)
    const double zeta = (b - a) / (2.0 * g);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
    const double2 e = make_double2(gr / g, gi / g);
    const double2 se = cscale(e, sn), sec = cscale(cconj(e), sn);
    for (int i = threadIdx.x; i < rx; i += SVD_NT) {
        const double2 u = xp[i], v = xq[i];
        xp[i] = csub(cscale(u, c), cmul(sec, v));
        xq[i] = cadd(cmul(se, u), cscale(v, c));
    }
    double2* vp = V + (int64_t)rv * p;
    double2* vq = V + (int64_t)rv * q;
    for (int i = threadIdx.x; i < rv; i += SVD_NT) {
        const double2 u = vp[i], v = vq[i];
        vp[i] = csub(cscale(u, c), cmul(sec, v));
        vq[i] = cadd(cmul(se, u), cscale(v, c));
    }
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// nu[j] = ||X[:, j]||^2, one block per column
__global__ __launch_bounds__(256) void k_svd_colnorms(const double2* X, int rx, double* nu)
{
    __shared__ double red[4];
    const double2* x = X + (int64_t)rx * blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < rx; i += 256) s += cabs2(x[i]);
    s = block_sum256(s, red);
    if (threadIdx.x == 0) nu[blockIdx.x] = s;
}

// site i (m x k, ld m) <- V[:, perm[t]]; site i+1 (k x n, ld k) <- sc conj(X[:, perm[t]])^T
template <typename T>
__global__ __launch_bounds__(256) void k_svd_out(const double2* X, int n, const double2* V, int m, const int32_t* perm,
                                                 int k, double sc, T* A_out, T* B_out)
{
    const int64_t ta = (int64_t)m * k, tb = (int64_t)k * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < ta + tb; e += (int64_t)gridDim.x * 256) {
        if (e < ta) {
            const int64_t i = e % m, t = e / m;
            A_out[e] = from_d<T>(V[i + (int64_t)m * perm[t]]);
        } else {
            const int64_t f = e - ta, t = f % k, c = f / k;
            B_out[f] = from_d<T>(cscale(cconj(X[c + (int64_t)n * perm[t]]), sc));
        }
    }
}

#define SVD_SWEEPS_MAX 60

// The two-site update with truncated-SVD truncation: theta as in update_core
// (a1-a3), then the Jacobi SVD above.  Outputs as update_core's (A_out =
// U_k, B_out = S_k V_k^H renormalised); theta lives in the workspace, so the
// outputs may alias the inputs.
template <typename T>
static mps_status svd_update(int64_t chi_l, int64_t chi_m, int64_t chi_r, int64_t chi_cap, const T* A, const T* B,
                             const double* g, T* A_out, T* B_out, mps_update_info* info, void* work, int64_t work_bytes,
                             hipStream_t st)
{
    const int64_t m = 2 * chi_l, n = 2 * chi_r;
    int64_t k = chi_cap < m ? chi_cap : m;
    k = k < n ? k : n;
    Carver cv{(char*)work, work_bytes, 0};
    UpdateWs<T> w;
    if (!carve_update_ws<T>(cv, w, m, n, k, true)) return fail(MPS_ENOMEM, "svd update: workspace too small");
    double2* X = (double2*)cv.take(16 * n * m);
    double2* V = (double2*)cv.take(16 * m * m);
    double* nu = (double*)cv.take(8 * m);
    int32_t* perm = (int32_t*)cv.take(4 * m);
    int32_t* flag = (int32_t*)cv.take(256);
    if (!X || !V || !nu || !perm || !flag) return fail(MPS_ENOMEM, "svd update: workspace too small");
    QrcpDev<T>& d = w.d;
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, d.ctl, d.dsc);
    if (!zgemm<T>(st, OP_N, false, OP_N, false, m, n, chi_m, C_ONE, A, m, B, chi_m, C_ZERO, d.A, d.lda, w.gsplit,
                  w.gsplit_bytes))
        return fail(MPS_EINVAL, "svd update: gemm form unavailable");
    hipLaunchKernelGGL((k_gate_norms<T>), dim3((unsigned)chi_r), dim3(256), 0, st, d, chi_l, make_gate(g));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double*)d.npart, (int)chi_r, d.dsc,
                       (int)DSC_NORM2);
    {
        const int64_t tot = n * m > m * m ? n * m : m * m;
        const unsigned nb = (unsigned)(rup(tot, 256) < 4096 ? rup(tot, 256) : 4096);
        hipLaunchKernelGGL((k_svd_init<T>), dim3(nb), dim3(256), 0, st, (const T*)d.A, d.lda, (int)m, (int)n, X, V);
    }
    HIPCHK(hipGetLastError(), "svd update launch");
    const int cp = (int)(m + (m & 1));
    int sweeps = 0;
    for (; sweeps < SVD_SWEEPS_MAX && m > 1; ++sweeps) {
        hipLaunchKernelGGL(k_svd_flag_reset, dim3(1), dim3(64), 0, st, flag);
        for (int r = 0; r < cp - 1; ++r)
            hipLaunchKernelGGL(k_jacobi_round, dim3((unsigned)(cp / 2)), dim3(SVD_NT), 0, st, X, (int)n, (int)m, V,
                               (int)m, r, (const double*)d.dsc, flag);
        int32_t h = 0;
        HIPCHK(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st), "svd flag readback");
        HIPCHK(hipStreamSynchronize(st), "svd sweep sync");
        if (!h) break;
    }
    hipLaunchKernelGGL(k_svd_colnorms, dim3((unsigned)m), dim3(256), 0, st, (const double2*)X, (int)n, nu);
    std::vector<double> hnu(m);
    double dsc[DSC_COUNT];
    HIPCHK(hipMemcpyAsync(hnu.data(), nu, sizeof(double) * m, hipMemcpyDeviceToHost, st), "svd norms readback");
    HIPCHK(hipMemcpyAsync(dsc, d.dsc, sizeof(dsc), hipMemcpyDeviceToHost, st), "svd readback");
    HIPCHK(hipStreamSynchronize(st), "svd sync");
    const double s_all = dsc[DSC_NORM2];
    if (!isfinite(s_all)) return fail(MPS_ENUMERIC, "update: non-finite theta");
    // the k largest squared norms, ties to the smaller column
    std::vector<int32_t> order(m);
    for (int64_t j = 0; j < m; ++j) order[j] = (int32_t)j;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return hnu[x] > hnu[y]; });
    double s_eps = 0.0;
    for (int64_t r = k; r < m; ++r) s_eps += hnu[order[r]];
    const double kept = s_all - s_eps;
    const double sc = kept > 0.0 ? 1.0 / sqrt(kept) : 1.0;
    HIPCHK(hipMemcpyAsync(perm, order.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st), "svd order upload");
    {
        const int64_t tot = m * k + k * n;
        const unsigned nb = (unsigned)(rup(tot, 256) < 4096 ? rup(tot, 256) : 4096);
        hipLaunchKernelGGL((k_svd_out<T>), dim3(nb), dim3(256), 0, st, (const double2*)X, (int)n, (const double2*)V,
                           (int)m, (const int32_t*)perm, (int)k, sc, A_out, B_out);
    }
    HIPCHK(hipGetLastError(), "svd output launch");
    HIPCHK(hipStreamSynchronize(st), "svd output sync");
    if (info) {
        info->k = k;
        info->trunc_err_sq = s_eps;
        info->norm_sq = s_all;
        info->retained = s_all > 0 ? 1.0 - s_eps / s_all : 1.0;
        info->fallback = 0;
        info->panels = 0;
        info->refreshes = 0;
        info->window_misses = 0;
        info->learned_err_sq = -1.0;
        info->qrcp_err_sq = -1.0;
    }
    return MPS_OK;
}
