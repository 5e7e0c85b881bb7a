// MPO application by zip-up (paper Sec. III-C.3), and loading a given state
// into a context (the input of the random-saturation IQFT, Sec. III-D.1).
// Included by abi.hip after context.hpp.
//
// An MPO on the sites first .. first + ns - 1 has site tensors W_t[a, s', s, b]
// with bonds m_0 = 1, m_1, ..., m_ns = 1 (a < m_t, b < m_{t+1}; s is the input
// and s' the output physical index).  Zip-up with the orthogonality centre at
// `first`: a matrix C (rows: the new left bond, columns l + chi a over the old
// left bond l of the site and the MPO bond a; at the first site C is the
// identity) is carried from site to site.  At site i
//     T[(l' + chi' s'), (r + chi_r b)] = sum_{l, a, s} C[l', l + chi a] A_i[l, s, r] W[a, s', s, b],
// formed as m_a GEMMs X_a = C_a A_i and one pass that contracts (a, s) with
// W; T is truncated by pivoted QR to k = min(2 chi', chi_r m_b, the bond
// cap); Q becomes the new (left-canonical) site i and R P^T the next C.  At
// the last site (m_b = 1) T itself is the new site and the orthogonality
// centre.  With everything left of it left-canonical and everything right of
// it right-canonical, ||T||^2 there is the norm of the truncated state, i.e.
// the norm fidelity factor of the whole application (Sec. III-E; the state
// was normalised and the MPO is unitary, as the inverse QFT's is); T is then
// normalised and the factor goes into the norm fidelity.

// MPO bonds up to 2 (the inverse QFT's): a zip-up sweep then never needs a
// bond beyond the context's storage bound (max_bond), so with the cap at or
// above the Schmidt bounds the application is exact.
#define MPO_BOND_MAX 2

struct MpoSite {
    double2 w[MPO_BOND_MAX * 2 * 2 * MPO_BOND_MAX];   // W[a, s', s, b] at a + ma (s' + 2 (s + 2 b))
    int ma, mb;
};

// One thread per (l', r): reads X_a[l', s, r] (ld chip, a at stride xs) for
// every a < ma and s, writes T[(l' + chip s'), (r + chir b)] for every s', b.
// Reads all its inputs before writing, so `out` may be X itself when ma = 1,
// mb = 1 and the layouts coincide.
template <typename T>
__global__ __launch_bounds__(256) void k_mpo_site(const T* X, int64_t xs, int64_t chip, int64_t chir, MpoSite W,
                                                  T* out, int64_t ldo)
{
    const int64_t total = chip * chir;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t l = e % chip, r = e / chip;
        double2 xin[MPO_BOND_MAX][2];
#pragma unroll
        for (int a = 0; a < MPO_BOND_MAX; ++a)
#pragma unroll
            for (int s = 0; s < 2; ++s)
                xin[a][s] = a < W.ma ? to_d(X[a * xs + l + chip * (s + 2 * r)]) : czero();
#pragma unroll
        for (int b = 0; b < MPO_BOND_MAX; ++b) {
            if (b >= W.mb) break;
#pragma unroll
            for (int sp = 0; sp < 2; ++sp) {
                double2 acc = czero();
#pragma unroll
                for (int a = 0; a < MPO_BOND_MAX; ++a) {
                    if (a >= W.ma) break;
#pragma unroll
                    for (int s = 0; s < 2; ++s) acc = cadd(acc, cmul(xin[a][s], W.w[a + W.ma * (sp + 2 * (s + 2 * b))]));
                }
                out[(l + chip * sp) + ldo * (r + chir * b)] = from_d<T>(acc);
            }
        }
    }
}

// slot[0] += sum |x_i|^2 over n entries (FP64); slot[0] zeroed beforehand.
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* x, int64_t n, double* slot)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s += cabs2(to_d(x[i]));
    s = block_sum256(s, red);
    if (threadIdx.x == 0) atomicAdd(slot, s);
}

__global__ void k_zero_slot(double* slot)
{
    if (threadIdx.x == 0) slot[0] = 0.0;
}

// x /= sqrt(slot[0]) (left as it is when the norm is zero)
template <typename T>
__global__ __launch_bounds__(256) void k_scale_by_norm(T* x, int64_t n, const double* slot)
{
    const double s2 = slot[0];
    const double f = s2 > 0.0 ? 1.0 / sqrt(s2) : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        x[i] = from_d<T>(cscale(to_d(x[i]), f));
}

// Normalise n entries at x to unit Frobenius norm; slot is one double of
// device scratch.  Returns ||x||^2 before the scaling when want_norm.
template <typename T>
static mps_status normalise_block(T* x, int64_t n, double* slot, hipStream_t st, double* norm2_out)
{
    const unsigned nb = (unsigned)(rup(n, 256) < 1024 ? rup(n, 256) : 1024);
    hipLaunchKernelGGL(k_zero_slot, dim3(1), dim3(64), 0, st, slot);
    hipLaunchKernelGGL((k_sumsq<T>), dim3(nb), dim3(256), 0, st, (const T*)x, n, slot);
    hipLaunchKernelGGL((k_scale_by_norm<T>), dim3(nb), dim3(256), 0, st, x, n, (const double*)slot);
    HIPCHK(hipGetLastError(), "normalise launch");
    if (norm2_out) {
        HIPCHK(hipMemcpyAsync(norm2_out, slot, sizeof(double), hipMemcpyDeviceToHost, st), "norm readback");
        HIPCHK(hipStreamSynchronize(st), "norm sync");
    }
    return MPS_OK;
}

template <typename T>
static mps_status ctx_move_to(mps_ctx* c, int target)
{
    while (c->centre < target) {
        mps_status r = ctx_move_right<T>(c);
        if (r != MPS_OK) return r;
    }
    while (c->centre > target) {
        mps_status r = ctx_move_left<T>(c);
        if (r != MPS_OK) return r;
    }
    return MPS_OK;
}

template <typename T>
static mps_status ctx_apply_mpo(mps_ctx* c, int first, int ns, const int32_t* md, const double* W,
                                double* log_retained)
{
    mps_status r = ctx_move_to<T>(c, first);
    if (r != MPS_OK) return r;
    const std::vector<int64_t> old = c->dims;   // the bonds of the sites as they are before the sweep
    const int64_t eb = (int64_t)sizeof(T);
    // the carried C at the end of the workspace, sized for the largest one:
    // k <= dmax rows, chi_r m_b <= MPO_BOND_MAX dmax columns
    const int64_t cbytes = (eb * c->dmax * MPO_BOND_MAX * c->dmax + 255) / 256 * 256;
    if (cbytes + 256 > c->ws_bytes) return fail(MPS_ENOMEM, "mps_apply_mpo: workspace too small");
    T* Cm = (T*)(c->ws + (c->ws_bytes - cbytes));
    double* slot = (double*)(c->ws + (c->ws_bytes - cbytes - 256));
    const int64_t ws_left = c->ws_bytes - cbytes - 256;
    int64_t chip = old[first];   // left bond of the current site after the sweep so far
    double lsum = 0.0;
    const double* wp = W;
    for (int t = 0; t < ns; ++t) {
        const int i = first + t;
        const int ma = md[t], mb = md[t + 1];
        MpoSite ws;
        ws.ma = ma;
        ws.mb = mb;
        for (int q = 0; q < 4 * ma * mb; ++q) ws.w[q] = make_double2(wp[2 * q], wp[2 * q + 1]);
        wp += 8 * ma * mb;
        const int64_t chi = old[i], chir = old[i + 1];
        const int64_t rows = 2 * chip, cols = chir * mb;
        const bool last = t == ns - 1;
        T* site = (T*)c->site[i];
        Carver cv{c->ws, ws_left, 0};
        UpdateWs<T> w;
        int64_t k = 0;
        if (!last) {
            const int64_t kcap = max_bond(c->n, i + 1, c->chi_max);
            k = rows < cols ? rows : cols;
            k = k < kcap ? k : kcap;
            if (!carve_update_ws<T>(cv, w, rows, cols, k, true))
                return fail(MPS_ENOMEM, "mps_apply_mpo: workspace too small at site %d", i);
        }
        // X_a = C_a A_i (chip x 2 chir each), or the site itself at the first site
        const T* X = site;
        int64_t xs = 0;
        if (t > 0) {
            T* Xw = (T*)cv.take(eb * ma * chip * 2 * chir);
            if (!Xw) return fail(MPS_ENOMEM, "mps_apply_mpo: workspace too small at site %d", i);
            for (int a = 0; a < ma; ++a)
                if (!zgemm<T>(c->st, OP_N, false, OP_N, false, chip, 2 * chir, chi, C_ONE, Cm + chip * chi * a, chip,
                              site, chi, C_ZERO, Xw + chip * 2 * chir * a, chip, nullptr, 0))
                    return fail(MPS_EINVAL, "mps_apply_mpo: gemm form unavailable");
            X = Xw;
            xs = chip * 2 * chir;
        }
        T* dst = last ? site : w.d.A;
        const int64_t ldo = last ? rows : w.d.lda;
        const unsigned nb = (unsigned)(rup(chip * chir, 256) < 4096 ? rup(chip * chir, 256) : 4096);
        hipLaunchKernelGGL((k_mpo_site<T>), dim3(nb), dim3(256), 0, c->st, X, xs, chip, chir, ws, dst, ldo);
        HIPCHK(hipGetLastError(), "mpo site launch");
        if (last) {
            double n2 = 0.0;
            r = normalise_block<T>(site, rows * chir, slot, c->st, &n2);
            if (r != MPS_OK) return r;
            if (!isfinite(n2) || !(n2 > 0.0)) return fail(MPS_ENUMERIC, "mps_apply_mpo: zero or non-finite state");
            lsum = log(n2);
            c->dims[i] = chip;
            c->centre = i;
            break;
        }
        // truncated pivoted QR of T: Q -> site i, R P^T (unit norm) -> C
        w.nb = panel_width(rows, cols);
        w.win = qr_window(w.nb, cols);
        w.d.tol = recompute_tol(c->prec);
        w.d.pivoting = 1;
        const int nparts = init_norms<T>(w, c->st);
        FactorOut<T> f;
        r = factorise<T>(w, nullptr, nullptr, nparts, c->st, f);
        if (r != MPS_OK) return r;
        QrcpDev<T>& du = f.use->d;
        HIPCHK(form_q<T>(*f.use, site, rows, c->st), "mpo Q");
        hipLaunchKernelGGL((k_rpt<T>), dim3((unsigned)cols), dim3(256), 0, c->st, (const T*)du.A, du.lda,
                           (const int32_t*)du.perm, k, cols, Cm, k, (const double*)du.dsc, 0);
        HIPCHK(hipGetLastError(), "mpo split launch");
        c->dims[i] = chip;
        c->dims[i + 1] = k;
        chip = k;
    }
    c->log_fid += lsum;
    if (log_retained) *log_retained = lsum;
    return MPS_OK;
}

extern "C" mps_status mps_apply_mpo(mps_ctx* ctx, int32_t first, int32_t n_sites, const int32_t* mdims,
                                    const double* W, double* log_retained)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (n_sites < 1 || first < 0 || first + n_sites > ctx->n)
        return fail(MPS_EINVAL, "mps_apply_mpo: sites %d .. %d out of range", (int)first, (int)(first + n_sites - 1));
    if (!mdims || !W) return fail(MPS_EINVAL, "mps_apply_mpo: NULL bond dimensions or tensors");
    if (mdims[0] != 1 || mdims[n_sites] != 1)
        return fail(MPS_EINVAL, "mps_apply_mpo: the outer MPO bonds must be 1");
    int64_t nw = 0;
    for (int t = 0; t < n_sites; ++t) {
        if (mdims[t + 1] < 1 || mdims[t + 1] > MPO_BOND_MAX)
            return fail(MPS_EINVAL, "mps_apply_mpo: MPO bond %d is %d (1 .. %d supported)", t + 1, (int)mdims[t + 1],
                        MPO_BOND_MAX);
        nw += 8 * (int64_t)mdims[t] * mdims[t + 1];
    }
    for (int64_t q = 0; q < nw; ++q)
        if (!isfinite(W[q])) return fail(MPS_ENUMERIC, "mps_apply_mpo: non-finite tensor entry");
    s = ctx->prec == MPS_FP64 ? ctx_apply_mpo<double2>(ctx, first, n_sites, mdims, W, log_retained)
                              : ctx_apply_mpo<float2>(ctx, first, n_sites, mdims, W, log_retained);
    if (s == MPS_EDEVICE || s == MPS_ENUMERIC) ctx->poisoned = true;
    return s;
}

// Load a state: site j (dims[j] x 2 x dims[j+1], entry (l, s, r) at
// l + dims[j] (s + 2 r), complex FP64 from the host) for every site, then a
// sweep of LQ moves from the last site to the first (right-canonical form,
// centre 0) and normalisation of site 0.  The norm fidelity restarts at 1.
template <typename T>
static mps_status ctx_load_state(mps_ctx* c, const int64_t* dims, const double* data)
{
    const double* p = data;
    std::vector<T> buf;
    for (int j = 0; j < c->n; ++j) {
        const int64_t ne = dims[j] * 2 * dims[j + 1];
        buf.resize(ne);
        for (int64_t q = 0; q < ne; ++q) {
            buf[q].x = p[2 * q];
            buf[q].y = p[2 * q + 1];
        }
        p += 2 * ne;
        HIPCHK(hipMemcpyAsync(c->site[j], buf.data(), sizeof(T) * ne, hipMemcpyHostToDevice, c->st), "load site");
        HIPCHK(hipStreamSynchronize(c->st), "load sync");
        c->dims[j] = dims[j];
    }
    c->dims[c->n] = dims[c->n];
    c->centre = c->n - 1;
    mps_status r = ctx_move_to<T>(c, 0);
    if (r != MPS_OK) return r;
    double* slot = (double*)(c->ws + c->ws_bytes - 256);
    double n2 = 0.0;
    r = normalise_block<T>((T*)c->site[0], 2 * c->dims[1], slot, c->st, &n2);
    if (r != MPS_OK) return r;
    if (!isfinite(n2) || !(n2 > 0.0)) return fail(MPS_ENUMERIC, "mps_load_state: zero or non-finite state");
    c->log_fid = 0.0;
    return MPS_OK;
}

extern "C" mps_status mps_load_state(mps_ctx* ctx, const int64_t* dims, const double* data)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (!dims || !data) return fail(MPS_EINVAL, "mps_load_state: NULL dims or data");
    if (dims[0] != 1 || dims[ctx->n] != 1) return fail(MPS_EINVAL, "mps_load_state: the outer bonds must be 1");
    int64_t total = 0;
    for (int j = 0; j < ctx->n; ++j) {
        if (dims[j + 1] < 1 || dims[j + 1] > max_bond(ctx->n, j + 1, ctx->chi_max))
            return fail(MPS_EINVAL, "mps_load_state: bond %d is %lld, beyond its cap %lld", j + 1,
                        (long long)dims[j + 1], (long long)max_bond(ctx->n, j + 1, ctx->chi_max));
        total += dims[j] * 2 * dims[j + 1];
    }
    for (int64_t q = 0; q < 2 * total; ++q)
        if (!isfinite(data[q])) return fail(MPS_ENUMERIC, "mps_load_state: non-finite entry");
    s = ctx->prec == MPS_FP64 ? ctx_load_state<double2>(ctx, dims, data) : ctx_load_state<float2>(ctx, dims, data);
    if (s == MPS_EDEVICE || s == MPS_ENUMERIC) ctx->poisoned = true;
    return s;
}
