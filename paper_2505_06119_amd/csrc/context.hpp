// Stateful MPS context (included at the end of abi.hip, after the error
// helpers and update_core).  The state is a chain of site tensors in a
// caller-provided device arena, kept normalised with one orthogonality centre;
// moves of the centre are unpivoted Householder QR (to the right) or LQ, done
// as the QR of the conjugate transpose (to the left) -- paper Sec. III-C.1.

template <typename T>
__global__ __launch_bounds__(256) void k_iota(int32_t* perm, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        perm[i] = (int32_t)i;
}

// dst (cols x rows, ldd) = src (rows x cols, lds)^H, through 32x32 LDS tiles.
template <typename T>
__global__ __launch_bounds__(256) void k_conj_transpose(const T* src, int64_t lds, int64_t rows, int64_t cols,
                                                        T* dst, int64_t ldd)
{
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + tx, c = c0 + q;
        if (r < rows && c < cols) tile[q][tx] = src[r + lds * c];
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t c = c0 + tx, r = r0 + q;   // dst row = c, dst col = r
        if (r < rows && c < cols) {
            T v = tile[tx][q];
            v.y = -v.y;
            dst[c + ldd * r] = v;
        }
    }
}

// out[r] = sum_l v[l] * S[l + ld*r]  (row vector times matrix, FP64 accumulate)
template <typename T>
__global__ __launch_bounds__(256) void k_vecmat(const double2* v, const T* S, int64_t ld, int64_t rows,
                                                int64_t cols, double2* out)
{
    __shared__ double red_lds[8];
    __shared__ double red_out[2];
    const int64_t r = blockIdx.x;
    if (r >= cols) return;
    double2 acc = czero();
    for (int64_t l = threadIdx.x; l < rows; l += 256) acc = cadd(acc, cmul(v[l], to_d(S[l + ld * r])));
    double a[2] = {acc.x, acc.y};
    block_sum_vec<2>(a, red_lds, red_out);
    if (threadIdx.x == 0) out[r] = make_double2(red_out[0], red_out[1]);
}

struct mps_ctx {
    mps_config cfg;
    int n;
    int64_t chi_max;
    mps_precision prec;
    hipStream_t st;
    std::vector<int64_t> dims;   // n + 1 bond dimensions
    std::vector<int64_t> cap;    // per-site capacity in elements
    std::vector<char*> site;
    char* ws;
    int64_t ws_bytes;
    char* tmp;                   // max site capacity
    char* rbuf;                  // dmax * dmax elements
    double2* vec0;
    double2* vec1;
    int32_t centre;
    double log_fid;
    bool poisoned;
    bool has_net;          // pivot network set (learned mode)
    mps_learned_cfg lcfg;
    ChainOp* chain_ops;    // device: operations of the small-bond chains of one call
    double* chain_info;    // device: ||theta||^2, eps^2 per chained update
    int64_t chain_cap;     // capacity of chain_ops (entries)
    int64_t dmax;          // largest bond dimension the state can reach
    int32_t trunc;         // mps_truncation of the two-site updates
};

// Storage bound of bond b (between sites b-1 and b): the cap chi, the
// Schmidt bound 2^b of the b sites on its left, and twice the Schmidt bound
// 2^(n-b) of the sites on its right.  The factor 2 is the room an MPO of bond
// 2 needs while a left-to-right zip-up sweep crosses the bond: the matrix
// truncated there still carries the MPO bond on its right (see mpo.hpp).
static int64_t max_bond(int n, int b, int64_t chi)
{
    int64_t d = chi;
    const int e1 = b, e2 = n - b + 1;
    if (e1 < 62 && ((int64_t)1 << e1) < d) d = (int64_t)1 << e1;
    if (e2 < 62 && ((int64_t)1 << e2) < d) d = (int64_t)1 << e2;
    return d;
}

struct CtxLayout {
    std::vector<int64_t> off;   // site offsets
    std::vector<int64_t> cap;
    int64_t dmax, ws_off, ws_bytes, tmp_off, rbuf_off, vec_off, chain_off, chain_cap, total;
};

// Operations one call can chain: every gate of a layer needs its update and
// at most n_sites centre moves in all (the centre crosses each bond at most
// once per direction change, and a layer's bonds are increasing).
static int64_t chain_capacity(int n_sites) { return 3 * (int64_t)n_sites + 8; }

static bool ctx_layout(const mps_config* cfg, CtxLayout& L)
{
    const int n = cfg->n_sites;
    const int64_t eb = elem_bytes(cfg->prec);
    L.off.assign(n, 0);
    L.cap.assign(n, 0);
    int64_t pos = 0, maxcap = 0;
    L.dmax = 1;
    for (int j = 0; j < n; ++j) {
        const int64_t dl = max_bond(n, j, cfg->chi_max), dr = max_bond(n, j + 1, cfg->chi_max);
        if (dl > L.dmax) L.dmax = dl;
        L.cap[j] = dl * 2 * dr;
        maxcap = L.cap[j] > maxcap ? L.cap[j] : maxcap;
        L.off[j] = pos;
        pos += (L.cap[j] * eb + 255) / 256 * 256;
    }
    const int64_t m = 2 * L.dmax;
    L.ws_off = pos;
    L.ws_bytes = (cfg->prec == MPS_FP64 ? update_ws_bytes<double2>(m, m, L.dmax)
                                        : update_ws_bytes<float2>(m, m, L.dmax)) +
                 16 * eb * (m * m + 64);
    if (cfg->pivot == MPS_PIVOT_LEARNED)
        L.ws_bytes += cfg->prec == MPS_FP64 ? learn_ws_bytes<double2>(m, m, L.dmax, PN_ELL_MAX)
                                            : learn_ws_bytes<float2>(m, m, L.dmax, PN_ELL_MAX);
    pos += (L.ws_bytes + 255) / 256 * 256;
    L.tmp_off = pos;
    pos += (maxcap * eb + 255) / 256 * 256;
    L.rbuf_off = pos;
    pos += (L.dmax * L.dmax * eb + 255) / 256 * 256;
    L.vec_off = pos;
    pos += 2 * ((L.dmax * 16 + 255) / 256 * 256);
    L.chain_off = pos;
    L.chain_cap = chain_capacity(n);
    pos += (L.chain_cap * (int64_t)sizeof(ChainOp) + 255) / 256 * 256 + (16 * (int64_t)(n + 1) + 255) / 256 * 256;
    L.total = pos + 256;
    return true;
}

static bool cfg_valid(const mps_config* cfg)
{
    return cfg && cfg->n_sites >= 2 && cfg->n_sites <= 4096 && cfg->chi_max >= 1 && cfg->chi_max <= (1 << 16) &&
           valid_prec(cfg->prec) && (cfg->pivot == MPS_PIVOT_QRCP || cfg->pivot == MPS_PIVOT_LEARNED);
}

extern "C" int64_t mps_arena_bytes(const mps_config* cfg)
{
    if (!cfg_valid(cfg)) return -1;
    CtxLayout L;
    ctx_layout(cfg, L);
    return L.total;
}

template <typename T>
static mps_status ctx_init_sites(mps_ctx* c)
{
    std::vector<T> one(2);
    one[0].x = 1; one[0].y = 0;
    one[1].x = 0; one[1].y = 0;
    for (int j = 0; j < c->n; ++j)
        HIPCHK(hipMemcpyAsync(c->site[j], one.data(), 2 * sizeof(T), hipMemcpyHostToDevice, c->st), "init site");
    HIPCHK(hipStreamSynchronize(c->st), "init sync");
    return MPS_OK;
}

extern "C" mps_status mps_create(const mps_config* cfg, void* dev_arena, int64_t arena_bytes, void* hip_stream,
                                 mps_ctx** out)
{
    if (!out) return fail(MPS_EINVAL, "mps_create: out is NULL");
    *out = nullptr;
    if (!cfg_valid(cfg)) return fail(MPS_EINVAL, "mps_create: invalid configuration");
    if (!dev_arena) return fail(MPS_EINVAL, "mps_create: arena is NULL");
    if (cfg->pivot == MPS_PIVOT_LEARNED && cfg->mlp_weights) {
        mps_learned_cfg lc;
        lc.params = cfg->mlp_weights;
        lc.sketch_rows = cfg->sketch_rows;
        lc.verify = cfg->learned_verify;
        lc.seed = cfg->seed;
        lc.fallback_ratio = cfg->fallback_ratio;
        if (!learned_cfg_valid(&lc))
            return fail(MPS_EINVAL, "mps_create: invalid learned-pivot settings (sketch_rows, learned_verify, "
                                    "fallback_ratio)");
    }
    CtxLayout L;
    ctx_layout(cfg, L);
    if (arena_bytes < L.total)
        return fail(MPS_ENOMEM, "mps_create: arena needs %lld bytes, got %lld", (long long)L.total,
                    (long long)arena_bytes);
    char* base = (char*)(((uintptr_t)dev_arena + 255) & ~(uintptr_t)255);
    mps_ctx* c = new mps_ctx();
    c->cfg = *cfg;
    c->n = cfg->n_sites;
    c->chi_max = cfg->chi_max;
    c->prec = cfg->prec;
    c->st = (hipStream_t)hip_stream;
    c->dims.assign(c->n + 1, 1);
    c->cap = L.cap;
    c->site.resize(c->n);
    for (int j = 0; j < c->n; ++j) c->site[j] = base + L.off[j];
    c->ws = base + L.ws_off;
    c->ws_bytes = L.ws_bytes;
    c->tmp = base + L.tmp_off;
    c->rbuf = base + L.rbuf_off;
    c->vec0 = (double2*)(base + L.vec_off);
    c->vec1 = (double2*)(base + L.vec_off + (L.dmax * 16 + 255) / 256 * 256);
    c->chain_ops = (ChainOp*)(base + L.chain_off);
    c->chain_cap = L.chain_cap;
    c->dmax = L.dmax;
    c->chain_info = (double*)(base + L.chain_off + (L.chain_cap * (int64_t)sizeof(ChainOp) + 255) / 256 * 256);
    c->centre = 0;
    c->log_fid = 0.0;
    c->poisoned = false;
    c->has_net = false;
    if (cfg->pivot == MPS_PIVOT_LEARNED && cfg->mlp_weights) {
        c->lcfg.params = cfg->mlp_weights;
        c->lcfg.sketch_rows = cfg->sketch_rows;
        c->lcfg.verify = cfg->learned_verify;
        c->lcfg.seed = cfg->seed;
        c->lcfg.fallback_ratio = cfg->fallback_ratio;
        c->has_net = true;
    }
    c->trunc = MPS_TRUNC_QRCP;
    mps_status s = c->prec == MPS_FP64 ? ctx_init_sites<double2>(c) : ctx_init_sites<float2>(c);
    if (s != MPS_OK) {
        delete c;
        return s;
    }
    *out = c;
    return MPS_OK;
}

extern "C" mps_status mps_destroy(mps_ctx* ctx)
{
    if (!ctx) return fail(MPS_EINVAL, "mps_destroy: NULL context");
    delete ctx;
    return MPS_OK;
}

// Unpivoted QR of M (m x n, ld m) in the context workspace: Q (m x k', ldq)
// and R (k' x n, ld k') into rbuf.  k' = min(m, n).
// Unpivoted Householder QR of the m x n matrix M (or of M^H when transpose_in:
// M is then given as the n x m matrix with leading dimension ld_in), k =
// min(m, n): Q (m x k, ldq) and R (k x n, ld k) into R_out.  The workspace
// (ws, ws_bytes) holds the factorisation.  A centre move (Sec. III-C.1).
template <typename T>
static mps_status move_qr(char* ws, int64_t ws_bytes, hipStream_t st, const T* M, int64_t m, int64_t n,
                          bool transpose_in, int64_t ld_in, T* Q, int64_t ldq, T* R_out, int64_t* kout)
{
    const int64_t k = m < n ? m : n;
    Carver cv{ws, ws_bytes, 0};
    UpdateWs<T> w;
    if (!carve_update_ws<T>(cv, w, m, n, k, true)) return fail(MPS_ENOMEM, "centre move: workspace too small");
    w.nb = panel_width(m, n);
    w.d.tol = 0.0;
    w.d.pivoting = 0;
    if (transpose_in) {
        dim3 grid((unsigned)rup(n, 32), (unsigned)rup(m, 32));
        hipLaunchKernelGGL((k_conj_transpose<T>), grid, dim3(256), 0, st, M, ld_in, n, m, w.d.A, w.d.lda);
    } else {
        dim3 grid((unsigned)(rup(m, 256) < 64 ? rup(m, 256) : 64), (unsigned)n);
        hipLaunchKernelGGL((k_copy_cols<T>), grid, dim3(256), 0, st, M, ld_in, w.d.A, w.d.lda, m);
    }
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st, w.d.ctl, w.d.dsc);
    hipLaunchKernelGGL((k_iota<T>), dim3((unsigned)rup(n, 256)), dim3(256), 0, st, w.d.perm, n);
    HIPCHK(hipGetLastError(), "centre move launch");
    HIPCHK(run_qrcp<T>(w, st, nullptr, 0), "centre move QR");
    HIPCHK(form_q<T>(w, Q, ldq, st), "centre move Q");
    hipLaunchKernelGGL((k_rpt<T>), dim3((unsigned)n), dim3(256), 0, st, (const T*)w.d.A, w.d.lda,
                       (const int32_t*)w.d.perm, k, n, R_out, k, (const double*)w.d.dsc, 0);
    HIPCHK(hipGetLastError(), "centre move R");
    *kout = k;
    return MPS_OK;
}

template <typename T>
static mps_status ctx_qr(mps_ctx* c, const T* M, int64_t m, int64_t n, bool transpose_in, int64_t ld_in, T* Q,
                         int64_t ldq, int64_t* kout)
{
    return move_qr<T>(c->ws, c->ws_bytes, c->st, M, m, n, transpose_in, ld_in, Q, ldq, (T*)c->rbuf, kout);
}

template <typename T>
static mps_status ctx_move_right(mps_ctx* c)
{
    const int s = c->centre;
    const int64_t chl = c->dims[s], chr = c->dims[s + 1], chr2 = c->dims[s + 2];
    T* A = (T*)c->site[s];
    int64_t k = 0;
    mps_status r = ctx_qr<T>(c, A, 2 * chl, chr, false, 2 * chl, A, 2 * chl, &k);
    if (r != MPS_OK) return r;
    // site s+1 <- R (k x chr) * B (chr x 2 chr2)
    T* B = (T*)c->site[s + 1];
    if (!zgemm<T>(c->st, OP_N, false, OP_N, false, k, 2 * chr2, chr, C_ONE, (const T*)c->rbuf, k, B, chr, C_ZERO,
                  (T*)c->tmp, k, nullptr, 0))
        return fail(MPS_EINVAL, "centre move: gemm form unavailable");
    HIPCHK(hipMemcpyAsync(B, c->tmp, sizeof(T) * k * 2 * chr2, hipMemcpyDeviceToDevice, c->st), "centre move copy");
    c->dims[s + 1] = k;
    c->centre = s + 1;
    return MPS_OK;
}

template <typename T>
static mps_status ctx_move_left(mps_ctx* c)
{
    const int s = c->centre;
    const int64_t chl = c->dims[s], chr = c->dims[s + 1], chl2 = c->dims[s - 1];
    T* A = (T*)c->site[s];
    // LQ of A (chl x 2chr): A^H = Q' R', A = R'^H Q'^H
    int64_t k = 0;
    mps_status r = ctx_qr<T>(c, A, 2 * chr, chl, true, chl, (T*)c->tmp, 2 * chr, &k);
    if (r != MPS_OK) return r;
    {
        dim3 grid((unsigned)rup(2 * chr, 32), (unsigned)rup(k, 32));
        hipLaunchKernelGGL((k_conj_transpose<T>), grid, dim3(256), 0, c->st, (const T*)c->tmp, 2 * chr, 2 * chr,
                           k, A, k);
    }
    // site s-1 (2chl2 x chl) <- site s-1 * R'^H
    T* P = (T*)c->site[s - 1];
    if (!zgemm<T>(c->st, OP_N, false, OP_C, false, 2 * chl2, k, chl, C_ONE, P, 2 * chl2, (const T*)c->rbuf, k,
                  C_ZERO, (T*)c->tmp, 2 * chl2, nullptr, 0))
        return fail(MPS_EINVAL, "centre move: gemm form unavailable");
    HIPCHK(hipMemcpyAsync(P, c->tmp, sizeof(T) * 2 * chl2 * k, hipMemcpyDeviceToDevice, c->st), "centre move copy");
    c->dims[s] = k;
    c->centre = s - 1;
    return MPS_OK;
}

// Largest bond dimension of an operation that runs in a small-bond chain
// (mps_set_small_bond_limit; 0: every operation takes the multi-kernel path).
static int g_chain_dim = CH_DIM_MAX;

// Gates t = 0 .. ng-1 on bonds idx[t] with sequential semantics.  The centre
// moves and updates are planned first; consecutive operations whose bond
// dimensions are all <= the chain limit run as one k_chain launch, the others
// on the multi-kernel path in between.  Norm fidelities are accumulated in
// gate order after one read-back of the chained updates' norms.
template <typename T>
static mps_status ctx_run_gates(mps_ctx* c, int64_t ng, const int32_t* idx, const double* g, mps_update_info* info)
{
    struct Step {
        int kind, s, t;
        bool fused;
    };
    int lim = c->cfg.pivot == MPS_PIVOT_QRCP ? g_chain_dim : 0;
    // every bond dimension during the call is <= c->dmax (the structural
    // bound), and a chained operation's are <= lim: matrices of at most mat rows
    const int64_t mat = 2 * (c->dmax < lim ? c->dmax : (int64_t)lim);
    if (lim > 0 && chain_ws_bytes(mat) > c->ws_bytes) lim = 0;
    const int64_t half = lim > 0 ? mat / 2 : 0;   // = min(dmax, lim)
    auto small = [&](int64_t a, int64_t b, int64_t d) { return a <= half && b <= half && d <= half; };

    // plan: the operations and the bond dimensions they produce
    std::vector<int64_t> dims = c->dims;
    int centre = c->centre;
    std::vector<Step> steps;
    std::vector<ChainOp> ops;
    int nslots = 0;
    for (int64_t t = 0; t < ng; ++t) {
        const int i = idx[t];
        const int target = centre <= i ? i : i + 1;
        while (centre != target) {
            ChainOp op = {};
            const int s = centre;
            if (centre < target) {
                op.kind = CH_RIGHT;
                op.dl = (int32_t)dims[s];
                op.dr = (int32_t)dims[s + 1];
                op.dx = (int32_t)dims[s + 2];
                op.k = (int32_t)(2 * dims[s] < dims[s + 1] ? 2 * dims[s] : dims[s + 1]);
                op.s0 = c->site[s];
                op.s1 = c->site[s + 1];
                dims[s + 1] = op.k;
                ++centre;
            } else {
                op.kind = CH_LEFT;
                op.dl = (int32_t)dims[s];
                op.dr = (int32_t)dims[s + 1];
                op.dx = (int32_t)dims[s - 1];
                op.k = (int32_t)(2 * dims[s + 1] < dims[s] ? 2 * dims[s + 1] : dims[s]);
                op.s0 = c->site[s];
                op.s1 = c->site[s - 1];
                dims[s] = op.k;
                --centre;
            }
            const bool f = small(op.dl, op.dr, op.dx);
            steps.push_back({op.kind, s, (int)t, f});
            if (f) ops.push_back(op);
        }
        ChainOp op = {};
        op.kind = c->trunc == MPS_TRUNC_SVD ? CH_UPDATE_SVD : CH_UPDATE;
        op.dl = (int32_t)dims[i];
        op.dm = (int32_t)dims[i + 1];
        op.dr = (int32_t)dims[i + 2];
        int64_t k = c->chi_max < 2 * dims[i] ? c->chi_max : 2 * dims[i];
        k = k < 2 * dims[i + 2] ? k : 2 * dims[i + 2];
        op.k = (int32_t)k;
        op.s0 = c->site[i];
        op.s1 = c->site[i + 1];
        for (int q = 0; q < 16; ++q) op.g[q] = make_double2(g[32 * t + 2 * q], g[32 * t + 2 * q + 1]);
        const bool f = small(op.dl, op.dm, op.dr);
        if (f) op.slot = nslots++;
        steps.push_back({CH_UPDATE, i, (int)t, f});
        if (f) ops.push_back(op);
        dims[i + 1] = k;
        centre = i + 1;
    }
    if ((int64_t)ops.size() > c->chain_cap) return fail(MPS_EINVAL, "gates: too many chained operations");
    if (!ops.empty())
        HIPCHK(hipMemcpyAsync(c->chain_ops, ops.data(), sizeof(ChainOp) * ops.size(), hipMemcpyHostToDevice, c->st),
               "chain upload");

    // execute
    Carver cv{c->ws, c->ws_bytes, 0};
    ChainWs cw;
    cw.M = (double2*)cv.take(16 * mat * mat);
    cw.Q = (double2*)cv.take(16 * mat * mat);
    cw.P = (double2*)cv.take(16 * mat * mat);
    cw.tau = (double2*)cv.take(16 * mat);
    cw.nu = (double*)cv.take(8 * mat);
    cw.perm = (int32_t*)cv.take(4 * mat);
    std::vector<double> retained(ng, 1.0);
    std::vector<int> slot_of(ng, -1);
    size_t next_op = 0;
    for (size_t q = 0; q < steps.size();) {
        const Step& st = steps[q];
        if (st.fused) {
            size_t e = q;
            while (e < steps.size() && steps[e].fused) ++e;
            const size_t nops = e - q;
            hipLaunchKernelGGL((k_chain<T>), dim3(1), dim3(CH_NT), 0, c->st, (const ChainOp*)(c->chain_ops + next_op),
                               (int)nops, cw, c->chain_info);
            HIPCHK(hipGetLastError(), "chain launch");
            for (size_t u = 0; u < nops; ++u) {
                const ChainOp& op = ops[next_op + u];
                const Step& su = steps[q + u];
                if (op.kind == CH_RIGHT) {
                    c->dims[su.s + 1] = op.k;
                    c->centre = su.s + 1;
                } else if (op.kind == CH_LEFT) {
                    c->dims[su.s] = op.k;
                    c->centre = su.s - 1;
                } else {
                    c->dims[su.s + 1] = op.k;
                    c->centre = su.s + 1;
                    slot_of[su.t] = op.slot;
                }
            }
            next_op += nops;
            q = e;
            continue;
        }
        mps_status r = MPS_OK;
        if (st.kind == CH_RIGHT) r = ctx_move_right<T>(c);
        else if (st.kind == CH_LEFT) r = ctx_move_left<T>(c);
        else {
            mps_update_info loc;
            const int i = st.s;
            const mps_learned_cfg* lc = c->cfg.pivot == MPS_PIVOT_LEARNED ? &c->lcfg : nullptr;
            if (c->trunc == MPS_TRUNC_SVD)
                r = svd_update<T>(c->dims[i], c->dims[i + 1], c->dims[i + 2], c->chi_max, (const T*)c->site[i],
                                  (const T*)c->site[i + 1], g + 32 * st.t, (T*)c->site[i], (T*)c->site[i + 1], &loc,
                                  c->ws, c->ws_bytes, c->st);
            else
                r = update_core<T>(c->dims[i], c->dims[i + 1], c->dims[i + 2], c->chi_max, c->prec,
                                   (const T*)c->site[i], (const T*)c->site[i + 1], g + 32 * st.t, (T*)c->site[i],
                                   (T*)c->site[i + 1], 1, lc, &loc, c->ws, c->ws_bytes, c->st);
            if (r == MPS_OK) {
                c->dims[i + 1] = loc.k;
                c->centre = i + 1;
                retained[st.t] = loc.retained;
                if (info) info[st.t] = loc;
            }
        }
        if (r != MPS_OK) return r;
        ++q;
    }
    if (nslots > 0) {
        std::vector<double> h(2 * (size_t)nslots);
        HIPCHK(hipMemcpyAsync(h.data(), c->chain_info, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->st),
               "chain read-back");
        HIPCHK(hipStreamSynchronize(c->st), "chain sync");
        bool finite = true;
        for (int64_t t = 0; t < ng; ++t) {
            const int sl = slot_of[t];
            if (sl < 0) continue;
            const double n2 = h[2 * sl], e2 = h[2 * sl + 1];
            finite = finite && isfinite(n2) && isfinite(e2);
            retained[t] = n2 > 0.0 ? 1.0 - e2 / n2 : 1.0;
            if (info) {
                mps_update_info& u = info[t];
                u.k = c->dims[idx[t] + 1];
                u.trunc_err_sq = e2;
                u.norm_sq = n2;
                u.retained = retained[t];
                u.fallback = 0;
                u.panels = 0;
                u.refreshes = 0;
                u.window_misses = 0;
                u.learned_err_sq = -1.0;
                u.qrcp_err_sq = c->trunc == MPS_TRUNC_SVD ? -1.0 : e2;
            }
        }
        if (!finite) return fail(MPS_ENUMERIC, "chained update: non-finite theta");
    } else {
        HIPCHK(hipStreamSynchronize(c->st), "gates sync");
    }
    for (int64_t t = 0; t < ng; ++t)
        if (retained[t] > 0) c->log_fid += log(retained[t]);
    return MPS_OK;
}

extern "C" mps_status mps_set_truncation(mps_ctx* ctx, int32_t mode)
{
    if (!ctx) return fail(MPS_EINVAL, "mps_set_truncation: NULL context");
    if (mode != MPS_TRUNC_QRCP && mode != MPS_TRUNC_SVD)
        return fail(MPS_EINVAL, "mps_set_truncation: unknown mode %d", (int)mode);
    if (mode == MPS_TRUNC_SVD && ctx->cfg.pivot != MPS_PIVOT_QRCP)
        return fail(MPS_EINVAL, "mps_set_truncation: SVD truncation needs pivot = MPS_PIVOT_QRCP");
    ctx->trunc = mode;
    return MPS_OK;
}

extern "C" mps_status mps_set_small_bond_limit(int32_t max_dim)
{
    if (max_dim < 0 || max_dim > CH_DIM_MAX)
        return fail(MPS_EINVAL, "mps_set_small_bond_limit: %d outside 0..%d", (int)max_dim, CH_DIM_MAX);
    g_chain_dim = max_dim;
    return MPS_OK;
}

extern "C" mps_status mps_set_pivot_network(mps_ctx* ctx, const mps_learned_cfg* cfg)
{
    if (!ctx) return fail(MPS_EINVAL, "mps_set_pivot_network: NULL context");
    if (ctx->cfg.pivot != MPS_PIVOT_LEARNED)
        return fail(MPS_EINVAL, "mps_set_pivot_network: context was not created for learned pivots");
    if (!learned_cfg_valid(cfg)) return fail(MPS_EINVAL, "mps_set_pivot_network: invalid mps_learned_cfg");
    ctx->lcfg = *cfg;
    ctx->has_net = true;
    return MPS_OK;
}

static mps_status ctx_check(const mps_ctx* c)
{
    if (!c) return fail(MPS_EINVAL, "NULL context");
    if (c->poisoned)
        return fail(MPS_ESTATE, "context unusable after an earlier device failure or non-finite result");
    return MPS_OK;
}

extern "C" mps_status mps_apply_gate(mps_ctx* ctx, int32_t i, const double* g, mps_update_info* info)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (i < 0 || i >= ctx->n - 1) return fail(MPS_EINVAL, "mps_apply_gate: bond %d out of range", (int)i);
    if (!g) return fail(MPS_EINVAL, "mps_apply_gate: NULL gate");
    if (!gate_finite(g)) return fail(MPS_ENUMERIC, "mps_apply_gate: non-finite gate entry");
    if (ctx->cfg.pivot == MPS_PIVOT_LEARNED && !ctx->has_net)
        return fail(MPS_EINVAL, "mps_apply_gate: learned pivots need mps_set_pivot_network first");
    const int32_t one = i;
    s = ctx->prec == MPS_FP64 ? ctx_run_gates<double2>(ctx, 1, &one, g, info)
                              : ctx_run_gates<float2>(ctx, 1, &one, g, info);
    // a non-finite theta has already rewritten sites: the state is lost
    if (s == MPS_EDEVICE || s == MPS_ENUMERIC) ctx->poisoned = true;
    return s;
}

extern "C" mps_status mps_apply_layer(mps_ctx* ctx, int64_t n, const int32_t* idx, const double* g,
                                      mps_update_info* info)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (n < 0 || (n > 0 && (!idx || !g))) return fail(MPS_EINVAL, "mps_apply_layer: bad arrays");
    if (ctx->cfg.pivot == MPS_PIVOT_LEARNED && !ctx->has_net)
        return fail(MPS_EINVAL, "mps_apply_layer: learned pivots need mps_set_pivot_network first");
    for (int64_t t = 0; t < n; ++t) {
        if (idx[t] < 0 || idx[t] >= ctx->n - 1)
            return fail(MPS_EINVAL, "mps_apply_layer: bond %d out of range", (int)idx[t]);
        if (t > 0 && idx[t] < idx[t - 1] + 2)
            return fail(MPS_EINVAL, "mps_apply_layer: bonds must be disjoint and increasing");
        if (!gate_finite(g + 32 * t)) return fail(MPS_ENUMERIC, "mps_apply_layer: non-finite gate entry");
    }
    if (n == 0) return MPS_OK;
    s = ctx->prec == MPS_FP64 ? ctx_run_gates<double2>(ctx, n, idx, g, info) : ctx_run_gates<float2>(ctx, n, idx, g, info);
    if (s == MPS_EDEVICE || s == MPS_ENUMERIC) ctx->poisoned = true;
    return s;
}

template <typename T>
static mps_status ctx_amplitude(mps_ctx* c, const uint8_t* bits, double* out)
{
    double2 one = make_double2(1.0, 0.0);
    HIPCHK(hipMemcpyAsync(c->vec0, &one, sizeof(one), hipMemcpyHostToDevice, c->st), "amplitude init");
    double2* v = c->vec0;
    double2* wv = c->vec1;
    for (int j = 0; j < c->n; ++j) {
        const int64_t chl = c->dims[j], chr = c->dims[j + 1];
        const T* S = (const T*)c->site[j] + chl * bits[j];
        hipLaunchKernelGGL((k_vecmat<T>), dim3((unsigned)chr), dim3(256), 0, c->st, (const double2*)v, S, 2 * chl,
                           chl, chr, wv);
        double2* t = v;
        v = wv;
        wv = t;
    }
    double2 res;
    HIPCHK(hipMemcpyAsync(&res, v, sizeof(res), hipMemcpyDeviceToHost, c->st), "amplitude readback");
    HIPCHK(hipStreamSynchronize(c->st), "amplitude sync");
    const double s = exp(0.5 * c->log_fid);
    out[0] = res.x * s;
    out[1] = res.y * s;
    return MPS_OK;
}

extern "C" mps_status mps_amplitude(mps_ctx* ctx, const uint8_t* bits, double* out)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (!bits || !out) return fail(MPS_EINVAL, "mps_amplitude: NULL argument");
    for (int j = 0; j < ctx->n; ++j)
        if (bits[j] > 1) return fail(MPS_EINVAL, "mps_amplitude: bit %d is not 0/1", j);
    s = ctx->prec == MPS_FP64 ? ctx_amplitude<double2>(ctx, bits, out) : ctx_amplitude<float2>(ctx, bits, out);
    if (s == MPS_EDEVICE) ctx->poisoned = true;
    return s;
}

extern "C" mps_status mps_log_norm_fidelity(const mps_ctx* ctx, double* out)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (!out) return fail(MPS_EINVAL, "mps_log_norm_fidelity: NULL out");
    *out = ctx->log_fid;
    return MPS_OK;
}

extern "C" mps_status mps_bond_dims(const mps_ctx* ctx, int64_t* dims)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (!dims) return fail(MPS_EINVAL, "mps_bond_dims: NULL out");
    for (int b = 0; b <= ctx->n; ++b) dims[b] = ctx->dims[b];
    return MPS_OK;
}

extern "C" mps_status mps_centre(const mps_ctx* ctx, int32_t* out)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (!out) return fail(MPS_EINVAL, "mps_centre: NULL out");
    *out = ctx->centre;
    return MPS_OK;
}

extern "C" mps_status mps_get_site(mps_ctx* ctx, int32_t j, void* dst, int64_t dst_bytes)
{
    mps_status s = ctx_check(ctx);
    if (s != MPS_OK) return s;
    if (j < 0 || j >= ctx->n) return fail(MPS_EINVAL, "mps_get_site: site %d out of range", (int)j);
    const int64_t bytes = ctx->dims[j] * 2 * ctx->dims[j + 1] * elem_bytes(ctx->prec);
    if (!dst || dst_bytes < bytes) return fail(MPS_EINVAL, "mps_get_site: need %lld bytes", (long long)bytes);
    HIPCHK(hipMemcpyAsync(dst, ctx->site[j], bytes, hipMemcpyDeviceToDevice, ctx->st), "mps_get_site copy");
    HIPCHK(hipStreamSynchronize(ctx->st), "mps_get_site sync");
    return MPS_OK;
}

// ---------------------------------------------------------------------------
// Stateless centre move on explicit sites (Sec. III-C.1), the operation a
// context performs before an update whose bond is away from the centre.
// ---------------------------------------------------------------------------
template <typename T>
static int64_t move_ws_bytes_t(int64_t chi_l, int64_t chi_c, int64_t chi_r, int direction)
{
    const int64_t m = direction > 0 ? 2 * chi_l : 2 * chi_r, n = chi_c;
    const int64_t k = m < n ? m : n;
    Carver cv{nullptr, (int64_t)1 << 62, 0};
    UpdateWs<T> w;
    carve_update_ws<T>(cv, w, m, n, k, true);
    cv.take((int64_t)sizeof(T) * k * n);        // R
    if (direction < 0) cv.take((int64_t)sizeof(T) * m * k);   // Q' before its conjugate transpose
    return cv.used + 256;
}

extern "C" int64_t mps_move_work_bytes(int64_t chi_l, int64_t chi_c, int64_t chi_r, mps_precision prec,
                                       int32_t direction)
{
    if (chi_l < 1 || chi_c < 1 || chi_r < 1 || !valid_prec(prec) || (direction != 1 && direction != -1)) return -1;
    return prec == MPS_FP64 ? move_ws_bytes_t<double2>(chi_l, chi_c, chi_r, direction)
                            : move_ws_bytes_t<float2>(chi_l, chi_c, chi_r, direction);
}

template <typename T>
static mps_status move_impl(int64_t chi_l, int64_t chi_c, int64_t chi_r, int direction, const T* A, const T* B,
                            T* A_out, T* B_out, int64_t* k_out, void* work, int64_t work_bytes, hipStream_t st)
{
    const int64_t m = direction > 0 ? 2 * chi_l : 2 * chi_r, n = chi_c;
    const int64_t k = m < n ? m : n;
    Carver cv{(char*)work, work_bytes, 0};
    UpdateWs<T> probe;
    if (!carve_update_ws<T>(cv, probe, m, n, k, true)) return fail(MPS_ENOMEM, "mps_move_centre: work too small");
    const int64_t ws_used = cv.used;
    T* R = (T*)cv.take((int64_t)sizeof(T) * k * n);
    T* Qt = direction < 0 ? (T*)cv.take((int64_t)sizeof(T) * m * k) : nullptr;
    if (!R || (direction < 0 && !Qt)) return fail(MPS_ENOMEM, "mps_move_centre: work too small");
    int64_t kk = 0;
    mps_status s;
    if (direction > 0) {
        // A (2 chi_l x chi_c) = Q R;  A_out = Q, B_out = R B
        s = move_qr<T>((char*)work, ws_used, st, A, m, n, false, m, A_out, m, R, &kk);
        if (s != MPS_OK) return s;
        if (!zgemm<T>(st, OP_N, false, OP_N, false, k, 2 * chi_r, chi_c, C_ONE, (const T*)R, k, B, chi_c, C_ZERO,
                      B_out, k, nullptr, 0))
            return fail(MPS_EINVAL, "mps_move_centre: gemm form unavailable");
    } else {
        // B (chi_c x 2 chi_r): B^H = Q' R', B = R'^H Q'^H;  B_out = Q'^H, A_out = A R'^H
        s = move_qr<T>((char*)work, ws_used, st, B, m, n, true, chi_c, Qt, m, R, &kk);
        if (s != MPS_OK) return s;
        dim3 grid((unsigned)rup(m, 32), (unsigned)rup(k, 32));
        hipLaunchKernelGGL((k_conj_transpose<T>), grid, dim3(256), 0, st, (const T*)Qt, m, m, k, B_out, k);
        if (!zgemm<T>(st, OP_N, false, OP_C, false, 2 * chi_l, k, chi_c, C_ONE, A, 2 * chi_l, (const T*)R, k, C_ZERO,
                      A_out, 2 * chi_l, nullptr, 0))
            return fail(MPS_EINVAL, "mps_move_centre: gemm form unavailable");
    }
    HIPCHK(hipGetLastError(), "mps_move_centre launch");
    HIPCHK(hipStreamSynchronize(st), "mps_move_centre sync");
    if (k_out) *k_out = kk;
    return MPS_OK;
}

extern "C" mps_status mps_move_centre(int64_t chi_l, int64_t chi_c, int64_t chi_r, mps_precision prec,
                                      int32_t direction, const void* A, const void* B, void* A_out, void* B_out,
                                      int64_t* k_out, void* work, int64_t work_bytes, void* hip_stream)
{
    if (chi_l < 1 || chi_c < 1 || chi_r < 1) return fail(MPS_EINVAL, "mps_move_centre: dimensions must be >= 1");
    if (chi_l > (1 << 19) || chi_c > (1 << 20) || chi_r > (1 << 19))
        return fail(MPS_EINVAL, "mps_move_centre: dimension too large");
    if (!valid_prec(prec)) return fail(MPS_EINVAL, "mps_move_centre: bad precision %d", (int)prec);
    if (direction != 1 && direction != -1) return fail(MPS_EINVAL, "mps_move_centre: direction must be +1 or -1");
    if (!A || !B || !A_out || !B_out || !work) return fail(MPS_EINVAL, "mps_move_centre: null pointer");
    const int64_t need = mps_move_work_bytes(chi_l, chi_c, chi_r, prec, direction);
    if (work_bytes < need)
        return fail(MPS_ENOMEM, "mps_move_centre: need %lld work bytes, got %lld", (long long)need,
                    (long long)work_bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == MPS_FP64)
        return move_impl<double2>(chi_l, chi_c, chi_r, direction, (const double2*)A, (const double2*)B,
                                  (double2*)A_out, (double2*)B_out, k_out, work, work_bytes, st);
    return move_impl<float2>(chi_l, chi_c, chi_r, direction, (const float2*)A, (const float2*)B, (float2*)A_out,
                             (float2*)B_out, k_out, work, work_bytes, st);
}
