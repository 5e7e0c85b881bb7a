// Autotuner of the pivoted-QR tiles per bond bucket (included at the end of
// abi.hip).  A layer of a circuit holds updates of very different sizes (bond
// dimensions from 2 to the cap); the panel width nb and the candidate-window
// width W that make the pivoted QR fastest differ between them.  For each
// bucket chi = 128, 256, ... the tuner times one synthetic two-site update
// (chi_l = chi_m = chi_r = chi) per candidate pair (nb, W) on the caller's
// stream and keeps the fastest; later factorisations look their tiles up by
// their column count.  The pivots do not depend on the tiles (a window panel
// keeps only the steps the full greedy search would take), so tuning changes
// speed only.

// B[r, :] *= exp(-r / scale): the middle bond of the synthetic pair carries a
// decaying spectrum, as the headline workload's does.
template <typename T>
__global__ __launch_bounds__(256) void k_scale_rows(T* B, int64_t rows, int64_t cols, double scale)
{
    const int64_t total = rows * cols;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
        const int64_t r = q % rows;
        B[q] = from_d<T>(cscale(to_d(B[q]), exp(-(double)r / scale)));
    }
}

#define TUNE_MAX_BUCKETS 8
static const int g_tune_cands[][2] = {{16, 128}, {16, 256}, {32, 128}, {32, 256}, {32, 512}, {64, 256}, {64, 512},
                                      {32, 0}};
#define TUNE_NCANDS ((int)(sizeof(g_tune_cands) / sizeof(g_tune_cands[0])))

static int64_t tune_layout(int32_t chi, mps_precision prec, int64_t* off_b, int64_t* off_ao, int64_t* off_bo,
                           int64_t* off_ws)
{
    const int64_t eb = elem_bytes(prec), c = chi;
    const int64_t site = (2 * c * c * eb + 255) / 256 * 256;
    *off_b = site;
    *off_ao = 2 * site;
    *off_bo = 3 * site;
    *off_ws = 4 * site;
    return 4 * site + mps_update_work_bytes(c, c, c, c, prec, MPS_PIVOT_QRCP);
}

extern "C" int64_t mps_autotune_work_bytes(int32_t chi_max, mps_precision prec)
{
    if (chi_max < 128 || chi_max > 8192 || !valid_prec(prec)) return -1;
    int32_t chi = 128;
    while (chi * 2 <= chi_max) chi *= 2;
    int64_t b, ao, bo, ws;
    return tune_layout(chi, prec, &b, &ao, &bo, &ws);
}

template <typename T>
static mps_status tune_bucket(int32_t chi, mps_precision prec, char* work, int64_t work_bytes, hipStream_t st,
                              mps_tune_entry* e)
{
    int64_t ob, oao, obo, ows;
    tune_layout(chi, prec, &ob, &oao, &obo, &ows);
    T* A = (T*)work;
    T* B = (T*)(work + ob);
    T* Ao = (T*)(work + oao);
    T* Bo = (T*)(work + obo);
    const int64_t c = chi;
    const unsigned blocks = (unsigned)(rup(2 * c * c, 256) < 4096 ? rup(2 * c * c, 256) : 4096);
    hipLaunchKernelGGL((k_sketch_omega<T>), dim3(blocks), dim3(256), 0, st, A, 2 * c, c, (uint64_t)(977 + chi));
    hipLaunchKernelGGL((k_sketch_omega<T>), dim3(blocks), dim3(256), 0, st, B, c, 2 * c, (uint64_t)(1977 + chi));
    hipLaunchKernelGGL((k_scale_rows<T>), dim3(blocks), dim3(256), 0, st, B, c, 2 * c, 150.0 * (double)chi / 1024.0);
    HIPCHK(hipGetLastError(), "autotune inputs");
    static const double gate[32] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0.7071067811865476, 0, 0, 0, 0.7071067811865476,
                                    0, 0, 0, 0.7071067811865476, 0, 0, 0, -0.7071067811865476, 0, 0, 0, 0, 0, 0, 1, 0};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "autotune event");
    HIPCHK(hipEventCreate(&e1), "autotune event");
    const int save_nb = g_panel_width, save_win = g_qr_window;
    double best = 1e300, def = -1.0;
    int best_nb = 32, best_win = QR_WIN_DEFAULT;
    mps_status s = MPS_OK;
    for (int q = 0; q < TUNE_NCANDS && s == MPS_OK; ++q) {
        g_panel_width = g_tune_cands[q][0];
        g_qr_window = g_tune_cands[q][1];
        float ms = 0.0f, tot = 0.0f;
        for (int rep = 0; rep < 3 && s == MPS_OK; ++rep) {   // one warm-up, two timed
            if (hipEventRecord(e0, st) != hipSuccess) {
                s = fail(MPS_EDEVICE, "autotune: event record failed");
                break;
            }
            s = update_core<T>(c, c, c, c, prec, A, B, gate, Ao, Bo, 1, nullptr, nullptr, work + ows,
                               work_bytes - ows, st);
            if (s != MPS_OK) break;
            if (hipEventRecord(e1, st) != hipSuccess) {
                s = fail(MPS_EDEVICE, "autotune: event record failed");
                break;
            }
            if (hipEventSynchronize(e1) != hipSuccess) {
                s = fail(MPS_EDEVICE, "autotune: event synchronisation failed");
                break;
            }
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                s = fail(MPS_EDEVICE, "autotune: event timing failed");
                break;
            }
            if (rep > 0) tot += ms;
        }
        const double t = tot / 2.0;
        if (s == MPS_OK && t < best) {
            best = t;
            best_nb = g_tune_cands[q][0];
            best_win = g_tune_cands[q][1];
        }
        if (g_tune_cands[q][0] == 32 && g_tune_cands[q][1] == QR_WIN_DEFAULT) def = t;
    }
    g_panel_width = save_nb;
    g_qr_window = save_win;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != MPS_OK) return s;
    e->n_max = 0;
    e->panel_width = best_nb;
    e->qr_window = best_win;
    e->ms = best;
    e->ms_default = def;
    return MPS_OK;
}

extern "C" mps_status mps_autotune(int32_t chi_max, mps_precision prec, void* work, int64_t work_bytes,
                                   void* hip_stream, mps_tune_entry* table, int32_t max_entries, int32_t* n_entries)
{
    if (chi_max < 128 || chi_max > 8192) return fail(MPS_EINVAL, "mps_autotune: chi_max %d not in [128, 8192]", chi_max);
    if (!valid_prec(prec)) return fail(MPS_EINVAL, "mps_autotune: bad precision %d", (int)prec);
    if (!work || !table || max_entries < 1) return fail(MPS_EINVAL, "mps_autotune: null pointer or no room");
    const int64_t need = mps_autotune_work_bytes(chi_max, prec);
    if (work_bytes < need)
        return fail(MPS_ENOMEM, "mps_autotune: need %lld work bytes, got %lld", (long long)need, (long long)work_bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<mps_tune_entry> found;
    for (int32_t chi = 128; chi <= chi_max && (int)found.size() < max_entries && (int)found.size() < TUNE_MAX_BUCKETS;
         chi *= 2) {
        mps_tune_entry e;
        mps_status s = prec == MPS_FP64 ? tune_bucket<double2>(chi, prec, (char*)work, work_bytes, st, &e)
                                        : tune_bucket<float2>(chi, prec, (char*)work, work_bytes, st, &e);
        if (s != MPS_OK) return s;
        // the bucket covers column counts up to the geometric midpoint to the next one
        e.n_max = (int64_t)(2.0 * chi * 1.41421356237);
        found.push_back(e);
    }
    if (!found.empty()) found.back().n_max = (int64_t)1 << 40;
    g_tune.assign(found.begin(), found.end());
    for (size_t q = 0; q < found.size(); ++q) table[q] = found[q];
    if (n_entries) *n_entries = (int32_t)found.size();
    return MPS_OK;
}

extern "C" mps_status mps_clear_autotune(void)
{
    g_tune.clear();
    return MPS_OK;
}
