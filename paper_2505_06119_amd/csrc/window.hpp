// Candidate-window panels for the delayed-update QRCP.
//
// The pivot sequence of column-pivoted QR is decided by greedy argmax steps
// over the downdated residual column norms.  Over the next nb steps, the
// greedy choices almost always come from the few hundred columns with the
// largest residual norms at the start of the panel.  A window panel exploits
// this while computing exactly the greedy factorisation:
//
//   1. select     the W columns with the largest residual norms (ties: smaller
//                 original index first, the argmax order) and swap them to
//                 positions p0 .. p0+W-1; keep a copy of that state;
//   2. factorise  up to nb pivot steps with the per-step kernels, restricted
//                 to the window: the per-step GEMV reads m x W instead of the
//                 whole trailing block;
//   3. verify     apply the panel's block reflector to the columns outside the
//                 window only as far as needed for their R rows
//                     W_o = V^H A_o,  W2 = T^H W_o,  R12 = A_o[p0:j, :] - V_top W2
//                 and replay the greedy test for every step t: the outside
//                 column's norm before step t (downdated by R12 rows 0..t-1)
//                 must lose against the window's pivot of that step, and must
//                 not fall under the recomputation threshold before it;
//   4. accept     t* = the first step that fails (or nb): when t* < nb the
//                 window state is restored and exactly t* steps are redone
//                 (the kernels are deterministic, so these are the same
//                 steps), then the outside columns receive the block update
//                 A_o -= V W2 with the first t* reflectors and the window's
//                 remaining columns the usual V F^H update.
//
// Every accepted step is therefore the step the full greedy search would have
// taken on the same downdated norms; only the HBM traffic changes: the
// trailing block is read once and written once per panel (two GEMMs) instead
// of read once per pivot step.
#pragma once
#include "qrcp.hpp"

#define WIN_SORT_MAX 8192   // remaining columns the one-block selection handles
#define QR_WIN_MAX 512      // largest window (workspace for the saved state)

// Exclusive prefix count of `flag` over the threads of a 1024-thread block;
// *total receives the block total.  `wsum` is LDS scratch of 16 ints.
__device__ __forceinline__ int block_scan_flags1024(bool flag, int* wsum, int* total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(flag);
    const int inwave = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inwave;
}

// Exclusive prefix sum of v over the threads of a 1024-thread block; *total
// receives the block total.  `wsum` is LDS scratch of 16 ints.
__device__ __forceinline__ int block_scan_counts1024(int v, int* wsum, int* total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, MPS_WAVE);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// Step 1a (one block of 1024 threads): choose the window among the remaining
// columns [p0, n) -- the W largest residual norms, found by a radix select
// on the norms' bit patterns (non-negative doubles order like their bits),
// equal norms at the threshold taken in column order -- and write the swap
// plan that brings them to [p0, p0+W): plan[0] = number of pairs, then pairs
// (a, b) of column positions to exchange, then from plan[1 + 2W] one entry
// per window slot: the position of the column that moves into it, or -1.  The first pivot (largest norm,
// smallest key on ties) is always in the window; its argmax partial for the
// post-swap positions goes to cpart[0], cflag[0].
// Requires W <= 1024, W < n - p0 <= WIN_SORT_MAX.
template <typename T>
__global__ __launch_bounds__(1024) void k_window_select(QrcpDev<T> d, int64_t p0, int W, int32_t* plan,
                                                        ArgBest* wcp)
{
    __shared__ uint64_t s_b[WIN_SORT_MAX];   // norm bits
    __shared__ int32_t s_key[WIN_SORT_MAX];
    __shared__ uint8_t s_in[WIN_SORT_MAX];
    __shared__ int32_t s_win[1024];           // window entries (column offsets), in column order
    __shared__ int32_t s_d[1024];
    __shared__ uint32_t s_hist[256];
    __shared__ int wsum[16];
    __shared__ int s_sel[4];                  // chosen digit, count still needed, done flag
    __shared__ ArgBest s_best[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int L = (int)(d.n - p0);
    constexpr int PER = WIN_SORT_MAX / 1024;

    // load; global argmax (larger norm, then smaller key) on the way
    ArgBest best;
    best.val = -1.0;
    best.key = 0x7fffffff;
    best.slot = -1;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int q = tid + 1024 * u;
        if (q < L) {
            const double v = d.nu[p0 + q];
            const int32_t key = d.perm[p0 + q];
            s_b[q] = (uint64_t)__double_as_longlong(v > 0.0 ? v : 0.0);
            s_key[q] = key;
            if (arg_better(v, key, best.val, best.key)) {
                best.val = v;
                best.key = key;
                best.slot = q;
            }
        }
        s_in[q] = 0;
    }
    best = wave_argmax(best);
    if (lane == 0) s_best[wid] = best;

    // radix select of the W-th largest bit pattern, 8 bits per pass from the top
    uint64_t prefix = 0, mask = 0;
    int need = W;
    bool all_in = false;
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (tid < 256) s_hist[tid] = 0;
        __syncthreads();
        // Norms of similar size share the top digits, so most entries of a
        // pass land in one bin.  Each thread first merges runs of equal digits
        // among its entries; when every lane of a wave holds a single run of
        // one digit, the wave adds its total with one atomic instead of 64.
        uint32_t run_d = 0xffffffffu, run_c = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = tid + 1024 * u;
            if (q < L && (s_b[q] & mask) == prefix) {
                const uint32_t dg = (uint32_t)(s_b[q] >> shift) & 255u;
                if (dg == run_d) {
                    ++run_c;
                } else {
                    if (run_c) atomicAdd(&s_hist[run_d], run_c);
                    run_d = dg;
                    run_c = 1;
                }
            }
        }
        {
            const uint32_t d0 = (uint32_t)__shfl((int)run_d, 0, MPS_WAVE);
            if (__all(run_c == 0 || run_d == d0)) {
                uint32_t tot = run_c;
                for (int off = 32; off > 0; off >>= 1) tot += (uint32_t)__shfl_xor((int)tot, off, MPS_WAVE);
                if (lane == 0 && tot) atomicAdd(&s_hist[d0], tot);
            } else if (run_c) {
                atomicAdd(&s_hist[run_d], run_c);
            }
        }
        __syncthreads();
        if (tid < 64) {
            // wave 0: lane l holds bins 255-4l .. 252-4l (descending); the bin
            // where the count from the top reaches `need` is found with one
            // exclusive scan over the lanes
            const int lane = tid;
            int h[4], own = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                h[u] = (int)s_hist[255 - 4 * lane - u];
                own += h[u];
            }
            int incl = own;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off, MPS_WAVE);
                if (lane >= off) incl += t;
            }
            int cum = incl - own;   // count in bins above this lane's
            const bool here = cum < need && incl >= need;
            if (here) {
                int dig = 0, before = cum;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (before + h[u] >= need) {
                        dig = 255 - 4 * lane - u;
                        break;
                    }
                    before += h[u];
                }
                s_sel[0] = dig;
                s_sel[1] = need - before;                               // still needed from this bin
                s_sel[2] = (int)s_hist[dig] == need - before ? 1 : 0;   // the whole bin is taken
            }
        }
        __syncthreads();
        prefix |= (uint64_t)s_sel[0] << shift;
        mask |= (uint64_t)255 << shift;
        need = s_sel[1];
        all_in = s_sel[2] != 0;
        __syncthreads();
        if (all_in) break;
    }
    // membership: above the threshold prefix, or at it (all of them when the
    // bin was taken whole, else the first `need` in column order).  Here each
    // thread owns PER consecutive columns, so one block scan of the per-thread
    // counts ranks every column at the threshold in column order.
    {
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = PER * tid + u;
            cnt += (q < L && (s_b[q] & mask) == prefix) ? 1 : 0;
        }
        int tot = 0;
        int rank = block_scan_counts1024(cnt, wsum, &tot);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = PER * tid + u;
            const bool valid = q < L;
            const uint64_t hb = valid ? (s_b[q] & mask) : 0;
            const bool above = valid && hb > prefix;
            const bool at = valid && hb == prefix;
            const bool take = above || (at && (all_in || rank < need));
            rank += at ? 1 : 0;
            if (take) s_in[q] = 1;
        }
    }
    __syncthreads();
    // the global argmax must be in the window (it is, unless ties at the threshold left it out)
    if (tid == 0) {
        ArgBest b = s_best[0];
        for (int w = 1; w < 16; ++w)
            if (arg_better(s_best[w].val, s_best[w].key, b.val, b.key)) b = s_best[w];
        s_best[0] = b;
        s_sel[3] = s_in[b.slot] ? -1 : b.slot;
    }
    __syncthreads();
    // compact the window in column order (one scan of per-thread member counts)
    {
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = PER * tid + u;
            cnt += (q < L && s_in[q]) ? 1 : 0;
        }
        int tot = 0;
        int base = block_scan_counts1024(cnt, wsum, &tot);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = PER * tid + u;
            if (q < L && s_in[q]) {
                if (base < W) s_win[base] = q;
                ++base;
            }
        }
    }
    __syncthreads();
    if (tid == 0 && s_sel[3] >= 0) {
        // replace the last member by the argmax (ties at the threshold only)
        s_in[s_win[W - 1]] = 0;
        s_win[W - 1] = s_sel[3];
        s_in[s_sel[3]] = 1;
    }
    __syncthreads();
    const int qe = tid < W ? s_win[tid] : 0;   // window entry -> column offset
    // displaced positions inside [0, W) and window columns outside it, paired in order
    int nd = 0, nv = 0;
    const bool disp = tid < W && !s_in[tid];
    const int id = block_scan_flags1024(disp, wsum, &nd);
    if (disp) s_d[id] = tid;
    const bool vac = tid < W && qe >= W;
    const int iv = block_scan_flags1024(vac, wsum, &nv);
    __syncthreads();
    if (vac) {
        plan[1 + 2 * iv] = (int32_t)(p0 + s_d[iv]);
        plan[2 + 2 * iv] = (int32_t)(p0 + qe);
        plan[1 + 2 * W + s_d[iv]] = (int32_t)(p0 + qe);   // the slot's incoming column
    }
    if (tid < W && !disp) plan[1 + 2 * W + tid] = -1;      // slot already holds a window column
    const ArgBest b0 = s_best[0];
    if (tid == 0) plan[0] = nv;
    // first partial: the argmax, at its post-swap position; and one partial per
    // window column (post-swap position p0 + b in wcp[b]) for the window steps
    if (tid < W) {
        const int64_t pos = p0 + (vac ? s_d[iv] : qe);
        ArgBest b;
        b.val = __longlong_as_double((long long)s_b[qe]);
        b.key = s_key[qe];
        b.slot = (int32_t)pos;
        wcp[pos - p0] = b;
        if (qe == b0.slot) {
            d.cpart[0] = b;
            d.cflag[0] = 0;
        }
    }
}

// Step 1b (block q = window slot p0 + q): carry out the plan -- a slot with an
// incoming column b exchanges all m rows, norm, reference norm and key with
// it -- and, with save, keep a copy of the slot's new column (wsave[:, q], ld
// lds) and of its norms and key (snu, snuref, sperm).  grid: W blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_window_place(QrcpDev<T> d, int64_t p0, int W, const int32_t* plan, T* wsave,
                                                      int64_t lds, double* snu, double* snuref, int32_t* sperm,
                                                      int save)
{
    const int q = blockIdx.x;
    const int64_t a = p0 + q, b = plan[1 + 2 * W + q];
    if (b < 0 && !save) return;   // nothing moves into this slot
    T* ca = d.A + d.lda * a;
    T* cb = d.A + d.lda * (b >= 0 ? b : a);
    T* cs = wsave + lds * q;
    for (int64_t i0 = threadIdx.x; i0 < d.m; i0 += 256 * 8) {
        T x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + 256 * u;
            const int64_t ic = i < d.m ? i : d.m - 1;
            x[u] = ca[ic];
            y[u] = cb[ic];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + 256 * u;
            if (i < d.m) {
                if (b >= 0) {
                    ca[i] = y[u];
                    cb[i] = x[u];
                }
                if (save) cs[i] = b >= 0 ? y[u] : x[u];
            }
        }
    }
    if (threadIdx.x == 0) {
        if (b >= 0) {
            const double t0 = d.nu[a]; d.nu[a] = d.nu[b]; d.nu[b] = t0;
            const double t1 = d.nuref[a]; d.nuref[a] = d.nuref[b]; d.nuref[b] = t1;
            const int32_t t2 = d.perm[a]; d.perm[a] = d.perm[b]; d.perm[b] = t2;
        }
        if (save) {
            snu[q] = d.nu[a];
            snuref[q] = d.nuref[a];
            sperm[q] = d.perm[a];
        }
    }
}

// Copy the window's norms and keys to (dir = 0) or from (dir = 1) the save area.
template <typename T>
__global__ __launch_bounds__(256) void k_window_meta(QrcpDev<T> d, int64_t p0, int W, double* snu, double* snuref,
                                                     int32_t* sperm, int dir)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= W) return;
    if (dir == 0) {
        snu[q] = d.nu[p0 + q];
        snuref[q] = d.nuref[p0 + q];
        sperm[q] = d.perm[p0 + q];
    } else {
        d.nu[p0 + q] = snu[q];
        d.nuref[p0 + q] = snuref[q];
        d.perm[p0 + q] = sperm[q];
    }
}

// Step 3: greedy replay for the columns [c0, c0 + nout) outside the window.
// R12 (nbe x nout, leading dimension ldr) holds their R rows of the panel.
// ctl[CTL_TFAIL] = first failing step, ctl[CTL_TFLAG] = first step after which
// a norm falls under the recomputation threshold, plus one (nbe+1 when none):
// minima over the columns, per block by shuffles, across blocks by atomic
// minimum on values k_ctl_panel set to INT_MAX.  One thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_window_check(QrcpDev<T> d, const T* R12, int64_t ldr, int64_t c0,
                                                      int64_t nout, int nbe)
{
    __shared__ int s_min[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t q = (int64_t)blockIdx.x * 256 + tid;
    int tfail = nbe + 1, tflag = nbe + 1;
    if (q < nout) {
        const int64_t c = c0 + q;
        double s = d.nu[c];
        const double lim = d.tol * d.nuref[c];
        const int32_t key = d.perm[c];
        // rows in chunks of 8 loaded ahead (clamped, unconditional), so the
        // early exits do not serialise one load per step
        const T* rq = R12 + ldr * q;
        bool done = false;
        for (int t0 = 0; t0 < nbe && !done; t0 += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = rq[t0 + u < nbe ? t0 + u : nbe - 1];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u;
                if (done || t >= nbe) break;
                const double pv = d.pivval[t];
                if (arg_better(s, key, pv, d.pivkey[t])) {
                    tfail = t;
                    done = true;
                    break;
                }
                double nn = s - cabs2(to_d(v[u]));
                if (nn < 0.0) nn = 0.0;
                if (nn <= lim) {
                    tflag = t + 1;
                    done = true;
                    break;
                }
                s = nn;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        tfail = min(tfail, __shfl_xor(tfail, off, MPS_WAVE));
        tflag = min(tflag, __shfl_xor(tflag, off, MPS_WAVE));
    }
    if (lane == 0) {
        s_min[0][wid] = tfail;
        s_min[1][wid] = tflag;
    }
    __syncthreads();
    if (tid == 0) {
        atomicMin(d.ctl + CTL_TFAIL, min(min(s_min[0][0], s_min[0][1]), min(s_min[0][2], s_min[0][3])));
        atomicMin(d.ctl + CTL_TFLAG, min(min(s_min[1][0], s_min[1][1]), min(s_min[1][2], s_min[1][3])));
    }
}

// Step 4 (no recomputation pending): downdate the outside columns' norms by
// their R rows 0 .. nbe-1 in R12 (the values the replay used), with the
// per-step clamp of the step kernel.  One thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_window_commit(QrcpDev<T> d, const T* R12, int64_t ldr, int64_t c0,
                                                       int64_t nout, int nbe)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nout) return;
    const int64_t c = c0 + q;
    const T* rq = R12 + ldr * q;
    double s = d.nu[c];
    int t = 0;
    for (; t + 8 <= nbe; t += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = rq[t + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double nn = s - cabs2(to_d(v[u]));
            s = nn < 0.0 ? 0.0 : nn;
        }
    }
    for (; t < nbe; ++t) {
        const double nn = s - cabs2(to_d(rq[t]));
        s = nn < 0.0 ? 0.0 : nn;
    }
    d.nu[c] = s;
}

// Argmax partials of the current norms of columns [c0, n) (256 per block),
// for a panel that starts without a preceding step kernel.
template <typename T>
__global__ __launch_bounds__(256) void k_nu_argmax(QrcpDev<T> d, int64_t c0)
{
    __shared__ ArgBest arg_lds[4];
    const int64_t c = c0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    ArgBest b;
    b.val = -1.0;
    b.key = 0x7fffffff;
    b.slot = -1;
    if (c < d.n) {
        b.val = d.nu[c];
        b.key = d.perm[c];
        b.slot = (int32_t)c;
    }
    b = block_argmax256(b, arg_lds);
    if (threadIdx.x == 0) {
        d.cpart[blockIdx.x] = b;
        d.cflag[blockIdx.x] = 0;
    }
}

// ---------------------------------------------------------------------------
// Right-looking pivot step inside a window (one launch per step).  Block b
// owns the window column at position p0 + b and keeps it current: every step
// applies the new reflector to it (H^H a = a - conj(tau) v (v^H a)) and
// recomputes its residual norm exactly, so no norm is downdated inside the
// window.  Columns do not move during the panel: the pivots are recorded in
// wpiv and put in place by k_window_order / k_window_gather at the panel end.
//   cin[b] / cout[b]: the argmax partial of column p0 + b before / after this
//   step (slot -1 once it is a pivot); the two buffers alternate between
//   steps, so no block reads a partial another block of the same launch writes.
// Every block reads all W partials, finds the pivot, loads the pivot column
// (rows j..m, shared through L2) and forms the reflector with the same
// arithmetic as every other block.  The pivot's block stores beta and v in
// vbuf[:, jj] (column p itself is read by all blocks during the step and is
// left as it is).  grid: W blocks of NT threads; requires m - j <= NT * RPT.
// ---------------------------------------------------------------------------
#define WSTEP_NT 512    // threads per block (8 waves)
#define WSTEP_RPT 16    // rows per thread
#define WSTEP_NW (WSTEP_NT / 64)

__device__ __forceinline__ ArgBest e0_dead()
{
    ArgBest z;
    z.val = -1.0;
    z.key = 0x7fffffff;
    z.slot = -1;
    return z;
}

template <int NW>
__device__ __forceinline__ double block_sum_ws(double v, double* lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += lds[w];
    return s;
}

// four block sums in one round
template <int NW>
__device__ __forceinline__ void block_sum_ws4(double& a, double& b, double& c, double& e, double* lds /* 4 * NW */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    e = wave_sum(e);
    __syncthreads();
    if (lane == 0) {
        lds[wid] = a;
        lds[NW + wid] = b;
        lds[2 * NW + wid] = c;
        lds[3 * NW + wid] = e;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0, sc = 0.0, se = 0.0;
    for (int w = 0; w < NW; ++w) {
        sa += lds[w];
        sb += lds[NW + w];
        sc += lds[2 * NW + w];
        se += lds[3 * NW + w];
    }
    a = sa;
    b = sb;
    c = sc;
    e = se;
}

// The new residual norm of a live column comes from the same reduction round
// as the reflector: with c = conj(tau) (v^H a) scale, the rows below the
// pivot become a_i - c x_i, so
//     sum |a_i - c x_i|^2 = sum |a_i|^2 - 2 Re(conj(c) sum conj(x_i) a_i)
//                            + |c|^2 sum |x_i|^2,
// all three sums taken over the stored column and pivot column in FP64.  The
// norm is thus exact for the column as it stood at the step's start, moved
// by one reflector analytically; when that cancels below 1e-6 of sum |a_i|^2
// it is recomputed from the updated column instead (a second reduction).
// NT threads per block with RPT rows each (NT * RPT >= m - j): 512 x 16 for
// the large factorisations, smaller blocks when few rows remain.
template <typename T, int NT = WSTEP_NT, int RPT = WSTEP_RPT>
__global__ __launch_bounds__(NT) void k_window_step(QrcpDev<T> d, int64_t j, int64_t p0, int jj, const ArgBest* cin,
                                                      ArgBest* cout, int32_t* wpiv, T* vbuf, int32_t* wstep, T* gbuf, int ldg)
{
    constexpr int NW = NT / 64;
    __shared__ double s_red[4 * NW];
    __shared__ ArgBest s_arg[NW];
    __shared__ double2 s_alpha, s_aj;
    const int tid = threadIdx.x, lane = tid & 63;
    const int W = gridDim.x, b = blockIdx.x;
    const int64_t c = p0 + b;
    const int m = (int)d.m, j0 = (int)j;   // rows fit 32 bits here
    T* colc = d.A + d.lda * c;
    const int32_t stop = d.ctl[CTL_STOP];

    // independent loads first: the first NT partials (all of them when
    // W <= NT), this block's own partial, this column's rows j.., its key
    const ArgBest e = cin[tid < W ? tid : 0];
    const int32_t own_slot = cin[b].slot;
    const int32_t key_c = d.perm[c];
    T a[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = j0 + tid + NT * q;
        a[q] = colc[i < m ? i : m - 1];
    }
    ArgBest best = e0_dead();
    if (tid < W && e.slot >= 0) best = e;
    for (int t = tid + NT; t < W; t += NT) {   // windows wider than the block
        const ArgBest f = cin[t];
        if (f.slot >= 0 && arg_better(f.val, f.key, best.val, best.key)) best = f;
    }
    best = wave_argmax(best);
    if (lane == 0) s_arg[tid >> 6] = best;
    __syncthreads();
    ArgBest bb = s_arg[0];
    for (int w = 1; w < NW; ++w)
        if (arg_better(s_arg[w].val, s_arg[w].key, bb.val, bb.key)) bb = s_arg[w];
    if (stop || bb.slot < 0) return;   // uniform over the block
    // a dead block is the pivot of an earlier step i of this panel: it forms
    // the Gram entry G[i, jj] = v_i^H v_jj of the panel's reflectors instead
    const bool dead = own_slot < 0;
    const int gi = dead ? wstep[b] : -1;
    if (dead && tid == 0) cout[b] = e0_dead();
    if (dead && (gi < 0 || gi >= jj)) return;
    const int64_t p = bb.slot;

    // the pivot column and its reflector (identical arithmetic in every block)
    T x[RPT];   // kept in the storage type, converted at each use
    const T* colp = d.A + d.lda * p;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = j0 + tid + NT * q;
        x[q] = colp[i < m ? i : m - 1];
    }
    if (gi >= 0) {
        // dead block: v_i (rows j.. of vbuf column i) takes the place of the
        // column, and g = sum_{r>j} conj(v_i[r]) x_r is formed below
        const T* vi = vbuf + d.lda * gi;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = j0 + tid + NT * q;
            a[q] = vi[i < m ? i : m - 1];
        }
    }
    // one reduction round for ||x_rest||^2, g = sum_{i>j} conj(x_i) a_i and
    // ||a_rest||^2; then v^H a = a_j + conj(scale) g with v = (1, scale * x_rest)
    const bool want_norm = gi < 0;
    double rest = 0.0, gre = 0.0, gim = 0.0, sa = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = j0 + tid + NT * q;
        if (i > j0 && i < m) {
            const double2 xi = to_d(x[q]);
            const double2 ai = to_d(a[q]);
            rest += cabs2(xi);
            // live: conj(x) a; dead: conj(v_i) x
            const double2 t = gi >= 0 ? cmulc(ai, xi) : cmulc(xi, ai);
            gre += t.x;
            gim += t.y;
            if (want_norm) sa += cabs2(ai);
        }
    }
    if (tid == 0) {
        s_alpha = to_d(x[0]);
        s_aj = to_d(a[0]);
    }
    block_sum_ws4<NW>(rest, gre, gim, sa, s_red);   // its barriers also publish s_alpha, s_aj
    const double2 alpha = s_alpha;
    double2 tau, scale;
    double beta;
    if (rest == 0.0 && alpha.y == 0.0) {
        tau = czero();
        scale = czero();
        beta = alpha.x;
    } else {
        const double nrm = sqrt(cabs2(alpha) + rest);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        scale = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
    }

    if (gi >= 0) {
        // G[i, jj] = conj(v_i[j]) * 1 + scale * sum_{r>j} conj(v_i[r]) x_r
        if (tid == 0)
            gbuf[gi + ldg * jj] = from_d<T>(cadd(cconj(s_aj), cmul(scale, make_double2(gre, gim))));
        return;
    }
    if (c == p) {
        // this column is the pivot: beta and v go to vbuf[j.., jj]
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = j0 + tid + NT * q;
            if (i == j0) vbuf[i + d.lda * jj] = from_d<T>(make_double2(beta, 0.0));
            else if (i < m) vbuf[i + d.lda * jj] = from_d<T>(cmul(scale, to_d(x[q])));
        }
        if (tid == 0) {
            d.tau[j] = tau;
            d.diagR[j] = beta;
            d.pivval[jj] = bb.val;
            d.pivkey[jj] = bb.key;
            d.ctl[CTL_JDONE] = (int32_t)(j + 1);
            wpiv[jj] = (int32_t)c;
            wstep[b] = jj;
            cout[b] = e0_dead();
        }
        return;
    }

    // w = v^H a, coef = conj(tau) w; the rows below j move by -coef scale x
    const double2 g = make_double2(gre, gim);
    const double2 wv = cadd(s_aj, cmul(cconj(scale), g));
    const double2 coef = cmul(cconj(tau), wv);
    const double2 cs = cmul(coef, scale);
    double nn = sa - 2.0 * (cs.x * g.x + cs.y * g.y) + cabs2(cs) * rest;
    const bool recompute = want_norm && !(nn > 1e-6 * sa);   // uniform: from block-wide sums
    if (tid == 0 && !recompute) {
        ArgBest mine;
        mine.val = nn > 0.0 ? nn : 0.0;
        mine.key = key_c;
        mine.slot = (int32_t)c;
        cout[b] = mine;
        if (want_norm) d.nu[c] = mine.val;
    }
    // a -= conj(tau) v (v^H a)
    double ne = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = j0 + tid + NT * q;
        if (i < m) {
            const double2 vi = i == j0 ? make_double2(1.0, 0.0) : cmul(scale, to_d(x[q]));
            const T an = from_d<T>(csub(to_d(a[q]), cmul(coef, vi)));
            colc[i] = an;
            if (recompute && i > j0) ne += cabs2(to_d(an));
        }
    }
    if (recompute) {
        ne = block_sum_ws<NW>(ne, s_red);
        if (tid == 0) {
            ArgBest mine;
            mine.val = ne;
            mine.key = key_c;
            mine.slot = (int32_t)c;
            cout[b] = mine;
            d.nu[c] = ne;
        }
    }
}

// ---------------------------------------------------------------------------
// Unpivoted panel in column order as one launch (a centre move, or QR with a
// known column order).  Block b owns column p0 + b of the window [p0, p0 + W)
// and keeps its rows p0.. in registers for the whole panel.  Step s belongs
// to block s (s < nsteps): it waits for steps 0 .. s-1, applies each
// reflector to its column as it arrives, forms its own Householder reflector
// (xLARFG convention, FP64), stores the column (R rows above the diagonal,
// the reflected rows from the diagonal on: the x that later blocks read),
// tau, R_ss and the FP64 scale of v, publishes flags[s] = epoch, and only
// then writes beta and v into vbuf[:, s] (read after the launch).  Blocks
// from nsteps on apply all nsteps reflectors and store their column.  Each
// reflector reaches a column with the arithmetic of a right-looking step:
// w = a_j + conj(scale) x^H a over the rows below j, a -= conj(tau) w v with
// v = (1, scale x).
//
// Block b only ever waits for blocks below b.  Workgroups are dispatched in
// index order, so the lowest unfinished block always runs and the panel
// makes progress whatever the number of resident blocks.  Each wait is
// bounded all the same: a wait that runs out (which correct operation never
// reaches) poisons the block's column and the factorisation's epsilon with
// NaN instead of hanging, so the caller's finiteness checks report it.
// Publication: every thread of the pivot block fences its stores at agent
// scope (the L2s of the chip's dies are not coherent with one another),
// then one thread stores the flag with release semantics; a waiting block's
// thread 0 reads the flag and fences with acquire semantics before the
// block barrier that releases its other threads to read the column.
// flags[] must hold values other than epoch when the panel starts.
// ---------------------------------------------------------------------------
#define FIXED_WAIT_LIMIT (1 << 20)   // polls of one flag (about a second): far beyond any panel

template <int NW>
__device__ __forceinline__ void block_sum_ws2(double& a, double& b, double* lds /* 2 * NW */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane == 0) {
        lds[wid] = a;
        lds[NW + wid] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < NW; ++w) {
        sa += lds[w];
        sb += lds[NW + w];
    }
    a = sa;
    b = sb;
}

// A double2 written by another block of the running kernel: two relaxed
// agent-scope atomic loads, so the compiler cannot serve it from the scalar
// cache (which the acquire fence does not make coherent).
__device__ __forceinline__ double2 ld_published(const double2* p)
{
    const double* q = (const double*)p;
    return make_double2(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

template <typename T, int NT, int RPT>
__global__ __launch_bounds__(NT) void k_fixed_panel(QrcpDev<T> d, int64_t p0, int nsteps, int32_t epoch,
                                                     int32_t* flags, double2* vscale, int32_t* wpiv, T* vbuf)
{
    constexpr int NW = NT / 64;
    __shared__ double s_red[2 * NW];
    __shared__ double2 s_aj;
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int64_t c = p0 + b;
    const int m = (int)d.m, r0 = (int)p0;   // rows fit 32 bits here
    const T zero = from_d<T>(czero());
    T* colc = d.A + d.lda * c;
    T a[RPT];   // rows r0 + tid + NT q; zeros past the matrix
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = r0 + tid + NT * q;
        const T v = colc[i < m ? i : m - 1];
        a[q] = i < m ? v : zero;
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    const int nref = b < nsteps ? b : nsteps;
    for (int s = 0; s < nref; ++s) {
        const int js = r0 + s;
        if (tid == 0) {
            int it = 0;
            while (__hip_atomic_load(flags + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                if (++it >= FIXED_WAIT_LIMIT) {
                    s_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (s_fail) break;   // uniform: read after the barrier
        // x: the rows of column p0 + s below js (zeros elsewhere)
        const T* xs = d.A + d.lda * (p0 + s);
        T x[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = r0 + tid + NT * q;
            const T v = xs[i < m ? i : m - 1];
            x[q] = (i > js && i < m) ? v : zero;
        }
        const double2 sc = ld_published(vscale + s);
        const double2 tau = ld_published(d.tau + js);
        if (tid == s) s_aj = to_d(a[0]);   // row js of this column
        double gre = 0.0, gim = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const double2 g = cmulc(to_d(x[q]), to_d(a[q]));
            gre += g.x;
            gim += g.y;
        }
        block_sum_ws2<NW>(gre, gim, s_red);   // its barriers also publish s_aj
        const double2 wv = cadd(s_aj, cmul(cconj(sc), make_double2(gre, gim)));
        const double2 coef = cmul(cconj(tau), wv);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            double2 vi = cmul(sc, to_d(x[q]));
            if (q == 0 && tid == s) vi = make_double2(1.0, 0.0);
            a[q] = from_d<T>(csub(to_d(a[q]), cmul(coef, vi)));
        }
        __syncthreads();   // s_aj is rewritten by the next step
    }
    if (s_fail) {
        const T bad = from_d<T>(make_double2(__builtin_nan(""), 0.0));
#pragma unroll
        for (int q = 0; q < RPT; ++q) a[q] = bad;
        if (tid == 0) d.dsc[DSC_EPS2] = __builtin_nan("");
    }
    if (b >= nsteps) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = r0 + tid + NT * q;
            if (i < m) colc[i] = a[q];
        }
        return;
    }
    // this block's own step: reflector of rows jb.. of its column
    const int jb = r0 + b;
    if (tid == b) s_aj = to_d(a[0]);
    double rest = 0.0, dummy = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        double2 ai = to_d(a[q]);
        if (q == 0 && tid <= b) ai = czero();
        rest += cabs2(ai);
    }
    block_sum_ws2<NW>(rest, dummy, s_red);
    const double2 alpha = s_aj;
    double2 tau, scale;
    double beta;
    if (rest == 0.0 && alpha.y == 0.0) {
        tau = czero();
        scale = czero();
        beta = alpha.x;
    } else {
        const double nrm = sqrt(cabs2(alpha) + rest);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        scale = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
    }
    // what the later blocks read first (the column, its scalars), then the
    // flag; beta and v are read only after the launch
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = r0 + tid + NT * q;
        if (i < m) colc[i] = a[q];
    }
    if (tid == 0) {
        d.tau[jb] = tau;
        d.diagR[jb] = beta;
        vscale[b] = scale;
        wpiv[b] = (int32_t)c;
        if (b == nsteps - 1) d.ctl[CTL_JDONE] = r0 + nsteps;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flags + b, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    T* vb = vbuf + d.lda * b;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = r0 + tid + NT * q;
        if (i == jb) vb[i] = from_d<T>(make_double2(beta, 0.0));
        else if (i > jb && i < m) vb[i] = from_d<T>(cmul(scale, to_d(a[q])));
    }
}

// flags of k_fixed_panel set to a value no panel uses (epochs are p0 + 1 >= 1)
__global__ void k_fixed_flags_reset(int32_t* flags, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = 0;
}

// First partials of a pivoted panel whose window is every remaining column
// (one per column, from the current norms).  One block of W <= 1024 threads.
template <typename T>
__global__ __launch_bounds__(1024) void k_nu_partials(QrcpDev<T> d, ArgBest* cp, int64_t p0, int W)
{
    const int b = threadIdx.x;
    if (b < W) {
        ArgBest a;
        a.val = d.nu[p0 + b];
        a.key = d.perm[p0 + b];
        a.slot = (int32_t)(p0 + b);
        cp[b] = a;
    }
}

// Panel end of the right-looking window steps: the moves that put the pivots
// first (in step order).  Pivot q goes to slot q; a non-pivot column sitting
// in one of the slots 0..nbe-1 goes to a slot a pivot vacated (both taken in
// slot order); every other column stays, so at most 2 nbe columns move (the
// order of the non-pivot columns does not matter: the next panel reselects
// its window by norm, ties by key).  mv[0] = number of moves; move t is
// (mv[1+3t], mv[2+3t], mv[3+3t]) = (target slot, source column, pivot step or
// -1).  One block of up to 1024 threads (W <= 1024).
__global__ __launch_bounds__(1024) void k_window_order(const int32_t* wpiv, int nbe, int64_t p0, int W, int32_t* mv)
{
    __shared__ int32_t s_ispiv[1024];
    __shared__ int32_t s_d[1024];
    __shared__ int wsum[16];
    const int tid = threadIdx.x;
    if (tid < W) s_ispiv[tid] = 0;
    __syncthreads();
    if (tid < nbe) s_ispiv[wpiv[tid] - p0] = 1;
    __syncthreads();
    // non-pivot slots below nbe (sources) and pivot slots from nbe on (targets)
    const bool src = tid < nbe && !s_ispiv[tid];
    int nd = 0, ne = 0;
    const int rd = block_scan_flags1024(src, wsum, &nd);
    if (src) s_d[rd] = tid;
    const bool dst = tid >= nbe && tid < W && s_ispiv[tid];
    const int re = block_scan_flags1024(dst, wsum, &ne);
    __syncthreads();
    if (tid < nbe) {
        mv[1 + 3 * tid] = tid;
        mv[2 + 3 * tid] = wpiv[tid];
        mv[3 + 3 * tid] = tid;
    }
    if (dst) {
        const int t = nbe + re;
        mv[1 + 3 * t] = tid;
        mv[2 + 3 * t] = (int32_t)(p0 + s_d[re]);
        mv[3 + 3 * t] = -1;
    }
    if (tid == 0) mv[0] = nbe + ne;
}

// dir 0: tmp[:, t] = the final form of move t's column (for pivot step q:
// rows above p0 + q from A, beta and v from vbuf[:, q]; otherwise all rows
// from A), and its scalars into snu/snuref/sperm.  dir 1: the target slot
// receives tmp[:, t] and the scalars.  grid: (row chunks, >= mv[0]).
template <typename T>
__global__ __launch_bounds__(256) void k_window_gather(QrcpDev<T> d, const int32_t* mv, int64_t p0, const T* vbuf,
                                                       T* tmp, double* snu, double* snuref, int32_t* sperm, int dir)
{
    const int t = blockIdx.y;
    if (t >= mv[0]) return;
    const int64_t tgt = p0 + mv[1 + 3 * t], src = mv[2 + 3 * t];
    const int q = mv[3 + 3 * t];
    const int64_t vrow = q >= 0 ? p0 + q : d.m;   // first row taken from vbuf
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d.m; i += (int64_t)gridDim.x * 256) {
        if (dir == 0) tmp[i + d.lda * t] = i >= vrow ? vbuf[i + d.lda * q] : d.A[i + d.lda * src];
        else d.A[i + d.lda * tgt] = tmp[i + d.lda * t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (dir == 0) {
            snu[t] = d.nu[src];
            snuref[t] = d.nuref[src];
            sperm[t] = d.perm[src];
        } else {
            d.nu[tgt] = snu[t];
            d.nuref[tgt] = snuref[t];
            d.perm[tgt] = sperm[t];
        }
    }
}
