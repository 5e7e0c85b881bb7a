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

// Step 1a (one block of 1024 threads): choose the window among the remaining
// columns [p0, n) -- the W largest residual norms, found by a radix select
// on the norms' bit patterns (non-negative doubles order like their bits),
// equal norms at the threshold taken in column order -- and write the swap
// plan that brings them to [p0, p0+W): plan[0] = number of pairs, then pairs
// (a, b) of column positions to exchange.  The first pivot (largest norm,
// smallest key on ties) is always in the window; its argmax partial for the
// post-swap positions goes to cpart[0], cflag[0].
// Requires W <= 1024, W < n - p0 <= WIN_SORT_MAX.
template <typename T>
__global__ __launch_bounds__(1024) void k_window_select(QrcpDev<T> d, int64_t p0, int W, int32_t* plan)
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
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = tid + 1024 * u;
            if (q < L && (s_b[q] & mask) == prefix) atomicAdd(&s_hist[(s_b[q] >> shift) & 255], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int cum = 0, dig = 0;
            for (int bb = 255; bb >= 0; --bb) {
                const int h = (int)s_hist[bb];
                if (cum + h >= need) {
                    dig = bb;
                    break;
                }
                cum += h;
            }
            s_sel[0] = dig;
            s_sel[1] = need - cum;                               // still needed from this bin
            s_sel[2] = (int)s_hist[dig] == need - cum ? 1 : 0;   // the whole bin is taken
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
    // bin was taken whole, else the first `need` in column order)
    int taken_eq = 0;
    for (int u = 0; u < PER; ++u) {
        const int q0 = 1024 * u;
        const int q = tid + q0;
        const bool valid = q < L;
        const uint64_t hb = valid ? (s_b[q] & mask) : 0;
        const bool above = valid && hb > prefix;
        const bool at = valid && hb == prefix;
        int tot = 0;
        const int rank = block_scan_flags1024(at, wsum, &tot);
        const bool take = above || (at && (all_in || taken_eq + rank < need));
        if (take) s_in[q] = 1;
        taken_eq += tot;
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
    // compact the window in column order
    int base = 0;
    for (int u = 0; u < PER; ++u) {
        const int q = tid + 1024 * u;
        const bool f = q < L && s_in[q];
        int tot = 0;
        const int r = block_scan_flags1024(f, wsum, &tot);
        if (f && base + r < W) s_win[base + r] = q;
        base += tot;
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
    }
    const ArgBest b0 = s_best[0];
    if (tid == 0) plan[0] = nv;
    // first partial: the argmax, at its post-swap position
    if (tid < W && qe == b0.slot) {
        ArgBest b = b0;
        b.slot = (int32_t)(p0 + (vac ? s_d[iv] : qe));
        d.cpart[0] = b;
        d.cflag[0] = 0;
    }
}

// Step 1b: exchange the planned column pairs (all m rows, norms, keys).
// grid: W blocks (one pair each; blocks past plan[0] return).
template <typename T>
__global__ __launch_bounds__(256) void k_window_swap(QrcpDev<T> d, const int32_t* plan)
{
    const int q = blockIdx.x;
    if (q >= plan[0]) return;
    const int64_t a = plan[1 + 2 * q], b = plan[2 + 2 * q];
    for (int64_t i = threadIdx.x; i < d.m; i += 256) {
        const T x = d.A[i + d.lda * a], y = d.A[i + d.lda * b];
        d.A[i + d.lda * a] = y;
        d.A[i + d.lda * b] = x;
    }
    if (threadIdx.x == 0) {
        const double t0 = d.nu[a]; d.nu[a] = d.nu[b]; d.nu[b] = t0;
        const double t1 = d.nuref[a]; d.nuref[a] = d.nuref[b]; d.nuref[b] = t1;
        const int32_t t2 = d.perm[a]; d.perm[a] = d.perm[b]; d.perm[b] = t2;
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
// Per block: wpart[2b] = first failing step, wpart[2b+1] = first step after
// which a norm falls under the recomputation threshold, plus one (both nbe+1
// when none).  One thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_window_check(QrcpDev<T> d, const T* R12, int64_t ldr, int64_t c0,
                                                      int64_t nout, int nbe, int32_t* wpart)
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
        for (int t = 0; t < nbe; ++t) {
            const double pv = d.pivval[t];
            if (s > pv || (s == pv && key < d.pivkey[t])) {
                tfail = t;
                break;
            }
            double nn = s - cabs2(to_d(R12[t + ldr * q]));
            if (nn < 0.0) nn = 0.0;
            if (nn <= lim) {
                tflag = t + 1;
                break;
            }
            s = nn;
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
        wpart[2 * blockIdx.x] = min(min(s_min[0][0], s_min[0][1]), min(s_min[0][2], s_min[0][3]));
        wpart[2 * blockIdx.x + 1] = min(min(s_min[1][0], s_min[1][1]), min(s_min[1][2], s_min[1][3]));
    }
}

// Minimum over the check partials into ctl[CTL_TFAIL], ctl[CTL_TFLAG].
__global__ __launch_bounds__(256) void k_window_reduce(const int32_t* wpart, int nparts, int32_t* ctl)
{
    __shared__ int s_min[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int a = 0x7fffffff, b = 0x7fffffff;
    for (int q = tid; q < nparts; q += 256) {
        a = min(a, wpart[2 * q]);
        b = min(b, wpart[2 * q + 1]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a = min(a, __shfl_xor(a, off, MPS_WAVE));
        b = min(b, __shfl_xor(b, off, MPS_WAVE));
    }
    if (lane == 0) {
        s_min[0][wid] = a;
        s_min[1][wid] = b;
    }
    __syncthreads();
    if (tid == 0) {
        ctl[CTL_TFAIL] = min(min(s_min[0][0], s_min[0][1]), min(s_min[0][2], s_min[0][3]));
        ctl[CTL_TFLAG] = min(min(s_min[1][0], s_min[1][1]), min(s_min[1][2], s_min[1][3]));
    }
}

// Step 4 (no recomputation pending): downdate the outside columns' norms by
// their R rows r0 .. r0+nbe-1, now stored in A, with the per-step clamp of
// the step kernel.  One thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_window_commit(QrcpDev<T> d, int64_t r0, int64_t c0, int64_t nout, int nbe)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nout) return;
    const int64_t c = c0 + q;
    double s = d.nu[c];
    for (int t = 0; t < nbe; ++t) {
        const double nn = s - cabs2(to_d(d.A[r0 + t + d.lda * c]));
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
