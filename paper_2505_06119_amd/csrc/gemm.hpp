// Complex GEMM on the gfx950 matrix cores:  C = alpha * op(A) op(B) + beta * C
//
// Column-major operands.  op(X) is X or its conjugate transpose X^H.  A complex
// product is four real MFMAs (v_mfma_f32_16x16x4f32 for complex64 storage,
// v_mfma_f64_16x16x4f64 for complex128) into separate real / imaginary
// accumulators.  Each 256-thread workgroup computes a (32*WM) x (32*WN) tile of
// C with a 2 x 2 arrangement of waves; each wave owns (16*WM) x (16*WN).  The
// MFMA is fed with the B fragment as its first operand so that the 16 lanes
// of a lane group hold 16 consecutive *rows* of one C column: the epilogue's
// stores are then contiguous in column-major memory.  Output register e of
// lane l holds MFMA row 4*(l/16)+e for the f32 instruction and row l/16+4e for
// the f64 one (checked on gfx950).
//
// An operand can be read as a unit lower-trapezoidal matrix (the stored
// Householder vectors below a diagonal: entries above the diagonal read as 0,
// the diagonal as 1) -- the "V" of a block reflector I - V T V^H.
//
// Tall-skinny products (small M*N, long K) are split along K into partial
// products that a second kernel sums in FP64, in a fixed order.
#pragma once
#include "common.hpp"

struct GemmArgs {
    int64_t M, N, K;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    void* C;
    int64_t ldc;
    double2 alpha, beta;
    int64_t kchunk;   // split-K: number of K per z-slice (multiple of BK)
    void* part;       // split-K partial products (z x M x N, ld M), or null
};

template <typename T> struct MfmaOps;
template <> struct MfmaOps<float2> {
    typedef float S;
    typedef floatx4 Acc;
    static __device__ __forceinline__ Acc mma(S a, S b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output row of accumulator register e held by this lane
    static __device__ __forceinline__ int drow(int lane, int e) { return 4 * (lane >> 4) + e; }
};
template <> struct MfmaOps<double2> {
    typedef double S;
    typedef doublex4 Acc;
    static __device__ __forceinline__ Acc mma(S a, S b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the f64 variant interleaves its output rows across the 4 registers
    static __device__ __forceinline__ int drow(int lane, int e) { return (lane >> 4) + 4 * e; }
};

template <typename T>
__device__ __forceinline__ T load_masked(const T* base, int64_t ld, int64_t sr, int64_t sc, bool mask)
{
    if (mask) {
        if (sr < sc) { T z; z.x = 0; z.y = 0; return z; }
        if (sr == sc) { T o; o.x = 1; o.y = 0; return o; }
    }
    return base[sr + ld * sc];
}

#define GEMM_BK 16
#define GEMM_PAD 1

// PF: load the C tile (beta != 0) into registers before the K loop, so that
// its HBM latency overlaps the operand loads and the MFMAs -- for short-K
// updates, whose cost is the C read and write.
// BK: K depth of one LDS stage.  Long-K slices of small-tile products use 64
// (complex64) or 32 (complex128), so that each stage streams more of the
// operands per synchronisation.
template <typename T, int WM, int WN, bool CA, bool CB, bool MA, bool MB, bool PF = false, int BK = GEMM_BK,
          bool G3 = false>
__global__ __launch_bounds__(256) void k_zgemm(GemmArgs g)
{
    typedef typename MfmaOps<T>::S S;
    typedef typename MfmaOps<T>::Acc Acc;
    constexpr int BM = 32 * WM, BN = 32 * WN;
    __shared__ S As_re[BK][BM + GEMM_PAD], As_im[BK][BM + GEMM_PAD];
    __shared__ S Bs_re[BK][BN + GEMM_PAD], Bs_im[BK][BN + GEMM_PAD];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * BM, col0 = (int64_t)blockIdx.y * BN;
    const int wr = (wid >> 1) * (16 * WM), wc = (wid & 1) * (16 * WN);
    const T* A = (const T*)g.A;
    const T* B = (const T*)g.B;

    int64_t kbeg = 0, kend = g.K;
    if (g.part) {
        kbeg = (int64_t)blockIdx.z * g.kchunk;
        kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
    }

    T* C = (T*)g.C;
    T* P = (T*)g.part;
    const bool use_beta = (g.beta.x != 0.0 || g.beta.y != 0.0) && !P;
    T cpf[PF ? WM : 1][PF ? WN : 1][4];
    if constexpr (PF) {
        if (use_beta) {
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const int64_t r = row0 + wr + 16 * i + (lane & 15);
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t c = col0 + wc + 16 * j + MfmaOps<T>::drow(lane, e);
                        const int64_t rc = r < g.M ? r : g.M - 1, cc = c < g.N ? c : g.N - 1;
                        cpf[i][j][e] = C[rc + g.ldc * cc];
                    }
            }
        }
    }

    // G3: three real products per complex one, P1 = Br Ar, P2 = Bi Ai and
    // P3 = (Br + Bi)(Ar + Ai) in acc_re, acc_im, acc_s (re = P1 - P2,
    // im = P3 - P1 - P2); otherwise four, straight into re and im
    Acc acc_re[WM][WN], acc_im[WM][WN], acc_s[G3 ? WM : 1][G3 ? WN : 1];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc_re[i][j][e] = 0;
                acc_im[i][j][e] = 0;
                if constexpr (G3) acc_s[i][j][e] = 0;
            }

    // The next K tile is loaded into registers while the current one is
    // multiplied out of LDS.
    constexpr int AEL = BM * BK / 256;
    constexpr int BEL = BN * BK / 256;
    T ra[AEL], rb[BEL];
    auto load_tile = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < AEL; ++q) {
            int r, kk;
            if (!CA) { r = (tid + 256 * q) % BM; kk = (tid + 256 * q) / BM; }
            else     { kk = (tid + 256 * q) % BK; r = (tid + 256 * q) / BK; }
            const int64_t gr = row0 + r, gk = k0 + kk;
            T v;
            v.x = 0;
            v.y = 0;
            if (gr < g.M && gk < kend)
                v = CA ? load_masked(A, g.lda, gk, gr, MA) : load_masked(A, g.lda, gr, gk, MA);
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < BEL; ++q) {
            int c, kk;
            if (!CB) { kk = (tid + 256 * q) % BK; c = (tid + 256 * q) / BK; }
            else     { c = (tid + 256 * q) % BN; kk = (tid + 256 * q) / BN; }
            const int64_t gc = col0 + c, gk = k0 + kk;
            T v;
            v.x = 0;
            v.y = 0;
            if (gc < g.N && gk < kend)
                v = CB ? load_masked(B, g.ldb, gc, gk, MB) : load_masked(B, g.ldb, gk, gc, MB);
            rb[q] = v;
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int q = 0; q < AEL; ++q) {
            int r, kk;
            if (!CA) { r = (tid + 256 * q) % BM; kk = (tid + 256 * q) / BM; }
            else     { kk = (tid + 256 * q) % BK; r = (tid + 256 * q) / BK; }
            As_re[kk][r] = ra[q].x;
            As_im[kk][r] = CA ? -ra[q].y : ra[q].y;
        }
#pragma unroll
        for (int q = 0; q < BEL; ++q) {
            int c, kk;
            if (!CB) { kk = (tid + 256 * q) % BK; c = (tid + 256 * q) / BK; }
            else     { c = (tid + 256 * q) % BN; kk = (tid + 256 * q) / BN; }
            Bs_re[kk][c] = rb[q].x;
            Bs_im[kk][c] = CB ? -rb[q].y : rb[q].y;
        }
    };

    if (kbeg < kend) load_tile(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
        store_tile();
        __syncthreads();
        if (k0 + BK < kend) load_tile(k0 + BK);
#pragma unroll 4
        for (int ks = 0; ks < BK; ks += 4) {
            const int kk = ks + (lane >> 4);
            S ar[WM], ai[WM], br[WN], bi[WN], nbi[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                ar[i] = As_re[kk][wr + 16 * i + (lane & 15)];
                ai[i] = As_im[kk][wr + 16 * i + (lane & 15)];
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                br[j] = Bs_re[kk][wc + 16 * j + (lane & 15)];
                bi[j] = Bs_im[kk][wc + 16 * j + (lane & 15)];
                nbi[j] = -bi[j];
            }
            if constexpr (G3) {
                S as[WM], bs[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) as[i] = ar[i] + ai[i];
#pragma unroll
                for (int j = 0; j < WN; ++j) bs[j] = br[j] + bi[j];
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        acc_re[i][j] = MfmaOps<T>::mma(br[j], ar[i], acc_re[i][j]);
                        acc_im[i][j] = MfmaOps<T>::mma(bi[j], ai[i], acc_im[i][j]);
                        acc_s[i][j] = MfmaOps<T>::mma(bs[j], as[i], acc_s[i][j]);
                    }
            } else {
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        acc_re[i][j] = MfmaOps<T>::mma(br[j], ar[i], acc_re[i][j]);
                        acc_re[i][j] = MfmaOps<T>::mma(nbi[j], ai[i], acc_re[i][j]);
                        acc_im[i][j] = MfmaOps<T>::mma(bi[j], ar[i], acc_im[i][j]);
                        acc_im[i][j] = MfmaOps<T>::mma(br[j], ai[i], acc_im[i][j]);
                    }
            }
        }
        __syncthreads();
    }

    // ---- epilogue: lane holds C[row = .. + lane%16][col = .. + drow(lane, e)];
    //      the C loads of one row block are issued together ----
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int64_t r = row0 + wr + 16 * i + (lane & 15);
        T cv[WN][4];
        if constexpr (PF) {
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) cv[j][e] = cpf[i][j][e];
        } else if (use_beta) {
            // unconditional loads from clamped indices (a conditional load would
            // wait for its data before the next one issues)
            const int64_t rc = r < g.M ? r : g.M - 1;
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t c = col0 + wc + 16 * j + MfmaOps<T>::drow(lane, e);
                    cv[j][e] = C[rc + g.ldc * (c < g.N ? c : g.N - 1)];
                }
        }
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = col0 + wc + 16 * j + MfmaOps<T>::drow(lane, e);
                if (r >= g.M || c >= g.N) continue;
                double2 v = make_double2((double)acc_re[i][j][e], (double)acc_im[i][j][e]);
                if constexpr (G3) {
                    const double p1 = acc_re[i][j][e], p2 = acc_im[i][j][e], p3 = acc_s[i][j][e];
                    v = make_double2(p1 - p2, p3 - p1 - p2);
                }
                if (P) {
                    P[(int64_t)blockIdx.z * g.M * g.N + r + g.M * c] = from_d<T>(v);
                } else {
                    v = cmul(g.alpha, v);
                    if (use_beta) v = cadd(v, cmul(g.beta, to_d(cv[j][e])));
                    C[r + g.ldc * c] = from_d<T>(v);
                }
            }
    }
}

// Sum split-K partial products in a fixed order (FP64) and apply alpha/beta.
template <typename T>
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs g, int nz)
{
    const int64_t total = g.M * g.N;
    const T* P = (const T*)g.part;
    T* C = (T*)g.C;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        double2 s = czero();
        for (int z = 0; z < nz; ++z) s = cadd(s, to_d(P[(int64_t)z * total + idx]));
        const int64_t r = idx % g.M, c = idx / g.M;
        double2 v = cmul(g.alpha, s);
        if (g.beta.x != 0.0 || g.beta.y != 0.0) v = cadd(v, cmul(g.beta, to_d(C[r + g.ldc * c])));
        C[r + g.ldc * c] = from_d<T>(v);
    }
}

// ---------------------------------------------------------------------------
// Rank-K update  C += alpha A B  for K <= KD (32 or 64): the trailing update
// A_o -= V W2 of a QR panel and the Q update of the blocked Q formation.
// Memory-bound (16 bytes of C traffic per KD complex MACs), so it is laid out
// for streaming C rather than for operand reuse:
//   * each wave keeps its 32 rows of A (the panel's V, read once, masked to
//     the unit lower trapezoid when MA) in registers as MFMA fragments;
//   * it walks its block's column range in chunks of 16 columns, loading the
//     next chunk's C tile and B fragments before the current chunk's MFMAs,
//     so that HBM traffic overlaps the matrix-core work;
//   * the contraction index is split so that lane group q (lanes 16q..16q+15)
//     covers k = q*KD/4 .. (q+1)*KD/4-1: B fragments are then KD/4 contiguous
//     elements of one B column per lane (16-byte loads).
// Entries k >= K of A and B are zeroed, so B may hold anything there.  beta
// is 1.  Grid: (ceil(M / 128), column ranges of cps columns, cps a multiple
// of 16); 256 threads (four waves stacked in rows).
// ---------------------------------------------------------------------------
template <typename T, int KD, bool MA, bool G3 = false>
__global__ __launch_bounds__(256) void k_zrank(GemmArgs g, int64_t cps)
{
    typedef typename MfmaOps<T>::S S;
    typedef typename MfmaOps<T>::Acc Acc;
    constexpr int QK = KD / 4;                 // contraction indices per lane group
    constexpr int NV = QK * (int)sizeof(T) / 16;   // 16-byte loads per B fragment
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int grp = lane >> 4, l16 = lane & 15;
    const int64_t M = g.M, N = g.N, K = g.K;
    const int64_t r0 = (int64_t)blockIdx.x * 128 + wid * 32;
    const int64_t cbeg = (int64_t)blockIdx.y * cps;
    const int64_t cend = cbeg + cps < N ? cbeg + cps : N;
    if (r0 >= M || cbeg >= cend) return;
    const T* A = (const T*)g.A;
    const T* B = (const T*)g.B;
    T* C = (T*)g.C;
    const S alr = (S)g.alpha.x, ali = (S)g.alpha.y;

    S are[2][QK], aim[2][QK], asu[G3 ? 2 : 1][G3 ? QK : 1];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t r = r0 + 16 * i + l16;
        const int64_t rc = r < M ? r : M - 1;
#pragma unroll
        for (int q = 0; q < QK; ++q) {
            const int k = QK * grp + q;
            const int kc = k < K ? k : 0;
            T v = A[rc + g.lda * kc];
            if (MA) {
                if (r < k) { v.x = 0; v.y = 0; }
                if (r == k) { v.x = 1; v.y = 0; }
            }
            if (k >= K) { v.x = 0; v.y = 0; }
            are[i][q] = v.x;
            aim[i][q] = v.y;
            if constexpr (G3) asu[i][q] = v.x + v.y;
        }
    }
    const int64_t ra = r0 + l16, rb = r0 + 16 + l16;
    const int64_t rca = ra < M ? ra : M - 1, rcb = rb < M ? rb : M - 1;
    T cv[2][2][4];
    T bv[2][QK];
    auto load = [&](int buf, int64_t c0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t c = c0 + MfmaOps<T>::drow(lane, e);
            const int64_t cc = c < N ? c : N - 1;
            cv[buf][0][e] = C[rca + g.ldc * cc];
            cv[buf][1][e] = C[rcb + g.ldc * cc];
        }
        const int64_t c = c0 + l16;
        const int64_t cc = c < N ? c : N - 1;
        const float4* bp = (const float4*)(B + QK * grp + g.ldb * cc);
#pragma unroll
        for (int h = 0; h < NV; ++h) {
            const float4 t = bp[h];
            if constexpr (sizeof(T) == 8) {
                bv[buf][2 * h] = make_float2(t.x, t.y);
                bv[buf][2 * h + 1] = make_float2(t.z, t.w);
            } else {
                bv[buf][h] = *(const T*)&t;
            }
        }
    };
    auto compute = [&](int buf, int64_t c0) {
        S bre[QK], bim[QK], nbi[QK];
#pragma unroll
        for (int q = 0; q < QK; ++q) {
            const bool live = QK * grp + q < K;
            bre[q] = live ? (S)bv[buf][q].x : (S)0;
            bim[q] = live ? (S)bv[buf][q].y : (S)0;
            nbi[q] = -bim[q];
        }
        // G3: P1 = Br Ar, P2 = Bi Ai, P3 = (Br + Bi)(Ar + Ai) in pr, pi, ps;
        // otherwise the real and imaginary parts directly in pr, pi
        Acc pr[2], pi[2], ps[G3 ? 2 : 1];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                pr[i][e] = 0;
                pi[i][e] = 0;
                if constexpr (G3) ps[i][e] = 0;
            }
#pragma unroll
        for (int q = 0; q < QK; ++q)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if constexpr (G3) {
                    pr[i] = MfmaOps<T>::mma(bre[q], are[i][q], pr[i]);
                    pi[i] = MfmaOps<T>::mma(bim[q], aim[i][q], pi[i]);
                    ps[i] = MfmaOps<T>::mma(bre[q] + bim[q], asu[i][q], ps[i]);
                } else {
                    pr[i] = MfmaOps<T>::mma(bre[q], are[i][q], pr[i]);
                    pr[i] = MfmaOps<T>::mma(nbi[q], aim[i][q], pr[i]);
                    pi[i] = MfmaOps<T>::mma(bim[q], are[i][q], pi[i]);
                    pi[i] = MfmaOps<T>::mma(bre[q], aim[i][q], pi[i]);
                }
            }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t r = i ? rb : ra;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t c = c0 + MfmaOps<T>::drow(lane, e);
                S xr = pr[i][e], xi = pi[i][e];
                if constexpr (G3) {
                    xr = pr[i][e] - pi[i][e];
                    xi = ps[i][e] - pr[i][e] - pi[i][e];
                }
                T o = cv[buf][i][e];
                o.x += alr * xr - ali * xi;
                o.y += alr * xi + ali * xr;
                if (r < M && c < cend) C[r + g.ldc * c] = o;
            }
        }
    };
    // two register buffers: chunk c+16 loads while chunk c computes
    load(0, cbeg);
    for (int64_t c0 = cbeg;;) {
        const int64_t c1 = c0 + 16;
        if (c1 < cend) load(1, c1);
        compute(0, c0);
        if (c1 >= cend) break;
        const int64_t c2 = c1 + 16;
        if (c2 < cend) load(0, c2);
        compute(1, c1);
        if (c2 >= cend) break;
        c0 = c2;
    }
}

// C (M x N) += alpha A B with A M x K (unit lower trapezoidal when mask_a),
// B K x N (ldb >= 32 for K <= 32, >= 64 otherwise; 16-byte aligned columns),
// K <= 64.  Complex64 only: the complex128 fragments would need the whole
// register file (one wave per SIMD), where the LDS-tiled zgemm does better.
// Returns false for what it does not take (the caller then uses zgemm with
// beta = 1).
template <typename T>
static bool zrank_update(hipStream_t st, bool mask_a, int64_t M, int64_t N, int64_t K, double2 alpha, const T* A,
                         int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc)
{
    if constexpr (sizeof(T) != 8) {
        return false;
    } else {
    if (M <= 0 || N <= 0 || K <= 0) return true;
    const int kd = K <= 32 ? 32 : 64;
    if (K > 64 || ldb < kd || ((uintptr_t)B & 15) != 0 || (ldb * (int64_t)sizeof(T)) % 16 != 0) return false;
    GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    g.alpha = alpha; g.beta = make_double2(1.0, 0.0);
    g.kchunk = K; g.part = nullptr;
    // rank <= 32: about 1500 blocks (six per CU) measured best, the longer
    // column ranges amortising the V fragment loads; rank 64: about 3000
    const int64_t rblk = (M + 127) / 128;
    const int64_t target = kd == 32 ? 1536 : 3072;
    int64_t splits = (target + rblk - 1) / rblk;
    int64_t cps = (N + splits - 1) / splits;
    cps = (cps + 15) / 16 * 16;
    splits = (N + cps - 1) / cps;
    dim3 grid((unsigned)rblk, (unsigned)splits);
    if (kd == 32) {   // three products per complex one (the rank-64 form has no registers for it)
        if (mask_a) hipLaunchKernelGGL((k_zrank<T, 32, true, true>), grid, dim3(256), 0, st, g, cps);
        else hipLaunchKernelGGL((k_zrank<T, 32, false, true>), grid, dim3(256), 0, st, g, cps);
    } else {
        if (mask_a) hipLaunchKernelGGL((k_zrank<T, 64, true>), grid, dim3(256), 0, st, g, cps);
        else hipLaunchKernelGGL((k_zrank<T, 64, false>), grid, dim3(256), 0, st, g, cps);
    }
    return true;
    }
}

enum GemmOp { OP_N = 0, OP_C = 1 };

// Bytes of split-K scratch the launcher may need for an M x N product.
static inline int64_t gemm_splitk_bytes(int64_t M, int64_t N, int64_t K, int64_t elem)
{
    (void)K;
    return 16 * M * N * elem;   // at most 16 slices
}

template <typename T, int WM, int WN, bool CA, bool CB, bool MA, bool MB, bool PF = false, int BK = GEMM_BK,
          bool G3 = false>
static void launch_gemm_cfg(GemmArgs g, hipStream_t st, int nz)
{
    constexpr int BM = 32 * WM, BN = 32 * WN;
    dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)((g.N + BN - 1) / BN), (unsigned)nz);
    hipLaunchKernelGGL((k_zgemm<T, WM, WN, CA, CB, MA, MB, PF, BK, G3>), grid, dim3(256), 0, st, g);
}

// Tile shapes per storage type: complex64 uses 128 x 128 tiles for large
// products; complex128 uses 128 x 64 (its LDS staging is twice as large).
template <typename T> struct GemmTile;
template <> struct GemmTile<float2> { static constexpr int WM = 4, WN = 4; };
template <> struct GemmTile<double2> { static constexpr int WM = 4, WN = 2; };

template <typename T, bool CA, bool CB, bool MA, bool MB>
static void launch_gemm_t(GemmArgs g, hipStream_t st, void* scratch, int64_t scratch_bytes, int* nz_out)
{
    if (g.M <= 0 || g.N <= 0) return;
    constexpr int BWM = GemmTile<T>::WM, BWN = GemmTile<T>::WN;
    // Large tiles only pay off for long K; a rank-k update with k <= 64 is
    // memory-bound and wants many resident blocks to overlap C traffic.
    const bool big = g.M >= 512 && g.N >= 512 && g.K > 64;
    // at most 32 rows (the V^H A products of a panel): 32 x 128 tiles
    const bool thin = !big && g.M <= 32;
    const int64_t BM = big ? 32 * BWM : (thin ? 32 : 64), BN = big ? 32 * BWN : (thin ? 128 : 64);
    const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    int nz = 1;
    if (g.K > 0 && tiles < 256 && g.K >= 512 && scratch) {
        // enough K slices for ~1024 blocks: a short-M, long-K product streams
        // its B operand and needs every CU busy with several blocks, while each
        // slice's partial product costs a write and a read of M x N
        int64_t want = 1024 / tiles;
        int64_t maxz = g.K / 128;
        nz = (int)(want < maxz ? want : maxz);
        if (nz > 64) nz = 64;
        if (nz < 1) nz = 1;
        const int64_t fit = scratch_bytes / (g.M * g.N * (int64_t)sizeof(T));
        if (nz > fit) nz = (int)(fit > 1 ? fit : 1);
    }
    // deep K stages for long slices of a small-tile product
    constexpr int DBK = sizeof(T) == 8 ? 32 : 16;
    const bool deep = !big && (nz > 1 ? g.K / nz : g.K) >= 256;
    const int64_t bk = deep ? DBK : GEMM_BK;
    if (nz > 1) {
        int64_t chunk = (g.K + nz - 1) / nz;
        chunk = (chunk + bk - 1) / bk * bk;
        nz = (int)((g.K + chunk - 1) / chunk);
        g.kchunk = chunk;
        g.part = scratch;
    } else {
        g.part = nullptr;
        g.kchunk = g.K;
    }
    const bool beta_nz = g.beta.x != 0.0 || g.beta.y != 0.0;
    if (big)   // complex128's big tile has no registers left for the third accumulator
        launch_gemm_cfg<T, BWM, BWN, CA, CB, MA, MB, false, GEMM_BK, sizeof(T) == 8>(g, st, nz);
    else if (nz == 1 && beta_nz && g.K <= 64 && !thin)
        launch_gemm_cfg<T, 2, 2, CA, CB, MA, MB, true>(g, st, nz);
    else if (thin && deep)
        launch_gemm_cfg<T, 1, 4, CA, CB, MA, MB, false, DBK, true>(g, st, nz);
    else if (thin)
        launch_gemm_cfg<T, 1, 4, CA, CB, MA, MB, false, GEMM_BK, true>(g, st, nz);
    else if (deep)
        launch_gemm_cfg<T, 2, 2, CA, CB, MA, MB, false, DBK, true>(g, st, nz);
    else
        launch_gemm_cfg<T, 2, 2, CA, CB, MA, MB, false, GEMM_BK, true>(g, st, nz);
    if (nz_out) *nz_out = g.part ? nz : 1;
    if (g.part && !nz_out) {
        int64_t total = g.M * g.N;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL((k_splitk_reduce<T>), dim3((unsigned)blocks), dim3(256), 0, st, g, nz);
    }
}

// Runtime dispatch over the operand forms used by the library.  Returns false
// for a combination that has no instantiation.  With nz_out, a product split
// along K leaves its *nz_out partial products unreduced in scratch (slice z at
// scratch + z M N, ld M; alpha and beta not applied) for the caller to reduce;
// *nz_out = 1 means C holds the product.
template <typename T>
static bool zgemm(hipStream_t st, GemmOp opa, bool maska, GemmOp opb, bool maskb,
                  int64_t M, int64_t N, int64_t K, double2 alpha,
                  const T* A, int64_t lda, const T* B, int64_t ldb, double2 beta, T* C, int64_t ldc,
                  void* scratch, int64_t scratch_bytes, int* nz_out = nullptr)
{
    GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    g.kchunk = K; g.part = nullptr;
    const int key = (opa == OP_C ? 8 : 0) | (opb == OP_C ? 4 : 0) | (maska ? 2 : 0) | (maskb ? 1 : 0);
    switch (key) {
    case 0:  launch_gemm_t<T, false, false, false, false>(g, st, scratch, scratch_bytes, nz_out); return true;
    case 4:  launch_gemm_t<T, false, true, false, false>(g, st, scratch, scratch_bytes, nz_out); return true;
    case 8:  launch_gemm_t<T, true, false, false, false>(g, st, scratch, scratch_bytes, nz_out); return true;
    case 2:  launch_gemm_t<T, false, false, true, false>(g, st, scratch, scratch_bytes, nz_out); return true;
    case 10: launch_gemm_t<T, true, false, true, false>(g, st, scratch, scratch_bytes, nz_out); return true;
    case 11: launch_gemm_t<T, true, false, true, true>(g, st, scratch, scratch_bytes, nz_out); return true;
    case 12: launch_gemm_t<T, true, true, false, false>(g, st, scratch, scratch_bytes, nz_out); return true;
    default: return false;
    }
}
