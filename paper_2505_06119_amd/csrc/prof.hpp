// Optional per-kernel timing with HIP events on the launch stream.  In mode 1
// (mps_profile(1)) every timed launch is bracketed by an event pair; in a
// sampled mode s >= 2 only one pivot-step launch (class PK_STEP_C: k_step_c
// or k_window_step) in s is, so that the event markers barely perturb the run
// they measure.  The pairs are
// resolved at the next host synchronisation point of the library and
// accumulated per kernel class together with the algorithmic bytes and flops
// of each launch.  Process-global; meant for single-threaded use.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>

enum {
    PK_CONTRACT = 0,  // theta0 = A B (MFMA GEMM)
    PK_GATE = 1,      // gate + FP64 column norms
    PK_STEP_A = 2,    // pivot swap, bring-up, reflector
    PK_STEP_C = 3,    // trailing GEMV, F column, pivot row, downdate
    PK_TRAIL = 4,     // panel-end MFMA updates A -= V F^H and A -= V W2
    PK_NORMS = 5,     // exact norm recomputation / ||R22||
    PK_UNGQR = 6,     // Q formation
    PK_SPLIT = 7,     // R P^T scatter
    PK_PROPOSE = 8,   // learned proposal: sketch, features, scores, order, gather
    PK_WINDOW = 9,    // candidate-window selection, swaps, saves and greedy replay
    PK_PANEL = 10,    // W = V^H A over the trailing columns (the first half of the block-reflector update)
    PK_REFL = 11,     // block reflector bookkeeping: V^H V, T, T^H W, the R rows outside a window
    PK_COUNT = 12
};

struct ProfAcc {
    int64_t launches;
    double total_ms;
    double alg_bytes;
    double alg_flops;
};

struct ProfState {
    bool on = false;
    int stride = 1;        // 1: every launch of every class; s >= 2: one k_step_c launch in s
    int64_t counter = 0;
    struct Rec {
        hipEvent_t a, b;
        int cls;
        double bytes, flops;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    ProfAcc acc[PK_COUNT] = {};
};

static ProfState g_prof;

static hipEvent_t prof_event()
{
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Returns an opaque begin event (or null when this launch is not timed).
// cls names the kernel class where the sampled mode has to know it.
static inline hipEvent_t prof_begin(hipStream_t st, int cls = -1)
{
    if (!g_prof.on) return nullptr;
    if (g_prof.stride > 1 && (cls != PK_STEP_C || (g_prof.counter++ % g_prof.stride) != 0)) return nullptr;
    hipEvent_t e = prof_event();
    if (e) (void)hipEventRecord(e, st);
    return e;
}

static inline void prof_end(hipEvent_t begin, hipStream_t st, int cls, double bytes, double flops)
{
    if (!g_prof.on || !begin) return;
    hipEvent_t e = prof_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    g_prof.pending.push_back({begin, e, cls, bytes, flops});
}

// Call after the stream has been synchronised.
static inline void prof_flush()
{
    for (auto& r : g_prof.pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            ProfAcc& a = g_prof.acc[r.cls];
            a.launches++;
            a.total_ms += ms;
            a.alg_bytes += r.bytes;
            a.alg_flops += r.flops;
        }
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.pending.clear();
}
