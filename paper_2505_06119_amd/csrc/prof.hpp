// Optional per-kernel timing with HIP events on the launch stream.  In mode 1
// (mps_profile(1)) every timed launch is bracketed by an event pair.  In a
// sampled mode s >= 2 the pivot steps are timed in whole runs: one run of
// back-to-back window-step launches (a panel's steps) in s gets a single
// event pair and counts as that many launches, and one k_step_c launch in s
// outside the window is bracketed on its own; nothing else is timed, so the
// markers barely perturb the run they measure.  The pairs are resolved once
// both events have completed (at a host synchronisation point of the library)
// and accumulated per kernel class together with the algorithmic bytes and
// flops of each launch.  Process-global; meant for single-threaded use.
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
    int stride = 1;        // 1: every launch of every class; s >= 2: sampled pivot steps
    int64_t counter = 0;   // k_step_c launches seen in the sampled mode
    int64_t runs = 0;      // window-step runs seen in the sampled mode
    struct Rec {
        hipEvent_t a, b;
        int cls;
        double bytes, flops;
        int64_t n;   // launches the pair brackets
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

// The begin event of a run of back-to-back pivot-step launches, in the
// sampled mode only (one run in stride); null otherwise.
static inline hipEvent_t prof_begin_run(hipStream_t st)
{
    if (!g_prof.on || g_prof.stride <= 1 || (g_prof.runs++ % g_prof.stride) != 0) return nullptr;
    hipEvent_t e = prof_event();
    if (e) (void)hipEventRecord(e, st);
    return e;
}

// n: the launches between begin and this end (bytes and flops are their sums)
static inline void prof_end(hipEvent_t begin, hipStream_t st, int cls, double bytes, double flops, int64_t n = 1)
{
    if (!g_prof.on || !begin) return;
    hipEvent_t e = prof_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    g_prof.pending.push_back({begin, e, cls, bytes, flops, n});
}

// Resolves the pairs whose end event has completed; the others stay pending.
static inline void prof_flush()
{
    size_t keep = 0;
    for (size_t i = 0; i < g_prof.pending.size(); ++i) {
        ProfState::Rec& r = g_prof.pending[i];
        if (hipEventQuery(r.b) == hipErrorNotReady) {
            g_prof.pending[keep++] = r;
            continue;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            ProfAcc& a = g_prof.acc[r.cls];
            a.launches += r.n;
            a.total_ms += ms;
            a.alg_bytes += r.bytes;
            a.alg_flops += r.flops;
        }
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.pending.resize(keep);
}
