// Private declarations of the solver driver shared by api.cpp (single
// image) and batch.cpp (many images). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/ddi.h"
#include "internal.h"

namespace ddi {

// One resolution level of a plan's pyramid.
struct Level {
    int h = 0, w = 0;
    const float* f = nullptr;
    const uint8_t* c = nullptr;
    float* fown = nullptr;
    uint8_t* cown = nullptr;
    float* u[2] = {nullptr, nullptr};
    uint64_t* mbits = nullptr;  // column-transposed unknown-pixel bits
    bool own_u0 = false;
    SweepArgs sw;
};

// Record a failed HIP call and return DDI_EHIP.
int hip_fail(hipError_t e);

BlockGrid make_grid(int h, int w, int block, int overlap);
SweepArgs make_sweep(int h, int w, int channels, int block, int overlap, float alpha, int k,
                     float local_tol = 0.f);
// DDI_OK when a gfx950 device is current.
int check_device();
// Device bytes ddi_create allocates for these sizes and parameters.
size_t plan_device_bytes(int h, int w, int C, const ddi_params& prm);
// Finest-level sweeps of this plan use unchanged-block flags
// (skip_unchanged, float32 ORAS, a grid where launch_sweep accepts them).
bool use_skip(const ddi_params& prm, const SweepArgs& a0);
// The finest level's sweeps of this plan run their blocks in the order
// of the CG steps of the level-2 blocks over them (order_blocks).
bool use_order(const ddi_params& prm, int h, int w, int C);
// Sweep geometry of level l (0 = finest) of a plan for h x w x C.
SweepArgs level_sweep(int h, int w, int C, const ddi_params& prm, int l);
// coarse_solver = 1 on a coarsest level too large for one workgroup: the
// solve runs on a grid of workgroups (launch_coarse_cg_grid).
bool use_coarse_grid(const ddi_params& prm, int h, int w);
// Levels a plan builds for h x w: `levels`, fewer once a level is 1 x 1.
int level_count(int h, int w, int levels);
// DDI_OK for 1 <= h, w; 1 <= channels <= 4; h * w <= 2^30.
int check_dims(int h, int w, int channels);

// True when the byte ranges [a, a + na) and [b, b + nb) share a byte (null
// pointers never overlap): outputs of a call must not alias its inputs.
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace ddi

#define DDI_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return ddi::hip_fail(e_); \
    } while (0)

struct ddi_plan {
    int h = 0, w = 0, C = 0;
    ddi_params p;
    size_t bytes = 0;  // device memory the plan holds
    hipStream_t s = nullptr;
    std::vector<ddi::Level> lv;
    double* part = nullptr;
    size_t part_n = 0;
    double* red = nullptr;   // [C + 2] stats, [C] norms, [C] CG step totals,
                             // [C] first-sweep CG steps, [2C] skip totals
    double* host = nullptr;  // pinned mirror of red
    double* cgcnt = nullptr; // timing: per finest-level block, CG steps, whole
                             // skips and skipped write-backs (three planes)
    int* flg = nullptr;      // block keys (CG steps) of the finest level for the
                             // skips of the batched solve, two arrays (sweep
                             // parity); null: no skipping
    void* cgw = nullptr;     // coarse_solver = 1 on a coarsest level over
                             // kCoarseMaxPixels: the grid solve's workspace
    int* keys2 = nullptr;    // order_blocks: CG steps per level-2 block of its
                             // last sweep, and the dispatch table of the
    int* order = nullptr;    // finest level's sweeps built from them
    bool order_on = false;   // the solve being enqueued built that table
    int* ctl = nullptr;      // device stop test: done, sweeps, error, -, rel (double)
    void* hctl = nullptr;    // pinned mirror of ctl
    int* dmirror = nullptr;  // hctl as the device sees it (k_decide writes it), or null
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t ev_ctl = nullptr;  // after the control-word read-back of a batch
    // a solve enqueued by ddi_solve_async and not yet waited for
    struct Pending {
        bool active = false, timing = false;
        const float* f = nullptr;
        const uint8_t* c = nullptr;
        float* u = nullptr;
        hipStream_t s = nullptr;
        int start0 = 0, done_upto = 0;
        // the work enqueued since the last check ends with a stop test that
        // writes the host mirror of the control words (no copy needed)
        bool mirrored = false;
    };
    Pending pend;
    std::vector<hipEvent_t> sweep_ev;  // 2 per finest-level sweep (timing)
    std::vector<double> sweep_ms;      // device ms of each finest sweep, last solve
    int last_sweeps = -1;              // finest-level sweeps of the previous solve
    // graph mode: a plan-owned stream, and the instantiated graph of the
    // solve's first batch with the key it was captured for
    hipStream_t gs = nullptr;
    hipEvent_t ev_in = nullptr;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        const void* f = nullptr;
        const void* c = nullptr;
        const void* u = nullptr;
        int start = -1, batch = -1;
        long last_use = 0;
    };
    // a few instantiated graphs (the start buffer and first batch follow the
    // sweeps the previous solve needed, so they alternate between values)
    static constexpr int kGraphs = 4;
    Graph graphs[kGraphs];
    long graph_clock = 0;
    // storage = 1: bfloat16 right-hand side and ping-pong corrections of
    // the refinement equation on the finest level
    uint16_t* r16 = nullptr;
    uint16_t* d16[2] = {nullptr, nullptr};
    // method = 1 (multilevel CG): r, p[2], q planes sized for the finest
    // level, the CG scalars [rho, alpha, beta] x C, per-level statistics
    // [L][C + 2], and the CG steps each level needed last time
    float* cg_vec = nullptr;
    double* cg_sc = nullptr;
    std::vector<int> last_iters;
    // method = 2 (Krylov-accelerated ORAS): the basis V_0..V_m and the
    // preconditioned vectors Z_0..Z_{m-1} (finest-level planes), the
    // per-channel cycle state, scalars [hcol (m+1) x C][hn2 C][beta2 C], and
    // the dot-product partials [wg][m+1][C]
    float* kry_vec = nullptr;
    ddi::KryState* kry_state = nullptr;
    double* kry_sc = nullptr;
    double* kry_part = nullptr;
    // the finest level's first sweep of the solve being enqueued prolongs
    // from this source (fuse_prolong)
    ddi::ProSrc pro0{};
    bool pro0_on = false;
};

// Multilevel CG solve (mlcg.cpp); the level-0 pointers are set.
int solve_mlcg(ddi_plan* P, ddi_stats* st);
// Krylov-accelerated ORAS solve (krylov.cpp); the level-0 pointers are set.
int solve_krylov(ddi_plan* P, ddi_stats* st);
// Pyramid, statistics, transposed masks, coarsest level and coarse-to-fine
// passes down to the finest level's start in buffer start0 (api.cpp); it
// also zeroes the stop-test control word ctl[0..4).
int plan_enqueue_front(ddi_plan* P, int start0, hipStream_t s, bool fuse_l0);
