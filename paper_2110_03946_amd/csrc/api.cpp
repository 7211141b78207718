// Solver driver and C ABI (include/ddi.h) of the multilevel ORAS inpainting
// library. Host code only: it owns the device buffers of a plan and
// enqueues the kernels (sweep.hip, levels.hip, outer.hip, coarse.hip) on the
// plan's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan.h"

using namespace ddi;

static_assert(DDI_COARSE_MAX_PIXELS == kCoarseMaxPixels, "coarse solve size limit");

namespace {
// per host thread: plans may be driven from several threads at once
thread_local int g_last_hip = 0;
}  // namespace

int ddi::hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return DDI_EHIP;
}

namespace ddi {

BlockGrid make_grid(int h, int w, int block, int overlap) {
    BlockGrid g;
    g.h = h;
    g.w = w;
    g.bh = std::min(block, h);
    g.bw = std::min(block, w);
    g.nby = block_count(h, block, overlap);
    g.nbx = block_count(w, block, overlap);
    g.sy = g.nby > 1 ? block - overlap : std::max(g.bh, 1);
    g.sx = g.nbx > 1 ? block - overlap : std::max(g.bw, 1);
    return g;
}

SweepArgs make_sweep(int h, int w, int channels, int block, int overlap, float alpha, int k,
                     float local_tol) {
    SweepArgs a;
    a.local_tol2 = local_tol * local_tol;
    a.g = make_grid(h, w, block, overlap);
    a.channels = channels;
    a.cpitch = (int64_t)h * w;
    a.alpha = alpha;
    a.k = k;
    return a;
}

int check_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return DDI_ENODEV;
    int dev = 0;
    DDI_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    DDI_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DDI_ENODEV;
    return DDI_OK;
}

int level_count(int h, int w, int levels) {
    // stop halving once the level is a single pixel
    int L = 1;
    while (L < levels) {
        int hl = h, wl = w;
        for (int i = 0; i < L; ++i) {
            hl = (hl + 1) / 2;
            wl = (wl + 1) / 2;
        }
        if (hl == 1 && wl == 1) break;
        ++L;
    }
    return L;
}

bool use_skip(const ddi_params& prm, const SweepArgs& a0) {
    return prm.skip_unchanged == 1 && prm.storage == 0 && prm.method == 0 && sweep_skip_ok(a0);
}

// Level grids of a plan (level 0 = finest).
SweepArgs level_sweep(int h, int w, int C, const ddi_params& prm, int l) {
    for (int i = 0; i < l; ++i) {
        h = (h + 1) / 2;
        w = (w + 1) / 2;
    }
    if (l == 0) return make_sweep(h, w, C, prm.block, prm.overlap, prm.robin_alpha, 1);
    const int cb = prm.coarse_block ? prm.coarse_block : prm.block;
    const int co = prm.coarse_overlap >= 0 ? prm.coarse_overlap : prm.overlap;
    return make_sweep(h, w, C, cb, co, prm.robin_alpha, 1);
}

bool use_order(const ddi_params& prm, int h, int w, int C) {
    // the finest sweeps' dispatch table comes from the level-2 sweep's
    // CG steps and is built inside the level-1 sweep: three levels of 64-row
    // blocks, levels 2 and 1 each running a sweep; the table's counting sort
    // takes grids of < 2^16 blocks
    if (prm.order_blocks != 1 || prm.storage != 0 || prm.method != 0) return false;
    const int L = level_count(h, w, prm.levels);
    if (L < 3 || prm.coarse_sweeps < 1) return false;
    if (L == 3 && !(prm.coarse_solver == 0 && prm.coarsest_sweeps > 0)) return false;
    const SweepArgs a0 = level_sweep(h, w, C, prm, 0);
    return sweep_prolong_ok(a0) && sweep_prolong_ok(level_sweep(h, w, C, prm, 1)) &&
           sweep_prolong_ok(level_sweep(h, w, C, prm, 2)) &&
           (int64_t)sweep_partials(a0) * C < 65536 && a0.g.nby + a0.g.nbx <= kOrderMaxAxes;
}

// Size of the coarsest level a plan builds for h x w.
static void coarsest_dims(const ddi_params& prm, int h, int w, int* hl, int* wl) {
    *hl = h;
    *wl = w;
    for (int l = 1; l < level_count(h, w, prm.levels); ++l) {
        *hl = (*hl + 1) / 2;
        *wl = (*wl + 1) / 2;
    }
}

bool use_coarse_grid(const ddi_params& prm, int h, int w) {
    if (prm.coarse_solver != 1) return false;
    int hl, wl;
    coarsest_dims(prm, h, w, &hl, &wl);
    return (int64_t)hl * wl > kCoarseMaxPixels;
}

size_t plan_device_bytes(int h, int w, int C, const ddi_params& prm) {
    const int L = level_count(h, w, prm.levels);
    size_t bytes = 0, part_n = 0;
    int hl = h, wl = w;
    for (int l = 0; l < L; ++l) {
        const size_t n = (size_t)hl * wl, nf = n * C;
        if (l > 0) bytes += nf * sizeof(float) + n + nf * sizeof(float);  // f, c, u[0]
        bytes += nf * sizeof(float);                                      // u[1]
        bytes += (size_t)mask_bit_groups(hl) * wl * sizeof(uint64_t);     // mbits
        SweepArgs a;
        if (l == 0) {
            a = make_sweep(hl, wl, C, prm.block, prm.overlap, prm.robin_alpha, prm.local_iters);
        } else {
            const int cb = prm.coarse_block ? prm.coarse_block : prm.block;
            const int co = prm.coarse_overlap >= 0 ? prm.coarse_overlap : prm.overlap;
            a = make_sweep(hl, wl, C, cb, co, prm.robin_alpha, 1);
        }
        part_n = std::max(part_n, (size_t)sweep_partials(a) * C);
        part_n = std::max(part_n, (size_t)residual_partials(hl, wl) * C);
        hl = (hl + 1) / 2;
        wl = (wl + 1) / 2;
    }
    part_n = std::max(part_n, std::max<size_t>((size_t)coarsen_partials(h, w), 1024) * (C + 2));
    bytes += part_n * sizeof(double);
    bytes += (6 * (size_t)C + 2) * sizeof(double) + 64;  // red, ctl
    {
        const SweepArgs a0 = make_sweep(h, w, C, prm.block, prm.overlap, prm.robin_alpha, 1);
        if (use_skip(prm, a0)) bytes += 2 * (size_t)sweep_partials(a0) * C * sizeof(int);
        if (use_order(prm, h, w, C))
            bytes += ((size_t)sweep_partials(a0) +
                      (size_t)sweep_partials(level_sweep(h, w, C, prm, 2))) * C * sizeof(int);
    }
    if (prm.storage == 1) bytes += 3 * (size_t)C * h * w * sizeof(uint16_t);
    if (use_coarse_grid(prm, h, w)) {
        int hl, wl;
        coarsest_dims(prm, h, w, &hl, &wl);
        bytes += coarse_grid_bytes(hl, wl, C);
    }
    if (prm.method == 1)
        bytes += 4 * (size_t)C * h * w * sizeof(float) + (3 * (size_t)C + L * ((size_t)C + 2)) *
                                                             sizeof(double);
    if (prm.method == 2) {
        const size_t m = prm.krylov_restart;
        bytes += (2 * m + 1) * (size_t)C * h * w * sizeof(float) + (size_t)C * sizeof(KryState) +
                 ((m + 1) * C + 2 * (size_t)C) * sizeof(double) +
                 (size_t)residual_partials(h, w) * (m + 1) * C * sizeof(double);
    }
    if (prm.timing) {
        const SweepArgs a0 = make_sweep(h, w, C, prm.block, prm.overlap, prm.robin_alpha, 1);
        bytes += 3 * (size_t)sweep_partials(a0) * C * sizeof(double);
    }
    return bytes;
}

int check_dims(int h, int w, int channels) {
    if (h < 1 || w < 1 || channels < 1 || channels > 4) return DDI_EINVAL;
    if ((int64_t)h * w > (int64_t)1 << 30) return DDI_EINVAL;
    return DDI_OK;
}


}  // namespace ddi

namespace {

// Device scratch a step call needs, freed on scope exit.
struct Scratch {
    void* p = nullptr;
    ~Scratch() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace



extern "C" {

int ddi_default_params(ddi_params* p) {
    if (!p) return DDI_EINVAL;
    p->block = 64;
    p->overlap = 4;
    p->levels = 4;
    p->local_iters = 16;
    p->robin_alpha = 0.25f;
    p->coarse_sweeps = 2;
    p->coarsest_sweeps = 3;
    p->rel_tol = 1e-4;
    p->min_sweeps = 2;
    p->max_sweeps = 50;
    p->check_every = 1;
    p->final_residual = 1;
    p->timing = 0;
    p->coarse_block = 0;
    p->coarse_overlap = -1;
    p->coarse_local_iters = 0;
    p->local_tol = 0.f;
    p->use_graph = 0;
    p->coarse_solver = 0;
    p->coarse_cg_iters = 500;
    p->coarse_cg_tol = 1e-10;
    p->storage = 0;
    p->inner_sweeps = 2;
    p->method = 0;
    p->fuse_prolong = 1;
    p->krylov_restart = 8;
    p->skip_unchanged = 1;
    p->order_blocks = 1;
    return DDI_OK;
}

int ddi_check_params(int height, int width, int channels, const ddi_params* p) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!p) return DDI_EINVAL;
    if (p->block < 2 || p->block > DDI_MAX_BLOCK) return DDI_EINVAL;
    if (p->overlap < 0 || p->overlap >= p->block) return DDI_EINVAL;
    if (p->levels < 1 || p->levels > 16) return DDI_EINVAL;
    if (p->local_iters < 1) return DDI_EINVAL;
    if (!(p->robin_alpha > 0.f && p->robin_alpha <= 1.f)) return DDI_EINVAL;
    if (p->coarse_sweeps < 0 || p->coarsest_sweeps < 0) return DDI_EINVAL;
    if (!(p->rel_tol >= 0.0)) return DDI_EINVAL;
    if (p->min_sweeps < 0 || p->max_sweeps < p->min_sweeps) return DDI_EINVAL;
    if (p->check_every < 1) return DDI_EINVAL;
    const int cb = p->coarse_block ? p->coarse_block : p->block;
    const int co = p->coarse_overlap >= 0 ? p->coarse_overlap : p->overlap;
    if (p->coarse_block != 0 && (p->coarse_block < 2 || p->coarse_block > DDI_MAX_BLOCK))
        return DDI_EINVAL;
    if (p->coarse_overlap < -1 || co >= cb) return DDI_EINVAL;
    if (p->coarse_local_iters < 0) return DDI_EINVAL;
    if (!(p->local_tol >= 0.f) || p->local_tol > 1e6f) return DDI_EINVAL;
    if (p->use_graph != 0 && p->use_graph != 1) return DDI_EINVAL;
    if (p->coarse_solver != 0 && p->coarse_solver != 1) return DDI_EINVAL;
    if (p->coarse_cg_iters < 1 || !(p->coarse_cg_tol >= 0.0)) return DDI_EINVAL;
    if (p->storage != 0 && p->storage != 1) return DDI_EINVAL;
    if (p->inner_sweeps < 1) return DDI_EINVAL;
    if (p->method < 0 || p->method > 2) return DDI_EINVAL;
    if (p->method != 0 && p->storage != 0) return DDI_EINVAL;
    if (p->krylov_restart < 1 || p->krylov_restart > kKryMaxM) return DDI_EINVAL;
    if (p->fuse_prolong != 0 && p->fuse_prolong != 1) return DDI_EINVAL;
    if (p->skip_unchanged != 0 && p->skip_unchanged != 1) return DDI_EINVAL;
    if (p->order_blocks != 0 && p->order_blocks != 1) return DDI_EINVAL;
    return DDI_OK;
}

int ddi_destroy(ddi_plan* plan) {
    if (!plan) return DDI_OK;
    for (Level& l : plan->lv) {
        if (l.fown) (void)hipFree(l.fown);
        if (l.cown) (void)hipFree(l.cown);
        if (l.mbits) (void)hipFree(l.mbits);
        for (int i = 0; i < 2; ++i)
            if (l.u[i] && (i == 1 || l.own_u0)) (void)hipFree(l.u[i]);
    }
    if (plan->r16) (void)hipFree(plan->r16);
    if (plan->cg_vec) (void)hipFree(plan->cg_vec);
    if (plan->cg_sc) (void)hipFree(plan->cg_sc);
    if (plan->kry_vec) (void)hipFree(plan->kry_vec);
    if (plan->kry_state) (void)hipFree(plan->kry_state);
    if (plan->kry_sc) (void)hipFree(plan->kry_sc);
    if (plan->kry_part) (void)hipFree(plan->kry_part);
    for (uint16_t* d : plan->d16)
        if (d) (void)hipFree(d);
    if (plan->part) (void)hipFree(plan->part);
    if (plan->red) (void)hipFree(plan->red);
    if (plan->cgcnt) (void)hipFree(plan->cgcnt);
    if (plan->flg) (void)hipFree(plan->flg);
    if (plan->cgw) (void)hipFree(plan->cgw);
    if (plan->keys2) (void)hipFree(plan->keys2);
    if (plan->order) (void)hipFree(plan->order);
    if (plan->ctl) (void)hipFree(plan->ctl);
    if (plan->hctl) (void)hipHostFree(plan->hctl);
    if (plan->host) (void)hipHostFree(plan->host);
    if (plan->e0) (void)hipEventDestroy(plan->e0);
    if (plan->e1) (void)hipEventDestroy(plan->e1);
    if (plan->ev_ctl) (void)hipEventDestroy(plan->ev_ctl);
    for (hipEvent_t e : plan->sweep_ev) (void)hipEventDestroy(e);
    for (ddi_plan::Graph& g : plan->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (plan->ev_in) (void)hipEventDestroy(plan->ev_in);
    if (plan->gs) (void)hipStreamDestroy(plan->gs);
    delete plan;
    return DDI_OK;
}

int ddi_create(ddi_plan** out, int height, int width, int channels, const ddi_params* p,
               void* stream) {
    if (!out) return DDI_EINVAL;
    *out = nullptr;
    ddi_params prm;
    if (p)
        prm = *p;
    else
        ddi_default_params(&prm);
    int e = ddi_check_params(height, width, channels, &prm);
    if (e) return e;
    e = check_device();
    if (e) return e;

    ddi_plan* P = new (std::nothrow) ddi_plan;
    if (!P) return DDI_ENOMEM;
    P->h = height;
    P->w = width;
    P->C = channels;
    P->p = prm;
    P->s = (hipStream_t)stream;

    const int L = level_count(height, width, prm.levels);
    P->lv.resize(L);
    size_t part_n = 0;
    int hl = height, wl = width;
    for (int l = 0; l < L; ++l) {
        Level& lev = P->lv[l];
        lev.h = hl;
        lev.w = wl;
        if (l == 0) {
            lev.sw = make_sweep(hl, wl, channels, prm.block, prm.overlap, prm.robin_alpha,
                                prm.local_iters, prm.local_tol);
        } else {
            const int cb = prm.coarse_block ? prm.coarse_block : prm.block;
            const int co = prm.coarse_overlap >= 0 ? prm.coarse_overlap : prm.overlap;
            const int ck = prm.coarse_local_iters ? prm.coarse_local_iters : prm.local_iters;
            lev.sw = make_sweep(hl, wl, channels, cb, co, prm.robin_alpha, ck, prm.local_tol);
        }
        const size_t n = (size_t)hl * wl;
        const size_t nf = n * channels;
        auto fail = [&](hipError_t err) {
            ddi_destroy(P);
            if (err == hipErrorOutOfMemory) return DDI_ENOMEM;
            return hip_fail(err);
        };
        hipError_t err;
        if (l > 0) {
            if ((err = hipMalloc(&lev.fown, nf * sizeof(float))) != hipSuccess) return fail(err);
            if ((err = hipMalloc(&lev.cown, n)) != hipSuccess) return fail(err);
            if ((err = hipMalloc(&lev.u[0], nf * sizeof(float))) != hipSuccess) return fail(err);
            lev.own_u0 = true;
            lev.f = lev.fown;
            lev.c = lev.cown;
        }
        if ((err = hipMalloc(&lev.u[1], nf * sizeof(float))) != hipSuccess) return fail(err);
        if ((err = hipMalloc(&lev.mbits, (size_t)mask_bit_groups(hl) * wl * sizeof(uint64_t))) !=
            hipSuccess)
            return fail(err);
        part_n = std::max(part_n, (size_t)sweep_partials(lev.sw) * channels);
        const size_t res_wg = (size_t)residual_partials(hl, wl);
        part_n = std::max(part_n, res_wg * channels);
        hl = (hl + 1) / 2;
        wl = (wl + 1) / 2;
    }
    // statistics partials: the first coarsening (level 0 -> 1) or, for a
    // single level, the statistics kernel (at most 1024 workgroups)
    {
        const size_t nwg = std::max<size_t>((size_t)coarsen_partials(height, width), 1024);
        part_n = std::max(part_n, nwg * (channels + 2));
    }
    P->part_n = part_n;
    hipError_t err;
    if ((err = hipMalloc(&P->part, part_n * sizeof(double))) != hipSuccess) {
        ddi_destroy(P);
        return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
    }
    const size_t nred = 6 * channels + 2;
    if ((err = hipMalloc(&P->red, nred * sizeof(double))) != hipSuccess ||
        (err = hipHostMalloc(&P->host, nred * sizeof(double), hipHostMallocDefault)) !=
            hipSuccess ||
        (err = hipMalloc(&P->ctl, 64)) != hipSuccess ||
        (err = hipHostMalloc(&P->hctl, 64, hipHostMallocDefault)) != hipSuccess ||
        // e0 only starts the solve's timer: no system-scope fence
        (err = hipEventCreateWithFlags(&P->e0, hipEventDisableSystemFence)) != hipSuccess ||
        (err = hipEventCreate(&P->e1)) != hipSuccess ||
        (err = hipEventCreate(&P->ev_ctl)) != hipSuccess) {
        ddi_destroy(P);
        return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
    }
    // the stop test writes the control words' host copy itself (pinned
    // memory the device can address); without that address, a copy after it
    void* dm = nullptr;
    if (hipHostGetDevicePointer(&dm, P->hctl, 0) == hipSuccess && dm)
        P->dmirror = static_cast<int*>(dm);
    else
        (void)hipGetLastError();
    if (prm.storage == 1) {
        const size_t nv = (size_t)channels * height * width * sizeof(uint16_t);
        if ((err = hipMalloc(&P->r16, nv)) != hipSuccess ||
            (err = hipMalloc(&P->d16[0], nv)) != hipSuccess ||
            (err = hipMalloc(&P->d16[1], nv)) != hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
    }
    if (prm.method == 1) {
        const size_t nv = (size_t)channels * height * width * sizeof(float);
        if ((err = hipMalloc(&P->cg_vec, 4 * nv)) != hipSuccess ||
            (err = hipMalloc(&P->cg_sc, (size_t)(3 * channels + L * (channels + 2)) *
                                            sizeof(double))) != hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
        P->last_iters.assign(L, -1);
    }
    if (prm.method == 2) {
        const size_t m = prm.krylov_restart;
        const size_t nv = (size_t)channels * height * width * sizeof(float);
        if ((err = hipMalloc(&P->kry_vec, (2 * m + 1) * nv)) != hipSuccess ||
            (err = hipMalloc(&P->kry_state, (size_t)channels * sizeof(KryState))) !=
                hipSuccess ||
            (err = hipMalloc(&P->kry_sc, ((m + 1) * channels + 2 * (size_t)channels) *
                                             sizeof(double))) != hipSuccess ||
            (err = hipMalloc(&P->kry_part, (size_t)residual_partials(height, width) * (m + 1) *
                                               channels * sizeof(double))) != hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
    }
    if (prm.use_graph && !prm.timing && prm.storage == 0 && prm.method == 0) {
        // a stream of our own (default priority): the caller's may be the
        // legacy default stream, which cannot be captured
        if ((err = hipStreamCreate(&P->gs)) != hipSuccess ||
            (err = hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming)) != hipSuccess) {
            ddi_destroy(P);
            return hip_fail(err);
        }
    }
    if (use_skip(prm, P->lv[0].sw)) {
        const size_t nfl = 2 * (size_t)sweep_partials(P->lv[0].sw) * channels;
        if ((err = hipMalloc(&P->flg, nfl * sizeof(int))) != hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
    }
    if (use_order(prm, height, width, channels)) {
        const size_t nfl = (size_t)sweep_partials(P->lv[0].sw) * channels;
        const size_t nk = (size_t)sweep_partials(P->lv[2].sw) * channels;
        if ((err = hipMalloc(&P->order, nfl * sizeof(int))) != hipSuccess ||
            (err = hipMalloc(&P->keys2, nk * sizeof(int))) != hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
    }
    if (use_coarse_grid(prm, height, width)) {
        const Level& top = P->lv.back();
        if ((err = hipMalloc(&P->cgw, coarse_grid_bytes(top.h, top.w, channels))) !=
            hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
    }
    if (prm.timing) {
        const size_t nc = 3 * (size_t)sweep_partials(P->lv[0].sw) * channels;
        if ((err = hipMalloc(&P->cgcnt, nc * sizeof(double))) != hipSuccess) {
            ddi_destroy(P);
            return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
        }
        if ((err = launch_clear(P->cgcnt, (int)nc, P->s)) != hipSuccess ||
            (err = hipStreamSynchronize(P->s)) != hipSuccess) {
            ddi_destroy(P);
            return hip_fail(err);
        }
        const int per = prm.storage == 1 ? prm.inner_sweeps : 1;
        P->sweep_ev.assign(2 * (size_t)std::max(prm.max_sweeps, 1) * per, nullptr);
        // timing-only events: no system-scope fence (no L2 writeback and
        // invalidate between sweeps); the host reads their times only after
        // synchronizing on a later default event of the same stream
        for (hipEvent_t& ev : P->sweep_ev) {
            if ((err = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence)) != hipSuccess) {
                ddi_destroy(P);
                return hip_fail(err);
            }
        }
    }
    P->bytes = plan_device_bytes(height, width, channels, prm);
    *out = P;
    return DDI_OK;
}

int ddi_plan_footprint(int height, int width, int channels, const ddi_params* p,
                       size_t* bytes) {
    if (!bytes) return DDI_EINVAL;
    ddi_params prm;
    if (p)
        prm = *p;
    else
        ddi_default_params(&prm);
    const int e = ddi_check_params(height, width, channels, &prm);
    if (e) return e;
    *bytes = plan_device_bytes(height, width, channels, prm);
    return DDI_OK;
}

int ddi_plan_bytes(const ddi_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return DDI_EINVAL;
    *bytes = plan->bytes;
    return DDI_OK;
}

// max over channels of sqrt(rsq / ||b||^2); the stats occupy host[0..C+2).
static double rel_from_host(const ddi_plan* P, const double* rsq) {
    double worst = 0.0;
    for (int k = 0; k < P->C; ++k) {
        const double b2 = P->host[k];
        double rel;
        if (b2 > 0.0)
            rel = std::sqrt(rsq[k] / b2);
        else
            rel = rsq[k] > 0.0 ? INFINITY : 0.0;
        worst = std::max(worst, rel);
    }
    return worst;
}

// Pyramid, input statistics, transposed masks, coarsest level and the
// coarse-to-fine passes down to the start of the finest level, enqueued on
// `s`. The finest level starts in buffer `start0` (0 = u). With
// fuse_prolong, the first sweep on each coarser level reads the level
// above it directly; fuse_l0 extends that to the finest level, whose
// prolongation is then left to enqueue_sweeps (P->pro0).
static int enqueue_front(ddi_plan* P, int start0, hipStream_t s, bool fuse_l0) {
    return plan_enqueue_front(P, start0, s, fuse_l0);
}

}  // extern "C"

int plan_enqueue_front(ddi_plan* P, int start0, hipStream_t s, bool fuse_l0) {
    const int C = P->C;
    const int L = (int)P->lv.size();
    const ddi_params& prm = P->p;
    const Level& L0 = P->lv[0];
    int nwg = 0;
    if (L > 1)
        DDI_HIP(launch_coarsen(L0.f, L0.c, P->h, P->w, C, P->lv[1].fown, P->lv[1].cown, P->part,
                               &nwg, s));
    else
        DDI_HIP(launch_stats(L0.f, L0.c, P->h, P->w, C, P->part, &nwg, s));
    // the statistics' column sums (P->part -> P->red) run in the transposed-
    // mask launch below; nothing writes P->part before it
    // the coarser levels two at a time where the widths allow it (one launch
    // makes both, bit for bit as two would)
    for (int l = 1; l + 1 < L;) {
        Level& a = P->lv[l];
        Level& b = P->lv[l + 1];
        if (l + 2 < L) {
            Level& d = P->lv[l + 2];
            if (coarsen2_ok(a.f, a.c, b.fown, b.cown, d.fown, d.cown, a.w)) {
                DDI_HIP(launch_coarsen2(a.f, a.c, a.h, a.w, C, b.fown, b.cown, d.fown, d.cown, s));
                l += 2;
                continue;
            }
        }
        DDI_HIP(launch_coarsen(a.f, a.c, a.h, a.w, C, b.fown, b.cown, nullptr, nullptr, s));
        ++l;
    }
    {
        const uint8_t* cs[kMaxLevels];
        uint64_t* mbs[kMaxLevels];
        int hs[kMaxLevels], ws[kMaxLevels];
        for (int l = 0; l < L; ++l) {
            cs[l] = P->lv[l].c;
            mbs[l] = P->lv[l].mbits;
            hs[l] = P->lv[l].h;
            ws[l] = P->lv[l].w;
        }
        // the same launch clears the stop-test control word of this solve,
        // sums the input statistics and, unless the coarsest level is solved
        // in float64, makes its initial guess u = c ? f : 0
        const int top = L - 1;
        const int cur = (top == 0) ? start0 : 0;
        const Level& t = P->lv[top];
        const InitJob ini{t.f, t.c, t.u[cur], (int64_t)t.h * t.w, C};
        DDI_HIP(launch_mask_bits_levels(L, cs, hs, ws, mbs, s, P->ctl, 4, P->part, nwg, C + 2,
                                        C + 2, P->red, prm.coarse_solver == 1 ? nullptr : &ini));
    }
    const int top = L - 1;
    int cur = (top == 0) ? start0 : 0;
    if (prm.coarse_solver == 1 && P->cgw) {
        const Level& t = P->lv[top];
        DDI_HIP(launch_coarse_cg_grid(t.f, t.c, t.h, t.w, C, t.u[cur], prm.coarse_cg_iters,
                                      prm.coarse_cg_tol, coarse_grid_workgroups(t.h, t.w, C),
                                      P->cgw, P->ctl, s));
    } else if (prm.coarse_solver == 1)
        DDI_HIP(launch_coarse_cg(P->lv[top].f, P->lv[top].c, P->lv[top].h, P->lv[top].w, C,
                                 P->lv[top].u[cur], prm.coarse_cg_iters, prm.coarse_cg_tol, s));
    // (otherwise the initial guess came with the transposed masks)
    P->pro0_on = false;
    P->order_on = false;
    // set: this level's first sweep prolongs from it (only when the level
    // has coarse_sweeps > 0 sweeps to fuse into)
    const ProSrc* from = nullptr;
    ProSrc src;
    for (int l = top; l >= 1; --l) {
        Level& lev = P->lv[l];
        const int n = (l == top) ? (prm.coarse_solver == 1 ? 0 : prm.coarsest_sweeps)
                                 : prm.coarse_sweeps;
        // order_blocks: level 2 leaves its blocks' CG steps, and the first
        // level-1 sweep turns them into the dispatch table of the finest
        // level's first sweep in an extra workgroup
        int* kout = (l == 2 && P->keys2) ? P->keys2 : nullptr;
        OrderArgs job;
        const OrderArgs* jp = nullptr;
        if (l == 1 && P->order && n > 0) {
            job.keys = P->keys2;
            job.order = P->order;
            job.g = L0.sw.g;
            job.cg = P->lv[2].sw.g;
            job.channels = C;
            job.scale = 4;
            jp = &job;
            P->order_on = true;
        }
        for (int i = 0; i < n; ++i) {
            if (i == 0 && from)
                DDI_HIP(launch_sweep_prolong(*from, lev.mbits, lev.u[1 - cur], P->part, nullptr,
                                             nullptr, lev.sw, s, kout, nullptr,
                                             i == 0 ? jp : nullptr));
            else
                DDI_HIP(launch_sweep(lev.u[cur], lev.mbits, lev.u[1 - cur], P->part, nullptr,
                                     nullptr, lev.sw, s, nullptr, kout, nullptr,
                                     i == 0 ? jp : nullptr));
            cur ^= 1;
        }
        from = nullptr;
        Level& fine = P->lv[l - 1];
        const int dst = (l == 1) ? start0 : 0;
        const bool fuse = prm.fuse_prolong == 1 && sweep_prolong_ok(fine.sw) &&
                          (l == 1 ? fuse_l0 : prm.coarse_sweeps > 0);
        if (fuse) {
            src = ProSrc{lev.u[cur], lev.h, lev.w, fine.f, fine.c};
            from = &src;
            if (l == 1) {
                P->pro0 = src;
                P->pro0_on = true;
            }
        } else {
            DDI_HIP(launch_prolong(lev.u[cur], lev.h, lev.w, fine.f, fine.c, fine.h, fine.w, C,
                                   fine.u[dst], s));
        }
        cur = dst;
    }
    return DDI_OK;
}

extern "C" {

static bool is_check(const ddi_params& prm, int n) {
    return n >= prm.min_sweeps && (n - prm.min_sweeps) % prm.check_every == 0;
}

// Finest-level sweeps [from, to) starting from buffer start0, each followed
// by the device stop test where it applies (and after the last allowed).
static int enqueue_sweeps(ddi_plan* P, int from, int to, int start0, bool timing,
                          hipStream_t s) {
    const ddi_params& prm = P->p;
    Level& L0 = P->lv[0];
    const int nb = sweep_partials(L0.sw);
    int* ctl = P->ctl;
    double* drel = reinterpret_cast<double*>(ctl + 4);
    for (int i = from; i < to; ++i) {
        const int c0 = start0 ^ (i & 1);
        // every sweep runs its blocks in the order built by level 1: the
        // blocks the coarse level found heavy stay the ones that take most
        // CG steps in the later sweeps too, so they start first in each
        const int* order = P->order_on ? P->order : nullptr;
        // with timing, the launch records the kernel's own start and end
        hipEvent_t ev0 = timing ? P->sweep_ev[2 * i] : nullptr;
        hipEvent_t ev1 = timing ? P->sweep_ev[2 * i + 1] : nullptr;
        if (i == 0 && P->pro0_on)
            DDI_HIP(launch_sweep_prolong(P->pro0, L0.mbits, L0.u[c0 ^ 1], P->part,
                                         timing ? P->cgcnt : nullptr, ctl, L0.sw, s, nullptr,
                                         order, nullptr, ev0, ev1));
        else if (i == 0 && order)
            DDI_HIP(launch_sweep(L0.u[c0], L0.mbits, L0.u[c0 ^ 1], P->part,
                                 timing ? P->cgcnt : nullptr, ctl, L0.sw, s, nullptr,
                                 P->flg ? P->flg + (i & 1) * nb * P->C : nullptr, order, nullptr,
                                 ev0, ev1));
        else if (P->flg) {
            // sweep i writes the flags of parity i & 1 and reads those of the
            // sweep before (from the third sweep on: the first sweep's
            // output buffer is the only one the solve has written yet)
            const int nfl = nb * P->C;
            DDI_HIP(launch_sweep(L0.u[c0], L0.mbits, L0.u[c0 ^ 1], P->part,
                                 timing ? P->cgcnt : nullptr, ctl, L0.sw, s,
                                 i >= 2 ? P->flg + ((i - 1) & 1) * nfl : nullptr,
                                 P->flg + (i & 1) * nfl, order, nullptr, ev0, ev1));
        } else {
            DDI_HIP(launch_sweep(L0.u[c0], L0.mbits, L0.u[c0 ^ 1], P->part,
                                 timing ? P->cgcnt : nullptr, ctl, L0.sw, s, nullptr, nullptr,
                                 nullptr, nullptr, ev0, ev1));
        }
        if (timing && i == 0)  // the first sweep's CG steps on their own
            DDI_HIP(launch_reduce(P->cgcnt, nb, P->C, P->C, P->red + 3 * P->C + 2, s));
        if (is_check(prm, i + 1) || i + 1 == prm.max_sweeps)
            DDI_HIP(launch_decide(P->part, nb, P->C, P->red, ctl, drel,
                                  is_check(prm, i + 1) ? prm.rel_tol : -1.0, i + 1, s,
                                  P->dmirror));
    }
    return DDI_OK;
}

// storage = 1: the coarse-to-fine start (built by the first residual pass
// where the finest level's start can be fused), then refinement steps k =
// 0, 1, ...: r_k = b - A u_k (bfloat16, float64 norm, device stop test), then
// inner_sweeps correction sweeps on A d = r_k from d = 0 (bfloat16), and
// u_{k+1} = u_k + d fused into the next residual pass. u_k lives in buffer
// start0 ^ (k & 1) of the finest level; steps are enqueued ahead in batches
// like the float32 sweeps, and exit at once after the stop test passed.
static int solve_refine(ddi_plan* P, const float* f, const uint8_t* c, float* u, ddi_stats* st) {
    const int C = P->C;
    const ddi_params& prm = P->p;
    Level& L0 = P->lv[0];
    const bool timing = !P->sweep_ev.empty();
    hipStream_t s = P->s;
    const int m = prm.inner_sweeps;
    const int kmax = prm.max_sweeps;
    DDI_HIP(hipEventRecord(P->e0, s));
    const int expect = P->last_sweeps >= 0 ? P->last_sweeps : std::max(prm.min_sweeps, 1);
    const int start0 = std::min(expect, kmax) & 1;
    // also clears the control word; where the finest level's start can be
    // fused (P->pro0_on), the first residual pass builds it
    int e = enqueue_front(P, start0, s, true);
    if (e) return e;
    int* ctl = P->ctl;
    double* drel = reinterpret_cast<double*>(ctl + 4);
    const int nres = residual_partials(P->h, P->w);
    auto enqueue_steps = [&](int from, int to) -> int {
        for (int k = from; k < to; ++k) {
            const int a = start0 ^ (k & 1);
            const float* usrc = k == 0 ? L0.u[start0] : L0.u[a ^ 1];
            const uint16_t* dk = k == 0 ? nullptr : P->d16[(m - 1) & 1];
            if (k == 0 && P->pro0_on)
                DDI_HIP(launch_start_residual(P->pro0, P->h, P->w, C, L0.u[start0], P->r16,
                                              P->part, ctl, nullptr, s));
            else
                DDI_HIP(launch_refine_residual(f, c, usrc, dk, P->h, P->w, C,
                                               k == 0 ? nullptr : L0.u[a], P->r16, P->part, ctl,
                                               nullptr, s));
            const bool chk = is_check(prm, k);
            if (chk || k == kmax)
                DDI_HIP(launch_decide(P->part, nres, C, P->red, ctl, drel, chk ? prm.rel_tol : -1.0,
                                      k, s));
            if (k == kmax) break;
            for (int j = 0; j < m; ++j) {
                const int ev = k * m + j;
                if (timing) DDI_HIP(hipEventRecord(P->sweep_ev[2 * ev], s));
                DDI_HIP(launch_sweep_corr(j == 0 ? nullptr : P->d16[(j - 1) & 1], P->r16, L0.mbits,
                                          P->d16[j & 1], P->part, timing ? P->cgcnt : nullptr, ctl,
                                          L0.sw, s));
                if (timing) DDI_HIP(hipEventRecord(P->sweep_ev[2 * ev + 1], s));
            }
        }
        return DDI_OK;
    };
    int done = 0, k_end = kmax;
    bool converged = false;
    double rel = INFINITY;
    int batch = std::min(kmax + 1, expect + 1);
    while (done <= kmax) {
        const int to = std::min(kmax + 1, done + batch);
        if ((e = enqueue_steps(done, to))) return e;
        done = to;
        batch = 2;
        DDI_HIP(hipMemcpyAsync(P->hctl, P->ctl, 4 * sizeof(int) + sizeof(double),
                               hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
        const int* hc = reinterpret_cast<const int*>(P->hctl);
        if (hc[2] == 1) return DDI_EINVAL;
        if (hc[2] == 2) return DDI_ESINGULAR;
        if (hc[2] == 3) return DDI_ESTALL;
        double rel2;
        std::memcpy(&rel2, hc + 4, sizeof(rel2));
        rel = std::sqrt(rel2);
        if (hc[0] != 0) {
            k_end = hc[1];
            converged = true;
            break;
        }
    }
    P->last_sweeps = k_end;
    const int cur = start0 ^ (k_end & 1);
    if (cur == 1)
        DDI_HIP(hipMemcpyAsync(u, L0.u[1], (size_t)C * P->h * P->w * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    if (timing) {
        const int nb = sweep_partials(L0.sw);
        DDI_HIP(launch_reduce(P->cgcnt, nb, C, C, P->red + 2 * C + 2, s, true));
        DDI_HIP(hipMemcpyAsync(P->host + 2 * C + 2, P->red + 2 * C + 2, C * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    DDI_HIP(hipEventRecord(P->e1, s));
    DDI_HIP(hipEventSynchronize(P->e1));
    float ms = 0.f;
    DDI_HIP(hipEventElapsedTime(&ms, P->e0, P->e1));
    double sweep_ms = 0.0, nsteps = 0.0;
    P->sweep_ms.clear();
    for (int i = 0; timing && i < k_end * m; ++i) {
        float t = 0.f;
        DDI_HIP(hipEventElapsedTime(&t, P->sweep_ev[2 * i], P->sweep_ev[2 * i + 1]));
        sweep_ms += t;
        P->sweep_ms.push_back(t);  // the correction sweeps, in order
    }
    for (int k = 0; timing && k < C; ++k) nsteps += P->host[2 * C + 2 + k];
    if (st) {
        st->sweeps = k_end * m;
        st->refinements = k_end;
        st->converged = converged ? 1 : 0;
        st->rel_residual = rel;
        st->ms = ms;
        st->sweep_ms = sweep_ms;
        st->cg_steps = nsteps;
    }
    return converged ? DDI_OK : DDI_ENOCONV;
}

static int enqueue_check(ddi_plan* P);

// Enqueues a solve up to the first host check: pyramid, coarse levels, the
// first batch of finest-level sweeps with their device stop tests, then the
// read-back of the control word (and, with timing, of the CG step counts),
// recorded by ev_ctl. The finest level ping-pongs between u (index 0) and
// the plan's buffer (index 1). It starts in the buffer that makes the
// expected final iterate -- as many sweeps as the previous solve needed --
// land in u, so that usually no copy is needed at the end. Once a stop test
// passes, the sweeps still enqueued exit at once.
static int begin_solve(ddi_plan* P, const float* f, const uint8_t* c, float* u) {
    const ddi_params& prm = P->p;
    Level& L0 = P->lv[0];
    L0.f = f;
    L0.c = c;
    L0.u[0] = u;
    ddi_plan::Pending& q = P->pend;
    q = ddi_plan::Pending();
    q.f = f;
    q.c = c;
    q.u = u;
    q.timing = !P->sweep_ev.empty();
    const bool graph = P->gs != nullptr;
    hipStream_t s = graph ? P->gs : P->s;
    q.s = s;
    if (graph) {
        // order the plan's stream after work the caller queued before
        DDI_HIP(hipEventRecord(P->ev_in, P->s));
        DDI_HIP(hipStreamWaitEvent(s, P->ev_in, 0));
    }
    DDI_HIP(hipEventRecord(P->e0, s));

    const int expect = P->last_sweeps >= 0 ? P->last_sweeps : std::max(prm.min_sweeps, 1);
    q.start0 = std::min(expect, prm.max_sweeps) & 1;
    int batch = std::min(prm.max_sweeps, std::max(expect, prm.min_sweeps));
    if (batch > 0) {
        int upto = std::max(1, batch);
        while (upto < prm.max_sweeps && !is_check(prm, upto)) ++upto;
        batch = std::min(upto, prm.max_sweeps);
    }
    if (q.timing) DDI_HIP(launch_clear(P->cgcnt, 3 * sweep_partials(L0.sw) * P->C, s));

    if (graph) {
        // one graph per (f, c, u, start buffer, first batch); later solves
        // with the same key replay it
        ddi_plan::Graph* hit = nullptr;
        for (ddi_plan::Graph& gr : P->graphs)
            if (gr.exec && gr.f == f && gr.c == c && gr.u == u && gr.start == q.start0 &&
                gr.batch == batch)
                hit = &gr;
        if (!hit) {
            // replace the least recently used entry
            hit = &P->graphs[0];
            for (ddi_plan::Graph& gr : P->graphs)
                if (gr.last_use < hit->last_use) hit = &gr;
            if (hit->exec) {
                (void)hipGraphExecDestroy(hit->exec);
                hit->exec = nullptr;
            }
            hipGraph_t g = nullptr;
            DDI_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            int e = enqueue_front(P, q.start0, s, batch > 0);  // clears the control word
            if (!e) e = enqueue_sweeps(P, 0, batch, q.start0, false, s);
            hipError_t he = hipStreamEndCapture(s, &g);
            if (e) {
                if (g) (void)hipGraphDestroy(g);
                return e;
            }
            if (he != hipSuccess) return hip_fail(he);
            he = hipGraphInstantiate(&hit->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (he != hipSuccess) {
                hit->exec = nullptr;
                return hip_fail(he);
            }
            hit->f = f;
            hit->c = c;
            hit->u = u;
            hit->start = q.start0;
            hit->batch = batch;
        }
        hit->last_use = ++P->graph_clock;
        DDI_HIP(hipGraphLaunch(hit->exec, s));
        q.done_upto = batch;
    } else {
        int e = enqueue_front(P, q.start0, s, batch > 0);  // clears the control word
        if (e) return e;
        e = enqueue_sweeps(P, 0, batch, q.start0, q.timing, s);
        if (e) return e;
        q.done_upto = batch;
    }
    // every path that ran sweeps ended with a stop test that wrote the mirror
    q.mirrored = batch > 0 && P->dmirror != nullptr;
    q.active = true;
    return enqueue_check(P);
}

// Read-back of the control word (and of the CG step counts with timing),
// recorded by ev_ctl.
static int enqueue_check(ddi_plan* P) {
    const int C = P->C;
    hipStream_t s = P->pend.s;
    if (P->pend.timing) {
        const int nb = sweep_partials(P->lv[0].sw);
        DDI_HIP(launch_reduce(P->cgcnt, nb, C, C, P->red + 2 * C + 2, s));
        DDI_HIP(launch_reduce(P->cgcnt + (size_t)nb * C, nb, C, C, P->red + 4 * C + 2, s));
        DDI_HIP(launch_reduce(P->cgcnt + 2 * (size_t)nb * C, nb, C, C, P->red + 5 * C + 2, s));
        DDI_HIP(hipMemcpyAsync(P->host + 2 * C + 2, P->red + 2 * C + 2, 4 * C * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    if (!P->pend.mirrored)
        DDI_HIP(hipMemcpyAsync(P->hctl, P->ctl, 4 * sizeof(int) + sizeof(double),
                               hipMemcpyDeviceToHost, s));
    P->pend.mirrored = false;
    DDI_HIP(hipEventRecord(P->ev_ctl, s));
    return DDI_OK;
}

// Waits for the enqueued sweeps, enqueues more batches while the stop test
// has not passed, then finishes: the optional final residual, the move of
// the result into u, and the statistics. Only this plan's work is waited for
// (events), so solves of other plans queued behind it keep the GPU busy.
static int finish_solve(ddi_plan* P, ddi_stats* st) {
    ddi_plan::Pending& q = P->pend;
    if (!q.active) return DDI_EINVAL;
    q.active = false;
    const int C = P->C;
    const ddi_params& prm = P->p;
    Level& L0 = P->lv[0];
    hipStream_t s = q.s;
    const float* f = q.f;
    const uint8_t* c = q.c;
    float* u = q.u;
    if (st) std::memset(st, 0, sizeof(*st));

    bool validated = false, converged = false;
    double rel = INFINITY;
    int sweeps = 0;
    int done_upto = q.done_upto;
    for (;;) {
        DDI_HIP(hipEventSynchronize(P->ev_ctl));
        const int* hc = reinterpret_cast<const int*>(P->hctl);
        validated = done_upto > 0;
        if (hc[2] == 1) return DDI_EINVAL;
        if (hc[2] == 2) return DDI_ESINGULAR;
        if (hc[2] == 3) return DDI_ESTALL;
        if (done_upto > 0) {
            double rel2;
            std::memcpy(&rel2, hc + 4, sizeof(rel2));
            rel = std::sqrt(rel2);
        }
        if (hc[0] != 0) {
            sweeps = hc[1];
            converged = true;
            break;
        }
        sweeps = done_upto;
        if (done_upto >= prm.max_sweeps) break;
        int upto = std::min(prm.max_sweeps, done_upto + 2);
        while (upto < prm.max_sweeps && !is_check(prm, upto)) ++upto;
        int e = enqueue_sweeps(P, done_upto, upto, q.start0, q.timing, s);
        if (e) return e;
        done_upto = upto;
        q.mirrored = P->dmirror != nullptr;
        if ((e = enqueue_check(P))) return e;
    }
    int cur = q.start0 ^ (sweeps & 1);
    P->last_sweeps = sweeps;

    // ---- final residual of the returned iterate; move it into u ----
    hipEvent_t end = P->ev_ctl;
    if (prm.final_residual || !validated) {
        int rwg = 0;
        DDI_HIP(launch_residual(f, c, L0.u[cur], P->h, P->w, C, nullptr,
                                cur == 1 ? u : nullptr, P->part, &rwg, s));
        DDI_HIP(launch_reduce(P->part, rwg, C, C, P->red + C + 2, s));
        DDI_HIP(hipMemcpyAsync(P->host, P->red, (2 * C + 2) * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        DDI_HIP(hipEventRecord(P->e1, s));
        DDI_HIP(hipEventSynchronize(P->e1));
        end = P->e1;
        validated = true;
        if (P->host[C + 1] > 0.0) return DDI_EINVAL;
        if (P->host[C] <= 0.0) return DDI_ESINGULAR;
        if (prm.final_residual) {
            rel = rel_from_host(P, P->host + C + 2);
            converged = rel <= prm.rel_tol || converged;
        }
    } else if (cur == 1) {
        DDI_HIP(hipMemcpyAsync(u, L0.u[1], (size_t)C * P->h * P->w * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
        DDI_HIP(hipEventRecord(P->e1, s));
        DDI_HIP(hipEventSynchronize(P->e1));
        end = P->e1;
    }
    double nsteps = 0.0, steps0 = 0.0, nskip = 0.0, nunwr = 0.0;
    for (int k = 0; q.timing && k < C; ++k) {
        nsteps += P->host[2 * C + 2 + k];
        steps0 += P->host[3 * C + 2 + k];
        nskip += P->host[4 * C + 2 + k];
        nunwr += P->host[5 * C + 2 + k];
    }
    float ms = 0.f;
    DDI_HIP(hipEventElapsedTime(&ms, P->e0, end));
    double sweep_ms = 0.0, first_ms = 0.0;
    P->sweep_ms.clear();
    for (int i = 0; q.timing && i < sweeps; ++i) {
        float t = 0.f;
        DDI_HIP(hipEventElapsedTime(&t, P->sweep_ev[2 * i], P->sweep_ev[2 * i + 1]));
        sweep_ms += t;
        P->sweep_ms.push_back(t);
        if (i == 0) first_ms = t;
    }
    if (st) {
        st->sweeps = sweeps;
        st->converged = converged ? 1 : 0;
        st->rel_residual = rel;
        st->ms = ms;
        st->sweep_ms = sweep_ms;
        st->cg_steps = nsteps;
        st->first_sweep_ms = first_ms;
        st->first_cg_steps = steps0;
        st->skipped_blocks = nskip;
        st->unwritten_blocks = nunwr;
    }
    return converged ? DDI_OK : DDI_ENOCONV;
}

// u (written) must not share memory with f or c (read throughout the solve).
static bool solve_aliases(const ddi_plan* P, const float* f, const uint8_t* c, const float* u) {
    const size_t nimg = (size_t)P->C * P->h * P->w * sizeof(float);
    return overlaps(u, nimg, f, nimg) || overlaps(u, nimg, c, (size_t)P->h * P->w);
}

int ddi_solve(ddi_plan* P, const float* f, const uint8_t* c, float* u, ddi_stats* st) {
    if (!P || !f || !c || !u) return DDI_EINVAL;
    if (P->pend.active || solve_aliases(P, f, c, u)) return DDI_EINVAL;
    if (P->p.storage == 1 || P->p.method != 0) {
        Level& L0 = P->lv[0];
        L0.f = f;
        L0.c = c;
        L0.u[0] = u;
        if (st) std::memset(st, 0, sizeof(*st));
        if (P->p.method == 1) return solve_mlcg(P, st);
        if (P->p.method == 2) return solve_krylov(P, st);
        return solve_refine(P, f, c, u, st);
    }
    int e = begin_solve(P, f, c, u);
    if (e) {
        P->pend.active = false;
        return e;
    }
    return finish_solve(P, st);
}

int ddi_solve_async(ddi_plan* P, const float* f, const uint8_t* c, float* u) {
    if (!P || !f || !c || !u || solve_aliases(P, f, c, u)) return DDI_EINVAL;
    if (P->pend.active || P->p.storage != 0 || P->p.method != 0) return DDI_EINVAL;
    int e = begin_solve(P, f, c, u);
    if (e) P->pend.active = false;
    return e;
}

int ddi_solve_wait(ddi_plan* P, ddi_stats* st) {
    if (!P || !P->pend.active) return DDI_EINVAL;
    return finish_solve(P, st);
}

const char* ddi_strerror(int code) {
    switch (code) {
        case DDI_OK: return "ok";
        case DDI_EINVAL: return "invalid argument";
        case DDI_ESINGULAR: return "mask has no known pixel (singular system)";
        case DDI_ENOMEM: return "out of device memory";
        case DDI_ENOCONV: return "no convergence within max_sweeps";
        case DDI_EHIP: return "HIP runtime error";
        case DDI_ENODEV: return "no gfx950 device";
        case DDI_ESCRATCH: return "input too large for the fixed no-allocation scratch";
        case DDI_ESTALL: return "a grid barrier of the float64 coarse solve timed out";
        default: return "unknown error";
    }
}

int ddi_last_hip_error(void) { return g_last_hip; }

int ddi_sweep_times(const ddi_plan* P, double* ms, int n, int* count) {
    if (!P || n < 0 || (n > 0 && !ms)) return DDI_EINVAL;
    const int m = (int)P->sweep_ms.size();
    for (int i = 0; i < std::min(n, m); ++i) ms[i] = P->sweep_ms[i];
    if (count) *count = m;
    return DDI_OK;
}

int ddi_block_count(int n, int block, int overlap) {
    if (n < 1 || block < 1 || overlap < 0 || overlap >= block) return DDI_EINVAL;
    return block_count(n, block, overlap);
}

int ddi_block_range(int n, int block, int overlap, int k, int* origin, int* own_lo,
                    int* own_hi) {
    const int nb = ddi_block_count(n, block, overlap);
    if (nb < 0 || k < 0 || k >= nb) return DDI_EINVAL;
    const BlockGrid g = make_grid(n, n, block, overlap);
    int lo, hi;
    owner_range(k, nb, g.sx, n, g.bw, &lo, &hi);
    if (origin) *origin = block_origin(k, g.sx, n, g.bw);
    if (own_lo) *own_lo = lo;
    if (own_hi) *own_hi = hi;
    return DDI_OK;
}

// ---- steps one by one ----

int ddi_residual(const float* f, const uint8_t* c, const float* u, int height, int width,
                 int channels, float* r, double* rsq, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!f || !c || !u) return DDI_EINVAL;
    const size_t nimg = (size_t)channels * height * width * sizeof(float);
    if (overlaps(r, nimg, f, nimg) || overlaps(r, nimg, u, nimg) ||
        overlaps(r, nimg, c, (size_t)height * width))
        return DDI_EINVAL;
    if ((e = check_device())) return e;
    hipStream_t s = (hipStream_t)stream;
    const size_t nwg = (size_t)residual_partials(height, width);
    Scratch part, red;
    DDI_HIP(hipMalloc(&part.p, nwg * channels * sizeof(double)));
    DDI_HIP(hipMalloc(&red.p, channels * sizeof(double)));
    int n = 0;
    DDI_HIP(launch_residual(f, c, u, height, width, channels, r, nullptr, (double*)part.p, &n, s));
    DDI_HIP(launch_reduce((double*)part.p, n, channels, channels, (double*)red.p, s));
    if (rsq) {
        DDI_HIP(hipMemcpyAsync(rsq, red.p, channels * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    DDI_HIP(hipStreamSynchronize(s));
    return DDI_OK;
}

int ddi_coarsen(const float* f, const uint8_t* c, int height, int width, int channels,
                float* fc, uint8_t* cc, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!f || !c || !fc || !cc) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        const size_t ncs = (size_t)((height + 1) / 2) * ((width + 1) / 2);
        const size_t hw = (size_t)height * width;
        if (overlaps(fc, channels * ncs * sizeof(float), f, nimg) ||
            overlaps(fc, channels * ncs * sizeof(float), c, hw) || overlaps(cc, ncs, f, nimg) ||
            overlaps(cc, ncs, c, hw) || overlaps(fc, channels * ncs * sizeof(float), cc, ncs))
            return DDI_EINVAL;
    }
    if ((e = check_device())) return e;
    DDI_HIP(launch_coarsen(f, c, height, width, channels, fc, cc, nullptr, nullptr,
                           (hipStream_t)stream));
    return DDI_OK;
}

int ddi_prolong(const float* uc, int hc, int wc, const float* f, const uint8_t* c, int height,
                int width, int channels, float* u, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!uc || !f || !c || !u) return DDI_EINVAL;
    if (hc != (height + 1) / 2 || wc != (width + 1) / 2) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        if (overlaps(u, nimg, uc, (size_t)channels * hc * wc * sizeof(float)) ||
            overlaps(u, nimg, f, nimg) || overlaps(u, nimg, c, (size_t)height * width))
            return DDI_EINVAL;
    }
    if ((e = check_device())) return e;
    DDI_HIP(launch_prolong(uc, hc, wc, f, c, height, width, channels, u, (hipStream_t)stream));
    return DDI_OK;
}

int ddi_coarse_solve(const float* f, const uint8_t* c, int height, int width, int channels,
                     float* u, int max_iter, double tol, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!f || !c || !u || max_iter < 1 || !(tol >= 0.0)) return DDI_EINVAL;
    if ((int64_t)height * width > kCoarseMaxPixels) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        if (overlaps(u, nimg, f, nimg) || overlaps(u, nimg, c, (size_t)height * width))
            return DDI_EINVAL;
    }
    if ((e = check_device())) return e;
    DDI_HIP(launch_coarse_cg(f, c, height, width, channels, u, max_iter, tol,
                             (hipStream_t)stream));
    return DDI_OK;
}

int ddi_coarse_grid_bytes(int height, int width, int channels, size_t* bytes) {
    if (!bytes) return DDI_EINVAL;
    const int e = check_dims(height, width, channels);
    if (e) return e;
    *bytes = coarse_grid_bytes(height, width, channels);
    return DDI_OK;
}

int ddi_coarse_grid_debug_spin_limit(long polls) {
    set_coarse_grid_spin_limit(polls);
    return DDI_OK;
}

int ddi_coarse_solve_grid(const float* f, const uint8_t* c, int height, int width, int channels,
                          float* u, int max_iter, double tol, int workgroups, void* work,
                          size_t work_bytes, int* steps, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!f || !c || !u || !work || max_iter < 1 || !(tol >= 0.0)) return DDI_EINVAL;
    if (workgroups < 0 || workgroups > kGridCgMaxWg) return DDI_EINVAL;
    const size_t need = coarse_grid_bytes(height, width, channels);
    if (work_bytes < need || ((uintptr_t)work & 255) != 0) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        const size_t nc = (size_t)height * width;
        if (overlaps(u, nimg, f, nimg) || overlaps(u, nimg, c, nc) ||
            overlaps(work, need, f, nimg) || overlaps(work, need, c, nc) ||
            overlaps(work, need, u, nimg))
            return DDI_EINVAL;
    }
    if ((e = check_device())) return e;
    hipStream_t s = (hipStream_t)stream;
    const int g = workgroups ? workgroups : coarse_grid_workgroups(height, width, channels);
    DDI_HIP(launch_coarse_cg_grid(f, c, height, width, channels, u, max_iter, tol, g, work,
                                  nullptr, s));
    if (steps) {
        int hs[4 + 1] = {};
        DDI_HIP(hipMemcpyAsync(hs, coarse_grid_status(work), sizeof(int), hipMemcpyDeviceToHost,
                               s));
        DDI_HIP(hipMemcpyAsync(hs + 1, coarse_grid_steps(work), 4 * sizeof(int),
                               hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
        if (hs[0] != 0) return DDI_ESTALL;
        for (int k = 0; k < channels; ++k) steps[k] = hs[1 + k];
    }
    return DDI_OK;
}

int ddi_refine_residual(const float* f, const uint8_t* c, const float* u, const uint16_t* d,
                        int height, int width, int channels, float* u_next, uint16_t* rhs,
                        double* rsq, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!f || !c || !u || !rhs || (d && !u_next)) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        const size_t nb16 = nimg / 2, hw = (size_t)height * width;
        const void* in[4] = {f, c, u, d};
        const size_t nin[4] = {nimg, hw, nimg, nb16};
        for (int i = 0; i < 4; ++i)
            if (overlaps(rhs, nb16, in[i], nin[i]) ||
                (d && overlaps(u_next, nimg, in[i], nin[i])))
                return DDI_EINVAL;
        if (overlaps(rhs, nb16, u_next, d ? nimg : 0)) return DDI_EINVAL;
    }
    if ((e = check_device())) return e;
    hipStream_t s = (hipStream_t)stream;
    const size_t nwg = (size_t)residual_partials(height, width);
    Scratch part, red;
    DDI_HIP(hipMalloc(&part.p, nwg * channels * sizeof(double)));
    DDI_HIP(hipMalloc(&red.p, channels * sizeof(double)));
    int n = 0;
    DDI_HIP(launch_refine_residual(f, c, u, d, height, width, channels, u_next, rhs,
                                   (double*)part.p, nullptr, &n, s));
    DDI_HIP(launch_reduce((double*)part.p, n, channels, channels, (double*)red.p, s));
    if (rsq)
        DDI_HIP(hipMemcpyAsync(rsq, red.p, channels * sizeof(double), hipMemcpyDeviceToHost, s));
    DDI_HIP(hipStreamSynchronize(s));
    return DDI_OK;
}

int ddi_refine_start(const float* uc, int hc, int wc, const float* f, const uint8_t* c,
                     int height, int width, int channels, float* u, uint16_t* rhs, double* rsq,
                     void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!uc || !f || !c || !u || !rhs) return DDI_EINVAL;
    if (hc != (height + 1) / 2 || wc != (width + 1) / 2) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        const size_t nb16 = nimg / 2, hw = (size_t)height * width;
        const void* in[3] = {uc, f, c};
        const size_t nin[3] = {(size_t)channels * hc * wc * sizeof(float), nimg, hw};
        for (int i = 0; i < 3; ++i)
            if (overlaps(u, nimg, in[i], nin[i]) || overlaps(rhs, nb16, in[i], nin[i]))
                return DDI_EINVAL;
        if (overlaps(rhs, nb16, u, nimg)) return DDI_EINVAL;
    }
    if ((e = check_device())) return e;
    hipStream_t s = (hipStream_t)stream;
    const size_t nwg = (size_t)residual_partials(height, width);
    Scratch part, red;
    DDI_HIP(hipMalloc(&part.p, nwg * channels * sizeof(double)));
    DDI_HIP(hipMalloc(&red.p, channels * sizeof(double)));
    int n = 0;
    DDI_HIP(launch_start_residual(ProSrc{uc, hc, wc, f, c}, height, width, channels, u, rhs,
                                  (double*)part.p, nullptr, &n, s));
    DDI_HIP(launch_reduce((double*)part.p, n, channels, channels, (double*)red.p, s));
    if (rsq)
        DDI_HIP(hipMemcpyAsync(rsq, red.p, channels * sizeof(double), hipMemcpyDeviceToHost, s));
    DDI_HIP(hipStreamSynchronize(s));
    return DDI_OK;
}

int ddi_correction_sweep(const uint16_t* d_in, const uint16_t* rhs, const uint8_t* c,
                         uint16_t* d_out, int height, int width, int channels, int block,
                         int overlap, float robin_alpha, int local_iters, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!rhs || !c || !d_out) return DDI_EINVAL;
    {
        const size_t nb16 = (size_t)channels * height * width * sizeof(uint16_t);
        if (overlaps(d_out, nb16, d_in, nb16) || overlaps(d_out, nb16, rhs, nb16) ||
            overlaps(d_out, nb16, c, (size_t)height * width))
            return DDI_EINVAL;
    }
    if (block < 2 || block > DDI_MAX_BLOCK || overlap < 0 || overlap >= block) return DDI_EINVAL;
    if (!(robin_alpha > 0.f && robin_alpha <= 1.f) || local_iters < 1) return DDI_EINVAL;
    if ((e = check_device())) return e;
    hipStream_t s = (hipStream_t)stream;
    const SweepArgs a = make_sweep(height, width, channels, block, overlap, robin_alpha,
                                   local_iters);
    Scratch part, mb;
    DDI_HIP(hipMalloc(&part.p, (size_t)sweep_partials(a) * channels * sizeof(double)));
    DDI_HIP(hipMalloc(&mb.p, (size_t)mask_bit_groups(height) * width * sizeof(uint64_t)));
    DDI_HIP(launch_mask_bits(c, height, width, (uint64_t*)mb.p, s));
    DDI_HIP(launch_sweep_corr(d_in, rhs, (const uint64_t*)mb.p, d_out, (double*)part.p, nullptr,
                              nullptr, a, s));
    DDI_HIP(hipStreamSynchronize(s));
    return DDI_OK;
}

int ddi_oras_sweep(const float* u_in, const uint8_t* c, float* u_out, int height, int width,
                   int channels, int block, int overlap, float robin_alpha, int local_iters,
                   double* rsq, void* stream) {
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (!u_in || !c || !u_out) return DDI_EINVAL;
    {
        const size_t nimg = (size_t)channels * height * width * sizeof(float);
        if (overlaps(u_out, nimg, u_in, nimg) || overlaps(u_out, nimg, c, (size_t)height * width))
            return DDI_EINVAL;
    }
    if (block < 2 || block > DDI_MAX_BLOCK || overlap < 0 || overlap >= block) return DDI_EINVAL;
    if (!(robin_alpha > 0.f && robin_alpha <= 1.f) || local_iters < 1) return DDI_EINVAL;
    if ((e = check_device())) return e;
    hipStream_t s = (hipStream_t)stream;
    const SweepArgs a = make_sweep(height, width, channels, block, overlap, robin_alpha,
                                   local_iters);
    const int nb = sweep_partials(a);
    Scratch part, red, mb;
    DDI_HIP(hipMalloc(&part.p, (size_t)nb * channels * sizeof(double)));
    DDI_HIP(hipMalloc(&red.p, channels * sizeof(double)));
    DDI_HIP(hipMalloc(&mb.p, (size_t)mask_bit_groups(height) * width * sizeof(uint64_t)));
    DDI_HIP(launch_mask_bits(c, height, width, (uint64_t*)mb.p, s));
    DDI_HIP(launch_sweep(u_in, (const uint64_t*)mb.p, u_out, (double*)part.p, nullptr, nullptr, a,
                         s));
    DDI_HIP(launch_reduce((double*)part.p, nb, channels, channels, (double*)red.p, s));
    if (rsq) {
        DDI_HIP(hipMemcpyAsync(rsq, red.p, channels * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    DDI_HIP(hipStreamSynchronize(s));
    return DDI_OK;
}

}  // extern "C"
