// Batched solve (include/ddi.h, ddi_batch_*): many images of uneven size
// solved together, each step of the multilevel ORAS scheme (Sec. 3-4) run
// as one launch over the work items of every image -- (image, block,
// channel) for the sweeps, (image, level, tile) for the level kernels. Each
// image keeps its own pyramid, stop test and device control word; images
// that have converged drop out of the work list at the next host check and
// their sweeps still in flight exit at once.
//
// Per-launch work lists (job tables) are written on the host into a pinned
// arena and uploaded with one copy per batch of launches, so a solve costs
// the same number of launches as a single image.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan.h"

using namespace ddi;

namespace {

constexpr int kCtlInts = 8;  // per image: done, sweeps, error, -, rel (double), -

// Sweep instances: (rows per wave, ragged) pairs of launch_sweep_batch.
constexpr int kInstances = 8;
int instance_index(int bh) {
    int rpw;
    bool ragged;
    sweep_instance(bh, &rpw, &ragged);
    const int r = rpw == 64 ? 0 : rpw == 32 ? 1 : rpw == 16 ? 2 : 3;
    return 2 * r + (ragged ? 1 : 0);
}
int instance_rpw(int idx) {
    static const int rpw[4] = {64, 32, 16, 8};
    return rpw[idx / 2];
}

// Host-side builder of the job tables of one upload. With h == nullptr it
// only counts bytes (used at create to size the arena).
struct Arena {
    char* h = nullptr;
    char* d = nullptr;
    size_t cap = 0, used = 0;
    template <class T>
    const T* put(const std::vector<T>& v) {
        used = (used + 63) & ~size_t(63);
        const size_t bytes = v.size() * sizeof(T);
        const T* dp = reinterpret_cast<const T*>(d + used);
        if (h && used + bytes <= cap && bytes) std::memcpy(h + used, v.data(), bytes);
        used += bytes;
        return dp;
    }
    bool overflow() const { return used > cap; }
};

// One sweep launch per instance present in the job list.
struct SweepLaunch {
    const SweepJob* jobs;
    int njobs, total_wg, inst;
};

}  // namespace

struct ddi_batch {
    int n = 0, C = 0;
    hipStream_t s = nullptr;
    std::vector<ddi_plan*> plans;
    int min_sweeps = 0, max_sweeps = 0, check_every = 1;
    bool timing = false;
    int* ctl = nullptr;    // device [n][kCtlInts]
    int* hctl = nullptr;   // pinned mirror
    char* djob = nullptr;  // device job arena
    char* hjob = nullptr;  // pinned staging of the arena
    size_t jcap = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<hipEvent_t> sweep_ev;  // 2 per finest-level sweep (timing)
};

namespace {

bool is_check(const ddi_batch* B, int n) {
    return n >= B->min_sweeps && (n - B->min_sweeps) % B->check_every == 0;
}

// Groups sweep jobs by instance into consecutive tables of the arena.
void put_sweeps(Arena& A, const std::vector<SweepJob>& jobs, std::vector<SweepLaunch>& out) {
    out.clear();
    for (int inst = 0; inst < kInstances; ++inst) {
        std::vector<SweepJob> v;
        int wg = 0;
        for (const SweepJob& j : jobs) {
            if (instance_index(j.a.g.bh) != inst) continue;
            // fused jobs are built only for split blocks (k_sweep2_batch)
            SweepJob k = j;
            k.wg0 = wg;
            wg += sweep_partials(j.a) * j.a.channels;
            v.push_back(k);
        }
        if (v.empty()) continue;
        out.push_back({A.put(v), (int)v.size(), wg, inst});
    }
}

hipError_t run_sweeps(const std::vector<SweepLaunch>& ls, hipStream_t s) {
    for (const SweepLaunch& l : ls) {
        hipError_t e = launch_sweep_batch(l.jobs, l.njobs, l.total_wg, instance_rpw(l.inst),
                                          (l.inst & 1) != 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Everything of one solve up to the start of the finest level, as a list
// of deferred launches built against the arena (so that the tables are
// uploaded before the first launch is enqueued).
struct Front {
    struct Step {
        enum Kind { Coarsen, CoarsenOne, StatsOne, Reduce, MaskBits, Init, CoarseCg,
                    CoarseGrid, Sweep, Prolong, ProlongOne } kind;
        const void* jobs = nullptr;
        int njobs = 0, total_wg = 0;
        std::vector<SweepLaunch> sweeps;
        int img = -1, level = -1, dst = 0, src = 0;
    };
    std::vector<Step> steps;
    std::vector<int> nwg;  // statistics rows per image
};

// ORAS sweeps an image runs on level l >= 1 of its pyramid.
int coarse_sweeps_at(const ddi_plan* P, int l) {
    const int L = (int)P->lv.size();
    if (l != L - 1) return P->p.coarse_sweeps;
    return P->p.coarse_solver == 1 ? 0 : P->p.coarsest_sweeps;
}

// Builds the front for images with start buffers start0 (finest level).
// Pointers of level 0 must be set in the plans already.
void build_front(ddi_batch* B, const std::vector<int>& start0, Arena& A, Front& F) {
    const int n = B->n, C = B->C;
    int Lmax = 0;
    for (ddi_plan* P : B->plans) Lmax = std::max(Lmax, (int)P->lv.size());
    F.steps.clear();
    F.nwg.assign(n, 0);

    // pyramid and input statistics (from the first coarsening)
    for (int l = 0; l + 1 < Lmax || (l == 0 && Lmax == 1); ++l) {
        std::vector<LevelJob> jobs;
        int wg = 0;
        for (int i = 0; i < n; ++i) {
            ddi_plan* P = B->plans[i];
            const int L = (int)P->lv.size();
            if (l == 0 && L == 1) {
                Front::Step st;
                st.kind = Front::Step::StatsOne;
                st.img = i;
                F.steps.push_back(st);
                F.nwg[i] = stats_rows(P->h, P->w);
                continue;
            }
            if (l + 1 >= L) continue;
            const Level& a = P->lv[l];
            const Level& b = P->lv[l + 1];
            if (!coarsen4_ok(a.f, a.c, b.fown, b.cown, a.w)) {
                Front::Step st;
                st.kind = Front::Step::CoarsenOne;
                st.img = i;
                st.level = l;
                F.steps.push_back(st);
                if (l == 0) F.nwg[i] = coarsen_rows(a.f, a.c, b.fown, b.cown, a.h, a.w);
                continue;
            }
            LevelJob j{};
            j.f = a.f;
            j.c = a.c;
            j.fo = b.fown;
            j.co = b.cown;
            j.stats = l == 0 ? P->part : nullptr;
            j.h = a.h;
            j.w = a.w;
            j.hc = b.h;
            j.wc = b.w;
            const int nw = coarsen4_grid(a.h, a.w, &j.gx, &j.rows);
            j.wg0 = wg;
            wg += nw;
            if (l == 0) F.nwg[i] = nw;
            jobs.push_back(j);
        }
        if (!jobs.empty()) {
            Front::Step st;
            st.kind = Front::Step::Coarsen;
            st.jobs = A.put(jobs);
            st.njobs = (int)jobs.size();
            st.total_wg = wg;
            F.steps.push_back(st);
        }
        if (Lmax == 1) break;
    }
    {
        std::vector<ReduceJob> jobs;
        for (int i = 0; i < n; ++i) {
            ReduceJob j{};
            j.partial = B->plans[i]->part;
            j.out = B->plans[i]->red;
            j.nrows = F.nwg[i];
            j.stride = C + 2;
            jobs.push_back(j);
        }
        Front::Step st;
        st.kind = Front::Step::Reduce;
        st.jobs = A.put(jobs);
        st.njobs = n;
        F.steps.push_back(st);
    }

    // transposed masks of every (image, level)
    {
        std::vector<LevelJob> jobs;
        int wg = 0;
        for (int i = 0; i < n; ++i) {
            for (const Level& lev : B->plans[i]->lv) {
                LevelJob j{};
                j.c = lev.c;
                j.mbits = lev.mbits;
                j.h = lev.h;
                j.w = lev.w;
                const int nw = mask_bits_grid(lev.h, lev.w, &j.gx);
                j.wg0 = wg;
                wg += nw;
                jobs.push_back(j);
            }
        }
        Front::Step st;
        st.kind = Front::Step::MaskBits;
        st.jobs = A.put(jobs);
        st.njobs = (int)jobs.size();
        st.total_wg = wg;
        F.steps.push_back(st);
    }

    // start on each image's coarsest level: u = c ? f : 0, or its float64
    // solve
    std::vector<int> cur(n, 0);
    {
        std::vector<LevelJob> jobs;
        std::vector<CoarseJob> cg;
        std::vector<Front::Step> grid;
        int wg = 0;
        for (int i = 0; i < n; ++i) {
            ddi_plan* P = B->plans[i];
            const int top = (int)P->lv.size() - 1;
            cur[i] = top == 0 ? start0[i] : 0;
            const Level& lev = P->lv[top];
            if (P->p.coarse_solver == 1 && P->cgw) {
                // a coarsest level too large for one workgroup: its own
                // grid solve
                Front::Step st;
                st.kind = Front::Step::CoarseGrid;
                st.img = i;
                st.dst = cur[i];
                grid.push_back(st);
                continue;
            }
            if (P->p.coarse_solver == 1) {
                CoarseJob j{};
                j.f = lev.f;
                j.c = lev.c;
                j.u = lev.u[cur[i]];
                j.h = lev.h;
                j.w = lev.w;
                j.max_iter = P->p.coarse_cg_iters;
                j.tol2 = P->p.coarse_cg_tol * P->p.coarse_cg_tol;
                cg.push_back(j);
                continue;
            }
            LevelJob j{};
            j.f = lev.f;
            j.c = lev.c;
            j.u = lev.u[cur[i]];
            j.h = lev.h;
            j.w = lev.w;
            j.wg0 = wg;
            wg += init_grid(lev.h, lev.w);
            jobs.push_back(j);
        }
        if (!jobs.empty()) {
            Front::Step st;
            st.kind = Front::Step::Init;
            st.jobs = A.put(jobs);
            st.njobs = (int)jobs.size();
            st.total_wg = wg;
            F.steps.push_back(st);
        }
        if (!cg.empty()) {
            Front::Step st;
            st.kind = Front::Step::CoarseCg;
            st.jobs = A.put(cg);
            st.njobs = (int)cg.size();
            F.steps.push_back(st);
        }
        for (const Front::Step& st : grid) F.steps.push_back(st);
    }

    // coarse levels, coarsest first: sweeps, then prolongation one level down
    // (fused into the first sweep of the finer level where it has one: the
    // image's pending source `from`)
    std::vector<ProSrc> from(n, ProSrc{});
    for (ddi_plan* P : B->plans) P->pro0_on = false;
    for (int l = Lmax - 1; l >= 1; --l) {
        int nmax = 0;
        for (ddi_plan* P : B->plans) {
            const int L = (int)P->lv.size();
            if (L <= l) continue;
            nmax = std::max(nmax, coarse_sweeps_at(P, l));
        }
        for (int k = 0; k < nmax; ++k) {
            std::vector<SweepJob> jobs;
            for (int i = 0; i < n; ++i) {
                ddi_plan* P = B->plans[i];
                const int L = (int)P->lv.size();
                if (L <= l) continue;
                const int ni = coarse_sweeps_at(P, l);
                if (k >= ni) continue;
                Level& lev = P->lv[l];
                SweepJob j{};
                j.uin = lev.u[cur[i]];
                j.mbits = lev.mbits;
                j.uout = lev.u[cur[i] ^ 1];
                j.partial = P->part;
                j.a = lev.sw;
                if (k == 0 && from[i].uc) {
                    j.uin = nullptr;
                    j.pro = from[i];
                }
                jobs.push_back(j);
                cur[i] ^= 1;
            }
            Front::Step st;
            st.kind = Front::Step::Sweep;
            put_sweeps(A, jobs, st.sweeps);
            F.steps.push_back(st);
        }
        std::vector<LevelJob> jobs;
        int wg = 0;
        for (int i = 0; i < n; ++i) {
            ddi_plan* P = B->plans[i];
            if ((int)P->lv.size() <= l) continue;
            const Level& lev = P->lv[l];
            Level& fine = P->lv[l - 1];
            const int dst = l == 1 ? start0[i] : 0;
            from[i] = ProSrc{};
            const bool fuse = P->p.fuse_prolong == 1 && sweep_prolong_ok(fine.sw) &&
                              (l == 1 ? B->max_sweeps > 0 : coarse_sweeps_at(P, l - 1) > 0);
            if (fuse) {
                from[i] = ProSrc{lev.u[cur[i]], lev.h, lev.w, fine.f, fine.c};
                if (l == 1) {
                    P->pro0 = from[i];
                    P->pro0_on = true;
                }
            } else if (!prolong4_ok(lev.u[cur[i]], fine.f, fine.c, fine.u[dst], fine.w)) {
                Front::Step st;
                st.kind = Front::Step::ProlongOne;
                st.img = i;
                st.level = l;
                st.src = cur[i];
                st.dst = dst;
                F.steps.push_back(st);
            } else {
                LevelJob j{};
                j.uc = lev.u[cur[i]];
                j.hc = lev.h;
                j.wc = lev.w;
                j.f = fine.f;
                j.c = fine.c;
                j.h = fine.h;
                j.w = fine.w;
                j.u = fine.u[dst];
                j.wg0 = wg;
                wg += prolong4_grid(fine.h, fine.w, &j.gx);
                jobs.push_back(j);
            }
            cur[i] = dst;
        }
        if (!jobs.empty()) {
            Front::Step st;
            st.kind = Front::Step::Prolong;
            st.jobs = A.put(jobs);
            st.njobs = (int)jobs.size();
            st.total_wg = wg;
            F.steps.push_back(st);
        }
    }
}

int enqueue_front(ddi_batch* B, const Front& F) {
    hipStream_t s = B->s;
    const int C = B->C;
    for (const Front::Step& st : F.steps) {
        hipError_t e = hipSuccess;
        switch (st.kind) {
            case Front::Step::Coarsen:
                e = launch_coarsen_batch((const LevelJob*)st.jobs, st.njobs, st.total_wg, C, s);
                break;
            case Front::Step::CoarsenOne: {
                ddi_plan* P = B->plans[st.img];
                const Level& a = P->lv[st.level];
                const Level& b = P->lv[st.level + 1];
                e = launch_coarsen(a.f, a.c, a.h, a.w, C, b.fown, b.cown,
                                   st.level == 0 ? P->part : nullptr, nullptr, s);
                break;
            }
            case Front::Step::StatsOne: {
                ddi_plan* P = B->plans[st.img];
                e = launch_stats(P->lv[0].f, P->lv[0].c, P->h, P->w, C, P->part, nullptr, s);
                break;
            }
            case Front::Step::Reduce:
                e = launch_reduce_batch((const ReduceJob*)st.jobs, st.njobs, C + 2, s);
                break;
            case Front::Step::MaskBits:
                e = launch_mask_bits_batch((const LevelJob*)st.jobs, st.njobs, st.total_wg, s);
                break;
            case Front::Step::Init:
                e = launch_init_batch((const LevelJob*)st.jobs, st.njobs, st.total_wg, C, s);
                break;
            case Front::Step::CoarseCg:
                e = launch_coarse_cg_batch((const CoarseJob*)st.jobs, st.njobs, C, s);
                break;
            case Front::Step::CoarseGrid: {
                ddi_plan* P = B->plans[st.img];
                const Level& t = P->lv.back();
                e = launch_coarse_cg_grid(t.f, t.c, t.h, t.w, C, t.u[st.dst],
                                          P->p.coarse_cg_iters, P->p.coarse_cg_tol,
                                          coarse_grid_workgroups(t.h, t.w, C), P->cgw,
                                          B->ctl + (size_t)st.img * kCtlInts, s);
                break;
            }
            case Front::Step::Sweep:
                e = run_sweeps(st.sweeps, s);
                break;
            case Front::Step::Prolong:
                e = launch_prolong_batch((const LevelJob*)st.jobs, st.njobs, st.total_wg, C, s);
                break;
            case Front::Step::ProlongOne: {
                ddi_plan* P = B->plans[st.img];
                const Level& lev = P->lv[st.level];
                Level& fine = P->lv[st.level - 1];
                e = launch_prolong(lev.u[st.src], lev.h, lev.w, fine.f, fine.c, fine.h, fine.w, C,
                                   fine.u[st.dst], s);
                break;
            }
        }
        if (e != hipSuccess) return hip_fail(e);
    }
    return DDI_OK;
}

// Finest-level tables for the images in `act`: sweep tables for both
// parities and the decide tables (stop test, and the non-passing test after
// the last allowed sweep when that is not a check point).
struct FineTables {
    std::vector<SweepLaunch> sweep[2];  // sweeps 2, 3, ... by parity
    std::vector<SweepLaunch> early[2];  // sweeps 0 and 1: no unchanged-block flags to read
    std::vector<SweepLaunch> first;  // sweep 0 with fused prolongations (empty: early[0])
    const DecideJob* decide[2] = {nullptr, nullptr};
    int ndecide = 0;
};

void build_fine(ddi_batch* B, const std::vector<int>& act, const std::vector<int>& start0,
                Arena& A, FineTables& T, bool with_first) {
    T.first.clear();
    if (with_first) {
        std::vector<SweepJob> jobs;
        bool any = false;
        for (int i : act) {
            ddi_plan* P = B->plans[i];
            Level& L0 = P->lv[0];
            SweepJob j{};
            j.uin = L0.u[start0[i]];
            j.mbits = L0.mbits;
            j.uout = L0.u[start0[i] ^ 1];
            j.partial = P->part;
            j.cg_steps = B->timing ? P->cgcnt : nullptr;
            j.ctl = B->ctl + (size_t)i * kCtlInts;
            j.a = L0.sw;
            if (P->pro0_on) {
                j.uin = nullptr;
                j.pro = P->pro0;
                any = true;
            }
            jobs.push_back(j);
        }
        if (any) put_sweeps(A, jobs, T.first);
    }
    // sweep k of parity q = k & 1 writes the image's unchanged-block flags
    // q and, from the third sweep on, reads those of the sweep before
    // (launch_sweep); images whose plan keeps no flags run every block
    for (int late = 0; late < 2; ++late) {
        for (int q = 0; q < 2; ++q) {
            std::vector<SweepJob> jobs;
            for (int i : act) {
                ddi_plan* P = B->plans[i];
                Level& L0 = P->lv[0];
                const int c0 = start0[i] ^ q;
                SweepJob j{};
                j.uin = L0.u[c0];
                j.mbits = L0.mbits;
                j.uout = L0.u[c0 ^ 1];
                j.partial = P->part;
                j.cg_steps = B->timing ? P->cgcnt : nullptr;
                j.ctl = B->ctl + (size_t)i * kCtlInts;
                j.a = L0.sw;
                if (P->flg) {
                    const size_t nfl = (size_t)sweep_partials(L0.sw) * P->C;
                    j.fout = P->flg + q * nfl;
                    j.fin = late ? P->flg + (q ^ 1) * nfl : nullptr;
                }
                jobs.push_back(j);
            }
            put_sweeps(A, jobs, late ? T.sweep[q] : T.early[q]);
        }
    }
    for (int t = 0; t < 2; ++t) {
        std::vector<DecideJob> jobs;
        for (int i : act) {
            ddi_plan* P = B->plans[i];
            DecideJob j{};
            j.partial = P->part;
            j.stats = P->red;
            j.ctl = B->ctl + (size_t)i * kCtlInts;
            j.rel = reinterpret_cast<double*>(B->ctl + (size_t)i * kCtlInts + 4);
            j.tol2 = t == 0 ? P->p.rel_tol * P->p.rel_tol : -1.0;
            j.nb = sweep_partials(P->lv[0].sw);
            j.min_n = P->p.min_sweeps;
            jobs.push_back(j);
        }
        T.decide[t] = A.put(jobs);
    }
    T.ndecide = (int)act.size();
}

int enqueue_fine(ddi_batch* B, const FineTables& T, int from, int to) {
    hipStream_t s = B->s;
    for (int i = from; i < to; ++i) {
        if (B->timing) DDI_HIP(hipEventRecord(B->sweep_ev[2 * i], s));
        DDI_HIP(run_sweeps(i == 0 && !T.first.empty() ? T.first
                           : i < 2                      ? T.early[i]
                                                        : T.sweep[i & 1],
                           s));
        if (B->timing) DDI_HIP(hipEventRecord(B->sweep_ev[2 * i + 1], s));
        const bool chk = is_check(B, i + 1);
        if (chk || i + 1 == B->max_sweeps)
            DDI_HIP(launch_decide_batch(T.decide[chk ? 0 : 1], T.ndecide, B->C, i + 1, s));
    }
    return DDI_OK;
}

int upload(ddi_batch* B, const Arena& A) {
    if (A.overflow()) return DDI_EINVAL;  // sized at create: cannot happen
    if (A.used)
        DDI_HIP(hipMemcpyAsync(B->djob, B->hjob, A.used, hipMemcpyHostToDevice, B->s));
    return DDI_OK;
}

// Sweeps to enqueue in a batch starting after `done` enqueued sweeps.
int next_upto(const ddi_batch* B, int done, int first_len) {
    int upto = std::min(B->max_sweeps, std::max(done + 1, first_len > 0 ? first_len : done + 2));
    while (upto < B->max_sweeps && !is_check(B, upto)) ++upto;
    return upto;
}

}  // namespace

extern "C" {

int ddi_batch_destroy(ddi_batch* B) {
    if (!B) return DDI_OK;
    for (ddi_plan* P : B->plans) ddi_destroy(P);
    if (B->ctl) (void)hipFree(B->ctl);
    if (B->hctl) (void)hipHostFree(B->hctl);
    if (B->djob) (void)hipFree(B->djob);
    if (B->hjob) (void)hipHostFree(B->hjob);
    if (B->e0) (void)hipEventDestroy(B->e0);
    if (B->e1) (void)hipEventDestroy(B->e1);
    for (hipEvent_t e : B->sweep_ev) (void)hipEventDestroy(e);
    delete B;
    return DDI_OK;
}

int ddi_batch_create(ddi_batch** out, int n, const int* heights, const int* widths,
                     int channels, const ddi_params* p, int n_params, void* stream) {
    if (!out) return DDI_EINVAL;
    *out = nullptr;
    if (n < 1 || !heights || !widths) return DDI_EINVAL;
    if (p ? (n_params != 1 && n_params != n) : n_params != 0) return DDI_EINVAL;
    std::vector<ddi_params> prm(n);
    for (int i = 0; i < n; ++i) {
        if (p)
            prm[i] = p[n_params == 1 ? 0 : i];
        else
            ddi_default_params(&prm[i]);
        prm[i].use_graph = 0;
        int e = ddi_check_params(heights[i], widths[i], channels, &prm[i]);
        if (e) return e;
        // batches run float32 ORAS
        if (prm[i].storage != 0 || prm[i].method != 0) return DDI_EINVAL;
        if (prm[i].max_sweeps != prm[0].max_sweeps || prm[i].check_every != prm[0].check_every ||
            prm[i].timing != prm[0].timing)
            return DDI_EINVAL;
    }
    int e = check_device();
    if (e) return e;
    ddi_batch* B = new (std::nothrow) ddi_batch;
    if (!B) return DDI_ENOMEM;
    B->n = n;
    B->C = channels;
    B->s = (hipStream_t)stream;
    // the stop tests start with the smallest min_sweeps; each image's test
    // passes only from its own on
    B->min_sweeps = prm[0].min_sweeps;
    for (int i = 1; i < n; ++i) B->min_sweeps = std::min(B->min_sweeps, prm[i].min_sweeps);
    B->max_sweeps = prm[0].max_sweeps;
    B->check_every = prm[0].check_every;
    B->timing = prm[0].timing != 0;
    B->plans.assign(n, nullptr);
    for (int i = 0; i < n; ++i) {
        if ((e = ddi_create(&B->plans[i], heights[i], widths[i], channels, &prm[i], stream))) {
            ddi_batch_destroy(B);
            return e;
        }
    }
    auto fail = [&](hipError_t err) {
        ddi_batch_destroy(B);
        return err == hipErrorOutOfMemory ? DDI_ENOMEM : hip_fail(err);
    };
    hipError_t err;
    const size_t ctl_bytes = (size_t)n * kCtlInts * sizeof(int);
    if ((err = hipMalloc(&B->ctl, ctl_bytes)) != hipSuccess) return fail(err);
    if ((err = hipHostMalloc(&B->hctl, ctl_bytes, hipHostMallocDefault)) != hipSuccess)
        return fail(err);
    // e0 only starts the solve's timer: no system-scope fence
    if ((err = hipEventCreateWithFlags(&B->e0, hipEventDisableSystemFence)) != hipSuccess)
        return fail(err);
    if ((err = hipEventCreate(&B->e1)) != hipSuccess) return fail(err);
    if (B->timing) {
        B->sweep_ev.assign(2 * (size_t)B->max_sweeps, nullptr);
        // timing only: no system-scope fence between sweeps
        for (hipEvent_t& ev : B->sweep_ev)
            if ((err = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence)) != hipSuccess)
                return fail(err);
    }
    // size the job arena: the front plus the finest-level tables of all
    // images (a dry run of the builders; pointers do not matter here, but
    // the width-4 eligibility does, so count with aligned dummies)
    {
        Arena A;
        Front F;
        std::vector<int> start0(n, 0), act(n);
        for (int i = 0; i < n; ++i) {
            act[i] = i;
            Level& L0 = B->plans[i]->lv[0];
            L0.f = reinterpret_cast<const float*>(uintptr_t(256));
            L0.c = reinterpret_cast<const uint8_t*>(uintptr_t(256));
            L0.u[0] = reinterpret_cast<float*>(uintptr_t(256));
        }
        build_front(B, start0, A, F);
        FineTables T;
        build_fine(B, act, start0, A, T, true);
        for (int i = 0; i < n; ++i) {
            Level& L0 = B->plans[i]->lv[0];
            L0.f = nullptr;
            L0.c = nullptr;
            L0.u[0] = nullptr;
        }
        B->jcap = A.used + 64;
    }
    if ((err = hipMalloc(&B->djob, B->jcap)) != hipSuccess) return fail(err);
    if ((err = hipHostMalloc(&B->hjob, B->jcap, hipHostMallocDefault)) != hipSuccess)
        return fail(err);
    *out = B;
    return DDI_OK;
}

int ddi_batch_solve(ddi_batch* B, const float* const* f, const uint8_t* const* c,
                    float* const* u, ddi_stats* st, int* status) {
    if (!B || !f || !c || !u) return DDI_EINVAL;
    const int n = B->n, C = B->C;
    for (int i = 0; i < n; ++i)
        if (!f[i] || !c[i] || !u[i]) return DDI_EINVAL;
    // every output must be disjoint from every input and from the other
    // outputs: one launch reads and writes all images at once
    for (int i = 0; i < n; ++i) {
        const ddi_plan* Pi = B->plans[i];
        const size_t ni = (size_t)C * Pi->h * Pi->w * sizeof(float);
        for (int j = 0; j < n; ++j) {
            const ddi_plan* Pj = B->plans[j];
            const size_t nj = (size_t)C * Pj->h * Pj->w * sizeof(float);
            if (overlaps(u[i], ni, f[j], nj) || overlaps(u[i], ni, c[j], (size_t)Pj->h * Pj->w) ||
                (j != i && overlaps(u[i], ni, u[j], nj)))
                return DDI_EINVAL;
        }
    }
    if (st) std::memset(st, 0, sizeof(*st) * n);
    std::vector<int> code(n, DDI_OK);
    hipStream_t s = B->s;

    // start buffers: as many sweeps as each image needed last time
    std::vector<int> start0(n), sweeps(n, 0), act, expect(n);
    std::vector<double> rel(n, INFINITY);
    std::vector<char> converged(n, 0), validated(n, 0);
    for (int i = 0; i < n; ++i) {
        ddi_plan* P = B->plans[i];
        Level& L0 = P->lv[0];
        L0.f = f[i];
        L0.c = c[i];
        L0.u[0] = u[i];
        expect[i] = P->last_sweeps >= 0 ? P->last_sweeps : std::max(B->min_sweeps, 1);
        start0[i] = std::min(expect[i], B->max_sweeps) & 1;
        act.push_back(i);
    }
    // the first batch of finest sweeps: as many as the images holding three
    // quarters of the pixels needed last time. The images expected to need
    // more continue after one host check in tables of their own, so the
    // launches of the longest-running images do not carry the blocks of
    // every converged image (each such block still costs a dispatch).
    int first;
    {
        std::vector<std::pair<int, double>> ep;
        double total = 0.0;
        for (int i = 0; i < n; ++i) {
            const double px = (double)B->plans[i]->h * B->plans[i]->w;
            ep.push_back({expect[i], px});
            total += px;
        }
        std::sort(ep.begin(), ep.end());
        double acc = 0.0;
        int n75 = ep.back().first;
        for (const auto& e : ep) {
            acc += e.second;
            if (acc >= 0.75 * total) {
                n75 = e.first;
                break;
            }
        }
        first = std::min(B->max_sweeps, std::max(n75, B->min_sweeps));
    }

    DDI_HIP(hipEventRecord(B->e0, s));
    Arena A;
    A.h = B->hjob;
    A.d = B->djob;
    A.cap = B->jcap;
    Front F;
    build_front(B, start0, A, F);
    FineTables T;
    build_fine(B, act, start0, A, T, true);
    int e = upload(B, A);
    if (e) return e;
    // the control words first: the front's float64 grid solves report a
    // stalled barrier there
    DDI_HIP(launch_clear_int(B->ctl, n * kCtlInts, s));
    if ((e = enqueue_front(B, F))) return e;

    int done_upto = 0;
    bool first_batch = true;
    while (done_upto < B->max_sweeps) {
        // later batches: up to the largest count the running images needed
        // last time, then two sweeps per check
        int want = first;
        if (!first_batch) {
            want = 0;
            for (int i : act) want = std::max(want, expect[i]);
            if (want <= done_upto) want = 0;
        }
        const int upto = next_upto(B, done_upto, want);
        if (!first_batch) {
            // rebuild the finest-level tables for the images still running
            Arena R;
            R.h = B->hjob;
            R.d = B->djob;
            R.cap = B->jcap;
            build_fine(B, act, start0, R, T, false);
            if ((e = upload(B, R))) return e;
        }
        first_batch = false;
        if ((e = enqueue_fine(B, T, done_upto, upto))) return e;
        done_upto = upto;
        DDI_HIP(hipMemcpyAsync(B->hctl, B->ctl, (size_t)n * kCtlInts * sizeof(int),
                               hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
        std::vector<int> still;
        for (int i : act) {
            const int* hc = B->hctl + (size_t)i * kCtlInts;
            validated[i] = 1;
            double rel2;
            std::memcpy(&rel2, hc + 4, sizeof(rel2));
            rel[i] = std::sqrt(rel2);
            if (hc[2] != 0) {
                code[i] = hc[2] == 1 ? DDI_EINVAL : hc[2] == 2 ? DDI_ESINGULAR : DDI_ESTALL;
                sweeps[i] = hc[1];
            } else if (hc[0] != 0) {
                sweeps[i] = hc[1];
                converged[i] = 1;
            } else {
                sweeps[i] = done_upto;
                still.push_back(i);
            }
        }
        act.swap(still);
        if (act.empty()) break;
    }

    // final residual of the returned iterate, or a copy into u
    bool need_sync = false;
    for (int i = 0; i < n; ++i) {
        if (code[i]) continue;
        ddi_plan* P = B->plans[i];
        Level& L0 = P->lv[0];
        const int cur = start0[i] ^ (sweeps[i] & 1);
        P->last_sweeps = sweeps[i];
        if (P->p.final_residual || !validated[i]) {
            int rwg = 0;
            DDI_HIP(launch_residual(f[i], c[i], L0.u[cur], P->h, P->w, C, nullptr,
                                    cur == 1 ? u[i] : nullptr, P->part, &rwg, s));
            DDI_HIP(launch_reduce(P->part, rwg, C, C, P->red + C + 2, s));
            DDI_HIP(hipMemcpyAsync(P->host, P->red, (2 * C + 2) * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
            need_sync = true;
        } else if (cur == 1) {
            DDI_HIP(hipMemcpyAsync(u[i], L0.u[1], (size_t)C * P->h * P->w * sizeof(float),
                                   hipMemcpyDeviceToDevice, s));
        }
        if (B->timing) {
            // CG steps, whole skips and skipped write-backs (three planes)
            const int nb = sweep_partials(L0.sw);
            DDI_HIP(launch_reduce(P->cgcnt, nb, C, C, P->red + 2 * C + 2, s, true));
            DDI_HIP(launch_reduce(P->cgcnt + (size_t)nb * C, nb, C, C, P->red + 4 * C + 2, s,
                                  true));
            DDI_HIP(launch_reduce(P->cgcnt + 2 * (size_t)nb * C, nb, C, C, P->red + 5 * C + 2,
                                  s, true));
            DDI_HIP(hipMemcpyAsync(P->host + 2 * C + 2, P->red + 2 * C + 2, 4 * C * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
        }
    }
    DDI_HIP(hipEventRecord(B->e1, s));
    DDI_HIP(hipEventSynchronize(B->e1));
    (void)need_sync;
    float ms = 0.f;
    DDI_HIP(hipEventElapsedTime(&ms, B->e0, B->e1));
    double sweep_ms = 0.0;
    int max_sw = 0;
    for (int i = 0; i < n; ++i) max_sw = std::max(max_sw, sweeps[i]);
    for (int i = 0; B->timing && i < std::min(max_sw, done_upto); ++i) {
        float t = 0.f;
        DDI_HIP(hipEventElapsedTime(&t, B->sweep_ev[2 * i], B->sweep_ev[2 * i + 1]));
        sweep_ms += t;
    }
    int ret = DDI_OK;
    for (int i = 0; i < n; ++i) {
        ddi_plan* P = B->plans[i];
        if (!code[i]) {
            if (!validated[i]) {
                if (P->host[C + 1] > 0.0) code[i] = DDI_EINVAL;
                else if (P->host[C] <= 0.0) code[i] = DDI_ESINGULAR;
            }
        }
        if (!code[i] && P->p.final_residual) {
            double worst = 0.0;
            for (int k = 0; k < C; ++k) {
                const double b2 = P->host[k], r2 = P->host[C + 2 + k];
                worst = std::max(worst, b2 > 0.0 ? std::sqrt(r2 / b2) : (r2 > 0.0 ? INFINITY : 0.0));
            }
            rel[i] = worst;
            converged[i] = converged[i] || worst <= P->p.rel_tol;
        }
        if (!code[i] && !converged[i]) code[i] = DDI_ENOCONV;
        if (status) status[i] = code[i];
        if (st) {
            st[i].sweeps = sweeps[i];
            st[i].converged = converged[i];
            st[i].rel_residual = rel[i];
            st[i].ms = ms;
            st[i].sweep_ms = sweep_ms;
            double steps = 0.0, skipped = 0.0, unwritten = 0.0;
            for (int k = 0; B->timing && !code[i] && k < C; ++k) {
                steps += P->host[2 * C + 2 + k];
                skipped += P->host[4 * C + 2 + k];
                unwritten += P->host[5 * C + 2 + k];
            }
            st[i].cg_steps = steps;
            st[i].skipped_blocks = skipped;
            st[i].unwritten_blocks = unwritten;
        }
        if (ret == DDI_OK && code[i] != DDI_OK) ret = code[i];
    }
    return ret;
}

}  // extern "C"
