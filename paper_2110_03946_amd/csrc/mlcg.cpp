// Multilevel conjugate gradients (method = 1): the comparator the paper
// measures ORAS against (Sec. 5). The same pyramid and coarse-to-fine start
// as the ORAS solve (Sec. 4); on every level, global CG on the unknown
// pixels (Hestenes-Stiefel, float32 vectors, float64 dot products, scalars
// kept on the device) until ||b - A u|| <= rel_tol ||b|| on that level.
// Steps are enqueued in batches sized by the previous solve; a device stop
// test after every step makes the steps still enqueued exit at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.h"

using namespace ddi;

namespace {

// CG on one level; x holds the start (u = f on the mask) and receives the
// result. Returns the steps taken in *iters and the last tested relative
// residual in *rel.
int cg_level(ddi_plan* P, int l, float* x, int* iters, double* rel, bool* conv) {
    const int C = P->C;
    const ddi_params& prm = P->p;
    const Level& lev = P->lv[l];
    const int h = lev.h, w = lev.w;
    hipStream_t s = P->s;
    const size_t nv = (size_t)C * P->h * P->w;
    float* r = P->cg_vec;
    float* pv[2] = {P->cg_vec + nv, P->cg_vec + 2 * nv};
    float* q = P->cg_vec + 3 * nv;
    double* sc = P->cg_sc;
    double* b2 = P->cg_sc + 3 * C + (size_t)l * (C + 2);
    int* ctl = P->ctl;
    const int nres = residual_partials(h, w);

    // statistics of this level (||C f||^2 per channel) and the initial residual
    int nwg = 0;
    DDI_HIP(launch_stats(lev.f, lev.c, h, w, C, P->part, &nwg, s));
    DDI_HIP(launch_reduce(P->part, nwg, C + 2, C + 2, b2, s));
    DDI_HIP(launch_clear_int(ctl, 4, s));
    DDI_HIP(launch_residual(lev.f, lev.c, x, h, w, C, r, nullptr, P->part, nullptr, s));
    DDI_HIP(launch_cg_scalars(P->part, nres, C, sc, b2, ctl, prm.rel_tol, 2, 0, s));

    const int cap = prm.max_sweeps;
    int done = 0;
    int batch = P->last_iters[l] > 0 ? P->last_iters[l] : 16;
    *conv = false;
    for (;;) {
        const int to = std::min(cap, done + std::max(batch, 1));
        for (int it = done; it < to; ++it) {
            DDI_HIP(launch_cg_dir_matvec(r, pv[it & 1], pv[(it + 1) & 1], q, lev.c, h, w, C,
                                         sc + 2 * C, it == 0, P->part, ctl, nullptr, s));
            DDI_HIP(launch_cg_scalars(P->part, nres, C, sc, b2, ctl, -1.0, 0, it + 1, s));
            DDI_HIP(launch_cg_update(x, r, pv[(it + 1) & 1], q, h, w, C, sc + C, P->part, ctl, s));
            DDI_HIP(launch_cg_scalars(P->part, nres, C, sc, b2, ctl, prm.rel_tol, 1, it + 1, s));
        }
        done = to;
        DDI_HIP(hipMemcpyAsync(P->hctl, ctl, 4 * sizeof(int) + sizeof(double),
                               hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
        const int* hc = reinterpret_cast<const int*>(P->hctl);
        double rel2;
        std::memcpy(&rel2, hc + 4, sizeof(rel2));
        *rel = std::sqrt(rel2);
        if (hc[0] != 0) {
            *iters = hc[1];
            *conv = true;
            break;
        }
        *iters = done;
        if (done >= cap) break;
        batch = 8;
    }
    P->last_iters[l] = std::max(*iters, 1);
    return DDI_OK;
}

}  // namespace

int solve_mlcg(ddi_plan* P, ddi_stats* st) {
    const int C = P->C;
    const int L = (int)P->lv.size();
    hipStream_t s = P->s;
    Level& L0 = P->lv[0];
    DDI_HIP(hipEventRecord(P->e0, s));
    // pyramid, and the input checks on the finest level
    int nwg = 0;
    if (L > 1)
        DDI_HIP(launch_coarsen(L0.f, L0.c, P->h, P->w, C, P->lv[1].fown, P->lv[1].cown, P->part,
                               &nwg, s));
    else
        DDI_HIP(launch_stats(L0.f, L0.c, P->h, P->w, C, P->part, &nwg, s));
    DDI_HIP(launch_reduce(P->part, nwg, C + 2, C + 2, P->red, s));
    for (int l = 1; l + 1 < L; ++l)
        DDI_HIP(launch_coarsen(P->lv[l].f, P->lv[l].c, P->lv[l].h, P->lv[l].w, C,
                               P->lv[l + 1].fown, P->lv[l + 1].cown, nullptr, nullptr, s));
    DDI_HIP(hipMemcpyAsync(P->host, P->red, (C + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
    DDI_HIP(hipStreamSynchronize(s));
    if (P->host[C + 1] > 0.0) return DDI_EINVAL;
    if (P->host[C] <= 0.0) return DDI_ESINGULAR;

    double total = 0.0, rel = INFINITY;
    int fine_iters = 0;
    bool conv = false;
    for (int l = L - 1; l >= 0; --l) {
        Level& lev = P->lv[l];
        float* x = lev.u[0];  // the caller's u on level 0
        if (l == L - 1)
            DDI_HIP(launch_init(lev.f, lev.c, lev.h, lev.w, C, x, s));
        else
            DDI_HIP(launch_prolong(P->lv[l + 1].u[0], P->lv[l + 1].h, P->lv[l + 1].w, lev.f, lev.c,
                                   lev.h, lev.w, C, x, s));
        int iters = 0;
        int e = cg_level(P, l, x, &iters, &rel, &conv);
        if (e) return e;
        total += iters;
        if (l == 0) fine_iters = iters;
    }
    DDI_HIP(hipEventRecord(P->e1, s));
    DDI_HIP(hipEventSynchronize(P->e1));
    float ms = 0.f;
    DDI_HIP(hipEventElapsedTime(&ms, P->e0, P->e1));
    if (st) {
        st->sweeps = fine_iters;
        st->converged = conv ? 1 : 0;
        st->rel_residual = rel;
        st->ms = ms;
        st->cg_steps = total;
    }
    return conv ? DDI_OK : DDI_ENOCONV;
}
