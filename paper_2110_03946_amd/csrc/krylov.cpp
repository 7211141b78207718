// Krylov-accelerated ORAS (method = 2; not in the paper): the multilevel
// coarse-to-fine start of Sec. 4, then flexible GMRES(m) on the finest level
// per channel (Saad's flexible inner-outer GMRES), each basis vector
// preconditioned by one ORAS sweep (Sec. 3) on the correction equation
// A d = v from d = 0. Local CG with a step cap is not a linear map of its
// right-hand side, hence the flexible variant: the preconditioned vectors
// z_j are kept and the cycle's update is u += Z y.
//
// One cycle is enqueued at a time: the residual r = b - A u and beta, then
// m Arnoldi steps (preconditioner sweep; w = A z with the dot products
// (w, v_i); w -= sum h_i v_i with ||w||; Givens update and stop test on the
// device; normalisation), the back substitution and u += Z y. Once the
// device stop test passes, the rest of the cycle exits at once; the host
// waits once per cycle. A stop on the least-squares estimate is confirmed
// on the recomputed residual b - A u at the next cycle start.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.h"

using namespace ddi;

int solve_krylov(ddi_plan* P, ddi_stats* st) {
    const int C = P->C;
    const ddi_params& prm = P->p;
    Level& L0 = P->lv[0];
    const int h = P->h, w = P->w;
    hipStream_t s = P->s;
    const int m = prm.krylov_restart;
    const int64_t n = (int64_t)h * w;
    const int64_t vstride = (int64_t)C * n;
    float* u = L0.u[0];
    float* V = P->kry_vec;                 // V_0 .. V_m
    float* Z = P->kry_vec + (m + 1) * vstride;  // Z_0 .. Z_{m-1}
    double* hcol = P->kry_sc;              // [(m + 1) C]
    double* hn2 = hcol + (size_t)(m + 1) * C;
    double* beta2 = hn2 + C;
    int* ctl = P->ctl;
    const double tol2 = prm.rel_tol * prm.rel_tol;
    const int nres = residual_partials(h, w);
    // the preconditioner's local CG runs its local_iters steps: the local
    // stop is an absolute threshold on the block residual, which the unit
    // basis vectors (entries ~ 1/sqrt(pixels)) would meet before any step
    SweepArgs pre = L0.sw;
    pre.local_tol2 = 0.f;

    DDI_HIP(hipEventRecord(P->e0, s));
    // u = the coarse-to-fine start; the front also clears the control word
    int e = plan_enqueue_front(P, 0, s, false);
    if (e) return e;

    int total = 0;
    bool converged = false, checked = false;
    double rel = INFINITY;
    while (true) {
        // cycle start: r = b - A u into V_0, beta = ||r||, stop test
        int nwg = 0;
        DDI_HIP(launch_residual(L0.f, L0.c, u, h, w, C, V, nullptr, P->part, &nwg, s));
        DDI_HIP(launch_reduce(P->part, nwg, C, C, beta2, s));
        DDI_HIP(launch_kry_start(P->kry_state, beta2, P->red, C, ctl, tol2, total, s));
        DDI_HIP(launch_kry_scale(V, V, beta2, n, C, ctl, false, s));
        const int steps = std::min(m, prm.max_sweeps - total);
        for (int j = 0; j < steps; ++j) {
            float* vj = V + j * vstride;
            float* zj = Z + j * vstride;
            float* vn = V + (j + 1) * vstride;
            DDI_HIP(launch_sweep_c32(nullptr, vj, L0.mbits, zj, P->part, nullptr, ctl, pre, s));
            DDI_HIP(launch_kry_matvec_dots(zj, L0.c, h, w, C, vn, V, vstride, j + 1, P->kry_part,
                                           ctl, s));
            DDI_HIP(launch_reduce(P->kry_part, nres, (j + 1) * C, (j + 1) * C, hcol, s));
            DDI_HIP(launch_kry_orth(vn, V, vstride, j + 1, hcol, h, w, C, P->part, ctl, s));
            DDI_HIP(launch_reduce(P->part, nres, C, C, hn2, s));
            DDI_HIP(launch_kry_givens(P->kry_state, hcol, hn2, j, C, ctl, tol2, total, s));
            DDI_HIP(launch_kry_scale(vn, vn, hn2, n, C, ctl, false, s));
        }
        DDI_HIP(launch_kry_backsolve(P->kry_state, C, s));
        DDI_HIP(launch_kry_combine(u, Z, vstride, P->kry_state, n, C, s));
        DDI_HIP(hipMemcpyAsync(P->hctl, ctl, 4 * sizeof(int) + sizeof(double),
                               hipMemcpyDeviceToHost, s));
        if (!checked)
            DDI_HIP(hipMemcpyAsync(P->host, P->red, (C + 2) * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
        if (!checked) {
            if (P->host[C + 1] > 0.0) return DDI_EINVAL;
            if (P->host[C] <= 0.0) return DDI_ESINGULAR;
            checked = true;
        }
        const int* hc = reinterpret_cast<const int*>(P->hctl);
        if (hc[2] == 3) return DDI_ESTALL;  // the float64 coarse grid solve stalled
        double rel2;
        std::memcpy(&rel2, hc + 4, sizeof(rel2));
        rel = std::sqrt(rel2);
        if (hc[0] != 0 && hc[1] == total) {
            // the test at the cycle start passed: the residual of u itself
            converged = true;
            break;
        }
        if (hc[0] != 0) {
            // the least-squares estimate passed within the cycle; in float32
            // it can drift below the true residual, so the next cycle start
            // confirms it on b - A u (or the iteration goes on)
            total = hc[1];
            DDI_HIP(launch_clear_int(ctl, 1, s));
            continue;
        }
        total += steps;
        if (steps == 0 || total >= prm.max_sweeps) break;
    }

    // the residual of the returned iterate, for the statistics
    if (prm.final_residual) {
        int rwg = 0;
        DDI_HIP(launch_residual(L0.f, L0.c, u, h, w, C, nullptr, nullptr, P->part, &rwg, s));
        DDI_HIP(launch_reduce(P->part, rwg, C, C, P->red + C + 2, s));
        DDI_HIP(hipMemcpyAsync(P->host, P->red, (2 * C + 2) * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
        double worst = 0.0;
        for (int k = 0; k < C; ++k) {
            const double b2 = P->host[k], r2 = P->host[C + 2 + k];
            worst = std::max(worst, b2 > 0.0 ? std::sqrt(r2 / b2) : (r2 > 0.0 ? INFINITY : 0.0));
        }
        rel = worst;
        converged = rel <= prm.rel_tol || converged;
    }
    DDI_HIP(hipEventRecord(P->e1, s));
    DDI_HIP(hipEventSynchronize(P->e1));
    float ms = 0.f;
    DDI_HIP(hipEventElapsedTime(&ms, P->e0, P->e1));
    if (st) {
        st->sweeps = total;
        st->converged = converged ? 1 : 0;
        st->rel_residual = rel;
        st->ms = ms;
    }
    return converged ? DDI_OK : DDI_ENOCONV;
}
