// Float64 solves of the coarsest level for gfx950 (the system of Sec. 2,
// eq. 6, on the coarse grid) and their launchers: conjugate gradients in one
// workgroup per channel for levels that fit its LDS, and on a grid of
// workgroups meeting at grid barriers for larger ones.
#include <atomic>

#include "device.h"

namespace ddi {
namespace {

// ---------------------------------------------------------------------------
// Float64 solve of the coarsest level (Sec. 2 system, eq. 6, on the coarse
// grid): conjugate gradients on the unknown pixels, known pixels fixed at
// their value, in one workgroup per channel. Thread t owns pixels t,
// t + kCgTpb, ... of the level; the search direction lives in LDS for the
// neighbour reads of the matvec; the two dot products of a step are
// fixed-order block reductions. Starts from u = c ? f : 0 and stops once
// ||r||^2 <= tol2 ||C f||^2 or after max_iter steps.
// ---------------------------------------------------------------------------
constexpr int kCgTpb = 1024;
constexpr int kCgPer = kCoarseMaxPixels / kCgTpb;

// Sum of v over the workgroup, returned to every thread (fixed order).
__device__ __forceinline__ double cg_block_sum(double v, double* red) {
    v = wave_sum_d(v);
    const int wv = threadIdx.x >> 6;
    __syncthreads();  // earlier readers of red are done
    if ((threadIdx.x & 63) == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kCgTpb / 64; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ void coarse_cg_body(const float* __restrict__ f,
                                               const uint8_t* __restrict__ c, int h, int w,
                                               float* __restrict__ u, int max_iter, double tol2,
                                               int ch, double* __restrict__ sh,
                                               double* __restrict__ red) {
    const int n = h * w;
    const float* F = f + (int64_t)ch * n;
    float* U = u + (int64_t)ch * n;
    const int t = threadIdx.x;
    double x[kCgPer], r[kCgPer], p[kCgPer];
    bool unk[kCgPer];
    // in-image neighbours of each owned pixel: bit 0 up, 1 down, 2 left,
    // 3 right
    int nbm[kCgPer];
    // start: u = c ? f : 0, staged for the residual's neighbour reads
    double b2 = 0.0;
#pragma unroll
    for (int j = 0; j < kCgPer; ++j) {
        const int i = t + j * kCgTpb;
        const bool in = i < n;
        const bool known = in && c[i] != 0;
        unk[j] = in && !known;
        const int yy = in ? i / w : 0, xx = i - yy * w;
        nbm[j] = (yy > 0 ? 1 : 0) | (yy < h - 1 ? 2 : 0) | (xx > 0 ? 4 : 0) | (xx < w - 1 ? 8 : 0);
        x[j] = known ? (double)F[i] : 0.0;
        b2 += known ? x[j] * x[j] : 0.0;
        if (in) sh[i] = x[j];
    }
    b2 = cg_block_sum(b2, red);  // also orders the writes of sh before the reads
    // r = b - A x: for an unknown pixel the sum over in-image neighbours of
    // (x_q - x_p); 0 on the mask
    double rho = 0.0;
#pragma unroll
    for (int j = 0; j < kCgPer; ++j) {
        const int i = t + j * kCgTpb;
        double rv = 0.0;
        if (unk[j]) {
            if (nbm[j] & 1) rv += sh[i - w] - x[j];
            if (nbm[j] & 2) rv += sh[i + w] - x[j];
            if (nbm[j] & 4) rv += sh[i - 1] - x[j];
            if (nbm[j] & 8) rv += sh[i + 1] - x[j];
        }
        r[j] = rv;
        p[j] = rv;
        rho += rv * rv;
    }
    rho = cg_block_sum(rho, red);
    const double stop = tol2 * b2;
    for (int it = 0; it < max_iter && rho > stop; ++it) {
        __syncthreads();  // all reads of sh from the previous step are done
#pragma unroll
        for (int j = 0; j < kCgPer; ++j) {
            const int i = t + j * kCgTpb;
            if (i < n) sh[i] = p[j];
        }
        __syncthreads();
        double q[kCgPer];
        double pq = 0.0;
#pragma unroll
        for (int j = 0; j < kCgPer; ++j) {
            const int i = t + j * kCgTpb;
            double qv = 0.0;
            if (unk[j]) {
                // (A p)_i = deg_i p_i - sum of the neighbours' p (p = 0 on
                // the mask), deg_i = number of in-image neighbours
                double s = 0.0, deg = 0.0;
                if (nbm[j] & 1) { s += sh[i - w]; deg += 1.0; }
                if (nbm[j] & 2) { s += sh[i + w]; deg += 1.0; }
                if (nbm[j] & 4) { s += sh[i - 1]; deg += 1.0; }
                if (nbm[j] & 8) { s += sh[i + 1]; deg += 1.0; }
                qv = deg * p[j] - s;
            }
            q[j] = qv;
            pq += p[j] * qv;
        }
        pq = cg_block_sum(pq, red);
        if (!(pq > 0.0)) break;
        const double alpha = rho / pq;
        double rr = 0.0;
#pragma unroll
        for (int j = 0; j < kCgPer; ++j) {
            x[j] += alpha * p[j];
            r[j] -= alpha * q[j];
            rr += r[j] * r[j];
        }
        rr = cg_block_sum(rr, red);
        const double beta = rr / rho;
        rho = rr;
#pragma unroll
        for (int j = 0; j < kCgPer; ++j) p[j] = r[j] + beta * p[j];
    }
#pragma unroll
    for (int j = 0; j < kCgPer; ++j) {
        const int i = t + j * kCgTpb;
        if (i < n) U[i] = (float)x[j];
    }
}

__global__ __launch_bounds__(kCgTpb) void k_coarse_cg64(const float* __restrict__ f,
                                                        const uint8_t* __restrict__ c, int h,
                                                        int w, float* __restrict__ u,
                                                        int max_iter, double tol2) {
    __shared__ double sh[kCoarseMaxPixels];
    __shared__ double red[kCgTpb / 64];
    coarse_cg_body(f, c, h, w, u, max_iter, tol2, blockIdx.x, sh, red);
}

// Several images: workgroup (job j, channel k) = blockIdx.x = j * channels + k.
__global__ __launch_bounds__(kCgTpb) void k_coarse_cg64_batch(const CoarseJob* __restrict__ jobs,
                                                              int channels) {
    __shared__ double sh[kCoarseMaxPixels];
    __shared__ double red[kCgTpb / 64];
    const CoarseJob& J = jobs[blockIdx.x / channels];
    coarse_cg_body(J.f, J.c, J.h, J.w, J.u, J.max_iter, J.tol2, blockIdx.x % channels, sh, red);
}

// ---------------------------------------------------------------------------
// Float64 solve of the coarsest level on a grid of workgroups, for levels
// larger than one workgroup's LDS holds: the CG of coarse_cg_body (same
// system, start, stop test and per-channel ending), its vectors in global
// memory, the workgroups meeting at grid barriers.
//
// Workgroup g owns a contiguous range of pixels. At the start it numbers the
// unknown pixels of its range in pixel order after those of the ranges
// before it (so the numbering is that of the image), records each unknown's
// pixel and, per pixel, its number (-1 on the mask), then each unknown's
// four neighbours as numbers (-1 known, -2 outside the image). The CG
// vectors are kept per unknown in that numbering, so the steps touch no
// known pixel and test no mask byte. One step:
//   1. p = r + beta p_old (p = r in the first step) into the step's
//      direction buffer, q = A p with the neighbours' p formed from their r
//      and p_old by the same expression, and the partial p.q;
//   2. barrier; alpha = rho / p.q per channel from the partials of all
//      workgroups (each sums the same table in the same order, so every
//      workgroup holds the same alpha); x += alpha p, r -= alpha q, and the
//      partial r.r;
//   3. barrier; beta = r.r / rho, rho = r.r and the stop test.
// A channel that meets its tolerance, or whose p.q is not positive, stops
// updating; the solve ends once every channel has stopped or after max_iter
// steps.
// ---------------------------------------------------------------------------
constexpr int kGcgTpb = 256;
constexpr unsigned kGcgSpinLimit = 1u << 20;  // polls of one barrier wait (1-2 s)
std::atomic<unsigned> g_gcg_spin_limit{kGcgSpinLimit};  // host: the limit launches pass
constexpr int kGcgCtlInts = 64;               // control words, cleared per launch

struct GcgWork {
    unsigned* arrive;  // barrier arrivals
    unsigned* gen;     // barriers completed
    int* status;       // 0; 1 once a barrier wait exceeded its bound
    int* steps;        // CG steps per channel
    double* part;      // [3][kGridCgMaxWg][4]: r.r, ||C f||^2, p.q
    int* cnt;          // [kGridCgMaxWg] unknowns in each workgroup's range
    int* idx;          // [n] pixel of unknown k
    int* map;          // [n] unknown number of pixel j, -1 on the mask
    int4* nb;          // [n] neighbours of unknown k (up, down, left, right)
    double *x, *r, *pd0, *pd1, *q;  // [channels][n] by unknown number
};

__host__ __device__ inline size_t gcg_round(size_t n) { return (n + 255) & ~(size_t)255; }

__host__ __device__ inline GcgWork gcg_layout(void* work, int64_t n, int channels) {
    unsigned char* b = (unsigned char*)work;
    GcgWork W;
    W.arrive = (unsigned*)b;
    W.gen = (unsigned*)b + 16;
    W.status = (int*)b + 32;
    W.steps = (int*)b + 48;
    b += kGcgCtlInts * sizeof(int);
    W.part = (double*)b;
    b += gcg_round(3 * kGridCgMaxWg * 4 * sizeof(double));
    W.cnt = (int*)b;
    b += gcg_round(kGridCgMaxWg * sizeof(int));
    W.idx = (int*)b;
    b += gcg_round((size_t)n * sizeof(int));
    W.map = (int*)b;
    b += gcg_round((size_t)n * sizeof(int));
    W.nb = (int4*)b;
    b += gcg_round((size_t)n * sizeof(int4));
    const size_t vb = gcg_round((size_t)n * channels * sizeof(double));
    W.x = (double*)b;
    W.r = (double*)(b + vb);
    W.pd0 = (double*)(b + 2 * vb);
    W.pd1 = (double*)(b + 3 * vb);
    W.q = (double*)(b + 4 * vb);
    return W;
}

// All workgroups of the launch meet here; the generation count `gen` is the
// caller's copy of W.gen. Every thread's earlier global writes are visible
// to every workgroup after it. Returns false on every workgroup once the
// status word is set: a wait that exceeded `limit` polls sets it (limit 0:
// every wait that does not end at once), and the other waits end on it.
__device__ bool gcg_barrier(const GcgWork& W, unsigned nwg, unsigned limit, unsigned& gen,
                            int* ok_sh) {
    // the workgroup barrier waits for every wave's stores; one agent-scope
    // release by thread 0 then writes them back for the other XCDs, and one
    // acquire invalidates the caches the workgroup reads through
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned a =
            __hip_atomic_fetch_add(W.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == nwg - 1) {
            __hip_atomic_store(W.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(W.gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned polls = 0;
            // relaxed polls (an acquire per poll would invalidate the caches
            // every time); the acquire fence below follows the last one
            while (__hip_atomic_load(W.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(W.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                    break;
                if (polls++ >= limit) {
                    __hip_atomic_store(W.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        *ok_sh = __hip_atomic_load(W.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    ++gen;
    return *ok_sh != 0;
}

// Row blockIdx.x of tab = this workgroup's sums of v[0..4) (fixed order).
__device__ void gcg_partial(double (&v)[4], double* __restrict__ tab, double (*red)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum_d(v[k]);
    __syncthreads();  // earlier readers of red are done
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[threadIdx.x >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kGcgTpb / 64; ++j) t += red[j][threadIdx.x];
        tab[blockIdx.x * 4 + threadIdx.x] = t;
    }
}

// out[k] = sum over the nwg rows of tab (fixed order, the same in every
// workgroup), returned to every thread.
__device__ void gcg_total(const double* __restrict__ tab, unsigned nwg, double (*red)[4],
                          double* out_sh, double (&out)[4]) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (unsigned g = threadIdx.x; g < nwg; g += kGcgTpb) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += tab[g * 4 + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum_d(v[k]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[threadIdx.x >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kGcgTpb / 64; ++j) t += red[j][threadIdx.x];
        out_sh[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = out_sh[k];
}

// Workgroup sum of an int (every thread receives it).
__device__ int gcg_isum(int v, int* sh) {
    __syncthreads();  // earlier readers of sh are done
    if (threadIdx.x == 0) *sh = 0;
    __syncthreads();
    if (v) atomicAdd(sh, v);
    __syncthreads();
    return *sh;
}

// The search direction at an unknown: r, or r + beta p_old.
__device__ __forceinline__ double gcg_dir(bool first, double beta, double r, double pold) {
    return first ? r : fma(beta, pold, r);
}

__global__ __launch_bounds__(kGcgTpb) void k_coarse_cg64_grid(
    const float* __restrict__ f, const uint8_t* __restrict__ c, int h, int w, int channels,
    float* __restrict__ u, int max_iter, double tol2, GcgWork W, int* __restrict__ ctl,
    unsigned spin_limit) {
    __shared__ double red[kGcgTpb / 64][4];
    __shared__ double tot_sh[4];
    __shared__ int ok_sh, isum_sh, wcnt_sh[kGcgTpb / 64];
    const unsigned nwg = gridDim.x;
    unsigned gen = 0;
    const uint32_t n = (uint32_t)h * (uint32_t)w;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // this workgroup's pixel range
    const uint32_t len = (n + nwg - 1) / nwg;
    const uint32_t lo = min(blockIdx.x * len, n), hi = min(lo + len, n);
    double* T_rr = W.part;
    double* T_b2 = W.part + kGridCgMaxWg * 4;
    double* T_pq = W.part + 2 * kGridCgMaxWg * 4;

    // ---- numbering: count the range's unknowns; ||C f||^2 on its known pixels
    int mine = 0;
    double vb[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t j = lo + t; j < hi; j += kGcgTpb) {
        if (c[j] == 0) {
            ++mine;
            continue;
        }
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            if (ch < channels) {
                const double fv = (double)f[(size_t)ch * n + j];
                vb[ch] += fv * fv;
            }
        }
    }
    const int count = gcg_isum(mine, &isum_sh);
    if (t == 0) W.cnt[blockIdx.x] = count;
    gcg_partial(vb, T_b2, red);
    bool ok = gcg_barrier(W, nwg, spin_limit, gen, &ok_sh);
    int first_k = 0;  // number of this range's first unknown
    if (ok) {
        first_k = gcg_isum(t < blockIdx.x ? W.cnt[t] : 0, &isum_sh);
        // numbers in pixel order: per 256-pixel chunk, the unknowns before a
        // pixel in its wave (ballot) and in the waves before it
        int base = first_k;
        for (uint32_t j0 = lo; j0 < hi; j0 += kGcgTpb) {
            const uint32_t j = j0 + t;
            const bool unk = j < hi && c[j] == 0;
            const uint64_t m = __ballot(unk);
            const int below = __popcll(m & ((1ull << lane) - 1ull));
            __syncthreads();  // earlier readers of wcnt_sh are done
            if (lane == 0) wcnt_sh[wv] = __popcll(m);
            __syncthreads();
            int before = 0, all = 0;
#pragma unroll
            for (int i = 0; i < kGcgTpb / 64; ++i) {
                const int v = wcnt_sh[i];
                before += (i < (int)wv) ? v : 0;
                all += v;
            }
            if (j < hi) {
                const int k = base + before + below;
                W.map[j] = unk ? k : -1;
                if (unk) W.idx[k] = (int)j;
            }
            base += all;
        }
        ok = gcg_barrier(W, nwg, spin_limit, gen, &ok_sh);
    }
    const int k_lo = first_k, k_hi = first_k + count;  // this workgroup's unknowns

    // ---- neighbours and the start: x = 0 on the unknowns (u = c ? f : 0),
    // r = b - A x = the sum of the known in-image neighbours' f
    double vr[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok) {
        for (int k = k_lo + (int)t; k < k_hi; k += kGcgTpb) {
            const uint32_t j = (uint32_t)W.idx[k];
            const uint32_t y = j / (uint32_t)w, x = j - y * (uint32_t)w;
            int4 e;
            e.x = y > 0 ? W.map[j - w] : -2;
            e.y = y + 1 < (uint32_t)h ? W.map[j + w] : -2;
            e.z = x > 0 ? W.map[j - 1] : -2;
            e.w = x + 1 < (uint32_t)w ? W.map[j + 1] : -2;
            W.nb[k] = e;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (ch >= channels) break;
                const float* F = f + (size_t)ch * n;
                double rv = 0.0;
                if (e.x == -1) rv += (double)F[j - w];
                if (e.y == -1) rv += (double)F[j + w];
                if (e.z == -1) rv += (double)F[j - 1];
                if (e.w == -1) rv += (double)F[j + 1];
                W.x[(size_t)ch * n + k] = 0.0;
                W.r[(size_t)ch * n + k] = rv;
                vr[ch] += rv * rv;
            }
        }
        gcg_partial(vr, T_rr, red);
        ok = gcg_barrier(W, nwg, spin_limit, gen, &ok_sh);
    }
    double rho[4] = {0.0, 0.0, 0.0, 0.0}, stop[4] = {0.0, 0.0, 0.0, 0.0};
    double beta[4] = {0.0, 0.0, 0.0, 0.0};
    bool active[4] = {false, false, false, false};
    int steps[4] = {0, 0, 0, 0};
    if (ok) {
        double b2[4];
        gcg_total(T_b2, nwg, red, tot_sh, b2);
        gcg_total(T_rr, nwg, red, tot_sh, rho);
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            stop[ch] = tol2 * b2[ch];
            active[ch] = ch < channels && rho[ch] > stop[ch];
        }
    }
    for (int it = 0; ok && it < max_iter; ++it) {
        if (!(active[0] || active[1] || active[2] || active[3])) break;
        const bool first = it == 0;
        const double* Pold = (it & 1) ? W.pd1 : W.pd0;
        double* Pnew = (it & 1) ? W.pd0 : W.pd1;
        // 1. direction and A p; (A p)_k = deg_k p_k - the sum of the unknown
        // neighbours' p (p = 0 on the mask), neighbours in the order up,
        // down, left, right
        double vq[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = k_lo + (int)t; k < k_hi; k += kGcgTpb) {
            const int4 e = W.nb[k];
            const double deg = (double)((e.x != -2) + (e.y != -2) + (e.z != -2) + (e.w != -2));
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (ch >= channels) break;
                if (!active[ch]) continue;
                const size_t o = (size_t)ch * n;
                const double* __restrict__ R = W.r + o;
                const double* __restrict__ PO = Pold + o;
                const double b = beta[ch];
                auto dir = [&](int m) {
                    return gcg_dir(first, b, R[m], first ? 0.0 : PO[m]);
                };
                const double pv = dir(k);
                double sn = 0.0;
                if (e.x >= 0) sn += dir(e.x);
                if (e.y >= 0) sn += dir(e.y);
                if (e.z >= 0) sn += dir(e.z);
                if (e.w >= 0) sn += dir(e.w);
                const double qv = deg * pv - sn;
                Pnew[o + k] = pv;
                W.q[o + k] = qv;
                vq[ch] += pv * qv;
            }
        }
        gcg_partial(vq, T_pq, red);
        if (!(ok = gcg_barrier(W, nwg, spin_limit, gen, &ok_sh))) break;
        double pq[4], alpha[4];
        gcg_total(T_pq, nwg, red, tot_sh, pq);
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            if (active[ch] && !(pq[ch] > 0.0)) active[ch] = false;
            alpha[ch] = active[ch] ? rho[ch] / pq[ch] : 0.0;
        }
        // 2. x += alpha p, r -= alpha q
        double vr2[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = k_lo + (int)t; k < k_hi; k += kGcgTpb) {
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (ch >= channels) break;
                if (!active[ch]) continue;
                const size_t o = (size_t)ch * n + k;
                W.x[o] += alpha[ch] * Pnew[o];
                const double rv = W.r[o] - alpha[ch] * W.q[o];
                W.r[o] = rv;
                vr2[ch] += rv * rv;
            }
        }
        gcg_partial(vr2, T_rr, red);
        if (!(ok = gcg_barrier(W, nwg, spin_limit, gen, &ok_sh))) break;
        double rr[4];
        gcg_total(T_rr, nwg, red, tot_sh, rr);
        // 3. beta, rho and the stop test of the channels that stepped
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            if (!active[ch]) continue;
            beta[ch] = rr[ch] / rho[ch];
            rho[ch] = rr[ch];
            ++steps[ch];
            active[ch] = rho[ch] > stop[ch];
        }
    }
    if (!ok) {
        if (ctl && t == 0) {
            ctl[2] = 3;
            ctl[0] = 1;
        }
        return;
    }
    if (blockIdx.x == 0 && t == 0) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) W.steps[ch] = steps[ch];
    }
    // u = f on the mask, the rounded iterate elsewhere (this range's pixels)
    for (uint32_t j = lo + t; j < hi; j += kGcgTpb) {
        const int k = W.map[j];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            if (ch >= channels) break;
            const size_t o = (size_t)ch * n;
            u[o + j] = k < 0 ? f[o + j] : (float)W.x[o + k];
        }
    }
}

}  // namespace

hipError_t launch_coarse_cg(const float* f, const uint8_t* c, int h, int w, int channels,
                            float* u, int max_iter, double tol, hipStream_t s) {
    if ((int64_t)h * w > kCoarseMaxPixels || channels < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_coarse_cg64, dim3(channels), dim3(kCgTpb), 0, s, f, c, h, w, u,
                       max_iter, tol * tol);
    return hipGetLastError();
}

size_t coarse_grid_bytes(int h, int w, int channels) {
    const size_t n = (size_t)h * w;
    return kGcgCtlInts * sizeof(int) + gcg_round(3 * kGridCgMaxWg * 4 * sizeof(double)) +
           gcg_round(kGridCgMaxWg * sizeof(int)) + 2 * gcg_round(n * sizeof(int)) +
           gcg_round(n * 4 * sizeof(int)) + 5 * gcg_round(n * channels * sizeof(double));
}

int coarse_grid_workgroups(int h, int w, int channels) {
    // about 8 pixels per thread in the numbering and the final write, at
    // most 64 workgroups: every barrier costs each workgroup a cache
    // write-back and invalidate
    (void)channels;
    const int64_t n = (int64_t)h * w;
    const int64_t g = (n + 8 * kGcgTpb - 1) / (8 * kGcgTpb);
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 64);
}

void set_coarse_grid_spin_limit(long polls) {
    g_gcg_spin_limit = polls < 0 ? kGcgSpinLimit
                                 : (unsigned)std::min<long>(polls, (long)0xffffffffu);
}

const int* coarse_grid_status(const void* work) { return (const int*)work + 32; }
const int* coarse_grid_steps(const void* work) { return (const int*)work + 48; }

hipError_t launch_coarse_cg_grid(const float* f, const uint8_t* c, int h, int w, int channels,
                                 float* u, int max_iter, double tol, int wgs, void* work,
                                 int* ctl, hipStream_t s) {
    if (channels < 1 || channels > 4 || wgs < 1 || wgs > kGridCgMaxWg || !work ||
        ((uintptr_t)work & 255) != 0 || (int64_t)h * w > (int64_t(1) << 30))
        return hipErrorInvalidValue;
    if (hipError_t e = launch_clear_int((int*)work, kGcgCtlInts, s)) return e;
    const GcgWork W = gcg_layout(work, (int64_t)h * w, channels);
    hipLaunchKernelGGL(k_coarse_cg64_grid, dim3(wgs), dim3(kGcgTpb), 0, s, f, c, h, w, channels,
                       u, max_iter, tol * tol, W, ctl, g_gcg_spin_limit.load());
    return hipGetLastError();
}

hipError_t launch_coarse_cg_batch(const CoarseJob* jobs, int njobs, int channels, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_coarse_cg64_batch, dim3(njobs * channels), dim3(kCgTpb), 0, s, jobs,
                       channels);
    return hipGetLastError();
}

}  // namespace ddi
