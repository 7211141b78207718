// Global solvers on one level for gfx950 and their launchers: the conjugate
// gradients of the multilevel-CG comparison (Sec. 5) and the flexible GMRES
// that takes ORAS sweeps as its preconditioner. Both are column-walk stencil
// kernels with float64 dot products per channel and their scalars kept on
// the device.
#include "device.h"

namespace ddi {
namespace {

// ---------------------------------------------------------------------------
// Global conjugate gradients on one level (the multilevel-CG comparator of
// Sec. 5): float32 vectors of all channels, float64 dot products per
// channel, scalars kept on the device. The vectors vanish on the mask (r,
// p, q) and x = f there, so the masked 5-point operator needs no branches
// beyond the in-image tests.
// ---------------------------------------------------------------------------

// p_out = r + beta p_in (beta per channel; first: p_out = r), q = A p_out on
// unknown pixels (0 on the mask), partial[wg][ch] = sum p_out q. Column
// walk: p_out is formed once per pixel from r and p_in and shared with the
// neighbours through registers and DPP.
__global__ __launch_bounds__(64 * kWalkWaves) void k_cg_dir_matvec(
    const float* __restrict__ r, const float* __restrict__ pin, float* __restrict__ pout,
    float* __restrict__ q, const uint8_t* __restrict__ c, int h, int w, int channels,
    const double* __restrict__ beta, int first, double* __restrict__ partial,
    const int* __restrict__ ctl) {
    constexpr int R = kWalkRows;
    if (ctl[0] != 0) return;
    const Walk k = walk_geom(h, w);
    const int ch = blockIdx.z;
    const int64_t n = (int64_t)h * w;
    const uint32_t W = w;
    const float* __restrict__ RR = r + ch * n;
    const float* __restrict__ P = pin + ch * n;
    const float b = first ? 0.f : (float)beta[ch];
    auto pn = [&](uint32_t j) -> float {
        return first ? at32(RR, j) : at32(RR, j) + b * at32(P, j);
    };
    float v[R + 2], e[R];
    uint32_t cm[R];
#pragma unroll
    for (int t = 0; t < R + 2; ++t)
        v[t] = pn(walk_vrow(k, h, t) * W + k.xc);
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const uint32_t row = walk_row(k, h, t) * W;
        cm[t] = at32(c, row + k.xc);
        e[t] = k.edge ? pn(row + k.xe) : 0.f;
    }
    const int nr = k.y1 - k.y0;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const float cur = v[t + 1];
        float lft = from_left(cur), rgt = from_right(cur);
        if (k.lane == 0) lft = e[t];
        if (k.lane == 63) rgt = e[t];
        if (k.x == 0) lft = cur;
        if (k.x + 1 >= w) rgt = cur;
        const float qv =
            cm[t] == 0 ? ((cur - v[t]) + (cur - v[t + 2])) + ((cur - lft) + (cur - rgt)) : 0.f;
        if (k.inb && t < nr) {
            const uint32_t i = walk_out(k, W, t);
            put32(pout + ch * n, i, cur);
            put32(q + ch * n, i, qv);
            acc += (double)cur * (double)qv;
        }
    }
    walk_partial(acc, partial, channels);
}

// x += alpha p, r -= alpha q (alpha per channel), partial[wg][ch] = sum r^2,
// over the column-walk layout (same partial rows as the other CG kernels).
__global__ __launch_bounds__(64 * kWalkWaves) void k_cg_update(
    float* __restrict__ xv, float* __restrict__ r, const float* __restrict__ p,
    const float* __restrict__ q, int h, int w, int channels, const double* __restrict__ alpha,
    double* __restrict__ partial, const int* __restrict__ ctl) {
    constexpr int R = kWalkRows;
    if (ctl[0] != 0) return;
    const Walk k = walk_geom(h, w);
    const int ch = blockIdx.z;
    const int64_t n = (int64_t)h * w;
    const uint32_t W = w;
    const float a = (float)alpha[ch];
    float* __restrict__ X = xv + ch * n;
    float* __restrict__ RR = r + ch * n;
    const float* __restrict__ P = p + ch * n;
    const float* __restrict__ Q = q + ch * n;
    const int nr = k.y1 - k.y0;
    double acc = 0.0;
    if (k.inb) {
        float xs[R], rs[R], ps[R], qs[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const uint32_t i = walk_row(k, h, t) * W + k.xc;
            xs[t] = at32(X, i);
            rs[t] = at32(RR, i);
            ps[t] = at32(P, i);
            qs[t] = at32(Q, i);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (t < nr) {
                const uint32_t i = walk_out(k, W, t);
                put32(X, i, xs[t] + a * ps[t]);
                const float rv = rs[t] - a * qs[t];
                put32(RR, i, rv);
                acc += (double)rv * (double)rv;
            }
        }
    }
    walk_partial(acc, partial, channels);
}

// The CG scalars of one step from the partials of the last dot product,
// in one workgroup (fixed-order sums). stage 0 (after the matvec): alpha =
// rho / (p.q). stage 1 (after the update): rr = r.r, beta = rr / rho, rho =
// rr, and the stop test max_k rr_k / b2_k <= tol2 (sets ctl[0], ctl[1] =
// n). stage 2 (initial residual): rho = r.r and the same test. sc holds
// [rho, alpha, beta] x channels; b2 = ||C f||^2 per channel.
template <int NC>
__global__ __launch_bounds__(kDecideTpb) void k_cg_scalars(const double* __restrict__ partial,
                                                           int nb, double* __restrict__ sc,
                                                           const double* __restrict__ b2,
                                                           int* __restrict__ ctl, double tol2,
                                                           int stage, int n) {
    if (ctl[0] != 0) return;
    __shared__ double sm[kDecideTpb / 64][NC];
    double v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = 0.0;
    for (int i = threadIdx.x; i < nb; i += kDecideTpb) {
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] += partial[(int64_t)i * NC + k];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = wave_sum_d(v[k]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) sm[threadIdx.x >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double worst = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        double t = 0.0;
        for (int j = 0; j < kDecideTpb / 64; ++j) t += sm[j][k];
        double* rho = sc + k;
        double* alpha = sc + NC + k;
        double* beta = sc + 2 * NC + k;
        if (stage == 0) {
            *alpha = t > 0.0 ? *rho / t : 0.0;
        } else {
            if (stage == 1) *beta = *rho > 0.0 ? t / *rho : 0.0;
            *rho = t;
            const double q = b2[k] > 0.0 ? t / b2[k] : (t > 0.0 ? INFINITY : 0.0);
            worst = fmax(worst, q);
        }
    }
    if (stage != 0) {
        reinterpret_cast<double*>(ctl + 4)[0] = worst;
        if (worst <= tol2) {
            ctl[1] = n;
            ctl[0] = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Krylov-accelerated ORAS: flexible GMRES(m) on A u = b per channel, each
// basis vector v_j preconditioned by one ORAS sweep on the correction
// equation (z_j = k_sweep*_c32 from d = 0), classical Gram-Schmidt, the
// Hessenberg least-squares problem updated by Givens rotations on the device.
// ---------------------------------------------------------------------------

// Workgroup sum of acc into *dst (fixed order), column-walk workgroups.
__device__ __forceinline__ void walk_sum_to(double acc, double* __restrict__ dst) {
    acc = wave_sum_d(acc);
    __shared__ double sm[kWalkWaves];
    __syncthreads();  // an earlier call's readers are done
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kWalkWaves; ++j) t += sm[j];
        *dst = t;
    }
}

// w = A z (eq. 6; 0 on the mask, where z vanishes) and the dot products
// (w, v_i) for i < nv: partial[(wg * nv + i) * C + ch], wg = workgroup of
// the column walk.
__global__ __launch_bounds__(64 * kWalkWaves) void k_kry_matvec_dots(
    const float* __restrict__ z, const uint8_t* __restrict__ c, int h, int w, int channels,
    float* __restrict__ wout, const float* __restrict__ V, int64_t vstride, int nv,
    double* __restrict__ partial, const int* __restrict__ ctl) {
    constexpr int R = kWalkRows;
    if (ctl[0] != 0) return;
    const Walk k = walk_geom(h, w);
    const int ch = blockIdx.z;
    const int64_t n = (int64_t)h * w;
    const uint32_t W = w;
    const float* __restrict__ Z = z + ch * n;
    float v[R + 2], e[R];
    uint32_t cm[R];
#pragma unroll
    for (int t = 0; t < R + 2; ++t)
        v[t] = at32(Z, walk_vrow(k, h, t) * W + k.xc);
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const uint32_t row = walk_row(k, h, t) * W;
        cm[t] = at32(c, row + k.xc);
        e[t] = k.edge ? at32(Z, row + k.xe) : 0.f;
    }
    const int nr = k.y1 - k.y0;
    float wv[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const float cur = v[t + 1];
        float lft = from_left(cur), rgt = from_right(cur);
        if (k.lane == 0) lft = e[t];
        if (k.lane == 63) rgt = e[t];
        if (k.x == 0) lft = cur;
        if (k.x + 1 >= w) rgt = cur;
        const float q =
            cm[t] == 0 ? ((cur - v[t]) + (cur - v[t + 2])) + ((cur - lft) + (cur - rgt)) : 0.f;
        wv[t] = q;
        if (k.inb && t < nr) put32(wout + ch * n, walk_out(k, W, t), q);
    }
    const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    for (int i = 0; i < nv; ++i) {
        const float* __restrict__ Vi = V + i * vstride + ch * n;
        double acc = 0.0;
        if (k.inb) {
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (t < nr) acc += (double)wv[t] * (double)at32(Vi, walk_out(k, W, t));
        }
        walk_sum_to(acc, partial + (wg * nv + i) * channels + ch);
    }
}

// w -= sum_{i < nv} h_i v_i with h_i = hcol[i * C + ch] (rounded to float32),
// partial[wg * C + ch] = ||w||^2.
__global__ __launch_bounds__(64 * kWalkWaves) void k_kry_orth(
    float* __restrict__ wv, const float* __restrict__ V, int64_t vstride, int nv,
    const double* __restrict__ hcol, int h, int w, int channels, double* __restrict__ partial,
    const int* __restrict__ ctl) {
    constexpr int R = kWalkRows;
    if (ctl[0] != 0) return;
    const Walk k = walk_geom(h, w);
    const int ch = blockIdx.z;
    const int64_t n = (int64_t)h * w;
    const uint32_t W = w;
    float* __restrict__ Wp = wv + ch * n;
    const int nr = k.y1 - k.y0;
    double acc = 0.0;
    if (k.inb) {
        float x[R];
#pragma unroll
        for (int t = 0; t < R; ++t) x[t] = at32(Wp, walk_row(k, h, t) * W + k.xc);
        for (int i = 0; i < nv; ++i) {
            const float hi = (float)hcol[i * channels + ch];
            const float* __restrict__ Vi = V + i * vstride + ch * n;
#pragma unroll
            for (int t = 0; t < R; ++t)
                x[t] -= hi * at32(Vi, walk_row(k, h, t) * W + k.xc);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (t < nr) {
                put32(Wp, walk_out(k, W, t), x[t]);
                acc += (double)x[t] * (double)x[t];
            }
        }
    }
    walk_partial(acc, partial, channels);
}

// dst = src / sqrt(norm2[ch]) per channel (0 where the norm is 0); skipped
// once the solve has converged unless force.
__global__ __launch_bounds__(256) void k_kry_scale(const float* __restrict__ src,
                                                   float* __restrict__ dst,
                                                   const double* __restrict__ norm2, int64_t n,
                                                   const int* __restrict__ ctl, int force) {
    if (!force && ctl[0] != 0) return;
    const int ch = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double s2 = norm2[ch];
    const float inv = s2 > 0.0 ? (float)(1.0 / sqrt(s2)) : 0.f;
    dst[ch * n + i] = src[ch * n + i] * inv;
}

// Cycle start: beta = ||r|| per channel (beta2 = ||r||^2), g = beta e_1;
// the stop test on the residual of the current u.
template <int NC>
__global__ __launch_bounds__(64) void k_kry_start(KryState* __restrict__ st,
                                                  const double* __restrict__ beta2,
                                                  const double* __restrict__ b2,
                                                  int* __restrict__ ctl, double tol2, int total) {
    if (ctl[0] != 0) return;
    __shared__ double q[NC];
    const int ch = threadIdx.x;
    if (ch < NC) {
        KryState& S = st[ch];
        S.bnorm2 = b2[ch];
        S.steps = 0;
        for (int i = 0; i <= kKryMaxM; ++i) S.g[i] = 0.0;
        S.g[0] = sqrt(fmax(beta2[ch], 0.0));
        q[ch] = b2[ch] > 0.0 ? beta2[ch] / b2[ch] : (beta2[ch] > 0.0 ? INFINITY : 0.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double worst = 0.0;
        for (int k = 0; k < NC; ++k) worst = fmax(worst, q[k]);
        reinterpret_cast<double*>(ctl + 4)[0] = worst;
        if (worst <= tol2) {
            ctl[1] = total;
            ctl[0] = 1;
        }
    }
}

// Step j of the cycle: the new Hessenberg column (dots hcol[i * C + ch],
// i <= j, and sqrt(hn2[ch]) below the diagonal), the earlier rotations
// applied to it, a new rotation that zeroes the subdiagonal, and the
// least-squares residual |g_{j+1}|; the stop test (sets ctl[0] with ctl[1]
// = total + j + 1 once max_k g_{j+1}^2 / ||b_k||^2 <= tol2).
template <int NC>
__global__ __launch_bounds__(64) void k_kry_givens(KryState* __restrict__ st,
                                                   const double* __restrict__ hcol,
                                                   const double* __restrict__ hn2, int j,
                                                   int* __restrict__ ctl, double tol2,
                                                   int total) {
    if (ctl[0] != 0) return;
    __shared__ double q[NC];
    const int ch = threadIdx.x;
    if (ch < NC) {
        KryState& S = st[ch];
        double* col = S.R + j * (kKryMaxM + 1);
        for (int i = 0; i <= j; ++i) col[i] = hcol[i * NC + ch];
        double sub = sqrt(fmax(hn2[ch], 0.0));
        for (int i = 0; i < j; ++i) {
            const double a = col[i], b = col[i + 1];
            col[i] = S.cs[i] * a + S.sn[i] * b;
            col[i + 1] = -S.sn[i] * a + S.cs[i] * b;
        }
        const double r = sqrt(col[j] * col[j] + sub * sub);
        const double cs = r > 0.0 ? col[j] / r : 1.0, sn = r > 0.0 ? sub / r : 0.0;
        S.cs[j] = cs;
        S.sn[j] = sn;
        col[j] = r > 0.0 ? r : col[j];
        S.g[j + 1] = -sn * S.g[j];
        S.g[j] = cs * S.g[j];
        S.steps = j + 1;
        const double res2 = S.g[j + 1] * S.g[j + 1];
        q[ch] = S.bnorm2 > 0.0 ? res2 / S.bnorm2 : (res2 > 0.0 ? INFINITY : 0.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double worst = 0.0;
        for (int k = 0; k < NC; ++k) worst = fmax(worst, q[k]);
        reinterpret_cast<double*>(ctl + 4)[0] = worst;
        if (worst <= tol2) {
            ctl[1] = total + j + 1;
            ctl[0] = 1;
        }
    }
}

// y = R^-1 g over the cycle's steps (back substitution; a zero pivot gives
// y_i = 0), one thread per channel.
template <int NC>
__global__ __launch_bounds__(64) void k_kry_backsolve(KryState* __restrict__ st) {
    const int ch = threadIdx.x;
    if (ch >= NC) return;
    KryState& S = st[ch];
    for (int i = S.steps - 1; i >= 0; --i) {
        double t = S.g[i];
        for (int l = i + 1; l < S.steps; ++l) t -= S.R[l * (kKryMaxM + 1) + i] * S.y[l];
        const double d = S.R[i * (kKryMaxM + 1) + i];
        S.y[i] = d != 0.0 ? t / d : 0.0;
    }
}

// u += sum_{i < steps} y_i z_i per channel (z_i vanish on the mask, so u = f
// there is kept exactly).
__global__ __launch_bounds__(256) void k_kry_combine(float* __restrict__ u,
                                                     const float* __restrict__ Z, int64_t zstride,
                                                     const KryState* __restrict__ st, int64_t n) {
    const int ch = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const KryState& S = st[ch];
    float x = u[ch * n + i];
    for (int l = 0; l < S.steps; ++l) x += (float)S.y[l] * Z[l * zstride + ch * n + i];
    u[ch * n + i] = x;
}

}  // namespace

hipError_t launch_kry_matvec_dots(const float* z, const uint8_t* c, int h, int w, int channels,
                                  float* wout, const float* V, int64_t vstride, int nv,
                                  double* partial, const int* ctl, hipStream_t s) {
    if (nv < 1 || nv > kKryMaxM + 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kry_matvec_dots, walk_grid(h, w, channels), dim3(64 * kWalkWaves), 0, s,
                       z, c, h, w, channels, wout, V, vstride, nv, partial, ctl);
    return hipGetLastError();
}

hipError_t launch_kry_orth(float* wv, const float* V, int64_t vstride, int nv,
                           const double* hcol, int h, int w, int channels, double* partial,
                           const int* ctl, hipStream_t s) {
    if (nv < 1 || nv > kKryMaxM + 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kry_orth, walk_grid(h, w, channels), dim3(64 * kWalkWaves), 0, s, wv, V,
                       vstride, nv, hcol, h, w, channels, partial, ctl);
    return hipGetLastError();
}

hipError_t launch_kry_scale(const float* src, float* dst, const double* norm2, int64_t n,
                            int channels, const int* ctl, bool force, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256), channels);
    hipLaunchKernelGGL(k_kry_scale, grid, dim3(256), 0, s, src, dst, norm2, n, ctl,
                       force ? 1 : 0);
    return hipGetLastError();
}

#define DDI_KRY_NC(KERNEL, ...)                                                              \
    switch (channels) {                                                                      \
        case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(1), dim3(64), 0, s, __VA_ARGS__); break; \
        case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(1), dim3(64), 0, s, __VA_ARGS__); break; \
        case 3: hipLaunchKernelGGL(KERNEL<3>, dim3(1), dim3(64), 0, s, __VA_ARGS__); break; \
        case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(1), dim3(64), 0, s, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                                \
    }

hipError_t launch_kry_start(KryState* st, const double* beta2, const double* b2, int channels,
                            int* ctl, double tol2, int total, hipStream_t s) {
    DDI_KRY_NC(k_kry_start, st, beta2, b2, ctl, tol2, total)
    return hipGetLastError();
}

hipError_t launch_kry_givens(KryState* st, const double* hcol, const double* hn2, int j,
                             int channels, int* ctl, double tol2, int total, hipStream_t s) {
    if (j < 0 || j >= kKryMaxM) return hipErrorInvalidValue;
    DDI_KRY_NC(k_kry_givens, st, hcol, hn2, j, ctl, tol2, total)
    return hipGetLastError();
}

hipError_t launch_kry_backsolve(KryState* st, int channels, hipStream_t s) {
    DDI_KRY_NC(k_kry_backsolve, st)
    return hipGetLastError();
}
#undef DDI_KRY_NC

hipError_t launch_kry_combine(float* u, const float* Z, int64_t zstride, const KryState* st,
                              int64_t n, int channels, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256), channels);
    hipLaunchKernelGGL(k_kry_combine, grid, dim3(256), 0, s, u, Z, zstride, st, n);
    return hipGetLastError();
}

hipError_t launch_cg_dir_matvec(const float* r, const float* pin, float* pout, float* q,
                                const uint8_t* c, int h, int w, int channels,
                                const double* beta, bool first, double* partial, const int* ctl,
                                int* nwg, hipStream_t s) {
    const dim3 grid = walk_grid(h, w, channels);
    if (nwg) *nwg = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_cg_dir_matvec, grid, dim3(64 * kWalkWaves), 0, s, r, pin, pout, q, c, h,
                       w, channels, beta, first ? 1 : 0, partial, ctl);
    return hipGetLastError();
}

hipError_t launch_cg_update(float* x, float* r, const float* p, const float* q, int h, int w,
                            int channels, const double* alpha, double* partial, const int* ctl,
                            hipStream_t s) {
    const dim3 grid = walk_grid(h, w, channels);
    hipLaunchKernelGGL(k_cg_update, grid, dim3(64 * kWalkWaves), 0, s, x, r, p, q, h, w, channels,
                       alpha, partial, ctl);
    return hipGetLastError();
}

hipError_t launch_cg_scalars(const double* partial, int nb, int channels, double* sc,
                             const double* b2, int* ctl, double tol, int stage, int n,
                             hipStream_t s) {
    const double tol2 = tol < 0.0 ? -1.0 : tol * tol;
    switch (channels) {
#define DDI_CASE(NC)                                                                          \
    case NC:                                                                                  \
        hipLaunchKernelGGL(k_cg_scalars<NC>, dim3(1), dim3(kDecideTpb), 0, s, partial, nb, sc, \
                           b2, ctl, tol2, stage, n);                                          \
        break;
        DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ddi
