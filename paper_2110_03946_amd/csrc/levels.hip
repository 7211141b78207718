// Level kernels of multilevel ORAS inpainting for gfx950 and their
// launchers: the transposed mask bits, level transfer, statistics,
// residuals, reductions and the stop test.
//
//   k_mask_bits*   column-transposed unknown-pixel bits of a mask.
//   k_coarsen*     dyadic subsampling of mask and known values (Sec. 4), with
//                  ||C f||^2 per channel, the known-pixel count and the bad
//                  mask bytes of the finer level.
//   k_init         u = c ? f : 0 on the coarsest level.
//   k_prolong*     u = c ? f : bilinear(coarse u) (Sec. 4 coarse-to-fine start).
//   k_residual_walk  r = b - A u (eq. 7) with float64 partial norms; column-
//                  walking waves keep the vertical stencil in registers.
//   k_reduce*      fixed-order float64 sums of per-workgroup partials.
//   k_decide*      the relative-residual stop test on the device.
#include "device.h"

namespace ddi {
namespace {

// Zero fill (a kernel rather than hipMemsetAsync, so that the solve can be
// captured into a graph).
__global__ void k_clear(double* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Column-transposed unknown-pixel bits of a mask: word (g, x) holds bit j
// = 1 iff pixel (64 g + j, x) is unknown (0 beyond the image). One extra
// all-zero group row follows the last one.
__global__ __launch_bounds__(256) void k_mask_bits(const uint8_t* __restrict__ c, int h, int w,
                                                   int groups, uint64_t* __restrict__ mbits) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int gy = blockIdx.y;
    if (x >= w) return;
    uint64_t bits = 0;
    if (gy < groups - 1) {
        uint8_t m[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            const int y = min(gy * 64 + j, h - 1);
            m[j] = c[(int64_t)y * w + x];
        }
#pragma unroll
        for (int j = 0; j < 64; ++j)
            if (gy * 64 + j < h && m[j] == 0) bits |= 1ull << j;
    }
    mbits[(int64_t)gy * w + x] = bits;
}

// ---------------------------------------------------------------------------
// Level transfer and statistics
// ---------------------------------------------------------------------------

template <int NC>
__global__ __launch_bounds__(kTpb) void k_coarsen(const float* __restrict__ f,
                                                  const uint8_t* __restrict__ c,
                                                  int h, int w, float* __restrict__ fc,
                                                  uint8_t* __restrict__ cc, int hc, int wc,
                                                  double* __restrict__ stats) {
    const int64_t n = (int64_t)hc * wc;
    const int64_t idx = (int64_t)blockIdx.x * kTpb + threadIdx.x;
    double st[NC + 2];
#pragma unroll
    for (int j = 0; j < NC + 2; ++j) st[j] = 0.0;
    if (idx < n) {
        const int I = (int)(idx / wc), J = (int)(idx - (int64_t)I * wc);
        double s[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) s[k] = 0.0;
        int cnt = 0;
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2) {
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                const int i = 2 * I + a2, j = 2 * J + b2;
                if (i < h && j < w) {
                    const int64_t fi = (int64_t)i * w + j;
                    const uint8_t cv = c[fi];
                    if (cv != 0) {
                        ++cnt;
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            const double fv = f[k * (int64_t)h * w + fi];
                            s[k] += fv;
                            st[k] += fv * fv;
                        }
                    }
                    st[NC] += cv != 0 ? 1.0 : 0.0;
                    st[NC + 1] += cv > 1 ? 1.0 : 0.0;
                }
            }
        }
        cc[idx] = cnt > 0 ? 1 : 0;
#pragma unroll
        for (int k = 0; k < NC; ++k)
            fc[k * n + idx] = cnt > 0 ? (float)(s[k] / (double)cnt) : 0.f;
    }
    if (stats) block_reduce<NC + 2>(st, stats + (int64_t)blockIdx.x * (NC + 2));
}

template <int NC>
__global__ __launch_bounds__(kTpb) void k_stats(const float* __restrict__ f,
                                                const uint8_t* __restrict__ c, int64_t n,
                                                double* __restrict__ stats) {
    double st[NC + 2];
#pragma unroll
    for (int j = 0; j < NC + 2; ++j) st[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTpb + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kTpb) {
        const uint8_t cv = c[i];
        if (cv != 0) {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const double fv = f[k * n + i];
                st[k] += fv * fv;
            }
        }
        st[NC] += cv != 0 ? 1.0 : 0.0;
        st[NC + 1] += cv > 1 ? 1.0 : 0.0;
    }
    block_reduce<NC + 2>(st, stats + (int64_t)blockIdx.x * (NC + 2));
}

// Coarsening for widths divisible by 4: a thread makes coarse pixels
// (I, 2t) and (I, 2t + 1) from fine rows 2I, 2I + 1 and columns 4t .. 4t+3
// with one u32 mask load and one float4 per channel and row. Each
// workgroup walks `rows` coarse rows (up to 4 on large levels, so the
// statistics partials stay few; 1 on small ones, for parallelism). Same
// arithmetic as k_coarsen (float64 sum of <= 4 known values).

template <int NC>
__device__ __forceinline__ void coarsen4_body(const float* __restrict__ f,
                                              const uint8_t* __restrict__ c, int h, int w,
                                              float* __restrict__ fc, uint8_t* __restrict__ cc,
                                              int hc, int wc, int rows,
                                              double* __restrict__ stats, int bx, int by,
                                              int gx) {
    const int t = bx * kTpb + threadIdx.x;  // pair of coarse columns
    const int64_t n = (int64_t)h * w, ncs = (int64_t)hc * wc;
    double st[NC + 2];
#pragma unroll
    for (int j = 0; j < NC + 2; ++j) st[j] = 0.0;
    if (4 * t < w) {
        for (int I = by * rows; I < min(hc, (by + 1) * rows); ++I) {
            uint32_t m[2] = {0u, 0u};
            float4 fv[2][NC];
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
                const int y = 2 * I + a2;
                if (y < h) {
                    const int64_t i = coarsen4_in(y, w, t);
                    m[a2] = *reinterpret_cast<const uint32_t*>(c + i);
#pragma unroll
                    for (int k = 0; k < NC; ++k)
                        fv[a2][k] = m[a2] ? *reinterpret_cast<const float4*>(f + k * n + i)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
            double sm[2][NC];
            int cnt[2] = {0, 0};
#pragma unroll
            for (int k = 0; k < NC; ++k) sm[0][k] = sm[1][k] = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
#pragma unroll
                for (int b2 = 0; b2 < 4; ++b2) {
                    const uint32_t cv = (m[a2] >> (8 * b2)) & 0xffu;
                    const int J = b2 >> 1;
                    if (cv != 0) {
                        ++cnt[J];
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            const float4 q = fv[a2][k];
                            const double v = b2 == 0 ? q.x : b2 == 1 ? q.y : b2 == 2 ? q.z : q.w;
                            sm[J][k] += v;
                            st[k] += v * v;
                        }
                    }
                    st[NC] += cv != 0 ? 1.0 : 0.0;
                    st[NC + 1] += cv > 1 ? 1.0 : 0.0;
                }
            }
            const int64_t o = coarsen4_out(I, wc, t);
            *reinterpret_cast<uint16_t*>(cc + o) =
                (uint16_t)((cnt[0] > 0 ? 1 : 0) | ((cnt[1] > 0 ? 1 : 0) << 8));
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                float2 out;
                out.x = cnt[0] > 0 ? (float)(sm[0][k] / (double)cnt[0]) : 0.f;
                out.y = cnt[1] > 0 ? (float)(sm[1][k] / (double)cnt[1]) : 0.f;
                *reinterpret_cast<float2*>(fc + k * ncs + o) = out;
            }
        }
    }
    if (stats) block_reduce<NC + 2>(st, stats + ((int64_t)by * gx + bx) * (NC + 2));
}

template <int NC>
__global__ __launch_bounds__(kTpb) void k_coarsen4(const float* __restrict__ f,
                                                   const uint8_t* __restrict__ c, int h, int w,
                                                   float* __restrict__ fc,
                                                   uint8_t* __restrict__ cc, int hc, int wc,
                                                   int rows, double* __restrict__ stats) {
    coarsen4_body<NC>(f, c, h, w, fc, cc, hc, wc, rows, stats, blockIdx.x, blockIdx.y,
                      gridDim.x);
}

// Two levels of coarsening in one launch (level a -> a + 1 -> a + 2), for
// widths divisible by 8: a thread makes the coarse pixels (I, 2t) and
// (I, 2t + 1) of level a + 2 from rows 2I, 2I + 1 and columns 4t .. 4t + 3
// of level a + 1, which it makes itself (and writes) from rows 4I .. 4I + 3
// and columns 8t .. 8t + 7 of level a. Each level takes the arithmetic of
// k_coarsen4 (float64 sum of <= 4 known values, one rounding to float32),
// so the two levels equal two k_coarsen4 launches bit for bit.
template <int NC>
__device__ __forceinline__ void coarsen2x_body(const float* __restrict__ f,
                                               const uint8_t* __restrict__ c, int h, int w,
                                               float* __restrict__ fm, uint8_t* __restrict__ cm,
                                               int hm, int wm, float* __restrict__ fc,
                                               uint8_t* __restrict__ cc, int hc, int wc,
                                               int rows, int bx, int by) {
    const int t = bx * kTpb + threadIdx.x;
    if (8 * t >= w) return;
    const int64_t n = (int64_t)h * w, nm = (int64_t)hm * wm, ncs = (int64_t)hc * wc;
    for (int I = by * rows; I < min(hc, (by + 1) * rows); ++I) {
        float mv[2][4][NC];
        int mk[2][4];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int Y = 2 * I + r;  // row of level a + 1
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                mk[r][j] = 0;
#pragma unroll
                for (int k = 0; k < NC; ++k) mv[r][j][k] = 0.f;
            }
            if (Y >= hm) continue;
            uint2 m[2] = {make_uint2(0u, 0u), make_uint2(0u, 0u)};
            float4 fv[2][2][NC];
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
                const int y = 2 * Y + a2;
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    fv[a2][0][k] = fv[a2][1][k] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (y < h) {
                    const int64_t i = coarsen8_in(y, w, t);
                    m[a2] = *reinterpret_cast<const uint2*>(c + i);
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        if (m[a2].x) fv[a2][0][k] = *reinterpret_cast<const float4*>(f + k * n + i);
                        if (m[a2].y)
                            fv[a2][1][k] = *reinterpret_cast<const float4*>(f + k * n + i + 4);
                    }
                }
            }
            double sm[4][NC];
            int cnt[4] = {0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int k = 0; k < NC; ++k) sm[j][k] = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2) {
#pragma unroll
                for (int b2 = 0; b2 < 8; ++b2) {
                    const uint32_t word = b2 < 4 ? m[a2].x : m[a2].y;
                    const uint32_t cv = (word >> (8 * (b2 & 3))) & 0xffu;
                    const int J = b2 >> 1;
                    if (cv != 0) {
                        ++cnt[J];
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            const float4 q = fv[a2][b2 >> 2][k];
                            const int e = b2 & 3;
                            sm[J][k] += e == 0 ? q.x : e == 1 ? q.y : e == 2 ? q.z : q.w;
                        }
                    }
                }
            }
            const int64_t o = coarsen8_mid(Y, wm, t);
            *reinterpret_cast<uint32_t*>(cm + o) =
                (uint32_t)(cnt[0] > 0 ? 1 : 0) | ((uint32_t)(cnt[1] > 0 ? 1 : 0) << 8) |
                ((uint32_t)(cnt[2] > 0 ? 1 : 0) << 16) | ((uint32_t)(cnt[3] > 0 ? 1 : 0) << 24);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[j] = cnt[j] > 0 ? (float)(sm[j][k] / (double)cnt[j]) : 0.f;
                    mv[r][j][k] = v[j];
                }
                *reinterpret_cast<float4*>(fm + k * nm + o) = make_float4(v[0], v[1], v[2], v[3]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) mk[r][j] = cnt[j] > 0 ? 1 : 0;
        }
        // level a + 2 from the level a + 1 values just made
        double s2[2][NC];
        int c2[2] = {0, 0};
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < NC; ++k) s2[j][k] = 0.0;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int b2 = 0; b2 < 4; ++b2) {
                if (mk[r][b2]) {
                    ++c2[b2 >> 1];
#pragma unroll
                    for (int k = 0; k < NC; ++k) s2[b2 >> 1][k] += mv[r][b2][k];
                }
            }
        }
        const int64_t o2 = coarsen4_out(I, wc, t);
        *reinterpret_cast<uint16_t*>(cc + o2) =
            (uint16_t)((c2[0] > 0 ? 1 : 0) | ((c2[1] > 0 ? 1 : 0) << 8));
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            float2 out;
            out.x = c2[0] > 0 ? (float)(s2[0][k] / (double)c2[0]) : 0.f;
            out.y = c2[1] > 0 ? (float)(s2[1][k] / (double)c2[1]) : 0.f;
            *reinterpret_cast<float2*>(fc + k * ncs + o2) = out;
        }
    }
}

template <int NC>
__global__ __launch_bounds__(kTpb) void k_coarsen2x(const float* __restrict__ f,
                                                    const uint8_t* __restrict__ c, int h, int w,
                                                    float* __restrict__ fm,
                                                    uint8_t* __restrict__ cm, int hm, int wm,
                                                    float* __restrict__ fc,
                                                    uint8_t* __restrict__ cc, int hc, int wc,
                                                    int rows) {
    coarsen2x_body<NC>(f, c, h, w, fm, cm, hm, wm, fc, cc, hc, wc, rows, blockIdx.x, blockIdx.y);
}

template <int NC>
__global__ __launch_bounds__(kTpb) void k_coarsen4_batch(const LevelJob* __restrict__ jobs,
                                                         int njobs) {
    const int lb = blockIdx.x;
    const LevelJob& J = jobs[find_job(jobs, njobs, lb)];
    const int local = lb - J.wg0;
    coarsen4_body<NC>(J.f, J.c, J.h, J.w, J.fo, J.co, J.hc, J.wc, J.rows, J.stats,
                      local % J.gx, local / J.gx, J.gx);
}

// Prolongation for widths divisible by 4: a thread writes fine pixels
// (y, 4t .. 4t+3) of all channels with one u32 mask load, float4 loads of f
// where the mask is set, and float4 stores. Fine columns 4t .. 4t+3 mix the
// coarse columns (2t, 2t-1), (2t, 2t+1), (2t+1, 2t), (2t+1, 2t+2) (nearer
// first, clamped), so a thread reads coarse columns 2t - 1 .. 2t + 2 of the
// two coarse rows of fine row y: one float2 (2t, 2t + 1: in range and 8-byte
// aligned since the coarse width is even) and two scalars per row and
// channel. Every load is issued before the first result is computed. The
// same pro_mix expression as the fused first sweep and k_prolong.
template <int NC>
__device__ __forceinline__ void prolong4_body(const float* __restrict__ uc, int hc, int wc,
                                              const float* __restrict__ f,
                                              const uint8_t* __restrict__ c, int h, int w,
                                              float* __restrict__ u, int bx, int y) {
    const int t = bx * kTpb + threadIdx.x;
    if (4 * t >= w) return;
    const int64_t n = (int64_t)h * w, ncs = (int64_t)hc * wc;
    const Pro4Addr pa = prolong4_addr(y, t, w, hc, wc);
    const int64_t i = pa.fine;
    const uint32_t m = *reinterpret_cast<const uint32_t*>(c + i);
    // nearer and farther coarse rows of fine row y
    const int J0 = pa.J0, jl = pa.jl, jr = pa.jr;
    // ---- all loads: the coarse values first (unconditional), then f
    // where the mask is set; 32-bit element offsets inside a plane ----
    float2 mn[NC], mf[NC];
    float ln[NC], lf[NC], en[NC], ef[NC];
    const uint32_t on = pa.rn, of = pa.rf;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const float* C = uc + k * ncs;
        mn[k] = *reinterpret_cast<const float2*>(C + (on + J0));
        mf[k] = *reinterpret_cast<const float2*>(C + (of + J0));
        ln[k] = C[on + jl];
        lf[k] = C[of + jl];
        en[k] = C[on + jr];
        ef[k] = C[of + jr];
    }
    float4 fk[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) fk[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (m) {
#pragma unroll
        for (int k = 0; k < NC; ++k) fk[k] = *reinterpret_cast<const float4*>(f + k * n + i);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        // columns first (each coarse row), then rows
        const float o0 = pro_mix(pro_mix(mn[k].x, ln[k]), pro_mix(mf[k].x, lf[k]));
        const float o1 = pro_mix(pro_mix(mn[k].x, mn[k].y), pro_mix(mf[k].x, mf[k].y));
        const float o2 = pro_mix(pro_mix(mn[k].y, mn[k].x), pro_mix(mf[k].y, mf[k].x));
        const float o3 = pro_mix(pro_mix(mn[k].y, en[k]), pro_mix(mf[k].y, ef[k]));
        float4 out;
        out.x = (m & 0xffu) ? fk[k].x : o0;
        out.y = (m & 0xff00u) ? fk[k].y : o1;
        out.z = (m & 0xff0000u) ? fk[k].z : o2;
        out.w = (m & 0xff000000u) ? fk[k].w : o3;
        *reinterpret_cast<float4*>(u + k * n + i) = out;
    }
}

template <int NC>
__global__ __launch_bounds__(kTpb) void k_prolong4(const float* __restrict__ uc, int hc, int wc,
                                                   const float* __restrict__ f,
                                                   const uint8_t* __restrict__ c, int h, int w,
                                                   float* __restrict__ u) {
    const int gx = (w / 4 + kTpb - 1) / kTpb;
    const int L = xcd_band(blockIdx.x, gridDim.x);
    prolong4_body<NC>(uc, hc, wc, f, c, h, w, u, L % gx, L / gx);
}

template <int NC>
__global__ __launch_bounds__(kTpb) void k_prolong4_batch(const LevelJob* __restrict__ jobs,
                                                         int njobs) {
    const int lb = xcd_band(blockIdx.x, gridDim.x);
    const LevelJob& J = jobs[find_job(jobs, njobs, lb)];
    const int local = lb - J.wg0;
    prolong4_body<NC>(J.uc, J.hc, J.wc, J.f, J.c, J.h, J.w, J.u, local % J.gx, local / J.gx);
}

// u = c ? f : 0 for several images (one grid1d range per job).
__global__ __launch_bounds__(kTpb) void k_init_batch(const LevelJob* __restrict__ jobs, int njobs,
                                                     int channels) {
    const int lb = blockIdx.x;
    const LevelJob& J = jobs[find_job(jobs, njobs, lb)];
    const int64_t n = (int64_t)J.h * J.w;
    const int64_t i = (int64_t)(lb - J.wg0) * kTpb + threadIdx.x;
    if (i >= n) return;
    const bool known = J.c[i] != 0;
    for (int k = 0; k < channels; ++k) J.u[k * n + i] = known ? J.f[k * n + i] : 0.f;
}

// Transposed masks of several (image, level) pairs: job range = gx x groups.
__global__ __launch_bounds__(256) void k_mask_bits_batch(const LevelJob* __restrict__ jobs,
                                                         int njobs) {
    const int lb = blockIdx.x;
    const LevelJob& J = jobs[find_job(jobs, njobs, lb)];
    const int local = lb - J.wg0;
    const int h = J.h, w = J.w;
    const int x = (local % J.gx) * 256 + threadIdx.x;
    const int gy = local / J.gx;
    const int groups = mask_bit_groups(h);
    if (x >= w || gy >= groups) return;
    uint64_t bits = 0;
    if (gy < groups - 1) {
        uint8_t m[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) m[j] = J.c[(int64_t)min(gy * 64 + j, h - 1) * w + x];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            if (gy * 64 + j < h && m[j] == 0) bits |= 1ull << j;
    }
    J.mbits[(int64_t)gy * w + x] = bits;
}

// Column-transposed masks of several levels in one launch (grid.z = level).
struct MaskBitsLevels {
    const uint8_t* c[kMaxLevels];
    uint64_t* mbits[kMaxLevels];
    int h[kMaxLevels], w[kMaxLevels];
    int* clear;  // optional: nclear ints zeroed by the first workgroup
    int nclear;
    // optional column sums (the k_reduce of the input statistics, folded
    // into this launch): the extra z slice's workgroup j < ncols writes
    // out[j] = sum_i part[i * stride + j] in k_reduce's order
    const double* part;
    double* out;
    int nrows, stride, ncols;
    // optional initial guess u = c ? f : 0 of one level (the k_init of the
    // coarsest level, folded into this launch): a further z slice
    const float* init_f;
    const uint8_t* init_c;
    float* init_u;
    int64_t init_n;
    int init_ch;
};

__global__ __launch_bounds__(256) void k_mask_bits_levels(MaskBitsLevels L, int nlev) {
    if ((int)blockIdx.z == nlev + (L.ncols > 0 ? 1 : 0)) {  // the initial-guess slice
        const int64_t nth = (int64_t)gridDim.x * gridDim.y * 256;
        for (int64_t i = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
             i < L.init_n; i += nth) {
            const bool known = L.init_c[i] != 0;
            for (int k = 0; k < L.init_ch; ++k)
                L.init_u[k * L.init_n + i] = known ? L.init_f[k * L.init_n + i] : 0.f;
        }
        return;
    }
    if ((int)blockIdx.z == nlev) {  // the column-sum slice (uniform per workgroup)
        const int j = blockIdx.x;
        if (blockIdx.y != 0 || j >= L.ncols) return;
        double acc[1] = {0.0};
        for (int i = threadIdx.x; i < L.nrows; i += kTpb) acc[0] += L.part[(int64_t)i * L.stride + j];
        block_reduce<1>(acc, L.out + j);
        return;
    }
    if (L.clear && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 &&
        (int)threadIdx.x < L.nclear)
        L.clear[threadIdx.x] = 0;
    const int lv = blockIdx.z;
    const int h = L.h[lv], w = L.w[lv];
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int gy = blockIdx.y;
    const int groups = mask_bit_groups(h);
    if (x >= w || gy >= groups) return;
    const uint8_t* c = L.c[lv];
    uint64_t bits = 0;
    if (gy < groups - 1) {
        uint8_t m[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) m[j] = c[(int64_t)min(gy * 64 + j, h - 1) * w + x];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            if (gy * 64 + j < h && m[j] == 0) bits |= 1ull << j;
    }
    L.mbits[lv][(int64_t)gy * w + x] = bits;
}

__global__ __launch_bounds__(kTpb) void k_init(const float* __restrict__ f,
                                               const uint8_t* __restrict__ c, int64_t n,
                                               int channels, float* __restrict__ u) {
    const int64_t i = (int64_t)blockIdx.x * kTpb + threadIdx.x;
    if (i >= n) return;
    const bool known = c[i] != 0;
    for (int k = 0; k < channels; ++k) u[k * n + i] = known ? f[k * n + i] : 0.f;
}

// One thread per coarse cell (I, J) writes the fine pixels 2I + a, 2J + b:
// along each axis the nearer coarse sample is the cell itself and the
// farther its neighbour on the fine pixel's side (clamped), mixed by
// pro_mix, columns first.
__global__ __launch_bounds__(kTpb) void k_prolong(const float* __restrict__ uc, int hc, int wc,
                                                  const float* __restrict__ f,
                                                  const uint8_t* __restrict__ c, int h, int w,
                                                  int channels, float* __restrict__ u) {
    const int J = blockIdx.x * 64 + (threadIdx.x & 63);
    const int I = blockIdx.y * (kTpb / 64) + (threadIdx.x >> 6);
    if (I >= hc || J >= wc) return;
    const int64_t n = (int64_t)h * w, nc = (int64_t)hc * wc;
    const int Im = max(I - 1, 0), Ip = min(I + 1, hc - 1);
    const int Jm = max(J - 1, 0), Jp = min(J + 1, wc - 1);
    for (int k = 0; k < channels; ++k) {
        const float* C = uc + k * nc;
        float q[3][3];
        const int rr[3] = {Im, I, Ip}, cc[3] = {Jm, J, Jp};
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2) q[a2][b2] = C[(int64_t)rr[a2] * wc + cc[b2]];
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2) {
            const int y = 2 * I + a2;
            if (y >= h) break;
            const int rf = a2 == 0 ? 0 : 2;  // farther row: above for even y
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                const int x = 2 * J + b2;
                if (x >= w) break;
                const int cf = b2 == 0 ? 0 : 2;
                const int64_t i = (int64_t)y * w + x;
                const float out = c[i] != 0 ? f[k * n + i]
                                            : pro_mix(pro_mix(q[1][1], q[1][cf]),
                                                      pro_mix(q[rf][1], q[rf][cf]));
                u[k * n + i] = out;
            }
        }
    }
}

// Residual r = b - A v of eq. 7 with v = u (d == nullptr) or v = u + d (d in
// bfloat16: the refinement update). Outputs, each optional: r (float32),
// rhs (bfloat16 of r), vout (v; with ucopy semantics for d == nullptr),
// and the float64 partials of ||r||^2. Skipped once ctl[0] is set.
// FIXED: v equals f on the mask (the refinement keeps u = f and d = 0
// there), so r is 0 there and f is not read: on an unknown pixel the
// stencil takes its known neighbours' values from v.
template <bool REF, bool FIXED = false>
__global__ __launch_bounds__(64 * kWalkWaves) void k_residual_walk(
    const float* __restrict__ f, const uint8_t* __restrict__ c, const float* __restrict__ u,
    const uint16_t* __restrict__ d, int h, int w, int channels, float* __restrict__ r,
    uint16_t* __restrict__ rhs, float* __restrict__ vout, double* __restrict__ partial,
    const int* __restrict__ ctl) {
    constexpr int R = kWalkRows;
    if (ctl && ctl[0] != 0) return;
    const Walk k = walk_geom(h, w);
    const int ch = blockIdx.z;
    const int64_t n = (int64_t)h * w;
    const uint32_t W = w;
    const float* __restrict__ U = u + ch * n;
    const uint16_t* __restrict__ D = REF ? d + ch * n : nullptr;
    const float* __restrict__ F = f + ch * n;
    auto val = [&](uint32_t j) -> float {
        if constexpr (REF) return at32(U, j) + bf16_to_f(at32(D, j));
        else return at32(U, j);
    };
    // every load of the band first: rows y0 - 1 .. y0 + R (clamped to the
    // image: the clamped rows are the reflecting boundary), mask bytes,
    // edge columns, then f where the mask is set
    float v[R + 2], e[R];
    uint32_t cm[R];
#pragma unroll
    for (int t = 0; t < R + 2; ++t)
        v[t] = val(walk_vrow(k, h, t) * W + k.xc);
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const uint32_t row = walk_row(k, h, t) * W;
        cm[t] = at32(c, row + k.xc);
        e[t] = k.edge ? val(row + k.xe) : 0.f;
    }
    float fv[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        if constexpr (FIXED)
            fv[t] = 0.f;
        else
            fv[t] = cm[t] ? at32(F, walk_row(k, h, t) * W + k.xc) : 0.f;
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
        const float ry = cm[t] ? (FIXED ? 0.f : fv[t] - cur)
                               : ((v[t] - cur) + (v[t + 2] - cur)) + ((lft - cur) + (rgt - cur));
        if (k.inb && t < nr) {
            const uint32_t i = walk_out(k, W, t);
            acc += (double)ry * (double)ry;
            if (r) put32(r + ch * n, i, ry);
            if (rhs) put32(rhs + ch * n, i, f_to_bf16(ry));
            if (vout) put32(vout + ch * n, i, cur);
        }
    }
    walk_partial(acc, partial, channels);
}

// The first residual of the refinement fused with the coarse-to-fine start
// (Sec. 4): v = c ? f : the bilinear prolongation of the coarse plane, with
// the arithmetic of k_prolong4 (each coarse row mixed in x, then the nearer
// and farther row mixed in y), written to vout; rhs = bfloat16(b - A v),
// 0 on the mask (v = f there), and the float64 partials of ||b - A v||^2
// laid out as k_residual_walk's. The walk's kWalkRows + 2 rows y0 - 1 + t
// share kWalkRows / 2 + 2 coarse rows, from y0 / 2 - 1 on: row t takes
// index (t + 1) / 2 as the nearer row and the one after it (t even: odd
// fine row) or before it as the farther. The outside column of an edge
// lane (x - 1 for lane 0, x + 1 for lane 63, used only inside the image)
// takes the lane's two coarse columns with the roles of nearer and farther
// swapped. Skipped once ctl[0] is set.
__global__ __launch_bounds__(64 * kWalkWaves) void k_start_residual_walk(
    ProSrc S, int h, int w, uint16_t* __restrict__ rhs, float* __restrict__ vout,
    double* __restrict__ partial, const int* __restrict__ ctl) {
    constexpr int R = kWalkRows;
    constexpr int NQ = R / 2 + 2;
    if (ctl && ctl[0] != 0) return;
    const Walk k = walk_geom(h, w);
    const int ch = blockIdx.z;
    const int64_t n = (int64_t)h * w;
    const uint32_t W = w;
    const float* __restrict__ F = S.f + ch * n;
    const float* __restrict__ Uc = S.uc + (int64_t)ch * S.hc * S.wc;
    const uint32_t cn = k.xc >> 1, cf = (uint32_t)pro_far((int)k.xc, S.wc);
    const int cb = (k.y0 >> 1) - 1;
    // the loads that wait for nothing: mask bytes and coarse rows
    uint32_t cm[R + 2], ce[R];
#pragma unroll
    for (int t = 0; t < R + 2; ++t) cm[t] = at32(S.c, walk_vrow(k, h, t) * W + k.xc);
#pragma unroll
    for (int t = 0; t < R; ++t) ce[t] = k.edge ? at32(S.c, walk_row(k, h, t) * W + k.xe) : 0u;
    float qn[NQ], qf[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const uint32_t row = (uint32_t)min(max(cb + i, 0), S.hc - 1) * (uint32_t)S.wc;
        qn[i] = at32(Uc, row + cn);
        qf[i] = at32(Uc, row + cf);
    }
    // f where the mask is set
    float fv[R + 2], fe[R];
#pragma unroll
    for (int t = 0; t < R + 2; ++t) fv[t] = cm[t] ? at32(F, walk_vrow(k, h, t) * W + k.xc) : 0.f;
#pragma unroll
    for (int t = 0; t < R; ++t) fe[t] = ce[t] ? at32(F, walk_row(k, h, t) * W + k.xe) : 0.f;
    float hq[NQ], he[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        hq[i] = pro_mix(qn[i], qf[i]);
        he[i] = pro_mix(qf[i], qn[i]);
    }
    float v[R + 2], e[R];
#pragma unroll
    for (int t = 0; t < R + 2; ++t) {
        const int ni = (t + 1) / 2, fi = (t & 1) ? ni - 1 : ni + 1;
        v[t] = cm[t] ? fv[t] : pro_mix(hq[ni], hq[fi]);
        if (t >= 1 && k.y0 - 1 + t > h - 1) v[t] = v[t - 1];  // the clamp of walk_vrow
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int ni = (t + 2) / 2, fi = ((t + 1) & 1) ? ni - 1 : ni + 1;
        e[t] = ce[t] ? fe[t] : pro_mix(he[ni], he[fi]);
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
        const float ry = cm[t + 1] ? 0.f
                                   : ((v[t] - cur) + (v[t + 2] - cur)) + ((lft - cur) + (rgt - cur));
        if (k.inb && t < nr) {
            const uint32_t i = walk_out(k, W, t);
            acc += (double)ry * (double)ry;
            put32(rhs + ch * n, i, f_to_bf16(ry));
            put32(vout + ch * n, i, cur);
        }
    }
    walk_partial(acc, partial, gridDim.z);
}

__global__ __launch_bounds__(kTpb) void k_reduce(double* __restrict__ partial, int nrows,
                                                 int stride, double* __restrict__ out, int zero) {
    const int j = blockIdx.x;
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < nrows; i += kTpb) {
        double* p = partial + (int64_t)i * stride + j;
        s[0] += *p;
        if (zero) *p = 0.0;  // each element is read and cleared by one thread
    }
    block_reduce<1>(s, out + j);
}

// Column sums of several images' partials: workgroup (job j, column k).
__global__ __launch_bounds__(kTpb) void k_reduce_batch(const ReduceJob* __restrict__ jobs,
                                                       int ncols) {
    const ReduceJob& J = jobs[blockIdx.x / ncols];
    const int j = blockIdx.x % ncols;
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < J.nrows; i += kTpb) s[0] += J.partial[(int64_t)i * J.stride + j];
    block_reduce<1>(s, J.out + j);
}

// Stop test on the device after finest-level sweep number n (1-based),
// launched only at the sweeps where the test applies. ctl[0] = done,
// ctl[1] = the sweep after which the test passed, ctl[2] = error (1: mask
// byte > 1, 2: empty mask). stats = [||b_k||^2 (k < C), known pixels, bad
// mask bytes]. rel[0] receives max_k ||r_k||^2 / ||b_k||^2 of the sweep's
// input. One workgroup sums the [block][channel] partials of all channels
// in one pass, in a fixed order.

template <int NC>
__device__ __forceinline__ void decide_body(const double* __restrict__ partial, int nb,
                                            const double* __restrict__ stats,
                                            int* __restrict__ ctl, double* __restrict__ rel,
                                            double tol2, int n, int min_n) {
    if (ctl[0] != 0) return;  // an earlier test passed: sweep n did not run
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
    if (threadIdx.x == 0) {
        double worst = 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            double rsq = 0.0;
            for (int j = 0; j < kDecideTpb / 64; ++j) rsq += sm[j][k];
            const double b2 = stats[k];
            const double q = b2 > 0.0 ? rsq / b2 : (rsq > 0.0 ? INFINITY : 0.0);
            worst = fmax(worst, q);
        }
        rel[0] = worst;
        int err = 0;
        if (stats[NC + 1] > 0.0) err = 1;
        else if (!(stats[NC] > 0.0)) err = 2;
        if (err) {
            ctl[2] = err;
            ctl[1] = n;
            ctl[0] = 1;
        } else if (worst <= tol2 && n >= min_n) {
            ctl[1] = n;
            ctl[0] = 1;
        }
    }
}

// mirror (may be null): host-mapped memory that receives ctl[0 .. 4) and
// then rel[0], written by the thread that decides, so the host reads the
// outcome without a copy launch.
template <int NC>
__global__ __launch_bounds__(kDecideTpb) void k_decide(const double* __restrict__ partial, int nb,
                                                       const double* __restrict__ stats,
                                                       int* __restrict__ ctl,
                                                       double* __restrict__ rel, double tol2,
                                                       int n, int* __restrict__ mirror) {
    decide_body<NC>(partial, nb, stats, ctl, rel, tol2, n, 0);
    if (mirror && threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) mirror[j] = ctl[j];
        const long long bits = __double_as_longlong(rel[0]);
        mirror[4] = static_cast<int>(bits);
        mirror[5] = static_cast<int>(bits >> 32);
    }
}

// One stop test per image after finest-level sweep n: workgroup j tests
// job j; an image's test passes only from its own min_sweeps on.
template <int NC>
__global__ __launch_bounds__(kDecideTpb) void k_decide_batch(const DecideJob* __restrict__ jobs,
                                                             int n) {
    const DecideJob& J = jobs[blockIdx.x];
    decide_body<NC>(J.partial, J.nb, J.stats, J.ctl, J.rel, J.tol2, n, J.min_n);
}

__global__ void k_clear_int(int* __restrict__ p, int n) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_decide(const double* partial, int nb, int channels, const double* stats,
                         int* ctl, double* rel, double tol, int n, hipStream_t s, int* mirror) {
    const double tol2 = tol < 0.0 ? -1.0 : tol * tol;  // negative: never passes
    switch (channels) {
#define DDI_CASE(NC)                                                                          \
    case NC:                                                                                  \
        hipLaunchKernelGGL(k_decide<NC>, dim3(1), dim3(kDecideTpb), 0, s, partial, nb, stats, \
                           ctl, rel, tol2, n, mirror);                                        \
        break;
        DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_clear_int(int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_int, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_clear(double* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_clear, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_mask_bits_levels(int n, const uint8_t* const* c, const int* h, const int* w,
                                  uint64_t* const* mbits, hipStream_t s, int* clear,
                                  int nclear, const double* part, int nrows, int stride,
                                  int ncols, double* out, const InitJob* init) {
    if (n < 1 || n > kMaxLevels || nclear < 0 || nclear > 256) return hipErrorInvalidValue;
    const bool sums = part && out && nrows > 0 && ncols > 0;
    if (sums && (stride < ncols || ncols > 65535)) return hipErrorInvalidValue;
    const bool ini = init && init->f && init->c && init->u && init->n > 0 && init->channels > 0;
    if (init && !ini) return hipErrorInvalidValue;
    MaskBitsLevels L;
    L.clear = nclear > 0 ? clear : nullptr;
    L.nclear = nclear;
    L.part = part;
    L.out = out;
    L.nrows = sums ? nrows : 0;
    L.stride = stride;
    L.ncols = sums ? ncols : 0;
    L.init_f = ini ? init->f : nullptr;
    L.init_c = ini ? init->c : nullptr;
    L.init_u = ini ? init->u : nullptr;
    L.init_n = ini ? init->n : 0;
    L.init_ch = ini ? init->channels : 0;
    int gx = 1, gy = 1;
    for (int i = 0; i < n; ++i) {
        L.c[i] = c[i];
        L.mbits[i] = mbits[i];
        L.h[i] = h[i];
        L.w[i] = w[i];
        gx = max(gx, (w[i] + 255) / 256);
        gy = max(gy, mask_bit_groups(h[i]));
    }
    if (sums) gx = max(gx, ncols);
    hipLaunchKernelGGL(k_mask_bits_levels, dim3(gx, gy, n + (sums ? 1 : 0) + (ini ? 1 : 0)),
                       dim3(256), 0, s, L, n);
    return hipGetLastError();
}

hipError_t launch_mask_bits(const uint8_t* c, int h, int w, uint64_t* mbits, hipStream_t s) {
    const int groups = mask_bit_groups(h);
    hipLaunchKernelGGL(k_mask_bits, dim3((w + 255) / 256, groups), dim3(256), 0, s, c, h, w,
                       groups, mbits);
    return hipGetLastError();
}

static int coarsen4_rows(int hc, int gx) { return std::max(1, std::min(4, hc * gx / 2048)); }

int coarsen_partials(int h, int w) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    int n = grid1d((int64_t)hc * wc);  // fallback path
    if (w % 4 == 0) {
        const int gx = (w / 4 + kTpb - 1) / kTpb;
        const int rows = coarsen4_rows(hc, gx);
        n = std::max(n, gx * ((hc + rows - 1) / rows));
    }
    return n;
}

hipError_t launch_coarsen(const float* f, const uint8_t* c, int h, int w, int channels,
                          float* fc, uint8_t* cc, double* stats, int* nwg, hipStream_t s) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    if (coarsen4_ok(f, c, fc, cc, w)) {
        const int gx = (w / 4 + kTpb - 1) / kTpb;
        const int rows = coarsen4_rows(hc, gx);
        dim3 grid(gx, (hc + rows - 1) / rows);
        if (nwg) *nwg = (int)(grid.x * grid.y);
        switch (channels) {
#define DDI_CASE(NC)                                                                         \
    case NC:                                                                                 \
        hipLaunchKernelGGL(k_coarsen4<NC>, grid, dim3(kTpb), 0, s, f, c, h, w, fc, cc, hc, wc, \
                           rows, stats);                                                     \
        break;
            DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int grid = grid1d((int64_t)hc * wc);
    if (nwg) *nwg = grid;
    switch (channels) {
#define DDI_CASE(NC)                                                                       \
    case NC:                                                                               \
        hipLaunchKernelGGL(k_coarsen<NC>, dim3(grid), dim3(kTpb), 0, s, f, c, h, w, fc, cc, \
                           hc, wc, stats);                                                 \
        break;
        DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool coarsen2_ok(const float* f, const uint8_t* c, const float* fm, const uint8_t* cm,
                 const float* fc, const uint8_t* cc, int w) {
    return w % 8 == 0 && aligned(f, 16) && aligned(c, 8) && aligned(fm, 16) && aligned(cm, 4) &&
           aligned(fc, 8) && aligned(cc, 2);
}

int coarsen2_grid(int h, int w, int* gx, int* rows) {
    const int hm = (h + 1) / 2, hc = (hm + 1) / 2;
    *gx = (w / 8 + kTpb - 1) / kTpb;
    *rows = coarsen4_rows(hc, *gx);
    return *gx * ((hc + *rows - 1) / *rows);
}

hipError_t launch_coarsen2(const float* f, const uint8_t* c, int h, int w, int channels,
                           float* fm, uint8_t* cm, float* fc, uint8_t* cc, hipStream_t s) {
    if (!coarsen2_ok(f, c, fm, cm, fc, cc, w)) return hipErrorInvalidValue;
    const int hm = (h + 1) / 2, wm = w / 2, hc = (hm + 1) / 2, wc = wm / 2;
    int gx = 0, rows = 0;
    const int ng = coarsen2_grid(h, w, &gx, &rows);
    const dim3 grid(gx, ng / gx);
    switch (channels) {
#define DDI_CASE(NC)                                                                          \
    case NC:                                                                                  \
        hipLaunchKernelGGL(k_coarsen2x<NC>, grid, dim3(kTpb), 0, s, f, c, h, w, fm, cm, hm, wm, \
                           fc, cc, hc, wc, rows);                                             \
        break;
        DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stats(const float* f, const uint8_t* c, int h, int w, int channels,
                        double* stats, int* nwg, hipStream_t s) {
    const int64_t n = (int64_t)h * w;
    int grid = grid1d(n);
    if (grid > 1024) grid = 1024;
    if (nwg) *nwg = grid;
    switch (channels) {
#define DDI_CASE(NC)                                                                   \
    case NC:                                                                           \
        hipLaunchKernelGGL(k_stats<NC>, dim3(grid), dim3(kTpb), 0, s, f, c, n, stats); \
        break;
        DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(const float* f, const uint8_t* c, int h, int w, int channels, float* u,
                       hipStream_t s) {
    const int64_t n = (int64_t)h * w;
    hipLaunchKernelGGL(k_init, dim3(grid1d(n)), dim3(kTpb), 0, s, f, c, n, channels, u);
    return hipGetLastError();
}

hipError_t launch_prolong(const float* uc, int hc, int wc, const float* f, const uint8_t* c,
                          int h, int w, int channels, float* u, hipStream_t s) {
    if (prolong4_ok(uc, f, c, u, w)) {
        dim3 grid(((w / 4 + kTpb - 1) / kTpb) * h);
        switch (channels) {
#define DDI_CASE(NC)                                                                          \
    case NC:                                                                                  \
        hipLaunchKernelGGL(k_prolong4<NC>, grid, dim3(kTpb), 0, s, uc, hc, wc, f, c, h, w, u); \
        break;
            DDI_CASE(1) DDI_CASE(2) DDI_CASE(3) DDI_CASE(4)
#undef DDI_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    dim3 grid((wc + 63) / 64, (hc + kTpb / 64 - 1) / (kTpb / 64));
    hipLaunchKernelGGL(k_prolong, grid, dim3(kTpb), 0, s, uc, hc, wc, f, c, h, w, channels, u);
    return hipGetLastError();
}

int residual_partials(int h, int w) {
    const dim3 g = walk_grid(h, w, 1);
    return (int)(g.x * g.y);
}

hipError_t launch_residual(const float* f, const uint8_t* c, const float* u, int h, int w,
                           int channels, float* r, float* ucopy, double* partial, int* nwg,
                           hipStream_t s) {
    const dim3 grid = walk_grid(h, w, channels);
    if (nwg) *nwg = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_residual_walk<false>, grid, dim3(64 * kWalkWaves), 0, s, f, c, u,
                       nullptr, h, w, channels, r, nullptr, ucopy, partial, nullptr);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nrows, int stride, int ncols, double* out,
                         hipStream_t s, bool zero) {
    hipLaunchKernelGGL(k_reduce, dim3(ncols), dim3(kTpb), 0, s, const_cast<double*>(partial),
                       nrows, stride, out, zero ? 1 : 0);
    return hipGetLastError();
}

bool coarsen4_ok(const float* f, const uint8_t* c, const float* fc, const uint8_t* cc, int w) {
    return w % 4 == 0 && aligned(f, 16) && aligned(c, 4) && aligned(fc, 8) && aligned(cc, 2);
}

bool prolong4_ok(const float* uc, const float* f, const uint8_t* c, const float* u, int w) {
    return w % 4 == 0 && aligned(uc, 8) && aligned(f, 16) && aligned(c, 4) && aligned(u, 16);
}

int coarsen_rows(const float* f, const uint8_t* c, const float* fc, const uint8_t* cc, int h,
                 int w) {
    int gx, rows;
    if (coarsen4_ok(f, c, fc, cc, w)) return coarsen4_grid(h, w, &gx, &rows);
    return grid1d((int64_t)((h + 1) / 2) * ((w + 1) / 2));
}

int stats_rows(int h, int w) { return std::min(grid1d((int64_t)h * w), 1024); }

int coarsen4_grid(int h, int w, int* gx, int* rows) {
    const int hc = (h + 1) / 2;
    *gx = (w / 4 + kTpb - 1) / kTpb;
    *rows = coarsen4_rows(hc, *gx);
    return *gx * ((hc + *rows - 1) / *rows);
}

int prolong4_grid(int h, int w, int* gx) {
    *gx = (w / 4 + kTpb - 1) / kTpb;
    return *gx * h;
}

int init_grid(int h, int w) { return grid1d((int64_t)h * w); }

int mask_bits_grid(int h, int w, int* gx) {
    *gx = (w + 255) / 256;
    return *gx * mask_bit_groups(h);
}

#define DDI_NC_SWITCH(KERNEL, GRID, BLOCK, ...)                                           \
    switch (channels) {                                                                  \
        case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(GRID), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
        case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
        case 3: hipLaunchKernelGGL(KERNEL<3>, dim3(GRID), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
        case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(GRID), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                            \
    }

hipError_t launch_coarsen_batch(const LevelJob* jobs, int njobs, int total_wg, int channels,
                                hipStream_t s) {
    if (total_wg <= 0) return hipSuccess;
    DDI_NC_SWITCH(k_coarsen4_batch, total_wg, kTpb, jobs, njobs)
    return hipGetLastError();
}

hipError_t launch_prolong_batch(const LevelJob* jobs, int njobs, int total_wg, int channels,
                                hipStream_t s) {
    if (total_wg <= 0) return hipSuccess;
    DDI_NC_SWITCH(k_prolong4_batch, total_wg, kTpb, jobs, njobs)
    return hipGetLastError();
}

hipError_t launch_decide_batch(const DecideJob* jobs, int njobs, int channels, int n,
                               hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    DDI_NC_SWITCH(k_decide_batch, njobs, kDecideTpb, jobs, n)
    return hipGetLastError();
}
#undef DDI_NC_SWITCH

hipError_t launch_init_batch(const LevelJob* jobs, int njobs, int total_wg, int channels,
                             hipStream_t s) {
    if (total_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_batch, dim3(total_wg), dim3(kTpb), 0, s, jobs, njobs, channels);
    return hipGetLastError();
}

hipError_t launch_mask_bits_batch(const LevelJob* jobs, int njobs, int total_wg, hipStream_t s) {
    if (total_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mask_bits_batch, dim3(total_wg), dim3(256), 0, s, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const ReduceJob* jobs, int njobs, int ncols, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_batch, dim3(njobs * ncols), dim3(kTpb), 0, s, jobs, ncols);
    return hipGetLastError();
}

hipError_t launch_start_residual(const ProSrc& S, int h, int w, int channels, float* vout,
                                 uint16_t* rhs, double* partial, const int* ctl, int* nwg,
                                 hipStream_t s) {
    if (S.hc != (h + 1) / 2 || S.wc != (w + 1) / 2) return hipErrorInvalidValue;
    const dim3 grid = walk_grid(h, w, channels);
    if (nwg) *nwg = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_start_residual_walk, grid, dim3(64 * kWalkWaves), 0, s, S, h, w, rhs,
                       vout, partial, ctl);
    return hipGetLastError();
}

hipError_t launch_refine_residual(const float* f, const uint8_t* c, const float* u,
                                  const uint16_t* d, int h, int w, int channels, float* unext,
                                  uint16_t* rhs, double* partial, const int* ctl, int* nwg,
                                  hipStream_t s) {
    const dim3 grid = walk_grid(h, w, channels);
    if (nwg) *nwg = (int)(grid.x * grid.y);
    // u = f and d = 0 on the mask (the caller's precondition): f is not read
    if (d)
        hipLaunchKernelGGL((k_residual_walk<true, true>), grid, dim3(64 * kWalkWaves), 0, s, f, c,
                           u, d, h, w, channels, nullptr, rhs, unext, partial, ctl);
    else
        hipLaunchKernelGGL((k_residual_walk<false, true>), grid, dim3(64 * kWalkWaves), 0, s, f,
                           c, u, nullptr, h, w, channels, nullptr, rhs, nullptr, partial, ctl);
    return hipGetLastError();
}

}  // namespace ddi
