// HIP kernels for gfx950 (CDNA4, wave64) of multilevel ORAS inpainting.
//
//   k_sweep     one ORAS iteration (Sec. 3 eqs. 7-9): block residual, k-step
//               local CG with the Robin interface weight, owned write-back.
//               One wave64 per (block, channel): lanes are block columns, the
//               block's rows live in registers, horizontal neighbours come
//               from DPP lane shifts, CG dot products are wave reductions
//               (DPP row shifts + readlane). No LDS barriers.
//   k_coarsen   dyadic subsampling of mask and known values (Sec. 4).
//   k_stats     ||C f||^2 per channel, known-pixel count, bad mask bytes.
//   k_init      u = c ? f : 0 on the coarsest level.
//   k_prolong   u = c ? f : bilinear(coarse u) (Sec. 4 coarse-to-fine start).
//   k_residual_walk  r = b - A u (eq. 7), float64 partial norms; column-
//               walking waves keep the vertical stencil in registers.
//   k_reduce    fixed-order float64 sums of per-workgroup partials.
//
// All reductions run in a fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <atomic>

#include <hip/hip_ext.h>

#include "access.h"
#include "internal.h"

namespace ddi {
namespace {

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------

// GCN DPP controls: wave_shr:1 moves data one lane up (lane i receives lane
// i - 1), wave_shl:1 one lane down; row_shr:n shifts inside 16-lane rows.
// With bound_ctrl set, lanes whose source does not exist receive 0.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}

// Value held by lane i - 1 (0 in lane 0).
__device__ __forceinline__ float from_left(float x) { return dpp<kDppWaveShr1>(x); }
// Value held by lane i + 1 (0 in lane 63).
__device__ __forceinline__ float from_right(float x) { return dpp<kDppWaveShl1>(x); }

__device__ __forceinline__ float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Sum over the 64 lanes, returned uniformly (fixed order).
__device__ __forceinline__ float wave_sum(float x) {
    x += dpp<0x111>(x);  // row_shr:1
    x += dpp<0x112>(x);  // row_shr:2
    x += dpp<0x114>(x);  // row_shr:4
    x += dpp<0x118>(x);  // row_shr:8 -> lane 15 of each row holds the row sum
    return (readlane(x, 15) + readlane(x, 31)) + (readlane(x, 47) + readlane(x, 63));
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// q where bit `bit` of `bits` is set, +0 elsewhere: a sign-extended bit
// field (v_bfe_i32) ANDed with q. Branch-free, and opaque enough that the
// compiler does not turn it into per-row lane masks held in scalar registers.
__device__ __forceinline__ float mask_keep(uint32_t bits, int bit, float q) {
    const int sel = __builtin_amdgcn_sbfe((int)bits, bit, 1);
    return __int_as_float(__float_as_int(q) & sel);
}

// bfloat16 storage of the correction equation: widen by a 16-bit shift,
// narrow with round-to-nearest-even (inputs are finite).
__device__ __forceinline__ float bf16_to_f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// The same selection with the bit field extract written out: the compiler
// otherwise turns a one-bit v_bfe_i32 into and + compare + select (three
// instructions for two).
__device__ __forceinline__ float mask_bfe(uint32_t bits, int bit, float q) {
    int sel;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(sel) : "v"(bits), "s"(bit));
    return __int_as_float(__float_as_int(q) & sel);
}

// Byte masks: byte k of a word is 0xff where row 4 j + k of the column is
// unknown (bit 4 j + k of the 32-bit mask word), 0 elsewhere.
__device__ __forceinline__ uint32_t mask_bytes(uint32_t bits, int j) {
    const uint32_t nib = (bits >> (4 * j)) & 0xfu;
    return ((nib * 0x00204081u) & 0x01010101u) * 0xffu;
}

// q where byte K of the byte mask m is 0xff, +0 where it is 0: one AND whose
// first operand is that byte sign-extended to 32 bits (an SDWA operand
// select), so a masked row costs one instruction instead of an extract and
// an AND.
template <int K>
__device__ __forceinline__ float mask_byte(uint32_t m, float q) {
    uint32_t out;
    asm("v_and_b32_sdwa %0, sext(%1), %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_%3 src1_sel:DWORD"
        : "=v"(out)
        : "v"(m), "v"(__float_as_uint(q)), "i"(K));
    return __uint_as_float(out);
}
// The same with the byte index as an argument; in unrolled loops it is a
// constant and the switch folds away.
__device__ __forceinline__ float mask_byte(uint32_t m, int k, float q) {
    switch (k & 3) {
        case 0: return mask_byte<0>(m, q);
        case 1: return mask_byte<1>(m, q);
        case 2: return mask_byte<2>(m, q);
        default: return mask_byte<3>(m, q);
    }
}

// Mask of one block column, built from the bits of the unknown pixels.
// Float storage (1 = unknown) for short columns; the bits themselves for
// 64-row columns, where registers are scarce.
template <int RPW, bool BITS>
struct ColMask;

template <int RPW>
struct ColMask<RPW, false> {
    float m[RPW];
    __device__ __forceinline__ void load(uint32_t lo, uint32_t hi) {
#pragma unroll
        for (int y = 0; y < RPW; ++y)
            m[y] = (((y < 32 ? lo : hi) >> (y & 31)) & 1u) ? 1.f : 0.f;
    }
    __device__ __forceinline__ float apply(int y, float q) const { return q * m[y]; }
    __device__ __forceinline__ void refresh() {}
};

template <int RPW>
struct ColMask<RPW, true> {
    uint32_t b[2];
    __device__ __forceinline__ void load(uint32_t lo, uint32_t hi) { b[0] = lo; b[1] = hi; }
    __device__ __forceinline__ float apply(int y, float q) const {
        return mask_keep(b[y >> 5], y & 31, q);
    }
    // Re-define the words once per CG step so that the 64 per-row bit
    // extracts stay inside the loop instead of occupying 64 registers.
    __device__ __forceinline__ void refresh() { asm volatile("" : "+v"(b[0]), "+v"(b[1])); }
};

// ---------------------------------------------------------------------------
// One ORAS sweep
// ---------------------------------------------------------------------------
//
// Block b = (by, bx) of channel ch covers rows [y0, y0 + bh) and columns
// [x0, x0 + bw); lane l holds column x0 + l (lanes >= bw idle). Row y of the
// block is register index y (RPW >= bh; RAGGED when bh < RPW).
//
// Local matrix (one row per unknown pixel p of the block): diagonal = number
// of in-image neighbours inside the block + alpha * number of in-image
// neighbours outside it; -1 towards every unknown neighbour inside the
// block. Known pixels are homogeneous Dirichlet (their correction is 0).
// This is R_i A R_i^T of eq. 7 for alpha = 1 (RAS) and the Robin-modified
// ORAS matrix otherwise (Sec. 3). The diagonal depends only on the position:
// dmid for inner rows (per lane), dtop / dbot for the first / last row.
//
// LDS: the block's u with a one-pixel halo is staged first (the halo copies
// the nearest image pixel where the image ends, which is exactly the
// reflecting boundary of eq. 3); the same memory then parks the CG vector
// q = A p between the matvec and the update when QLDS is set (64-row blocks
// do not fit v, r, p and q in 256 VGPRs).
constexpr int kTileW = kMaxBlock + 2;

// The sweep of logical block lb (channel-major over the block grid) of one
// image, with the block's tile in `lds` ((RPW + 2) x kTileW floats).
//
// CORR = false: the iterate u (float32) of A u = b; the block residual is
// b - A u = L u on unknown pixels.
// CORR = true: the correction d (bfloat16) of the refinement equation
// A d = rhs (d = 0 on the mask, rhs = b - A u of the float32 iterate,
// stored in bfloat16); the block residual is rhs - A d = rhs + L d on
// unknown pixels. uin == nullptr stands for d = 0. Arithmetic is float32 in
// both cases; only the loads widen and the stores narrow.
// CORR and F32: the same correction equation with d and rhs in float32 (the
// preconditioner of the Krylov method).
template <int RPW, bool RAGGED, bool QLDS, bool MBITS, bool CORR = false, bool F32 = false>
__device__ __forceinline__ void sweep_body(const void* __restrict__ uin_v,
                                           const void* __restrict__ rhs,
                                           const uint64_t* __restrict__ mbits,
                                           void* __restrict__ uout_v,
                                           double* __restrict__ partial,
                                           double* __restrict__ cg_steps,
                                           const int* __restrict__ ctl, const SweepArgs& a,
                                           int lb, float* __restrict__ lds) {
    constexpr int TW = kTileW;  // floats per tile row in LDS
    constexpr int CO = 1;       // tile column of block column 0
    // a solve that has already met its stop test skips the sweeps it had
    // enqueued ahead (ctl[0] is set by k_decide)
    if (ctl && ctl[0] != 0) return;

    const int lane = threadIdx.x;
    const BlockGrid g = a.g;
    const Blk kb = blk_geo(g, lb);
    const int ch = kb.ch, b = kb.b, y0 = kb.y0, x0 = kb.x0;
    const int oylo = kb.oylo, oyhi = kb.oyhi, oxlo = kb.oxlo, oxhi = kb.oxhi;

    const float* __restrict__ U = CORR ? nullptr : (const float*)uin_v + ch * a.cpitch;
    const uint16_t* __restrict__ U16 =
        CORR && !F32 && uin_v ? (const uint16_t*)uin_v + ch * a.cpitch : nullptr;
    const float* __restrict__ UF = CORR && F32 && uin_v ? (const float*)uin_v + ch * a.cpitch
                                                        : nullptr;
    const bool on = lane < g.bw;
    const int x = x0 + lane;
    const int nrows = RAGGED ? g.bh : RPW;
    const bool has_top = y0 > 0;
    const bool has_bot = y0 + nrows < g.h;
    const bool has_left = x0 > 0;
    const bool has_right = x0 + g.bw < g.w;

    // ---- stage u (rows y0-1 .. y0+RPW, columns x0-1 .. x0+bw) ----
    // Rows and columns are clamped to the image: a clamped halo copies the
    // border pixel, i.e. the reflecting boundary. All loads are issued
    // before the first LDS write (no branches between them). Offsets are
    // 32-bit element indices into one channel plane (planes hold < 2^30
    // pixels), so each load is one scalar base plus a vector offset.
    auto stage = [&](auto ld) {
        const uint32_t xc = tile_col(kb, g, lane);
        const uint32_t Wd = g.w;
        float col[RPW + 2];
        if constexpr (!RAGGED) {
            // rows y0 .. y0+RPW-1 lie in the image; only the two halo rows
            // can fall outside it (then they copy the border row)
            const Tile2Rows tr = tile1_rows(kb, RPW, Wd, xc);
            uint32_t off = tr.mid0;
            col[0] = ld(tr.first);
#pragma unroll
            for (int t = 1; t <= RPW; ++t) {
                col[t] = ld(off);
                if (t < RPW) off += Wd;
            }
            col[RPW + 1] = ld(tr.last);
        } else {
#pragma unroll
            for (int t = 0; t < RPW + 2; ++t) col[t] = ld(tile_row(kb, g, t) * Wd + xc);
        }
        // halo columns: lane l fetches row l - 1 (and rows 63, 64 in a
        // second pass for lanes 0, 1)
        const uint32_t xl = halo_left(kb), xr = halo_right(kb, g);
        const int t1 = lane, t2 = 64 + lane;
        const uint32_t r1 = tile_row(kb, g, t1) * (uint32_t)g.w;
        const float hl1 = ld(r1 + xl), hr1 = ld(r1 + xr);
        float hl2 = 0.f, hr2 = 0.f;
        if (t2 < RPW + 2) {
            const uint32_t r2 = tile_row(kb, g, t2) * (uint32_t)g.w;
            hl2 = ld(r2 + xl);
            hr2 = ld(r2 + xr);
        }
        if (on) {
#pragma unroll
            for (int t = 0; t < RPW + 2; ++t) lds[t * TW + lane + CO] = col[t];
        }
        if (t1 < RPW + 2) {
            lds[t1 * TW + CO - 1] = hl1;
            lds[t1 * TW + CO + g.bw] = hr1;
        }
        if (t2 < RPW + 2) {
            lds[t2 * TW + CO - 1] = hl2;
            lds[t2 * TW + CO + g.bw] = hr2;
        }
    };
    if constexpr (!CORR) {
        stage([&](uint32_t i) { return U[i]; });
    } else if constexpr (F32) {
        if (UF)
            stage([&](uint32_t i) { return UF[i]; });
        else
            stage([](uint32_t) { return 0.f; });
    } else {
        if (U16)
            stage([&](uint32_t i) { return bf16_to_f(U16[i]); });
        else
            stage([](uint32_t) { return 0.f; });
    }
    // unknown-pixel bits of this column: bit y <-> row y0 + y
    uint32_t mlo = 0u, mhi = 0u;
    if (on) {
        const MaskWords mw = mask_words(kb, (uint32_t)g.w, x);
        const uint64_t* mb = mbits + mw.w0;
        uint64_t bits = mb[0] >> mw.sh;
        if (mw.sh) bits |= mb[g.w] << (64 - mw.sh);
        if (nrows < 64) bits &= (1ull << (nrows & 63)) - 1ull;
        mlo = (uint32_t)bits;
        mhi = (uint32_t)(bits >> 32);
    }
    __syncthreads();

    // ---- residual of u_in on the block (eq. 7) and its owned norm ----
    // One pass over the rows also fills w = u_in (the iterate the local
    // correction is added to) and rho = r.r. The owned-pixel norm is summed
    // per lane over the block's rows in float32 (<= 64 terms) and in float64
    // from there on (across lanes and blocks).
    float r[RPW], w[RPW];
    float rho_l0 = 0.f, rho_l1 = 0.f, own_l = 0.f;
    {
        const int ylo = oylo - y0, yhi = oyhi - y0;
        const float* col = lds + lane + CO;
        float uup = col[0];
        float uy = col[TW];
        const uint16_t* R16 = nullptr;
        const float* RF = nullptr;
        if constexpr (CORR && !F32)
            R16 = (const uint16_t*)rhs + ch * a.cpitch + (uint32_t)(on ? x : x0);
        if constexpr (CORR && F32)
            RF = (const float*)rhs + ch * a.cpitch + (uint32_t)(on ? x : x0);
#pragma unroll
        for (int y = 0; y < RPW; ++y) {
            const float udn = col[(y + 2) * TW];
            const float ul = col[(y + 1) * TW - 1];
            const float ur = col[(y + 1) * TW + 1];
            float lap = ((uup - uy) + (udn - uy)) + ((ul - uy) + (ur - uy));
            if constexpr (CORR) {
                const uint32_t yy = RAGGED ? min(y0 + y, g.h - 1) : y0 + y;
                if constexpr (F32)
                    lap = RF[yy * (uint32_t)g.w] + lap;
                else
                    lap = bf16_to_f(R16[yy * (uint32_t)g.w]) + lap;
            }
            const float ry = mask_keep(y < 32 ? mlo : mhi, y & 31, lap);
            r[y] = ry;
            w[y] = uy;
            const float rq = ry * ry;
            if (y & 1) rho_l1 += rq; else rho_l0 += rq;
            own_l += (y >= ylo && y < yhi) ? rq : 0.f;
            uup = uy;
            uy = udn;
        }
    }
    {
        const bool own_col = on && x >= oxlo && x < oxhi;
        const double rsq = wave_sum_d(own_col ? (double)own_l : 0.0);
        if (lane == 0) partial[(int64_t)b * a.channels + ch] = rsq;
    }

    ColMask<RPW, MBITS> mk;
    mk.load(mlo, mhi);

    // ---- local CG (Sec. 4) from v = 0 ----
    const float al = a.alpha;
    const float wl = (lane > 0) ? 1.f : (has_left ? al : 0.f);
    const float wr = (lane < g.bw - 1) ? 1.f : (has_right ? al : 0.f);
    const float dmid = 2.f + wl + wr;
    const float dtop = dmid - 1.f + (has_top ? al : 0.f);
    const float dbot = dmid - 1.f + (has_bot ? al : 0.f);

    // w = u_in + v: the correction is accumulated straight into the block's
    // own values, so the write-back needs no second read of u_in
    float p[RPW];
#pragma unroll
    for (int y = 0; y < RPW; ++y) p[y] = r[y];
    float rho = wave_sum(rho_l0 + rho_l1);
    // optional absolute stop: mean square local residual below local_tol^2
    const float rho_stop = a.local_tol2 * (float)(g.bh * g.bw);

    __syncthreads();  // the staged tile is dead; its LDS now holds q
    float4* qs = reinterpret_cast<float4*>(lds);
    float qreg[QLDS ? 1 : RPW];
    int it = 0;
    for (; it < a.k; ++it) {
        if (!(rho > rho_stop)) break;
        mk.refresh();
        // q = A_loc p, pq = p . q
        float pq0 = 0.f, pq1 = 0.f;
        float q4[4];
        // keep the last-row test inside the loop (64 hoisted compares would
        // exhaust the scalar registers)
        int last = nrows - 1;
        if constexpr (RAGGED) asm volatile("" : "+s"(last));
#pragma unroll
        for (int y = 0; y < RPW; ++y) {
            float s = ((y > 0) ? p[y - 1] : 0.f) + ((y < RPW - 1) ? p[y + 1] : 0.f);
            s += from_left(p[y]);
            s += from_right(p[y]);
            float d;
            if (!RAGGED) {
                d = (y == 0) ? dtop : ((y == RPW - 1) ? dbot : dmid);
            } else {
                d = dmid;
                if (y == 0) d = dtop;
                if (y == last) d = (y == 0) ? dtop + dbot - dmid : dbot;
            }
            const float q = mk.apply(y, d * p[y] - s);
            if (y & 1) pq1 += p[y] * q; else pq0 += p[y] * q;
            if constexpr (QLDS) {
                q4[y & 3] = q;
                if ((y & 3) == 3)
                    qs[(y >> 2) * 64 + lane] = make_float4(q4[0], q4[1], q4[2], q4[3]);
            } else {
                qreg[y] = q;
            }
        }
        const float pq = wave_sum(pq0 + pq1);
        if (!(pq > 0.f)) {
            ++it;  // the matvec of this step was done
            break;
        }
        const float alpha = rho / pq;
        float rr0 = 0.f, rr1 = 0.f;
        float4 qn;
        if constexpr (QLDS) qn = qs[lane];
#pragma unroll
        for (int y = 0; y < RPW; ++y) {
            float q;
            if constexpr (QLDS) {
                // one float4 group in flight ahead of the one in use
                if ((y & 3) == 0) {
                    q4[0] = qn.x; q4[1] = qn.y; q4[2] = qn.z; q4[3] = qn.w;
                    if (y + 4 < RPW) qn = qs[((y >> 2) + 1) * 64 + lane];
                }
                q = q4[y & 3];
            } else {
                q = qreg[y];
            }
            w[y] += alpha * p[y];
            r[y] -= alpha * q;
            if (y & 1) rr1 += r[y] * r[y]; else rr0 += r[y] * r[y];
            if constexpr (QLDS) {
                if ((y & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
        const float rr = wave_sum(rr0 + rr1);
        const float beta = rr / rho;
        rho = rr;
#pragma unroll
        for (int y = 0; y < RPW; ++y) p[y] = r[y] + beta * p[y];
    }

    // executed CG steps, accumulated in this block's own slot (one wave per
    // block and launch, launches in stream order: no race)
    if (cg_steps && lane == 0) cg_steps[(int64_t)b * a.channels + ch] += (double)it;

    // ---- restricted prolongation: u_out = u_in + v on owned pixels (eq. 9)
    if (on && x >= oxlo && x < oxhi) {
        uint32_t off = out_base(y0, (uint32_t)g.w, x);
        if constexpr (!CORR || F32) {
            float* __restrict__ UO = (float*)uout_v + ch * a.cpitch;
#pragma unroll
            for (int y = 0; y < RPW; ++y) {
                const int yy = y0 + y;
                if ((!RAGGED || y < nrows) && yy >= oylo && yy < oyhi) UO[off] = w[y];
                off += (uint32_t)g.w;
            }
        } else {
            uint16_t* __restrict__ UO = (uint16_t*)uout_v + ch * a.cpitch;
#pragma unroll
            for (int y = 0; y < RPW; ++y) {
                const int yy = y0 + y;
                if ((!RAGGED || y < nrows) && yy >= oylo && yy < oyhi) UO[off] = f_to_bf16(w[y]);
                off += (uint32_t)g.w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One ORAS sweep with two waves per 64 x 64 block
// ---------------------------------------------------------------------------
//
// The same computation as sweep_body for full 64-row blocks, split over a
// 128-thread workgroup: wave wi holds block rows 32 wi .. 32 wi + 31 in
// registers (all four CG vectors, no parking in LDS), the two waves of a
// block run on different SIMDs of the CU, and at about 150 VGPRs three
// waves share each SIMD instead of two. Per CG step the waves meet three
// times in LDS: to swap the boundary rows of p (row 31 <-> row 32) for the
// matvec, and to add their halves of p.q and r.r (wave 0's half first, so
// both waves hold bitwise equal scalars and take the same branches).
// Word 3 of a raw buffer resource on gfx950 (32-bit data, no swizzle) and a
// vector offset that its range check rejects (the load returns 0).
constexpr int kBufferDword3 = 0x00020000;
constexpr uint32_t kBufferOutside = 0x80000000u;
// Floor of the split sweep's local CG: it stops once r.r or p.Ap is at most
// this (a residual of 1e-15 grey levels per block).
constexpr float kCgFloor = 1e-30f;
// LDS floats of a split sweep: the 66 x 66 tile, then the exchange area
// (two p rows, then the per-wave scalars).
constexpr int kSplitLds = (2 * kSplitRows + 2) * kTileW + 2 * 64 + 8;

// This wave's share of a split block's tile, held in registers between the
// loads and the LDS stores: tile rows 33 wi .. 33 wi + 32 of its column
// (tile row t = image row y0 - 1 + t, clamped: the reflecting boundary),
// one row of each halo column, and the block's 64 unknown-pixel bits.
struct Tile2 {
    float col[kSplitRows + 1];
    float hl, hr;
    uint32_t mlo, mhi;
};

// Element i of a plane through a 32-bit byte offset: a uniform base plus an
// unsigned 32-bit offset maps onto one global load with a scalar base
// (element offsets are below 2^30, so the byte offset fits).
template <class T>
__device__ __forceinline__ T at32(const T* base, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void put32(T* base, uint32_t i, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}

// Tile loaders: ld(i) reads element i of the plane, ld.bytes(b) the element
// at byte offset b of a float32 plane (b / 2 for bfloat16).
struct LoadF32 {
    const float* p;
    __device__ __forceinline__ float operator()(uint32_t i) const { return at32(p, i); }
    __device__ __forceinline__ float bytes(uint32_t b) const {
        return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + b);
    }
};
struct LoadBf16 {
    const uint16_t* p;
    __device__ __forceinline__ float operator()(uint32_t i) const { return bf16_to_f(at32(p, i)); }
    __device__ __forceinline__ float bytes(uint32_t b) const {
        return bf16_to_f(*reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(p) + (b >> 1)));
    }
};
struct LoadZero {
    __device__ __forceinline__ float operator()(uint32_t) const { return 0.f; }
    __device__ __forceinline__ float bytes(uint32_t) const { return 0.f; }
};

// Loads (no waits): ld(i) returns the widened value at element offset i of
// the block's channel plane (the plane base is uniform, the offsets 32-bit,
// so every load is one scalar base plus a vector offset).
template <class LD>
__device__ __forceinline__ void tile2_load(Tile2& T, const Blk& k, const SweepArgs& a,
                                           const uint64_t* __restrict__ mbits, LD ld) {
    constexpr int RPW = kSplitRows;
    const BlockGrid& g = a.g;
    const int lane = threadIdx.x & 63;
    const int wi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool on = lane < g.bw;
    const int x = k.x0 + lane;
    const uint32_t xc = tile_col(k, g, lane);
    const uint32_t Wd = g.w;
    // tile row t0 + j = image row y0 - 1 + t0 + j; only tile rows 0 and 65
    // (first of wave 0, last of wave 1) can lie outside the image
    const Tile2Rows tr = tile2_rows(k, wi, Wd, xc);
    T.col[0] = ld(tr.first);
    // byte offsets: one add per row
    const uint32_t bstride = Wd * 4u;
    uint32_t boff = tr.mid0 * 4u;
#pragma unroll
    for (int j = 1; j < RPW; ++j) {
        T.col[j] = ld.bytes(boff);
        boff += bstride;
    }
    T.col[RPW] = ld(tr.last);
    const uint32_t xl = halo_left(k), xr = halo_right(k, g);
    const int th = wi == 0 ? lane : 64 + lane;
    const uint32_t r1 = tile_row(k, g, min(th, 2 * RPW + 1)) * Wd;
    T.hl = ld(r1 + xl);
    T.hr = ld(r1 + xr);
    uint64_t bits = 0;
    if (on) {
        const MaskWords mw = mask_words(k, Wd, x);
        const uint64_t* mb = mbits + mw.w0;
        bits = mb[0] >> mw.sh;
        if (mw.sh) bits |= mb[g.w] << (64 - mw.sh);
    }
    T.mlo = (uint32_t)bits;
    T.mhi = (uint32_t)(bits >> 32);
}

// Bilinear prolongation (Sec. 4; cell-centred, the reading this build
// takes of the paper's coarse-to-fine step): fine pixel y sits at coarse
// coordinate y/2 - 1/4, so along each axis it mixes the coarse sample y >> 1
// with weight 3/4 and that sample's neighbour on the fine pixel's side with
// weight 1/4, the neighbour index clamped to the coarse grid (where both
// weights fall on one sample, which the mix returns exactly). Columns first,
// then rows. Each mix is one rounding of the exact weighted sum of two
// float32 values: the 1/4 product is exact and the 3/4 one is fused.
__device__ __forceinline__ float pro_mix(float near, float far) {
    return __builtin_fmaf(0.75f, near, 0.25f * far);
}
// The prolonged value of fine pixel (y, x) from the coarse plane Uc.
__device__ __forceinline__ float pro_pixel(const ProSrc& S, const float* __restrict__ Uc,
                                           int y, int x) {
    const ProCell p = pro_cell(y, x, S.hc, S.wc);
    return pro_mix(pro_mix(Uc[p.nn], Uc[p.nf]), pro_mix(Uc[p.fn], Uc[p.ff]));
}

// tile2_load for a first sweep: the tile of the prolonged iterate, built
// from the coarse plane and f. The wave's 33 rows ybase .. ybase + 32 need
// coarse rows F0 .. F0 + 17 (F0 = (ybase - 1) >> 1): fine row ybase + j
// takes coarse rows F0 + (s >> 1) (nearer) and the one before or after it
// (s = 1 + Q + j, Q = (ybase - 1) & 1), so the 18 column-mixed coarse rows
// are shared by the fine rows. known: bit j set where row j of this lane is
// a known pixel (its value is f). Every load is a uniform row base plus the
// lane's column. Image rows outside the image (tile rows 0 and 65 at the
// border) are computed clamped and then replaced by their reflection.
template <int Q>
__device__ __forceinline__ void tile2_prolong_rows(Tile2& T, const ProSrc& S,
                                                   const float* __restrict__ Uc,
                                                   const float* __restrict__ F,
                                                   const ProRows& P, uint32_t xc, uint32_t Wd,
                                                   uint32_t klo, uint32_t khi) {
    constexpr int RPW = kSplitRows;
    constexpr int NQ = RPW / 2 + 2;
    const int hmax = P.hmax;
    // Buffer loads: the row offset is a scalar operand and the lane's column
    // the vector offset, so a row costs no vector instruction; a lane that
    // is not known in a row of f gets an offset past the plane, which the
    // buffer's range check turns into 0 without a memory access.
    const uint32_t fbytes = Wd * (uint32_t)(hmax + 1) * 4u;
    const __amdgpu_buffer_rsrc_t rf =
        __builtin_amdgcn_make_buffer_rsrc((void*)F, (short)0, (int)fbytes, kBufferDword3);
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Uc, (short)0, (int)((uint32_t)S.hc * (uint32_t)S.wc * 4u), kBufferDword3);
    const uint32_t xb = xc * 4u, cnb = (xc >> 1) * 4u, cfb = (uint32_t)pro_far((int)xc, S.wc) * 4u;
    // all loads first: f (0 where not known), then the coarse pairs
    float fv[RPW + 1];
    int sel[RPW + 1];
#pragma unroll
    for (int j = 0; j < RPW + 1; ++j) {
        const int y = pro_frow(P, j);
        sel[j] = j < 32 ? __builtin_amdgcn_sbfe((int)klo, j, 1)
                        : __builtin_amdgcn_sbfe((int)khi, j - 32, 1);
        const uint32_t off = (xb & (uint32_t)sel[j]) | (kBufferOutside & ~(uint32_t)sel[j]);
        fv[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                              rf, (int)off, (int)((uint32_t)y * Wd * 4u), 0));
    }
    float qn[NQ], qf[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int so = (int)((uint32_t)pro_crow(P, i, S.hc) * (uint32_t)S.wc * 4u);
        qn[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)cnb, so, 0));
        qf[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)cfb, so, 0));
    }
    float hq[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) hq[i] = pro_mix(qn[i], qf[i]);
#pragma unroll
    for (int j = 0; j < RPW + 1; ++j) {
        const int sj = 1 + Q + j;
        const int in = sj >> 1, ifar = (sj & 1) ? in + 1 : in - 1;
        const float v = pro_mix(hq[in], hq[ifar]);
        // known rows take f
        T.col[j] = __uint_as_float((__float_as_uint(fv[j]) & (uint32_t)sel[j]) |
                                   (__float_as_uint(v) & ~(uint32_t)sel[j]));
    }
}

__device__ __forceinline__ void tile2_load_prolong(Tile2& T, const Blk& k, const SweepArgs& a,
                                                   const uint64_t* __restrict__ mbits,
                                                   const ProSrc& S) {
    constexpr int RPW = kSplitRows;
    const BlockGrid& g = a.g;
    const int lane = threadIdx.x & 63;
    const int wi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool on = lane < g.bw;
    const int x = k.x0 + lane;
    const uint32_t xc = tile_col(k, g, lane);
    const uint32_t Wd = g.w;
    const float* __restrict__ Uc = S.uc + (int64_t)k.ch * S.hc * S.wc;
    const float* __restrict__ F = S.f + k.ch * a.cpitch;
    uint64_t bits = 0;
    if (on) {
        const MaskWords mw = mask_words(k, Wd, x);
        const uint64_t* mb = mbits + mw.w0;
        bits = mb[0] >> mw.sh;
        if (mw.sh) bits |= mb[g.w] << (64 - mw.sh);
    }
    T.mlo = (uint32_t)bits;
    T.mhi = (uint32_t)(bits >> 32);
    // known pixels of this wave's 33 rows: the block's bits, and the mask
    // byte for the halo row (above the block for wave 0, below for wave 1)
    const ProRows P = pro_rows(k, g, wi, xc);
    const uint32_t hknown = (P.hin && at32(S.c, P.hrow) != 0) ? 1u : 0u;
    // bit j of (klo, khi): tile row j of this wave is known
    uint32_t klo, khi;
    if (wi == 0) {
        klo = (~T.mlo << 1) | hknown;
        khi = (~T.mlo) >> 31;
    } else {
        klo = ~T.mhi;
        khi = hknown;
    }
    if ((P.ybase - 1) & 1)
        tile2_prolong_rows<1>(T, S, Uc, F, P, xc, Wd, klo, khi);
    else
        tile2_prolong_rows<0>(T, S, Uc, F, P, xc, Wd, klo, khi);
    // reflecting border: the clamped tile row repeats its neighbour
    if (wi == 0 && !k.has_top) T.col[0] = T.col[1];
    if (wi == 1 && !k.has_bot) T.col[RPW] = T.col[RPW - 1];
    // halo columns: one pixel each per lane th (tile row th)
    const int xl = (int)halo_left(k), xr = (int)halo_right(k, g);
    const int th = wi == 0 ? lane : 64 + lane;
    const int r1 = (int)tile_row(k, g, min(th, 2 * RPW + 1));
    const uint32_t ro = (uint32_t)r1 * Wd;
    const bool kl = at32(S.c, ro + xl) != 0, kr = at32(S.c, ro + xr) != 0;
    const float fl = kl ? at32(F, ro + xl) : 0.f;
    const float fr = kr ? at32(F, ro + xr) : 0.f;
    const float pl = pro_pixel(S, Uc, r1, xl), pr = pro_pixel(S, Uc, r1, xr);
    T.hl = kl ? fl : pl;
    T.hr = kr ? fr : pr;
}

__device__ __forceinline__ void tile2_store(const Tile2& T, const SweepArgs& a,
                                            float* __restrict__ lds) {
    constexpr int RPW = kSplitRows;
    constexpr int TW = kTileW;
    constexpr int CO = 1;
    const int lane = threadIdx.x & 63;
    const int wi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t0 = wi * (RPW + 1);
    if (lane < a.g.bw) {
#pragma unroll
        for (int j = 0; j < RPW + 1; ++j) lds[(t0 + j) * TW + lane + CO] = T.col[j];
    }
    const int th = wi == 0 ? lane : 64 + lane;
    if (th < 2 * RPW + 2) {
        lds[th * TW + CO - 1] = T.hl;
        lds[th * TW + CO + a.g.bw] = T.hr;
    }
}

// Residual, local CG and owned write-back of one split block whose tile is
// in LDS (staged and followed by a barrier). QL: q parked in the wave's half
// of the tile.
// keep: the previous sweep left this block's owned pixels unchanged, so the
// output buffer already holds the input's values there; a block that then
// runs no CG step skips its write-back. fout (may be null) receives the CG
// steps the block ran (0: its output equals its input on its owned pixels).
template <bool CORR, bool QL, bool F32 = false>
__device__ __forceinline__ void sweep2_compute(const Blk& k, uint32_t mw,
                                               const void* __restrict__ rhs,
                                               void* __restrict__ uout_v,
                                               double* __restrict__ partial,
                                               double* __restrict__ cg_steps,
                                               const SweepArgs& a, float* __restrict__ lds,
                                               int* __restrict__ fout = nullptr, int lb = 0,
                                               bool keep = false) {
    constexpr int RPW = kSplitRows;
    constexpr int TW = kTileW;
    constexpr int CO = 1;
    const BlockGrid& g = a.g;
    const int lane = threadIdx.x & 63;
    const int wi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool on = lane < g.bw;
    const int x = k.x0 + lane;
    float* xrow = lds + (2 * RPW + 2) * TW;  // [2][64] boundary rows of p
    float* xs = xrow + 2 * 64;               // [4] per-wave scalars, then 2 doubles
    double* xd = reinterpret_cast<double*>(xs + 4);

    // ---- residual of this wave's rows, owned norm ----
    // The Laplacian as a sum of neighbour differences: near the fixed point
    // the residual is tiny against the grey values, and differences of
    // neighbours keep it accurate where (sum of neighbours) - 4 u would
    // cancel. Each row's contribution to the owned norm is weighted by a
    // wave-uniform 0/1 factor (one fused multiply-add with a scalar operand
    // instead of a select and an add).
    float r[RPW], w[RPW];
    float rho_l0 = 0.f, rho_l1 = 0.f, own_l = 0.f;
    const int ry0 = k.y0 + RPW * wi;
    {
        // owned rows of this wave as a uniform bit mask
        const int ylo = max(k.oylo - ry0, 0), yhi = min(k.oyhi - ry0, RPW);
        const uint32_t ownrows = yhi > ylo ? (uint32_t)(((1ull << (yhi - ylo)) - 1) << ylo) : 0u;
        const float* col = lds + lane + CO + RPW * wi * TW;
        float uup = col[0];
        float uy = col[TW];
        const uint16_t* R16 = nullptr;
        const float* RF = nullptr;
        if constexpr (CORR && !F32) R16 = (const uint16_t*)rhs + k.ch * a.cpitch;
        if constexpr (CORR && F32) RF = (const float*)rhs + k.ch * a.cpitch;
        uint32_t roff = (uint32_t)ry0 * (uint32_t)g.w + (uint32_t)(on ? x : k.x0);
#pragma unroll
        for (int y = 0; y < RPW; ++y) {
            const float udn = col[(y + 2) * TW];
            const float ul = col[(y + 1) * TW - 1];
            const float ur = col[(y + 1) * TW + 1];
            float lap = ((uup - uy) + (udn - uy)) + ((ul - uy) + (ur - uy));
            if constexpr (CORR) {
                if constexpr (F32)
                    lap = at32(RF, roff) + lap;
                else
                    lap = bf16_to_f(at32(R16, roff)) + lap;
                roff += (uint32_t)g.w;
            }
            const float ry = mask_bfe(mw, y, lap);
            r[y] = ry;
            w[y] = uy;
            const float rq = ry * ry;
            if (y & 1) rho_l1 += rq; else rho_l0 += rq;
            const uint32_t wrow = ((ownrows >> y) & 1u) ? 0x3f800000u : 0u;  // 1.f or 0
            own_l = __builtin_fmaf(rq, __uint_as_float(wrow), own_l);
            uup = uy;
            uy = udn;
        }
    }
    {
        const bool own_col = on && x >= k.oxlo && x < k.oxhi;
        const double rsq = wave_sum_d(own_col ? (double)own_l : 0.0);
        const float rw = wave_sum(rho_l0 + rho_l1);
        if (lane == 0) {
            xd[wi] = rsq;
            xs[wi] = rw;
        }
    }
    __syncthreads();
    float rho = xs[0] + xs[1];
    if (wi == 0 && lane == 0) partial[(int64_t)k.b * a.channels + k.ch] = xd[0] + xd[1];

    // ---- local CG from v = 0 (same local matrix as sweep_body) ----
    const float al = a.alpha;
    const float wl = (lane > 0) ? 1.f : (k.has_left ? al : 0.f);
    const float wr = (lane < g.bw - 1) ? 1.f : (k.has_right ? al : 0.f);
    const float dmid = 2.f + wl + wr;
    const float dfirst = wi == 0 ? dmid - 1.f + (k.has_top ? al : 0.f) : dmid;
    const float dlast = wi == 1 ? dmid - 1.f + (k.has_bot ? al : 0.f) : dmid;

    float p[RPW];
    float q[QL ? 1 : RPW];
    float4* qs = reinterpret_cast<float4*>(lds) + wi * (RPW / 4) * 64;
#pragma unroll
    for (int y = 0; y < RPW; ++y) p[y] = r[y];
    // a floor on the local residual and on p.Ap: below it the block's
    // correction is far under a float32 ulp of any grey value, and the
    // reciprocals of the CG scalars stay finite
    const float rho_stop = fmaxf(a.local_tol2 * (float)(g.bh * g.bw), kCgFloor);
    uint32_t mb[RPW / 4];
#pragma unroll
    for (int j = 0; j < RPW / 4; ++j) mb[j] = mask_bytes(mw, j);
    int it = 0;
    for (; it < a.k; ++it) {
        if (!(rho > rho_stop)) break;
        // swap boundary rows: wave 0 sends row 31, wave 1 row 0
        xrow[wi * 64 + lane] = wi == 0 ? p[RPW - 1] : p[0];
        __syncthreads();
        const float pnb = xrow[(1 - wi) * 64 + lane];
        float pq0 = 0.f, pq1 = 0.f;
        float q4[4];
#pragma unroll
        for (int y = 0; y < RPW; ++y) {
            const float up = y > 0 ? p[y - 1] : (wi == 1 ? pnb : 0.f);
            const float dn = y < RPW - 1 ? p[y + 1] : (wi == 0 ? pnb : 0.f);
            float s = up + dn;
            s += from_left(p[y]);
            s += from_right(p[y]);
            const float d = y == 0 ? dfirst : (y == RPW - 1 ? dlast : dmid);
            const float qy = mask_byte(mb[y >> 2], y, d * p[y] - s);
            if constexpr (QL) {
                q4[y & 3] = qy;
                if ((y & 3) == 3) qs[(y >> 2) * 64 + lane] = make_float4(q4[0], q4[1], q4[2], q4[3]);
            } else {
                q[y] = qy;
            }
            if (y & 1) pq1 += p[y] * qy; else pq0 += p[y] * qy;
        }
        const float pqw = wave_sum(pq0 + pq1);
        if (lane == 0) xs[2 + wi] = pqw;
        __syncthreads();
        const float pq = xs[2] + xs[3];
        if (!(pq > kCgFloor)) {
            ++it;
            break;
        }
        // the CG scalars through one reciprocal (about 1 ulp): a tiny
        // perturbation of the step lengths, off the critical path of the
        // exact quotient's scaling and fix-up sequence
        const float alpha = rho * __builtin_amdgcn_rcpf(pq);
        float rr0 = 0.f, rr1 = 0.f;
        float4 qn;
        if constexpr (QL) qn = qs[lane];
#pragma unroll
        for (int y = 0; y < RPW; ++y) {
            float qy;
            if constexpr (QL) {
                if ((y & 3) == 0) {
                    q4[0] = qn.x; q4[1] = qn.y; q4[2] = qn.z; q4[3] = qn.w;
                    if (y + 4 < RPW) qn = qs[((y >> 2) + 1) * 64 + lane];
                }
                qy = q4[y & 3];
            } else {
                qy = q[y];
            }
            w[y] += alpha * p[y];
            r[y] -= alpha * qy;
            if (y & 1) rr1 += r[y] * r[y]; else rr0 += r[y] * r[y];
        }
        const float rrw = wave_sum(rr0 + rr1);
        if (lane == 0) xs[wi] = rrw;
        __syncthreads();
        const float rr = xs[0] + xs[1];
        const float beta = rr * __builtin_amdgcn_rcpf(rho);
        rho = rr;
#pragma unroll
        for (int y = 0; y < RPW; ++y) p[y] = r[y] + beta * p[y];
    }

    if (cg_steps && wi == 0 && lane == 0) cg_steps[(int64_t)k.b * a.channels + k.ch] += (double)it;
    if (fout && wi == 0 && lane == 0) fout[lb] = it;
    if (keep && it == 0) {  // output already equals the input here
        // timing counters: plane 2 counts blocks whose write-back was skipped
        if (cg_steps && wi == 0 && lane == 0)
            cg_steps[2 * (int64_t)a.g.nby * a.g.nbx * a.channels + (int64_t)k.b * a.channels +
                     k.ch] += 1.0;
        return;
    }

    // ---- restricted prolongation on owned pixels (eq. 9): the row test is
    // wave-uniform, the column test per lane ----
    if (on && x >= k.oxlo && x < k.oxhi) {
        const int ylo = k.oylo - ry0, yhi = k.oyhi - ry0;
        uint32_t off = out_base(ry0, (uint32_t)g.w, x);
        if constexpr (!CORR || F32) {
            float* __restrict__ UO = (float*)uout_v + k.ch * a.cpitch;
#pragma unroll
            for (int y = 0; y < RPW; ++y) {
                if (y >= ylo && y < yhi) put32(UO, off, w[y]);
                off += (uint32_t)g.w;
            }
        } else {
            uint16_t* __restrict__ UO = (uint16_t*)uout_v + k.ch * a.cpitch;
#pragma unroll
            for (int y = 0; y < RPW; ++y) {
                if (y >= ylo && y < yhi) put32(UO, off, f_to_bf16(w[y]));
                off += (uint32_t)g.w;
            }
        }
    }
}

// One split block (tile loaded, stored, computed). PRO: the input iterate
// is the prolongation of pro (uin_v unused).
// Workgroup position pos runs logical block pos, or with a dispatch table
// (order_run) the block of entry pos.
// fin (may be null): the CG steps of the previous sweep's blocks (0 = block
// left unchanged, see sweep2_compute), fout those of this sweep. A block
// whose tile lies in blocks that the previous sweep all left unchanged has
// the same input as then, so the same residual and again no CG step: it
// keeps its partial and its output (which already holds these values) and
// exits. Each tile lies in the owned pixels of its own block and its 8
// neighbours (the host passes fin only for grids where this holds).
template <bool CORR, bool QL, bool PRO = false, bool F32 = false>
__device__ __forceinline__ void sweep2_body(const void* __restrict__ uin_v,
                                            const void* __restrict__ rhs,
                                            const uint64_t* __restrict__ mbits,
                                            void* __restrict__ uout_v,
                                            double* __restrict__ partial,
                                            double* __restrict__ cg_steps,
                                            const int* __restrict__ ctl, const SweepArgs& a,
                                            int pos, float* __restrict__ lds,
                                            const ProSrc* pro = nullptr,
                                            const int* __restrict__ fin = nullptr,
                                            int* __restrict__ fout = nullptr,
                                            const int* __restrict__ order = nullptr) {
    // the control word, the table entry and the keys are uniform loads, read
    // by both waves, so both take the same decisions
    const int stop = ctl ? ctl[0] : 0;
    const int lb = order ? order[pos] : pos;
    bool keep = false, same = false;
    const Blk k = blk_geo(a.g, lb);
    if (fin) {
        const int* F = fin + (int64_t)k.ch * a.g.nby * a.g.nbx;
        int cell[9];
        flag_cells(k, a.g, cell);
        const int own = F[cell[0]];
        const int nb = (F[cell[1]] | F[cell[2]] | F[cell[3]]) | (F[cell[4]] | F[cell[5]]) |
                       (F[cell[6]] | F[cell[7]] | F[cell[8]]);
        keep = own == 0;
        same = (own | nb) == 0;
    }
    if (stop != 0) return;
    if (same) {
        if (threadIdx.x == 0) {
            if (fout) fout[lb] = 0;
            // timing counters: plane 1 counts blocks skipped whole
            if (cg_steps)
                cg_steps[(int64_t)a.g.nby * a.g.nbx * a.channels + (int64_t)k.b * a.channels +
                         k.ch] += 1.0;
        }
        return;
    }
    Tile2 T;
    if constexpr (PRO) {
        tile2_load_prolong(T, k, a, mbits, *pro);
    } else if constexpr (!CORR) {
        tile2_load(T, k, a, mbits, LoadF32{(const float*)uin_v + k.ch * a.cpitch});
    } else if constexpr (F32) {
        const float* UF = (const float*)uin_v;
        if (UF)
            tile2_load(T, k, a, mbits, LoadF32{UF + k.ch * a.cpitch});
        else
            tile2_load(T, k, a, mbits, LoadZero{});
    } else {
        const uint16_t* U16 = (const uint16_t*)uin_v;
        if (U16)
            tile2_load(T, k, a, mbits, LoadBf16{U16 + k.ch * a.cpitch});
        else
            tile2_load(T, k, a, mbits, LoadZero{});
    }
    tile2_store(T, a, lds);
    const uint32_t mw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) ? T.mhi : T.mlo;
    __syncthreads();
    sweep2_compute<CORR, QL, F32>(k, mw, rhs, uout_v, partial, cg_steps, a, lds, fout, lb, keep);
}

// ---------------------------------------------------------------------------
// Dispatch order of a sweep (blocks with the longest local solves first)
// ---------------------------------------------------------------------------
//
// One workgroup of NT threads sorts the blocks of a grid into kOrderBuckets
// buckets by a key per block, stably (a counting sort): thread t owns the
// t-th contiguous run of the logical block order, counts its blocks per
// bucket in registers, a workgroup-wide exclusive scan of those counts (four
// 16-bit counters packed per 64-bit word) gives every thread its first rank
// in each bucket, and the thread then writes its run's blocks to
// consecutive ranks. Buckets run from the most CG steps down to none. The
// key of a block is that of the block of a coarser grid over its centre.
// Equal buckets keep their logical order, so consecutive workgroups still
// cover neighbouring blocks. sh: LDS for the coarse keys and two axis
// tables (cap ints); wsum: NT / 64 words of LDS.
constexpr int kOrderBuckets = 8;
static_assert(kOrderMaxAxes < kSplitLds, "axis tables of a dispatch table fit in a sweep's LDS");

// Bucket of a block whose coarse block ran `key` CG steps (0 = first).
__device__ __forceinline__ int order_bucket_of(int key) {
    return key >= 12 ? 0 : key >= 8 ? 1 : key >= 5 ? 2 : key >= 3 ? 3 : 6 - min(max(key, 0), 2);
}

// Exclusive scan of v over the workgroup (threads in order); *total gets
// the workgroup sum.
template <int NT>
__device__ __forceinline__ uint64_t order_scan(uint64_t v, uint64_t* wsum, uint64_t* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const uint64_t t = wsum[w];
        if (w < wv) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <int NT>
__device__ void order_run(const OrderArgs& A, int* __restrict__ sh, int cap,
                          uint64_t* __restrict__ wsum) {
    const BlockGrid& g = A.g;
    const BlockGrid& c = A.cg;
    const int tid = threadIdx.x;
    const int nblk = g.nby * g.nbx, n = nblk * A.channels;
    const int nk = c.nby * c.nbx * A.channels;
    // coarse block row / column over each fine block's centre
    int* cby_of = sh;
    int* cbx_of = sh + g.nby;
    for (int y = tid; y < g.nby; y += NT)
        cby_of[y] = min(((block_origin(y, g.sy, g.h, g.bh) + g.bh / 2) / A.scale) / c.sy,
                        c.nby - 1);
    for (int x = tid; x < g.nbx; x += NT)
        cbx_of[x] = min(((block_origin(x, g.sx, g.w, g.bw) + g.bw / 2) / A.scale) / c.sx,
                        c.nbx - 1);
    const int* K = A.keys;
    int* sk = sh + g.nby + g.nbx;
    if (nk <= cap - g.nby - g.nbx) {
        for (int i = tid; i < nk; i += NT) sk[i] = A.keys[i];
        K = sk;
    }
    __syncthreads();
    const int per = (n + NT - 1) / NT;
    const int lo = min(tid * per, n), hi = min(lo + per, n);
    const int ch0 = lo / nblk, by0 = (lo - ch0 * nblk) / g.nbx, bx0 = lo - ch0 * nblk - by0 * g.nbx;
    auto bucket = [&](int ch, int by, int bx) {
        return order_bucket_of(K[(ch * c.nby + cby_of[by]) * c.nbx + cbx_of[bx]]);
    };
    uint64_t c03 = 0, c47 = 0;
    {
        int ch = ch0, by = by0, bx = bx0;
        for (int i = lo; i < hi; ++i) {
            const int bk = bucket(ch, by, bx);
            if (bk < 4) c03 += 1ull << (16 * bk); else c47 += 1ull << (16 * (bk - 4));
            if (++bx == g.nbx) {
                bx = 0;
                if (++by == g.nby) { by = 0; ++ch; }
            }
        }
    }
    uint64_t t03, t47;
    const uint64_t r03 = order_scan<NT>(c03, wsum, &t03);
    const uint64_t r47 = order_scan<NT>(c47, wsum, &t47);
    int rank[kOrderBuckets];
    {
        int base = 0;
#pragma unroll
        for (int k = 0; k < kOrderBuckets; ++k) {
            const uint64_t tw = k < 4 ? t03 : t47, rw = k < 4 ? r03 : r47;
            const int sh16 = 16 * (k & 3);
            rank[k] = base + (int)((rw >> sh16) & 0xffff);
            base += (int)((tw >> sh16) & 0xffff);
        }
    }
    int ch = ch0, by = by0, bx = bx0;
    for (int i = lo; i < hi; ++i) {
        const int bk = bucket(ch, by, bx);
        int r = 0;
#pragma unroll
        for (int k = 0; k < kOrderBuckets; ++k)
            if (bk == k) r = rank[k]++;
        A.order[r] = i;
        if (++bx == g.nbx) {
            bx = 0;
            if (++by == g.nby) { by = 0; ++ch; }
        }
    }
}

// The extra last workgroup of a sweep launch that carries an order job
// builds the dispatch table of a later sweep instead of running a block.
__device__ __forceinline__ bool order_job(const OrderArgs& job, float* __restrict__ lds) {
    if (!job.order || blockIdx.x != gridDim.x - 1) return false;
    __shared__ uint64_t wsum[2];
    order_run<128>(job, reinterpret_cast<int*>(lds), kSplitLds, wsum);
    return true;
}

#ifndef DDI_SPLIT_QL
#define DDI_SPLIT_QL 1
#endif
#ifndef DDI_SPLIT_WAVES
#define DDI_SPLIT_WAVES 4
#endif
template <bool CORR>
__global__ __launch_bounds__(128, DDI_SPLIT_WAVES) void k_sweep2(const void* __restrict__ uin,
                                                const uint16_t* __restrict__ rhs,
                                                const uint64_t* __restrict__ mbits,
                                                void* __restrict__ uout,
                                                double* __restrict__ partial,
                                                double* __restrict__ cg_steps,
                                                const int* __restrict__ ctl, SweepArgs a,
                                                const int* __restrict__ fin,
                                                int* __restrict__ fout,
                                                const int* __restrict__ order, OrderArgs job) {
    __shared__ __attribute__((aligned(16))) float lds[kSplitLds];
    if (order_job(job, lds)) return;
    const int nwg = gridDim.x - (job.order ? 1 : 0);
    sweep2_body<CORR, DDI_SPLIT_QL>(uin, rhs, mbits, uout, partial, cg_steps, ctl, a,
                                    xcd_remap(blockIdx.x, nwg), lds, nullptr, fin, fout,
                                    order);
}

// k_sweep2 whose input iterate is the bilinear prolongation of a coarser
// level, computed in the tile load.
__global__ __launch_bounds__(128, DDI_SPLIT_WAVES) void k_sweep2_pro(ProSrc pro,
                                                    const uint64_t* __restrict__ mbits,
                                                    float* __restrict__ uout,
                                                    double* __restrict__ partial,
                                                    double* __restrict__ cg_steps,
                                                    const int* __restrict__ ctl, SweepArgs a,
                                                    int* __restrict__ fout,
                                                    const int* __restrict__ order,
                                                    OrderArgs job) {
    __shared__ __attribute__((aligned(16))) float lds[kSplitLds];
    if (order_job(job, lds)) return;
    const int nwg = gridDim.x - (job.order ? 1 : 0);
    sweep2_body<false, DDI_SPLIT_QL, true>(nullptr, nullptr, mbits, uout, partial, cg_steps, ctl,
                                           a, xcd_remap(blockIdx.x, nwg), lds, &pro, nullptr,
                                           fout, order);
}


// Zero fill (a kernel rather than hipMemsetAsync, so that the solve can be
// captured into a graph).
__global__ void k_clear(double* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <int RPW, bool RAGGED, bool QLDS, bool MBITS>
__global__ __launch_bounds__(64) void k_sweep(const float* __restrict__ uin,
                                              const uint64_t* __restrict__ mbits,
                                              float* __restrict__ uout,
                                              double* __restrict__ partial,
                                              double* __restrict__ cg_steps,
                                              const int* __restrict__ ctl, SweepArgs a) {
    __shared__ __attribute__((aligned(16))) float lds[(RPW + 2) * kTileW];
    sweep_body<RPW, RAGGED, QLDS, MBITS>(uin, nullptr, mbits, uout, partial, cg_steps, ctl, a,
                                         xcd_remap(blockIdx.x, gridDim.x), lds);
}

// One sweep of the refinement equation A d = rhs with d and rhs in
// bfloat16 (din == nullptr: d = 0).
template <int RPW, bool RAGGED, bool QLDS, bool MBITS>
__global__ __launch_bounds__(64) void k_sweep_corr(const uint16_t* __restrict__ din,
                                                   const uint16_t* __restrict__ rhs,
                                                   const uint64_t* __restrict__ mbits,
                                                   uint16_t* __restrict__ dout,
                                                   double* __restrict__ partial,
                                                   double* __restrict__ cg_steps,
                                                   const int* __restrict__ ctl, SweepArgs a) {
    __shared__ __attribute__((aligned(16))) float lds[(RPW + 2) * kTileW];
    sweep_body<RPW, RAGGED, QLDS, MBITS, true>(din, rhs, mbits, dout, partial, cg_steps, ctl, a,
                                               xcd_remap(blockIdx.x, gridDim.x), lds);
}

// One sweep of the correction equation A d = rhs with d and rhs in float32
// (din == nullptr: d = 0): the ORAS preconditioner of the Krylov method.
template <int RPW, bool RAGGED, bool QLDS, bool MBITS>
__global__ __launch_bounds__(64) void k_sweep_c32(const float* __restrict__ din,
                                                  const float* __restrict__ rhs,
                                                  const uint64_t* __restrict__ mbits,
                                                  float* __restrict__ dout,
                                                  double* __restrict__ partial,
                                                  double* __restrict__ cg_steps,
                                                  const int* __restrict__ ctl, SweepArgs a) {
    __shared__ __attribute__((aligned(16))) float lds[(RPW + 2) * kTileW];
    sweep_body<RPW, RAGGED, QLDS, MBITS, true, true>(din, rhs, mbits, dout, partial, cg_steps,
                                                     ctl, a, xcd_remap(blockIdx.x, gridDim.x),
                                                     lds);
}

// Split (two-wave) variant for full 64-row blocks.
__global__ __launch_bounds__(128, DDI_SPLIT_WAVES) void k_sweep2_c32(
    const float* __restrict__ din, const float* __restrict__ rhs,
    const uint64_t* __restrict__ mbits, float* __restrict__ dout, double* __restrict__ partial,
    double* __restrict__ cg_steps, const int* __restrict__ ctl, SweepArgs a) {
    __shared__ __attribute__((aligned(16))) float lds[kSplitLds];
    sweep2_body<true, DDI_SPLIT_QL, false, true>(din, rhs, mbits, dout, partial, cg_steps, ctl,
                                                 a, xcd_remap(blockIdx.x, gridDim.x), lds);
}

// Index of the job whose workgroup range holds logical workgroup lb (jobs
// sorted by wg0, jobs[0].wg0 == 0).
template <class Job>
__device__ __forceinline__ int find_job(const Job* __restrict__ jobs, int njobs, int lb) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg0 <= lb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One ORAS sweep over the blocks of several images in one launch; the
// logical workgroup order runs image after image, so the XCD interleave
// keeps neighbouring blocks of an image together.
template <int RPW, bool RAGGED, bool QLDS, bool MBITS>
__global__ __launch_bounds__(64) void k_sweep_batch(const SweepJob* __restrict__ jobs,
                                                    int njobs) {
    __shared__ __attribute__((aligned(16))) float lds[(RPW + 2) * kTileW];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const SweepJob& J = jobs[find_job(jobs, njobs, lb)];
    sweep_body<RPW, RAGGED, QLDS, MBITS>(J.uin, nullptr, J.mbits, J.uout, J.partial, J.cg_steps,
                                         J.ctl, J.a, lb - J.wg0, lds);
}

// Split-sweep variant of k_sweep_batch (every job has full 64-row blocks).
__global__ __launch_bounds__(128, DDI_SPLIT_WAVES) void k_sweep2_batch(const SweepJob* __restrict__ jobs,
                                                      int njobs) {
    __shared__ __attribute__((aligned(16))) float lds[kSplitLds];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const SweepJob& J = jobs[find_job(jobs, njobs, lb)];
    if (J.pro.uc)  // uniform per workgroup
        sweep2_body<false, DDI_SPLIT_QL, true>(nullptr, nullptr, J.mbits, J.uout, J.partial,
                                               J.cg_steps, J.ctl, J.a, lb - J.wg0, lds, &J.pro);
    else
        sweep2_body<false, DDI_SPLIT_QL>(J.uin, nullptr, J.mbits, J.uout, J.partial, J.cg_steps,
                                         J.ctl, J.a, lb - J.wg0, lds, nullptr, J.fin, J.fout);
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

constexpr int kTpb = 256;

// Fixed-order block reduction of NV doubles per thread into out[0..NV):
// wave sums, then thread 0 adds the kTpb / 64 wave results in order.
template <int NV>
__device__ void block_reduce(double (&val)[NV], double* out) {
    __shared__ double sm[kTpb / 64][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) val[j] = wave_sum_d(val[j]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) sm[threadIdx.x >> 6][j] = val[j];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kTpb / 64; ++i) s += sm[i][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

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
};

__global__ __launch_bounds__(256) void k_mask_bits_levels(MaskBitsLevels L, int nlev) {
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

// ---------------------------------------------------------------------------
// Column-walking stencil kernels. A workgroup is kWalkWaves waves side by
// side, each covering 64 consecutive columns of a band of kWalkRows rows;
// every lane walks down its column and keeps the rows above and below in
// registers, so each value is loaded once. Horizontal neighbours come from
// the neighbouring lanes (DPP); the columns just left and right of a wave
// come from one extra load per row in lanes 0 and 63. A missing neighbour
// at the image border takes the pixel's own value, so its difference is
// 0: the reflecting boundary. One float64 partial per workgroup and
// channel, in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Walk walk_geom(int h, int w) {
    return walk_at(h, w, blockIdx.x, blockIdx.y, threadIdx.x);
}

// Sum of acc over the workgroup into partial[wg][ch] (fixed order).
__device__ __forceinline__ void walk_partial(double acc, double* __restrict__ partial,
                                             int channels) {
    acc = wave_sum_d(acc);
    __shared__ double sm[kWalkWaves];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kWalkWaves; ++j) t += sm[j];
        partial[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * channels + blockIdx.z] = t;
    }
}

// Residual r = b - A v of eq. 7 with v = u (d == nullptr) or v = u + d (d in
// bfloat16: the refinement update). Outputs, each optional: r (float32),
// rhs (bfloat16 of r), vout (v; with ucopy semantics for d == nullptr),
// and the float64 partials of ||r||^2. Skipped once ctl[0] is set.
template <bool REF>
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
    for (int t = 0; t < R; ++t)
        fv[t] = cm[t] ? at32(F, walk_row(k, h, t) * W + k.xc) : 0.f;
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
        const float ry = cm[t] ? fv[t] - cur
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
constexpr int kDecideTpb = 1024;

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

template <int NC>
__global__ __launch_bounds__(kDecideTpb) void k_decide(const double* __restrict__ partial, int nb,
                                                       const double* __restrict__ stats,
                                                       int* __restrict__ ctl,
                                                       double* __restrict__ rel, double tol2,
                                                       int n) {
    decide_body<NC>(partial, nb, stats, ctl, rel, tol2, n, 0);
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Full 64-row blocks take the two-wave split sweep.
#ifndef DDI_SPLIT
#define DDI_SPLIT 1
#endif
static bool use_split(const SweepArgs& a) { return DDI_SPLIT && a.g.bh == 2 * kSplitRows; }

// Along one axis, does every block's tile (the block and its one-pixel
// halo, clamped to the level) lie in the pixels owned by the block and its
// two neighbours? Then a sweep may skip blocks whose 3 x 3 neighbourhood the
// previous sweep left unchanged.
static bool skip_axis_ok(int n, int nb, int stride, int size) {
    for (int k = 0; k < nb; ++k) {
        const int o = block_origin(k, stride, n, size);
        const int lo = std::max(o - 1, 0), hi = std::min(o + size, n - 1);
        int l0, h0, l2, h2;
        owner_range(std::max(k - 1, 0), nb, stride, n, size, &l0, &h0);
        owner_range(std::min(k + 1, nb - 1), nb, stride, n, size, &l2, &h2);
        if (lo < l0 || hi >= h2) return false;
    }
    return true;
}
static bool skip_grid_ok(const BlockGrid& g) {
    return skip_axis_ok(g.h, g.nby, g.sy, g.bh) && skip_axis_ok(g.w, g.nbx, g.sx, g.bw);
}


// A launch, or with timing events (ev0, ev1 non-null) a launch whose
// dispatch packet records the kernel's own start and end in them (no
// dispatch gap inside the bracket).
template <class K, class... Args>
static hipError_t launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t ev0,
                               hipEvent_t ev1, Args... args) {
    if (ev0 && ev1)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev0, ev1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return hipGetLastError();
}

template <int RPW, bool QLDS, bool MBITS>
static hipError_t sweep_rpw(const float* uin, const uint64_t* mbits, float* uout,
                            double* partial, double* cg_steps, const int* ctl,
                            const SweepArgs& a, hipStream_t s, const int* fin = nullptr,
                            int* fout = nullptr, const int* order = nullptr,
                            const OrderArgs* job = nullptr, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr) {
    const int grid = a.g.nby * a.g.nbx * a.channels;
    if (use_split(a)) {
        const OrderArgs j = job ? *job : OrderArgs{};
        return launch_timed(k_sweep2<false>, dim3(grid + (job ? 1 : 0)), dim3(128), s, ev0, ev1,
                            (const void*)uin, (const uint16_t*)nullptr, mbits, (void*)uout,
                            partial, cg_steps, ctl, a, fin, fout, order, j);
    }
    if (a.g.bh == RPW)
        return launch_timed(k_sweep<RPW, false, QLDS, MBITS>, dim3(grid), dim3(64), s, ev0, ev1,
                            uin, mbits, uout, partial, cg_steps, ctl, a);
    return launch_timed(k_sweep<RPW, true, QLDS, MBITS>, dim3(grid), dim3(64), s, ev0, ev1, uin,
                        mbits, uout, partial, cg_steps, ctl, a);
}

template <int RPW, bool QLDS, bool MBITS>
static hipError_t sweep_corr_rpw(const uint16_t* din, const uint16_t* rhs,
                                 const uint64_t* mbits, uint16_t* dout, double* partial,
                                 double* cg_steps, const int* ctl, const SweepArgs& a,
                                 hipStream_t s) {
    const int grid = a.g.nby * a.g.nbx * a.channels;
    if (use_split(a)) {
        hipLaunchKernelGGL((k_sweep2<true>), dim3(grid), dim3(128), 0, s, din, rhs, mbits, dout,
                           partial, cg_steps, ctl, a, (const int*)nullptr, (int*)nullptr,
                           (const int*)nullptr, OrderArgs{});
        return hipGetLastError();
    }
    if (a.g.bh == RPW)
        hipLaunchKernelGGL((k_sweep_corr<RPW, false, QLDS, MBITS>), dim3(grid), dim3(64), 0, s,
                           din, rhs, mbits, dout, partial, cg_steps, ctl, a);
    else
        hipLaunchKernelGGL((k_sweep_corr<RPW, true, QLDS, MBITS>), dim3(grid), dim3(64), 0, s,
                           din, rhs, mbits, dout, partial, cg_steps, ctl, a);
    return hipGetLastError();
}

template <int RPW, bool QLDS, bool MBITS>
static hipError_t sweep_c32_rpw(const float* din, const float* rhs, const uint64_t* mbits,
                                float* dout, double* partial, double* cg_steps, const int* ctl,
                                const SweepArgs& a, hipStream_t s) {
    const int grid = a.g.nby * a.g.nbx * a.channels;
    if (use_split(a)) {
        hipLaunchKernelGGL(k_sweep2_c32, dim3(grid), dim3(128), 0, s, din, rhs, mbits, dout,
                           partial, cg_steps, ctl, a);
        return hipGetLastError();
    }
    if (a.g.bh == RPW)
        hipLaunchKernelGGL((k_sweep_c32<RPW, false, QLDS, MBITS>), dim3(grid), dim3(64), 0, s,
                           din, rhs, mbits, dout, partial, cg_steps, ctl, a);
    else
        hipLaunchKernelGGL((k_sweep_c32<RPW, true, QLDS, MBITS>), dim3(grid), dim3(64), 0, s,
                           din, rhs, mbits, dout, partial, cg_steps, ctl, a);
    return hipGetLastError();
}

hipError_t launch_sweep_c32(const float* din, const float* rhs, const uint64_t* mbits,
                            float* dout, double* partial, double* cg_steps, const int* ctl,
                            const SweepArgs& a, hipStream_t s) {
    const int bh = a.g.bh;
    if (a.g.bw < 1 || a.g.bw > kMaxBlock || bh < 1 || bh > kMaxBlock) return hipErrorInvalidValue;
    if (bh > 32)
        return sweep_c32_rpw<64, true, true>(din, rhs, mbits, dout, partial, cg_steps, ctl, a, s);
    if (bh > 16)
        return sweep_c32_rpw<32, false, false>(din, rhs, mbits, dout, partial, cg_steps, ctl, a,
                                               s);
    if (bh > 8)
        return sweep_c32_rpw<16, false, false>(din, rhs, mbits, dout, partial, cg_steps, ctl, a,
                                               s);
    return sweep_c32_rpw<8, false, false>(din, rhs, mbits, dout, partial, cg_steps, ctl, a, s);
}

static dim3 walk_grid(int h, int w, int channels);

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

hipError_t launch_sweep_corr(const uint16_t* din, const uint16_t* rhs, const uint64_t* mbits,
                             uint16_t* dout, double* partial, double* cg_steps, const int* ctl,
                             const SweepArgs& a, hipStream_t s) {
    const int bh = a.g.bh;
    if (a.g.bw < 1 || a.g.bw > kMaxBlock || bh < 1 || bh > kMaxBlock) return hipErrorInvalidValue;
    if (bh > 32)
        return sweep_corr_rpw<64, true, true>(din, rhs, mbits, dout, partial, cg_steps, ctl, a, s);
    if (bh > 16)
        return sweep_corr_rpw<32, false, false>(din, rhs, mbits, dout, partial, cg_steps, ctl, a,
                                                s);
    if (bh > 8)
        return sweep_corr_rpw<16, false, false>(din, rhs, mbits, dout, partial, cg_steps, ctl, a,
                                                s);
    return sweep_corr_rpw<8, false, false>(din, rhs, mbits, dout, partial, cg_steps, ctl, a, s);
}

static bool order_job_ok(const OrderArgs* job) {
    // the axis tables live in the sweep's LDS; counts are 16-bit fields
    return !job || (job->order && job->keys && job->scale >= 1 &&
                    (int64_t)job->g.nby * job->g.nbx * job->channels < 65536 &&
                    job->g.nby + job->g.nbx <= kOrderMaxAxes && job->cg.sy >= 1 &&
                    job->cg.sx >= 1);
}

hipError_t launch_sweep(const float* uin, const uint64_t* mbits, float* uout,
                        double* partial, double* cg_steps, const int* ctl, const SweepArgs& a,
                        hipStream_t s, const int* fin, int* fout, const int* order,
                        const OrderArgs* job, hipEvent_t ev0, hipEvent_t ev1) {
    const int bh = a.g.bh;
    if (a.g.bw < 1 || a.g.bw > kMaxBlock || bh < 1 || bh > kMaxBlock) return hipErrorInvalidValue;
    if ((fout || order || job) && !use_split(a)) return hipErrorInvalidValue;
    if (fin && !(use_split(a) && skip_grid_ok(a.g))) return hipErrorInvalidValue;
    if (!order_job_ok(job)) return hipErrorInvalidValue;
    if (bh > 32)
        return sweep_rpw<64, true, true>(uin, mbits, uout, partial, cg_steps, ctl, a, s, fin,
                                         fout, order, job, ev0, ev1);
    if (bh > 16)
        return sweep_rpw<32, false, false>(uin, mbits, uout, partial, cg_steps, ctl, a, s, nullptr,
                                           nullptr, nullptr, nullptr, ev0, ev1);
    if (bh > 8)
        return sweep_rpw<16, false, false>(uin, mbits, uout, partial, cg_steps, ctl, a, s, nullptr,
                                           nullptr, nullptr, nullptr, ev0, ev1);
    return sweep_rpw<8, false, false>(uin, mbits, uout, partial, cg_steps, ctl, a, s, nullptr,
                                      nullptr, nullptr, nullptr, ev0, ev1);
}

bool sweep_prolong_ok(const SweepArgs& a) { return use_split(a); }

bool sweep_skip_ok(const SweepArgs& a) { return use_split(a) && skip_grid_ok(a.g); }

hipError_t launch_sweep_prolong(const ProSrc& src, const uint64_t* mbits, float* uout,
                                double* partial, double* cg_steps, const int* ctl,
                                const SweepArgs& a, hipStream_t s, int* fout,
                                const int* order, const OrderArgs* job, hipEvent_t ev0,
                                hipEvent_t ev1) {
    if (!use_split(a) || a.g.bw < 1 || a.g.bw > kMaxBlock || !src.uc || !src.f || !src.c ||
        src.hc != (a.g.h + 1) / 2 || src.wc != (a.g.w + 1) / 2 || !order_job_ok(job))
        return hipErrorInvalidValue;
    const int grid = a.g.nby * a.g.nbx * a.channels;
    const OrderArgs j = job ? *job : OrderArgs{};
    return launch_timed(k_sweep2_pro, dim3(grid + (job ? 1 : 0)), dim3(128), s, ev0, ev1, src,
                        mbits, uout, partial, cg_steps, ctl, a, fout, order, j);
}

hipError_t launch_decide(const double* partial, int nb, int channels, const double* stats,
                         int* ctl, double* rel, double tol, int n, hipStream_t s) {
    const double tol2 = tol < 0.0 ? -1.0 : tol * tol;  // negative: never passes
    switch (channels) {
#define DDI_CASE(NC)                                                                          \
    case NC:                                                                                  \
        hipLaunchKernelGGL(k_decide<NC>, dim3(1), dim3(kDecideTpb), 0, s, partial, nb, stats, \
                           ctl, rel, tol2, n);                                                \
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
                                  int ncols, double* out) {
    if (n < 1 || n > kMaxLevels || nclear < 0 || nclear > 256) return hipErrorInvalidValue;
    const bool sums = part && out && nrows > 0 && ncols > 0;
    if (sums && (stride < ncols || ncols > 65535)) return hipErrorInvalidValue;
    MaskBitsLevels L;
    L.clear = nclear > 0 ? clear : nullptr;
    L.nclear = nclear;
    L.part = part;
    L.out = out;
    L.nrows = sums ? nrows : 0;
    L.stride = stride;
    L.ncols = sums ? ncols : 0;
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
    hipLaunchKernelGGL(k_mask_bits_levels, dim3(gx, gy, n + (sums ? 1 : 0)), dim3(256), 0, s, L,
                       n);
    return hipGetLastError();
}

hipError_t launch_mask_bits(const uint8_t* c, int h, int w, uint64_t* mbits, hipStream_t s) {
    const int groups = mask_bit_groups(h);
    hipLaunchKernelGGL(k_mask_bits, dim3((w + 255) / 256, groups), dim3(256), 0, s, c, h, w,
                       groups, mbits);
    return hipGetLastError();
}

static int grid1d(int64_t n) { return (int)((n + kTpb - 1) / kTpb); }

static bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

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

static dim3 walk_grid(int h, int w, int channels) {
    return dim3(walk_groups_x(w), walk_groups_y(h), channels);
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

// ---------------------------------------------------------------------------
// batched launchers (one launch for the jobs of many images)
// ---------------------------------------------------------------------------

void sweep_instance(int bh, int* rpw, bool* ragged) {
    *rpw = bh > 32 ? 64 : bh > 16 ? 32 : bh > 8 ? 16 : 8;
    *ragged = bh != *rpw;
}

bool sweep_split(int bh) { return DDI_SPLIT && bh == 2 * kSplitRows; }

hipError_t launch_sweep_batch(const SweepJob* jobs, int njobs, int total_wg, int rpw,
                              bool ragged, hipStream_t s) {
    if (total_wg <= 0 || njobs <= 0) return hipSuccess;
    if (rpw == 64 && !ragged && DDI_SPLIT) {
        hipLaunchKernelGGL(k_sweep2_batch, dim3(total_wg), dim3(128), 0, s, jobs, njobs);
        return hipGetLastError();
    }
#define DDI_SB(R, G, Q, M)                                                                   \
    hipLaunchKernelGGL((k_sweep_batch<R, G, Q, M>), dim3(total_wg), dim3(64), 0, s, jobs, njobs)
    switch (rpw) {
        case 64: if (ragged) DDI_SB(64, true, true, true); else DDI_SB(64, false, true, true); break;
        case 32: if (ragged) DDI_SB(32, true, false, false); else DDI_SB(32, false, false, false); break;
        case 16: if (ragged) DDI_SB(16, true, false, false); else DDI_SB(16, false, false, false); break;
        case 8: if (ragged) DDI_SB(8, true, false, false); else DDI_SB(8, false, false, false); break;
        default: return hipErrorInvalidValue;
    }
#undef DDI_SB
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
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(64), 0, s, (int*)work, kGcgCtlInts);
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

hipError_t launch_refine_residual(const float* f, const uint8_t* c, const float* u,
                                  const uint16_t* d, int h, int w, int channels, float* unext,
                                  uint16_t* rhs, double* partial, const int* ctl, int* nwg,
                                  hipStream_t s) {
    const dim3 grid = walk_grid(h, w, channels);
    if (nwg) *nwg = (int)(grid.x * grid.y);
    if (d)
        hipLaunchKernelGGL(k_residual_walk<true>, grid, dim3(64 * kWalkWaves), 0, s, f, c, u, d,
                           h, w, channels, nullptr, rhs, unext, partial, ctl);
    else
        hipLaunchKernelGGL(k_residual_walk<false>, grid, dim3(64 * kWalkWaves), 0, s, f, c, u,
                           nullptr, h, w, channels, nullptr, rhs, nullptr, partial, ctl);
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
