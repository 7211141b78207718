// ORAS sweep kernels for gfx950 (wave64) and their launchers.
//
//   k_sweep2       one ORAS iteration (Sec. 3, eqs. 7-9) over full 64 x 64
//                  blocks, two waves per block: block residual, k-step local
//                  CG with the Robin interface weight, owned write-back.
//   k_sweep2_pro   the same with the tile formed from the coarser level by
//                  the bilinear prolongation (Sec. 4): a level's first sweep.
//   k_sweep        one wave64 per (block, channel), for the other block
//                  heights.
//   k_sweep_corr, k_sweep_c32, k_sweep2_c32
//                  sweeps of a correction equation (bfloat16 or float32).
//   k_sweep_batch, k_sweep2_batch
//                  one sweep over the blocks of many images.
// A sweep launch may carry one extra workgroup that sorts the blocks of the
// next sweep into its dispatch order (longest local solves first).
#include "device.h"

namespace ddi {
namespace {

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

// The two mask words holding a block column's 64 unknown-pixel bits, and
// the bits themselves (bit y <-> row y0 + y). Both words are always loaded
// (the transposed mask has one all-zero group row past the last, so the
// second exists) and combined without a branch: the loads issue together
// with the tile's, and the bits cost no extra memory round trip whatever
// y0 % 64 is.
struct BlockWords {
    uint64_t lo, hi;
    int sh;
};
__device__ __forceinline__ BlockWords block_words(const uint64_t* __restrict__ mbits,
                                                  const MaskWords& mw, uint32_t W) {
    return {mbits[mw.w0], mbits[mw.w0 + W], mw.sh};
}
__device__ __forceinline__ uint64_t block_bits(const BlockWords& b) {
    // (hi << 1) << (63 - sh): hi << (64 - sh) without the undefined shift by 64
    return (b.lo >> b.sh) | ((b.hi << 1) << (63 - b.sh));
}

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
        uint64_t bits = block_bits(block_words(mbits, mask_words(kb, (uint32_t)g.w, x), (uint32_t)g.w));
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
// Word 3 of a raw buffer resource on gfx950 (32-bit data, no swizzle).
constexpr int kBufferDword3 = 0x00020000;
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
    // the mask words first, combined after the tile loads are issued (idle
    // lanes read the last column's words and drop them)
    const BlockWords bw = block_words(mbits, mask_words(k, Wd, min(x, g.w - 1)), Wd);
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
    const uint64_t bits = on ? block_bits(bw) : 0ull;
    T.mlo = (uint32_t)bits;
    T.mhi = (uint32_t)(bits >> 32);
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
// are shared by the fine rows. Row j of a lane takes f where that pixel is
// known: the block's mask bits bw, and the mask byte hbyte for the halo row
// (above the block for wave 0, below for wave 1). Every load is a uniform
// row base plus the lane's column. f is loaded in every row, known or not:
// nearly every 128-byte line of f holds a known pixel at 4 % density, and
// the loads then go out with the coarse ones, before the mask words are
// waited for. Image rows outside the image (tile rows 0 and 65 at the
// border) are computed clamped and then replaced by their reflection.
template <int Q>
__device__ __forceinline__ void tile2_prolong_rows(Tile2& T, const ProSrc& S,
                                                   const float* __restrict__ Uc,
                                                   const float* __restrict__ F,
                                                   const ProRows& P, uint32_t xc, uint32_t Wd,
                                                   const BlockWords& bw, uint32_t hbyte, bool on,
                                                   int wi) {
    constexpr int RPW = kSplitRows;
    constexpr int NQ = RPW / 2 + 2;
    const int hmax = P.hmax;
    // Buffer loads: the row offset is a scalar operand and the lane's column
    // the vector offset, so a row costs no vector instruction.
    const uint32_t fbytes = Wd * (uint32_t)(hmax + 1) * 4u;
    const __amdgpu_buffer_rsrc_t rf =
        __builtin_amdgcn_make_buffer_rsrc((void*)F, (short)0, (int)fbytes, kBufferDword3);
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Uc, (short)0, (int)((uint32_t)S.hc * (uint32_t)S.wc * 4u), kBufferDword3);
    const uint32_t xb = xc * 4u, cnb = (xc >> 1) * 4u, cfb = (uint32_t)pro_far((int)xc, S.wc) * 4u;
    // all loads first: f, then the coarse pairs
    float fv[RPW + 1];
    int sel[RPW + 1];
#pragma unroll
    for (int j = 0; j < RPW + 1; ++j) {
        const int y = pro_frow(P, j);
        fv[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                              rf, (int)xb, (int)((uint32_t)y * Wd * 4u), 0));
    }
    float qn[NQ], qf[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int so = (int)((uint32_t)pro_crow(P, i, S.hc) * (uint32_t)S.wc * 4u);
        qn[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)cnb, so, 0));
        qf[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)cfb, so, 0));
    }
    // the mask words and the halo byte are consumed only after every load
    // of the tile is issued
    const uint64_t bits = on ? block_bits(bw) : 0ull;
    T.mlo = (uint32_t)bits;
    T.mhi = (uint32_t)(bits >> 32);
    const uint32_t hknown = (P.hin & (hbyte != 0)) ? 1u : 0u;
    uint32_t klo, khi;
    if (wi == 0) {
        klo = (~T.mlo << 1) | hknown;
        khi = (~T.mlo) >> 31;
    } else {
        klo = ~T.mhi;
        khi = hknown;
    }
#pragma unroll
    for (int j = 0; j < RPW + 1; ++j)
        sel[j] = j < 32 ? __builtin_amdgcn_sbfe((int)klo, j, 1)
                        : __builtin_amdgcn_sbfe((int)khi, j - 32, 1);
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
    const BlockWords bw = block_words(mbits, mask_words(k, Wd, min(x, g.w - 1)), Wd);
    // known pixels of this wave's 33 rows: the block's bits, and the mask
    // byte for the halo row (above the block for wave 0, below for wave 1)
    const ProRows P = pro_rows(k, g, wi, xc);
    const uint32_t hbyte = at32(S.c, P.hrow);  // clamped: always in the plane
    if ((P.ybase - 1) & 1)
        tile2_prolong_rows<1>(T, S, Uc, F, P, xc, Wd, bw, hbyte, on, wi);
    else
        tile2_prolong_rows<0>(T, S, Uc, F, P, xc, Wd, bw, hbyte, on, wi);
    // reflecting border: the clamped tile row repeats its neighbour
    if (wi == 0 && !k.has_top) T.col[0] = T.col[1];
    if (wi == 1 && !k.has_bot) T.col[RPW] = T.col[RPW - 1];
    // halo columns: one pixel each per lane th (tile row th)
    const int xl = (int)halo_left(k), xr = (int)halo_right(k, g);
    const int th = wi == 0 ? lane : 64 + lane;
    const int r1 = (int)tile_row(k, g, min(th, 2 * RPW + 1));
    const uint32_t ro = (uint32_t)r1 * Wd;
    const bool kl = at32(S.c, ro + xl) != 0, kr = at32(S.c, ro + xr) != 0;
    const float fl = at32(F, ro + xl);
    const float fr = at32(F, ro + xr);
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
    int used = g.nby + g.nbx;
    int* sk = sh + used;
    if (nk <= cap - used) {
        for (int i = tid; i < nk; i += NT) sk[i] = A.keys[i];
        K = sk;
        used += nk;
    }
    // the count pass leaves each block's bucket here for the write pass
    // (one byte per block, where the LDS holds them)
    uint8_t* bks = n <= 4 * (cap - used) ? reinterpret_cast<uint8_t*>(sh + used) : nullptr;
    __syncthreads();
    const int per = (n + NT - 1) / NT;
    const int lo = min(tid * per, n), hi = min(lo + per, n);
    const int ch0 = lo / nblk, by0 = (lo - ch0 * nblk) / g.nbx, bx0 = lo - ch0 * nblk - by0 * g.nbx;
    auto bucket = [&](int ch, int by, int bx) {
        return order_bucket_of(K[(ch * c.nby + cby_of[by]) * c.nbx + cbx_of[bx]]);
    };
    // the bucket lookups of consecutive blocks are independent: unrolled,
    // their LDS latencies overlap
    uint64_t c03 = 0, c47 = 0;
    {
        int ch = ch0, by = by0, bx = bx0;
#pragma unroll 4
        for (int i = lo; i < hi; ++i) {
            const int bk = bucket(ch, by, bx);
            if (bks) bks[i] = (uint8_t)bk;
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
#pragma unroll 4
    for (int i = lo; i < hi; ++i) {
        const int bk = bks ? (int)bks[i] : bucket(ch, by, bx);
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

}  // namespace

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

}  // namespace ddi
