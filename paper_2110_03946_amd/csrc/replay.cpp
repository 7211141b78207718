// Host replay of the kernels' global-memory offsets: every thread of every
// launch that a float32 ORAS plan of a given size makes (transposed-mask
// bits, coarsening, the sweeps of every level including the first sweep
// that builds its tile from the coarser level, prolongation, the
// column-walking stencil kernels), with the offsets computed by the same
// functions the kernels use (access.h), each checked against the size of the
// buffer it addresses. Host code only: nothing runs on a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "access.h"
#include "plan.h"

using namespace ddi;

namespace {

struct Replay {
    long long checked = 0, bad = 0;
    char first[512] = {0};

    // element offset `off` (and `span` consecutive elements) of buffer
    // `buf` of `size` elements
    void at(const char* kernel, const char* buf, int64_t off, int64_t size, int span = 1) {
        ++checked;
        if (off >= 0 && off + span <= size) return;
        if (bad++ == 0)
            std::snprintf(first, sizeof first, "%s: %s[%lld..%lld] outside [0, %lld)", kernel,
                          buf, (long long)off, (long long)(off + span - 1), (long long)size);
    }
    void check(const char* kernel, const char* what, bool ok) {
        ++checked;
        if (ok) return;
        if (bad++ == 0) std::snprintf(first, sizeof first, "%s: %s", kernel, what);
    }
};

// Transposed-mask bits of an h x w level.
void replay_mask_bits(Replay& R, int h, int w) {
    const int groups = mask_bit_groups(h);
    const int64_t n = (int64_t)h * w, nm = (int64_t)groups * w;
    const int gx = (w + 255) / 256;
    for (int gy = 0; gy < groups; ++gy)
        for (int bx = 0; bx < gx; ++bx)
            for (int t = 0; t < 256; ++t) {
                const int x = bx * 256 + t;
                if (x >= w) continue;
                if (gy < groups - 1)
                    for (int j = 0; j < 64; ++j)
                        R.at("k_mask_bits", "c", (int64_t)std::min(gy * 64 + j, h - 1) * w + x, n);
                R.at("k_mask_bits", "mbits", (int64_t)gy * w + x, nm);
            }
}

// Coarsening h x w -> hc x wc: both variants (the four-column one when the
// width allows it, whichever the buffers' alignment selects).
void replay_coarsen(Replay& R, int h, int w) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    const int64_t n = (int64_t)h * w, nc = (int64_t)hc * wc;
    if (w % 4 == 0) {
        int gx = 0, rows = 0;
        const int ng = coarsen4_grid(h, w, &gx, &rows);
        const int gy = ng / gx;
        R.check("k_coarsen4", "grid covers the coarse rows", (int64_t)gy * rows >= hc);
        for (int by = 0; by < gy; ++by)
            for (int bx = 0; bx < gx; ++bx)
                for (int tid = 0; tid < 256; ++tid) {
                    const int t = bx * 256 + tid;
                    if (4 * t >= w) continue;
                    for (int I = by * rows; I < std::min(hc, (by + 1) * rows); ++I) {
                        for (int a2 = 0; a2 < 2; ++a2) {
                            const int y = 2 * I + a2;
                            if (y >= h) continue;
                            R.at("k_coarsen4", "c (4 bytes)", coarsen4_in(y, w, t), n, 4);
                            R.at("k_coarsen4", "f (float4)", coarsen4_in(y, w, t), n, 4);
                        }
                        R.at("k_coarsen4", "cc (2 bytes) / fc (float2)", coarsen4_out(I, wc, t),
                             nc, 2);
                    }
                }
    }
    const int grid = init_grid(hc, wc);
    for (int b = 0; b < grid; ++b)
        for (int tid = 0; tid < 256; ++tid) {
            const int64_t idx = (int64_t)b * 256 + tid;
            if (idx >= nc) continue;
            const int I = (int)(idx / wc), J = (int)(idx - (int64_t)I * wc);
            for (int a2 = 0; a2 < 2; ++a2)
                for (int b2 = 0; b2 < 2; ++b2) {
                    const int i = 2 * I + a2, j = 2 * J + b2;
                    if (i < h && j < w) R.at("k_coarsen", "c / f", (int64_t)i * w + j, n);
                }
            R.at("k_coarsen", "cc / fc", idx, nc);
        }
}

// Two levels of coarsening in one launch (k_coarsen2x): h x w -> middle ->
// coarsest, for widths divisible by 8.
void replay_coarsen2(Replay& R, int h, int w) {
    const int hm = (h + 1) / 2, wm = w / 2, hc = (hm + 1) / 2, wc = wm / 2;
    const int64_t n = (int64_t)h * w, nm = (int64_t)hm * wm, nc = (int64_t)hc * wc;
    int gx = 0, rows = 0;
    const int ng = coarsen2_grid(h, w, &gx, &rows);
    const int gy = ng / gx;
    R.check("k_coarsen2x", "grid covers the coarsest rows", (int64_t)gy * rows >= hc);
    for (int by = 0; by < gy; ++by)
        for (int bx = 0; bx < gx; ++bx)
            for (int tid = 0; tid < 256; ++tid) {
                const int t = bx * 256 + tid;
                if (8 * t >= w) continue;
                for (int I = by * rows; I < std::min(hc, (by + 1) * rows); ++I) {
                    for (int r = 0; r < 2; ++r) {
                        const int Y = 2 * I + r;
                        if (Y >= hm) continue;
                        for (int a2 = 0; a2 < 2; ++a2) {
                            const int y = 2 * Y + a2;
                            if (y >= h) continue;
                            R.at("k_coarsen2x", "c (8 bytes)", coarsen8_in(y, w, t), n, 8);
                            R.at("k_coarsen2x", "f (2 float4)", coarsen8_in(y, w, t), n, 8);
                        }
                        R.at("k_coarsen2x", "middle c (4 bytes) / f (float4)",
                             coarsen8_mid(Y, wm, t), nm, 4);
                    }
                    R.at("k_coarsen2x", "coarsest c (2 bytes) / f (float2)", coarsen4_out(I, wc, t),
                         nc, 2);
                }
            }
}

// Prolongation hc x wc -> h x w: both variants.
void replay_prolong(Replay& R, int h, int w) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    const int64_t n = (int64_t)h * w, nc = (int64_t)hc * wc;
    if (w % 4 == 0) {
        int gx = 0;
        const int grid = prolong4_grid(h, w, &gx);
        std::vector<char> seen(grid, 0);
        for (int b = 0; b < grid; ++b) {
            const int L = xcd_band(b, grid);
            R.check("k_prolong4", "workgroup numbering in range", L >= 0 && L < grid);
            if (L < 0 || L >= grid) continue;
            R.check("k_prolong4", "workgroup numbering one to one", !seen[L]);
            seen[L] = 1;
            const int bx = L % gx, y = L / gx;
            R.check("k_prolong4", "row in the image", y < h);
            for (int tid = 0; tid < 256; ++tid) {
                const int t = bx * 256 + tid;
                if (4 * t >= w) continue;
                const Pro4Addr a = prolong4_addr(y, t, w, hc, wc);
                R.at("k_prolong4", "c (4 bytes) / f / u (float4)", a.fine, n, 4);
                R.at("k_prolong4", "uc (float2, nearer row)", a.rn + a.J0, nc, 2);
                R.at("k_prolong4", "uc (float2, farther row)", a.rf + a.J0, nc, 2);
                R.at("k_prolong4", "uc (left)", a.rn + a.jl, nc);
                R.at("k_prolong4", "uc (left)", a.rf + a.jl, nc);
                R.at("k_prolong4", "uc (right)", a.rn + a.jr, nc);
                R.at("k_prolong4", "uc (right)", a.rf + a.jr, nc);
            }
        }
    }
    const int gx = (wc + 63) / 64, gy = (hc + 3) / 4;
    for (int by = 0; by < gy; ++by)
        for (int bx = 0; bx < gx; ++bx)
            for (int tid = 0; tid < 256; ++tid) {
                const int J = bx * 64 + (tid & 63), I = by * 4 + (tid >> 6);
                if (I >= hc || J >= wc) continue;
                const int rr[3] = {std::max(I - 1, 0), I, std::min(I + 1, hc - 1)};
                const int cc[3] = {std::max(J - 1, 0), J, std::min(J + 1, wc - 1)};
                for (int a2 = 0; a2 < 3; ++a2)
                    for (int b2 = 0; b2 < 3; ++b2)
                        R.at("k_prolong", "uc", (int64_t)rr[a2] * wc + cc[b2], nc);
                for (int a2 = 0; a2 < 2; ++a2)
                    for (int b2 = 0; b2 < 2; ++b2) {
                        const int y = 2 * I + a2, x = 2 * J + b2;
                        if (y < h && x < w) R.at("k_prolong", "c / f / u", (int64_t)y * w + x, n);
                    }
            }
}

// The column-walking kernels over h x w (residual, CG, Krylov steps).
void replay_walk(Replay& R, int h, int w) {
    const int64_t n = (int64_t)h * w;
    const uint32_t W = (uint32_t)w;
    for (int by = 0; by < walk_groups_y(h); ++by)
        for (int bx = 0; bx < walk_groups_x(w); ++bx)
            for (int tid = 0; tid < 64 * kWalkWaves; ++tid) {
                const Walk k = walk_at(h, w, bx, by, tid);
                R.check("walk", "band in the image", k.y0 < h && k.y1 > k.y0);
                for (int t = 0; t < kWalkRows + 2; ++t)
                    R.at("walk", "vertical stencil row", (int64_t)walk_vrow(k, h, t) * W + k.xc, n);
                for (int t = 0; t < kWalkRows; ++t) {
                    const int64_t row = (int64_t)walk_row(k, h, t) * W;
                    R.at("walk", "band row (c, f)", row + k.xc, n);
                    if (k.edge) R.at("walk", "edge column", row + k.xe, n);
                    if (k.inb && t < k.y1 - k.y0) R.at("walk", "written row", walk_out(k, W, t), n);
                }
            }
}

// The first refinement residual built with the coarse-to-fine start, over
// an h x w level whose coarser level is ceil(h/2) x ceil(w/2): its coarse
// rows and columns, and the index rules it relies on (the coarse rows of
// each in-image fine row, and an edge lane's outside column taking the
// lane's coarse columns swapped).
void replay_start_walk(Replay& R, int h, int w) {
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    const int64_t nc = (int64_t)hc * wc;
    constexpr int NQ = kWalkRows / 2 + 2;
    for (int by = 0; by < walk_groups_y(h); ++by)
        for (int bx = 0; bx < walk_groups_x(w); ++bx)
            for (int tid = 0; tid < 64 * kWalkWaves; ++tid) {
                const Walk k = walk_at(h, w, bx, by, tid);
                const int cn = (int)k.xc >> 1, cf = pro_far((int)k.xc, wc);
                const int cb = (k.y0 >> 1) - 1;
                auto crow = [&](int i) { return std::min(std::max(cb + i, 0), hc - 1); };
                for (int i = 0; i < NQ; ++i) {
                    R.at("k_start_residual_walk", "coarse row, nearer column",
                         (int64_t)crow(i) * wc + cn, nc);
                    R.at("k_start_residual_walk", "coarse row, farther column",
                         (int64_t)crow(i) * wc + cf, nc);
                }
                for (int t = 0; t < kWalkRows + 2; ++t) {
                    const int y = k.y0 - 1 + t;
                    if (y < 0 || y >= h) continue;
                    const int ni = (t + 1) / 2, fi = (t & 1) ? ni - 1 : ni + 1;
                    R.check("k_start_residual_walk", "nearer coarse row of a fine row",
                            crow(ni) == (y >> 1));
                    R.check("k_start_residual_walk", "farther coarse row of a fine row",
                            crow(fi) == pro_far(y, hc));
                }
                const bool used = k.inb && ((k.lane == 0 && k.x > 0) || (k.lane == 63 && k.x + 1 < w));
                if (used)
                    R.check("k_start_residual_walk", "edge column: the lane's coarse columns swapped",
                            ((int)k.xe >> 1) == cf && pro_far((int)k.xe, wc) == cn);
            }
}

// Block data the sweeps index per block: partials, timing counters, flags.
void replay_block_data(Replay& R, const char* kernel, const SweepArgs& a, const Blk& k, int lb) {
    const int nb = sweep_partials(a), C = a.channels;
    R.at(kernel, "partial", (int64_t)k.b * C + k.ch, (int64_t)nb * C);
    R.at(kernel, "cg_steps (plane 1)", (int64_t)nb * C + (int64_t)k.b * C + k.ch,
         3 * (int64_t)nb * C);
    R.at(kernel, "flags out", lb, (int64_t)nb * C);
    int cell[9];
    flag_cells(k, a.g, cell);
    for (int i = 0; i < 9; ++i)
        R.at(kernel, "flags in", (int64_t)k.ch * nb + cell[i], (int64_t)nb * C);
}

// One sweep of level geometry a: the kernel the launcher picks, every block,
// every thread; with `pro` also the first sweep that builds its tile from
// the coarser level (hc x wc).
void replay_sweep(Replay& R, const SweepArgs& a, bool pro) {
    const BlockGrid& g = a.g;
    const int h = g.h, w = g.w, C = a.channels;
    const int64_t n = (int64_t)h * w;
    const int64_t nm = (int64_t)mask_bit_groups(h) * w;
    const uint32_t W = (uint32_t)w;
    const int nblk = g.nby * g.nbx * C;
    // the workgroup numbering is a permutation of the blocks
    {
        std::vector<char> seen(nblk, 0);
        for (int b = 0; b < nblk; ++b) {
            const int lb = xcd_remap(b, nblk);
            R.check("sweep", "workgroup numbering in range", lb >= 0 && lb < nblk);
            if (lb < 0 || lb >= nblk) continue;
            R.check("sweep", "workgroup numbering one to one", !seen[lb]);
            seen[lb] = 1;
        }
    }
    const bool split = sweep_prolong_ok(a);
    const int hc = (h + 1) / 2, wc = (w + 1) / 2;
    const int64_t nc = (int64_t)hc * wc;
    for (int lb = 0; lb < nblk; ++lb) {
        const Blk k = blk_geo(g, lb);
        R.check("sweep", "block inside the level",
                k.y0 >= 0 && k.x0 >= 0 && k.y0 + g.bh <= h && k.x0 + g.bw <= w && k.ch < C);
        if (split) {
            R.check("k_sweep2", "a full 64-row block", g.bh == 2 * kSplitRows);
            replay_block_data(R, "k_sweep2", a, k, lb);
            for (int wi = 0; wi < 2; ++wi)
                for (int lane = 0; lane < 64; ++lane) {
                    const uint32_t xc = tile_col(k, g, lane);
                    const bool on = lane < g.bw;
                    const int x = k.x0 + lane;
                    const Tile2Rows tr = tile2_rows(k, wi, W, xc);
                    R.at("k_sweep2", "tile row 0", tr.first, n);
                    for (int j = 1; j < kSplitRows; ++j)
                        R.at("k_sweep2", "tile rows 1..31", tr.mid0 + (int64_t)(j - 1) * W, n);
                    R.at("k_sweep2", "tile row 32", tr.last, n);
                    const int th = wi == 0 ? lane : 64 + lane;
                    const int64_t r1 = (int64_t)tile_row(k, g, std::min(th, 2 * kSplitRows + 1)) * W;
                    R.at("k_sweep2", "halo left", r1 + halo_left(k), n);
                    R.at("k_sweep2", "halo right", r1 + halo_right(k, g), n);
                    {  // every lane, idle lanes at the last column
                        const MaskWords mw = mask_words(k, W, std::min(x, w - 1));
                        R.at("k_sweep2", "mask word", mw.w0, nm);
                        R.at("k_sweep2", "second mask word", (int64_t)mw.w0 + W, nm);
                    }
                    const int ry0 = k.y0 + kSplitRows * wi;
                    if (on && x >= k.oxlo && x < k.oxhi)
                        for (int y = 0; y < kSplitRows; ++y)
                            if (ry0 + y >= k.oylo && ry0 + y < k.oyhi)
                                R.at("k_sweep2", "owned write-back",
                                     out_base(ry0, W, x) + (int64_t)y * W, n);
                    if (!pro) continue;
                    // the first sweep's tile from the coarser level
                    const ProRows P = pro_rows(k, g, wi, xc);
                    R.at("k_sweep2_pro", "halo row mask byte", P.hrow, n);  // loaded always
                    for (int j = 0; j <= kSplitRows; ++j)
                        R.at("k_sweep2_pro", "f (every row)",
                             (int64_t)pro_frow(P, j) * W + xc, n);
                    const int64_t cn = xc >> 1, cf = pro_far((int)xc, wc);
                    for (int i = 0; i < kSplitRows / 2 + 2; ++i) {
                        const int64_t row = (int64_t)pro_crow(P, i, hc) * wc;
                        R.at("k_sweep2_pro", "coarse row (nearer column)", row + cn, nc);
                        R.at("k_sweep2_pro", "coarse row (farther column)", row + cf, nc);
                    }
                    const int xl = (int)halo_left(k), xr = (int)halo_right(k, g);
                    R.at("k_sweep2_pro", "halo c / f", r1 + xl, n);
                    R.at("k_sweep2_pro", "halo c / f", r1 + xr, n);
                    const int y1 = (int)(r1 / W);
                    for (int side = 0; side < 2; ++side) {
                        const ProCell pc = pro_cell(y1, side ? xr : xl, hc, wc);
                        R.at("k_sweep2_pro", "halo coarse samples", pc.nn, nc);
                        R.at("k_sweep2_pro", "halo coarse samples", pc.nf, nc);
                        R.at("k_sweep2_pro", "halo coarse samples", pc.fn, nc);
                        R.at("k_sweep2_pro", "halo coarse samples", pc.ff, nc);
                    }
                }
            continue;
        }
        // one wave per block: RPW rows in registers (64, 32, 16 or 8 by the
        // block height, as the launcher picks), ragged when the block has
        // fewer rows
        const int rpw = g.bh > 32 ? 64 : g.bh > 16 ? 32 : g.bh > 8 ? 16 : 8;
        const bool ragged = g.bh != rpw;
        const int nrows = ragged ? g.bh : rpw;
        R.at("k_sweep", "partial", (int64_t)k.b * C + k.ch, (int64_t)sweep_partials(a) * C);
        for (int lane = 0; lane < 64; ++lane) {
            const uint32_t xc = tile_col(k, g, lane);
            const bool on = lane < g.bw;
            const int x = k.x0 + lane;
            if (!ragged) {
                const Tile2Rows tr = tile1_rows(k, rpw, W, xc);
                R.at("k_sweep", "tile row 0", tr.first, n);
                for (int t = 1; t <= rpw; ++t)
                    R.at("k_sweep", "tile rows", tr.mid0 + (int64_t)(t - 1) * W, n);
                R.at("k_sweep", "tile row RPW + 1", tr.last, n);
            } else {
                for (int t = 0; t < rpw + 2; ++t)
                    R.at("k_sweep", "tile rows (ragged)", (int64_t)tile_row(k, g, t) * W + xc, n);
            }
            const int64_t r1 = (int64_t)tile_row(k, g, lane) * W;
            R.at("k_sweep", "halo", r1 + halo_left(k), n);
            R.at("k_sweep", "halo", r1 + halo_right(k, g), n);
            if (64 + lane < rpw + 2) {
                const int64_t r2 = (int64_t)tile_row(k, g, 64 + lane) * W;
                R.at("k_sweep", "halo (second pass)", r2 + halo_left(k), n);
                R.at("k_sweep", "halo (second pass)", r2 + halo_right(k, g), n);
            }
            if (on) {
                const MaskWords mw = mask_words(k, W, x);
                R.at("k_sweep", "mask word", mw.w0, nm);
                R.at("k_sweep", "second mask word", (int64_t)mw.w0 + W, nm);
            }
            if (on && x >= k.oxlo && x < k.oxhi)
                for (int y = 0; y < rpw; ++y)
                    if (y < nrows && k.y0 + y >= k.oylo && k.y0 + y < k.oyhi)
                        R.at("k_sweep", "owned write-back", out_base(k.y0, W, x) + (int64_t)y * W,
                             n);
        }
    }
}

}  // namespace

extern "C" int ddi_selfcheck_access(int height, int width, int channels, const ddi_params* p,
                                    long long* checked, long long* violations, char* first,
                                    int first_len) {
    ddi_params prm;
    if (p)
        prm = *p;
    else
        ddi_default_params(&prm);
    const int e = ddi_check_params(height, width, channels, &prm);
    if (e) return e;
    Replay R;
    const int L = level_count(height, width, prm.levels);
    int h = height, w = width;
    for (int l = 0; l < L; ++l) {
        replay_mask_bits(R, h, w);
        const SweepArgs a = level_sweep(height, width, channels, prm, l);
        R.check("level", "sweep geometry of the level", a.g.h == h && a.g.w == w);
        // a level below the coarsest starts from the coarser one: its first
        // sweep may build the tile from it
        replay_sweep(R, a, l + 1 < L && sweep_prolong_ok(a));
        replay_walk(R, h, w);
        if (l == 0 && L > 1) replay_start_walk(R, h, w);
        if (l + 1 < L) {
            replay_coarsen(R, h, w);
            replay_prolong(R, h, w);
        }
        if (l >= 1 && l + 2 < L && w % 8 == 0) replay_coarsen2(R, h, w);
        h = (h + 1) / 2;
        w = (w + 1) / 2;
    }
    if (checked) *checked = R.checked;
    if (violations) *violations = R.bad;
    if (first && first_len > 0) {
        std::strncpy(first, R.first, (size_t)first_len - 1);
        first[first_len - 1] = 0;
    }
    return DDI_OK;
}
