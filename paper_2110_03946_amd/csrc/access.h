// Index arithmetic of the kernels' global-memory accesses: the element
// offsets a thread of a launch reads and writes, as functions of the launch
// geometry and the thread's position. The kernels take their offsets from
// these functions, and the host replay (replay.cpp, ddi_selfcheck_access)
// runs the same functions over every thread of every launch a plan makes and
// checks each offset against the buffer it addresses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

#define DDI_HD __host__ __device__ __forceinline__

namespace ddi {

// ---------------------------------------------------------------------------
// Workgroup numbering over the XCDs
// ---------------------------------------------------------------------------

// Workgroups are handed to the 8 XCDs of the chip round-robin (workgroup i
// runs on XCD i mod 8). Renumber them so that each XCD works through runs
// of kXcdChunk consecutive blocks of the logical order (XCD j takes runs j,
// j + 8, j + 16, ...): horizontal neighbours, which share halo and overlap
// cache lines, meet in the same L2, while costly regions of the image are
// still spread over all XCDs. A tail shorter than 8 runs keeps its order.
constexpr int kXcds = 8;
constexpr int kXcdChunk = 16;

// Workgroup b of n -> logical index: XCD j (= b mod 8) takes one
// contiguous band of the logical order, so that row-streaming kernels whose
// neighbouring rows share reads (prolongation: four fine rows read each
// coarse row) fetch them into one L2 only. A tail shorter than 8 keeps its
// order.
DDI_HD int xcd_band(int b, int n) {
    const int full = n - n % kXcds;
    if (b >= full) return b;
    return (b % kXcds) * (full / kXcds) + b / kXcds;
}

DDI_HD int xcd_remap(int b, int n) {
    const int full = n - n % (kXcds * kXcdChunk);
    if (b >= full) return b;
    const int j = b % kXcds, i = b / kXcds;
    return (j + kXcds * (i / kXcdChunk)) * kXcdChunk + i % kXcdChunk;
}

// ---------------------------------------------------------------------------
// Sweeps: a block's tile, mask words, owned write-back, neighbour flags
// ---------------------------------------------------------------------------

// Rows per wave of a full 64-row block swept by two waves.
constexpr int kSplitRows = 32;

// Geometry of one block of the grid (logical index lb, channel-major).
struct Blk {
    int ch, b, y0, x0, oylo, oyhi, oxlo, oxhi;
    bool has_top, has_bot, has_left, has_right;
};

DDI_HD Blk blk_geo(const BlockGrid& g, int lb) {
    Blk k;
    const int nblk = g.nby * g.nbx;
    k.ch = lb / nblk;
    k.b = lb - k.ch * nblk;
    const int by = k.b / g.nbx;
    const int bx = k.b - by * g.nbx;
    k.y0 = block_origin(by, g.sy, g.h, g.bh);
    k.x0 = block_origin(bx, g.sx, g.w, g.bw);
    owner_range(by, g.nby, g.sy, g.h, g.bh, &k.oylo, &k.oyhi);
    owner_range(bx, g.nbx, g.sx, g.w, g.bw, &k.oxlo, &k.oxhi);
    k.has_top = k.y0 > 0;
    k.has_bot = k.y0 + g.bh < g.h;
    k.has_left = k.x0 > 0;
    k.has_right = k.x0 + g.bw < g.w;
    return k;
}

// Column that lane `lane` loads: its block column, or the block's first
// column for lanes right of the block (their values are not used).
DDI_HD uint32_t tile_col(const Blk& k, const BlockGrid& g, int lane) {
    return (uint32_t)(lane < g.bw ? k.x0 + lane : k.x0);
}

// Image row of tile row t (tile row t = image row y0 - 1 + t), clamped to
// the image: a clamped row repeats the border row (reflecting boundary).
DDI_HD uint32_t tile_row(const Blk& k, const BlockGrid& g, int t) {
    return (uint32_t)min(max(k.y0 - 1 + t, 0), g.h - 1);
}

// Wave wi of a two-wave block loads tile rows 33 wi .. 33 wi + 32 of its
// column xc: the first and last of them may lie outside the image (then
// they are the border row), rows 1 .. 31 are mid0 + (j - 1) W.
struct Tile2Rows {
    uint32_t first, mid0, last;
};
DDI_HD Tile2Rows tile2_rows(const Blk& k, int wi, uint32_t W, uint32_t xc) {
    const int t0 = wi * (kSplitRows + 1);
    const int yfirst = (wi == 0 && !k.has_top) ? k.y0 : k.y0 - 1 + t0;
    const int ylast =
        (wi == 1 && !k.has_bot) ? k.y0 + 2 * kSplitRows - 1 : k.y0 - 1 + t0 + kSplitRows;
    Tile2Rows r;
    r.first = (uint32_t)yfirst * W + xc;
    r.mid0 = (uint32_t)(k.y0 + t0) * W + xc;
    r.last = (uint32_t)ylast * W + xc;
    return r;
}

// A one-wave block of RPW full rows (rows y0 .. y0 + RPW - 1 in the image):
// tile row 0 at `first`, rows 1 .. RPW at mid0 + (t - 1) W, row RPW + 1 at
// `last`.
DDI_HD Tile2Rows tile1_rows(const Blk& k, int rpw, uint32_t W, uint32_t xc) {
    const uint32_t off = (uint32_t)k.y0 * W + xc;
    Tile2Rows r;
    r.first = k.has_top ? off - W : off;
    r.mid0 = off;
    const uint32_t lastmid = off + (uint32_t)(rpw - 1) * W;
    r.last = k.has_bot ? lastmid + W : lastmid;
    return r;
}

// The halo columns left and right of the block (clamped to the image).
DDI_HD uint32_t halo_left(const Blk& k) { return (uint32_t)max(k.x0 - 1, 0); }
DDI_HD uint32_t halo_right(const Blk& k, const BlockGrid& g) {
    return (uint32_t)min(k.x0 + g.bw, g.w - 1);
}

// The block's unknown-pixel bits of column x (transposed mask, 64 rows per
// word): they start at bit sh = y0 % 64 of word w0 = (y0 / 64) W + x and,
// with sh != 0, continue in word w0 + W.
struct MaskWords {
    uint32_t w0;
    int sh;
};
DDI_HD MaskWords mask_words(const Blk& k, uint32_t W, int x) {
    MaskWords m;
    m.w0 = (uint32_t)(k.y0 >> 6) * W + (uint32_t)x;
    m.sh = k.y0 & 63;
    return m;
}

// Owned write-back of column x over rows row0 .. row0 + nrows - 1: element
// offset of row row0; a row y is written when row0 + y lies in [oylo, oyhi)
// and the column in [oxlo, oxhi).
DDI_HD uint32_t out_base(int row0, uint32_t W, int x) { return (uint32_t)row0 * W + (uint32_t)x; }

// Flags of the block and its 8 neighbours (clamped at the grid border),
// indices into the channel's nby x nbx flags: [0] the block, [1..8] the
// neighbours.
DDI_HD void flag_cells(const Blk& k, const BlockGrid& g, int* cells) {
    const int nbx = g.nbx, nby = g.nby;
    const int by = k.b / nbx, bx = k.b - by * nbx;
    const int r0 = max(by - 1, 0) * nbx, r1 = by * nbx, r2 = min(by + 1, nby - 1) * nbx;
    const int c0 = max(bx - 1, 0), c2 = min(bx + 1, nbx - 1);
    cells[0] = r1 + bx;
    cells[1] = r0 + c0;
    cells[2] = r0 + bx;
    cells[3] = r0 + c2;
    cells[4] = r1 + c0;
    cells[5] = r1 + c2;
    cells[6] = r2 + c0;
    cells[7] = r2 + bx;
    cells[8] = r2 + c2;
}

// ---------------------------------------------------------------------------
// Bilinear prolongation (Sec. 4): coarse samples of a fine pixel
// ---------------------------------------------------------------------------

// The farther coarse sample of fine index y on an axis of nc samples (the
// nearer one is y >> 1).
DDI_HD int pro_far(int y, int nc) {
    return (y & 1) ? min((y >> 1) + 1, nc - 1) : max((y >> 1) - 1, 0);
}

// Element offsets of the four coarse samples of fine pixel (y, x):
// (nearer row, nearer column), (nearer, farther), (farther, nearer),
// (farther, farther).
struct ProCell {
    uint32_t nn, nf, fn, ff;
};
DDI_HD ProCell pro_cell(int y, int x, int hc, int wc) {
    const uint32_t rn = (uint32_t)(y >> 1) * (uint32_t)wc;
    const uint32_t rf = (uint32_t)pro_far(y, hc) * (uint32_t)wc;
    const uint32_t cn = (uint32_t)(x >> 1), cf = (uint32_t)pro_far(x, wc);
    ProCell p;
    p.nn = rn + cn;
    p.nf = rn + cf;
    p.fn = rf + cn;
    p.ff = rf + cf;
    return p;
}

// A two-wave block's first sweep builds wave wi's 33 tile rows from the
// coarser level: fine rows ybase .. ybase + 32, coarse rows F0 .. F0 +
// kSplitRows / 2 + 1 (clamped), f of the known rows, and the mask byte of
// the halo row (above the block for wave 0, below it for wave 1).
struct ProRows {
    int ybase, F0, hmax;
    uint32_t hrow;  // element offset of the halo row's mask byte in column xc
    bool hin;       // that row lies in the image
};
DDI_HD ProRows pro_rows(const Blk& k, const BlockGrid& g, int wi, uint32_t xc) {
    ProRows P;
    P.ybase = k.y0 - 1 + wi * (kSplitRows + 1);
    P.F0 = (P.ybase - 1) >> 1;
    P.hmax = g.h - 1;
    const int yh = wi == 0 ? k.y0 - 1 : k.y0 + 2 * kSplitRows;
    P.hin = wi == 0 ? k.has_top : k.has_bot;
    P.hrow = (uint32_t)min(max(yh, 0), g.h - 1) * (uint32_t)g.w + xc;
    return P;
}
// Fine row of wave row j (0 .. kSplitRows) whose f a known lane reads.
DDI_HD int pro_frow(const ProRows& P, int j) {
    return (j == 0 || j == kSplitRows) ? min(max(P.ybase + j, 0), P.hmax) : P.ybase + j;
}
// Coarse row i (0 .. kSplitRows / 2 + 1) of the wave, clamped.
DDI_HD int pro_crow(const ProRows& P, int i, int hc) { return min(max(P.F0 + i, 0), hc - 1); }

// ---------------------------------------------------------------------------
// Column-walking stencil kernels
// ---------------------------------------------------------------------------

// A workgroup is kWalkWaves waves side by side, each covering 64
// consecutive columns of a band of kWalkRows rows.
constexpr int kWalkRows = 8;
constexpr int kWalkWaves = 4;

// Launch grid of a walk over h x w: workgroup columns and row bands.
DDI_HD int walk_groups_x(int w) { return (w + 64 * kWalkWaves - 1) / (64 * kWalkWaves); }
DDI_HD int walk_groups_y(int h) { return (h + kWalkRows - 1) / kWalkRows; }

struct Walk {
    int lane, x, y0, y1;
    uint32_t xc, xe;  // clamped column, and the edge column lanes 0 / 63 read
    bool inb, edge;
};

DDI_HD Walk walk_at(int h, int w, int bx, int by, int tid) {
    Walk k;
    k.lane = tid & 63;
    const int wv = tid >> 6;
    k.x = (bx * kWalkWaves + wv) * 64 + k.lane;
    k.inb = k.x < w;
    k.xc = k.inb ? k.x : w - 1;
    k.edge = k.lane == 0 || k.lane == 63;
    // from the clamped column, so that lane 0 of a wave lying wholly right of
    // the image still reads inside the row (its values are not used)
    k.xe = k.lane == 0 ? (uint32_t)max((int)k.xc - 1, 0) : (uint32_t)min(k.x + 1, w - 1);
    k.y0 = by * kWalkRows;
    k.y1 = min(k.y0 + kWalkRows, h);
    return k;
}

// Rows of a walk: the vertical stencil's row t (0 .. kWalkRows + 1, image
// row y0 - 1 + t, clamped) and the band's row t (0 .. kWalkRows - 1, image
// row y0 + t, clamped below).
DDI_HD uint32_t walk_vrow(const Walk& k, int h, int t) {
    return (uint32_t)min(max(k.y0 - 1 + t, 0), h - 1);
}
DDI_HD uint32_t walk_row(const Walk& k, int h, int t) { return (uint32_t)min(k.y0 + t, h - 1); }
// Element offset of the band's row t (t < y1 - y0) in the lane's column:
// where a walk writes.
DDI_HD uint32_t walk_out(const Walk& k, uint32_t W, int t) {
    return (uint32_t)(k.y0 + t) * W + k.xc;
}

// ---------------------------------------------------------------------------
// Level transfer
// ---------------------------------------------------------------------------

// k_coarsen4: thread t of a row makes coarse columns 2t, 2t + 1 from fine
// columns 4t .. 4t + 3 (one 4-byte mask load, one float4 per channel and
// fine row) and writes them as one 2-byte mask and one float2 per channel.
DDI_HD int64_t coarsen4_in(int y, int w, int t) { return (int64_t)y * w + 4 * t; }
DDI_HD int64_t coarsen4_out(int I, int wc, int t) { return (int64_t)I * wc + 2 * t; }

// k_coarsen2x (two levels in one launch): thread t reads columns 8t .. 8t + 7
// of the finer level's rows, writes columns 4t .. 4t + 3 of the middle
// level's rows and columns 2t, 2t + 1 of the coarsest (coarsen4_out).
DDI_HD int64_t coarsen8_in(int y, int w, int t) { return (int64_t)y * w + 8 * t; }
DDI_HD int64_t coarsen8_mid(int Y, int wm, int t) { return (int64_t)Y * wm + 4 * t; }

// k_prolong4: thread t of fine row y writes fine columns 4t .. 4t + 3 (one
// float4 per channel) from coarse columns 2t - 1 .. 2t + 2 (clamped; 2t and
// 2t + 1 as one float2) of the nearer and the farther coarse row.
struct Pro4Addr {
    int64_t fine;            // fine element offset of column 4t
    uint32_t rn, rf;         // element offsets of the two coarse rows
    int J0, jl, jr;          // coarse columns: the pair J0, J0 + 1 and the clamped ends
};
DDI_HD Pro4Addr prolong4_addr(int y, int t, int w, int hc, int wc) {
    Pro4Addr a;
    a.fine = (int64_t)y * w + 4 * t;
    a.rn = (uint32_t)(y >> 1) * (uint32_t)wc;
    a.rf = (uint32_t)pro_far(y, hc) * (uint32_t)wc;
    a.J0 = 2 * t;
    a.jl = max(a.J0 - 1, 0);
    a.jr = min(a.J0 + 2, wc - 1);
    return a;
}

}  // namespace ddi
