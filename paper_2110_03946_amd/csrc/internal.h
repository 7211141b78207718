// Internal declarations shared by the kernels (sweep.hip, levels.hip,
// outer.hip, coarse.hip) and the solver driver / C ABI (api.cpp, batch.cpp,
// mlcg.cpp, krylov.cpp). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddi {

// Overlapping block grid of one resolution level (Sec. 4: a block spans
// `size` pixels including the overlap, neighbours share `overlap` pixels,
// the last block is shifted back to end at the image border).
struct BlockGrid {
    int h, w;       // level size in pixels
    int bh, bw;     // block height / width after clamping to the image
    int sy, sx;     // strides: bh - overlap_y, bw - overlap_x (>= 1)
    int nby, nbx;   // number of blocks per axis
};

// Arguments of one ORAS sweep (Sec. 3, eqs. 7-9) over all channels.
struct SweepArgs {
    BlockGrid g;
    int channels;
    int64_t cpitch;   // elements between channel planes (= h * w)
    float alpha;      // Robin interface weight, 1 = RAS
    int k;            // local CG steps
    float local_tol2; // stop CG once r.r <= local_tol2 * block pixels (0: k steps)
};

// The coarse level a first sweep prolongs from (the bilinear prolongation
// of Sec. 4 fused into the tile load): the coarse iterate (hc x wc per
// channel) and the fine level's data and mask, the known pixels taking f.
// Largest restart length of the Krylov method (method = 2).
constexpr int kKryMaxM = 16;

// Per-channel state of a Krylov cycle (device memory): the rotated
// Hessenberg matrix R (column j at R[j * (kKryMaxM + 1)]), the Givens
// rotations, the right-hand side g of the least-squares problem and its
// solution y, ||b||^2, and the steps taken in the cycle.
struct KryState {
    double R[kKryMaxM * (kKryMaxM + 1)];
    double cs[kKryMaxM], sn[kKryMaxM];
    double g[kKryMaxM + 1];
    double y[kKryMaxM];
    double bnorm2;
    int steps, pad;
};

struct ProSrc {
    const float* uc;
    int hc, wc;
    const float* f;
    const uint8_t* c;
};

__host__ __device__ inline int block_origin(int k, int stride, int n, int size) {
    int o = k * stride;
    return o < n - size ? o : n - size;
}

// Pixels [lo, hi) along one axis owned by block k (Boolean partition of
// unity, eq. 10): the overlap with each neighbour is split in the middle,
// the lower half (rounded up) going to the lower block.
__host__ __device__ inline void owner_range(int k, int nb, int stride, int n,
                                            int size, int* lo, int* hi) {
    int o = block_origin(k, stride, n, size);
    if (k == 0) {
        *lo = 0;
    } else {
        int op = block_origin(k - 1, stride, n, size);
        *lo = o + (op + size - o + 1) / 2;
    }
    if (k == nb - 1) {
        *hi = n;
    } else {
        int on = block_origin(k + 1, stride, n, size);
        *hi = on + (o + size - on + 1) / 2;
    }
}

// Number of blocks of length `size` with overlap `ov` covering n pixels.
__host__ __device__ inline int block_count(int n, int size, int ov) {
    if (size >= n) return 1;
    int stride = size - ov;
    return (n - ov + stride - 1) / stride;
}

// One image's part of a batched sweep launch: its workgroups are the
// logical range [wg0, wg0 + blocks * channels).
struct SweepJob {
    const float* uin;
    const uint64_t* mbits;
    float* uout;
    double* partial;
    double* cg_steps;
    const int* ctl;
    SweepArgs a;
    int wg0;
    ProSrc pro;  // pro.uc set: the input is the prolongation of pro (uin unused;
                 // only for jobs with sweep_prolong_ok)
    const int* fin;  // unchanged-block flags of the previous sweep (or null)
    int* fout;       // this sweep's flags (or null); as in launch_sweep
};

// One image at one level for the batched level kernels (coarsening,
// prolongation, initial guess, transposed masks). Unused fields are null.
struct LevelJob {
    const float* f;       // level data (the finer level for coarsening/prolongation)
    const uint8_t* c;
    float* fo;            // coarsening output
    uint8_t* co;
    const float* uc;      // prolongation input (coarse iterate)
    float* u;             // prolongation / initial-guess output
    uint64_t* mbits;      // transposed-mask output
    double* stats;        // coarsening statistics partials (or null)
    int h, w, hc, wc;     // fine and coarse sizes
    int gx, rows;         // workgroup columns, coarse rows per workgroup
    int wg0;              // first workgroup of the job in the launch
};

// Largest level (pixels) the float64 coarsest-level solve takes: one
// workgroup holds the level's search direction in LDS.
constexpr int kCoarseMaxPixels = 8192;

// One image's float64 coarsest-level solve in a batched launch.
struct CoarseJob {
    const float* f;
    const uint8_t* c;
    float* u;
    int h, w, max_iter;
    double tol2;  // squared relative tolerance
};

// One image's stop test in a batched k_decide launch.
struct DecideJob {
    const double* partial;
    const double* stats;
    int* ctl;
    double* rel;
    double tol2;  // squared tolerance, < 0: never passes
    int nb;       // sweep partial rows (blocks)
    int min_n;    // the image's min_sweeps: an earlier test never passes
};

// One image's column sums in a batched reduction.
struct ReduceJob {
    const double* partial;
    double* out;
    int nrows, stride;
};

// ---- launchers (the .hip kernel files); all asynchronous on `s` ----

// Largest block edge the sweep kernel holds on chip (one wave64 per block:
// lanes are columns, rows live in registers).
constexpr int kMaxBlock = 64;

// Dispatch-table job of a sweep launch (order_run): sort the blocks of grid
// g (channels x g.nby x g.nbx, channel-major) by the CG steps `keys` of the
// blocks of a coarser grid cg (scale = fine / coarse pixel size) over their
// centres, most first, stably, into order[]. A sweep launch that carries a
// job runs it in one extra workgroup beside its blocks.
constexpr int kOrderMaxAxes = 2048;  // g.nby + g.nbx of a dispatch-table job
struct OrderArgs {
    const int* keys = nullptr;
    int* order = nullptr;
    BlockGrid g{}, cg{};
    int channels = 0, scale = 0;
};

// One ORAS sweep u_in -> u_out. `mbits` is the column-transposed mask of
// launch_mask_bits for the same level. When cg_steps is non-null, block b
// of channel ch adds the number of CG steps it ran to cg_steps[b * C + ch].
// When ctl is non-null and ctl[0] != 0 the sweep does nothing.
// Block keys (only where sweep_prolong_ok, i.e. 64-row blocks): fout (may
// be null) receives per block (index ch * blocks + b) the CG steps the block
// ran; 0 means the sweep left its owned pixels unchanged. fin (may be null;
// only where sweep_skip_ok) holds the keys of the previous sweep on the
// same level, whose input was u_out and whose output is u_in: a block that
// this sweep would leave unchanged and that the previous sweep left
// unchanged skips its write-back (u_out holds the values already), and a
// block whose 3 x 3 neighbourhood the previous sweep left unchanged is
// skipped whole (its partial keeps the previous value, which is its residual
// norm again). The result is bit for bit that of the sweep without keys.
// order (may be null; 64-row blocks): a dispatch table (OrderArgs) built
// before this launch; workgroup i runs block order[i]. job (may be null;
// 64-row blocks, a table of < 2^16 blocks): a dispatch table for a later
// sweep, built by this launch. With cg_steps, planes 1 and 2 of cg_steps
// (offsets blocks * C and 2 * blocks * C) count the blocks skipped whole and
// those whose write-back was skipped.
// ev0, ev1 (both or neither): timing events recorded by the launch itself
// at the kernel's start and end.
hipError_t launch_sweep(const float* uin, const uint64_t* mbits, float* uout,
                        double* partial, double* cg_steps, const int* ctl, const SweepArgs& a,
                        hipStream_t s, const int* fin = nullptr, int* fout = nullptr,
                        const int* order = nullptr, const OrderArgs* job = nullptr,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// True when a sweep of `a` can use unchanged-block keys: full 64-row
// blocks, each tile inside the owned pixels of its block and its 8
// neighbours.
bool sweep_skip_ok(const SweepArgs& a);

// True when the sweep of `a` can take its input from a coarser level
// (launch_sweep_prolong): full 64-row blocks.
bool sweep_prolong_ok(const SweepArgs& a);

// One ORAS sweep whose input iterate is the bilinear prolongation of
// src.uc (known pixels: src.f), computed while the tiles are loaded, so the
// prolonged iterate is never stored; otherwise as launch_sweep. Bit for bit
// the sweep of launch_prolong's output whenever the interpolation sums are
// exact in float64 (coarse values within a factor 2^26 of their neighbours).
hipError_t launch_sweep_prolong(const ProSrc& src, const uint64_t* mbits, float* uout,
                                double* partial, double* cg_steps, const int* ctl,
                                const SweepArgs& a, hipStream_t s, int* fout = nullptr,
                                const int* order = nullptr, const OrderArgs* job = nullptr,
                                hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Device stop test after finest-level sweep n (see k_decide): reduces the
// sweep's partials, stores max_k ||r_k||^2/||b_k||^2 in rel[0] and, when
// the test passes or the input statistics are invalid (ctl[2] = 1 bad mask
// byte, 2 empty mask), sets ctl[0] and records n in ctl[1]. mirror (may be
// null): device-visible host memory that receives ctl[0 .. 4) and then the
// 8 bytes of rel[0] at the end, whatever the outcome.
hipError_t launch_decide(const double* partial, int nb, int channels, const double* stats,
                         int* ctl, double* rel, double tol, int n, hipStream_t s,
                         int* mirror = nullptr);

// p[0..n) = 0 for ints.
hipError_t launch_clear_int(int* p, int n, hipStream_t s);

// Row groups of the transposed mask: ceil(h / 64) plus one zero group.
__host__ __device__ inline int mask_bit_groups(int h) { return (h + 63) / 64 + 1; }

// mbits[g * w + x], bit j = pixel (64 g + j, x) is unknown.
hipError_t launch_mask_bits(const uint8_t* c, int h, int w, uint64_t* mbits, hipStream_t s);

// Largest number of levels a plan holds.
constexpr int kMaxLevels = 16;

// The initial guess u = c ? f : 0 of one level (n pixels, channel planes
// n apart).
struct InitJob {
    const float* f;
    const uint8_t* c;
    float* u;
    int64_t n;
    int channels;
};
hipError_t launch_mask_bits_levels(int n, const uint8_t* const* c, const int* h, const int* w,
                                   uint64_t* const* mbits, hipStream_t s,
                                   int* clear = nullptr, int nclear = 0,
                                   const double* part = nullptr, int nrows = 0, int stride = 0,
                                   int ncols = 0, double* out = nullptr,
                                   const InitJob* init = nullptr);
// (above) The transposed masks of n levels in one launch; optionally also
// zeroes clear[0 .. nclear) (nclear <= 256), e.g. a solve's control word,
// writes the column sums out[j] = sum_i part[i * stride + j] for j < ncols
// bit for bit as launch_reduce does (e.g. the input statistics), and makes
// the initial guess of `init` bit for bit as launch_init does.

// p[0..n) = 0.
hipError_t launch_clear(double* p, int n, hipStream_t s);

// Coarsening (Sec. 4). When `stats` is non-null it also writes per-workgroup
// partials [nwg][channels + 2]: sum over known pixels of f^2 per channel,
// number of known pixels, number of mask bytes > 1. Returns the number of
// workgroups in *nwg.
hipError_t launch_coarsen(const float* f, const uint8_t* c, int h, int w,
                          int channels, float* fc, uint8_t* cc,
                          double* stats, int* nwg, hipStream_t s);
// Two levels at once (h x w -> middle -> coarsest, each as launch_coarsen
// would make it, bit for bit) when coarsen2_ok: widths divisible by 8 and
// aligned buffers. No statistics.
bool coarsen2_ok(const float* f, const uint8_t* c, const float* fm, const uint8_t* cm,
                 const float* fc, const uint8_t* cc, int w);
int coarsen2_grid(int h, int w, int* gx, int* rows);
hipError_t launch_coarsen2(const float* f, const uint8_t* c, int h, int w, int channels,
                           float* fm, uint8_t* cm, float* fc, uint8_t* cc, hipStream_t s);

// Workgroups (statistics partial rows) launch_coarsen uses for h x w,
// whichever path it takes.
int coarsen_partials(int h, int w);

// Same statistics without coarsening (single-level solves).
hipError_t launch_stats(const float* f, const uint8_t* c, int h, int w,
                        int channels, double* stats, int* nwg, hipStream_t s);

// u = c ? f : 0 (start on the coarsest level).
hipError_t launch_init(const float* f, const uint8_t* c, int h, int w,
                       int channels, float* u, hipStream_t s);

// u = c ? f : bilinear(uc) (coarse-to-fine initialisation, Sec. 4).
hipError_t launch_prolong(const float* uc, int hc, int wc, const float* f,
                          const uint8_t* c, int h, int w, int channels,
                          float* u, hipStream_t s);

// Residual r = b - A u (eq. 7): per-workgroup partial sums of r^2 per
// channel into partial[nwg][channels]; optionally writes r and/or copies u
// into ucopy. Returns the number of workgroups in *nwg.
hipError_t launch_residual(const float* f, const uint8_t* c, const float* u,
                           int h, int w, int channels, float* r,
                           float* ucopy, double* partial, int* nwg,
                           hipStream_t s);

// Workgroups (partial rows) of launch_residual for an h x w plane.
int residual_partials(int h, int w);

// out[j] = sum_i partial[i * stride + j] for j < ncols, fixed order; with
// zero = true the partials are cleared after being read.
hipError_t launch_reduce(const double* partial, int nrows, int stride,
                         int ncols, double* out, hipStream_t s, bool zero = false);

// ---- batched launchers: one launch for the jobs of many images; job
// arrays live in device memory, sorted by wg0 (the first job at 0) ----

// Register layout of the sweep for blocks of height bh.
void sweep_instance(int bh, int* rpw, bool* ragged);
// All jobs of one launch must share the sweep instance (rpw, ragged).
hipError_t launch_sweep_batch(const SweepJob* jobs, int njobs, int total_wg, int rpw,
                              bool ragged, hipStream_t s);
// Width-4 coarsening / prolongation (every w % 4 == 0, aligned buffers).
hipError_t launch_coarsen_batch(const LevelJob* jobs, int njobs, int total_wg, int channels,
                                hipStream_t s);
hipError_t launch_prolong_batch(const LevelJob* jobs, int njobs, int total_wg, int channels,
                                hipStream_t s);
hipError_t launch_init_batch(const LevelJob* jobs, int njobs, int total_wg, int channels,
                             hipStream_t s);
hipError_t launch_mask_bits_batch(const LevelJob* jobs, int njobs, int total_wg, hipStream_t s);
// Stop tests after finest-level sweep n (see launch_decide), one per job.
hipError_t launch_decide_batch(const DecideJob* jobs, int njobs, int channels, int n,
                               hipStream_t s);
hipError_t launch_reduce_batch(const ReduceJob* jobs, int njobs, int ncols, hipStream_t s);
// Whether the width-4 coarsening / prolongation applies (w % 4 == 0 and
// vector-aligned buffers); launch_coarsen / launch_prolong take it then.
bool coarsen4_ok(const float* f, const uint8_t* c, const float* fc, const uint8_t* cc, int w);
bool prolong4_ok(const float* uc, const float* f, const uint8_t* c, const float* u, int w);
// Statistics rows launch_coarsen / launch_stats write for these arguments.
int coarsen_rows(const float* f, const uint8_t* c, const float* fc, const uint8_t* cc, int h,
                 int w);
int stats_rows(int h, int w);
// Workgroups of one job (h, w: the finer level) and its per-job geometry.
int coarsen4_grid(int h, int w, int* gx, int* rows);
int prolong4_grid(int h, int w, int* gx);
int init_grid(int h, int w);
int mask_bits_grid(int h, int w, int* gx);

// ---- bfloat16 storage with float32 iterative refinement ----

// ---- Krylov-accelerated ORAS (method = 2) ----
// w = A z and (w, v_i) for i < nv (v_i = V + i * vstride): partials
// [wg][i][C] over residual_partials(h, w) workgroups.
hipError_t launch_kry_matvec_dots(const float* z, const uint8_t* c, int h, int w, int channels,
                                  float* wout, const float* V, int64_t vstride, int nv,
                                  double* partial, const int* ctl, hipStream_t s);
// w -= sum_i hcol[i * C + ch] v_i; partials [wg][C] of ||w||^2.
hipError_t launch_kry_orth(float* wv, const float* V, int64_t vstride, int nv,
                           const double* hcol, int h, int w, int channels, double* partial,
                           const int* ctl, hipStream_t s);
// dst = src / sqrt(norm2[ch]) (skipped after convergence unless force).
hipError_t launch_kry_scale(const float* src, float* dst, const double* norm2, int64_t n,
                            int channels, const int* ctl, bool force, hipStream_t s);
hipError_t launch_kry_start(KryState* st, const double* beta2, const double* b2, int channels,
                            int* ctl, double tol2, int total, hipStream_t s);
hipError_t launch_kry_givens(KryState* st, const double* hcol, const double* hn2, int j,
                             int channels, int* ctl, double tol2, int total, hipStream_t s);
hipError_t launch_kry_backsolve(KryState* st, int channels, hipStream_t s);
hipError_t launch_kry_combine(float* u, const float* Z, int64_t zstride, const KryState* st,
                              int64_t n, int channels, hipStream_t s);

// One ORAS sweep of the correction equation A d = rhs with d and rhs in
// float32 (din == nullptr: d = 0; d = 0 on the mask): the preconditioner of
// the Krylov method. Otherwise as launch_sweep.
hipError_t launch_sweep_c32(const float* din, const float* rhs, const uint64_t* mbits,
                            float* dout, double* partial, double* cg_steps, const int* ctl,
                            const SweepArgs& a, hipStream_t s);

// One ORAS sweep of the refinement equation A d = rhs (d = 0 on the mask):
// din, rhs, dout bfloat16 planes like u (din == nullptr: d = 0); float32
// arithmetic; otherwise as launch_sweep.
hipError_t launch_sweep_corr(const uint16_t* din, const uint16_t* rhs, const uint64_t* mbits,
                             uint16_t* dout, double* partial, double* cg_steps, const int* ctl,
                             const SweepArgs& a, hipStream_t s);

// The first refinement residual fused with the coarse-to-fine start: vout
// = c ? f : the bilinear prolongation of S.uc (bit for bit launch_prolong's),
// rhs = bfloat16(b - A vout), float64 partials as launch_residual's. S.hc
// and S.wc must be ceil(h / 2) and ceil(w / 2). Does nothing once ctl[0] != 0.
hipError_t launch_start_residual(const ProSrc& S, int h, int w, int channels, float* vout,
                                 uint16_t* rhs, double* partial, const int* ctl, int* nwg,
                                 hipStream_t s);

// unext = u + d (skipped when d == nullptr), rhs = bfloat16(b - A unext),
// float64 partials of ||b - A unext||^2 laid out as launch_residual's (same
// workgroup count). Requires u = f and d = 0 on the mask (f is not read).
// Does nothing once ctl[0] != 0.
hipError_t launch_refine_residual(const float* f, const uint8_t* c, const float* u,
                                  const uint16_t* d, int h, int w, int channels, float* unext,
                                  uint16_t* rhs, double* partial, const int* ctl, int* nwg,
                                  hipStream_t s);

// Float64 CG solve of the coarsest level (h * w <= kCoarseMaxPixels), one
// workgroup per channel: u = exact solution (rounded to float32) once
// ||b - A u|| <= tol ||C f||, or after max_iter steps.
hipError_t launch_coarse_cg(const float* f, const uint8_t* c, int h, int w, int channels,
                            float* u, int max_iter, double tol, hipStream_t s);
hipError_t launch_coarse_cg_batch(const CoarseJob* jobs, int njobs, int channels, hipStream_t s);

// The same float64 CG on a level of any size, run by `wgs` workgroups
// (1..kGridCgMaxWg) that stay resident for the whole solve and meet at grid
// barriers. work: coarse_grid_bytes(h, w, channels) bytes, 256-byte aligned,
// owned by the caller (control words, partial sums, five float64 vectors);
// the launcher clears its control words first. A barrier that waits longer
// than its bound (about a second: workgroups that never became resident)
// ends the solve on every workgroup and leaves a nonzero status word
// (coarse_grid_status); with ctl given it also sets ctl[2] = 3 and ctl[0] =
// 1, so that the plan's later sweeps and stop tests do nothing.
constexpr int kGridCgMaxWg = 256;
size_t coarse_grid_bytes(int h, int w, int channels);
int coarse_grid_workgroups(int h, int w, int channels);
// Device addresses inside `work`: the barrier status (int, 0 = ok) and the
// CG steps taken per channel (int[4]).
const int* coarse_grid_status(const void* work);
// Bound of every later grid-solve barrier wait, in polls (test hook; < 0:
// the default).
void set_coarse_grid_spin_limit(long polls);
const int* coarse_grid_steps(const void* work);
hipError_t launch_coarse_cg_grid(const float* f, const uint8_t* c, int h, int w, int channels,
                                 float* u, int max_iter, double tol, int wgs, void* work,
                                 int* ctl, hipStream_t s);

// ---- global conjugate gradients (multilevel-CG comparator) ----
// Partial rows of these kernels: residual_partials(h, w). All skip their
// work once ctl[0] != 0.
hipError_t launch_cg_dir_matvec(const float* r, const float* pin, float* pout, float* q,
                                const uint8_t* c, int h, int w, int channels,
                                const double* beta, bool first, double* partial, const int* ctl,
                                int* nwg, hipStream_t s);
hipError_t launch_cg_update(float* x, float* r, const float* p, const float* q, int h, int w,
                            int channels, const double* alpha, double* partial, const int* ctl,
                            hipStream_t s);
// stage 0: alpha = rho / p.q; 1: beta = r.r / rho, rho = r.r, stop test
// (tol < 0: never passes); 2: rho = r.r and the stop test. sc = [rho,
// alpha, beta] x channels.
hipError_t launch_cg_scalars(const double* partial, int nb, int channels, double* sc,
                             const double* b2, int* ctl, double tol, int stage, int n,
                             hipStream_t s);

// Partials per channel written by one sweep: one per block.
inline int sweep_partials(const SweepArgs& a) {
    return a.g.nby * a.g.nbx;
}

}  // namespace ddi
