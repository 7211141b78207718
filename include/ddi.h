/*
 * ddi.h -- C ABI of the MI355X (gfx950) multilevel ORAS solver for
 * homogeneous diffusion inpainting.
 *
 * Method: Kaemper & Weickert, "Domain decomposition algorithms for real-time
 * homogeneous diffusion inpainting in 4K" (arXiv 2110.03946).
 *   - The problem (Sec. 2, eqs. 5-6): per colour channel solve A u = b with
 *     A = C - (I - C) L and b = C f, where L is the 5-point Laplacian with
 *     reflecting image boundaries and C the 0/1 diagonal of the mask. Known
 *     pixels keep their value; unknown pixels satisfy the discrete Laplace
 *     equation.
 *   - The solver (Sec. 3 eqs. 7-10, Sec. 4): optimised restricted additive
 *     Schwarz over overlapping square blocks, each local problem solved by a
 *     few conjugate-gradient steps, with a Robin interface condition, a
 *     Boolean partition of unity, and a coarse-to-fine start from dyadically
 *     subsampled masks and values.
 *
 * Conventions for every entry point:
 *   - Images are planar, dense, row-major float32: channel k, row y, column x
 *     sits at index (k * height + y) * width + x. The mask is one dense
 *     height x width uint8 plane (1 = known pixel, 0 = to be inpainted)
 *     shared by all channels. Grey values are expected in [0, 255] but any
 *     finite values work.
 *   - Pointers named f, c, u, r, ... are DEVICE pointers (HIP global memory,
 *     e.g. the data_ptr() of a torch tensor on a ROCm device). They remain
 *     owned by the caller; the library never frees them. Input and output
 *     buffers must not overlap: every call checks the address ranges on the
 *     host and returns DDI_EINVAL when an output shares a byte with an
 *     input (or, in a batch, with another image's buffers).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it; calls that return results on the host
 *     synchronise that stream.
 *   - Every call returns DDI_OK (0) or a negative DDI_E* code; ddi_strerror
 *     turns it into text. On DDI_EHIP, ddi_last_hip_error gives the HIP
 *     error code of the failing runtime call.
 *   - Nothing here is thread-safe for one plan; use one plan per stream.
 *     Different plans may be driven from different host threads at once.
 */
#ifndef DDI_H
#define DDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define DDI_OK          0
#define DDI_EINVAL     (-1)  /* bad size, parameter or pointer; mask byte > 1 */
#define DDI_ESINGULAR  (-2)  /* no known pixel: A is singular (Sec. 2 needs K nonempty) */
#define DDI_ENOMEM     (-3)  /* device allocation failed */
#define DDI_ENOCONV    (-4)  /* max_sweeps reached before rel_tol */
#define DDI_EHIP       (-5)  /* a HIP runtime call failed */
#define DDI_ENODEV     (-6)  /* no usable gfx950 device */
#define DDI_ESCRATCH   (-7)  /* ddi_oras_sweep_noalloc: the call needs more than
                                DDI_NOALLOC_SCRATCH_BYTES of scratch */
#define DDI_ESTALL     (-8)  /* a grid-wide wait of the float64 coarse solve on
                                many workgroups exceeded its bound (its
                                workgroups were not all resident); the result
                                is not valid */

/* Largest block edge (pixels) the on-chip local solver supports. */
#define DDI_MAX_BLOCK 64

/* Fixed device scratch of ddi_oras_sweep_noalloc, per GPU (4 MiB). */
#define DDI_NOALLOC_SCRATCH_BYTES (4u << 20)

/* Largest level (pixels) of the one-workgroup-per-channel float64 coarse
 * solve (ddi_coarse_solve); larger coarsest levels of coarse_solver = 1 use
 * the grid solve (ddi_coarse_solve_grid). */
#define DDI_COARSE_MAX_PIXELS 8192

/*
 * Solver parameters. Fill with ddi_default_params, then override.
 *   block          S: edge of a square block, overlap included (Sec. 4),
 *                  2 <= S <= DDI_MAX_BLOCK. Blocks are cut to the image
 *                  when the image is smaller.
 *   overlap        o: pixels shared by neighbouring blocks, 0 <= o < S.
 *                  Block k starts at min(k (S - o), n - S).
 *   levels         resolution levels of the coarse-to-fine scheme (Sec. 4),
 *                  >= 1; level l has size ceil(n / 2^l).
 *   local_iters    k: CG steps per local solve (Sec. 4), >= 1.
 *   robin_alpha    weight of an interface neighbour in the local diagonal
 *                  (ORAS, Sec. 3): 1 = RAS (homogeneous Dirichlet at the
 *                  block interface), towards 0 = Neumann. 0 < alpha <= 1.
 *   coarse_sweeps  ORAS sweeps on each level between the coarsest and the
 *                  finest, >= 0.
 *   coarsest_sweeps ORAS sweeps on the coarsest level, >= 0.
 *   rel_tol        stop on the finest level once ||b - A u||_2 <= rel_tol
 *                  ||b||_2 holds in every channel (float64 norms), >= 0.
 *   min_sweeps     finest-level sweeps before the first stop test, >= 0.
 *   max_sweeps     cap on finest-level sweeps, >= min_sweeps.
 *   check_every    sweeps between stop tests, >= 1.
 *   final_residual 1: recompute ||b - A u|| of the returned u (float64) for
 *                  the stats; 0: report the last stop-test residual.
 *   timing         1: bracket every finest-level sweep with HIP events and
 *                  report their summed device time and CG step count in the
 *                  stats (costs one small kernel per solve).
 *   coarse_block   block edge on the coarser levels (0 = block); small
 *                  levels solve faster with more, smaller blocks.
 *   coarse_overlap overlap on the coarser levels (-1 = overlap).
 *   coarse_local_iters CG steps per local solve on the coarser levels
 *                  (0 = local_iters).
 *   local_tol      absolute stop of the local CG (grey levels): a block
 *                  stops early once its mean square local residual is at
 *                  most local_tol^2 (0 = always local_iters steps). Blocks
 *                  that are already converged then cost no CG work; the
 *                  fixed point of the iteration is unchanged.
 *   use_graph      1: capture the solve (everything up to and including the
 *                  first batch of finest-level sweeps) into a HIP graph on a
 *                  stream the plan owns, and replay it on later solves with
 *                  the same f, c and u pointers (ignored with timing = 1).
 *   coarse_solver  0: coarsest_sweeps ORAS sweeps on the coarsest level;
 *                  1: solve the coarsest level in float64 by conjugate
 *                  gradients: one workgroup per channel when the level has
 *                  at most DDI_COARSE_MAX_PIXELS pixels, else the grid
 *                  solve of ddi_coarse_solve_grid (many workgroups, grid
 *                  barriers; the plan holds its workspace).
 *   coarse_cg_iters cap on CG steps of coarse_solver = 1, >= 1.
 *   coarse_cg_tol  coarse_solver = 1 stops once ||b - A u||_2 <= tol ||b||_2
 *                  on the coarsest level (float64), >= 0.
 *   storage        0: the finest level iterates on u in float32 (ORAS sweeps
 *                  on A u = b). 1: mixed precision with iterative
 *                  refinement: after the coarse-to-fine start u_0 (float32),
 *                  refinement step k forms r_k = b - A u_k from the float32
 *                  u_k (stored in bfloat16, its norm in float64), runs
 *                  inner_sweeps ORAS sweeps on the correction equation
 *                  A d = r_k from d = 0 with d stored in bfloat16 (float32
 *                  arithmetic), and sets u_{k+1} = u_k + d in float32. The
 *                  stop test applies to r_k, so min_sweeps, max_sweeps and
 *                  check_every count refinement steps, and the returned u_k
 *                  is the iterate whose residual was tested. Single-image
 *                  plans only.
 *   inner_sweeps   correction sweeps per refinement step (storage = 1), >= 1.
 *   method         0: multilevel ORAS (the method). 1: multilevel conjugate
 *                  gradients, the comparator of Sec. 5: the same pyramid and
 *                  coarse-to-fine start, every level solved by global CG on
 *                  its unknown pixels (float32 vectors, float64 dot products)
 *                  to rel_tol; max_sweeps then caps the CG steps per level
 *                  and stats.sweeps counts the finest level's steps. Single-
 *                  image float32 plans only.
 *                  2: Krylov-accelerated ORAS (not in the paper): the same
 *                  coarse-to-fine start, then flexible GMRES(krylov_restart)
 *                  on the finest level per channel, each basis vector
 *                  preconditioned by one ORAS sweep (block, overlap,
 *                  robin_alpha, local_iters; local_tol, an absolute
 *                  threshold, does not apply to the unit basis vectors) on
 *                  the correction equation A d = v from d = 0; it stops once
 *                  max_k
 *                  ||b - A u||/||b|| <= rel_tol (signalled by the
 *                  least-squares estimate, confirmed on the recomputed
 *                  residual). max_sweeps caps the Krylov steps (one
 *                  preconditioner sweep each), stats.sweeps counts them.
 *                  Single-image float32 plans only.
 *   krylov_restart restart length m of method = 2, 1 <= m <= 16 (the plan
 *                  holds 2m + 1 finest-level vectors).
 *   fuse_prolong   1: the first ORAS sweep on a level after the coarse-to-
 *                  fine prolongation builds its tiles from the coarser
 *                  level's iterate and f (the prolongation is computed in
 *                  the sweep's tile load and never stored); levels whose
 *                  blocks are not 64 rows high, the finest level of
 *                  storage = 1 and max_sweeps = 0 keep the separate
 *                  prolongation. 0: always the separate prolongation. Both
 *                  give the same iterates whenever the interpolation sums
 *                  are exact in float64 (neighbouring coarse values within
 *                  a factor 2^26 of each other).
 *   skip_unchanged 1: finest-level ORAS sweeps after the second one skip
 *                  work the previous sweep made redundant. A block that the
 *                  previous sweep left unchanged (no local CG step) and
 *                  that runs no CG step again skips its write-back: the
 *                  output buffer, the previous sweep's input, already holds
 *                  these values on its owned pixels. A block whose 3 x 3
 *                  neighbourhood of blocks the previous sweep left unchanged
 *                  has the same input tile as then, hence the same residual
 *                  and again no CG step: it is skipped whole. The iterates
 *                  are bit for bit those of skip_unchanged = 0. Applies to
 *                  float32 single-image ORAS plans (storage = 0, method =
 *                  0) whose finest level has 64-row blocks and a grid where
 *                  every block's tile lies in its 3 x 3 neighbourhood
 *                  (overlap small against the block size); ignored
 *                  otherwise. 0: every sweep does all its work.
 *   order_blocks   1: each finest-level ORAS sweep runs its blocks in the
 *                  order of the local CG steps that the sweep of the level
 *                  two below the finest needed over the block's centre,
 *                  most first, so that the blocks with long local solves
 *                  start first and do not finish after the rest of the
 *                  launch (where the coarse level found the error large,
 *                  the later finest sweeps also need most steps). A
 *                  scheduling choice
 *                  only: the iterates are bit for bit those of 0. Applies
 *                  where the finest level has 64-row blocks and fewer than
 *                  65536 blocks over its channels, at most 1024 per axis
 *                  (float32 ORAS, storage = 0, method = 0); ignored
 *                  otherwise.
 */
typedef struct ddi_params {
    int block;
    int overlap;
    int levels;
    int local_iters;
    float robin_alpha;
    int coarse_sweeps;
    int coarsest_sweeps;
    double rel_tol;
    int min_sweeps;
    int max_sweeps;
    int check_every;
    int final_residual;
    int timing;
    int coarse_block;
    int coarse_overlap;
    int coarse_local_iters;
    float local_tol;
    int use_graph;
    int coarse_solver;
    int coarse_cg_iters;
    double coarse_cg_tol;
    int storage;
    int inner_sweeps;
    int method;
    int fuse_prolong;
    int krylov_restart;
    int skip_unchanged;
    int order_blocks;
} ddi_params;

/*
 * Result of a solve.
 *   sweeps        ORAS sweeps run on the finest level.
 *   converged     1 if rel_tol was met.
 *   rel_residual  max over channels of ||b - A u||_2 / ||b||_2 (float64)
 *                 for the returned u (final_residual = 1), or for the
 *                 iterate of the last stop test (final_residual = 0).
 *   ms            device time of the solve from HIP events, milliseconds.
 *   sweep_ms      with timing = 1: summed device time of the finest-level
 *                 sweeps (the solver's dominant kernel), milliseconds.
 *   cg_steps      with timing = 1: local CG steps run by the finest-level
 *                 sweeps, summed over blocks and channels (fewer than blocks
 *                 x local_iters when local_tol stops blocks early).
 *   refinements   storage = 1: refinement steps taken (the finest-level
 *                 sweeps are then refinements x inner_sweeps); 0 otherwise.
 *   first_sweep_ms, first_cg_steps
 *                 with timing = 1 and storage = 0: the part of sweep_ms and
 *                 cg_steps that falls on the first finest-level sweep (the
 *                 one that also computes the prolongation when
 *                 fuse_prolong applies); 0 otherwise.
 *   skipped_blocks, unwritten_blocks
 *                 with timing = 1 and skip_unchanged in effect: blocks (over
 *                 channels and finest-level sweeps) skipped whole, and
 *                 blocks that ran but skipped their write-back; 0
 *                 otherwise.
 */
typedef struct ddi_stats {
    int sweeps;
    int converged;
    double rel_residual;
    double ms;
    double sweep_ms;
    double cg_steps;
    int refinements;
    double first_sweep_ms;
    double first_cg_steps;
    double skipped_blocks;
    double unwritten_blocks;
} ddi_stats;

typedef struct ddi_plan ddi_plan;

/* Fill *p with the defaults: S = 64, o = 4, 4 levels, k = 16, alpha = 0.25,
 * 2 sweeps per coarser level, 3 on the coarsest, rel_tol = 1e-4,
 * min_sweeps = 2, max_sweeps = 50, check_every = 1, final_residual = 1,
 * timing = 0, coarse_block = 0, coarse_overlap = -1, coarse_local_iters = 0,
 * local_tol = 0, use_graph = 0, coarse_solver = 0, coarse_cg_iters = 500,
 * coarse_cg_tol = 1e-10, storage = 0, inner_sweeps = 2, method = 0,
 * fuse_prolong = 1, krylov_restart = 8, skip_unchanged = 1, order_blocks = 1. */
int ddi_default_params(ddi_params* p);

/* Check *p for one image size without touching the GPU (this includes the
 * size of the coarsest level when coarse_solver = 1). */
int ddi_check_params(int height, int width, int channels, const ddi_params* p);

/*
 * Create a plan for height x width images with `channels` channels sharing
 * one mask. Allocates every device buffer the solve needs (level pyramid,
 * ping-pong iterate, reduction partials) once; ddi_solve allocates nothing.
 * p == NULL uses the defaults. The plan keeps `stream`.
 * Errors: DDI_EINVAL (sizes or params), DDI_ENOMEM, DDI_ENODEV, DDI_EHIP.
 */
int ddi_create(ddi_plan** out, int height, int width, int channels,
               const ddi_params* p, void* stream);

/*
 * Inpaint: multilevel ORAS (Sec. 3-4) for all channels of f with mask c,
 * writing the result to u. f: channels x height x width float32; c: height x
 * width uint8; u: like f, fully written, with u = f bit for bit on the mask.
 * Synchronises the plan's stream (stop tests read float64 norms).
 * Errors: DDI_EINVAL (null pointer, u overlapping f or c, mask byte > 1),
 * DDI_ESINGULAR (empty mask), DDI_ENOCONV (u then holds the last iterate and
 * *st is filled), DDI_EHIP. st may be NULL.
 */
int ddi_solve(ddi_plan* plan, const float* f, const uint8_t* c, float* u,
              ddi_stats* st);

/*
 * ddi_solve in two halves, so that one host thread can keep the GPU busy
 * with several plans (e.g. consecutive frames on two plans sharing a
 * stream): ddi_solve_async enqueues the solve up to its first host check
 * (the pyramid, the coarse levels and as many finest-level sweeps as the
 * plan's previous solve needed, with their device stop tests) and returns;
 * ddi_solve_wait waits for that plan's work only (HIP events), enqueues
 * more sweeps if the stop test has not passed, finishes and fills *st.
 * Each plan holds at most one pending solve; f, c, u must stay valid until
 * the wait returns. st->ms then spans the plan's own enqueue-to-finish
 * interval on the stream, which includes work of other plans queued in
 * between. storage = 1 plans: use ddi_solve (DDI_EINVAL here).
 */
int ddi_solve_async(ddi_plan* plan, const float* f, const uint8_t* c, float* u);
int ddi_solve_wait(ddi_plan* plan, ddi_stats* st);

/* Release the plan and its device buffers. NULL is a no-op. */
int ddi_destroy(ddi_plan* plan);

/* Device memory (bytes) a plan for these sizes and parameters allocates,
 * without touching the GPU (p == NULL: defaults): what a server admitting
 * requests by HBM footprint charges for the plan, on top of the caller's
 * f, c and u. ddi_plan_bytes reports it for an existing plan. */
int ddi_plan_footprint(int height, int width, int channels,
                       const ddi_params* p, size_t* bytes);
int ddi_plan_bytes(const ddi_plan* plan, size_t* bytes);

/* ---- batched solve ------------------------------------------------------
 * Many images of uneven size solved together: every step of the scheme
 * (coarsening, transposed masks, the sweeps of each level, prolongation,
 * the stop tests) runs as one launch over the work items of all images, so
 * that small images fill the GPU together and a batch costs the launches of
 * one image. Each image keeps its own stop test; results equal those of
 * ddi_solve on each image with the same parameters (the same kernels run on
 * the same data), bit for bit.
 */
typedef struct ddi_batch ddi_batch;

/*
 * Create a batch plan for n images; image i is heights[i] x widths[i] with
 * `channels` channels (shared by all). p is NULL (defaults), one params
 * struct (n_params = 1) or one per image (n_params = n), e.g. picked per
 * size by a tuner. max_sweeps, check_every and timing must be equal across
 * images (the finest-level sweeps run in lock step); min_sweeps may differ:
 * the stop tests run after sweep m, m + check_every, ... (m the smallest
 * min_sweeps), and an image's test passes only from its own min_sweeps on.
 * use_graph is ignored. Allocates every device buffer once.
 * Errors: DDI_EINVAL, DDI_ENOMEM, DDI_ENODEV, DDI_EHIP.
 */
int ddi_batch_create(ddi_batch** out, int n, const int* heights,
                     const int* widths, int channels, const ddi_params* p,
                     int n_params, void* stream);

/*
 * Inpaint all images: f[i], c[i], u[i] are device pointers laid out as for
 * ddi_solve (host arrays of n pointers). st (n entries) and status (n codes:
 * DDI_OK, DDI_EINVAL for a mask byte > 1, DDI_ESINGULAR, DDI_ENOCONV,
 * DDI_ESTALL) may be NULL; st[i].ms and st[i].sweep_ms are those of the whole batch.
 * Returns DDI_OK when every image converged, else the first image's error
 * code in order (or DDI_EHIP / DDI_EINVAL for the call itself). Synchronises
 * the stream.
 */
int ddi_batch_solve(ddi_batch* b, const float* const* f,
                    const uint8_t* const* c, float* const* u, ddi_stats* st,
                    int* status);

/* Release the batch plan. NULL is a no-op. */
int ddi_batch_destroy(ddi_batch* b);

/*
 * Host self-check of the kernels' index arithmetic. Replays every global-
 * memory offset that the kernels of a float32 ORAS plan for height x width
 * x channels with parameters p (NULL: defaults) read or write -- the
 * transposed mask bits, both coarsening kernels, every level's sweeps (with
 * the first sweep of a level that builds its tile from the coarser level),
 * both prolongation kernels and the column-walking kernels -- computed by
 * the functions the kernels themselves use, over every thread of every
 * launch, and checks each offset against the buffer it addresses. No GPU is
 * used. *checked (may be NULL) receives the number of offsets checked,
 * *violations (may be NULL) the number outside their buffer, first (may be
 * NULL, first_len bytes) a description of the first such offset.
 * Errors: those of ddi_check_params.
 */
int ddi_selfcheck_access(int height, int width, int channels, const ddi_params* p,
                         long long* checked, long long* violations, char* first,
                         int first_len);

/* Text for an error code (static storage). */
const char* ddi_strerror(int code);

/* HIP error code of the last DDI_EHIP returned to the calling host thread
 * (0 if none). */
int ddi_last_hip_error(void);

/* With timing = 1: the device time of each finest-level ORAS sweep of the
 * plan's last solve: ms[i] for sweep i < n, *count (may be NULL) = sweeps
 * of that solve (0 without timing). Float32 solves (storage = 0, method =
 * 0): from events that the sweep launch itself records at the kernel's
 * start and end. Mixed precision (storage = 1): the correction sweeps in
 * order, from events recorded on the stream around each launch. Host only. */
int ddi_sweep_times(const ddi_plan* plan, double* ms, int n, int* count);

/* Geometry of the block grid the solver uses on an n-pixel axis: number of
 * blocks, and origin / owned range [lo, hi) of block k (k < count). Host
 * only; lets callers and tests check the partition of unity (eq. 10). */
int ddi_block_count(int n, int block, int overlap);
int ddi_block_range(int n, int block, int overlap, int k, int* origin,
                    int* own_lo, int* own_hi);

/* ---- the steps of the path, exposed one by one -------------------------
 * Each enqueues on `stream`; those returning host values synchronise it.
 * They allocate device scratch per call (unlike ddi_solve).
 */

/*
 * Residual r = b - A u of eq. 7 (the masked 5-point stencil), for all
 * channels: r_p = f_p - u_p on the mask, sum over in-image 4-neighbours q
 * of (u_q - u_p) elsewhere. r may be NULL (norms only). rsq (host,
 * `channels` doubles, may be NULL) receives sum_p r_p^2 per channel,
 * accumulated in float64.
 */
int ddi_residual(const float* f, const uint8_t* c, const float* u, int height,
                 int width, int channels, float* r, double* rsq, void* stream);

/*
 * One dyadic subsampling step (Sec. 4): coarse pixel (I, J) covers the
 * in-image fine pixels (2I + a, 2J + b), a, b in {0, 1}; it is known iff one
 * of them is, and its value is the float64 mean of the known fine values,
 * rounded to float32 (0 where unknown). fc: channels x ceil(h/2) x ceil(w/2)
 * float32, cc: ceil(h/2) x ceil(w/2) uint8.
 */
int ddi_coarsen(const float* f, const uint8_t* c, int height, int width,
                int channels, float* fc, uint8_t* cc, void* stream);

/*
 * Coarse-to-fine initialisation (Sec. 4): u = f on the mask, elsewhere the
 * bilinear interpolation of the coarse grid uc (channels x hc x wc) at the
 * fine pixel centre (y/2 - 1/4, x/2 - 1/4), clamped to the coarse grid.
 * Requires hc = ceil(height/2), wc = ceil(width/2).
 */
int ddi_prolong(const float* uc, int hc, int wc, const float* f,
                const uint8_t* c, int height, int width, int channels,
                float* u, void* stream);

/*
 * One ORAS iteration (Sec. 3, eqs. 7-9) on all channels, u_in -> u_out:
 * the residual of u_in restricted to each block, k CG steps on the block's
 * local matrix with Robin weight alpha at the interface, and the sum of the
 * restricted corrections over the Boolean partition of unity. u_in must
 * equal f on the mask (then u_out does too). rsq (host, may be NULL)
 * receives sum_p r_p^2 of u_in per channel in float64.
 */
int ddi_oras_sweep(const float* u_in, const uint8_t* c, float* u_out,
                   int height, int width, int channels, int block,
                   int overlap, float robin_alpha, int local_iters,
                   double* rsq, void* stream);

/*
 * ddi_oras_sweep for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops or harnesses that forbid hipMalloc). The
 * same sweep, the same arguments and bit for bit the same u_out and rsq; it
 * calls no hipMalloc or hipFree. Its scratch (the column-transposed mask
 * bits, one float64 norm partial per block and channel, and their
 * per-channel sums) is a fixed array of DDI_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends;
 * ddi_noalloc_scratch_bytes reports what a call of these sizes needs
 * (host only). Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap in time on one GPU race (issue them on
 * one stream, or order them). Synchronises `stream` only when rsq is given.
 * Errors: DDI_EINVAL (as ddi_oras_sweep, or u_out overlapping u_in or c),
 * DDI_ESCRATCH (the sizes need more than the fixed scratch), DDI_EHIP.
 */
int ddi_noalloc_scratch_bytes(int height, int width, int channels, int block,
                              int overlap, size_t* bytes);
int ddi_oras_sweep_noalloc(const float* u_in, const uint8_t* c, float* u_out,
                           int height, int width, int channels, int block,
                           int overlap, float robin_alpha, int local_iters,
                           double* rsq, void* stream);

/*
 * Float64 solve of A u = b (Sec. 2, eq. 6) on a small grid, the solver of
 * the coarsest level (coarse_solver = 1): conjugate gradients on the unknown
 * pixels in float64, one workgroup per channel, from u = c ? f : 0 until
 * ||b - A u||_2 <= tol ||b||_2 or max_iter steps; u (float32) receives the
 * rounded iterate, f on the mask. height * width <= DDI_COARSE_MAX_PIXELS.
 */
int ddi_coarse_solve(const float* f, const uint8_t* c, int height, int width,
                     int channels, float* u, int max_iter, double tol,
                     void* stream);

/*
 * The same float64 solve on a level of any size (height * width <= 2^30):
 * the conjugate gradients of ddi_coarse_solve, with the vectors in the
 * caller's workspace and `workgroups` workgroups (1..256; 0 = a default from
 * the size) that stay resident for the whole solve and meet at two grid
 * barriers per step. The per-channel partial sums of each dot product are
 * added in a fixed order, so the result does not depend on timing; it
 * differs from ddi_coarse_solve's only by the order of those sums.
 *   work, work_bytes  device workspace of at least ddi_coarse_grid_bytes
 *                     bytes, 256-byte aligned, not overlapping f, c or u;
 *                     owned by the caller, overwritten by the call (calls
 *                     that share one workspace must not overlap in time).
 *   steps             NULL: the call is asynchronous on `stream`. Else the
 *                     call waits for the stream and stores the CG steps each
 *                     channel took in steps[0..channels).
 * Errors: DDI_EINVAL (sizes, tolerances, pointers, a short or misaligned
 * workspace, u overlapping an input); DDI_ESTALL (only with steps given) if
 * a barrier wait exceeded its bound, when not every workgroup could run.
 */
int ddi_coarse_grid_bytes(int height, int width, int channels, size_t* bytes);
/*
 * Test hook of the DDI_ESTALL path: later grid solves of this process bound
 * each barrier wait by `polls` polls instead of the default (about two
 * seconds' worth); 0 makes every wait that does not end at once a stall, so
 * a solve on two or more workgroups reports DDI_ESTALL while every
 * workgroup still ends. polls < 0 restores the default.
 */
int ddi_coarse_grid_debug_spin_limit(long polls);
int ddi_coarse_solve_grid(const float* f, const uint8_t* c, int height, int width,
                          int channels, float* u, int max_iter, double tol,
                          int workgroups, void* work, size_t work_bytes,
                          int* steps, void* stream);

/*
 * The two steps of the mixed-precision refinement (storage = 1), exposed
 * for tests. bfloat16 planes (d, rhs) are uint16 bit patterns laid out like
 * u.
 *
 * ddi_refine_residual: u_next = u + d in float32 (d may be NULL: then u_next
 * is not written and u itself is used), rhs = bfloat16(b - A u_next) of
 * eq. 7 rounded to nearest even, rsq (host, channels doubles, may be NULL)
 * = sum of (b - A u_next)^2 per channel in float64. Requires u = f and
 * d = 0 on the mask, as the refinement keeps them: the residual is then 0
 * there, the stencil takes the known values from u, and f is not read.
 *
 * ddi_refine_start: the first residual of the refinement built with the
 * coarse-to-fine start (Sec. 4): u = c ? f : the bilinear interpolation of
 * the coarse grid uc (channels x hc x wc, hc = ceil(height/2), wc =
 * ceil(width/2)), bit for bit what ddi_prolong writes, and rhs and rsq as
 * ddi_refine_residual gives for that u (0 on the mask).
 *
 * ddi_correction_sweep: one ORAS iteration (Sec. 3, eqs. 7-9) on the
 * refinement equation A d = rhs with d = 0 on the mask: the block residual
 * rhs - A d_in (float32), k local CG steps, d_out = d_in + owned
 * corrections rounded to bfloat16. d_in may be NULL (d = 0).
 */
int ddi_refine_residual(const float* f, const uint8_t* c, const float* u,
                        const uint16_t* d, int height, int width, int channels,
                        float* u_next, uint16_t* rhs, double* rsq, void* stream);
int ddi_refine_start(const float* uc, int hc, int wc, const float* f,
                     const uint8_t* c, int height, int width, int channels,
                     float* u, uint16_t* rhs, double* rsq, void* stream);
int ddi_correction_sweep(const uint16_t* d_in, const uint16_t* rhs,
                         const uint8_t* c, uint16_t* d_out, int height,
                         int width, int channels, int block, int overlap,
                         float robin_alpha, int local_iters, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DDI_H */
