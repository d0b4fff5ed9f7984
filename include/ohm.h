/*
 * ohm.h -- C ABI of the MI355X library for the implicit ohmic-dissipation step
 * of Matsumoto (PASJ 2011, "An Implicit Scheme for Ohmic Dissipation with
 * Adaptive Mesh Refinement").
 *
 * One Crank-Nicolson step (section 2.1, eq. 7 with lambda = 1/2) solves
 *     L B = S,   L B = B + lambda dt div F(B)            (eqs. 12-13)
 *                S   = b - (1 - lambda) dt div F(b)      (eq. 14)
 * where F are the face fluxes of eqs. (4)-(6) with the differences (9)-(10)
 * and the face resistivity (11), on the cell-centred fields of a block-
 * structured AMR hierarchy with a periodic box.  The solve uses multigrid
 * (section 2.2): red-black smoothing (eq. 19, 21-23), averaging restriction and
 * trilinear prolongation, refluxing at coarse-fine faces (section 4).
 *
 * ---------------------------------------------------------------------------
 * Data layout (all fields live in device memory owned by the caller)
 * ---------------------------------------------------------------------------
 * A handle holds one or more independent problems.  Each problem has AMR
 * levels 0..nlevels-1 built from 8^3-cell blocks; level l has cell width
 * dx0 / 2^l and level 0 tiles the periodic box.
 *
 * "Field at AMR level l >= 0" (block layout):
 *     T[ncomp][nblocks(l)][8][8][8]          (x fastest inside a block)
 * where nblocks(l) counts the level-l blocks of every problem of the handle,
 * problem after problem, each problem's blocks in the order the caller gave.
 * "Field at multigrid level l < 0" (the coarsenings of the base grid, made by
 * the library when every axis is even, at least 4 cells, and the grid has
 * more than 64 cells):
 *     T[ncomp][ncells(l)]                    (dense layout)
 * where every problem that has that level contributes its cells in
 * z-y-x order (x fastest), problem after problem.
 * T is double (OHM_F64) or float (OHM_F32) and is the arithmetic type of the
 * call; every field of one call, resistivity included, has type T.
 * ncomp is 3 for B, S, R and 1 for eta.
 *
 * Ownership: the library never allocates, frees or retains caller memory.
 * The handle owns only its own metadata (block tables, per-problem scalars).
 *
 * Streams: every call is asynchronous on `stream` except where stated; the
 * caller keeps arguments alive until the stream has run the work.
 *
 * Errors: each call returns an ohm_status.  Argument and layout checks run on
 * the host before any launch and leave device memory untouched; the message
 * of the last failure of the calling thread is returned by ohm_last_error().
 */
#ifndef OHM_H
#define OHM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OHM_BLOCK 8
#define OHM_MAX_LEVELS 8

typedef enum {
    OHM_OK = 0,
    OHM_ERR_ARG = 1,        /* a null pointer, a bad size or enum value        */
    OHM_ERR_LAYOUT = 2,     /* blocks outside the box, duplicates, bad nesting */
    OHM_ERR_NOMEM = 3,      /* workspace too small / host allocation failed    */
    OHM_ERR_HIP = 4,        /* a HIP runtime call failed                        */
    OHM_ERR_NOCONV = 5,     /* max_iters reached before the tolerance          */
    OHM_ERR_NONFINITE = 6   /* a residual norm is NaN or infinite              */
} ohm_status;

typedef enum { OHM_F64 = 0, OHM_F32 = 1 } ohm_dtype;

typedef struct ohm_hier ohm_hier;

/* One independent periodic problem. */
typedef struct {
    int32_t nlevels;                          /* 1..OHM_MAX_LEVELS                     */
    int32_t base_blocks[3];                   /* level-0 box = 8*base_blocks[d] cells  */
    double dx0;                               /* level-0 cell width (cubic cells)      */
    int32_t nblocks[OHM_MAX_LEVELS];          /* blocks on each level                  */
    const int32_t *block_ijk[OHM_MAX_LEVELS]; /* host int32[nblocks][3]: block coords in
                                                 8-cell units of that level; level 0
                                                 must list every block of the box      */
} ohm_problem_desc;

/*
 * Build a handle for `nprob` problems.  Checks on the host that blocks lie in
 * the box, are unique, level 0 tiles the box and that each level l >= 1 is
 * properly nested: every cell within one level-(l-1) cell of a level-l block
 * (or of the 8^3 ghost block next to it) belongs to a level-(l-1) block.
 * Uploads the block tables with blocking copies on `stream`.
 * Returns OHM_ERR_LAYOUT for a bad hierarchy, OHM_ERR_ARG for bad arguments.
 */
ohm_status ohm_hier_create(const ohm_problem_desc *probs, int32_t nprob, hipStream_t stream,
                           ohm_hier **out);
ohm_status ohm_hier_destroy(ohm_hier *h);

/* Device bytes the handle itself holds: its block tables and reduction
 * scratch, plus the per-problem coefficient slots and the coarsest-grid
 * inverses that its first calls allocate (caller memory -- fields and the
 * step's workspace -- is not included). */
ohm_status ohm_hier_device_bytes(const ohm_hier *h, size_t *bytes);

/* Totals over all problems at `level` (>= 0: AMR level, < 0: multigrid level):
 * *nblocks (0 for level < 0), *ncells, and *nghost = coarse-fine ghost blocks. */
ohm_status ohm_hier_level_info(const ohm_hier *h, int32_t level, int64_t *nblocks,
                               int64_t *ncells, int64_t *nghost);
/* Per-problem placement at `level`: first cell of the problem inside a field of
 * that level (*cell_offset; -1 if the problem lacks the level) and, for levels
 * < 0, the dense grid size dims[3] (x, y, z).  Also the deepest multigrid level
 * of the problem (*min_level <= 0).  On levels < 0 every problem starts on a
 * 64-cell boundary; the cells between problems are unused. */
ohm_status ohm_hier_problem_info(const ohm_hier *h, int32_t prob, int32_t level,
                                 int64_t *cell_offset, int32_t dims[3], int32_t *min_level);

const char *ohm_last_error(void);

/*
 * Coarse-fine ghost fill (AMR levels >= 1).  Every ghost block of `level` --
 * an 8^3 block position next to a level block across a face, an edge or (where
 * the coarse cells its interpolation needs exist) a corner, but not part of
 * the level --
 * receives the cell-centred trilinear interpolant (27/9/3/1 over 64) of the
 * level-(level-1) field `coarse`.  The paper leaves its coarse-fine
 * interpolation unstated; this is the library's reading.
 *   coarse : T[ncomp][nblocks(level-1)][512]
 *   ghost  : T[ncomp][nghost(level)][512]   (output)
 * ncomp is 1 (resistivity) or 3.  A level without ghost blocks is a no-op.
 */
ohm_status ohm_fill_ghosts(ohm_hier *h, int32_t level, const void *coarse, void *ghost,
                           int32_t ncomp, ohm_dtype dtype, hipStream_t stream);

/*
 * Operator apply, eqs. (8)-(13):  out = B + coef[p] * div F(B)  on every cell
 * of `level` (covered cells included).  With coef = lambda dt this is L B;
 * with coef = -(1 - lambda) dt and B = b it is the source S of eq. (14).
 *   B, out : T[3][...] at `level`;  eta : T[1][...] at `level`;
 *   B_ghost, eta_ghost : ghost blocks of `level` filled by ohm_fill_ghosts
 *            (may be NULL when the level has no ghost blocks);
 *   coef   : host double[nprob].
 * `out` must not alias `B`.
 */
ohm_status ohm_apply(ohm_hier *h, int32_t level, const void *B, const void *B_ghost,
                     const void *eta, const void *eta_ghost, const double *coef, void *out,
                     ohm_dtype dtype, hipStream_t stream);

/*
 * Residual, eq. (20):  R = S - (B + lam_dt[p] div F(B))  on every cell of
 * `level`, written to R unless R is NULL.  If `norms` is not NULL it receives
 * (host double[nprob][3][2]) the sum of R_c^2 and max |R_c| per problem and
 * component; the call then synchronises `stream`.
 */
ohm_status ohm_residual(ohm_hier *h, int32_t level, const void *B, const void *B_ghost,
                        const void *S, const void *eta, const void *eta_ghost,
                        const double *lam_dt, void *R, double *norms, ohm_dtype dtype,
                        hipStream_t stream);

/*
 * ohm_residual for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc): the same
 * residual R (when R is not NULL) and the same norms, with every scratch
 * buffer in one static device array of 4 MiB per device, which the library
 * holds until the process ends.  Differences from ohm_residual:
 *   norms  : DEVICE double[nprob][3][2] (sum R_c^2, max |R_c|), written
 *            asynchronously on `stream`; the call never synchronises;
 *   lam_dt : host double[nprob], read when the call enqueues its work and
 *            passed to the device as kernel arguments (so is the block range
 *            of each problem): nothing is copied from host memory later, and
 *            a graph captured from the call replays the values it was given.
 * Returns OHM_ERR_NOMEM, before any launch, when the level needs more scratch
 * than the array holds: 48 bytes per block of `level` plus about 72 bytes per
 * problem with norms (about 87,000 blocks, 4.4e7 cells, for one problem).
 * Calls on one device share the array and keep the last call's contents:
 * calls that overlap on one device (several streams or host threads) race.
 * Nothing in the array needs to start at zero.
 */
ohm_status ohm_residual_noalloc(ohm_hier *h, int32_t level, const void *B, const void *B_ghost,
                                const void *S, const void *eta, const void *eta_ghost,
                                const double *lam_dt, void *R, double *norms, ohm_dtype dtype,
                                hipStream_t stream);

/*
 * Red-black smoother, eq. (19) with alpha of eqs. (21)-(23): `nsweeps` sweeps,
 * each a red half-sweep ((i+j+k) even in level-global cell indices) then a
 * black one.  All cells of a colour update together from the state at the
 * start of the half-sweep: B_c += R_c / (1 + alpha_c).  Ghost values are held
 * fixed.  `tmp` is caller scratch of the size of B; B holds the result.  On
 * levels where each of the 26 neighbour positions of every block is a level
 * block or a ghost block (all levels, unless some corner ghost would need
 * coarse cells that do not exist) and whose field and ghost arrays are at
 * most 4 GiB per component, one launch performs a whole sweep; it needs B, eta
 * and the ghost arrays aligned to 2 elements (OHM_ERR_ARG otherwise).  Other
 * levels take one launch per colour.
 * ordering: 0 = the paper's red-black; 1 = four colour classes
 * ((i+j) mod 2) + 2 ((j+k) mod 2), updated in that order with the same
 * update.  No two cells of a class share a stencil term, so on grids of even
 * extent a four-class sweep is an exact Gauss-Seidel sweep (red-black is a
 * Jacobi step inside each colour: the in-plane edge terms join same-colour
 * cells).  It takes four launches per sweep.  Other values: OHM_ERR_ARG.
 */
ohm_status ohm_smooth(ohm_hier *h, int32_t level, void *B, const void *B_ghost, const void *S,
                      const void *eta, const void *eta_ghost, const double *lam_dt,
                      int32_t nsweeps, int32_t ordering, void *tmp, ohm_dtype dtype, hipStream_t stream);

/*
 * Averaging restriction (section 2.2): each cell of level fine_level-1 that
 * lies under a fine_level block (all cells when fine_level <= 0) becomes the
 * mean of its 8 children; other coarse cells are left unchanged.
 *   fine : T[ncomp][...] at fine_level;  coarse : T[ncomp][...] at fine_level-1.
 */
ohm_status ohm_restrict(ohm_hier *h, int32_t fine_level, const void *fine, void *coarse,
                        int32_t ncomp, ohm_dtype dtype, hipStream_t stream);

/*
 * Trilinear prolongation (section 2.2, read as cell-centred trilinear, 27/9/3/1
 * over 64) from coarse_level to coarse_level+1, added to `fine`
 * (accumulate = 1) or written over it (accumulate = 0).  For coarse_level >= 0
 * the coarse neighbours of every fine block must be coarse blocks (nesting).
 */
ohm_status ohm_prolong(ohm_hier *h, int32_t coarse_level, const void *coarse, void *fine,
                       int32_t ncomp, int32_t accumulate, ohm_dtype dtype, hipStream_t stream);

/*
 * Refluxing (section 4): on every face between a leaf cell of `level` and a
 * cell covered by level+1, replace the coarse flux in `out` (the result of
 * ohm_apply with the same coef) by the mean of the 4 fine fluxes on that face,
 * i.e. out += coef * (F_fine_mean - F_coarse) * (+-1/h).  The fine fluxes use
 * the level+1 field with its ghost blocks.  Covered cells of `out` are set to
 * zero when zero_covered is 1.
 */
ohm_status ohm_reflux(ohm_hier *h, int32_t level, const void *B_coarse, const void *eta_coarse,
                      const void *B_fine, const void *B_fine_ghost, const void *eta_fine,
                      const void *eta_fine_ghost, const double *coef, void *out,
                      int32_t zero_covered, ohm_dtype dtype, hipStream_t stream);

/* Options of one Crank-Nicolson step. */
typedef struct {
    double lambda;        /* 0.5 = Crank-Nicolson (eq. 7); 1 = backward Euler    */
    double rtol;          /* stop when |S - L B|_2 <= rtol |S|_2 (composite leaf cells) */
    int32_t max_iters;    /* outer iterations                                       */
    int32_t nu_pre;       /* smoothing sweeps before / after the coarse correction */
    int32_t nu_post;
    int32_t n_vcycles;    /* V-cycles per multigrid application (per level in FMG)  */
    int32_t cycle;        /* 0 = V-cycle, 1 = full multigrid                        */
    int32_t outer;        /* 0 = iterative multigrid of eqs. (16)-(18), 1 = BiCGStab */
    int32_t precision;    /* 0 = FP64 everywhere, 1 = FP32 multigrid inside FP64 outer */
    int32_t coarse_sweeps;/* sweeps on a coarsest grid too large for a dense solve  */
    int32_t nu_coarse;    /* sweeps before and after on the levels below the base grid
                             (0 = nu_pre / nu_post)                                  */
    int32_t graph;        /* 1 = replay the device work of a step's start and of
                             each outer iteration as captured HIP graphs (kept in
                             the handle while workspace, eta pointers and options
                             stay the same)                                         */
    int32_t ordering;     /* smoother ordering, as for ohm_smooth: 0 = red-black
                             (fused sweeps), 1 = four colour classes (one launch per
                             class on every level)                                  */
    /* Multigrid over the AMR levels (hierarchies with more than one level;
       section 2.2, Table 1).  A composite V-cycle smooths each AMR level from
       zero with zero coarse-fine ghosts, restricts its residual under its
       blocks and takes its refluxed face fluxes out of the coarser leaf
       residual, solves the base grid (cycle, n_vcycles, nu_pre, nu_post), then
       prolongs and post-smooths each AMR level with ghosts from the coarser
       correction.                                                           */
    int32_t amr_fmg;      /* 0 = amr_vcycles composite V-cycles per multigrid
                             application; 1 = full multigrid over the AMR levels:
                             the base grid alone on the restricted right-hand
                             side, then per finer level the interpolated
                             correction and amr_vcycles composite V-cycles     */
    int32_t amr_vcycles;  /* >= 1; Table 1 "FMG on AMR": 4                       */
    int32_t amr_mlat;     /* further composite V-cycles on all levels (Table 1
                             "MLAT-FAS on AMR": 2); every composite V-cycle after
                             the first of an application starts from the FP64
                             composite residual of the correction so far       */
    int32_t nu_amr;       /* sweeps before and after on AMR levels >= 1 (0 =
                             nu_pre / nu_post)                                   */
} ohm_cn_opts;

typedef struct {
    int32_t iters;        /* outer iterations taken                                 */
    int32_t mg_apps;      /* multigrid applications                                 */
    double rel_res;       /* |S - L B|_2 / |S|_2 at exit (FP64)                     */
    double max_res[3];    /* max |R_c| at exit                                      */
} ohm_cn_stats;

void ohm_cn_default_opts(ohm_cn_opts *opts);

/* Bytes of device workspace ohm_cn_step needs for this handle and options. */
ohm_status ohm_cn_workspace_size(const ohm_hier *h, const ohm_cn_opts *opts, size_t *bytes);

/*
 * One Crank-Nicolson step on every problem of the handle.
 *   B[l]   : double[3][nblocks(l)][512], in: B^n, out: B^{n+1} (l = 0..max nlevels-1)
 *   eta[l] : double[nblocks(l)][512]
 *   dt     : host double[nprob]
 *   workspace : device memory of at least ohm_cn_workspace_size bytes, 256-byte aligned
 *   stats  : host ohm_cn_stats[nprob] (may be NULL)
 * The norms that test convergence reach the host through a pinned buffer of
 * the handle.  With BiCGStab the host queues the iterations it expects from
 * the previous step on the same handle (and, from the expected count on, the
 * verification and the copy to B) before it synchronises `stream`; a problem
 * leaves the iteration on the device at the iteration that converges it, so
 * results do not depend on how far ahead the host queued.  The iteration of
 * eqs. (16)-(18) synchronises once after the initial residual and once per
 * iteration.  B is complete when the call returns.
 * Returns OHM_ERR_NOCONV if a problem reached max_iters (B then holds the last
 * iterate and stats are filled) and OHM_ERR_NONFINITE on a non-finite norm
 * (B then keeps its input values if the norm was that of the initial
 * residual or of a BiCGStab iteration).
 */
ohm_status ohm_cn_step(ohm_hier *h, void *const B[], const void *const eta[], const double *dt,
                       const ohm_cn_opts *opts, void *workspace, size_t ws_bytes,
                       ohm_cn_stats *stats, hipStream_t stream);

/*
 * Explicit comparison scheme of section 3.3: nsteps steps of size dt[p] of the
 * predictor-corrector (Heun) update with the same flux divergence as the
 * implicit operator (eqs. 8-11), on the composite leaf cells of every problem
 * (coarse-fine faces refluxed as in ohm_cn_step, covered cells set to the mean
 * of their children after each stage):
 *   B* = B - dt div F(B),   B <- B - dt/2 (div F(B) + div F(B*)).
 *   B[l], eta[l] : as for ohm_cn_step (FP64, device)
 *   dt     : host double[nprob], > 0.  Stability is the caller's: with constant
 *            eta the largest eigenvalue of the flux divergence is 8 eta / h^2
 *            and the scheme is stable exactly for dt <= h^2 / (4 eta); with
 *            variable eta keep dt below about h^2 / (4 eta_max) on the finest
 *            level.
 *   workspace : device memory of at least ohm_explicit_workspace_size bytes,
 *            256-byte aligned (the same layout as the Crank-Nicolson workspace)
 * Asynchronous except for a final synchronisation of `stream`.  Returns
 * OHM_ERR_ARG for bad arguments, OHM_ERR_NOMEM for a short workspace.
 */
ohm_status ohm_explicit_workspace_size(const ohm_hier *h, size_t *bytes);
ohm_status ohm_explicit_step(ohm_hier *h, void *const B[], const void *const eta[], const double *dt, int nsteps,
                             void *workspace, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* OHM_H */
