// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "ohm.h"

namespace ohm {

constexpr int NB = 8;          // cells per block edge
constexpr int NC = 512;        // cells per block
constexpr int NXCD = 8;        // MI355X compute dies: workgroups are dealt round-robin

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
ohm_status fail(ohm_status st, const char *fmt, ...);

#define OHM_HIP(call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::ohm::fail(OHM_ERR_HIP, "%s failed: %s (%s:%d)", #call,         \
                               hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

#define OHM_TRY(...)                                                                \
    do {                                                                            \
        ohm_status s_ = (__VA_ARGS__);                                              \
        if (s_ != OHM_OK) return s_;                                                \
    } while (0)

ohm_status check_launch(const char *what);

// serialises graph capture against handle creation/destruction (which touch the
// device outside any stream) when several host threads share the library
std::mutex &capture_mutex();

// ---------------------------------------------------------------------------
// device-side tables of one AMR level (all problems of a handle)
// ---------------------------------------------------------------------------
// Neighbour entry of a block: >= 0 index of a same-level block; <= -1 means the
// ghost block -1-entry; NBR_NONE means absent (only for corners whose
// interpolation would need missing coarse cells).
constexpr int NBR_NONE = -(1 << 30);

struct AmrLevelDev {
    int nb = 0;                // blocks
    int ng = 0;                // coarse-fine ghost blocks
    bool complete27 = false;   // every block has all 26 neighbours as level blocks
    bool fused = false;        // every neighbour entry is a level or a ghost block
    int *nbr = nullptr;        // [nb][27] neighbour entries, index (dx+1)+3(dy+1)+9(dz+1)
    int *prob = nullptr;       // [nb] problem of each block
    int *ijk = nullptr;        // [nb][3] block coordinates at this level
    int *parent = nullptr;     // [nb] level-1 block containing the block (level >= 1)
    int *octant = nullptr;     // [nb] octant of the parent the block fills (x + 2y + 4z)
    int *gparent = nullptr;    // [ng] level-1 block containing each ghost block
    int *goctant = nullptr;    // [ng] its octant
    int *gprob = nullptr;      // [ng] problem of the ghost block
    uint8_t *cov = nullptr;    // [nb] octants covered by level+1 blocks (bit x+2y+4z)
    double *inv_h2 = nullptr;  // [nprob] 1 / h^2 of this level per problem (0 if absent)
    double *inv_h = nullptr;   // [nprob] 1 / h
    int *dense_map = nullptr;  // level 0 only: [nb] cell offset of the block's 4^3 coarse
                               // cells inside the problem's first dense level (-1 level)
    // refluxing: coarse cells of this level with faces next to covered cells
    int nrf = 0;
    int *rf = nullptr;         // [nrf][RF_INTS]
    int *rff = nullptr;        // faces of the entries, entry-major, faces in order: 8 entry + face
    int *rfs = nullptr;        // [nrf] index of each entry's first face in rff
    int nrfw = 0;              // workgroups of the refluxing kernel
    int *rfw = nullptr;        // [nrfw][4]: first entry, entries, first face, faces
};
constexpr int RF_INTS = 16;      // block, cell, facemask, 6 x fine block, 6 x fine base cell, problem
constexpr int RF_WG_FACES = 96;  // faces per refluxing workgroup (10 fluxes each)

// Dense multigrid level (below level 0)
struct DenseProbDev {
    int nx, ny, nz;
    int active;                // 1 if the level is not the problem's coarsest
    long long off;             // first cell of the problem in a field of this level
    double inv_h2;             // 1 / h^2 of this level
};

struct DenseLevelDev {
    int ncells = 0;
    int ntile = 0;             // 256-cell tiles of problems that are not coarsest here
    int *tiles = nullptr;      // [ntile][2]: problem, first cell
    int ntile_all = 0;         // tiles of every problem present
    int *tiles_all = nullptr;
    // smoothing: 8^3 tiles (fused sweeps) of problems whose grid has even
    // edges (the last tile along an edge that is not a multiple of 8 wraps
    // around), 256-cell tiles (two half-sweeps) of the others;
    // "all" variants cover every problem present, the others the problems
    // that are not coarsest here
    int nftile = 0, nftile_all = 0, nptile = 0, nptile_all = 0;
    int *ftiles = nullptr, *ftiles_all = nullptr, *ptiles = nullptr, *ptiles_all = nullptr;
    DenseProbDev *probs = nullptr;   // [nprob] (nx = 0 if the problem lacks the level)
};

}  // namespace ohm

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
struct ohm_prob_host {
    int nlevels;
    int bb[3];
    double dx0;
    int min_level;                   // deepest multigrid level (<= -1)
    int dims[16][3];                 // dense dims per depth d = -level (d >= 1)
    long long boff[OHM_MAX_LEVELS];  // first block of the problem at each AMR level
    int nb[OHM_MAX_LEVELS];
    long long doff[16];              // first cell at each dense depth
    std::vector<int32_t> blocks[OHM_MAX_LEVELS];
};

struct ohm_hier {
    int nprob = 0;
    int nlev = 0;                    // max AMR levels
    int min_level = 0;               // most negative multigrid level
    std::vector<ohm_prob_host> probs;
    ohm::AmrLevelDev amr[OHM_MAX_LEVELS];
    std::vector<int> nb_host;        // blocks per AMR level
    std::vector<int> ng_host;        // ghosts per AMR level
    ohm::DenseLevelDev dense[16];    // index d = -level
    long long dense_cells[16] = {0};
    // host copies read by the step code (cn.hip)
    std::vector<std::vector<int>> blk_prob_host;  // per level
    // scratch for per-problem scalars uploaded by the primitives
    double *d_scal = nullptr;        // [4 * nprob]
    double *d_part = nullptr;        // reduction partials
    size_t part_cap = 0;
    double *d_norms = nullptr;       // [nprob * 6]
    size_t table_bytes = 0;          // device bytes of the tables and scratch above
    // pinned host copies of norms: [8 * nprob] of reductions (a step's
    // start: |r|^2, |S|^2 at [0, 2 nprob); the verifying true residual at
    // [2 nprob, 3 nprob); an iteration of eqs. 16-18 at [0, nprob)), then the
    // iteration ring [2 * ITER_SLOTS * nprob], then the final norms of a
    // step [6 * nprob]
    double *h_dots = nullptr;
    int bicg_pred = 0;               // iterations the last step's first BiCGStab pass took
    char *h_stage = nullptr;         // pinned staging of a step's host-built tables
    size_t stage_bytes = 0;
    hipEvent_t stage_ev = nullptr;   // recorded after the staged upload
    bool stage_live = false;
    // ring of device slots for per-problem coefficients passed by the host to
    // the primitive calls (slot reuse waits on the event of its last use)
    double *d_ring = nullptr;        // [RING][nprob]
    hipEvent_t ring_ev[64] = {};
    bool ring_live[64] = {};
    int ring_pos = 0;
    // captured outer iteration of ohm_cn_step, reused while its key matches
    // replayed graphs, one per kind (0: iteration of eqs. 16-18, 1: BiCGStab
    // iteration, 2: start of a step), each valid for its workspace, resistivity
    // pointers and options
    struct GraphSlot {
        hipGraphExec_t exec = nullptr;
        std::vector<const void *> key;
        std::vector<char> opts;
    } graphs[3];
    hipStream_t cap_stream = nullptr;    // capture stream (the null stream cannot be captured)
    // solver state cache
    double *d_coarse_inv = nullptr;  // per-problem dense inverse of the coarsest grid
    double *d_coarse_eta = nullptr;  // coarsest resistivity each inverse was built from
    int *d_coarse_flags = nullptr;   // rebuild flags / forced rebuilds per job
    std::vector<long long> cinv_off; // element offset per problem, -1 if none
    std::vector<int> cinv_n;         // unknowns per problem
    std::vector<double> cinv_lamdt;  // lam_dt the inverse was built for
    std::vector<int> cinv_prec;
};

namespace ohm {

// launchers implemented in the kernel translation units ----------------------
enum { MODE_APPLY = 0, MODE_RESID = 1, MODE_SMOOTH = 2, MODE_RESID_RESTRICT = 3 };

// Colour classes of the smoother's orderings, in level-global cell indices
// (block-local indices have the same parities, block origins being multiples
// of 8).  colour 0 / 1: red / black of eq. (19), (i + j + k) mod 2; same-colour
// cells meet in the stencil's in-plane edge terms, so an update of one colour
// is a Jacobi step inside it.  colour 2 + m, m = 0..3: the four classes
// ((i + j) mod 2) + 2 ((j + k) mod 2), which give each of the 18 stencil
// neighbours of a cell (6 faces, 12 in-plane edges) another class than the
// cell's, so that on grids of even extent four class updates are one exact
// Gauss-Seidel sweep.
__device__ __forceinline__ bool in_colour(int i, int j, int k, int colour)
{
    return colour < 2 ? ((i + j + k) & 1) == colour : (((i + j) & 1) | (((j + k) & 1) << 1)) == colour - 2;
}

// Optional work fused into the block stencil kernel.  MODE_APPLY with ndot > 0
// also writes per-block partial dot products of the output with dot_y[q]
// (nullptr: with the output itself) to dot_part[block][ndot], summed in the
// same order as the stand-alone dot kernel.
struct StencilDots {
    const double *dot_y[2];
    int ndot;
    double *dot_part;
};

template <typename T>
ohm_status launch_blk_stencil(const ohm_hier *h, int level, int mode, const T *B, const T *Bg,
                              long long cs, long long gcs, const T *S, const T *eta, const T *etag,
                              const double *coef_dev, T *out, int colour, double *partials,
                              const uint8_t *cov_zero, const int *active, hipStream_t s,
                              StencilDots dots = StencilDots{{nullptr, nullptr}, 0, nullptr});
// level 0 -> first dense level: r = S - L e on the blocks, restricted (mean of
// the 8 children) straight into coarse; r itself is not stored
template <typename T>
ohm_status launch_resid_restrict_blk0(const ohm_hier *h, const T *B, const T *Bg, long long cs, long long gcs,
                                      const T *S, const T *eta, const T *etag, const double *coef_dev, T *coarse,
                                      long long ccs, const int *active, hipStream_t s);
// one fused red-black sweep B -> out (levels whose every neighbour entry is a
// level or ghost block; ghost values Bg / etag, held fixed, on levels that
// have ghosts); B == nullptr sweeps a zero input, with zero ghost values,
// without reading either; coarse != nullptr (level 0 only) sweeps
// B + P(coarse), the trilinear prolongation of the first dense level's field,
// without storing the corrected input; out64 (FP32 sweeps of a complete level
// with an input): the result is written as FP64 to out64 instead of out
template <typename T>
ohm_status launch_blk_sweep(const ohm_hier *h, int level, const T *B, long long cs, const T *S, const T *eta,
                            const double *coef_dev, T *out, const int *active, hipStream_t s,
                            const T *coarse = nullptr, long long ccs = 0, const T *Bg = nullptr, long long gcs = 0,
                            const T *etag = nullptr, double *out64 = nullptr);

template <typename T>
ohm_status launch_dense_stencil(const ohm_hier *h, int level, int mode, const T *B, const T *S,
                                const T *eta, const double *coef_dev, T *out, int colour,
                                bool coarsest_too, const int *active, hipStream_t s);

template <typename T>
ohm_status launch_restrict(const ohm_hier *h, int fine_level, const T *fine, long long fcs,
                           T *coarse, long long ccs, int ncomp, const int *active, hipStream_t s);
template <typename T>
ohm_status launch_prolong(const ohm_hier *h, int coarse_level, const T *coarse, long long ccs,
                          T *fine, long long fcs, int ncomp, int accumulate, const int *active,
                          hipStream_t s);
template <typename T>
ohm_status launch_fill_ghosts(const ohm_hier *h, int level, const T *coarse, long long ccs,
                              T *ghost, long long gcs, int ncomp, const int *active, hipStream_t s);
// out += coef (F_fine mean - F_coarse) (+-1/h) on faces between leaf cells of
// `level` and covered cells; Bc == nullptr takes the coarse field as zero
template <typename T>
ohm_status launch_reflux(const ohm_hier *h, int level, const T *Bc, long long ccs, const T *etac,
                         const T *Bf, long long fcs, const T *Bfg, long long fgcs, const T *etaf,
                         const T *etafg, const double *coef_dev, T *out, const int *active,
                         hipStream_t s);
template <typename T>
ohm_status launch_zero_covered(const ohm_hier *h, int level, T *out, long long cs, int ncomp,
                               hipStream_t s);

// per-problem reduction of per-block partials [block][k] into out[nprob][k]:
// range_dev holds [nprob][nrange][2] block ranges; quantities q < ksum are summed,
// the others maxed
ohm_status launch_reduce_problem(int nprob, int nrange, const long long *range_dev, const double *part, int k,
                                 int ksum, double *out, hipStream_t s);
template <typename T>
ohm_status launch_restrict_blk(const ohm_hier *h, int fine_level, const T *fine, long long fcs, T *coarse,
                               long long ccs, int ncomp, const int *active, hipStream_t s);
template <typename T>
// coarse_level -1 (first dense level -> level 0) may write base + P(coarse)
// into fine (base != fine) instead of accumulating in place
ohm_status launch_prolong_blk(const ohm_hier *h, int coarse_level, const T *coarse, long long ccs, T *fine,
                              long long fcs, int ncomp, int accumulate, const int *active, hipStream_t s,
                              const T *base = nullptr);

// dense multigrid levels (k_dense.hip)
// nsweeps fused or two-pass sweeps; the result is left in B, or, when `last`
// is given, wherever the fused sweeps end (B or tmp, returned in *last).
// flags: SMOOTH_ZERO: the input is zero and is not read; SMOOTH_FROM_TMP: the
// input is in tmp rather than B.  Sweep parities are arranged so that the
// fused tiles need no final copy when the count allows it.  coarse: the first
// sweep adds the trilinear prolongation of the next coarser level's field as
// it loads (coarse and last need a level of whole tiles, an input and a sweep).
// ordering 1: four-colour sweeps (four class launches each, see in_colour)
// instead of red-black; coarse and last are then not accepted.
enum { SMOOTH_ZERO = 1, SMOOTH_FROM_TMP = 2 };
template <typename T>
ohm_status launch_dense_smooth(const ohm_hier *h, int level, T *B, T *tmp, const T *S, const T *eta,
                               const double *coef_dev, int nsweeps, bool all, const int *active, hipStream_t s,
                               int flags = 0, const T *coarse = nullptr, T **last = nullptr, int ordering = 0);
// dense level -> next coarser: coarse = restriction of S - L B; res is scratch
// for handles where some continuing problem is not made of 8^3 tiles
template <typename T>
ohm_status launch_dense_resid_restrict(const ohm_hier *h, int level, const T *B, const T *S, const T *eta,
                                       const double *coef_dev, T *res, T *coarse, const int *active, hipStream_t s);
template <typename T>
ohm_status launch_dense_restrict(const ohm_hier *h, int fine_level, const T *fine, T *coarse, int ncomp,
                                 const int *active, hipStream_t s);
template <typename T>
ohm_status launch_dense_prolong(const ohm_hier *h, int coarse_level, const T *coarse, T *fine, int ncomp,
                                int accumulate, const int *active, hipStream_t s, const T *base = nullptr);
ohm_status coarse_sizes(const ohm_hier *h, size_t *inv_elems, size_t *aug_elems);
size_t coarse_job_bytes();
// Coarsest grids with at most 768 unknowns take a dense inverse kept in the
// handle.  coarse_plan fills, on the host, the job table of a step (per depth
// d, the jobs at slots d * nprob ...) and a force flag per job (lam_dt differs
// from the one the inverse was built for), and records the new lam_dt;
// launch_coarse_build then rebuilds, from the uploaded tables, every inverse
// that is forced or whose coarsest resistivity (eta_dense[d], FP64) changed.
// Scratch `aug` holds sum 2 n3^2 doubles.
void coarse_plan(ohm_hier *h, const double *lam_dt_host, void *jobs_host, int *force_host, int *njobs);
ohm_status ensure_coarse_storage(ohm_hier *h);   // the handle's inverse storage (before any capture)
size_t coarse_storage_bytes(const ohm_hier *h);  // device bytes ensure_coarse_storage allocates
ohm_status launch_coarse_build(ohm_hier *h, const double *const *eta_dense, const void *jobs_dev,
                               const int *force_dev, const int *njobs, double *aug, hipStream_t s);
template <typename T>
ohm_status launch_coarse_apply(const ohm_hier *h, int depth, const void *jobs_dev, int njobs, const double *inv,
                               const T *r, T *e, const int *active, hipStream_t s);

// vector kernels (k_vec.hip)
template <typename T>
ohm_status vfill(T *a, long long n, T v, hipStream_t s);
template <typename S, typename D>
ohm_status vconvert(const S *a, D *b, long long n, hipStream_t s);
template <typename S, typename D>
ohm_status vcopy_level(const S *a, long long acs, D *b, long long bcs, long long n, int ncomp, hipStream_t s,
                       const int *hold = nullptr);
ohm_status vdot(int nblk, const int *prob_of, const int *active, long long cs, const double *const *x,
                const double *const *y, int nq, double *part, hipStream_t s, double *copy = nullptr);
ohm_status vnorms(int nblk, const int *prob_of, const int *active, long long cs, const double *x, double *part,
                  hipStream_t s);
// p = r + beta (p - omega v) and s = r - alpha v per problem; c32 / c64, when
// given, also receive the result in FP32 / FP64 (the multigrid cycle's input)
ohm_status vbicg_p(int nblk, const int *prob_of, const int *active, long long cs, const double *scal,
                   const double *r, const double *v, double *p, hipStream_t s, float *c32 = nullptr,
                   double *c64 = nullptr);
ohm_status vbicg_s(int nblk, const int *prob_of, const int *active, long long cs, const double *scal,
                   const double *r, const double *v, double *sv, hipStream_t s, float *c32 = nullptr,
                   double *c64 = nullptr);
ohm_status vbicg_xr(int nblk, const int *prob_of, const int *active, long long cs, const double *scal, double *x,
                    const double *ph, const double *sh, const double *sv, const double *t, double *r,
                    const double *rhat, double *part, hipStream_t s);
// Record of the residual norms of consecutive BiCGStab iterations, so that the
// host can queue several iterations before it reads them: iteration j since
// the last restart stores {(r, r), (rhat, r)} of problem p at
// buf[2 (nprob (j mod ITER_SLOTS) + p)], and a problem whose (r, r) is not
// above tol2[p] (NaN included) leaves the active set (flags[p] = 0), so the
// iterations queued behind it skip it; a non-finite (r, r) of an active
// problem also sets *hold, which turns the copy of the result to the user's
// fields into a no-op (a step that fails leaves them as they were).
constexpr int ITER_SLOTS = 8;
struct IterRing {
    double *buf = nullptr;
    int *flags = nullptr;
    const double *tol2 = nullptr;
    int *hold = nullptr;
};
// per-problem sums of k <= 4 block partials into out[p][k], then the BiCGStab
// scalar update `stage` (< 0: none) for the active problems; stage 0 (restart)
// also resets every problem's iteration count, and stage 4 (end of an
// iteration) with ring.buf set records the norms in the ring as above
ohm_status launch_reduce_scal(int nprob, int nrange, const long long *range_dev, const double *part, int k,
                              double *out, int stage, const int *active, double *scal, hipStream_t s,
                              IterRing ring = IterRing());
// tol2[p] = rtol^2 max(|S|^2, 1e-300) from dots[2 p + 1] = |S|^2, and problems
// whose initial |r|^2 = dots[2 p] is not above it (NaN included) leave the
// active set; a non-finite initial |r|^2 sets *hold (see IterRing)
ohm_status launch_conv_init(int nprob, const double *dots, double rtol, double *tol2, int *active, int *hold,
                            hipStream_t s);
ohm_status vmean2(int nblk, const int *prob_of, const int *active, long long cs, double *x, const double *y,
                  hipStream_t s);
ohm_status vaxpy1(int nblk, const int *prob_of, const int *active, long long cs, double *x, const double *y,
                  hipStream_t s);
int scal_stride();

}  // namespace ohm
