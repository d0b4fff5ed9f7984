// One Crank-Nicolson step (eq. 7) on every problem of a handle.
//
// Outer iteration in FP64 on the composite leaf cells of the AMR hierarchy:
// either the iterative use of multigrid of eqs. (16)-(18) or BiCGStab, with a
// multigrid cycle as the (right) preconditioner.  The cycle runs in FP64 or,
// in mixed precision, in FP32 with the FP64 residual, update and coarsest
// solve around it.  Cycle: on AMR levels a coarse-grid-correction sweep over
// the levels (smooth on each level with coarse-fine ghosts, restrict the level
// residual under the finer blocks), then a V-cycle or full multigrid on the
// base grid and its coarsenings, with a dense FP64 solve on the coarsest grid.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

using namespace ohm;

namespace {

inline size_t al(size_t b) { return (b + 255) & ~size_t(255); }

struct Plan {
    int T32 = 0;                // 1: FP32 multigrid
    long long NBt = 0, NGt = 0; // blocks / ghost blocks over all AMR levels
    long long LB[OHM_MAX_LEVELS] = {0}, LG[OHM_MAX_LEVELS] = {0};
    size_t total = 0;
    // byte offsets
    size_t x, r, rhat, p, v, s, t, ph, sh, S, og, oeg;
    size_t rhs, e, tmp, res, mg_g, eta_t, eta_tg;
    size_t d_rhs[16], d_e[16], d_tmp[16], d_res[16], d_eta[16], d_eta64[16];
    size_t inv, aug, jobs, force, part, dots, scal, ranges, mlprob, active, cmask, coefs;
    size_t ring, tol2;          // norms of queued BiCGStab iterations, convergence thresholds
    size_t hold;                // set on the device when a norm is non-finite: no copy out
    size_t rf;                  // FMG over AMR levels: right-hand side restricted under finer blocks
    size_t inv_elems = 0, aug_elems = 0;
};

Plan make_plan(const ohm_hier *h, const ohm_cn_opts *o)
{
    Plan P;
    P.T32 = o->precision == 1;
    for (int l = 0; l < h->nlev; ++l) {
        P.LB[l] = P.NBt;
        P.LG[l] = P.NGt;
        P.NBt += h->nb_host[l];
        P.NGt += h->ng_host[l];
    }
    const size_t tb = P.T32 ? 4 : 8;
    const size_t V = 3 * (size_t)P.NBt * NC, G = 3 * (size_t)P.NGt * NC;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o_ = off;
        off += al(bytes);
        return o_;
    };
    P.x = take(8 * V);
    P.r = take(8 * V);
    P.rhat = take(8 * V);
    P.p = take(8 * V);
    P.v = take(8 * V);
    P.s = take(8 * V);
    P.t = take(8 * V);
    P.ph = take(8 * V);
    P.sh = take(8 * V);
    P.S = take(8 * V);
    P.rf = take(o->amr_fmg && h->nlev > 1 ? 8 * V : 8);
    P.og = take(8 * G + 8);
    P.oeg = take(8 * G / 3 + 8);
    P.rhs = take(tb * V);
    P.e = take(tb * V);
    P.tmp = take(tb * V);
    P.res = take(tb * V);
    P.mg_g = take(tb * G + 8);
    P.eta_t = take(P.T32 ? tb * V / 3 : 8);
    P.eta_tg = take(P.T32 ? tb * G / 3 + 8 : 8);
    for (int d = 1; d <= -h->min_level; ++d) {
        const size_t nc = (size_t)h->dense_cells[d];
        P.d_rhs[d] = take(tb * 3 * nc);
        P.d_e[d] = take(tb * 3 * nc);
        P.d_tmp[d] = take(tb * 3 * nc);
        P.d_res[d] = take(tb * 3 * nc);
        P.d_eta64[d] = take(8 * nc);
        // an FP64 cycle reads the FP64 resistivity itself
        P.d_eta[d] = P.T32 ? take(tb * nc) : P.d_eta64[d];
    }
    coarse_sizes(h, &P.inv_elems, &P.aug_elems);
    P.inv = take(8 * P.inv_elems + 8);
    P.aug = take(8 * P.aug_elems + 8);
    P.part = take(8 * (size_t)P.NBt * 8);
    P.dots = take(8 * (size_t)h->nprob * 8);
    P.scal = take(8 * (size_t)h->nprob * scal_stride());
    P.ring = take(8 * (size_t)h->nprob * 2 * ITER_SLOTS);
    P.tol2 = take(8 * (size_t)h->nprob);
    // tables the host builds each step, contiguous from jobs to coefs (one
    // staged upload): coarse jobs and force flags per depth, block ranges
    // per problem and level, block -> problem, active flags, coarse masks,
    // coefficients
    P.jobs = take(coarse_job_bytes() * (size_t)h->nprob * 17 + 8);
    P.force = take(4 * (size_t)h->nprob * 17);
    P.ranges = take(8 * (size_t)h->nprob * OHM_MAX_LEVELS * 2);
    P.mlprob = take(4 * (size_t)P.NBt);
    P.active = take(4 * (size_t)h->nprob);
    P.cmask = take(4 * (size_t)h->nprob * 17);
    P.hold = take(4);
    P.coefs = take(8 * (size_t)h->nprob * 4);
    P.total = off;
    return P;
}

bool valid_opts(const ohm_cn_opts *o)
{
    return o && o->lambda > 0.0 && o->lambda <= 1.0 && o->rtol > 0.0 && o->max_iters >= 1 && o->nu_pre >= 0 &&
           o->nu_post >= 0 && o->nu_pre + o->nu_post >= 1 && o->n_vcycles >= 1 && (o->cycle == 0 || o->cycle == 1) &&
           (o->outer == 0 || o->outer == 1) && (o->precision == 0 || o->precision == 1) && o->coarse_sweeps >= 0 &&
           o->nu_coarse >= 0 && (o->graph == 0 || o->graph == 1) && (o->ordering == 0 || o->ordering == 1) &&
           (o->amr_fmg == 0 || o->amr_fmg == 1) && o->amr_vcycles >= 1 && o->amr_mlat >= 0 && o->nu_amr >= 0;
}

// ---------------------------------------------------------------------------
template <typename T>
struct Solver {
    ohm_hier *h;
    const ohm_cn_opts *o;
    Plan P;
    char *ws;
    hipStream_t st;
    void *const *Buser;
    const void *const *Euser;
    // derived pointers
    const int *mlprob, *active;
    int *active_mut;
    double *lam_dt, *src_coef, *neg_lam_dt;
    long long VN, GN;            // component strides of multi-level vectors / ghosts
    std::vector<int> njobs;      // coarse jobs per depth
    std::vector<long long> ranges_host;

    template <typename U> U *at(size_t off) const { return (U *)(ws + off); }
    double *vec(size_t off, int l) const { return at<double>(off) + P.LB[l] * NC; }
    T *mg(size_t off, int l) const
    {
        T *base = (off == P.rhs && rhs_b) ? rhs_b : (off == P.e && e_b) ? e_b : at<T>(off);
        return base + P.LB[l] * NC;
    }
    T *rhs_b = nullptr, *e_b = nullptr;   // multigrid right-hand side / correction of this cycle
    const double *eta64(int l) const { return (const double *)Euser[l]; }
    const T *etaT(int l) const
    {
        if (P.T32) return at<T>(P.eta_t) + P.LB[l] * NC;
        return (const T *)Euser[l];
    }
    const double *etag64(int l) const { return at<double>(P.oeg) + P.LG[l] * NC; }
    const T *etagT(int l) const { return P.T32 ? at<T>(P.eta_tg) + P.LG[l] * NC : (const T *)etag64(l); }
    int nlev() const { return h->nlev; }

    // ---- outer composite operator (FP64) --------------------------------------
    // y = L x (mode APPLY, coef) or y = S - L x (mode RESID) on leaf cells;
    // covered cells of y are zero.
    // top >= 0: the composite operator of levels 0..top only (level top is
    // then the finest: its cells under finer blocks are its own unknowns)
    ohm_status composite(size_t xo, size_t yo, int mode, const double *coef, const double *reflux_coef, size_t So,
                         int top = -1)
    {
        const int L = top >= 0 ? top + 1 : nlev();
        for (int l = L - 1; l >= 1; --l)
            OHM_TRY(launch_restrict_blk<double>(h, l, vec(xo, l), VN, vec(xo, l - 1), VN, 3, active, st));
        for (int l = 1; l < L; ++l)
            OHM_TRY(launch_fill_ghosts<double>(h, l, vec(xo, l - 1), VN, at<double>(P.og) + P.LG[l] * NC, GN, 3,
                                               active, st));
        for (int l = 0; l < L; ++l)
            OHM_TRY(launch_blk_stencil<double>(h, l, mode, vec(xo, l), at<double>(P.og) + P.LG[l] * NC, VN, GN,
                                               So ? vec(So, l) : nullptr, eta64(l), etag64(l), coef, vec(yo, l), 0,
                                               nullptr, (l + 1 < L) ? h->amr[l].cov : nullptr, active, st));
        for (int l = 0; l + 1 < L; ++l)
            OHM_TRY(launch_reflux<double>(h, l, vec(xo, l), VN, eta64(l), vec(xo, l + 1), VN,
                                          at<double>(P.og) + P.LG[l + 1] * NC, GN, eta64(l + 1), etag64(l + 1),
                                          reflux_coef, vec(yo, l), active, st));
        return OHM_OK;
    }

    // per-problem reductions of per-block partials over all AMR levels
    ohm_status reduce(int k, int ksum, double *out)
    {
        return launch_reduce_problem(h->nprob, nlev(), at<long long>(P.ranges), at<double>(P.part), k, ksum, out, st);
    }

    ohm_status dots(const double *const *x, const double *const *y, int nq, int stage = -1, double *copy = nullptr)
    {
        OHM_TRY(vdot((int)P.NBt, mlprob, active, VN, x, y, nq, at<double>(P.part), st, copy));
        return reduce_scal(nq, stage);
    }
    // per-problem sums of the nq partials into dots, then BiCGStab scalar
    // update `stage` (< 0: none), one launch
    ohm_status reduce_scal(int nq, int stage)
    {
        return launch_reduce_scal(h->nprob, nlev(), at<long long>(P.ranges), at<double>(P.part), nq,
                                  at<double>(P.dots), stage, active, at<double>(P.scal), st);
    }

    // y = L x (lam dt) followed by the per-problem dots (xs[q], ys[q]), where
    // every xs[q] or ys[q] is y itself or another vector.  One level: the dot
    // partials come out of the operator kernel (same summation order as the
    // dot kernel); AMR: the refluxed operator first, then the dot kernel.
    ohm_status apply_dots(size_t xo, size_t yo, const double *const *xs, const double *const *ys, int nq,
                          int stage = -1)
    {
        if (nlev() == 1) {
            const double *y = at<double>(yo);
            StencilDots sd{{nullptr, nullptr}, nq, at<double>(P.part)};
            for (int q = 0; q < nq; ++q) {
                const double *other = xs[q] == y ? ys[q] : xs[q];
                sd.dot_y[q] = other == y ? nullptr : other;
            }
            OHM_TRY(launch_blk_stencil<double>(h, 0, MODE_APPLY, vec(xo, 0), at<double>(P.og) + P.LG[0] * NC, VN,
                                               GN, nullptr, eta64(0), etag64(0), lam_dt, vec(yo, 0), 0, nullptr,
                                               nullptr, active, st, sd));
            return reduce_scal(nq, stage);
        }
        OHM_TRY(composite(xo, yo, MODE_APPLY, lam_dt, lam_dt, 0));
        return dots(xs, ys, nq, stage);
    }

    // ---- multigrid cycle (precision T) ----------------------------------------
    // n sweeps on block level l, result in e.  flags as for dense levels:
    // SMOOTH_ZERO (zero input, not read) or SMOOTH_FROM_TMP (input in tmp)
    // coarse (level 0 only): the first sweep reads e + P(coarse), the
    // prolonged correction from the first dense level, without storing it
    // out64_: when set, the level-0 post-smoothing of the coming V-cycle writes
    // its last sweep as FP64 there (the preconditioned vector) and sets wrote64_
    double *out64_ = nullptr;
    bool wrote64_ = false;

    // fused sweeps are red-black and address each field (and ghost) array of
    // the level with 32-bit byte offsets; the four-colour ordering, and levels
    // above 4 GiB per component, take one launch per colour class (coarse and
    // out64 are for fused sweeps only)
    bool fused_blk(int l) const
    {
        const AmrLevelDev &A = h->amr[l];
        const unsigned long long lim = 0xFFFFFFFFull, per = (unsigned long long)NC * sizeof(T);
        return A.fused && o->ordering == 0 && (unsigned long long)A.nb * per <= lim &&
               (A.complete27 || (unsigned long long)A.ng * per <= lim);
    }
    ohm_status smooth_blk(int l, int n, int flags = 0, const T *coarse = nullptr, double *out64 = nullptr)
    {
        const bool zero = flags & SMOOTH_ZERO, from_tmp = (flags & SMOOTH_FROM_TMP) && !zero;
        T *e = mg(P.e, l), *tmp = mg(P.tmp, l);
        T *cur = from_tmp ? tmp : e;
        const T *gB = at<T>(P.mg_g) + P.LG[l] * NC, *gE = etagT(l);
        if (coarse && !(fused_blk(l) && n > 0)) return fail(OHM_ERR_ARG, "fused coarse correction without fused sweeps");
        if (fused_blk(l) && n > 0) {
            // fused sweeps ping-pong e <-> tmp; a zero input is not read, so
            // the first sweep writes whichever buffer makes the last land in e
            bool used64 = false;
            for (int k = 0; k < n; ++k) {
                T *dst;
                if (k == 0 && zero) {
                    dst = (n & 1) ? e : tmp;
                    OHM_TRY(launch_blk_sweep<T>(h, l, nullptr, VN, mg(P.rhs, l), etaT(l), lam_dt, dst, active, st,
                                                nullptr, 0, nullptr, GN, gE));
                } else if (k == 0 && coarse) {
                    dst = cur == e ? tmp : e;
                    used64 = k == n - 1 && out64;
                    OHM_TRY(launch_blk_sweep<T>(h, l, cur, VN, mg(P.rhs, l), etaT(l), lam_dt, dst, active, st, coarse,
                                                h->dense_cells[1], nullptr, 0, nullptr, used64 ? out64 : nullptr));
                } else {
                    dst = cur == e ? tmp : e;
                    used64 = k == n - 1 && out64;
                    OHM_TRY(launch_blk_sweep<T>(h, l, cur, VN, mg(P.rhs, l), etaT(l), lam_dt, dst, active, st,
                                                nullptr, 0, gB, GN, gE, used64 ? out64 : nullptr));
                }
                cur = dst;
            }
            if (used64) {
                wrote64_ = true;   // the result is in out64; e is not needed any more
                return OHM_OK;
            }
        } else {
            // one launch per colour class (two red-black, four for the
            // four-colour ordering), each a full out-of-place pass: a sweep
            // returns to the buffer it started from
            if (zero) OHM_TRY(zero_level(P.e, l));
            T *oth = cur == e ? tmp : e;
            const int ncol = o->ordering ? 4 : 2, c0 = o->ordering ? 2 : 0;
            for (int k = 0; k < n; ++k)
                for (int c = 0; c < ncol; ++c)
                    OHM_TRY(launch_blk_stencil<T>(h, l, MODE_SMOOTH, (c & 1) ? oth : cur, gB, VN, GN, mg(P.rhs, l),
                                                  etaT(l), etagT(l), lam_dt, (c & 1) ? cur : oth, c0 + c, nullptr,
                                                  nullptr, active, st));
        }
        if (cur != e)
            for (int c = 0; c < 3; ++c)
                OHM_TRY(vconvert<T, T>(cur + c * VN, e + c * VN, (long long)h->nb_host[l] * NC, st));
        return OHM_OK;
    }
    ohm_status resid_blk(int l)
    {
        return launch_blk_stencil<T>(h, l, MODE_RESID, mg(P.e, l), at<T>(P.mg_g) + P.LG[l] * NC, VN, GN,
                                     mg(P.rhs, l), etaT(l), etagT(l), lam_dt, mg(P.res, l), 0, nullptr, nullptr,
                                     active, st);
    }
    T *dv(size_t const *arr, int d) const { return at<T>(arr[d]); }
    ohm_status smooth_dense(int d, int n, const int *filter, bool all, int flags = 0, const T *coarse = nullptr,
                            T **last = nullptr)
    {
        return launch_dense_smooth<T>(h, -d, dv(P.d_e, d), dv(P.d_tmp, d), dv(P.d_rhs, d), dv(P.d_eta, d), lam_dt, n,
                                      all, filter, st, flags, coarse, last, o->ordering);
    }
    // where each dense level's current correction is: its e buffer, or its
    // tmp buffer when the post-smoothing sweeps ended there (no copy back)
    T *ecur[17] = {};
    T *ecur_of(int d) const { return ecur[d] ? ecur[d] : dv(P.d_e, d); }
    // post-smoothing of dense level d may leave its result in tmp only when no
    // problem takes its coarsest solve there (that solve writes e)
    bool may_end_in_tmp(int d) const { return njobs[d] == 0 && !has_big[d]; }
    // coarsest grids at depth d, from a zero guess: dense inverse for small
    // grids, FP-T smoothing sweeps for the others; writes e_d of every problem
    // that bottoms out at depth d
    ohm_status coarsest(int d)
    {
        ecur[d] = dv(P.d_e, d);
        void *jobs = at<char>(P.jobs) + coarse_job_bytes() * (size_t)h->nprob * d;
        if (njobs[d] > 0)
            OHM_TRY(launch_coarse_apply<T>(h, d, jobs, njobs[d], h->d_coarse_inv, dv(P.d_rhs, d), dv(P.d_e, d),
                                           active, st));
        if (has_big[d])
            OHM_TRY(smooth_dense(d, o->coarse_sweeps, at<int>(P.cmask) + (size_t)h->nprob * d, true, SMOOTH_ZERO));
        return OHM_OK;
    }
    ohm_status zero_level(size_t off, int l)
    {
        for (int c = 0; c < 3; ++c) OHM_TRY(vfill<T>(mg(off, l) + c * VN, (long long)h->nb_host[l] * NC, T(0), st));
        return OHM_OK;
    }
    std::vector<int> has_big;

    // V-cycle on the base stack at level lev (0 or dense -d); e at lev holds
    // the initial guess, or zero_guess says it is zero (and e is not read).
    // An odd post-smoothing count on fused levels prolongs into tmp
    // (tmp = e + P e_coarse) so that the sweeps end in e without a copy.
    ohm_status vcycle_base(int lev, bool zero_guess)
    {
        const int nu1 = o->nu_pre, nu2 = o->nu_post;
        const int zf = zero_guess ? SMOOTH_ZERO : 0;
        if (lev == 0) {
            OHM_TRY(smooth_blk(0, nu1, zf));
            OHM_TRY(launch_resid_restrict_blk0<T>(h, mg(P.e, 0), at<T>(P.mg_g) + P.LG[0] * NC, VN, GN, mg(P.rhs, 0),
                                                  etaT(0), etagT(0), lam_dt, dv(P.d_rhs, 1), h->dense_cells[1],
                                                  active, st));
            OHM_TRY(down_dense(1));
            const T *e1 = ecur_of(1);
            const bool fz = h->amr[0].complete27 && fused_blk(0);
            if (fz && nu2 > 0 && !(nu2 & 1)) {
                // even count: the first sweep adds the correction as it loads
                OHM_TRY(smooth_blk(0, nu2, 0, e1, out64_));
            } else if ((nu2 & 1) && fz) {
                OHM_TRY(launch_prolong_blk<T>(h, -1, e1, h->dense_cells[1], mg(P.tmp, 0), VN, 3, 1, active, st,
                                              mg(P.e, 0)));
                OHM_TRY(smooth_blk(0, nu2, SMOOTH_FROM_TMP, nullptr, out64_));
            } else {
                OHM_TRY(launch_prolong_blk<T>(h, -1, e1, h->dense_cells[1], mg(P.e, 0), VN, 3, 1, active, st));
                OHM_TRY(smooth_blk(0, nu2));
            }
            return OHM_OK;
        }
        const int d = -lev;
        const int nuc1 = o->nu_coarse > 0 ? o->nu_coarse : nu1, nuc2 = o->nu_coarse > 0 ? o->nu_coarse : nu2;
        const int f1 = zero_guess ? SMOOTH_ZERO : (ecur_of(d) == dv(P.d_tmp, d) ? SMOOTH_FROM_TMP : 0);
        OHM_TRY(smooth_dense(d, nuc1, active, false, f1));
        ecur[d] = dv(P.d_e, d);
        OHM_TRY(launch_dense_resid_restrict<T>(h, -d, dv(P.d_e, d), dv(P.d_rhs, d), dv(P.d_eta, d), lam_dt,
                                               dv(P.d_res, d), dv(P.d_rhs, d + 1), active, st));
        OHM_TRY(down_dense(d + 1));
        const T *ec = ecur_of(d + 1);
        if (nuc2 > 0 && h->dense[d].nptile == 0 && o->ordering == 0 && (!(nuc2 & 1) || may_end_in_tmp(d))) {
            // the first sweep adds the prolonged coarser correction as it
            // loads; the result stays where the last sweep put it
            T *last = nullptr;
            OHM_TRY(smooth_dense(d, nuc2, active, false, 0, ec, &last));
            ecur[d] = last;
        } else if (nuc2 & 1) {
            OHM_TRY(launch_dense_prolong<T>(h, -(d + 1), ec, dv(P.d_tmp, d), 3, 1, active, st,
                                            (const T *)dv(P.d_e, d)));
            OHM_TRY(smooth_dense(d, nuc2, active, false, SMOOTH_FROM_TMP));
        } else {
            OHM_TRY(launch_dense_prolong<T>(h, -(d + 1), ec, dv(P.d_e, d), 3, 1, active, st));
            OHM_TRY(smooth_dense(d, nuc2, active, false));
        }
        return OHM_OK;
    }
    // enter dense depth d with its rhs set: coarsest solves for the problems
    // bottoming out here, a zero-guess V-cycle for the others (between them
    // every problem present at depth d has e_d written, so no fill is needed)
    ohm_status down_dense(int d)
    {
        OHM_TRY(coarsest(d));
        if (h->dense[d].ntile > 0) OHM_TRY(vcycle_base(-d, true));
        return OHM_OK;
    }

    ohm_status fmg_base()
    {
        // restrict the right-hand side down the base stack, solve the coarsest
        // grids, then interpolate upward with n_vcycles V-cycles per level
        OHM_TRY(launch_restrict_blk<T>(h, 0, mg(P.rhs, 0), VN, dv(P.d_rhs, 1), h->dense_cells[1], 3, active, st));
        const int D = -h->min_level;
        for (int d = 1; d < D; ++d)
            OHM_TRY(launch_dense_restrict<T>(h, -d, dv(P.d_rhs, d), dv(P.d_rhs, d + 1), 3, active, st));
        for (int d = 1; d <= D; ++d) OHM_TRY(vfill<T>(dv(P.d_e, d), 3 * h->dense_cells[d], T(0), st));
        for (int d = 1; d <= D; ++d) OHM_TRY(coarsest(d));
        for (int d = D - 1; d >= 1; --d) {
            if (h->dense[d].ntile == 0) continue;
            OHM_TRY(launch_dense_prolong<T>(h, -(d + 1), ecur_of(d + 1), dv(P.d_e, d), 3, 0, active, st));
            ecur[d] = dv(P.d_e, d);
            for (int v = 0; v < o->n_vcycles; ++v) OHM_TRY(vcycle_base(-d, false));
        }
        OHM_TRY(launch_prolong_blk<T>(h, -1, ecur_of(1), h->dense_cells[1], mg(P.e, 0), VN, 3, 0, active, st));
        double *const o64 = out64_;
        for (int v = 0; v < o->n_vcycles; ++v) {
            out64_ = v == o->n_vcycles - 1 ? o64 : nullptr;
            OHM_TRY(vcycle_base(0, false));
        }
        out64_ = nullptr;
        return OHM_OK;
    }

    // z = M(r): the multigrid cycle applied to an FP64 multi-level vector
    // FP64 single-level problems run the cycle directly on the Krylov vectors
    // (the cycle only reads r and only writes z); otherwise r is copied, in
    // the cycle's precision, into its right-hand side first
    bool cycle_aliases() const { return !P.T32 && nlev() == 1; }
    int nu_amr_pre() const { return o->nu_amr > 0 ? o->nu_amr : o->nu_pre; }
    int nu_amr_post() const { return o->nu_amr > 0 ? o->nu_amr : o->nu_post; }
    // more than one composite V-cycle per application, or FMG over the levels
    bool amr_general() const { return nlev() > 1 && (o->amr_fmg || o->amr_vcycles > 1 || o->amr_mlat > 0); }

    // the base-grid multigrid on rhs(0) -> e(0); o64: FP64 output of a single
    // level's last post-sweep (or null)
    ohm_status base_cycle(double *o64)
    {
        if (o->cycle == 1) {
            out64_ = o64;
            OHM_TRY(fmg_base());
        } else {
            for (int v = 0; v < o->n_vcycles; ++v) {
                out64_ = v == o->n_vcycles - 1 ? o64 : nullptr;
                OHM_TRY(vcycle_base(0, v == 0));
            }
        }
        out64_ = nullptr;
        return OHM_OK;
    }

    // one composite V-cycle from a zero correction on levels 0..top, for the
    // right-hand side in rhs (precision T, levels 0..top); the correction is
    // left in e.  AMR levels, finest first: smooth with zero coarse-fine
    // ghosts, restrict the level residual under the finer blocks, and take
    // the refluxed fluxes of the level's correction out of the residual of
    // the coarser leaf cells next to it (the coarser correction is still zero
    // there): the coarser level then solves the composite residual
    ohm_status amr_vcycle(int top, double *o64)
    {
        if (top >= 1 && P.NGt > 0) OHM_TRY(vfill<T>(at<T>(P.mg_g), 3 * P.NGt * NC, T(0), st));
        for (int l = top; l >= 1; --l) {
            OHM_TRY(smooth_blk(l, nu_amr_pre(), SMOOTH_ZERO));
            OHM_TRY(resid_blk(l));
            OHM_TRY(launch_restrict_blk<T>(h, l, mg(P.res, l), VN, mg(P.rhs, l - 1), VN, 3, active, st));
            OHM_TRY(launch_reflux<T>(h, l - 1, nullptr, VN, etaT(l - 1), mg(P.e, l), VN, at<T>(P.mg_g) + P.LG[l] * NC,
                                     GN, etaT(l), etagT(l), neg_lam_dt, mg(P.rhs, l - 1), active, st));
        }
        wrote64_ = false;
        OHM_TRY(base_cycle(o64));
        for (int l = 1; l <= top; ++l) {
            OHM_TRY(launch_prolong_blk<T>(h, l - 1, mg(P.e, l - 1), VN, mg(P.e, l), VN, 3, 1, active, st));
            OHM_TRY(launch_fill_ghosts<T>(h, l, mg(P.e, l - 1), VN, at<T>(P.mg_g) + P.LG[l] * NC, GN, 3, active, st));
            OHM_TRY(smooth_blk(l, nu_amr_post()));
        }
        return OHM_OK;
    }

    // levels 0..top of a multi-level vector: FP64 src -> precision-T dst
    // (per component, the levels are contiguous from block 0)
    template <typename S, typename D>
    ohm_status convert_upto(const S *src, D *dst, int top)
    {
        const long long n = (top + 1 < nlev() ? P.LB[top + 1] : P.NBt) * NC;
        for (int c = 0; c < 3; ++c) OHM_TRY(vconvert<S, D>(src + c * VN, dst + c * VN, n, st));
        return OHM_OK;
    }

    ohm_status precond(size_t ro, size_t zo, bool rhs_ready = false)
    {
        if (amr_general()) return precond_amr(ro, zo);
        const long long n = 3 * P.NBt * NC;
        const int L = nlev();
        const bool alias = cycle_aliases();
        if (alias) {
            rhs_b = (T *)at<double>(ro);
            e_b = (T *)at<double>(zo);
        } else {
            rhs_b = e_b = nullptr;
            if (!rhs_ready) OHM_TRY(vconvert<double, T>(at<double>(ro), at<T>(P.rhs), n, st));
        }
        // one FP32 level: the last post-sweep writes the FP64 result directly
        double *const o64 = (P.T32 && L == 1 && h->amr[0].complete27 && fused_blk(0) &&
                             (unsigned long long)h->amr[0].nb * NC * sizeof(double) <= 0xFFFFFFFFull)
                                ? at<double>(zo)
                                : nullptr;
        OHM_TRY(amr_vcycle(L - 1, o64));
        if (!alias && !wrote64_) OHM_TRY(vconvert<T, double>(at<T>(P.e), at<double>(zo), n, st));
        rhs_b = e_b = nullptr;
        return OHM_OK;
    }

    // several composite V-cycles per application, or FMG over the AMR levels
    // (section 2.2, Table 1): every composite V-cycle after the first takes
    // the FP64 composite residual of the correction z so far (levels 0..top)
    // as its right-hand side and adds its correction to z.  The vector t is
    // free during an application in both outer iterations.
    ohm_status precond_amr(size_t ro, size_t zo)
    {
        const int L = nlev();
        rhs_b = e_b = nullptr;
        double *z = at<double>(zo), *t = at<double>(P.t);
        OHM_TRY(vfill<double>(z, 3 * VN, 0.0, st));
        auto cycle = [&](int top, size_t so) -> ohm_status {
            OHM_TRY(composite(zo, P.t, MODE_RESID, lam_dt, neg_lam_dt, so, top));
            OHM_TRY(convert_upto<double, T>(t, at<T>(P.rhs), top));
            OHM_TRY(amr_vcycle(top, nullptr));
            OHM_TRY(convert_upto<T, double>(at<T>(P.e), t, top));
            const int nblk = (int)(top + 1 < L ? P.LB[top + 1] : P.NBt);
            return vaxpy1(nblk, mlprob, active, VN, z, t, st);
        };
        if (!o->amr_fmg) {
            for (int k = 0; k < o->amr_vcycles + o->amr_mlat; ++k) OHM_TRY(cycle(L - 1, ro));
            return OHM_OK;
        }
        // FMG: the right-hand side restricted under the finer blocks (finest
        // first), the base grid alone, then level by level
        double *rf = at<double>(P.rf);
        OHM_TRY(vconvert<double, double>(at<double>(ro), rf, 3 * VN, st));
        for (int l = L - 1; l >= 1; --l)
            OHM_TRY(launch_restrict_blk<double>(h, l, vec(P.rf, l), VN, vec(P.rf, l - 1), VN, 3, active, st));
        OHM_TRY(convert_upto<double, T>(rf, at<T>(P.rhs), 0));
        OHM_TRY(base_cycle(nullptr));
        OHM_TRY(convert_upto<T, double>(at<T>(P.e), z, 0));
        for (int top = 1; top < L; ++top) {
            OHM_TRY(launch_prolong_blk<double>(h, top - 1, vec(zo, top - 1), VN, vec(zo, top), VN, 3, 0, active, st));
            const int n = o->amr_vcycles + (top == L - 1 ? o->amr_mlat : 0);
            for (int k = 0; k < n; ++k) OHM_TRY(cycle(top, P.rf));
        }
        return OHM_OK;
    }

    // ---- setup ----------------------------------------------------------------
    // A step starts with setup_host (tables staged in pinned memory, host
    // state), copy_in (x = B) and start_device (everything on the device up to
    // the norms of the initial residual; one captured graph when graphs are
    // on).  multigrid = false: only what the explicit scheme needs (tables,
    // coefficients, coarse-fine ghosts of eta).
    ohm_status setup_host(const double *dt, bool multigrid = true)
    {
        const int np = h->nprob, L = nlev();
        VN = P.NBt * NC;
        GN = P.NGt * NC;
        // the step's tables, built on the host in pinned staging memory laid
        // out like the workspace region from jobs to coefs, then one upload
        const size_t tab0 = P.jobs, tab_bytes = P.coefs + 8 * (size_t)np * 4 - P.jobs;
        if (h->stage_live) OHM_HIP(hipEventSynchronize(h->stage_ev));   // the previous upload is done
        h->stage_live = false;
        if (h->stage_bytes < tab_bytes) {
            if (h->h_stage) OHM_HIP(hipHostFree(h->h_stage));
            h->h_stage = nullptr;
            h->stage_bytes = 0;
            OHM_HIP(hipHostMalloc((void **)&h->h_stage, tab_bytes, hipHostMallocDefault));
            h->stage_bytes = tab_bytes;
        }
        if (!h->stage_ev) OHM_HIP(hipEventCreateWithFlags(&h->stage_ev, hipEventDisableTiming));
        char *stg = h->h_stage;
        auto host = [&](size_t off) { return stg + (off - tab0); };
        // multi-level block -> problem, per-problem block ranges
        {
            int *mp = (int *)host(P.mlprob);
            for (int l = 0; l < L; ++l) mp = std::copy(h->blk_prob_host[l].begin(), h->blk_prob_host[l].end(), mp);
        }
        ranges_host.assign((size_t)np * L * 2, 0);
        for (int p = 0; p < np; ++p)
            for (int l = 0; l < L; ++l) {
                const ohm_prob_host &Q = h->probs[p];
                long long b0 = 0, b1 = 0;
                if (l < Q.nlevels) {
                    b0 = P.LB[l] + Q.boff[l];
                    b1 = b0 + Q.nb[l];
                }
                ranges_host[2 * ((size_t)p * L + l)] = b0;
                ranges_host[2 * ((size_t)p * L + l) + 1] = b1;
            }
        std::copy(ranges_host.begin(), ranges_host.end(), (long long *)host(P.ranges));
        std::vector<double> coefs(4 * (size_t)np);
        for (int p = 0; p < np; ++p) {
            if (!(dt[p] > 0.0) || !std::isfinite(dt[p])) return fail(OHM_ERR_ARG, "dt[%d] must be positive", p);
            coefs[p] = o->lambda * dt[p];
            coefs[np + p] = -(1.0 - o->lambda) * dt[p];
            coefs[2 * np + p] = -o->lambda * dt[p];
        }
        std::copy(coefs.begin(), coefs.end(), (double *)host(P.coefs));
        std::vector<int> ones(np, 1);
        std::copy(ones.begin(), ones.end(), (int *)host(P.active));
        *(int *)host(P.hold) = 0;
        // coarsest grids: a dense inverse (job tables, force flags) or, for
        // grids above 768 unknowns, smoothing sweeps (mask per depth)
        njobs.assign(17, 0);
        has_big.assign(17, 0);
        {
            int *cm = (int *)host(P.cmask);
            std::fill(cm, cm + (size_t)np * 17, 0);
            for (int p = 0; p < np; ++p) {
                const ohm_prob_host &Q = h->probs[p];
                const int dd = -Q.min_level;
                const int *dm = Q.dims[dd];
                if (3LL * dm[0] * dm[1] * dm[2] > 768) {
                    has_big[dd] = 1;
                    cm[(size_t)np * dd + p] = 1;
                }
            }
        }
        if (multigrid) {
            coarse_plan(h, coefs.data(), host(P.jobs), (int *)host(P.force), njobs.data());
            OHM_TRY(ensure_coarse_storage(h));
        }
        act_dev = ones;
        mlprob = at<int>(P.mlprob);
        active_mut = at<int>(P.active);
        active = active_mut;
        lam_dt = at<double>(P.coefs);
        src_coef = lam_dt + np;
        neg_lam_dt = lam_dt + 2 * np;
        return OHM_OK;
    }

    // x = B (user fields), outside any captured graph (B may change per call)
    ohm_status copy_in()
    {
        for (int l = 0; l < nlev(); ++l)
            OHM_TRY(vcopy_level<double, double>((const double *)Buser[l], (long long)h->nb_host[l] * NC, vec(P.x, l),
                                                VN, (long long)h->nb_host[l] * NC, 3, st));
        return OHM_OK;
    }

    // the staged upload becomes safe to overwrite once the stream passes here
    ohm_status staged_done()
    {
        OHM_HIP(hipEventRecord(h->stage_ev, st));
        h->stage_live = true;
        return OHM_OK;
    }

    // device part of the start of a step: the staged tables, coarse-fine
    // ghosts of eta (FP64) and FP32 copies, dense-level resistivity, coarsest
    // inverses, S = b - (1 - lambda) dt div F(b), and (multigrid) the initial
    // residual with |r|^2 and |S|^2 copied to the pinned buffer, the stop
    // rule's thresholds and, for BiCGStab, the first restart
    ohm_status start_device(bool multigrid)
    {
        const int L = nlev();
        const size_t tab_bytes = P.coefs + 8 * (size_t)h->nprob * 4 - P.jobs;
        OHM_HIP(hipMemcpyAsync(at<char>(P.jobs), h->h_stage, tab_bytes, hipMemcpyHostToDevice, st));
        for (int l = 1; l < L; ++l)
            OHM_TRY(launch_fill_ghosts<double>(h, l, eta64(l - 1), (long long)h->nb_host[l - 1] * NC,
                                               at<double>(P.oeg) + P.LG[l] * NC, 0, 1, nullptr, st));
        if (!multigrid) return OHM_OK;
        if (P.T32) {
            for (int l = 0; l < L; ++l)
                OHM_TRY(vconvert<double, T>(eta64(l), at<T>(P.eta_t) + P.LB[l] * NC, (long long)h->nb_host[l] * NC, st));
            OHM_TRY(vconvert<double, T>(at<double>(P.oeg), at<T>(P.eta_tg), P.NGt * NC, st));
        }
        // resistivity of the dense levels: mean of the 8 children
        const int D = -h->min_level;
        for (int d = 1; d <= D; ++d) {
            if (d == 1)
                OHM_TRY(launch_restrict_blk<double>(h, 0, eta64(0), 0, at<double>(P.d_eta64[1]), 0, 1, nullptr, st));
            else
                OHM_TRY(launch_dense_restrict<double>(h, -(d - 1), at<double>(P.d_eta64[d - 1]), at<double>(P.d_eta64[d]),
                                                      1, nullptr, st));
            if (P.T32)
                OHM_TRY(vconvert<double, T>(at<double>(P.d_eta64[d]), at<T>(P.d_eta[d]), h->dense_cells[d], st));
        }
        // coarsest grids: dense inverses (kept in the handle, rebuilt when
        // lam_dt or the coarsest resistivity changes)
        if (P.inv_elems > 0) {
            std::vector<const double *> ed(17, nullptr);
            for (int d = 1; d <= D; ++d) ed[d] = at<double>(P.d_eta64[d]);
            OHM_TRY(launch_coarse_build(h, ed.data(), at<char>(P.jobs), at<int>(P.force), njobs.data(),
                                        at<double>(P.aug), st));
        }
        // S = b - (1 - lambda) dt div F(b) on leaf cells (x holds b)
        OHM_TRY(composite(P.x, P.S, MODE_APPLY, src_coef, src_coef, 0));
        // the initial residual and its norms
        OHM_TRY(composite(P.x, P.r, MODE_RESID, lam_dt, neg_lam_dt, P.S));
        // (r, r) and (S, S) per problem; for BiCGStab the same launch makes
        // the first restart (rhat = r, its scalars from (r, r))
        const double *xs[2] = {at<double>(P.r), at<double>(P.S)};
        if (o->outer == 1)
            OHM_TRY(dots(xs, xs, 2, 0, at<double>(P.rhat)));
        else
            OHM_TRY(dots(xs, xs, 2));
        OHM_TRY(copy_dots(2));
        // thresholds of the stop rule; problems the initial guess already
        // satisfies leave the active set before any iteration is queued
        return launch_conv_init(h->nprob, at<double>(P.dots), o->rtol, at<double>(P.tol2), active_mut, at<int>(P.hold),
                                st);
    }

    // |S|^2 per problem
    std::vector<double> Snorm2;

    // True residual S - L x into `into` (P.r, or P.t for a verification
    // queued before the host knows that the recurrence has converged: every
    // iteration rewrites t before reading it); its per-problem square norm
    // goes to the pinned buffer at h_dots[2 nprob + p] (the first 2 nprob
    // values hold |r|^2 and |S|^2 of the step's start).  It is formed for
    // every problem: a problem that stopped earlier has the same x as when
    // its residual was last formed, so it gets the same residual again.
    ohm_status true_residual(size_t into)
    {
        const int *keep = active;
        active = nullptr;
        ohm_status s = composite(P.x, into, MODE_RESID, lam_dt, neg_lam_dt, P.S);
        const double *xs[1] = {at<double>(into)};
        if (s == OHM_OK) s = dots(xs, xs, 1);
        active = keep;
        OHM_TRY(s);
        return copy_dots(1, 2 * (size_t)h->nprob);
    }

    // device flags as last uploaded (setup uploads all ones)
    std::vector<int> act_dev;
    ohm_status set_active(const std::vector<int> &a)
    {
        if (a == act_dev) return OHM_OK;
        OHM_HIP(hipMemcpyAsync(active_mut, a.data(), sizeof(int) * a.size(), hipMemcpyHostToDevice, st));
        act_dev = a;
        return OHM_OK;
    }

    // one BiCGStab iteration (device work only; the host reads the norms)
    ohm_status bicg_iter()
    {
            // beta and rho were formed by the scalar update that closed the
            // previous iteration (or the restart)
            // p and s also go straight into the cycle's right-hand side
            const bool cp = !cycle_aliases();
            float *c32 = cp && P.T32 ? (float *)at<T>(P.rhs) : nullptr;
            double *c64 = cp && !P.T32 ? (double *)at<T>(P.rhs) : nullptr;
            OHM_TRY(vbicg_p((int)P.NBt, mlprob, active, VN, at<double>(P.scal), at<double>(P.r),
                            at<double>(P.v), at<double>(P.p), st, c32, c64));
            OHM_TRY(precond(P.p, P.ph, cp));
            {
                const double *xs[1] = {at<double>(P.rhat)}, *ys[1] = {at<double>(P.v)};
                OHM_TRY(apply_dots(P.ph, P.v, xs, ys, 1, 2));
            }
            OHM_TRY(vbicg_s((int)P.NBt, mlprob, active, VN, at<double>(P.scal), at<double>(P.r),
                            at<double>(P.v), at<double>(P.s), st, c32, c64));
            OHM_TRY(precond(P.s, P.sh, cp));
            {
                const double *xs[2] = {at<double>(P.t), at<double>(P.t)},
                             *ys[2] = {at<double>(P.s), at<double>(P.t)};
                OHM_TRY(apply_dots(P.sh, P.t, xs, ys, 2, 3));
            }
            OHM_TRY(vbicg_xr((int)P.NBt, mlprob, active, VN, at<double>(P.scal), at<double>(P.x),
                             at<double>(P.ph), at<double>(P.sh), at<double>(P.s), at<double>(P.t),
                             at<double>(P.r), at<double>(P.rhat), at<double>(P.part), st));
            // (r, r) and (rhat, r) into the iteration ring, which goes to
            // the pinned buffer whole (one copy node)
            IterRing ring;
            ring.buf = at<double>(P.ring);
            ring.flags = active_mut;
            ring.tol2 = at<double>(P.tol2);
            ring.hold = at<int>(P.hold);
            OHM_TRY(launch_reduce_scal(h->nprob, nlev(), at<long long>(P.ranges), at<double>(P.part), 2,
                                       at<double>(P.dots), 4, active, at<double>(P.scal), st, ring));
            OHM_HIP(hipMemcpyAsync(h_ring(), at<double>(P.ring), sizeof(double) * 2 * ITER_SLOTS * h->nprob,
                                   hipMemcpyDeviceToHost, st));
            return OHM_OK;
    }
    // pinned regions after the first 8 nprob values: the iteration ring, then
    // the final norms of a step
    double *h_ring() const { return h->h_dots + 8 * (size_t)h->nprob; }
    double *h_final() const { return h->h_dots + (8 + 2 * ITER_SLOTS) * (size_t)h->nprob; }
    // the first nq * nprob norms to the handle's pinned host buffer (part of a
    // captured iteration: one node, no separate copy command); read after a
    // synchronisation of the stream
    // (at element `at_host` of the pinned buffer)
    ohm_status copy_dots(int nq, size_t at_host = 0)
    {
        OHM_HIP(hipMemcpyAsync(h->h_dots + at_host, at<double>(P.dots), sizeof(double) * nq * h->nprob,
                               hipMemcpyDeviceToHost, st));
        return OHM_OK;
    }

    // one iteration of eqs. (16)-(18): B += M(R); R = S - L B; |R|^2 per problem
    ohm_status ir_iter()
    {
        OHM_TRY(precond(P.r, P.ph));
        OHM_TRY(vaxpy1((int)P.NBt, mlprob, active, VN, at<double>(P.x), at<double>(P.ph), st));
        OHM_TRY(composite(P.x, P.r, MODE_RESID, lam_dt, neg_lam_dt, P.S));
        const double *xs[1] = {at<double>(P.r)};
        OHM_TRY(dots(xs, xs, 1));
        return copy_dots(1);
    }

    // the norms an iteration copied to the pinned buffer (stride nq)
    ohm_status read_dots(int nq, std::vector<double> &out)
    {
        OHM_HIP(hipStreamSynchronize(st));
        out.assign(h->nprob, 0.0);
        for (int p = 0; p < h->nprob; ++p) out[p] = h->h_dots[(size_t)p * nq];
        return OHM_OK;
    }

    // run `body` directly, or as a HIP graph captured once and replayed while
    // the workspace, the resistivity pointers and the options are unchanged
    template <typename F>
    ohm_status replay(int kind, F body)
    {
        if (!o->graph) return body();
        std::vector<const void *> key = {ws};
        for (int l = 0; l < nlev(); ++l) key.push_back(Euser[l]);
        // the options' bytes up to the end of their last field (not the
        // struct's tail padding, which callers need not initialise)
        std::vector<char> ob((const char *)o, (const char *)&o->nu_amr + sizeof(o->nu_amr));
        ohm_hier::GraphSlot &G = h->graphs[kind];
        if (!G.exec || G.key != key || G.opts != ob) {
            if (G.exec) {
                OHM_HIP(hipGraphExecDestroy(G.exec));
                G.exec = nullptr;
            }
            // record on the handle's own stream (the caller's may be the null
            // stream, which cannot be captured); replay on the caller's stream
            std::lock_guard<std::mutex> lock(capture_mutex());
            if (!h->cap_stream) OHM_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            hipStream_t user = st;
            st = h->cap_stream;
            OHM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            ohm_status s = body();
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(st, &g);
            st = user;
            if (s != OHM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            if (e != hipSuccess) return fail(OHM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                G.exec = nullptr;
                return fail(OHM_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
            }
            G.key = key;
            G.opts = ob;
        }
        OHM_HIP(hipGraphLaunch(G.exec, st));
        return OHM_OK;
    }

    // nsteps of the explicit predictor-corrector scheme on x (coefficient
    // slot neg_lam_dt holds -dt: the caller sets lambda = 1), then copy out
    ohm_status run_explicit(int nsteps)
    {
        const int L = nlev();
        for (int k = 0; k < nsteps; ++k) {
            OHM_TRY(composite(P.x, P.p, MODE_APPLY, neg_lam_dt, neg_lam_dt, 0));    // p = x - dt div F(x)
            OHM_TRY(composite(P.p, P.v, MODE_APPLY, neg_lam_dt, neg_lam_dt, 0));    // v = p - dt div F(p)
            OHM_TRY(vmean2((int)P.NBt, mlprob, nullptr, VN, at<double>(P.x), at<double>(P.v), st));
        }
        for (int l = L - 1; l >= 1; --l)
            OHM_TRY(launch_restrict_blk<double>(h, l, vec(P.x, l), VN, vec(P.x, l - 1), VN, 3, nullptr, st));
        for (int l = 0; l < L; ++l)
            OHM_TRY(vcopy_level<double, double>(vec(P.x, l), VN, (double *)Buser[l], (long long)h->nb_host[l] * NC,
                                                (long long)h->nb_host[l] * NC, 3, st));
        OHM_HIP(hipStreamSynchronize(st));
        return OHM_OK;
    }

    // one CN step: the start (captured once per workspace, resistivity and
    // options when graphs are on), then the outer iteration
    ohm_status step(const double *dt, ohm_cn_stats *stats)
    {
        OHM_TRY(setup_host(dt));
        OHM_TRY(copy_in());
        OHM_TRY(replay(2, [&]() { return start_device(true); }));
        OHM_TRY(staged_done());
        return run(stats);
    }

    ohm_status explicit_steps(const double *dt, int nsteps)
    {
        OHM_TRY(setup_host(dt, false));
        OHM_TRY(copy_in());
        OHM_TRY(start_device(false));
        OHM_TRY(staged_done());
        return run_explicit(nsteps);
    }

    // the end of a step, queued: norms of the true residual `res` (into the
    // pinned buffer), average-down of x over the AMR levels and the copy to
    // the user's fields (skipped on the device once a norm was non-finite).
    // It may be queued behind a true residual that turns out not to
    // converge: the iteration then resumes (values of x under finer blocks
    // are restored by every composite operator before use) and the end is
    // queued again.
    ohm_status finish_async(size_t res)
    {
        const int np = h->nprob, L = nlev();
        OHM_TRY(vnorms((int)P.NBt, mlprob, nullptr, VN, at<double>(res), at<double>(P.part), st));
        OHM_TRY(reduce(6, 3, at<double>(P.dots)));
        OHM_HIP(hipMemcpyAsync(h_final(), at<double>(P.dots), sizeof(double) * 6 * np, hipMemcpyDeviceToHost, st));
        for (int l = L - 1; l >= 1; --l)
            OHM_TRY(launch_restrict_blk<double>(h, l, vec(P.x, l), VN, vec(P.x, l - 1), VN, 3, nullptr, st));
        for (int l = 0; l < L; ++l)
            OHM_TRY(vcopy_level<double, double>(vec(P.x, l), VN, (double *)Buser[l], (long long)h->nb_host[l] * NC,
                                                (long long)h->nb_host[l] * NC, 3, st, at<int>(P.hold)));
        return OHM_OK;
    }

    ohm_status run(ohm_cn_stats *stats)
    {
        const int np = h->nprob;
        std::vector<int> iters(np, 0), mgapps(np, 0), act(np, 1);
        std::vector<double> r2(np), rfin(np, 0.0);
        Snorm2.assign(np, 0.0);
        auto converged = [&](int p, double v) {
            return !(v > o->rtol * o->rtol * std::fmax(Snorm2[p], 1e-300));
        };
        auto any = [](const std::vector<int> &a) {
            return std::any_of(a.begin(), a.end(), [](int x) { return x != 0; });
        };
        // |S|^2 and |r|^2 of the initial guess (start_device copied them and
        // took the same decisions on the device: k_conv_init).  A problem
        // stops being updated only right after a true residual that included
        // it, so at the end r holds every problem's residual at its final B.
        bool known = false;
        auto read_start = [&]() -> ohm_status {
            for (int p = 0; p < np; ++p) {
                r2[p] = h->h_dots[2 * p];
                Snorm2[p] = h->h_dots[2 * p + 1];
            }
            rfin = r2;
            for (int p = 0; p < np; ++p) {
                if (!std::isfinite(r2[p])) return fail(OHM_ERR_NONFINITE, "problem %d: non-finite residual", p);
                if (converged(p, r2[p])) act[p] = 0;
            }
            act_dev = act;
            known = true;
            return OHM_OK;
        };
        const int maxit = o->max_iters;
        bool finished = false;   // the end of the step is queued behind the last true residual
        if (o->outer == 0) {
            OHM_HIP(hipStreamSynchronize(st));
            OHM_TRY(read_start());
            // eqs. (16)-(18): R = S - L B; B <- B + M(R)
            for (int it = 0; it < maxit && any(act); ++it) {
                OHM_TRY(replay(0, [&]() { return ir_iter(); }));
                OHM_TRY(read_dots(1, r2));
                for (int p = 0; p < np; ++p)
                    if (act[p]) {
                        ++iters[p];
                        ++mgapps[p];
                        rfin[p] = r2[p];
                        if (!std::isfinite(r2[p])) return fail(OHM_ERR_NONFINITE, "problem %d: non-finite residual", p);
                        if (converged(p, r2[p])) act[p] = 0;
                    }
                OHM_TRY(set_active(act));
            }
        } else {
            // BiCGStab; restarted from the true residual when the recurrence
            // residual has converged but the true one has not.  The host
            // queues iterations ahead of its reads: the first pass of a step
            // queues as many as the previous step's first pass took before
            // its first read (the device drops each problem at the iteration
            // that converges it, so the iterations queued behind leave it
            // unchanged), later reads follow every iteration.  From the
            // predicted count on, the verifying true residual (into t) and the
            // end of the step are queued behind the iterations as well, so a
            // step whose prediction holds takes one synchronisation; when the
            // recurrence has not converged they are simply queued again.
            int it_total = 0, first_pass = -1;
            const int pred = h->bicg_pred;
            bool restarted = true;   // the step's start made the first restart
            while (it_total < maxit && (!known || any(act))) {
                // restart: rhat = r (copied by the dot kernel that forms
                // (r, r)), rho = alpha = omega = 1, and a first direction p = r
                // (the scalar stage sets beta = 0, which the direction update
                // reads as p = v = 0, so neither is filled)
                if (!restarted) {
                    const double *xs[1] = {at<double>(P.r)};
                    OHM_TRY(dots(xs, xs, 1, 0, at<double>(P.rhat)));
                }
                restarted = false;
                std::vector<int> inner(act);
                int since = 0;          // iterations since the restart (the ring's slot count)
                bool spec = false;      // a verification is queued behind the last iteration
                while (it_total < maxit) {
                    int nb = 1;
                    if (first_pass < 0 && since == 0) nb = std::max(1, std::min({pred, ITER_SLOTS, maxit - it_total}));
                    for (int j = 0; j < nb; ++j) OHM_TRY(replay(1, [&]() { return bicg_iter(); }));
                    it_total += nb;
                    spec = first_pass < 0 && pred > 0 && since + nb >= pred;
                    if (spec) {
                        OHM_TRY(true_residual(P.t));
                        OHM_TRY(finish_async(P.t));
                    }
                    OHM_HIP(hipStreamSynchronize(st));
                    if (!known) {
                        OHM_TRY(read_start());
                        inner = act;
                    }
                    int done_at = -1;
                    for (int j = 0; j < nb && done_at < 0; ++j) {
                        const double *d = h_ring() + 2 * (size_t)np * ((since + j) % ITER_SLOTS);
                        for (int p = 0; p < np; ++p)
                            if (inner[p]) {
                                ++iters[p];
                                mgapps[p] += 2;
                                if (!std::isfinite(d[2 * p]))
                                    return fail(OHM_ERR_NONFINITE, "problem %d: non-finite residual", p);
                                if (converged(p, d[2 * p])) inner[p] = 0;
                            }
                        if (!any(inner)) done_at = since + j + 1;
                    }
                    since += nb;
                    // the device dropped the same problems as the iterations ran
                    act_dev = inner;
                    if (done_at >= 0) {
                        if (first_pass < 0) first_pass = done_at;
                        break;
                    }
                }
                if (first_pass < 0) first_pass = since;
                if (!any(act)) break;   // every problem satisfied by its initial guess
                // verify with the true residual, the end of the step queued
                // behind it (unless both are queued already)
                if (!spec || any(inner)) {
                    OHM_TRY(true_residual(P.r));
                    OHM_TRY(finish_async(P.r));
                    OHM_HIP(hipStreamSynchronize(st));
                    spec = false;
                }
                finished = true;
                for (int p = 0; p < np; ++p)
                    if (act[p]) {
                        rfin[p] = h->h_dots[2 * (size_t)np + p];
                        if (converged(p, rfin[p])) act[p] = 0;
                    }
                if (any(act)) {
                    finished = false;
                    // the restart reads the true residual from r
                    if (spec)
                        OHM_TRY(vconvert<double, double>(at<double>(P.t), at<double>(P.r), 3 * VN, st));
                    OHM_TRY(set_active(act));
                }
            }
            h->bicg_pred = first_pass;
        }
        if (!finished) {
            OHM_TRY(finish_async(P.r));
            OHM_HIP(hipStreamSynchronize(st));
        }
        const double *nrm = h_final();
        ohm_status result = OHM_OK;
        for (int p = 0; p < np; ++p) {
            const double rel = std::sqrt(rfin[p] / std::max(Snorm2[p], 1e-300));
            if (stats) {
                stats[p].iters = iters[p];
                stats[p].mg_apps = mgapps[p];
                stats[p].rel_res = rel;
                for (int c = 0; c < 3; ++c) stats[p].max_res[c] = nrm[6 * p + 3 + c];
            }
            if (!std::isfinite(rfin[p])) result = fail(OHM_ERR_NONFINITE, "problem %d: non-finite residual", p);
            else if (!converged(p, rfin[p]) && result == OHM_OK)
                result = fail(OHM_ERR_NOCONV, "problem %d: relative residual %.3e after %d iterations", p, rel,
                              iters[p]);
        }
        return result;
    }
};

}  // namespace

extern "C" {

void ohm_cn_default_opts(ohm_cn_opts *o)
{
    if (!o) return;
    o->lambda = 0.5;
    o->rtol = 1e-10;
    o->max_iters = 100;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->n_vcycles = 1;
    o->cycle = 0;
    o->outer = 1;
    o->precision = 0;
    o->coarse_sweeps = 16;
    o->nu_coarse = 0;
    o->graph = 1;
    o->ordering = 0;
    o->amr_fmg = 0;
    o->amr_vcycles = 1;
    o->amr_mlat = 0;
    o->nu_amr = 0;
}

ohm_status ohm_cn_workspace_size(const ohm_hier *h, const ohm_cn_opts *opts, size_t *bytes)
{
    if (!h || !bytes) return fail(OHM_ERR_ARG, "NULL argument");
    if (!valid_opts(opts)) return fail(OHM_ERR_ARG, "invalid options");
    *bytes = make_plan(h, opts).total;
    return OHM_OK;
}

ohm_status ohm_cn_step(ohm_hier *h, void *const B[], const void *const eta[], const double *dt,
                       const ohm_cn_opts *opts, void *workspace, size_t ws_bytes, ohm_cn_stats *stats,
                       hipStream_t stream)
{
    if (!h) return fail(OHM_ERR_ARG, "handle is NULL");
    if (!B || !eta || !dt) return fail(OHM_ERR_ARG, "NULL argument");
    if (!valid_opts(opts)) return fail(OHM_ERR_ARG, "invalid options");
    for (int l = 0; l < h->nlev; ++l)
        if (!B[l] || !eta[l]) return fail(OHM_ERR_ARG, "B[%d] or eta[%d] is NULL", l, l);
    Plan P = make_plan(h, opts);
    if (!workspace || ws_bytes < P.total)
        return fail(OHM_ERR_NOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, P.total);
    if (((uintptr_t)workspace & 255) != 0) return fail(OHM_ERR_ARG, "workspace must be 256-byte aligned");
    if (opts->precision == 1) {
        Solver<float> S;
        S.h = h;
        S.o = opts;
        S.P = P;
        S.ws = (char *)workspace;
        S.st = stream;
        S.Buser = B;
        S.Euser = eta;
        return S.step(dt, stats);
    }
    Solver<double> S;
    S.h = h;
    S.o = opts;
    S.P = P;
    S.ws = (char *)workspace;
    S.st = stream;
    S.Buser = B;
    S.Euser = eta;
    return S.step(dt, stats);
}

ohm_status ohm_explicit_workspace_size(const ohm_hier *h, size_t *bytes)
{
    if (!h || !bytes) return fail(OHM_ERR_ARG, "NULL argument");
    ohm_cn_opts o;
    ohm_cn_default_opts(&o);
    o.precision = 0;
    *bytes = make_plan(h, &o).total;
    return OHM_OK;
}

ohm_status ohm_explicit_step(ohm_hier *h, void *const B[], const void *const eta[], const double *dt, int nsteps,
                             void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!h) return fail(OHM_ERR_ARG, "handle is NULL");
    if (!B || !eta || !dt) return fail(OHM_ERR_ARG, "NULL argument");
    if (nsteps < 0) return fail(OHM_ERR_ARG, "nsteps must be >= 0, got %d", nsteps);
    for (int l = 0; l < h->nlev; ++l)
        if (!B[l] || !eta[l]) return fail(OHM_ERR_ARG, "B[%d] or eta[%d] is NULL", l, l);
    ohm_cn_opts o;
    ohm_cn_default_opts(&o);
    o.precision = 0;
    o.lambda = 1.0;    // the coefficient slot -lambda dt is then -dt
    o.graph = 0;
    Plan P = make_plan(h, &o);
    if (!workspace || ws_bytes < P.total)
        return fail(OHM_ERR_NOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, P.total);
    if (((uintptr_t)workspace & 255) != 0) return fail(OHM_ERR_ARG, "workspace must be 256-byte aligned");
    Solver<double> S;
    S.h = h;
    S.o = &o;
    S.P = P;
    S.ws = (char *)workspace;
    S.st = stream;
    S.Buser = B;
    S.Euser = eta;
    return S.explicit_steps(dt, nsteps);
}

}  // extern "C"
