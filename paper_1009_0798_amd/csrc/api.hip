// C ABI entry points of the building blocks: argument checks on the host, then
// launches of the block-level or dense-level kernels.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "common.h"

using namespace ohm;

namespace {

constexpr int RING = 64;

// copy per-problem host coefficients into the next device slot
ohm_status coef_slot(ohm_hier *h, const double *host, hipStream_t s, double **dev, int *slot)
{
    if (!h->d_ring) {
        OHM_HIP(hipMalloc((void **)&h->d_ring, sizeof(double) * RING * h->nprob));
        for (int i = 0; i < RING; ++i) OHM_HIP(hipEventCreateWithFlags(&h->ring_ev[i], hipEventDisableTiming));
    }
    const int k = h->ring_pos;
    h->ring_pos = (k + 1) % RING;
    if (h->ring_live[k]) OHM_HIP(hipEventSynchronize(h->ring_ev[k]));
    double *d = h->d_ring + (size_t)k * h->nprob;
    OHM_HIP(hipMemcpyAsync(d, host, sizeof(double) * h->nprob, hipMemcpyHostToDevice, s));
    *dev = d;
    *slot = k;
    return OHM_OK;
}

ohm_status coef_done(ohm_hier *h, int slot, hipStream_t s)
{
    OHM_HIP(hipEventRecord(h->ring_ev[slot], s));
    h->ring_live[slot] = true;
    return OHM_OK;
}

ohm_status check_level(const ohm_hier *h, int level)
{
    if (!h) return fail(OHM_ERR_ARG, "handle is NULL");
    if (level >= h->nlev || level < h->min_level)
        return fail(OHM_ERR_ARG, "level %d outside %d..%d", level, h->min_level, h->nlev - 1);
    return OHM_OK;
}

ohm_status check_dtype(ohm_dtype d)
{
    if (d != OHM_F64 && d != OHM_F32) return fail(OHM_ERR_ARG, "unknown dtype %d", (int)d);
    return OHM_OK;
}

ohm_status check_coef(const ohm_hier *h, const double *c, const char *name)
{
    if (!c) return fail(OHM_ERR_ARG, "%s is NULL", name);
    for (int p = 0; p < h->nprob; ++p)
        if (!std::isfinite(c[p])) return fail(OHM_ERR_NONFINITE, "%s[%d] is not finite", name, p);
    return OHM_OK;
}

ohm_status need_ghosts(const ohm_hier *h, int level, const void *Bg, const void *eg)
{
    if (level >= 1 && h->ng_host[level] > 0 && (!Bg || !eg))
        return fail(OHM_ERR_ARG, "level %d has %d ghost blocks: ghost arrays are required", level, h->ng_host[level]);
    return OHM_OK;
}

long long level_cs(const ohm_hier *h, int level)
{
    return level >= 0 ? (long long)h->nb_host[level] * NC : h->dense_cells[-level];
}

template <typename T>
ohm_status stencil(ohm_hier *h, int level, int mode, const void *B, const void *Bg, const void *S, const void *eta,
                   const void *etag, const double *coef_dev, void *out, int colour, double *partials,
                   hipStream_t s)
{
    if (level >= 0)
        return launch_blk_stencil<T>(h, level, mode, (const T *)B, (const T *)Bg, level_cs(h, level),
                                     (long long)h->ng_host[level] * NC, (const T *)S, (const T *)eta,
                                     (const T *)etag, coef_dev, (T *)out, colour, partials, nullptr, nullptr, s);
    return launch_dense_stencil<T>(h, level, mode, (const T *)B, (const T *)S, (const T *)eta, coef_dev, (T *)out,
                                   colour, true, nullptr, s);
}

}  // namespace

extern "C" {

ohm_status ohm_fill_ghosts(ohm_hier *h, int32_t level, const void *coarse, void *ghost, int32_t ncomp,
                           ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, level));
    OHM_TRY(check_dtype(dtype));
    if (level < 1) return fail(OHM_ERR_ARG, "ghost fill needs an AMR level >= 1 (got %d)", level);
    if (ncomp != 1 && ncomp != 3) return fail(OHM_ERR_ARG, "ncomp must be 1 or 3");
    if (h->ng_host[level] == 0) return OHM_OK;
    if (!coarse || !ghost) return fail(OHM_ERR_ARG, "NULL field");
    const long long ccs = level_cs(h, level - 1), gcs = (long long)h->ng_host[level] * NC;
    if (dtype == OHM_F64)
        return launch_fill_ghosts<double>(h, level, (const double *)coarse, ccs, (double *)ghost, gcs, ncomp, nullptr,
                                          stream);
    return launch_fill_ghosts<float>(h, level, (const float *)coarse, ccs, (float *)ghost, gcs, ncomp, nullptr,
                                     stream);
}

ohm_status ohm_apply(ohm_hier *h, int32_t level, const void *B, const void *B_ghost, const void *eta,
                     const void *eta_ghost, const double *coef, void *out, ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, level));
    OHM_TRY(check_dtype(dtype));
    if (!B || !eta || !out) return fail(OHM_ERR_ARG, "NULL field");
    if (B == out) return fail(OHM_ERR_ARG, "out must not alias B");
    OHM_TRY(check_coef(h, coef, "coef"));
    OHM_TRY(need_ghosts(h, level, B_ghost, eta_ghost));
    double *cd;
    int slot;
    OHM_TRY(coef_slot(h, coef, stream, &cd, &slot));
    ohm_status st = dtype == OHM_F64
                        ? stencil<double>(h, level, MODE_APPLY, B, B_ghost, nullptr, eta, eta_ghost, cd, out, 0, nullptr, stream)
                        : stencil<float>(h, level, MODE_APPLY, B, B_ghost, nullptr, eta, eta_ghost, cd, out, 0, nullptr, stream);
    OHM_TRY(st);
    return coef_done(h, slot, stream);
}

ohm_status ohm_residual(ohm_hier *h, int32_t level, const void *B, const void *B_ghost, const void *S,
                        const void *eta, const void *eta_ghost, const double *lam_dt, void *R, double *norms,
                        ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, level));
    OHM_TRY(check_dtype(dtype));
    if (!B || !S || !eta) return fail(OHM_ERR_ARG, "NULL field");
    if (!R && !norms) return fail(OHM_ERR_ARG, "nothing to compute: R and norms are both NULL");
    if (R == B) return fail(OHM_ERR_ARG, "R must not alias B");
    if (norms && level < 0) return fail(OHM_ERR_ARG, "norms are available on AMR levels only");
    if (level < 0 && !R) return fail(OHM_ERR_ARG, "R is required on multigrid levels");
    OHM_TRY(check_coef(h, lam_dt, "lam_dt"));
    OHM_TRY(need_ghosts(h, level, B_ghost, eta_ghost));
    double *cd;
    int slot;
    OHM_TRY(coef_slot(h, lam_dt, stream, &cd, &slot));
    double *part = norms ? h->d_part : nullptr;
    ohm_status st = dtype == OHM_F64
                        ? stencil<double>(h, level, MODE_RESID, B, B_ghost, S, eta, eta_ghost, cd, R, 0, part, stream)
                        : stencil<float>(h, level, MODE_RESID, B, B_ghost, S, eta, eta_ghost, cd, R, 0, part, stream);
    OHM_TRY(st);
    OHM_TRY(coef_done(h, slot, stream));
    if (norms) {
        // one range per problem on this level
        std::vector<long long> rg(2 * h->nprob);
        for (int p = 0; p < h->nprob; ++p) {
            const ohm_prob_host &P = h->probs[p];
            rg[2 * p] = level < P.nlevels ? P.boff[level] : 0;
            rg[2 * p + 1] = level < P.nlevels ? P.boff[level] + P.nb[level] : 0;
        }
        long long *d_rg = (long long *)(h->d_part + 6 * (size_t)h->nb_host[level]);
        OHM_HIP(hipMemcpyAsync(d_rg, rg.data(), sizeof(long long) * rg.size(), hipMemcpyHostToDevice, stream));
        OHM_TRY(launch_reduce_problem(h->nprob, 1, d_rg, h->d_part, 6, 3, h->d_norms, stream));
        std::vector<double> tmp(6 * h->nprob);
        OHM_HIP(hipMemcpyAsync(tmp.data(), h->d_norms, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost, stream));
        OHM_HIP(hipStreamSynchronize(stream));
        for (int p = 0; p < h->nprob; ++p)
            for (int c = 0; c < 3; ++c) {
                norms[6 * p + 2 * c] = tmp[6 * p + c];
                norms[6 * p + 2 * c + 1] = tmp[6 * p + 3 + c];
            }
    }
    return OHM_OK;
}

ohm_status ohm_smooth(ohm_hier *h, int32_t level, void *B, const void *B_ghost, const void *S, const void *eta,
                      const void *eta_ghost, const double *lam_dt, int32_t nsweeps, int32_t ordering, void *tmp,
                      ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, level));
    OHM_TRY(check_dtype(dtype));
    if (!B || !S || !eta || !tmp) return fail(OHM_ERR_ARG, "NULL field");
    if (nsweeps < 0) return fail(OHM_ERR_ARG, "nsweeps must be >= 0");
    if (ordering != 0 && ordering != 1) return fail(OHM_ERR_ARG, "ordering must be 0 (red-black) or 1 (four colours)");
    if (tmp == B) return fail(OHM_ERR_ARG, "tmp must not alias B");
    OHM_TRY(check_coef(h, lam_dt, "lam_dt"));
    OHM_TRY(need_ghosts(h, level, B_ghost, eta_ghost));
    if (nsweeps == 0) return OHM_OK;
    double *cd;
    int slot;
    OHM_TRY(coef_slot(h, lam_dt, stream, &cd, &slot));
    // one fused launch per sweep where the level's arrays fit the sweep's
    // 32-bit offsets, else one launch per colour
    const unsigned long long per = (unsigned long long)NC * (dtype == OHM_F64 ? 8 : 4), lim = 0xFFFFFFFFull;
    if (level >= 0 && h->amr[level].fused && ordering == 0 && h->amr[level].nb * per <= lim &&
        (h->amr[level].complete27 || h->amr[level].ng * per <= lim)) {
        const long long cs = level_cs(h, level), gcs = (long long)h->ng_host[level] * NC;
        for (int k = 0; k < nsweeps; ++k) {
            const void *src = (k & 1) ? tmp : B;
            void *dst = (k & 1) ? B : tmp;
            ohm_status st =
                dtype == OHM_F64
                    ? launch_blk_sweep<double>(h, level, (const double *)src, cs, (const double *)S,
                                               (const double *)eta, cd, (double *)dst, nullptr, stream, nullptr, 0,
                                               (const double *)B_ghost, gcs, (const double *)eta_ghost)
                    : launch_blk_sweep<float>(h, level, (const float *)src, cs, (const float *)S, (const float *)eta,
                                              cd, (float *)dst, nullptr, stream, nullptr, 0, (const float *)B_ghost,
                                              gcs, (const float *)eta_ghost);
            OHM_TRY(st);
        }
        if (nsweeps & 1) OHM_HIP(hipMemcpyAsync(B, tmp, (size_t)(3 * cs) * (dtype == OHM_F64 ? 8 : 4),
                                                hipMemcpyDeviceToDevice, stream));
        return coef_done(h, slot, stream);
    }
    if (level < 0) {
        ohm_status st = dtype == OHM_F64
                            ? launch_dense_smooth<double>(h, level, (double *)B, (double *)tmp, (const double *)S,
                                                          (const double *)eta, cd, nsweeps, true, nullptr, stream, 0,
                                                          nullptr, nullptr, ordering)
                            : launch_dense_smooth<float>(h, level, (float *)B, (float *)tmp, (const float *)S,
                                                         (const float *)eta, cd, nsweeps, true, nullptr, stream, 0,
                                                         nullptr, nullptr, ordering);
        OHM_TRY(st);
        return coef_done(h, slot, stream);
    }
    // one out-of-place launch per colour class, B -> tmp -> B ...: an even
    // number per sweep, so each sweep ends in B
    const int ncol = ordering ? 4 : 2, c0 = ordering ? 2 : 0;
    for (int k = 0; k < nsweeps; ++k) {
        for (int c = 0; c < ncol; ++c) {
            const void *src = (c & 1) ? tmp : B;
            void *dst = (c & 1) ? B : tmp;
            ohm_status st =
                dtype == OHM_F64
                    ? stencil<double>(h, level, MODE_SMOOTH, src, B_ghost, S, eta, eta_ghost, cd, dst, c0 + c, nullptr, stream)
                    : stencil<float>(h, level, MODE_SMOOTH, src, B_ghost, S, eta, eta_ghost, cd, dst, c0 + c, nullptr, stream);
            OHM_TRY(st);
        }
    }
    return coef_done(h, slot, stream);
}

ohm_status ohm_restrict(ohm_hier *h, int32_t fine_level, const void *fine, void *coarse, int32_t ncomp,
                        ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, fine_level));
    OHM_TRY(check_level(h, fine_level - 1));
    OHM_TRY(check_dtype(dtype));
    if (!fine || !coarse) return fail(OHM_ERR_ARG, "NULL field");
    if (ncomp != 1 && ncomp != 3) return fail(OHM_ERR_ARG, "ncomp must be 1 or 3");
    if (fine_level >= 0) {
        const long long fcs = level_cs(h, fine_level), ccs = level_cs(h, fine_level - 1);
        if (dtype == OHM_F64)
            return launch_restrict_blk<double>(h, fine_level, (const double *)fine, fcs, (double *)coarse, ccs, ncomp,
                                               nullptr, stream);
        return launch_restrict_blk<float>(h, fine_level, (const float *)fine, fcs, (float *)coarse, ccs, ncomp, nullptr,
                                          stream);
    }
    if (dtype == OHM_F64)
        return launch_dense_restrict<double>(h, fine_level, (const double *)fine, (double *)coarse, ncomp, nullptr,
                                             stream);
    return launch_dense_restrict<float>(h, fine_level, (const float *)fine, (float *)coarse, ncomp, nullptr, stream);
}

ohm_status ohm_prolong(ohm_hier *h, int32_t coarse_level, const void *coarse, void *fine, int32_t ncomp,
                       int32_t accumulate, ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, coarse_level));
    OHM_TRY(check_level(h, coarse_level + 1));
    OHM_TRY(check_dtype(dtype));
    if (!fine || !coarse) return fail(OHM_ERR_ARG, "NULL field");
    if (ncomp != 1 && ncomp != 3) return fail(OHM_ERR_ARG, "ncomp must be 1 or 3");
    if (coarse_level >= -1) {
        const long long ccs = level_cs(h, coarse_level), fcs = level_cs(h, coarse_level + 1);
        if (dtype == OHM_F64)
            return launch_prolong_blk<double>(h, coarse_level, (const double *)coarse, ccs, (double *)fine, fcs, ncomp,
                                              accumulate ? 1 : 0, nullptr, stream);
        return launch_prolong_blk<float>(h, coarse_level, (const float *)coarse, ccs, (float *)fine, fcs, ncomp,
                                         accumulate ? 1 : 0, nullptr, stream);
    }
    if (dtype == OHM_F64)
        return launch_dense_prolong<double>(h, coarse_level, (const double *)coarse, (double *)fine, ncomp,
                                            accumulate ? 1 : 0, nullptr, stream);
    return launch_dense_prolong<float>(h, coarse_level, (const float *)coarse, (float *)fine, ncomp,
                                       accumulate ? 1 : 0, nullptr, stream);
}

ohm_status ohm_reflux(ohm_hier *h, int32_t level, const void *B_coarse, const void *eta_coarse, const void *B_fine,
                      const void *B_fine_ghost, const void *eta_fine, const void *eta_fine_ghost, const double *coef,
                      void *out, int32_t zero_covered, ohm_dtype dtype, hipStream_t stream)
{
    OHM_TRY(check_level(h, level));
    OHM_TRY(check_dtype(dtype));
    if (level < 0 || level + 1 >= h->nlev) return fail(OHM_ERR_ARG, "reflux needs AMR levels l and l+1");
    if (!B_coarse || !eta_coarse || !B_fine || !eta_fine || !out) return fail(OHM_ERR_ARG, "NULL field");
    OHM_TRY(need_ghosts(h, level + 1, B_fine_ghost, eta_fine_ghost));
    OHM_TRY(check_coef(h, coef, "coef"));
    double *cd;
    int slot;
    OHM_TRY(coef_slot(h, coef, stream, &cd, &slot));
    const long long ccs = level_cs(h, level), fcs = level_cs(h, level + 1), gcs = (long long)h->ng_host[level + 1] * NC;
    ohm_status st;
    if (dtype == OHM_F64)
        st = launch_reflux<double>(h, level, (const double *)B_coarse, ccs, (const double *)eta_coarse,
                                   (const double *)B_fine, fcs, (const double *)B_fine_ghost, gcs,
                                   (const double *)eta_fine, (const double *)eta_fine_ghost, cd, (double *)out, nullptr,
                                   stream);
    else
        st = launch_reflux<float>(h, level, (const float *)B_coarse, ccs, (const float *)eta_coarse,
                                  (const float *)B_fine, fcs, (const float *)B_fine_ghost, gcs, (const float *)eta_fine,
                                  (const float *)eta_fine_ghost, cd, (float *)out, nullptr, stream);
    OHM_TRY(st);
    OHM_TRY(coef_done(h, slot, stream));
    if (zero_covered) {
        if (dtype == OHM_F64) return launch_zero_covered<double>(h, level, (double *)out, ccs, 3, stream);
        return launch_zero_covered<float>(h, level, (float *)out, ccs, 3, stream);
    }
    return OHM_OK;
}

}  // extern "C"
