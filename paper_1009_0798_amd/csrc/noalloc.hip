// ohm_residual_noalloc: the residual of eq. (20) with its per-problem norms,
// for callers that cannot allocate device memory.  Its scratch (the per-problem
// coefficients, block ranges, the reduction's per-block partials and its
// per-problem sums) lives in one file-scope device array of fixed size instead
// of the handle's buffers, the per-call host scalars travel as kernel
// arguments, and the norms are written to caller device memory without a
// synchronisation or a copy, so the call can be captured into a HIP graph.
// The stencil and reduction kernels are those of ohm_residual.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

using namespace ohm;

namespace {

constexpr size_t SCRATCH_BYTES = size_t(4) << 20;   // 4 MiB per device
constexpr int MAX_DEVICES = 64;

// The array's name in host code is a host-side stand-in: kernels and copies
// use the device address obtained below, never `scratch` itself.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device, looked up once per device
ohm_status scratch_ptr(char **out)
{
    int dev = -1;
    OHM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(OHM_ERR_ARG, "device %d outside 0..%d", dev, MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(OHM_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = (char *)g_ptr[dev];
    return OHM_OK;
}

inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Per-call host scalars (coefficients, block ranges) reach the scratch through
// kernel arguments, 16 problems per launch: the values are copied when the
// kernel is enqueued, so a call captured into a graph replays them as they
// were, and no host buffer has to outlive the call.
constexpr int CHUNK = 16;
struct ScalarChunk {
    int first, n;
    double coef[CHUNK];
    long long lo[CHUNK], hi[CHUNK];
};

__global__ void __launch_bounds__(64) k_put_scalars(ScalarChunk c, double *__restrict__ coef,
                                                    long long *__restrict__ rg)
{
    const int t = threadIdx.x;
    if (t >= c.n) return;
    coef[c.first + t] = c.coef[t];
    if (rg) {
        rg[2 * (c.first + t)] = c.lo[t];
        rg[2 * (c.first + t) + 1] = c.hi[t];
    }
}

// [nprob][6] = (sum R_x^2, sum R_y^2, sum R_z^2, max|R_x|, max|R_y|, max|R_z|)
// -> [nprob][3][2] = (sum R_c^2, max |R_c|) per component
__global__ void __launch_bounds__(256) k_norm_pairs(int nprob, const double *__restrict__ in, double *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * nprob) return;
    const int p = t / 6, j = t % 6, c = j >> 1, m = j & 1;
    out[t] = in[6 * p + 3 * m + c];
}

}  // namespace

extern "C" ohm_status ohm_residual_noalloc(ohm_hier *h, int32_t level, const void *B, const void *B_ghost,
                                           const void *S, const void *eta, const void *eta_ghost,
                                           const double *lam_dt, void *R, double *norms, ohm_dtype dtype,
                                           hipStream_t stream)
{
    if (!h) return fail(OHM_ERR_ARG, "handle is NULL");
    if (level >= h->nlev || level < h->min_level)
        return fail(OHM_ERR_ARG, "level %d outside %d..%d", level, h->min_level, h->nlev - 1);
    if (dtype != OHM_F64 && dtype != OHM_F32) return fail(OHM_ERR_ARG, "unknown dtype %d", (int)dtype);
    if (!B || !S || !eta) return fail(OHM_ERR_ARG, "NULL field");
    if (!R && !norms) return fail(OHM_ERR_ARG, "nothing to compute: R and norms are both NULL");
    if (R == B) return fail(OHM_ERR_ARG, "R must not alias B");
    if (norms && level < 0) return fail(OHM_ERR_ARG, "norms are available on AMR levels only");
    if (level < 0 && !R) return fail(OHM_ERR_ARG, "R is required on multigrid levels");
    if (!lam_dt) return fail(OHM_ERR_ARG, "lam_dt is NULL");
    for (int p = 0; p < h->nprob; ++p)
        if (!std::isfinite(lam_dt[p])) return fail(OHM_ERR_NONFINITE, "lam_dt[%d] is not finite", p);
    if (level >= 1 && h->ng_host[level] > 0 && (!B_ghost || !eta_ghost))
        return fail(OHM_ERR_ARG, "level %d has %d ghost blocks: ghost arrays are required", level, h->ng_host[level]);

    // scratch layout: coefficients [nprob], block ranges [nprob][2], per-problem
    // sums [nprob][6], per-block partials [nblocks][6]
    const size_t np = (size_t)h->nprob;
    const size_t nb = level >= 0 ? (size_t)h->nb_host[level] : 0;
    const size_t o_coef = 0, o_rng = al256(8 * np), o_sum = o_rng + al256(16 * np), o_part = o_sum + al256(48 * np);
    const size_t need = norms ? o_part + 48 * nb : o_rng;
    if (need > SCRATCH_BYTES)
        return fail(OHM_ERR_NOMEM, "level %d with %zu problems and %zu blocks needs %zu bytes of scratch; the static "
                                   "scratch holds %zu", level, np, nb, need, SCRATCH_BYTES);
    char *base = nullptr;
    OHM_TRY(scratch_ptr(&base));
    double *coef = (double *)(base + o_coef);
    long long *d_rg = norms ? (long long *)(base + o_rng) : nullptr;
    for (size_t p0 = 0; p0 < np; p0 += CHUNK) {
        ScalarChunk c{};
        c.first = (int)p0;
        c.n = (int)std::min<size_t>(CHUNK, np - p0);
        for (int t = 0; t < c.n; ++t) {
            const ohm_prob_host &P = h->probs[p0 + t];
            c.coef[t] = lam_dt[p0 + t];
            c.lo[t] = level >= 0 && level < P.nlevels ? P.boff[level] : 0;
            c.hi[t] = level >= 0 && level < P.nlevels ? P.boff[level] + P.nb[level] : 0;
        }
        k_put_scalars<<<1, 64, 0, stream>>>(c, coef, d_rg);
        OHM_TRY(check_launch("scalar upload"));
    }
    double *part = norms ? (double *)(base + o_part) : nullptr;
    const long long cs = level >= 0 ? (long long)nb * NC : h->dense_cells[-level];
    if (level >= 0) {
        const long long gcs = (long long)h->ng_host[level] * NC;
        ohm_status st =
            dtype == OHM_F64
                ? launch_blk_stencil<double>(h, level, MODE_RESID, (const double *)B, (const double *)B_ghost, cs, gcs,
                                             (const double *)S, (const double *)eta, (const double *)eta_ghost, coef,
                                             (double *)R, 0, part, nullptr, nullptr, stream)
                : launch_blk_stencil<float>(h, level, MODE_RESID, (const float *)B, (const float *)B_ghost, cs, gcs,
                                            (const float *)S, (const float *)eta, (const float *)eta_ghost, coef,
                                            (float *)R, 0, part, nullptr, nullptr, stream);
        OHM_TRY(st);
    } else {
        ohm_status st =
            dtype == OHM_F64
                ? launch_dense_stencil<double>(h, level, MODE_RESID, (const double *)B, (const double *)S,
                                               (const double *)eta, coef, (double *)R, 0, true, nullptr, stream)
                : launch_dense_stencil<float>(h, level, MODE_RESID, (const float *)B, (const float *)S,
                                              (const float *)eta, coef, (float *)R, 0, true, nullptr, stream);
        OHM_TRY(st);
    }
    if (norms) {
        double *sums = (double *)(base + o_sum);
        OHM_TRY(launch_reduce_problem(h->nprob, 1, d_rg, part, 6, 3, sums, stream));
        const int n = 6 * h->nprob;
        k_norm_pairs<<<(n + 255) / 256, 256, 0, stream>>>(h->nprob, sums, norms);
        OHM_TRY(check_launch("norm pairs"));
    }
    return OHM_OK;
}
