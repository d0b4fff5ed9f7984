// Vector kernels of the outer Krylov / refinement iteration on multi-level
// block vectors [3][blocks of every AMR level][512]: fills, conversions,
// per-block partial dot products (reduced per problem in fixed order) and the
// BiCGStab updates with per-problem device scalars.
#include "common.h"

namespace ohm {

namespace {

__device__ __forceinline__ int xcd_block2(int w, int n)
{
    int q = n / NXCD, r = n % NXCD;
    int x = w % NXCD, i = w / NXCD;
    return x * q + min(x, r) + i;
}

template <typename T>
__global__ void k_fill(T *__restrict__ a, long long n, T v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = v;
}

template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ a, D *__restrict__ b, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (D)a[i];
}

// strided copy of one level (per-component strides differ between the user's
// per-level arrays and the multi-level vectors)
template <typename S, typename D>
__global__ void k_copy_level(const S *__restrict__ a, long long acs, D *__restrict__ b, long long bcs, long long n,
                             int ncomp, const int *__restrict__ hold)
{
    if (hold && *hold) return;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        for (int c = 0; c < ncomp; ++c) b[c * bcs + i] = (D)a[c * acs + i];
}

// per-block partial dots: q-th product is sum over the block of x[q] . y[q]
struct DotArgs {
    const double *x[3];
    const double *y[3];
    double *copy;   // when set, also receives x[0] (the products' operand, unchanged)
};

__global__ void __launch_bounds__(256)
k_dot(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs, DotArgs a, int nq,
      double *__restrict__ part)
{
    __shared__ double sred[3][4];
    const int b = xcd_block2(blockIdx.x, nblk);
    if (active && !active[prob_of[b]]) {
        if (threadIdx.x < nq) part[(long long)b * nq + threadIdx.x] = 0.0;
        return;
    }
    double acc[3] = {0, 0, 0};
    for (int t = threadIdx.x; t < 3 * NC; t += 256) {
        const int c = t / NC, cell = t % NC;
        const long long gi = c * cs + (long long)b * NC + cell;
        for (int q = 0; q < nq; ++q) acc[q] += a.x[q][gi] * a.y[q][gi];
        if (a.copy) a.copy[gi] = a.x[0][gi];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < nq; ++q) {
        double v = acc[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) sred[q][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        const int q = threadIdx.x;
        part[(long long)b * nq + q] = ((sred[q][0] + sred[q][1]) + sred[q][2]) + sred[q][3];
    }
}

// per-block sum of squares and max |x| per component -> part[b][6]
__global__ void __launch_bounds__(256)
k_norms(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs,
        const double *__restrict__ x, double *__restrict__ part)
{
    __shared__ double sred[6][4];
    const int b = xcd_block2(blockIdx.x, nblk);
    double ss[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    if (!(active && !active[prob_of[b]])) {
        for (int t = threadIdx.x; t < 3 * NC; t += 256) {
            const int c = t / NC;
            const double v = x[c * cs + (long long)b * NC + t % NC];
            ss[c] += v * v;
            mx[c] = fmax(mx[c], fabs(v));
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = 0; c < 3; ++c) {
        double a = ss[c], m = mx[c];
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_down(a, o, 64);
            m = fmax(m, __shfl_down(m, o, 64));
        }
        if (lane == 0) {
            sred[c][wv] = a;
            sred[3 + c][wv] = m;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = sred[k][0];
        for (int w = 1; w < 4; ++w) v = (k < 3) ? v + sred[k][w] : fmax(v, sred[k][w]);
        part[6 * (long long)b + k] = v;
    }
}

// Scalars per problem (double[SC_N]):
enum { SC_RHO = 0, SC_ALPHA, SC_OMEGA, SC_BETA, SC_RHONEW, SC_RR, SC_SS, SC_IT, SC_N = 16 };

// the result of a vector update, and optionally a copy of it in the
// multigrid cycle's precision (c32 or c64, same layout)
__device__ __forceinline__ void put(double *out, float *c32, double *c64, long long gi, double val)
{
    out[gi] = val;
    if (c32) c32[gi] = (float)val;
    if (c64) c64[gi] = val;
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(256)
k_bicg_p(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs,
         const double *__restrict__ scal, const double *__restrict__ r, const double *__restrict__ v,
         double *__restrict__ p, float *__restrict__ c32, double *__restrict__ c64)
{
    const int b = xcd_block2(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) return;
    const double beta = scal[SC_N * pr + SC_BETA], omega = scal[SC_N * pr + SC_OMEGA];
    if (beta == 0.0) {   // restart: p = r; p and v are not read (they hold no state yet)
        for (int t = threadIdx.x; t < 3 * NC; t += 256) {
            const long long gi = (t / NC) * cs + (long long)b * NC + t % NC;
            put(p, c32, c64, gi, r[gi]);
        }
        return;
    }
    for (int t = threadIdx.x; t < 3 * NC; t += 256) {
        const long long gi = (t / NC) * cs + (long long)b * NC + t % NC;
        put(p, c32, c64, gi, r[gi] + beta * (p[gi] - omega * v[gi]));
    }
}

// s = r - alpha v
__global__ void __launch_bounds__(256)
k_bicg_s(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs,
         const double *__restrict__ scal, const double *__restrict__ r, const double *__restrict__ v,
         double *__restrict__ s, float *__restrict__ c32, double *__restrict__ c64)
{
    const int b = xcd_block2(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) return;
    const double alpha = scal[SC_N * pr + SC_ALPHA];
    for (int t = threadIdx.x; t < 3 * NC; t += 256) {
        const long long gi = (t / NC) * cs + (long long)b * NC + t % NC;
        put(s, c32, c64, gi, r[gi] - alpha * v[gi]);
    }
}

// x += alpha ph + omega sh;  r = s - omega t;  partial (r, r) and (rhat, r)
__global__ void __launch_bounds__(256)
k_bicg_xr(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs,
          const double *__restrict__ scal, double *__restrict__ x, const double *__restrict__ ph,
          const double *__restrict__ sh, const double *__restrict__ s, const double *__restrict__ t_,
          double *__restrict__ r, const double *__restrict__ rhat, double *__restrict__ part)
{
    __shared__ double sred[2][4];
    const int b = xcd_block2(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) {
        if (threadIdx.x < 2) part[2 * (long long)b + threadIdx.x] = 0.0;
        return;
    }
    const double alpha = scal[SC_N * pr + SC_ALPHA], omega = scal[SC_N * pr + SC_OMEGA];
    double rr = 0.0, rh = 0.0;
    for (int t = threadIdx.x; t < 3 * NC; t += 256) {
        const long long gi = (t / NC) * cs + (long long)b * NC + t % NC;
        x[gi] += alpha * ph[gi] + omega * sh[gi];
        const double rn = s[gi] - omega * t_[gi];
        r[gi] = rn;
        rr += rn * rn;
        rh += rhat[gi] * rn;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        rr += __shfl_down(rr, o, 64);
        rh += __shfl_down(rh, o, 64);
    }
    if (lane == 0) {
        sred[0][wv] = rr;
        sred[1][wv] = rh;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        part[2 * (long long)b + threadIdx.x] =
            ((sred[threadIdx.x][0] + sred[threadIdx.x][1]) + sred[threadIdx.x][2]) + sred[threadIdx.x][3];
}

// x += y (iterative refinement update)
__global__ void __launch_bounds__(256)
k_axpy1(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs,
        double *__restrict__ x, const double *__restrict__ y)
{
    const int b = xcd_block2(blockIdx.x, nblk);
    if (active && !active[prob_of[b]]) return;
    for (int t = threadIdx.x; t < 3 * NC; t += 256) {
        const long long gi = (t / NC) * cs + (long long)b * NC + t % NC;
        x[gi] += y[gi];
    }
}

// x = (x + y) / 2 (the corrector of the explicit predictor-corrector step)
__global__ void __launch_bounds__(256)
k_mean2(int nblk, const int *__restrict__ prob_of, const int *__restrict__ active, long long cs,
        double *__restrict__ x, const double *__restrict__ y)
{
    const int b = xcd_block2(blockIdx.x, nblk);
    if (active && !active[prob_of[b]]) return;
    for (int t = threadIdx.x; t < 3 * NC; t += 256) {
        const long long gi = (t / NC) * cs + (long long)b * NC + t % NC;
        x[gi] = 0.5 * (x[gi] + y[gi]);
    }
}

// BiCGStab scalars of one problem from the reduced products d of the
// preceding dot kernel.  Stages 0 (restart) and 4 (after the x / r update)
// also form beta and rho for the next iteration's direction update.
__device__ __forceinline__ void scal_update(int stage, double *S, const double *d)
{
    switch (stage) {
    case 0:  // restart: rho = alpha = omega = 1, rho_new = (rhat, r) = (r, r)
        S[SC_RHO] = 1.0;
        S[SC_ALPHA] = 1.0;
        S[SC_OMEGA] = 1.0;
        S[SC_RHONEW] = d[0];
        S[SC_RR] = d[0];
        break;
    case 2:  // alpha = rho / (rhat, v)
        S[SC_ALPHA] = (d[0] != 0.0) ? S[SC_RHO] / d[0] : 0.0;
        break;
    case 3:  // omega = (t, s) / (t, t)
        S[SC_OMEGA] = (d[1] > 0.0) ? d[0] / d[1] : 0.0;
        break;
    case 4:  // after x/r update: d = {(r, r), (rhat, r)}
        S[SC_RR] = d[0];
        S[SC_RHONEW] = d[1];
        break;
    }
    if (stage == 0 || stage == 4) {  // beta from rho_new; rho <- rho_new
        const double rn = S[SC_RHONEW];
        S[SC_BETA] = (rn / S[SC_RHO]) * (S[SC_ALPHA] / S[SC_OMEGA]);
        S[SC_RHO] = rn;
    }
    // a restart starts the direction from p = v = 0, so its first p is r: the
    // direction update takes beta = 0 as "p = r" and reads neither p nor v
    if (stage == 0) S[SC_BETA] = 0.0;
}

// Per-problem sums of k block partials (part[block][k]) followed by the
// scalar update of `stage` (stage < 0: sums only).  One workgroup per problem,
// 256 threads per quantity; every sum is formed exactly as by the block
// reduction kernel (thread t owns the problem-local indices = t mod 256, wave
// shuffle, then the 4 wavefronts in order), so results do not depend on the
// other problems of the handle.  Every problem's iteration count (SC_IT) is
// reset by stage 0 and advanced by stage 4, active or not, so that the ring
// slot of an iteration is the same for all problems.
__global__ void __launch_bounds__(1024)
k_reduce_scal(int nrange, const long long *__restrict__ range, const double *__restrict__ part, int k,
              double *__restrict__ out, int stage, const int *active, double *__restrict__ scal, IterRing ring)
{
    __shared__ double sred[4][4];
    const int p = blockIdx.x;
    const int g = threadIdx.x >> 8, tid = threadIdx.x & 255;
    if (g < k) {
        double v = 0.0;
        long long base = 0;
        for (int r = 0; r < nrange; ++r) {
            const long long b0 = range[2 * ((long long)p * nrange + r)], b1 = range[2 * ((long long)p * nrange + r) + 1];
            const long long n = b1 - b0;
            const long long first = ((tid - base) % 256 + 256) % 256;
            // eight loads in flight, then the adds in index order
            long long i = first;
            for (; i + 7 * 256 < n; i += 8 * 256) {
                double a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = part[(b0 + i + 256 * u) * k + g];
#pragma unroll
                for (int u = 0; u < 8; ++u) v = v + a[u];
            }
            for (; i < n; i += 256) v = v + part[(b0 + i) * k + g];
            base += n;
        }
        for (int o = 32; o > 0; o >>= 1) v = v + __shfl_down(v, o, 64);
        if ((tid & 63) == 0) sred[g][tid >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d[4];
        for (int q = 0; q < k; ++q) {
            double t = sred[q][0];
            for (int w = 1; w < 4; ++w) t = t + sred[q][w];
            d[q] = t;
            out[(long long)p * k + q] = t;
        }
        double *S = scal + SC_N * p;
        const bool on = !(active && !active[p]);
        if (stage >= 0 && on) scal_update(stage, S, d);
        if (stage == 0) S[SC_IT] = 0.0;
        if (stage == 4 && ring.buf) {
            const int it = (int)S[SC_IT];
            double *slot = ring.buf + 2 * ((long long)gridDim.x * (it % ITER_SLOTS) + p);
            slot[0] = d[0];
            slot[1] = d[1];
            S[SC_IT] = (double)(it + 1);
            if (on && !(d[0] > ring.tol2[p])) ring.flags[p] = 0;
            if (on && !isfinite(d[0])) *ring.hold = 1;
        }
    }
}

// convergence thresholds and the initial active set (see launch_conv_init)
__global__ void k_conv_init(int nprob, const double *__restrict__ dots, double rtol, double *__restrict__ tol2,
                            int *__restrict__ active, int *__restrict__ hold)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    const double t = rtol * rtol * fmax(dots[2 * p + 1], 1e-300);
    tol2[p] = t;
    if (!(dots[2 * p] > t)) active[p] = 0;
    if (!isfinite(dots[2 * p])) *hold = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
static inline int grid_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 8192); }

template <typename T>
ohm_status vfill(T *a, long long n, T v, hipStream_t s)
{
    if (n <= 0) return OHM_OK;
    k_fill<T><<<grid_for(n), 256, 0, s>>>(a, n, v);
    return check_launch("fill");
}

template <typename S, typename D>
ohm_status vconvert(const S *a, D *b, long long n, hipStream_t s)
{
    if (n <= 0) return OHM_OK;
    k_convert<S, D><<<grid_for(n), 256, 0, s>>>(a, b, n);
    return check_launch("convert");
}

template <typename S, typename D>
ohm_status vcopy_level(const S *a, long long acs, D *b, long long bcs, long long n, int ncomp, hipStream_t s,
                       const int *hold)
{
    if (n <= 0) return OHM_OK;
    k_copy_level<S, D><<<grid_for(n), 256, 0, s>>>(a, acs, b, bcs, n, ncomp, hold);
    return check_launch("copy level");
}

ohm_status vdot(int nblk, const int *prob_of, const int *active, long long cs, const double *const *x,
                const double *const *y, int nq, double *part, hipStream_t s, double *copy)
{
    DotArgs a;
    a.copy = copy;
    for (int q = 0; q < 3; ++q) {
        a.x[q] = q < nq ? x[q] : nullptr;
        a.y[q] = q < nq ? y[q] : nullptr;
    }
    k_dot<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, a, nq, part);
    return check_launch("dot");
}

ohm_status vbicg_p(int nblk, const int *prob_of, const int *active, long long cs, const double *scal, const double *r,
                   const double *v, double *p, hipStream_t s, float *c32, double *c64)
{
    k_bicg_p<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, scal, r, v, p, c32, c64);
    return check_launch("bicg p");
}

ohm_status vbicg_s(int nblk, const int *prob_of, const int *active, long long cs, const double *scal, const double *r,
                   const double *v, double *sv, hipStream_t s, float *c32, double *c64)
{
    k_bicg_s<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, scal, r, v, sv, c32, c64);
    return check_launch("bicg s");
}

ohm_status vbicg_xr(int nblk, const int *prob_of, const int *active, long long cs, const double *scal, double *x,
                    const double *ph, const double *sh, const double *sv, const double *t, double *r,
                    const double *rhat, double *part, hipStream_t s)
{
    k_bicg_xr<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, scal, x, ph, sh, sv, t, r, rhat, part);
    return check_launch("bicg xr");
}

ohm_status launch_reduce_scal(int nprob, int nrange, const long long *range_dev, const double *part, int k,
                              double *out, int stage, const int *active, double *scal, hipStream_t s, IterRing ring)
{
    if (k < 1 || k > 4) return fail(OHM_ERR_ARG, "reduce + scalars takes 1 to 4 quantities, got %d", k);
    if (ring.buf && (stage != 4 || k < 2 || !ring.flags || !ring.tol2 || !ring.hold))
        return fail(OHM_ERR_ARG, "the iteration ring is written by stage 4 with two norms and needs flags and thresholds");
    k_reduce_scal<<<nprob, 256 * k, 0, s>>>(nrange, range_dev, part, k, out, stage, active, scal, ring);
    return check_launch("reduce + scalars");
}

ohm_status launch_conv_init(int nprob, const double *dots, double rtol, double *tol2, int *active, int *hold,
                            hipStream_t s)
{
    k_conv_init<<<(nprob + 63) / 64, 64, 0, s>>>(nprob, dots, rtol, tol2, active, hold);
    return check_launch("convergence thresholds");
}

ohm_status vmean2(int nblk, const int *prob_of, const int *active, long long cs, double *x, const double *y,
                  hipStream_t s)
{
    k_mean2<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, x, y);
    return check_launch("mean of two vectors");
}

ohm_status vaxpy1(int nblk, const int *prob_of, const int *active, long long cs, double *x, const double *y,
                  hipStream_t s)
{
    k_axpy1<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, x, y);
    return check_launch("axpy");
}


ohm_status vnorms(int nblk, const int *prob_of, const int *active, long long cs, const double *x, double *part,
                  hipStream_t s)
{
    k_norms<<<nblk, 256, 0, s>>>(nblk, prob_of, active, cs, x, part);
    return check_launch("norms");
}

int scal_stride() { return SC_N; }

template ohm_status vfill<double>(double *, long long, double, hipStream_t);
template ohm_status vfill<float>(float *, long long, float, hipStream_t);
template ohm_status vfill<int>(int *, long long, int, hipStream_t);
template ohm_status vconvert<double, float>(const double *, float *, long long, hipStream_t);
template ohm_status vconvert<float, double>(const float *, double *, long long, hipStream_t);
template ohm_status vconvert<double, double>(const double *, double *, long long, hipStream_t);
template ohm_status vconvert<float, float>(const float *, float *, long long, hipStream_t);
template ohm_status vcopy_level<double, double>(const double *, long long, double *, long long, long long, int,
                                                 hipStream_t, const int *);
template ohm_status vcopy_level<double, float>(const double *, long long, float *, long long, long long, int,
                                                hipStream_t, const int *);

}  // namespace ohm
