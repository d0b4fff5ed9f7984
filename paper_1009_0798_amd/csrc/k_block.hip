// Kernels on the 8^3-cell blocks of AMR levels: operator apply, residual and
// red-black half-sweep (one workgroup per block, block plus a one-cell face and
// edge halo staged in LDS), restriction, prolongation, coarse-fine ghost fill,
// refluxing and per-problem norm reductions.
#include "common.h"
#include <type_traits>
#include "stencil.h"
#include "sweep.h"

namespace ohm {

namespace {

constexpr int TW = NB + 2;             // tile edge with a one-cell halo
constexpr int TC = TW * TW * TW;       // tile cells

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// run of blocks (blocks are in Z-order, so a compact region whose halo stays
// in that XCD's L2).
__device__ __forceinline__ int xcd_block(int w, int n)
{
    int q = n / NXCD, r = n % NXCD;
    int x = w % NXCD, i = w / NXCD;
    return x * q + min(x, r) + i;
}

__device__ __forceinline__ int side(int c) { return c < 0 ? -1 : (c >= NB ? 1 : 0); }

// B (3 components) and eta of block b plus the one-cell halo into LDS: thread
// u < 200 owns tile column (x, y) = u mod 100 and five consecutive z, issues
// all its global loads, then stores them (ghost blocks for negative
// neighbour entries, zeros for absent corner blocks)
template <typename T>
__device__ __forceinline__ void load_tile_b_eta(T (*sB)[TC], T *sE, const T *f, const T *g, long long cs,
                                                long long gcs, const T *eta, const T *etag, const int *nbr)
{
    const int u = threadIdx.x;
    if (u >= 2 * TW * TW) return;
    const int col = u % (TW * TW), zh = u / (TW * TW);
    const int x = col % TW - 1, y = col / TW - 1;
    const int sx = side(x), sy = side(y);
    const int lxy = (x - NB * sx) + NB * (y - NB * sy);
    const int sxy = (sx + 1) + 3 * (sy + 1);
    T v[5][4];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int z = 5 * zh + k - 1, sz = side(z);
        const int n = nbr[sxy + 9 * (sz + 1)];
        const int li = lxy + NB * NB * (z - NB * sz);
        if (n >= 0) {
            const long long gi = (long long)n * NC + li;
            v[k][0] = f[gi];
            v[k][1] = f[cs + gi];
            v[k][2] = f[2 * cs + gi];
            v[k][3] = eta[gi];
        } else if (n != NBR_NONE) {
            const long long gi = (long long)(-1 - n) * NC + li;
            v[k][0] = g[gi];
            v[k][1] = g[gcs + gi];
            v[k][2] = g[2 * gcs + gi];
            v[k][3] = etag[gi];
        } else {
            v[k][0] = v[k][1] = v[k][2] = v[k][3] = T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int t = col + TW * TW * (5 * zh + k);
        sB[0][t] = v[k][0];
        sB[1][t] = v[k][1];
        sB[2][t] = v[k][2];
        sE[t] = v[k][3];
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256)
k_blk_stencil(int nblk, const int *__restrict__ nbr_tab, const int *__restrict__ prob_of,
              const uint8_t *__restrict__ cov_zero, const int *__restrict__ active,
              const double *__restrict__ inv_h2_p, const double *__restrict__ coef_p,
              const T *__restrict__ B, const T *__restrict__ Bg, long long cs, long long gcs,
              const T *__restrict__ S, const T *__restrict__ eta, const T *__restrict__ etag,
              T *__restrict__ out, int colour, double *__restrict__ partials, StencilDots dots,
              const int *__restrict__ dense_map, const DenseProbDev *__restrict__ dp, long long ccs)
{
    __shared__ T sB[3][TC];
    __shared__ T sE[1][TC];
    __shared__ int snbr[27];
    __shared__ double sred[6][4];
    const int b = xcd_block(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) {
        if (MODE == MODE_APPLY && threadIdx.x < dots.ndot) dots.dot_part[(long long)b * dots.ndot + threadIdx.x] = 0.0;
        return;
    }
    if (threadIdx.x < 27) snbr[threadIdx.x] = nbr_tab[27 * (long long)b + threadIdx.x];
    __syncthreads();
    load_tile_b_eta<T>(sB, sE[0], B, Bg, cs, gcs, eta, etag, snbr);
    // values read per cell after the stencil (S, or the other vector of the
    // first fused dot product that has one), loaded with the tile so that
    // their latency overlaps it
    constexpr bool HAS_S = MODE == MODE_RESID || MODE == MODE_RESID_RESTRICT || MODE == MODE_SMOOTH;
    T pS[2][3];
    double pY[2][3];
    int qy = -1;
    if (HAS_S) {
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
            for (int c = 0; c < 3; ++c) pS[half][c] = S[c * cs + (long long)b * NC + threadIdx.x + 256 * half];
    }
    if (MODE == MODE_APPLY) {
        for (int q = dots.ndot - 1; q >= 0; --q)
            if (dots.dot_y[q]) qy = q;
        if (qy >= 0)
#pragma unroll
            for (int half = 0; half < 2; ++half)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    pY[half][c] = dots.dot_y[qy][c * cs + (long long)b * NC + threadIdx.x + 256 * half];
    }
    __syncthreads();
    const T cih2 = T(coef_p[pr]) * T(inv_h2_p[pr]);
    const T c8 = cih2 * T(0.125), c2 = cih2 * T(0.5);
    const uint8_t cov = cov_zero ? cov_zero[b] : 0;
    double ss[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    T o[2][3];   // outputs kept for the fused dot products / restriction
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int cell = threadIdx.x + 256 * half;
        const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
        const int p = (x + 1) + TW * ((y + 1) + TW * (z + 1));
        const bool zero = (cov >> ((x >> 2) + 2 * (y >> 2) + 4 * (z >> 2))) & 1;
        const long long gi = (long long)b * NC + cell;
        T dvs[3], als[3];
        divF_all<T, TW>(sB[0], sB[1], sB[2], sE[0], p, dvs, als);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T LB = fma(c8, dvs[c], sB[c][p]);
            if (MODE == MODE_APPLY) {
                o[half][c] = zero ? T(0) : LB;
                out[c * cs + gi] = o[half][c];
            } else if (MODE == MODE_RESID_RESTRICT) {
                o[half][c] = zero ? T(0) : pS[half][c] - LB;
            } else if (MODE == MODE_RESID) {
                T r = zero ? T(0) : pS[half][c] - LB;
                if (out) out[c * cs + gi] = r;
                double rd = (double)r;
                ss[c] += rd * rd;
                mx[c] = fmax(mx[c], fabs(rd));
            } else {  // smoother half-sweep
                T v = sB[c][p];
                if (in_colour(x, y, z, colour)) v = relax_point(v, pS[half][c], dvs[c], als[c], c8, c2);
                out[c * cs + gi] = v;
            }
        }
    }
    if (MODE == MODE_APPLY && dots.ndot > 0) {
        // the stand-alone dot kernel's order: thread t sums its elements
        // (component 0, cells t and t + 256), (component 1, ...), (component 2, ...)
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int q = 0; q < dots.ndot; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const long long gi = (long long)b * NC + threadIdx.x + 256 * half;
                    const double y = q == qy ? pY[half][c]
                                     : (dots.dot_y[q] ? dots.dot_y[q][c * cs + gi] : (double)o[half][c]);
                    acc += (double)o[half][c] * y;
                }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if (lane == 0) sred[q][wv] = acc;
        }
        __syncthreads();
        if (threadIdx.x < dots.ndot) {
            const int q = threadIdx.x;
            dots.dot_part[(long long)b * dots.ndot + q] = ((sred[q][0] + sred[q][1]) + sred[q][2]) + sred[q][3];
        }
    }
    if (MODE == MODE_RESID_RESTRICT) {
        // r through LDS (the tile is no longer needed), then the mean of the 8
        // children of each coarse cell in the order of the restriction kernel
        __syncthreads();
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
            for (int c = 0; c < 3; ++c) sB[c][threadIdx.x + 256 * half] = o[half][c];
        __syncthreads();
        if (threadIdx.x < 64) {
            const int t = threadIdx.x;
            const int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
            const DenseProbDev q = dp[pr];
            const long long cidx = dense_map[b] + i + (long long)q.nx * (j + (long long)q.ny * k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T a = T(0);
#pragma unroll
                for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 2; ++dx) a += sB[c][(2 * i + dx) + NB * ((2 * j + dy) + NB * (2 * k + dz))];
                out[c * ccs + cidx] = a * T(0.125);
            }
        }
    }
    if (MODE == MODE_RESID && partials) {
        // wavefront reduction, then across the 4 wavefronts in fixed order
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
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
            int k = threadIdx.x;
            double v = sred[k][0];
            for (int w = 1; w < 4; ++w) v = (k < 3) ? v + sred[k][w] : fmax(v, sred[k][w]);
            partials[6 * (long long)b + k] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused red-black sweep on the blocks of a level whose blocks have all 26
// neighbours (the tile body is in sweep.h, shared with the dense levels)
// ---------------------------------------------------------------------------
struct BlockAddr {
    static constexpr bool ghosts = false;
    const int *nbr;   // 27 neighbour entries of the block (LDS)
    int b;
    __device__ __forceinline__ long long at(int x, int y, int z) const
    {
        const int sx = side(x), sy = side(y), sz = side(z);
        const int n = nbr[(sx + 1) + 3 * (sy + 1) + 9 * (sz + 1)];
        return (long long)n * NC + (x - NB * sx) + NB * ((y - NB * sy) + NB * (z - NB * sz));
    }
};

// Same, on a level whose neighbour entries may name coarse-fine ghost blocks
// (never absent ones); at() is used for level cells only.
template <typename T>
struct GhostBlockAddr {
    static constexpr bool ghosts = true;
    const int *nbr;
    const T *G;       // ghost blocks, component stride gcs
    long long gcs;
    const T *EG;      // resistivity of the ghost blocks
    __device__ __forceinline__ int entry(int x, int y, int z) const
    {
        return nbr[(side(x) + 1) + 3 * (side(y) + 1) + 9 * (side(z) + 1)];
    }
    __device__ __forceinline__ int local(int x, int y, int z) const
    {
        const int sx = side(x), sy = side(y), sz = side(z);
        return (x - NB * sx) + NB * ((y - NB * sy) + NB * (z - NB * sz));
    }
    __device__ __forceinline__ long long at(int x, int y, int z) const
    {
        return (long long)entry(x, y, z) * NC + local(x, y, z);
    }
};

// DIRECT (plain FP64 sweeps, MODE 0): the tile is staged by loads that write
// LDS directly instead of passing through registers.
// MODE 0: sweep B -> out; 1: zero input (B not read); 2: sweep of B plus the
// prolonged correction from the first dense level (coarse), B -> out; MODE 3
// and 4 as 0 and 1 on a level with coarse-fine ghost blocks (Bg, etag).  With
// O64 (MODE 0 or 2 of an FP32 sweep) the result is written as FP64 to out64.
template <typename T, int MODE, bool O64 = false, bool DIRECT = false>
__global__ void __launch_bounds__(SWEEP_THREADS)
k_blk_sweep(int nblk, const int *__restrict__ nbr_tab, const int *__restrict__ prob_of,
            const int *__restrict__ active, const double *__restrict__ inv_h2_p, const double *__restrict__ coef_p,
            const T *__restrict__ B, long long cs, const T *__restrict__ S, const T *__restrict__ eta,
            T *__restrict__ out, const int *__restrict__ ijk, const DenseProbDev *__restrict__ dp,
            const T *__restrict__ coarse, long long ccs, const T *__restrict__ Bg, long long gcs,
            const T *__restrict__ etag, double *__restrict__ out64 = nullptr)
{
    constexpr int TS = DIRECT ? TC2 + 64 : TC2;
    __shared__ T sB[3][TS];
    __shared__ T sE[TS];
    __shared__ T sC[MODE == 2 ? 3 * 512 : 1];
    __shared__ int snbr[27];
    const int b = xcd_block(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) return;
    if (threadIdx.x < 27) snbr[threadIdx.x] = nbr_tab[27 * (long long)b + threadIdx.x];
    __syncthreads();
    const T cih2 = T(coef_p[pr]) * T(inv_h2_p[pr]);
    if constexpr (DIRECT) {
        const BlockAddr A{snbr, b};
        fused_sweep_tile<T, false, BlockAddr, NoCoarse<T>, T, TS, true>(A, B, cs, S, eta, out, cih2, sB, sE);
        return;
    } else {
    if constexpr (MODE >= 3) {
        const GhostBlockAddr<T> A{snbr, Bg, gcs, etag};
        fused_sweep_tile<T, MODE == 4>(A, B, cs, S, eta, out, cih2, sB, sE);
    } else if constexpr (MODE == 2) {
        const BlockAddr A{snbr, b};
        TileCoarse<T> cor{coarse, ccs, dp[pr], 4 * ijk[3 * b] - 2, 4 * ijk[3 * b + 1] - 2, 4 * ijk[3 * b + 2] - 2,
                          sC, {}};
        if constexpr (O64)
            fused_sweep_tile<T, false, BlockAddr, TileCoarse<T>, double>(A, B, cs, S, eta, out64, cih2, sB, sE, cor);
        else
            fused_sweep_tile<T, false>(A, B, cs, S, eta, out, cih2, sB, sE, cor);
    } else {
        const BlockAddr A{snbr, b};
        if constexpr (O64)
            fused_sweep_tile<T, MODE == 1, BlockAddr, NoCoarse<T>, double>(A, B, cs, S, eta, out64, cih2, sB, sE);
        else
            fused_sweep_tile<T, MODE == 1>(A, B, cs, S, eta, out, cih2, sB, sE);
    }
    }
}

// ---------------------------------------------------------------------------
// restriction: fine block -> the octant of its parent block (AMR levels), and
// level-0 block -> the first dense level
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64)
k_restrict_blk(int nfine, const int *__restrict__ parent, const int *__restrict__ octant,
               const int *__restrict__ fprob, const int *__restrict__ active, const T *__restrict__ fine,
               long long fcs, T *__restrict__ coarse, long long ccs, int ncomp)
{
    const int b = xcd_block(blockIdx.x, nfine);
    if (active && !active[fprob[b]]) return;
    const int t = threadIdx.x;          // 4^3 coarse cells of the octant
    const int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
    const int o = octant[b];
    const int ci = 4 * (o & 1) + i, cj = 4 * ((o >> 1) & 1) + j, ck = 4 * (o >> 2) + k;
    const long long cidx = (long long)parent[b] * NC + ci + NB * (cj + NB * ck);
    for (int c = 0; c < ncomp; ++c) {
        const T *f = fine + c * fcs + (long long)b * NC;
        T s = T(0);
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) s += f[(2 * i + dx) + NB * ((2 * j + dy) + NB * (2 * k + dz))];
        coarse[c * ccs + cidx] = s * T(0.125);
    }
}

template <typename T>
__global__ void __launch_bounds__(64)
k_restrict_blk0_dense(int nblk, const int *__restrict__ dense_map, const int *__restrict__ prob_of,
                      const DenseProbDev *__restrict__ dp, const int *__restrict__ active,
                      const T *__restrict__ fine, long long fcs, T *__restrict__ coarse, long long ccs,
                      int ncomp)
{
    const int b = xcd_block(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) return;
    const int t = threadIdx.x;
    const int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
    const DenseProbDev q = dp[pr];
    const long long cidx = dense_map[b] + i + (long long)q.nx * (j + (long long)q.ny * k);
    for (int c = 0; c < ncomp; ++c) {
        const T *f = fine + c * fcs + (long long)b * NC;
        T s = T(0);
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) s += f[(2 * i + dx) + NB * ((2 * j + dy) + NB * (2 * k + dz))];
        coarse[c * ccs + cidx] = s * T(0.125);
    }
}

// ---------------------------------------------------------------------------
// prolongation (cell-centred trilinear, 27/9/3/1 over 64) into fine blocks or
// ghost blocks from their parent block (and its neighbours) one level coarser
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_prolong_blk(int nfine, const int *__restrict__ parent, const int *__restrict__ octant,
              const int *__restrict__ fprob, const int *__restrict__ active, const int *__restrict__ cnbr,
              const T *__restrict__ coarse, long long ccs, T *__restrict__ fine, long long fcs, int ncomp,
              int accumulate)
{
    // coarse region of the octant plus a one-cell halo: 6^3 cells
    __shared__ T sc[3][216];
    __shared__ int snbr[27];
    const int b = xcd_block(blockIdx.x, nfine);
    if (active && !active[fprob[b]]) return;
    const int pb = parent[b];
    const int o = octant[b];
    const int ox = 4 * (o & 1), oy = 4 * ((o >> 1) & 1), oz = 4 * (o >> 2);
    if (threadIdx.x < 27) snbr[threadIdx.x] = cnbr[27 * (long long)pb + threadIdx.x];
    __syncthreads();
    for (int t = threadIdx.x; t < 216; t += blockDim.x) {
        int x = ox - 1 + t % 6, y = oy - 1 + (t / 6) % 6, z = oz - 1 + t / 36;
        int sx = side(x), sy = side(y), sz = side(z);
        int n = snbr[(sx + 1) + 3 * (sy + 1) + 9 * (sz + 1)];
        int li = (x - NB * sx) + NB * ((y - NB * sy) + NB * (z - NB * sz));
        for (int c = 0; c < ncomp; ++c) sc[c][t] = (n >= 0) ? coarse[c * ccs + (long long)n * NC + li] : T(0);
    }
    __syncthreads();
    for (int cell = threadIdx.x; cell < NC; cell += blockDim.x) {
        const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
        // parent cell in the 6^3 tile and the side of the fine cell
        const int px = (x >> 1) + 1, py = (y >> 1) + 1, pz = (z >> 1) + 1;
        const int sx = (x & 1) ? 1 : -1, sy = (y & 1) ? 1 : -1, sz = (z & 1) ? 1 : -1;
        const int p0 = px + 6 * (py + 6 * pz);
        const int qx = sx, qy = 6 * sy, qz = 36 * sz;
        for (int c = 0; c < ncomp; ++c) {
            const T *C = sc[c];
            T v = T(27) * C[p0] + T(9) * (C[p0 + qx] + C[p0 + qy] + C[p0 + qz]) +
                  T(3) * (C[p0 + qx + qy] + C[p0 + qx + qz] + C[p0 + qy + qz]) + C[p0 + qx + qy + qz];
            v *= T(1.0 / 64.0);
            const long long gi = c * fcs + (long long)b * NC + cell;
            fine[gi] = accumulate ? fine[gi] + v : v;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_prolong_dense_blk0(int nblk, const int *__restrict__ ijk, const int *__restrict__ prob_of,
                     const DenseProbDev *__restrict__ dp, const int *__restrict__ active,
                     const T *__restrict__ coarse, long long ccs, const T *base, T *fine, long long fcs,
                     int ncomp)
{
    // the 6^3 coarse cells the block's 8^3 fine cells interpolate from (its
    // 4^3 parents and one layer around them, periodic) are staged in LDS
    __shared__ T sc[3][216];
    const int b = xcd_block(blockIdx.x, nblk);
    const int pr = prob_of[b];
    if (active && !active[pr]) return;
    const DenseProbDev q = dp[pr];
    const int bi = ijk[3 * b], bj = ijk[3 * b + 1], bk = ijk[3 * b + 2];
    const int i0 = 4 * bi - 1, j0 = 4 * bj - 1, k0 = 4 * bk - 1;
    for (int t = threadIdx.x; t < 216 * ncomp; t += blockDim.x) {
        const int c = t / 216, r = t % 216;
        const int i = (i0 + r % 6 + q.nx) % q.nx, j = (j0 + (r / 6) % 6 + q.ny) % q.ny, k = (k0 + r / 36 + q.nz) % q.nz;
        sc[c][r] = coarse[c * ccs + q.off + i + (long long)q.nx * (j + (long long)q.ny * k)];
    }
    __syncthreads();
    for (int cell = threadIdx.x; cell < NC; cell += blockDim.x) {
        const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
        // parent (local index 1..4 on each axis) and its neighbour on the child's side
        const int i = (x >> 1) + 1, j = (y >> 1) + 1, k = (z >> 1) + 1;
        const int i1 = i + ((x & 1) ? 1 : -1), j1 = j + ((y & 1) ? 1 : -1), k1 = k + ((z & 1) ? 1 : -1);
        auto at = [](int a, int bb, int cc) { return a + 6 * (bb + 6 * cc); };
        for (int c = 0; c < ncomp; ++c) {
            const T *C = sc[c];
            T v = T(27) * C[at(i, j, k)] + T(9) * (C[at(i1, j, k)] + C[at(i, j1, k)] + C[at(i, j, k1)]) +
                  T(3) * (C[at(i1, j1, k)] + C[at(i1, j, k1)] + C[at(i, j1, k1)]) + C[at(i1, j1, k1)];
            v *= T(1.0 / 64.0);
            const long long gi = c * fcs + (long long)b * NC + cell;
            fine[gi] = base ? base[gi] + v : v;
        }
    }
}

// ---------------------------------------------------------------------------
// refluxing (section 4): one thread per coarse leaf cell with coarse-fine faces
// ---------------------------------------------------------------------------
// value of component c at local coordinates (x,y,z) in [-1, 8] of block b
template <typename T>
__device__ __forceinline__ T fetch(const T *f, const T *g, long long cs, long long gcs, const int *nbr_tab,
                                   int b, int x, int y, int z, int c)
{
    int sx = side(x), sy = side(y), sz = side(z);
    int n = b;
    if (sx | sy | sz) n = nbr_tab[27 * (long long)b + (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1)];
    int li = (x - NB * sx) + NB * ((y - NB * sy) + NB * (z - NB * sz));
    if (n >= 0) return f[c * cs + (long long)n * NC + li];
    return g[c * gcs + (long long)(-1 - n) * NC + li];
}

// flux F_d[c] times h through the face between cell q and q + e_d (q local to
// block b, possibly one cell outside it)
template <typename T>
__device__ T face_flux_h(const T *Bf, const T *Bg, long long cs, long long gcs, const T *E, const T *Eg,
                         const int *nbr_tab, int b, const int q[3], int d, int c)
{
    int a[3] = {q[0], q[1], q[2]};
    int qd[3] = {q[0], q[1], q[2]};
    qd[d] += 1;
    auto F = [&](const int r[3], int comp) { return fetch<T>(Bf, Bg, cs, gcs, nbr_tab, b, r[0], r[1], r[2], comp); };
    auto Ee = [&](const int r[3]) { return fetch<T>(E, Eg, 0, 0, nbr_tab, b, r[0], r[1], r[2], 0); };
    T ef = (Ee(a) + Ee(qd)) * T(0.5);
    int p1[3] = {a[0], a[1], a[2]}, p2[3] = {a[0], a[1], a[2]}, p3[3] = {qd[0], qd[1], qd[2]},
        p4[3] = {qd[0], qd[1], qd[2]};
    p1[c] += 1;
    p2[c] -= 1;
    p3[c] += 1;
    p4[c] -= 1;
    T tr = (F(p1, d) + F(p3, d) - F(p2, d) - F(p4, d)) * T(0.25);
    return ef * (tr - (F(qd, c) - F(a, c)));
}

// Refluxing.  An entry is a leaf cell of level l with faces next to covered
// cells; each such face needs, for both tangential components, the coarse
// flux and the four fine fluxes through it.  A workgroup takes whole entries
// (at most RF_WG_FACES faces) and gives every one of the ten fluxes of a face
// its own thread, so each thread's loads are one neighbour lookup deep.  The
// face corrections and the entry sums are then formed in fixed orders: fine
// fluxes in child order, faces in face order.
template <typename T>
__global__ void __launch_bounds__(RF_WG_FACES * 10)
k_reflux(const int *__restrict__ rfw, const int *__restrict__ rff, const int *__restrict__ rfs,
         const int *__restrict__ rf, const int *__restrict__ active, const int *__restrict__ cnbr,
         const int *__restrict__ fnbr, const double *__restrict__ inv_h_c, const double *__restrict__ coef_p,
         const T *__restrict__ Bc, long long ccs, const T *__restrict__ Ec, const T *__restrict__ Bf,
         long long fcs, const T *__restrict__ Bfg, long long fgcs, const T *__restrict__ Ef,
         const T *__restrict__ Efg, T *__restrict__ out)
{
    __shared__ T sfl[RF_WG_FACES * 10];
    __shared__ T sadd[RF_WG_FACES][2];
    const int e0 = rfw[4 * blockIdx.x], ne = rfw[4 * blockIdx.x + 1], f0 = rfw[4 * blockIdx.x + 2],
              nf = rfw[4 * blockIdx.x + 3];
    const int t = threadIdx.x;
    // one flux: face i, tangential component ci (c = d + 1 + ci mod 3), k = 0
    // the coarse face, k = 1..4 the fine faces (children a1, a2 = (k-1)/2, (k-1)%2)
    {
        const int i = t / 10, ci = (t % 10) / 5, k = t % 5;
        if (i < nf) {
            const int it = rff[f0 + i];
            const int *ent = rf + RF_INTS * (long long)(it >> 3);
            const int f = it & 7, d = f >> 1, sg = (f & 1) ? -1 : 1;
            const int c = (d + 1 + ci) % 3;
            const int pr = ent[15];
            T v = T(0);
            if (!(active && !active[pr])) {
                if (k == 0) {
                    // coarse face: after cell p (sg = +1) or after p - e_d; a
                    // null coarse field stands for zero
                    const int cell = ent[1];
                    int q[3] = {cell & 7, (cell >> 3) & 7, cell >> 6};
                    if (sg < 0) q[d] -= 1;
                    if (Bc) v = face_flux_h<T>(Bc, Bc, ccs, ccs, Ec, Ec, cnbr, ent[0], q, d, c);
                } else {
                    // fine faces: the covered-side children start at the entry's
                    // fine base cell; the face is after the child (sg < 0) or
                    // after the child - e_d (sg > 0)
                    const int fbase = ent[9 + f];
                    int q[3] = {fbase & 7, (fbase >> 3) & 7, fbase >> 6};
                    q[(d + 1) % 3] += (k - 1) >> 1;
                    q[(d + 2) % 3] += (k - 1) & 1;
                    if (sg > 0) q[d] -= 1;
                    v = face_flux_h<T>(Bf, Bfg, fcs, fgcs, Ef, Efg, fnbr, ent[3 + f], q, d, c);
                }
            }
            sfl[t] = v;
        }
    }
    __syncthreads();
    // face correction per tangential component: sg (<F_fine> - F_coarse) / h
    if (t < 2 * nf) {
        const int i = t >> 1, ci = t & 1;
        const int it = rff[f0 + i];
        const int sg = (it & 1) ? -1 : 1;
        const T ih = T(inv_h_c[rf[RF_INTS * (long long)(it >> 3) + 15]]);  // fine fluxes carry h_f = h/2
        const T *fl = sfl + 10 * i + 5 * ci;
        const T Fc = fl[0] * ih;
        T Ff = fl[1];
        Ff += fl[2];
        Ff += fl[3];
        Ff += fl[4];
        Ff *= T(0.25) * (ih * T(2));
        sadd[i][ci] = T(sg) * (Ff - Fc) * ih;
    }
    __syncthreads();
    if (t < ne) {
        const int e = e0 + t;
        const int *en = rf + RF_INTS * (long long)e;
        const int pr = en[15];
        if (!(active && !active[pr])) {
            const T coef = T(coef_p[pr]);
            const int mask = en[2];
            const long long gi = (long long)en[0] * NC + en[1];
            T a[3] = {T(0), T(0), T(0)};
            int i = rfs[e] - f0;
            for (int ff = 0; ff < 6; ++ff)
                if ((mask >> ff) & 1) {
                    const int d = ff >> 1;
                    a[(d + 1) % 3] += sadd[i][0];
                    a[(d + 2) % 3] += sadd[i][1];
                    ++i;
                }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (a[c] != T(0)) out[c * ccs + gi] += coef * a[c];
        }
    }
}

template <typename T>
__global__ void k_zero_covered(int nblk, const uint8_t *__restrict__ cov, T *__restrict__ out, long long cs,
                               int ncomp)
{
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const uint8_t m = cov[b];
    if (!m) return;
    for (int cell = threadIdx.x; cell < NC; cell += blockDim.x) {
        const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
        if ((m >> ((x >> 2) + 2 * (y >> 2) + 4 * (z >> 2))) & 1)
            for (int c = 0; c < ncomp; ++c) out[c * cs + (long long)b * NC + cell] = T(0);
    }
}

// per-problem reduction of per-block partials (sums for k < ksum, max after):
// one workgroup per (problem, quantity); each thread walks a fixed strided
// subset of the problem's blocks (ranges per AMR level, in order), then a
// fixed-shape tree combines the threads -- the result depends only on the
// problem's own blocks, never on the other problems of the handle
__global__ void __launch_bounds__(256)
k_reduce_blocks(int nprob, int nrange, const long long *__restrict__ range, const double *__restrict__ part, int k,
                int ksum, double *__restrict__ out)
{
    __shared__ double sred[4];
    const int p = blockIdx.x / k, q = blockIdx.x % k;
    if (p >= nprob) return;   // uniform per workgroup, before any barrier
    const bool sum = q < ksum;
    double v = 0.0;
    long long base = 0;   // running block count of the problem (thread striding is global over its ranges)
    for (int r = 0; r < nrange; ++r) {
        const long long b0 = range[2 * ((long long)p * nrange + r)], b1 = range[2 * ((long long)p * nrange + r) + 1];
        const long long n = b1 - b0;
        // element i of this range has problem-local index base + i; thread t owns indices = t mod 256
        long long first = ((threadIdx.x - base) % 256 + 256) % 256;
        for (long long i = first; i < n; i += 256) {
            const double x = part[(b0 + i) * k + q];
            v = sum ? v + x : fmax(v, x);
        }
        base += n;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_down(v, o, 64);
        v = sum ? v + w : fmax(v, w);
    }
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sred[0];
        for (int w = 1; w < 4; ++w) t = sum ? t + sred[w] : fmax(t, sred[w]);
        out[(long long)p * k + q] = t;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
ohm_status launch_blk_stencil(const ohm_hier *h, int level, int mode, const T *B, const T *Bg, long long cs,
                              long long gcs, const T *S, const T *eta, const T *etag, const double *coef_dev,
                              T *out, int colour, double *partials, const uint8_t *cov_zero, const int *active,
                              hipStream_t s, StencilDots dots)
{
    const AmrLevelDev &L = h->amr[level];
    if (L.nb == 0) return OHM_OK;
    if (dots.ndot < 0 || dots.ndot > 2 || (dots.ndot > 0 && (mode != MODE_APPLY || !dots.dot_part)))
        return fail(OHM_ERR_ARG, "fused dot products need MODE_APPLY, 1 or 2 products and a partials buffer");
    dim3 grid(L.nb), blk(256);
#define ARGS L.nb, L.nbr, L.prob, cov_zero, active, L.inv_h2, coef_dev, B, Bg, cs, gcs, S, eta, etag, out, colour, \
             partials, dots, nullptr, nullptr, 0
    switch (mode) {
    case MODE_APPLY: k_blk_stencil<T, MODE_APPLY><<<grid, blk, 0, s>>>(ARGS); break;
    case MODE_RESID: k_blk_stencil<T, MODE_RESID><<<grid, blk, 0, s>>>(ARGS); break;
    case MODE_SMOOTH: k_blk_stencil<T, MODE_SMOOTH><<<grid, blk, 0, s>>>(ARGS); break;
    default: return fail(OHM_ERR_ARG, "unknown stencil mode %d", mode);
    }
#undef ARGS
    return check_launch("block stencil");
}

template <typename T>
ohm_status launch_resid_restrict_blk0(const ohm_hier *h, const T *B, const T *Bg, long long cs, long long gcs,
                                      const T *S, const T *eta, const T *etag, const double *coef_dev, T *coarse,
                                      long long ccs, const int *active, hipStream_t s)
{
    const AmrLevelDev &L = h->amr[0];
    if (L.nb == 0) return OHM_OK;
    if (h->min_level > -1) return fail(OHM_ERR_ARG, "no dense level below level 0");
    k_blk_stencil<T, MODE_RESID_RESTRICT><<<L.nb, 256, 0, s>>>(
        L.nb, L.nbr, L.prob, nullptr, active, L.inv_h2, coef_dev, B, Bg, cs, gcs, S, eta, etag, coarse, 0,
        nullptr, StencilDots{{nullptr, nullptr}, 0, nullptr}, L.dense_map, h->dense[1].probs, ccs);
    return check_launch("residual + restriction to dense");
}

template <typename T>
ohm_status launch_blk_sweep(const ohm_hier *h, int level, const T *B, long long cs, const T *S, const T *eta,
                            const double *coef_dev, T *out, const int *active, hipStream_t s, const T *coarse,
                            long long ccs, const T *Bg, long long gcs, const T *etag, double *out64)
{
    const AmrLevelDev &L = h->amr[level];
    if (L.nb == 0) return OHM_OK;
    if (out64) {
        if constexpr (std::is_same<T, float>::value) {
            if (!L.complete27 || !B)
                return fail(OHM_ERR_ARG, "an FP64 result needs a complete level and an input");
            if ((unsigned long long)L.nb * NC * sizeof(double) > 0xFFFFFFFFull)
                return fail(OHM_ERR_ARG, "level %d: FP64 result array above 4 GiB", level);
            if (((uintptr_t)B | (uintptr_t)eta | (uintptr_t)(cs * sizeof(T))) % (2 * sizeof(T)) != 0)
                return fail(OHM_ERR_ARG, "level %d: fused sweep needs B, eta and the component stride %zu-byte "
                                         "aligned", level, 2 * sizeof(T));
            if (coarse) {
                if (level != 0 || h->min_level > -1)
                    return fail(OHM_ERR_ARG, "a fused coarse correction needs level 0 and a dense level below it");
                k_blk_sweep<T, 2, true><<<L.nb, SWEEP_THREADS, 0, s>>>(
                    L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev, B, cs, S, eta, out, L.ijk, h->dense[1].probs,
                    coarse, ccs, nullptr, 0, nullptr, out64);
            } else {
                k_blk_sweep<T, 0, true><<<L.nb, SWEEP_THREADS, 0, s>>>(L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev,
                                                                       B, cs, S, eta, out, nullptr, nullptr, nullptr,
                                                                       0, nullptr, 0, nullptr, out64);
            }
            return check_launch("fused sweep to FP64");
        } else {
            return fail(OHM_ERR_ARG, "an FP64 result is for FP32 sweeps");
        }
    }
    if (!L.fused)
        return fail(OHM_ERR_ARG, "fused sweep needs every neighbour block of level %d as a level or ghost block", level);
    const bool gh = !L.complete27;
    if ((unsigned long long)L.nb * NC * sizeof(T) > 0xFFFFFFFFull ||
        (gh && (unsigned long long)L.ng * NC * sizeof(T) > 0xFFFFFFFFull))
        return fail(OHM_ERR_ARG, "level %d: fused sweep addresses each field array with 32-bit offsets (max 4 GiB)",
                    level);
    if (((uintptr_t)B | (uintptr_t)eta | (uintptr_t)(cs * sizeof(T))) % (2 * sizeof(T)) != 0)
        return fail(OHM_ERR_ARG, "level %d: fused sweep needs B, eta and the component stride %zu-byte aligned", level,
                    2 * sizeof(T));
    if (gh) {
        if (coarse) return fail(OHM_ERR_ARG, "a fused coarse correction needs level 0");
        if ((B && !Bg) || !etag) return fail(OHM_ERR_ARG, "level %d has ghost blocks: B_ghost and eta_ghost needed", level);
        if (((uintptr_t)Bg | (uintptr_t)etag | (uintptr_t)(gcs * sizeof(T))) % (2 * sizeof(T)) != 0)
            return fail(OHM_ERR_ARG, "level %d: fused sweep needs the ghost arrays and their stride %zu-byte aligned",
                        level, 2 * sizeof(T));
        if (B)
            k_blk_sweep<T, 3><<<L.nb, SWEEP_THREADS, 0, s>>>(L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev, B, cs, S,
                                                             eta, out, nullptr, nullptr, nullptr, 0, Bg, gcs, etag);
        else
            k_blk_sweep<T, 4><<<L.nb, SWEEP_THREADS, 0, s>>>(L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev, B, cs, S,
                                                             eta, out, nullptr, nullptr, nullptr, 0, nullptr, 0, etag);
        return check_launch("fused sweep with ghosts");
    }
    if (coarse) {
        if (level != 0 || h->min_level > -1 || !B)
            return fail(OHM_ERR_ARG, "a fused coarse correction needs level 0, a dense level below it and an input");
        k_blk_sweep<T, 2><<<L.nb, SWEEP_THREADS, 0, s>>>(L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev, B, cs, S, eta,
                                                         out, L.ijk, h->dense[1].probs, coarse, ccs, nullptr, 0,
                                                         nullptr);
    } else if (B) {
        // FP64 tiles go straight from global memory into LDS (16-byte pairs)
        k_blk_sweep<T, 0, false, std::is_same<T, double>::value><<<L.nb, SWEEP_THREADS, 0, s>>>(
            L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev, B, cs, S, eta, out, nullptr, nullptr, nullptr, 0, nullptr,
            0, nullptr);
    } else {
        k_blk_sweep<T, 1><<<L.nb, SWEEP_THREADS, 0, s>>>(L.nb, L.nbr, L.prob, active, L.inv_h2, coef_dev, B, cs, S, eta,
                                                         out, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr);
    }
    return check_launch("fused sweep");
}

template <typename T>
ohm_status launch_restrict_blk(const ohm_hier *h, int fine_level, const T *fine, long long fcs, T *coarse,
                               long long ccs, int ncomp, const int *active, hipStream_t s)
{
    if (fine_level >= 1) {
        const AmrLevelDev &L = h->amr[fine_level];
        if (L.nb == 0) return OHM_OK;
        k_restrict_blk<T><<<L.nb, 64, 0, s>>>(L.nb, L.parent, L.octant, L.prob, active, fine, fcs, coarse, ccs,
                                              ncomp);
        return check_launch("restrict");
    }
    const AmrLevelDev &L = h->amr[0];
    k_restrict_blk0_dense<T><<<L.nb, 64, 0, s>>>(L.nb, L.dense_map, L.prob, h->dense[1].probs, active, fine, fcs,
                                                 coarse, ccs, ncomp);
    return check_launch("restrict to dense");
}

template <typename T>
ohm_status launch_prolong_blk(const ohm_hier *h, int coarse_level, const T *coarse, long long ccs, T *fine,
                              long long fcs, int ncomp, int accumulate, const int *active, hipStream_t s,
                              const T *base)
{
    if (coarse_level >= 0) {
        if (base) return fail(OHM_ERR_ARG, "prolongation between block levels is in place");
        const AmrLevelDev &F = h->amr[coarse_level + 1];
        if (F.nb == 0) return OHM_OK;
        k_prolong_blk<T><<<F.nb, 256, 0, s>>>(F.nb, F.parent, F.octant, F.prob, active, h->amr[coarse_level].nbr,
                                              coarse, ccs, fine, fcs, ncomp, accumulate);
        return check_launch("prolong");
    }
    const AmrLevelDev &L = h->amr[0];
    if (base && !accumulate) return fail(OHM_ERR_ARG, "prolongation onto a base field must accumulate");
    if (ncomp < 1 || ncomp > 3) return fail(OHM_ERR_ARG, "prolongation takes 1 to 3 components, got %d", ncomp);
    if (accumulate && !base) base = fine;
    k_prolong_dense_blk0<T><<<L.nb, 256, 0, s>>>(L.nb, L.ijk, L.prob, h->dense[1].probs, active, coarse, ccs, base,
                                                 fine, fcs, ncomp);
    return check_launch("prolong from dense");
}

template <typename T>
ohm_status launch_fill_ghosts(const ohm_hier *h, int level, const T *coarse, long long ccs, T *ghost,
                              long long gcs, int ncomp, const int *active, hipStream_t s)
{
    const AmrLevelDev &L = h->amr[level];
    if (level < 1 || L.ng == 0) return OHM_OK;
    k_prolong_blk<T><<<L.ng, 256, 0, s>>>(L.ng, L.gparent, L.goctant, L.gprob, active, h->amr[level - 1].nbr,
                                          coarse, ccs, ghost, gcs, ncomp, 0);
    return check_launch("fill ghosts");
}

template <typename T>
ohm_status launch_reflux(const ohm_hier *h, int level, const T *Bc, long long ccs, const T *etac, const T *Bf,
                         long long fcs, const T *Bfg, long long fgcs, const T *etaf, const T *etafg,
                         const double *coef_dev, T *out, const int *active, hipStream_t s)
{
    const AmrLevelDev &L = h->amr[level];
    if (L.nrf == 0) return OHM_OK;
    k_reflux<T><<<L.nrfw, RF_WG_FACES * 10, 0, s>>>(L.rfw, L.rff, L.rfs, L.rf, active, L.nbr, h->amr[level + 1].nbr,
                                                   L.inv_h, coef_dev, Bc, ccs, etac, Bf, fcs, Bfg, fgcs, etaf, etafg,
                                                   out);
    return check_launch("reflux");
}

template <typename T>
ohm_status launch_zero_covered(const ohm_hier *h, int level, T *out, long long cs, int ncomp, hipStream_t s)
{
    const AmrLevelDev &L = h->amr[level];
    if (L.nb == 0) return OHM_OK;
    k_zero_covered<T><<<L.nb, 256, 0, s>>>(L.nb, L.cov, out, cs, ncomp);
    return check_launch("zero covered");
}

ohm_status launch_reduce_problem(int nprob, int nrange, const long long *range_dev, const double *part, int k,
                                 int ksum, double *out, hipStream_t s)
{
    k_reduce_blocks<<<nprob * k, 256, 0, s>>>(nprob, nrange, range_dev, part, k, ksum, out);
    return check_launch("reduce");
}

#define INST(T)                                                                                                 \
    template ohm_status launch_blk_sweep<T>(const ohm_hier *, int, const T *, long long, const T *, const T *,   \
                                            const double *, T *, const int *, hipStream_t, const T *, long long, \
                                            const T *, long long, const T *, double *);                         \
    template ohm_status launch_blk_stencil<T>(const ohm_hier *, int, int, const T *, const T *, long long,      \
                                              long long, const T *, const T *, const T *, const double *, T *,  \
                                              int, double *, const uint8_t *, const int *, hipStream_t,         \
                                              StencilDots);                                                     \
    template ohm_status launch_resid_restrict_blk0<T>(const ohm_hier *, const T *, const T *, long long,       \
                                                      long long, const T *, const T *, const T *,             \
                                                      const double *, T *, long long, const int *, hipStream_t);        \
    template ohm_status launch_restrict_blk<T>(const ohm_hier *, int, const T *, long long, T *, long long, int, \
                                               const int *, hipStream_t);                                       \
    template ohm_status launch_prolong_blk<T>(const ohm_hier *, int, const T *, long long, T *, long long, int,  \
                                              int, const int *, hipStream_t, const T *);                        \
    template ohm_status launch_fill_ghosts<T>(const ohm_hier *, int, const T *, long long, T *, long long, int,  \
                                              const int *, hipStream_t);                                        \
    template ohm_status launch_reflux<T>(const ohm_hier *, int, const T *, long long, const T *, const T *,      \
                                         long long, const T *, long long, const T *, const T *, const double *, \
                                         T *, const int *, hipStream_t);                                        \
    template ohm_status launch_zero_covered<T>(const ohm_hier *, int, T *, long long, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ohm
