// Kernels on the dense multigrid levels below the base grid (one thread per
// cell, 256-cell tiles that never straddle two problems) and the coarsest-grid
// solve (per-problem dense FP64 inverse built on the device).
#include "common.h"
#include "stencil.h"
#include "sweep.h"

namespace ohm {

namespace {

__device__ __forceinline__ int wrapd(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// gather the 3x3x3 neighbourhood (corners skipped) of cell (i,j,k)
template <typename T, typename Get>
__device__ __forceinline__ void gather(const DenseProbDev &q, int i, int j, int k, T *v, Get get)
{
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                if (dx != 0 && dy != 0 && dz != 0) {
                    v[t] = T(0);
                    continue;
                }
                const long long idx =
                    q.off + wrapd(i + dx, q.nx) + (long long)q.nx * (wrapd(j + dy, q.ny) + (long long)q.ny * wrapd(k + dz, q.nz));
                v[t] = get(idx);
            }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256)
k_dense_stencil(const int *__restrict__ tiles, const DenseProbDev *__restrict__ dp, const int *__restrict__ active,
                const double *__restrict__ coef_p, const T *__restrict__ B, const T *__restrict__ S,
                const T *__restrict__ eta, T *__restrict__ out, long long cs, int colour)
{
    const int pr = tiles[2 * blockIdx.x], start = tiles[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseProbDev q = dp[pr];
    const int n = q.nx * q.ny * q.nz;
    const int cell = start + threadIdx.x;
    if (cell >= n) return;
    const int i = cell % q.nx, j = (cell / q.nx) % q.ny, k = cell / (q.nx * q.ny);
    T b0[27], b1[27], b2[27], e[27];
    gather<T>(q, i, j, k, b0, [&](long long x) { return B[x]; });
    gather<T>(q, i, j, k, b1, [&](long long x) { return B[cs + x]; });
    gather<T>(q, i, j, k, b2, [&](long long x) { return B[2 * cs + x]; });
    gather<T>(q, i, j, k, e, [&](long long x) { return eta[x]; });
    const T cih2 = T(coef_p[pr]) * T(q.inv_h2);
    const T c8 = cih2 * T(0.125), c2 = cih2 * T(0.5);
    const long long gi = q.off + cell;
    const T *bc[3] = {b0, b1, b2};
    T dvs[3], als[3];
    divF_all<T, 3>(b0, b1, b2, e, 13, dvs, als);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T LB = fma(c8, dvs[c], bc[c][13]);
        if (MODE == MODE_APPLY) {
            out[c * cs + gi] = LB;
        } else if (MODE == MODE_RESID) {
            out[c * cs + gi] = S[c * cs + gi] - LB;
        } else {
            T v = bc[c][13];
            if (in_colour(i, j, k, colour)) v = relax_point(v, S[c * cs + gi], dvs[c], als[c], c8, c2);
            out[c * cs + gi] = v;
        }
    }
}

// Fused red-black sweep on 8^3 tiles of a dense level (periodic wrap).  A
// grid whose edges are even but not multiples of 8 is covered by
// ceil(n / 8) tiles per axis: the cells of the last tile past the edge are
// copies of cells at the start (an even period keeps their colour), computed
// from the same values as by the tile that owns them, so the duplicate
// stores write equal values.
__device__ __forceinline__ int wrap_cell(int i, int n)
{
    // i >= -2; past the first period only on grids narrower than a tile
    if (i < 0) return i + n;
    if (i >= n) {
        i -= n;
        if (i >= n) i %= n;
    }
    return i;
}

struct DenseAddr {
    static constexpr bool ghosts = false;
    DenseProbDev q;
    int ox, oy, oz;
    __device__ __forceinline__ long long at(int x, int y, int z) const
    {
        const int i = wrap_cell(ox + x, q.nx), j = wrap_cell(oy + y, q.ny), k = wrap_cell(oz + z, q.nz);
        return q.off + i + (long long)q.nx * (j + (long long)q.ny * k);
    }
};

__device__ __forceinline__ DenseAddr dense_tile(const DenseProbDev &q, int t)
{
    const int tx = (q.nx + 7) >> 3, ty = (q.ny + 7) >> 3;
    return DenseAddr{q, 8 * (t % tx), 8 * ((t / tx) % ty), 8 * (t / (tx * ty))};
}

// MODE 0: sweep B -> out; 1: zero input (B not read); 2: sweep of B plus the
// trilinear prolongation of the next coarser grid's field (coarse, problems
// cdp), B -> out, without storing the corrected input
template <typename T, int MODE>
__global__ void __launch_bounds__(SWEEP_THREADS)
k_dense_sweep(const int *__restrict__ ftiles, const DenseProbDev *__restrict__ dp, const int *__restrict__ active,
              const double *__restrict__ coef_p, const T *__restrict__ B, long long cs, const T *__restrict__ S,
              const T *__restrict__ eta, T *__restrict__ out, const T *__restrict__ coarse, long long ccs,
              const DenseProbDev *__restrict__ cdp)
{
    __shared__ T sB[3][TC2];
    __shared__ T sE[TC2];
    const int pr = ftiles[2 * blockIdx.x], t = ftiles[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseProbDev q = dp[pr];
    const DenseAddr A = dense_tile(q, t);
    const T cih2 = T(coef_p[pr]) * T(q.inv_h2);
    if constexpr (MODE == 2) {
        __shared__ T sC[3 * 512];
        TileCoarse<T> cor{coarse, ccs, cdp[pr], A.ox / 2 - 2, A.oy / 2 - 2, A.oz / 2 - 2, sC, {}};
        fused_sweep_tile<T, false>(A, B, cs, S, eta, out, cih2, sB, sE, cor);
    } else {
        fused_sweep_tile<T, MODE == 1>(A, B, cs, S, eta, out, cih2, sB, sE);
    }
}

// copy (src != nullptr) or zero the cells of the listed 8^3 tiles (3 components)
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_tile_copy(const int *__restrict__ ftiles, const DenseProbDev *__restrict__ dp, const int *__restrict__ active,
                  const T *__restrict__ src, T *__restrict__ dst, long long cs)
{
    const int pr = ftiles[2 * blockIdx.x], t = ftiles[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseAddr A = dense_tile(dp[pr], t);
    for (int cell = threadIdx.x; cell < 512; cell += 256) {
        const long long gi = A.at(cell & 7, (cell >> 3) & 7, cell >> 6);
        for (int c = 0; c < 3; ++c) dst[c * cs + gi] = src ? src[c * cs + gi] : T(0);
    }
}

// the same over 256-cell runs (prob, first cell) of a problem
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_run_copy(const int *__restrict__ runs, const DenseProbDev *__restrict__ dp, const int *__restrict__ active,
                 const T *__restrict__ src, T *__restrict__ dst, long long cs)
{
    const int pr = runs[2 * blockIdx.x], start = runs[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseProbDev q = dp[pr];
    const int cell = start + threadIdx.x;
    if (cell >= q.nx * q.ny * q.nz) return;
    const long long gi = q.off + cell;
    for (int c = 0; c < 3; ++c) dst[c * cs + gi] = src ? src[c * cs + gi] : T(0);
}

// r = S - L e on one 8^3 tile of a dense level (one-cell periodic halo in
// LDS) restricted straight to the next coarser level: the same residual and
// the same 8-child sums as k_dense_stencil<RESID> followed by k_dense_restrict
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_resid_restrict(const int *__restrict__ ftiles, const DenseProbDev *__restrict__ dp,
                       const DenseProbDev *__restrict__ cdp, const int *__restrict__ active,
                       const double *__restrict__ coef_p, const T *__restrict__ B, const T *__restrict__ S,
                       const T *__restrict__ eta, T *__restrict__ coarse, long long cs, long long ccs)
{
    constexpr int W = 10;
    __shared__ T sB[3][W * W * W];
    __shared__ T sE[W * W * W];
    const int pr = ftiles[2 * blockIdx.x], tile = ftiles[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseProbDev q = dp[pr];
    const DenseAddr A = dense_tile(q, tile);
    // thread u < 200 owns tile column (x, y) = u mod 100 and five z: all loads
    // first, then the LDS stores
    if (threadIdx.x < 2 * W * W) {
        const int col = threadIdx.x % (W * W), zh = threadIdx.x / (W * W);
        const int x = col % W - 1, y = col / W - 1;
        T v[5][4];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const long long gi = A.at(x, y, 5 * zh + k - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) v[k][c] = B[c * cs + gi];
            v[k][3] = eta[gi];
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int t = col + W * W * (5 * zh + k);
#pragma unroll
            for (int c = 0; c < 3; ++c) sB[c][t] = v[k][c];
            sE[t] = v[k][3];
        }
    }
    // S of this thread's two cells, loaded before the barrier so that its
    // latency overlaps the tile's
    T s2[2][3];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int cell = threadIdx.x + 256 * half;
        const long long gi = A.at(cell & 7, (cell >> 3) & 7, cell >> 6);
#pragma unroll
        for (int c = 0; c < 3; ++c) s2[half][c] = S[c * cs + gi];
    }
    __syncthreads();
    const T c8 = T(coef_p[pr]) * T(q.inv_h2) * T(0.125);
    T r[2][3];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int cell = threadIdx.x + 256 * half;
        const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
        const int p = (x + 1) + W * ((y + 1) + W * (z + 1));
        T dv[3], al[3];
        divF_all<T, W>(sB[0], sB[1], sB[2], sE, p, dv, al);
#pragma unroll
        for (int c = 0; c < 3; ++c) r[half][c] = s2[half][c] - fma(c8, dv[c], sB[c][p]);
    }
    __syncthreads();
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int c = 0; c < 3; ++c) sB[c][threadIdx.x + 256 * half] = r[half][c];
    __syncthreads();
    const int i = threadIdx.x & 3, j = (threadIdx.x >> 2) & 3, k = threadIdx.x >> 4;
    const DenseProbDev cq = cdp[pr];
    // a coarse cell past the grid's edge belongs to the tile that owns its
    // children (they are copies here)
    if (threadIdx.x < 64 && A.ox / 2 + i < cq.nx && A.oy / 2 + j < cq.ny && A.oz / 2 + k < cq.nz) {
        const long long ci = cq.off + (A.ox / 2 + i) + (long long)cq.nx * ((A.oy / 2 + j) + (long long)cq.ny * (A.oz / 2 + k));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T a = T(0);
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) a += sB[c][(2 * i + dx) + NB * ((2 * j + dy) + NB * (2 * k + dz))];
            coarse[c * ccs + ci] = a * T(0.125);
        }
    }
}

// dense level -d -> -(d+1): mean of 8 children; one thread per coarse cell
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_restrict(const int *__restrict__ ctiles, const DenseProbDev *__restrict__ cdp,
                 const DenseProbDev *__restrict__ fdp, const int *__restrict__ active, const T *__restrict__ fine,
                 long long fcs, T *__restrict__ coarse, long long ccs, int ncomp)
{
    const int pr = ctiles[2 * blockIdx.x], start = ctiles[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseProbDev c = cdp[pr], f = fdp[pr];
    const int cell = start + threadIdx.x;
    if (cell >= c.nx * c.ny * c.nz) return;
    const int i = cell % c.nx, j = (cell / c.nx) % c.ny, k = cell / (c.nx * c.ny);
    for (int m = 0; m < ncomp; ++m) {
        T s = T(0);
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    s += fine[m * fcs + f.off + (2 * i + dx) + (long long)f.nx * ((2 * j + dy) + (long long)f.ny * (2 * k + dz))];
        coarse[m * ccs + c.off + cell] = s * T(0.125);
    }
}

// dense -(d+1) -> -d trilinear prolongation; one thread per fine cell
template <typename T>
__global__ void __launch_bounds__(256)
k_dense_prolong(const int *__restrict__ ftiles, const DenseProbDev *__restrict__ fdp,
                const DenseProbDev *__restrict__ cdp, const int *__restrict__ active, const T *__restrict__ coarse,
                long long ccs, const T *base, T *fine, long long fcs, int ncomp)
{
    const int pr = ftiles[2 * blockIdx.x], start = ftiles[2 * blockIdx.x + 1];
    if (active && !active[pr]) return;
    const DenseProbDev f = fdp[pr], c = cdp[pr];
    const int cell = start + threadIdx.x;
    if (cell >= f.nx * f.ny * f.nz) return;
    const int X = cell % f.nx, Y = (cell / f.nx) % f.ny, Z = cell / (f.nx * f.ny);
    const int i = X >> 1, j = Y >> 1, k = Z >> 1;
    const int i1 = wrapd(i + ((X & 1) ? 1 : -1), c.nx), j1 = wrapd(j + ((Y & 1) ? 1 : -1), c.ny),
              k1 = wrapd(k + ((Z & 1) ? 1 : -1), c.nz);
    auto at = [&](int a, int b, int d) { return c.off + a + (long long)c.nx * (b + (long long)c.ny * d); };
    for (int m = 0; m < ncomp; ++m) {
        const T *C = coarse + m * ccs;
        T v = T(27) * C[at(i, j, k)] + T(9) * (C[at(i1, j, k)] + C[at(i, j1, k)] + C[at(i, j, k1)]) +
              T(3) * (C[at(i1, j1, k)] + C[at(i1, j, k1)] + C[at(i, j1, k1)]) + C[at(i1, j1, k1)];
        v *= T(1.0 / 64.0);
        const long long gi = m * fcs + f.off + cell;
        fine[gi] = base ? base[gi] + v : v;
    }
}

// ---------------------------------------------------------------------------
// coarsest grid: assemble L (FP64) column by column, invert by Gauss-Jordan
// with partial pivoting (one workgroup per problem), apply as a mat-vec
// ---------------------------------------------------------------------------
constexpr int COARSE_MAX_DEV = 768;

struct CoarseJob {
    int prob;
    int n3;              // unknowns = 3 * cells
    long long inv_off;   // element offset of the inverse
    long long aug_off;   // element offset of the [n3][2 n3] augmented matrix (scratch)
    long long eta_off;   // offset of the job's saved coarsest resistivity (cells)
    DenseProbDev q;
    double lam_dt;
};

__global__ void __launch_bounds__(256)
k_coarse_assemble(const CoarseJob *__restrict__ jobs, const int *__restrict__ flags, const double *__restrict__ eta,
                  double *__restrict__ aug)
{
    if (!flags[blockIdx.y]) return;
    const CoarseJob J = jobs[blockIdx.y];
    const int col = blockIdx.x;
    if (col >= J.n3) return;
    const int cells = J.n3 / 3;
    const int cj = col / cells, qj = col % cells;
    double *A = aug + J.aug_off;
    for (int row = threadIdx.x; row < J.n3; row += blockDim.x) {
        const int cr = row / cells, qr = row % cells;
        const int i = qr % J.q.nx, j = (qr / J.q.nx) % J.q.ny, k = qr / (J.q.nx * J.q.ny);
        double b[3][27], e[27];
        for (int m = 0; m < 3; ++m)
            gather<double>(J.q, i, j, k, b[m], [&](long long x) { return (m == cj && x == J.q.off + qj) ? 1.0 : 0.0; });
        gather<double>(J.q, i, j, k, e, [&](long long x) { return eta[x]; });
        double dvs[3], als[3];
        divF_all<double, 3>(b[0], b[1], b[2], e, 13, dvs, als);
        const double v = fma(J.lam_dt * J.q.inv_h2 * 0.125, dvs[cr], b[cr][13]);
        A[(long long)row * 2 * J.n3 + col] = v;
        A[(long long)row * 2 * J.n3 + J.n3 + col] = (row == col) ? 1.0 : 0.0;
    }
}

// does the coarsest resistivity of a job differ from the one its inverse was
// built with?  (flag = 1 also when the host forces a rebuild)
__global__ void __launch_bounds__(256)
k_coarse_check(const CoarseJob *__restrict__ jobs, const int *__restrict__ force, const double *__restrict__ eta,
               double *__restrict__ saved, int *__restrict__ flags)
{
    const CoarseJob J = jobs[blockIdx.x];
    const int cells = J.n3 / 3;
    __shared__ int diff;
    if (threadIdx.x == 0) diff = force[blockIdx.x];
    __syncthreads();
    double *sv = saved + J.eta_off;
    for (int t = threadIdx.x; t < cells; t += blockDim.x)
        if (sv[t] != eta[J.q.off + t]) diff = 1;
    __syncthreads();
    if (diff)
        for (int t = threadIdx.x; t < cells; t += blockDim.x) sv[t] = eta[J.q.off + t];
    if (threadIdx.x == 0) flags[blockIdx.x] = diff;
}

// Gauss-Jordan inversion with partial pivoting of a job with n <= 32 RG
// unknowns, the matrix held in registers.  Thread t of the 1024-thread
// workgroup owns rows ty + 32 i and columns tx + 32 j (i, j < RG) with
// ty = t mod 32, tx = t / 32, so the 32 owners of a column are one half of a
// wavefront.  Rows are never moved: step k takes as pivot the largest
// |A[r][k]| over the rows not pivoted yet (the lowest row on ties), scales
// that row and eliminates column k from every other row, and column k's
// storage then holds the column of the inverse-in-progress that the augmented
// form [A | I] would keep at the pivot row's identity column (in place).  With
// p_k the pivot row of step k and k(r) the step row r was pivot in, the
// inverse is inverse[k(r)][p_j] = S[r][j] for the stored matrix S.  Each step:
// the owners of column k reduce the candidates across their half-wavefront
// and publish the pivot and the multipliers, the pivot row's owners publish
// the scaled row (LDS, double-buffered by step parity), and every thread
// updates its 36 entries; nothing goes through global memory.  Column k sits
// in register slot k / 32, a compile-time index in the unrolled outer loop.
// Rows and columns at or beyond n are zero padding.  Against the augmented
// kernel below (one job of 192 unknowns): about 0.5 ms instead of 1.1 ms.
constexpr int RG = 6;

__global__ void __launch_bounds__(1024)
k_coarse_invert_reg(const CoarseJob *__restrict__ jobs, const int *__restrict__ flags,
                    const double *__restrict__ aug, double *__restrict__ inv)
{
    if (!flags[blockIdx.x]) return;
    const CoarseJob J = jobs[blockIdx.x];
    const int n = J.n3, w = 2 * n;
    if (n > 32 * RG) return;
    const double *A0 = aug + J.aug_off;
    const int ty = threadIdx.x & 31, tx = threadIdx.x >> 5;
    __shared__ double prow[2][32 * RG], fcol[2][32 * RG];
    __shared__ int piv_of_step[32 * RG], step_of_row[32 * RG];
    __shared__ int sp;
    __shared__ double spv;
    double a[RG][RG];
    bool used[RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) {
        const int r = ty + 32 * i;
        used[i] = r >= n;
#pragma unroll
        for (int j = 0; j < RG; ++j) {
            const int c = tx + 32 * j;
            a[i][j] = (r < n && c < n) ? A0[(long long)r * w + c] : 0.0;
        }
    }
    // column k = 32 jk + tk: jk is a compile-time register slot
#pragma unroll
    for (int jk = 0; jk < RG; ++jk) {
        for (int tk = 0; tk < 32; ++tk) {
            const int k = 32 * jk + tk;
            if (k >= n) break;
            const int buf = k & 1;
            if (tx == tk) {
                // a NaN ranks as infinite, so some row not pivoted yet is
                // always chosen (a non-finite matrix gives a non-finite
                // inverse, never an index outside the matrix); a lane without
                // such rows offers -1 and row n
                double best = -1.0, sg = 0.0;
                int id = n;
#pragma unroll
                for (int i = 0; i < RG; ++i) {
                    const double v = a[i][jk];
                    const double av = v != v ? INFINITY : fabs(v);
                    const bool take = !used[i] && av > best;
                    best = take ? av : best;
                    sg = take ? v : sg;
                    id = take ? ty + 32 * i : id;
                }
                // a lane's candidate rows increase with i and a later row
                // replaced an earlier one only when strictly larger: the
                // lowest row index wins ties
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 32), os = __shfl_xor(sg, off, 32);
                    const int oi = __shfl_xor(id, off, 32);
                    const bool take = ob > best || (ob == best && oi < id);
                    best = take ? ob : best;
                    sg = take ? os : sg;
                    id = take ? oi : id;
                }
                if (ty == 0) {
                    sp = id;
                    spv = sg;
                    piv_of_step[k] = id;
                    step_of_row[id] = k;
                }
#pragma unroll
                for (int i = 0; i < RG; ++i) {
                    const int r = ty + 32 * i;
                    fcol[buf][r] = r == id ? -1.0 : a[i][jk];
                }
            }
            __syncthreads();
            const int p = sp, ip = p >> 5, tp = p & 31;
            const double d = 1.0 / spv;
            if (ty == tp) {
                // the pivot row scaled by 1 / pivot; its column-k entry is d
#pragma unroll
                for (int j = 0; j < RG; ++j) {
                    double v = a[0][j];
#pragma unroll
                    for (int i = 1; i < RG; ++i) v = i == ip ? a[i][j] : v;
                    const int c = tx + 32 * j;
                    prow[buf][c] = (c == k ? 1.0 : v) * d;
                }
#pragma unroll
                for (int i = 0; i < RG; ++i) used[i] = used[i] || i == ip;
            }
            __syncthreads();
            double f[RG], y[RG];
#pragma unroll
            for (int i = 0; i < RG; ++i) f[i] = fcol[buf][ty + 32 * i];
#pragma unroll
            for (int j = 0; j < RG; ++j) y[j] = prow[buf][tx + 32 * j];
            // a - f y on every other row; the pivot row (multiplier -1, its
            // entries scaled by 0) becomes the scaled row y; then column k
            // becomes -f d (d on the pivot row)
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                const double keep = ty + 32 * i == p ? 0.0 : 1.0;
#pragma unroll
                for (int j = 0; j < RG; ++j) a[i][j] = fma(-f[i], y[j], a[i][j] * keep);
            }
            if (tx == tk) {
#pragma unroll
                for (int i = 0; i < RG; ++i) a[i][jk] = fma(-f[i], y[jk], 0.0);
            }
        }
    }
    __syncthreads();
    // stored transposed, as the mat-vec reads it: X[c][r] = inverse[r][c]
    double *X = inv + J.inv_off;
#pragma unroll
    for (int i = 0; i < RG; ++i) {
        const int r = ty + 32 * i;
        if (r >= n) continue;
        const int row = step_of_row[r];
#pragma unroll
        for (int j = 0; j < RG; ++j) {
            const int c = tx + 32 * j;
            if (c < n) X[(long long)piv_of_step[c] * n + row] = a[i][j];
        }
    }
}

// Gauss-Jordan inversion with partial pivoting of a job with more than 32 RG
// unknowns, one 32x32 workgroup per job, on the augmented matrix in memory.
// Without a row exchange, step k only meets columns k .. n+k of the augmented
// matrix [A | I] (the identity entries of the rows below k lie further right
// and are untouched).  A row exchange brings row p's identity entry, at column
// n+p, into the pivot row, so from the first exchange on every step works on
// all columns k .. 2n-1.  The pivot is read only after the exchange has been
// written and a barrier has passed.
__global__ void __launch_bounds__(1024)
k_coarse_invert(const CoarseJob *__restrict__ jobs, const int *__restrict__ flags, double *__restrict__ aug,
                double *__restrict__ inv)
{
    if (!flags[blockIdx.x]) return;
    const CoarseJob J = jobs[blockIdx.x];
    const int n = J.n3, w = 2 * n;
    if (n <= 32 * RG) return;
    double *A = aug + J.aug_off;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 32 + tx;
    __shared__ double sval[1024];
    __shared__ int sidx[1024];
    __shared__ double sfac[COARSE_MAX_DEV];
    __shared__ double srow[2 * COARSE_MAX_DEV];
    bool swapped = false;   // uniform over the workgroup: every thread reads the same sidx[0]
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = k;
        for (int r = k + tid; r < n; r += 1024) {
            const double a = fabs(A[r * w + k]);
            if (a > best) { best = a; bi = r; }
        }
        sval[tid] = best;
        sidx[tid] = bi;
        __syncthreads();
        for (int st = 512; st > 0; st >>= 1) {
            if (tid < st) {
                const double o = sval[tid + st];
                const int oi = sidx[tid + st];
                if (o > sval[tid] || (o == sval[tid] && oi < sidx[tid])) {
                    sval[tid] = o;
                    sidx[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int p = sidx[0];
        swapped = swapped || p != k;
        // live columns k .. k + ncol - 1
        const int ncol = swapped ? w - k : n + 1;
        if (p != k) {
            for (int cc = tid; cc < ncol; cc += 1024) {
                const int c = k + cc;
                const double vk = A[k * w + c], vp = A[p * w + c];
                A[k * w + c] = vp;
                A[p * w + c] = vk;
            }
        }
        __syncthreads();
        // scale the pivot row into LDS, then write it back; the multipliers of
        // the other rows are read in the same phase (column k only)
        const double d = 1.0 / A[k * w + k];
        for (int cc = tid; cc < ncol; cc += 1024) srow[cc] = A[k * w + k + cc] * d;
        for (int r = tid; r < n; r += 1024) sfac[r] = (r == k) ? 0.0 : A[r * w + k];
        __syncthreads();
        for (int cc = tid; cc < ncol; cc += 1024) A[k * w + k + cc] = srow[cc];
        for (int r = ty; r < n; r += 32) {
            const double f = sfac[r];
            if (f == 0.0) continue;
            for (int cc = tx; cc < ncol; cc += 32) A[r * w + k + cc] -= f * srow[cc];
        }
        __syncthreads();
    }
    // stored transposed: X[c][r] = inverse[r][c], so that the mat-vec reads
    // consecutive rows with consecutive lanes
    double *X = inv + J.inv_off;
    for (int r = ty; r < n; r += 32)
        for (int c = tx; c < n; c += 32) X[c * n + r] = A[r * w + n + c];
}

template <typename T>
__global__ void __launch_bounds__(512)
k_coarse_apply(const CoarseJob *__restrict__ jobs, const int *__restrict__ active, const double *__restrict__ inv,
               const T *__restrict__ r, T *__restrict__ e, long long cs)
{
    // workgroup (x, job): rows 64 x .. 64 x + 63 of the job's inverse; each of
    // the 8 wavefronts sums one contiguous slice of the columns, the slices are
    // then added in a fixed order
    const CoarseJob J = jobs[blockIdx.y];
    if (active && !active[J.prob]) return;
    const int n = J.n3, cells = n / 3;
    const int row0 = 64 * blockIdx.x;
    if (row0 >= n) return;
    __shared__ double sr[COARSE_MAX_DEV];
    __shared__ double part[8][64];
    for (int t = threadIdx.x; t < n; t += blockDim.x) sr[t] = (double)r[(t / cells) * cs + J.q.off + t % cells];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = row0 + lane;
    const double *X = inv + J.inv_off;
    const int per = (n + 7) / 8, c0 = w * per, c1 = min(n, c0 + per);
    double acc = 0.0;
    if (row < n) {
#pragma unroll 8
        for (int c = c0; c < c1; ++c) acc = fma(X[(long long)c * n + row], sr[c], acc);
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < n) {
        double v = part[0][lane];
        for (int k = 1; k < 8; ++k) v += part[k][lane];
        e[(row / cells) * cs + J.q.off + row % cells] = (T)v;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
ohm_status launch_dense_stencil(const ohm_hier *h, int level, int mode, const T *B, const T *S, const T *eta,
                                const double *coef_dev, T *out, int colour, bool coarsest_too, const int *active,
                                hipStream_t s)
{
    const DenseLevelDev &D = h->dense[-level];
    const int nt = coarsest_too ? D.ntile_all : D.ntile;
    const int *tl = coarsest_too ? D.tiles_all : D.tiles;
    if (nt == 0) return OHM_OK;
    const long long cs = D.ncells;
    switch (mode) {
    case MODE_APPLY:
        k_dense_stencil<T, MODE_APPLY><<<nt, 256, 0, s>>>(tl, D.probs, active, coef_dev, B, S, eta, out, cs, colour);
        break;
    case MODE_RESID:
        k_dense_stencil<T, MODE_RESID><<<nt, 256, 0, s>>>(tl, D.probs, active, coef_dev, B, S, eta, out, cs, colour);
        break;
    default:
        k_dense_stencil<T, MODE_SMOOTH><<<nt, 256, 0, s>>>(tl, D.probs, active, coef_dev, B, S, eta, out, cs, colour);
    }
    return check_launch("dense stencil");
}

// nsweeps red-black sweeps of dense level `level`: B holds the start and the
// result, tmp is scratch of the same size.  Problems whose grid is a whole
// number of 8^3 tiles get one fused launch per sweep, the others two
// half-sweep launches; the four-colour ordering takes four class launches per
// sweep on every problem.  all = every problem present, else the problems that
// are not coarsest at this level.
template <typename T>
ohm_status launch_dense_smooth(const ohm_hier *h, int level, T *B, T *tmp, const T *S, const T *eta,
                               const double *coef_dev, int nsweeps, bool all, const int *active, hipStream_t s,
                               int flags, const T *coarse, T **last, int ordering)
{
    const DenseLevelDev &D = h->dense[-level];
    const long long cs = D.ncells;
    const int nft = all ? D.nftile_all : D.nftile, npt = all ? D.nptile_all : D.nptile;
    const int *ft = all ? D.ftiles_all : D.ftiles, *pt = all ? D.ptiles_all : D.ptiles;
    const bool zero = flags & SMOOTH_ZERO, from_tmp = (flags & SMOOTH_FROM_TMP) && !zero;
    if (ordering != 0) {
        // four class launches per sweep over the 256-cell tiles of every
        // problem concerned, each a full out-of-place pass: a sweep returns to
        // the buffer it started from
        if (ordering != 1 || coarse || last)
            return fail(OHM_ERR_ARG, "dense level %d: ordering %d (0 or 1; 1 takes no fused coarse correction)",
                        level, ordering);
        const int nt = all ? D.ntile_all : D.ntile;
        const int *tl = all ? D.tiles_all : D.tiles;
        if (nt == 0) return OHM_OK;
        T *cur = from_tmp ? tmp : B, *oth = from_tmp ? B : tmp;
        if (zero) {
            k_dense_run_copy<T><<<nt, 256, 0, s>>>(tl, D.probs, active, nullptr, B, cs);
            OHM_TRY(check_launch("dense run zero"));
        }
        for (int k = 0; k < nsweeps; ++k)
            for (int m = 0; m < 4; ++m) {
                k_dense_stencil<T, MODE_SMOOTH><<<nt, 256, 0, s>>>(tl, D.probs, active, coef_dev, (m & 1) ? oth : cur,
                                                                   S, eta, (m & 1) ? cur : oth, cs, 2 + m);
                OHM_TRY(check_launch("dense colour-class update"));
            }
        if (cur != B) {
            k_dense_run_copy<T><<<nt, 256, 0, s>>>(tl, D.probs, active, cur, B, cs);
            OHM_TRY(check_launch("dense run copy"));
        }
        return OHM_OK;
    }
    if (nft > 0 && (unsigned long long)cs * sizeof(T) > 0xFFFFFFFFull)
        return fail(OHM_ERR_ARG, "dense level %d: fused sweep addresses each field array with 32-bit offsets", level);
    if ((coarse || last) && (npt > 0 || zero || nsweeps < 1 || -level >= -h->min_level))
        return fail(OHM_ERR_ARG, "dense level %d: a fused coarse correction or a result left in place needs whole "
                                 "tiles, an input, a sweep and a coarser level", level);
    const DenseLevelDev *Dc = coarse ? &h->dense[-level + 1] : nullptr;
    if (nft > 0) {
        // fused tiles ping-pong between B and tmp; a zero input is not read, so
        // the first sweep may write either buffer: pick the one that makes the
        // last sweep land in B
        T *cur = from_tmp ? tmp : B;
        for (int k = 0; k < nsweeps; ++k) {
            T *dst;
            if (k == 0 && zero) {
                dst = (nsweeps & 1) ? B : tmp;
                k_dense_sweep<T, 1><<<nft, SWEEP_THREADS, 0, s>>>(ft, D.probs, active, coef_dev, nullptr, cs, S, eta,
                                                                  dst, nullptr, 0, nullptr);
            } else if (k == 0 && coarse) {
                dst = cur == B ? tmp : B;
                k_dense_sweep<T, 2><<<nft, SWEEP_THREADS, 0, s>>>(ft, D.probs, active, coef_dev, cur, cs, S, eta,
                                                                  dst, coarse, Dc->ncells, Dc->probs);
            } else {
                dst = cur == B ? tmp : B;
                k_dense_sweep<T, 0><<<nft, SWEEP_THREADS, 0, s>>>(ft, D.probs, active, coef_dev, cur, cs, S, eta,
                                                                  dst, nullptr, 0, nullptr);
            }
            OHM_TRY(check_launch("dense fused sweep"));
            cur = dst;
        }
        if (last) {
            *last = cur;   // the caller takes the result where the sweeps left it
        } else if (nsweeps == 0 && zero) {
            k_dense_tile_copy<T><<<nft, 256, 0, s>>>(ft, D.probs, active, nullptr, B, cs);
            OHM_TRY(check_launch("dense tile zero"));
        } else if (cur != B) {
            k_dense_tile_copy<T><<<nft, 256, 0, s>>>(ft, D.probs, active, cur, B, cs);
            OHM_TRY(check_launch("dense tile copy"));
        }
    }
    if (npt > 0) {
        // two half-sweeps per sweep, each a full out-of-place pass: a sweep
        // returns to the buffer it started from
        T *cur = from_tmp ? tmp : B, *oth = from_tmp ? B : tmp;
        if (zero) {
            k_dense_run_copy<T><<<npt, 256, 0, s>>>(pt, D.probs, active, nullptr, B, cs);
            OHM_TRY(check_launch("dense run zero"));
        }
        for (int k = 0; k < nsweeps; ++k) {
            k_dense_stencil<T, MODE_SMOOTH><<<npt, 256, 0, s>>>(pt, D.probs, active, coef_dev, cur, S, eta, oth, cs, 0);
            OHM_TRY(check_launch("dense half-sweep"));
            k_dense_stencil<T, MODE_SMOOTH><<<npt, 256, 0, s>>>(pt, D.probs, active, coef_dev, oth, S, eta, cur, cs, 1);
            OHM_TRY(check_launch("dense half-sweep"));
        }
        if (cur != B) {
            k_dense_run_copy<T><<<npt, 256, 0, s>>>(pt, D.probs, active, cur, B, cs);
            OHM_TRY(check_launch("dense run copy"));
        }
    }
    return OHM_OK;
}

template <typename T>
ohm_status launch_dense_resid_restrict(const ohm_hier *h, int level, const T *B, const T *S, const T *eta,
                                       const double *coef_dev, T *res, T *coarse, const int *active, hipStream_t s)
{
    const DenseLevelDev &D = h->dense[-level], &C = h->dense[-level + 1];
    if (D.ntile == 0) return OHM_OK;
    if (D.nptile > 0 || D.nftile == 0) {
        // some continuing problem is not a whole number of 8^3 tiles
        OHM_TRY(launch_dense_stencil<T>(h, level, MODE_RESID, B, S, eta, coef_dev, res, 0, false, active, s));
        return launch_dense_restrict<T>(h, level, res, coarse, 3, active, s);
    }
    k_dense_resid_restrict<T><<<D.nftile, 256, 0, s>>>(D.ftiles, D.probs, C.probs, active, coef_dev, B, S, eta,
                                                        coarse, D.ncells, C.ncells);
    return check_launch("dense residual + restriction");
}

template <typename T>
ohm_status launch_dense_restrict(const ohm_hier *h, int fine_level, const T *fine, T *coarse, int ncomp,
                                 const int *active, hipStream_t s)
{
    const DenseLevelDev &F = h->dense[-fine_level], &C = h->dense[-fine_level + 1];
    if (C.ntile_all == 0) return OHM_OK;
    k_dense_restrict<T><<<C.ntile_all, 256, 0, s>>>(C.tiles_all, C.probs, F.probs, active, fine, F.ncells, coarse,
                                                    C.ncells, ncomp);
    return check_launch("dense restrict");
}

template <typename T>
ohm_status launch_dense_prolong(const ohm_hier *h, int coarse_level, const T *coarse, T *fine, int ncomp,
                                int accumulate, const int *active, hipStream_t s, const T *base)
{
    const DenseLevelDev &F = h->dense[-coarse_level - 1], &C = h->dense[-coarse_level];
    if (F.ntile == 0) return OHM_OK;
    if (base && !accumulate) return fail(OHM_ERR_ARG, "prolongation onto a base field must accumulate");
    if (accumulate && !base) base = fine;
    k_dense_prolong<T><<<F.ntile, 256, 0, s>>>(F.tiles, F.probs, C.probs, active, coarse, C.ncells, base, fine,
                                               F.ncells, ncomp);
    return check_launch("dense prolong");
}


constexpr int COARSE_MAX = 768;

ohm_status coarse_sizes(const ohm_hier *h, size_t *inv_elems, size_t *aug_elems)
{
    size_t a = 0, b = 0;
    for (const auto &P : h->probs) {
        const int *d = P.dims[-P.min_level];
        long long n3 = 3LL * d[0] * d[1] * d[2];
        if (n3 <= COARSE_MAX) {
            a += (size_t)(n3 * n3);
            b += (size_t)(2 * n3 * n3);
        }
    }
    *inv_elems = a;
    *aug_elems = b;
    return OHM_OK;
}

// Host-side job list, one per problem with a dense coarsest solve.
static std::vector<CoarseJob> coarse_jobs(const ohm_hier *h, const double *lam_dt_host, int depth_filter)
{
    std::vector<CoarseJob> jobs;
    long long io = 0, ao = 0, eo = 0;
    for (int p = 0; p < h->nprob; ++p) {
        const auto &P = h->probs[p];
        const int dd = -P.min_level;
        const int *d = P.dims[dd];
        const int n3 = 3 * d[0] * d[1] * d[2];
        if (n3 > COARSE_MAX) continue;
        CoarseJob J;
        J.prob = p;
        J.n3 = n3;
        J.inv_off = io;
        J.aug_off = ao;
        J.eta_off = eo;
        io += (long long)n3 * n3;
        ao += 2LL * n3 * n3;
        eo += n3 / 3;
        J.q.nx = d[0];
        J.q.ny = d[1];
        J.q.nz = d[2];
        J.q.active = 0;
        J.q.off = P.doff[dd];
        const double hh = P.dx0 * (double)(1 << dd);
        J.q.inv_h2 = 1.0 / (hh * hh);
        J.lam_dt = lam_dt_host ? lam_dt_host[p] : 0.0;
        if (depth_filter == 0 || depth_filter == dd) jobs.push_back(J);
    }
    return jobs;
}

void coarse_plan(ohm_hier *h, const double *lam_dt_host, void *jobs_host, int *force_host, int *njobs)
{
    for (int d = 0; d < 17; ++d) njobs[d] = 0;
    if (h->cinv_lamdt.size() != (size_t)h->nprob) h->cinv_lamdt.assign(h->nprob, -1.0);
    CoarseJob *J = (CoarseJob *)jobs_host;
    for (int d = 1; d <= -h->min_level; ++d) {
        const std::vector<CoarseJob> jobs = coarse_jobs(h, lam_dt_host, d);
        for (size_t j = 0; j < jobs.size(); ++j) {
            const int p = jobs[j].prob;
            J[(size_t)d * h->nprob + j] = jobs[j];
            force_host[(size_t)d * h->nprob + j] = (h->cinv_lamdt[p] != lam_dt_host[p]) ? 1 : 0;
            h->cinv_lamdt[p] = lam_dt_host[p];
        }
        njobs[d] = (int)jobs.size();
    }
}

size_t coarse_storage_bytes(const ohm_hier *h)
{
    size_t inv_elems = 0, aug_elems = 0, eta_elems = 0;
    coarse_sizes(h, &inv_elems, &aug_elems);
    if (inv_elems == 0) return 0;
    for (const CoarseJob &J : coarse_jobs(h, nullptr, 0)) eta_elems += (size_t)(J.n3 / 3);
    return sizeof(double) * (inv_elems + eta_elems) + sizeof(int) * (size_t)h->nprob;
}

ohm_status ensure_coarse_storage(ohm_hier *h)
{
    size_t inv_elems = 0, aug_elems = 0;
    coarse_sizes(h, &inv_elems, &aug_elems);
    if (inv_elems == 0 || h->d_coarse_inv) return OHM_OK;
    OHM_HIP(hipMalloc((void **)&h->d_coarse_inv, sizeof(double) * inv_elems));
    // saved resistivity: one slot of the coarsest grid's cells per job, at
    // the job's eta_off
    size_t eta_elems = 0;
    for (const CoarseJob &J : coarse_jobs(h, nullptr, 0)) eta_elems += (size_t)(J.n3 / 3);
    OHM_HIP(hipMalloc((void **)&h->d_coarse_eta, sizeof(double) * eta_elems));
    OHM_HIP(hipMalloc((void **)&h->d_coarse_flags, sizeof(int) * (size_t)h->nprob));
    return OHM_OK;
}

ohm_status launch_coarse_build(ohm_hier *h, const double *const *eta_dense, const void *jobs_dev,
                               const int *force_dev, const int *njobs, double *aug, hipStream_t s)
{
    // inverses live in the handle; each job is rebuilt only when forced (new
    // lam_dt) or when its coarsest resistivity differs from the saved copy
    size_t inv_elems = 0, aug_elems = 0;
    coarse_sizes(h, &inv_elems, &aug_elems);
    if (inv_elems == 0) return OHM_OK;
    if (!h->d_coarse_inv) return fail(OHM_ERR_ARG, "internal: coarse inverse storage not allocated");
    for (int d = 1; d <= -h->min_level; ++d) {
        if (njobs[d] == 0) continue;
        const CoarseJob *jd = (const CoarseJob *)jobs_dev + (size_t)d * h->nprob;
        const int *fo = force_dev + (size_t)d * h->nprob;
        int *fl = h->d_coarse_flags;   // reused per depth: the launches are stream-ordered
        int maxn = 0;
        for (const CoarseJob &J : coarse_jobs(h, nullptr, d)) maxn = std::max(maxn, J.n3);
        k_coarse_check<<<(unsigned)njobs[d], 256, 0, s>>>(jd, fo, eta_dense[d], h->d_coarse_eta, fl);
        OHM_TRY(check_launch("coarse check"));
        dim3 g(maxn, (unsigned)njobs[d]);
        k_coarse_assemble<<<g, 256, 0, s>>>(jd, fl, eta_dense[d], aug);
        OHM_TRY(check_launch("coarse assemble"));
        int minn = maxn;
        for (const CoarseJob &J : coarse_jobs(h, nullptr, d)) minn = std::min(minn, J.n3);
        // each kernel skips the jobs of the other's size range
        if (minn <= 32 * RG) {
            k_coarse_invert_reg<<<(unsigned)njobs[d], 1024, 0, s>>>(jd, fl, aug, h->d_coarse_inv);
            OHM_TRY(check_launch("coarse invert (registers)"));
        }
        if (maxn > 32 * RG) {
            k_coarse_invert<<<(unsigned)njobs[d], dim3(32, 32), 0, s>>>(jd, fl, aug, h->d_coarse_inv);
            OHM_TRY(check_launch("coarse invert"));
        }
    }
    return OHM_OK;
}

// x = inverse * r on the coarsest grid of every problem whose coarsest level is
// -depth (jobs_dev: that depth's slots of the step's job table)
template <typename T>
ohm_status launch_coarse_apply(const ohm_hier *h, int depth, const void *jobs_dev, int njobs, const double *inv,
                               const T *r, T *e, const int *active, hipStream_t s)
{
    if (njobs == 0) return OHM_OK;
    k_coarse_apply<T><<<dim3(COARSE_MAX_DEV / 64, njobs), 512, 0, s>>>((const CoarseJob *)jobs_dev, active, inv, r,
                                                                      e, h->dense[depth].ncells);
    return check_launch("coarse apply");
}


size_t coarse_job_bytes() { return sizeof(CoarseJob); }

#define INST(T)                                                                                                \
    template ohm_status launch_dense_smooth<T>(const ohm_hier *, int, T *, T *, const T *, const T *,           \
                                               const double *, int, bool, const int *, hipStream_t, int,       \
                                               const T *, T **, int);                                          \
    template ohm_status launch_dense_stencil<T>(const ohm_hier *, int, int, const T *, const T *, const T *,   \
                                                const double *, T *, int, bool, const int *, hipStream_t);     \
    template ohm_status launch_dense_restrict<T>(const ohm_hier *, int, const T *, T *, int, const int *,      \
                                                 hipStream_t);                                                 \
    template ohm_status launch_dense_resid_restrict<T>(const ohm_hier *, int, const T *, const T *, const T *, \
                                                       const double *, T *, T *, const int *, hipStream_t);    \
    template ohm_status launch_dense_prolong<T>(const ohm_hier *, int, const T *, T *, int, int, const int *,  \
                                                hipStream_t, const T *);                                       \
    template ohm_status launch_coarse_apply<T>(const ohm_hier *, int, const void *, int, const double *,       \
                                               const T *, T *, const int *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ohm
