// One fused red-black sweep (eq. 19 with alpha of eqs. 21-23) of an 8^3 tile.
//
// The tile and a two-cell halo are staged in LDS.  The red half-sweep is
// computed on the tile and, redundantly, on the red cells of the first halo
// layer that face the tile (their neighbours come from the second layer); the
// black half-sweep on the tile then reads those updated red values.  This is
// the same arithmetic as two separate half-sweeps.  `Addr::at(x, y, z)` gives
// the element offset of tile-local cell (x, y, z), -2 <= x, y, z <= 9, inside a
// component of the field; every such cell must exist (no coarse-fine ghosts).
#pragma once

#include "stencil.h"

namespace ohm {

constexpr int SWEEP_THREADS = 512;
constexpr int TW2 = 8 + 4;               // tile edge with a two-cell halo
constexpr int TC2 = TW2 * TW2 * TW2;

__device__ __forceinline__ int tix2(int x, int y, int z) { return (x + 2) + TW2 * ((y + 2) + TW2 * (z + 2)); }

template <typename T, typename Addr>
__device__ __forceinline__ void fused_sweep_tile(const Addr &A, const T *__restrict__ B, long long cs,
                                                 const T *__restrict__ S, const T *__restrict__ eta,
                                                 T *__restrict__ out, const T cih2, T (*sB)[TC2], T *sE)
{
    for (int t = threadIdx.x; t < TC2; t += SWEEP_THREADS) {
        const int x = t % TW2 - 2, y = (t / TW2) % TW2 - 2, z = t / (TW2 * TW2) - 2;
        const long long gi = A.at(x, y, z);
#pragma unroll
        for (int c = 0; c < 3; ++c) sB[c][t] = B[c * cs + gi];
        sE[t] = eta[gi];
    }
    __syncthreads();
    // red half-sweep: thread u < 256 takes tile cell u of the red colour,
    // 256 <= u < 448 a red first-layer face cell
    T red[3];
    int rp = -1;
    {
        const int u = threadIdx.x;
        if (u < 448) {
            int x, y, z;
            if (u < 256) {
                z = u >> 5;
                y = (u >> 2) & 7;
                x = 2 * (u & 3) + ((y + z) & 1);
            } else {
                const int v = u - 256, f = v >> 5, w = v & 31;
                const int d = f >> 1, s = (f & 1) ? 8 : -1;
                const int bb = w >> 2, a = 2 * (w & 3) + ((s + bb) & 1);
                if (d == 0) { x = s; y = a; z = bb; }
                else if (d == 1) { x = a; y = s; z = bb; }
                else { x = a; y = bb; z = s; }
            }
            const int p = tix2(x, y, z);
            rp = p;
            const long long gi = A.at(x, y, z);
            T dv[3], al[3];
            divF_all<T, TW2>(sB[0], sB[1], sB[2], sE, p, dv, al);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T LB = sB[c][p] + cih2 * dv[c];
                red[c] = sB[c][p] + (S[c * cs + gi] - LB) / (T(1) + cih2 * al[c]);
            }
        }
    }
    __syncthreads();
    if (rp >= 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) sB[c][rp] = red[c];
    __syncthreads();
    // black half-sweep on the tile (threads 0..255)
    {
        const int u = threadIdx.x;
        T blk[3];
        int p = -1;
        if (u < 256) {
            const int z = u >> 5, y = (u >> 2) & 7, x = 2 * (u & 3) + (1 - ((y + z) & 1));
            p = tix2(x, y, z);
            const long long gi = A.at(x, y, z);
            T dv[3], al[3];
            divF_all<T, TW2>(sB[0], sB[1], sB[2], sE, p, dv, al);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T LB = sB[c][p] + cih2 * dv[c];
                blk[c] = sB[c][p] + (S[c * cs + gi] - LB) / (T(1) + cih2 * al[c]);
            }
        }
        __syncthreads();
        if (p >= 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) sB[c][p] = blk[c];
    }
    __syncthreads();
    {
        const int cell = threadIdx.x;
        const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
        const int p = tix2(x, y, z);
        const long long gi = A.at(x, y, z);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c * cs + gi] = sB[c][p];
    }
}

}  // namespace ohm
