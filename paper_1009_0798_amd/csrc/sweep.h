// One fused red-black sweep (eq. 19 with alpha of eqs. 21-23) of an 8^3 tile.
//
// The tile and a two-cell halo are staged in LDS.  The red half-sweep is
// computed on the tile and, redundantly, on the red cells of the first halo
// layer that face the tile (their neighbours come from the second layer); the
// black half-sweep on the tile then reads those updated red values.  This is
// the same arithmetic as two separate half-sweeps.  `Addr::at(x, y, z)` gives
// the element offset of tile-local cell (x, y, z), -2 <= x, y, z <= 9, inside a
// component of the field.  Without `Addr::ghosts` every such cell is a level
// cell; with it, `Addr::entry(x, y, z)` is the neighbour entry of the cell's
// block (a level block, or ghost block -1-entry of the ghost arrays A.G, A.EG
// with component stride A.gcs), tile values of ghost blocks are loaded from
// those arrays, and first-layer red cells of ghost blocks keep their values
// (ghost values are fixed during smoothing).
// With ZERO the input field is zero and is not read (B may be null; so must
// be the ghost values): the red update reduces to S / diag and the tile starts
// from zeros, which gives the same values as a sweep over an explicitly zeroed
// field.  A `Coarse` object
// with active = true adds a coarse-grid correction to every tile value as it
// is loaded (prolongation fused into the first post-smoothing sweep); its
// load() issues the global reads of whatever it stages, stage() stores them in
// LDS (a barrier follows) and add(x, y, z, c, v) returns v plus the correction.
#pragma once

#include "common.h"
#include "stencil.h"

namespace ohm {

constexpr int SWEEP_THREADS = 512;
constexpr int TW2 = 8 + 4;               // tile edge with a two-cell halo
constexpr int TC2 = TW2 * TW2 * TW2;

__device__ __forceinline__ int tix2(int x, int y, int z) { return (x + 2) + TW2 * ((y + 2) + TW2 * (z + 2)); }

// two consecutive elements, loaded and stored as one 2 sizeof(T) access
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};

template <typename T>
struct NoCoarse {
    static constexpr bool active = false;
    __device__ __forceinline__ void load() {}
    __device__ __forceinline__ void stage() {}
    __device__ __forceinline__ T add(int, int, int, int, T v) const { return v; }
};

// Element at a byte offset from a wavefront-uniform base: the offset stays a
// 32-bit VGPR and the base an SGPR pair, so the 3 components and eta share one
// address computation.  The launchers check that every level array fits in
// 4 GiB.
template <typename T>
__device__ __forceinline__ T load_at(const T *base, unsigned off)
{
    return *(const T *)((const char *)base + off);
}
template <typename T>
__device__ __forceinline__ Pair<T> load_pair(const T *base, unsigned off)
{
    return *(const Pair<T> *)((const char *)base + off);
}
template <typename T>
__device__ __forceinline__ void store_at(T *base, unsigned off, T v)
{
    *(T *)((char *)base + off) = v;
}

// Trilinear correction (27/9/3/1 over 64) from the next coarser grid, a dense
// grid q, for the tile of fine origin 8 (i, j, k): the 8^3 coarse cells that
// hold the parents of the tile's cells and their neighbours (origin
// 4 (i, j, k) - 2, periodic) are staged in LDS; the weights and the order of
// the sum are those of the stand-alone prolongation kernels.
template <typename T>
struct TileCoarse {
    static constexpr bool active = true;
    const T *coarse;
    long long ccs;
    DenseProbDev q;
    int i0, j0, k0;
    T *sC;      // [3][512] in LDS
    T r[3];
    __device__ __forceinline__ void load()
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int t = threadIdx.x + SWEEP_THREADS * k, c = t >> 9, m = t & 511;
            const int i = (i0 + (m & 7) + q.nx) % q.nx, j = (j0 + ((m >> 3) & 7) + q.ny) % q.ny,
                      kk = (k0 + (m >> 6) + q.nz) % q.nz;
            r[k] = coarse[c * ccs + q.off + i + (long long)q.nx * (j + (long long)q.ny * kk)];
        }
    }
    __device__ __forceinline__ void stage()
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) sC[threadIdx.x + SWEEP_THREADS * k] = r[k];
    }
    __device__ __forceinline__ T add(int x, int y, int z, int c, T base) const
    {
        const int i = (x >> 1) + 2, j = (y >> 1) + 2, k = (z >> 1) + 2;
        const int i1 = i + ((x & 1) ? 1 : -1), j1 = j + ((y & 1) ? 1 : -1), k1 = k + ((z & 1) ? 1 : -1);
        const T *C = sC + 512 * c;
        auto at = [](int a, int bb, int cc) { return a + 8 * (bb + 8 * cc); };
        T v = T(27) * C[at(i, j, k)] + T(9) * (C[at(i1, j, k)] + C[at(i, j1, k)] + C[at(i, j, k1)]) +
              T(3) * (C[at(i1, j1, k)] + C[at(i1, j, k1)] + C[at(i, j1, k1)]) + C[at(i1, j1, k1)];
        v *= T(1.0 / 64.0);
        return base + v;
    }
};

// The result goes to `out` as TO (T, or double from an FP32 sweep), with the
// same element offsets and component stride as the input.
// 16 bytes from global memory straight into LDS: lane l of the wavefront
// writes dst + 16 l bytes (dst uniform over the wavefront)
__device__ __forceinline__ void lds_load16(const void *src, void *dst)
{
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)src,
                                     (void __attribute__((address_space(3))) *)dst, 16, 0, 0);
}

template <typename T, bool ZERO, typename Addr, typename Coarse = NoCoarse<T>, typename TO = T, int TS = TC2,
          bool DIRECT = false>
__device__ __forceinline__ void fused_sweep_tile(const Addr &A, const T *__restrict__ B, long long cs,
                                                 const T *__restrict__ S, const T *__restrict__ eta,
                                                 TO *__restrict__ out, const T cih2, T (*sB)[TS], T *sE,
                                                 Coarse cor = Coarse())
{
    const int u = threadIdx.x;
    const T *B0 = B, *B1 = ZERO ? B : B + cs, *B2 = ZERO ? B : B + 2 * cs;
    const T *S0 = S, *S1 = S + cs, *S2 = S + 2 * cs;
    if constexpr (DIRECT) {
        // FP64 tile pairs loaded straight into LDS: pair P = u + 512 k of
        // the 864 (plane-major, as tix2 lays them out) lands at element 2 P,
        // which is lane order within each wavefront; the lanes past the last
        // pair reload pair 863 into 64 elements of padding (TS >= TC2 + 64)
        static_assert(sizeof(T) == 8 && !ZERO && !Addr::ghosts && !Coarse::active && TS >= TC2 + 64,
                      "direct tile loads are for plain FP64 sweeps");
        constexpr int NPC = (TW2 / 2) * TW2, NP = NPC * TW2;
        const int w = u >> 6;
        // the waves of a group that issues its tile's loads take precedence
        // over the other resident group's updates until the loads are out
        __builtin_amdgcn_s_setprio(3);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int first = SWEEP_THREADS * k + 64 * w;
            if (first < NP) {
                const int P = min(u + SWEEP_THREADS * k, NP - 1);
                const int pc = P % NPC, z = P / NPC - 2;
                const int x = 2 * (pc % (TW2 / 2)) - 2, y = pc / (TW2 / 2) - 2;
                const unsigned off = (unsigned)A.at(x, y, z) * (unsigned)sizeof(T);
                lds_load16((const char *)B0 + off, &sB[0][2 * first]);
                lds_load16((const char *)B1 + off, &sB[1][2 * first]);
                lds_load16((const char *)B2 + off, &sB[2][2 * first]);
                lds_load16((const char *)eta + off, &sE[2 * first]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    } else {
    // tile load in pairs of x-neighbours (x even, so a pair never straddles a
    // block or a periodic wrap and is 2 sizeof(T) aligned): thread u < 432
    // owns pair column (px, y) = u mod 72 and the planes z = 2 (u / 72) - 2
    // and the next one; all global loads first, then the LDS stores
    constexpr int NPC = (TW2 / 2) * TW2;     // pair columns per plane
    const bool loader = u < 6 * NPC;
    const int pc = u % NPC, zq = u / NPC;
    const int x = 2 * (pc % (TW2 / 2)) - 2, y = pc / (TW2 / 2) - 2;
    Pair<T> v[2][4];
    if (Coarse::active) cor.load();
    if (loader) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int z = 2 * zq + k - 2;
            if constexpr (Addr::ghosts) {
                const int n = A.entry(x, y, z);
                const bool g = n < 0;
                const unsigned off = ((unsigned)(g ? -1 - n : n) * (unsigned)NC + (unsigned)A.local(x, y, z)) *
                                     (unsigned)sizeof(T);
                if (!ZERO) {
                    v[k][0] = load_pair(g ? A.G : B0, off);
                    v[k][1] = load_pair(g ? A.G + A.gcs : B1, off);
                    v[k][2] = load_pair(g ? A.G + 2 * A.gcs : B2, off);
                }
                v[k][3] = load_pair(g ? A.EG : eta, off);
            } else {
                const unsigned off = (unsigned)A.at(x, y, z) * (unsigned)sizeof(T);
                if (!ZERO) {
                    v[k][0] = load_pair(B0, off);
                    v[k][1] = load_pair(B1, off);
                    v[k][2] = load_pair(B2, off);
                }
                v[k][3] = load_pair(eta, off);
            }
        }
    }
    if (Coarse::active) {
        cor.stage();
        __syncthreads();
    }
    if (loader) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int z = 2 * zq + k - 2;
            const int t = tix2(x, y, z);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Pair<T> w;
                w.a = cor.add(x, y, z, c, ZERO ? T(0) : v[k][c].a);
                w.b = cor.add(x + 1, y, z, c, ZERO ? T(0) : v[k][c].b);
                *(Pair<T> *)&sB[c][t] = w;
            }
            *(Pair<T> *)&sE[t] = v[k][3];
        }
    }
    __syncthreads();
    }
    const T c8 = cih2 * T(0.125), c2 = cih2 * T(0.5);
    // the black cell of this thread and its S values, loaded before the red
    // half-sweep so that their latency overlaps it
    int pb = -1;
    T sbk[3];
    if (u < 256) {
        const int z = u >> 5, y = (u >> 2) & 7, x = 2 * (u & 3) + (1 - ((y + z) & 1));
        pb = tix2(x, y, z);
        const unsigned off = (unsigned)A.at(x, y, z) * (unsigned)sizeof(T);
        sbk[0] = load_at(S0, off);
        sbk[1] = load_at(S1, off);
        sbk[2] = load_at(S2, off);
    }
    // red half-sweep: thread u < 256 takes tile cell u of the red colour,
    // 256 <= u < 448 a red first-layer face cell
    T red[3];
    int rp = -1;
    if (u < 448) {
        int x, y, z;
        if (u < 256) {
            z = u >> 5;
            y = (u >> 2) & 7;
            x = 2 * (u & 3) + ((y + z) & 1);
        } else {
            const int w = u - 256, f = w >> 5, k = w & 31;
            const int d = f >> 1, s = (f & 1) ? 8 : -1;
            const int bb = k >> 2, a = 2 * (k & 3) + ((s + bb) & 1);
            if (d == 0) { x = s; y = a; z = bb; }
            else if (d == 1) { x = a; y = s; z = bb; }
            else { x = a; y = bb; z = s; }
        }
        bool upd = true;
        if constexpr (Addr::ghosts) upd = u < 256 || A.entry(x, y, z) >= 0;
        if (upd) {
            rp = tix2(x, y, z);
            const unsigned off = (unsigned)A.at(x, y, z) * (unsigned)sizeof(T);
            const T s3[3] = {load_at(S0, off), load_at(S1, off), load_at(S2, off)};
            T al[3];
            if (ZERO) {
                alpha_all<T, TW2>(sE, rp, al);
#pragma unroll
                for (int c = 0; c < 3; ++c) red[c] = relax_div(s3[c], fma(c2, al[c], T(1)));
            } else {
                T dv[3];
                divF_all<T, TW2>(sB[0], sB[1], sB[2], sE, rp, dv, al);
#pragma unroll
                for (int c = 0; c < 3; ++c) red[c] = relax_point(sB[c][rp], s3[c], dv[c], al[c], c8, c2);
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
        T blk[3];
        if (u < 256) {
            T dv[3], al[3];
            divF_all<T, TW2>(sB[0], sB[1], sB[2], sE, pb, dv, al);
#pragma unroll
            for (int c = 0; c < 3; ++c) blk[c] = relax_point(sB[c][pb], sbk[c], dv[c], al[c], c8, c2);
        }
        __syncthreads();
        if (pb >= 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) sB[c][pb] = blk[c];
    }
    __syncthreads();
    {
        const int x = u & 7, y = (u >> 3) & 7, z = u >> 6;
        const int p = tix2(x, y, z);
        const unsigned off = (unsigned)A.at(x, y, z) * (unsigned)sizeof(TO);
        store_at(out, off, TO(sB[0][p]));
        store_at(out + cs, off, TO(sB[1][p]));
        store_at(out + 2 * cs, off, TO(sB[2][p]));
    }
}

}  // namespace ohm
