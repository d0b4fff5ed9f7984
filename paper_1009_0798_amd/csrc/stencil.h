// Device-side discrete operator of eqs. (8)-(11) and the smoother diagonal of
// eqs. (21)-(23), on a cube of cells of edge W held in fast memory (LDS tile or
// registers).  All values are "times h^2": divide by h^2 for div F.
#pragma once

namespace ohm {

// h^2 (div F)_c at index p of a W^3 cube: sum over d != c of
// F_d[c](p + e_d/2) - F_d[c](p - e_d/2), where h F_d[c] = eta_face * (transverse
// four-point difference / 4 - normal difference).
template <typename T, int W>
__device__ __forceinline__ T divF_cube(const T *B0, const T *B1, const T *B2, const T *E, int p, int c)
{
    const int off[3] = {1, W, W * W};
    const T *Bt[3] = {B0, B1, B2};
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == c) continue;
        const int od = off[d], oc = off[c];
        const T *Bc = Bt[c];
        const T *Bd = Bt[d];
        T ep = (E[p] + E[p + od]) * T(0.5);
        T tp = (Bd[p + oc] + Bd[p + od + oc] - Bd[p - oc] - Bd[p + od - oc]) * T(0.25);
        T fp = ep * (tp - (Bc[p + od] - Bc[p]));
        T em = (E[p - od] + E[p]) * T(0.5);
        T tm = (Bd[p - od + oc] + Bd[p + oc] - Bd[p - od - oc] - Bd[p - oc]) * T(0.25);
        T fm = em * (tm - (Bc[p] - Bc[p - od]));
        acc += fp - fm;
    }
    return acc;
}

// h^2 alpha_c / lam_dt: the two d-face resistivities summed over d != c
template <typename T, int W>
__device__ __forceinline__ T alpha_cube(const T *E, int p, int c)
{
    const int off[3] = {1, W, W * W};
    T s = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == c) continue;
        s += (E[p - off[d]] + E[p]) * T(0.5) + (E[p] + E[p + off[d]]) * T(0.5);
    }
    return s;
}

}  // namespace ohm
