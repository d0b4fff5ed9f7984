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

namespace ohm {

// All three components at once: h^2 (div F)_c and h^2 alpha_c / lam_dt at index
// p of a W^3 cube, with every neighbour read from the cube once (46 reads
// instead of about 110 for three separate divF_cube calls).  Same expression
// tree as divF_cube / alpha_cube for each component.
template <typename T, int W>
__device__ __forceinline__ void divF_all(const T *__restrict__ Bx, const T *__restrict__ By, const T *__restrict__ Bz,
                                         const T *__restrict__ E, int p, T dv[3], T al[3])
{
    constexpr int ox = 1, oy = W, oz = W * W;
    const T half = T(0.5), quarter = T(0.25);
    const T e0 = E[p], exp_ = E[p + ox], exm = E[p - ox], eyp = E[p + oy], eym = E[p - oy], ezp = E[p + oz],
            ezm = E[p - oz];
    // B_x: p, p+-oy, p+-oz, p+-ox+-oy, p+-ox+-oz
    const T x0 = Bx[p], x_yp = Bx[p + oy], x_ym = Bx[p - oy], x_zp = Bx[p + oz], x_zm = Bx[p - oz];
    const T x_pp_y = Bx[p + ox + oy], x_pm_y = Bx[p + ox - oy], x_mp_y = Bx[p - ox + oy], x_mm_y = Bx[p - ox - oy];
    const T x_pp_z = Bx[p + ox + oz], x_pm_z = Bx[p + ox - oz], x_mp_z = Bx[p - ox + oz], x_mm_z = Bx[p - ox - oz];
    // B_y: p, p+-ox, p+-oz, p+-oy+-ox, p+-oy+-oz
    const T y0 = By[p], y_xp = By[p + ox], y_xm = By[p - ox], y_zp = By[p + oz], y_zm = By[p - oz];
    const T y_pp_x = By[p + oy + ox], y_pm_x = By[p + oy - ox], y_mp_x = By[p - oy + ox], y_mm_x = By[p - oy - ox];
    const T y_pp_z = By[p + oy + oz], y_pm_z = By[p + oy - oz], y_mp_z = By[p - oy + oz], y_mm_z = By[p - oy - oz];
    // B_z: p, p+-ox, p+-oy, p+-oz+-ox, p+-oz+-oy
    const T z0 = Bz[p], z_xp = Bz[p + ox], z_xm = Bz[p - ox], z_yp = Bz[p + oy], z_ym = Bz[p - oy];
    const T z_pp_x = Bz[p + oz + ox], z_pm_x = Bz[p + oz - ox], z_mp_x = Bz[p - oz + ox], z_mm_x = Bz[p - oz - ox];
    const T z_pp_y = Bz[p + oz + oy], z_pm_y = Bz[p + oz - oy], z_mp_y = Bz[p - oz + oy], z_mm_y = Bz[p - oz - oy];
    // face resistivities
    const T exf_p = (e0 + exp_) * half, exf_m = (exm + e0) * half;
    const T eyf_p = (e0 + eyp) * half, eyf_m = (eym + e0) * half;
    const T ezf_p = (e0 + ezp) * half, ezf_m = (ezm + e0) * half;
    // component x: d = y (B_d = B_y, transverse along x), d = z (B_d = B_z)
    {
        T acc = T(0);
        T tp = (y_xp + y_pp_x - y_xm - y_pm_x) * quarter;
        T fp = eyf_p * (tp - (x_yp - x0));
        T tm = (y_mp_x + y_xp - y_mm_x - y_xm) * quarter;
        T fm = eyf_m * (tm - (x0 - x_ym));
        acc += fp - fm;
        tp = (z_xp + z_pp_x - z_xm - z_pm_x) * quarter;
        fp = ezf_p * (tp - (x_zp - x0));
        tm = (z_mp_x + z_xp - z_mm_x - z_xm) * quarter;
        fm = ezf_m * (tm - (x0 - x_zm));
        acc += fp - fm;
        dv[0] = acc;
    }
    // component y: d = x (B_d = B_x, transverse along y), d = z (B_d = B_z)
    {
        T acc = T(0);
        T tp = (x_yp + x_pp_y - x_ym - x_pm_y) * quarter;
        T fp = exf_p * (tp - (y_xp - y0));
        T tm = (x_mp_y + x_yp - x_mm_y - x_ym) * quarter;
        T fm = exf_m * (tm - (y0 - y_xm));
        acc += fp - fm;
        tp = (z_yp + z_pp_y - z_ym - z_pm_y) * quarter;
        fp = ezf_p * (tp - (y_zp - y0));
        tm = (z_mp_y + z_yp - z_mm_y - z_ym) * quarter;
        fm = ezf_m * (tm - (y0 - y_zm));
        acc += fp - fm;
        dv[1] = acc;
    }
    // component z: d = x (B_d = B_x, transverse along z), d = y (B_d = B_y)
    {
        T acc = T(0);
        T tp = (x_zp + x_pp_z - x_zm - x_pm_z) * quarter;
        T fp = exf_p * (tp - (z_xp - z0));
        T tm = (x_mp_z + x_zp - x_mm_z - x_zm) * quarter;
        T fm = exf_m * (tm - (z0 - z_xm));
        acc += fp - fm;
        tp = (y_zp + y_pp_z - y_zm - y_pm_z) * quarter;
        fp = eyf_p * (tp - (z_yp - z0));
        tm = (y_mp_z + y_zp - y_mm_z - y_zm) * quarter;
        fm = eyf_m * (tm - (z0 - z_ym));
        acc += fp - fm;
        dv[2] = acc;
    }
    // alpha sums: the two d-face resistivities over d != c
    const T sx = exf_m + exf_p, sy = eyf_m + eyf_p, sz = ezf_m + ezf_p;
    al[0] = sy + sz;
    al[1] = sx + sz;
    al[2] = sx + sy;
}

}  // namespace ohm
