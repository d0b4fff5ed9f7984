// Device-side discrete operator of eqs. (8)-(11) and the smoother diagonal of
// eqs. (21)-(23), on a cube of cells of edge W held in fast memory (LDS tile or
// registers).
#pragma once

namespace ohm {

// All three components at index p of a W^3 cube, every neighbour read once:
//   dv[c] = 8 h^2 (div F)_c  and  al[c] = 2 h^2 alpha_c / lam_dt.
// Face fluxes are written without their power-of-two factors: with E the sum of
// the two cell resistivities at a face (twice the mean of eq. 11), t the
// transverse four-point sum (four times the difference of eq. 10) and n the
// normal difference (eq. 9), 8 h F = E (t - 4 n); scaling by 2, 4 or 8 is exact,
// so the callers fold the factors into their coefficients.  The central
// difference of B_d along c at p is shared by the +d and -d faces.
template <typename T, int W>
__device__ __forceinline__ void divF_all(const T *__restrict__ Bx, const T *__restrict__ By, const T *__restrict__ Bz,
                                         const T *__restrict__ E, int p, T dv[3], T al[3])
{
    constexpr int ox = 1, oy = W, oz = W * W;
    const T m4 = T(-4);
    const T e0 = E[p];
    const T Exp = e0 + E[p + ox], Exm = E[p - ox] + e0, Eyp = e0 + E[p + oy], Eym = E[p - oy] + e0,
            Ezp = e0 + E[p + oz], Ezm = E[p - oz] + e0;
    const T x0 = Bx[p], y0 = By[p], z0 = Bz[p];
    const T x_yp = Bx[p + oy], x_ym = Bx[p - oy], x_zp = Bx[p + oz], x_zm = Bx[p - oz];
    const T y_xp = By[p + ox], y_xm = By[p - ox], y_zp = By[p + oz], y_zm = By[p - oz];
    const T z_xp = Bz[p + ox], z_xm = Bz[p - ox], z_yp = Bz[p + oy], z_ym = Bz[p - oy];
    {   // component x: faces +-y (transverse d_x B_y) and +-z (d_x B_z)
        const T D = y_xp - y_xm;
        const T tp = D + (By[p + oy + ox] - By[p + oy - ox]), tm = (By[p - oy + ox] - By[p - oy - ox]) + D;
        const T gy = Eyp * fma(m4, x_yp - x0, tp) - Eym * fma(m4, x0 - x_ym, tm);
        const T D2 = z_xp - z_xm;
        const T tp2 = D2 + (Bz[p + oz + ox] - Bz[p + oz - ox]), tm2 = (Bz[p - oz + ox] - Bz[p - oz - ox]) + D2;
        const T gz = Ezp * fma(m4, x_zp - x0, tp2) - Ezm * fma(m4, x0 - x_zm, tm2);
        dv[0] = gy + gz;
    }
    {   // component y: faces +-x (d_y B_x) and +-z (d_y B_z)
        const T D = x_yp - x_ym;
        const T tp = D + (Bx[p + ox + oy] - Bx[p + ox - oy]), tm = (Bx[p - ox + oy] - Bx[p - ox - oy]) + D;
        const T gx = Exp * fma(m4, y_xp - y0, tp) - Exm * fma(m4, y0 - y_xm, tm);
        const T D2 = z_yp - z_ym;
        const T tp2 = D2 + (Bz[p + oz + oy] - Bz[p + oz - oy]), tm2 = (Bz[p - oz + oy] - Bz[p - oz - oy]) + D2;
        const T gz = Ezp * fma(m4, y_zp - y0, tp2) - Ezm * fma(m4, y0 - y_zm, tm2);
        dv[1] = gx + gz;
    }
    {   // component z: faces +-x (d_z B_x) and +-y (d_z B_y)
        const T D = x_zp - x_zm;
        const T tp = D + (Bx[p + ox + oz] - Bx[p + ox - oz]), tm = (Bx[p - ox + oz] - Bx[p - ox - oz]) + D;
        const T gx = Exp * fma(m4, z_xp - z0, tp) - Exm * fma(m4, z0 - z_xm, tm);
        const T D2 = y_zp - y_zm;
        const T tp2 = D2 + (By[p + oy + oz] - By[p + oy - oz]), tm2 = (By[p - oy + oz] - By[p - oy - oz]) + D2;
        const T gy = Eyp * fma(m4, z_yp - z0, tp2) - Eym * fma(m4, z0 - z_ym, tm2);
        dv[2] = gx + gy;
    }
    const T sx = Exm + Exp, sy = Eym + Eyp, sz = Ezm + Ezp;
    al[0] = sy + sz;
    al[1] = sx + sz;
    al[2] = sx + sy;
}

// al[c] = 2 h^2 alpha_c / lam_dt alone (same sums as divF_all)
template <typename T, int W>
__device__ __forceinline__ void alpha_all(const T *__restrict__ E, int p, T al[3])
{
    const T e0 = E[p];
    const T sx = (E[p - 1] + e0) + (e0 + E[p + 1]), sy = (E[p - W] + e0) + (e0 + E[p + W]),
            sz = (E[p - W * W] + e0) + (e0 + E[p + W * W]);
    al[0] = sy + sz;
    al[1] = sx + sz;
    al[2] = sx + sy;
}

// n / d for d >= 1 (the smoother's diagonal): hardware reciprocal, Newton steps
// (two in FP64, none in FP32) and one residual correction of the quotient; the
// result is within about one unit in the last place of the rounded quotient.
__device__ __forceinline__ float relax_div(float n, float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = n * r;
    return fmaf(fmaf(-d, q, n), r, q);
}
__device__ __forceinline__ double relax_div(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

// One point update of eq. (19) for the three components at p: with
// c8 = lam dt / (8 h^2) and c2 = lam dt / (2 h^2),
// B_c + (S_c - (B_c + c8 dv_c)) / (1 + c2 al_c).
template <typename T>
__device__ __forceinline__ T relax_point(T b, T s, T dv, T al, T c8, T c2)
{
    return b + relax_div(s - fma(c8, dv, b), fma(c2, al, T(1)));
}

}  // namespace ohm
