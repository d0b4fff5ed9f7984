/*
 * ohm_ref.c -- FP64 CPU oracle primitives for the implicit ohmic-dissipation
 * scheme of Matsumoto (PASJ 2011, "An Implicit Scheme for Ohmic Dissipation
 * with Adaptive Mesh Refinement").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP library and is written as a plain cell-by-cell transcription.
 *
 * Grid: one uniform periodic level of nx*ny*nz cubic cells of width h.
 * A vector field is double[3][nz][ny][nx] (x fastest); a scalar double[nz][ny][nx].
 * Face fluxes: F[d][c][cell p] is component c of the flux vector F_d on the
 * face between cell p and cell p + e_d.  Entries with c == d are zero.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

typedef struct { int nx, ny, nz; } dims_t;

static inline int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

/* linear index of cell (i,j,k) with periodic wrap */
static inline size_t at(dims_t g, int i, int j, int k)
{
    return ((size_t)wrap(k, g.nz) * g.ny + wrap(j, g.ny)) * g.nx + wrap(i, g.nx);
}

/* offset a cell index by unit vector e_d times s */
static inline void step(int d, int s, int *i, int *j, int *k)
{
    if (d == 0) *i += s; else if (d == 1) *j += s; else *k += s;
}

/*
 * Face fluxes, section 2.1, equations (4)-(6) with the differences (9)-(10)
 * and the face resistivity (11):
 *   F_d[c] = eta_face * ( d_c B_d  -  d_d B_c ),  c != d,
 * where d_d B_c is the compact difference across the face and d_c B_d is the
 * four-point transverse difference averaged over the two cells of the face.
 */
void oref_flux(int nx, int ny, int nz, double h, const double *B, const double *eta, double *F)
{
    dims_t g = {nx, ny, nz};
    size_t N = (size_t)nx * ny * nz;
    memset(F, 0, sizeof(double) * 9 * N);
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
        size_t p = at(g, i, j, k);
        for (int d = 0; d < 3; ++d) {
            int a = i, b = j, c_ = k;             /* the cell across the face */
            step(d, 1, &a, &b, &c_);
            size_t q = at(g, a, b, c_);
            double eta_f = 0.5 * (eta[p] + eta[q]);                 /* (11) */
            for (int c = 0; c < 3; ++c) {
                if (c == d) continue;
                const double *Bc = B + (size_t)c * N;
                const double *Bd = B + (size_t)d * N;
                double normal = (Bc[q] - Bc[p]) / h;                /* (9)  */
                /* (10): B_d at p +- e_c and p + e_d +- e_c */
                int i1 = i, j1 = j, k1 = k; step(c, 1, &i1, &j1, &k1);
                int i2 = i, j2 = j, k2 = k; step(c, -1, &i2, &j2, &k2);
                int i3 = a, j3 = b, k3 = c_; step(c, 1, &i3, &j3, &k3);
                int i4 = a, j4 = b, k4 = c_; step(c, -1, &i4, &j4, &k4);
                double trans = (Bd[at(g, i1, j1, k1)] + Bd[at(g, i3, j3, k3)]
                              - Bd[at(g, i2, j2, k2)] - Bd[at(g, i4, j4, k4)]) / (4.0 * h);
                F[((size_t)d * 3 + c) * N + p] = eta_f * (trans - normal);
            }
        }
    }
}

/* Divergence of face fluxes, equation (8): sum over d of the flux difference
 * between the two d-faces of the cell, divided by h. */
void oref_div(int nx, int ny, int nz, double h, const double *F, double *out)
{
    dims_t g = {nx, ny, nz};
    size_t N = (size_t)nx * ny * nz;
    for (int c = 0; c < 3; ++c)
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
        size_t p = at(g, i, j, k);
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            int a = i, b = j, c_ = k;
            step(d, -1, &a, &b, &c_);
            s += (F[((size_t)d * 3 + c) * N + p] - F[((size_t)d * 3 + c) * N + at(g, a, b, c_)]) / h;
        }
        out[(size_t)c * N + p] = s;
    }
}

/* out = B + coef * div F(B): the operator L of equation (13) when
 * coef = lambda*dt; with coef = -(1-lambda)*dt and B = b it is the source S
 * of equation (14). */
void oref_apply(int nx, int ny, int nz, double h, const double *B, const double *eta,
                double coef, double *out)
{
    size_t N = (size_t)nx * ny * nz;
    double *F = (double *)malloc(sizeof(double) * 9 * N);
    double *D = (double *)malloc(sizeof(double) * 3 * N);
    oref_flux(nx, ny, nz, h, B, eta, F);
    oref_div(nx, ny, nz, h, F, D);
    for (size_t t = 0; t < 3 * N; ++t) out[t] = B[t] + coef * D[t];
    free(F);
    free(D);
}

/* R = S - L B, equation (20) */
void oref_residual(int nx, int ny, int nz, double h, const double *B, const double *S,
                   const double *eta, double lam_dt, double *R)
{
    size_t N = (size_t)nx * ny * nz;
    oref_apply(nx, ny, nz, h, B, eta, lam_dt, R);
    for (size_t t = 0; t < 3 * N; ++t) R[t] = S[t] - R[t];
}

/* alpha_c of equations (21)-(23): lam_dt times the sum, over the two
 * directions d != c, of the two d-face resistivities divided by h^2. */
void oref_alpha(int nx, int ny, int nz, double h, const double *eta, double lam_dt, double *alpha)
{
    dims_t g = {nx, ny, nz};
    size_t N = (size_t)nx * ny * nz;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
        size_t p = at(g, i, j, k);
        double ef[3];                       /* eta_{-1/2} + eta_{+1/2} along d */
        for (int d = 0; d < 3; ++d) {
            int a = i, b = j, c_ = k; step(d, 1, &a, &b, &c_);
            int a2 = i, b2 = j, c2 = k; step(d, -1, &a2, &b2, &c2);
            ef[d] = 0.5 * (eta[p] + eta[at(g, a, b, c_)]) + 0.5 * (eta[p] + eta[at(g, a2, b2, c2)]);
        }
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int d = 0; d < 3; ++d) if (d != c) s += ef[d] / (h * h);
            alpha[(size_t)c * N + p] = lam_dt * s;
        }
    }
}

/*
 * One half-sweep of the red-black smoother, equation (19): every cell whose
 * colour (i+j+k) mod 2 equals `colour` receives B += R / (1 + alpha), with R
 * the residual (20) of the state at the start of the half-sweep (all cells of
 * the colour are updated together).
 */
void oref_rb_halfsweep(int nx, int ny, int nz, double h, double *B, const double *S,
                       const double *eta, double lam_dt, int colour)
{
    size_t N = (size_t)nx * ny * nz;
    double *R = (double *)malloc(sizeof(double) * 3 * N);
    double *al = (double *)malloc(sizeof(double) * 3 * N);
    oref_residual(nx, ny, nz, h, B, S, eta, lam_dt, R);
    oref_alpha(nx, ny, nz, h, eta, lam_dt, al);
    dims_t g = {nx, ny, nz};
    for (int c = 0; c < 3; ++c)
    for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
        if (((i + j + k) & 1) != colour) continue;
        size_t p = (size_t)c * N + at(g, i, j, k);
        B[p] += R[p] / (1.0 + al[p]);
    }
    free(R);
    free(al);
}

/* Averaging restriction: coarse cell = mean of its 8 children (per component). */
void oref_restrict(int nxc, int nyc, int nzc, int ncomp, const double *fine, double *coarse)
{
    dims_t gc = {nxc, nyc, nzc};
    dims_t gf = {2 * nxc, 2 * nyc, 2 * nzc};
    size_t Nc = (size_t)nxc * nyc * nzc, Nf = 8 * Nc;
    for (int c = 0; c < ncomp; ++c)
    for (int k = 0; k < nzc; ++k)
    for (int j = 0; j < nyc; ++j)
    for (int i = 0; i < nxc; ++i) {
        double s = 0.0;
        for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di)
            s += fine[(size_t)c * Nf + at(gf, 2 * i + di, 2 * j + dj, 2 * k + dk)];
        coarse[(size_t)c * Nc + at(gc, i, j, k)] = s / 8.0;
    }
}

/*
 * Cell-centred trilinear prolongation.  A fine cell sits in one octant of its
 * parent; along each axis the value is 3/4 of the parent plus 1/4 of the
 * coarse neighbour on the fine cell's side, giving the weights 27, 9, 3, 1
 * over 64.  The interpolant is ADDED to `fine` (coarse-grid correction).
 */
void oref_prolong_add(int nxc, int nyc, int nzc, int ncomp, const double *coarse, double *fine)
{
    dims_t gc = {nxc, nyc, nzc};
    dims_t gf = {2 * nxc, 2 * nyc, 2 * nzc};
    size_t Nc = (size_t)nxc * nyc * nzc, Nf = 8 * Nc;
    for (int c = 0; c < ncomp; ++c)
    for (int K = 0; K < gf.nz; ++K)
    for (int J = 0; J < gf.ny; ++J)
    for (int I = 0; I < gf.nx; ++I) {
        int i = I >> 1, j = J >> 1, k = K >> 1;
        int si = (I & 1) ? 1 : -1, sj = (J & 1) ? 1 : -1, sk = (K & 1) ? 1 : -1;
        double v = 0.0;
        for (int ck = 0; ck < 2; ++ck)
        for (int cj = 0; cj < 2; ++cj)
        for (int ci = 0; ci < 2; ++ci) {
            double w = (ci ? 0.25 : 0.75) * (cj ? 0.25 : 0.75) * (ck ? 0.25 : 0.75);
            v += w * coarse[(size_t)c * Nc + at(gc, i + ci * si, j + cj * sj, k + ck * sk)];
        }
        fine[(size_t)c * Nf + at(gf, I, J, K)] += v;
    }
}

/* threads the OpenMP loops above use */
#ifdef _OPENMP
#include <omp.h>
int oref_threads(void) { return omp_get_max_threads(); }
void oref_set_threads(int n) { omp_set_num_threads(n); }
#else
int oref_threads(void) { return 1; }
void oref_set_threads(int n) { (void)n; }
#endif
