/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the free-energy lattice Boltzmann
 * step analysed by Pooley & Furtado, "Eliminating spurious velocities in the
 * free energy lattice Boltzmann method".  It exists to check the GPU library;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source, header, table or helper with the GPU
 * library, and the GPU library never calls it.
 *
 * The method is an explicit iteration, so this file takes its steps in the
 * paper's order and notation:
 *   moments                     Section "Model", Eq. (rho)
 *   gradient / Laplacian        Eqs. (xderiv), (laplace); 3D Eq. (laplacian3d)
 *   van der Waals bulk pressure Eq. (p0); c_s^2 = dp0/drho, Appendix A
 *   lambda term                 Eq. (viscous)
 *   equilibrium                 Eq. (equilibrium), Eq. (feq0)
 *   body force (forcing scheme) Section "Using a forcing method"
 *   BGK collision + streaming   Eq. (latbolt)
 *
 * State representation: f[i][z][y][x] holds f_i(r,t), the population at
 * site r after streaming (the paper's f_i(r,t)).  All arrays are SoA with x
 * fastest.  Every boundary is periodic, except the binary stepper's optional
 * walls (below).  Units: dx = dt = c = 1.
 *
 * Readings of the paper taken here (each is listed with its justification in
 * the design notes of the repository):
 *  - the rest equilibrium is f0eq = rho - sum_{i>=1} f_i^eq (the printed
 *    "f_i" would make the definition vacuous; mass moment, Appendix A);
 *  - the w^t term carries kappa (Eq. (pt) and the kappa rho lap rho stencil
 *    label in Eq. (expand2));
 *  - w^xy_i = +1/4 on e5,e6 and -1/4 on e7,e8 (the constraint list after
 *    Eq. (fi)); the summary's "w^xy_5-8 = 1/4" loses the sign;
 *  - D3Q19: w_1-6 = w^p_1-6 = w^t_1-6 = 1/6 and w^xx_1,2 = w^yy_3,4 =
 *    w^zz_5,6 = 5/12 (the printed 1/3 values violate the second-moment
 *    condition of Appendix A and the stated reduction to 2D);
 *  - 3D body force g_a = -d_b (M_ab - delta_ab M_gg / 2), the kappa part of
 *    Eq. (pt), with the 3D gradient stencil;
 *  - the rest forcing term is F_0 = -sum_{i>=1} F_i (zeroth forcing moment);
 *  - the equilibrium and forcing use u = j / rho; the reported velocity of
 *    the forcing scheme is v = u + g / (2 rho) (end of Appendix A);
 *  - D3Q15 (section "Extension to 3D" states 19 velocities are necessary
 *    but gives no D3Q15 tables): weights with the second moments of
 *    Appendix A and an isotropic leading error where a choice remains, the
 *    corner weights of w^p, w^t, w^xx free (built in build_tables);
 *  - the binary fluid and its walls (not defined by the paper): see the
 *    binary section below.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int q;          /* 9 = D2Q9, 19 = D3Q19, 15 = D3Q15 (lattice comparison) */
    int scheme;     /* 0 = tuned equilibrium, 1 = momentum-conserving force */
    int nx, ny, nz; /* nz = 1 for D2Q9 */
    int lambda_on;  /* 1 = include the Galilean-invariance lambda terms */
    double a, b, T, kappa, tau;
    double B;       /* gradient stencil: off-axis coefficient */
    double D;       /* Laplacian stencil: off-axis coefficient */
    double F;       /* force stencil: off-axis coefficient */
    double wp_d, wt_d, wxx_d; /* equilibrium weights on the D2Q9 diagonals (D3Q15: corners) */
} orc_params;

/* ---- velocity sets ------------------------------------------------------ */

/* D2Q9 numbering of Section "Model": e1,2 = (+-1,0), e3,4 = (0,+-1),
 * e5,6 = (+-1,+-1), e7,8 = (-+1,+-1). */
static const int E2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}};

/* D3Q15 (for the lattice comparison; the paper gives no D3Q15 tables):
 * the faces e1..e6 as in D3Q19, then the eight cube corners in opposite
 * pairs. */
static const int E15[15][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

/* D3Q19 numbering of Section "Extension to 3D": faces e1..e6, then the
 * twelve square diagonals e7..e18 column by column as printed. */
static const int E3[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0},
    {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1},
    {1, 0, 1}, {-1, 0, 1}, {1, 0, -1}, {-1, 0, -1}};

typedef struct {
    int q, dim;
    int e[19][3];
    double w[19], wp[19], wt[19];
    double wm[6][19]; /* M-term weights: xx, yy, zz, xy, yz, zx */
    /* stencils as 3x3x3 arrays [slice][row][col]: slice 0,1,2 = z+1,z,z-1;
     * row 0,1,2 = y+1,y,y-1; col 0,1,2 = x-1,x,x+1 (the paper's layout) */
    double gx[3][3][3], gy[3][3][3], gz[3][3][3], lap[3][3][3];
    double fx[3][3][3], fy[3][3][3], fz[3][3][3];
} tables;

static void zero3(double s[3][3][3]) { memset(s, 0, sizeof(double) * 27); }

/* Build the gradient stencils of Eq. (xderiv) (2D) or Eq. (laplacian3d) (3D)
 * for the x direction with on-axis coefficient A and off-axis coefficient B,
 * then obtain y and z by rotating the lattice. */
static void build_gradient(int dim, double A, double B,
                           double sx[3][3][3], double sy[3][3][3], double sz[3][3][3])
{
    zero3(sx); zero3(sy); zero3(sz);
    if (dim == 2) {
        /* d_x = [ -B 0 B ; -A 0 A ; -B 0 B ] in the z = 0 slice */
        double m[3][3] = {{-B, 0, B}, {-A, 0, A}, {-B, 0, B}};
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                sx[1][r][c] = m[r][c];
                /* d_y: x and y interchanged, i.e. the stencil transposed so
                 * that the top row (y+1) carries +B +A +B */
                sy[1][r][c] = m[2 - c][2 - r];
            }
        return;
    }
    /* 3D: z = +-1 slices carry only (-B 0 B) on the middle row; the z = 0
     * slice is the full 2D pattern. */
    for (int s = 0; s < 3; s++)
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                int dx = c - 1, dy = 1 - r, dz = 1 - s;
                int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                /* x-derivative: odd in dx, touches faces (A) and edges (B) */
                if (dx != 0 && nnz == 1) sx[s][r][c] = A * dx;
                if (dx != 0 && nnz == 2) sx[s][r][c] = B * dx;
                if (dy != 0 && nnz == 1) sy[s][r][c] = A * dy;
                if (dy != 0 && nnz == 2) sy[s][r][c] = B * dy;
                if (dz != 0 && nnz == 1) sz[s][r][c] = A * dz;
                if (dz != 0 && nnz == 2) sz[s][r][c] = B * dz;
            }
}

static void build_laplacian(int dim, double C, double D, double s[3][3][3])
{
    zero3(s);
    if (dim == 2) {
        double m[3][3] = {{D, C, D}, {C, -4.0 * (C + D), C}, {D, C, D}};
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) s[1][r][c] = m[r][c];
        return;
    }
    double E = -6.0 * C - 12.0 * D;
    double top[3][3] = {{0, D, 0}, {D, C, D}, {0, D, 0}};
    double mid[3][3] = {{D, C, D}, {C, E, C}, {D, C, D}};
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            s[0][r][c] = top[r][c];
            s[1][r][c] = mid[r][c];
            s[2][r][c] = top[r][c];
        }
}

static void build_tables(const orc_params *p, tables *t)
{
    memset(t, 0, sizeof(*t));
    t->q = p->q;
    t->dim = (p->q == 9) ? 2 : 3;
    if (p->q == 15) {
        /* D3Q15, built as the paper builds D3Q19 (the paper gives no D3Q15
         * tables): the scalar terms on weights with sum w e_a e_b = delta_ab
         * (w: faces 1/3, corners 1/24, the isotropic fourth moment; w^p, w^t
         * with corner weights wp_d, wt_d, 1/24 for the same isotropy); the
         * kappa d_a d_b terms on weights meeting the second-moment conditions
         * of Appendix A (w^xx: x faces 1/4 - 4c, other faces -1/4 - 4c,
         * corners c, c free and passed as wxx_d; w^xy = e_x e_y / 8 on the
         * corners, the only velocities with e_x e_y != 0); the stencils on
         * faces and corners, B and D the corner coefficients (2A + 8B = 1,
         * C + 4D = 1 as for D3Q19; B = 1/24, D = 1/12 make their leading
         * error isotropic). */
        memcpy(t->e, E15, sizeof(E15));
        for (int i = 1; i <= 14; i++) {
            t->w[i] = (i <= 6) ? 1.0 / 3.0 : 1.0 / 24.0;
            /* w^p, w^t: corner weight wp_d / wt_d, faces from 2 w_f + 8 w_c = 1 */
            t->wp[i] = (i <= 6) ? 0.5 - 4.0 * p->wp_d : p->wp_d;
            t->wt[i] = (i <= 6) ? 0.5 - 4.0 * p->wt_d : p->wt_d;
        }
        const double c = p->wxx_d;
        for (int i = 1; i <= 14; i++) {
            const int *e = E15[i];
            for (int a = 0; a < 3; a++) {
                if (i <= 6) /* faces: along a, or not */
                    t->wm[a][i] = (e[a] != 0) ? 0.25 - 4.0 * c : -0.25 - 4.0 * c;
                else
                    t->wm[a][i] = c;
            }
            if (i > 6) {
                t->wm[3][i] = 0.125 * e[0] * e[1];
                t->wm[4][i] = 0.125 * e[1] * e[2];
                t->wm[5][i] = 0.125 * e[2] * e[0];
            }
        }
        const double A = (1.0 - 8.0 * p->B) / 2.0, C = 1.0 - 4.0 * p->D;
        zero3(t->gx); zero3(t->gy); zero3(t->gz); zero3(t->lap);
        for (int sl = 0; sl < 3; sl++)
            for (int r = 0; r < 3; r++)
                for (int cc = 0; cc < 3; cc++) {
                    int dx = cc - 1, dy = 1 - r, dz = 1 - sl;
                    int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nnz == 1) {
                        t->gx[sl][r][cc] = A * dx;
                        t->gy[sl][r][cc] = A * dy;
                        t->gz[sl][r][cc] = A * dz;
                        t->lap[sl][r][cc] = C;
                    } else if (nnz == 3) {
                        t->gx[sl][r][cc] = p->B * dx;
                        t->gy[sl][r][cc] = p->B * dy;
                        t->gz[sl][r][cc] = p->B * dz;
                        t->lap[sl][r][cc] = p->D;
                    }
                }
        t->lap[1][1][1] = -(6.0 * C + 8.0 * p->D);
        memcpy(t->fx, t->gx, sizeof(t->gx)); /* no forcing scheme on D3Q15 */
        memcpy(t->fy, t->gy, sizeof(t->gy));
        memcpy(t->fz, t->gz, sizeof(t->gz));
        return;
    }
    if (t->dim == 2) {
        memcpy(t->e, E2, sizeof(E2));
        for (int i = 1; i <= 8; i++) t->w[i] = (i <= 4) ? 1.0 / 3.0 : 1.0 / 12.0;
        /* constraints after Eq. (fi): 2 w_1-4 + 4 w_5-8 = 1 for p and t;
         * 2 w^xx_1-2 + 4 w^xx_5-8 = 1/2, 2 w^yy_1-2 + 4 w^yy_5-8 = -1/2,
         * x <-> y symmetry, w^xy_1-4 = 0, w^xy_5-6 = 1/4, w^xy_7-8 = -1/4 */
        for (int i = 1; i <= 8; i++) {
            int diag = (i >= 5);
            t->wp[i] = diag ? p->wp_d : 0.5 - 2.0 * p->wp_d;
            t->wt[i] = diag ? p->wt_d : 0.5 - 2.0 * p->wt_d;
            if (diag) {
                t->wm[0][i] = p->wxx_d;
                t->wm[1][i] = p->wxx_d;
                t->wm[3][i] = (i <= 6) ? 0.25 : -0.25;
            } else if (i <= 2) {
                t->wm[0][i] = 0.25 - 2.0 * p->wxx_d;
                t->wm[1][i] = -0.25 - 2.0 * p->wxx_d;
            } else {
                t->wm[0][i] = -0.25 - 2.0 * p->wxx_d;
                t->wm[1][i] = 0.25 - 2.0 * p->wxx_d;
            }
        }
        double A = (1.0 - 4.0 * p->B) / 2.0;  /* 2A + 4B = 1 */
        double C = 1.0 - 2.0 * p->D;          /* C + 2D = 1 */
        double Ef = (1.0 - 4.0 * p->F) / 2.0; /* force stencil, same form */
        build_gradient(2, A, p->B, t->gx, t->gy, t->gz);
        build_laplacian(2, C, p->D, t->lap);
        build_gradient(2, Ef, p->F, t->fx, t->fy, t->fz);
        return;
    }
    memcpy(t->e, E3, sizeof(E3));
    /* Eq. (3dres), with w_1-6 = 1/6 and the axial w^aa = 5/12 readings */
    for (int i = 1; i <= 18; i++) {
        t->w[i] = (i <= 6) ? 1.0 / 6.0 : 1.0 / 12.0;
        t->wp[i] = t->w[i];
        t->wt[i] = t->w[i];
    }
    double *wxx = t->wm[0], *wyy = t->wm[1], *wzz = t->wm[2];
    double *wxy = t->wm[3], *wyz = t->wm[4], *wzx = t->wm[5];
    wxx[1] = wxx[2] = 5.0 / 12.0;
    wyy[3] = wyy[4] = 5.0 / 12.0;
    wzz[5] = wzz[6] = 5.0 / 12.0;
    for (int i = 3; i <= 6; i++) wxx[i] = -1.0 / 3.0;
    wyy[1] = wyy[2] = wyy[5] = wyy[6] = -1.0 / 3.0;
    for (int i = 1; i <= 4; i++) wzz[i] = -1.0 / 3.0;
    for (int i = 7; i <= 10; i++) wxx[i] = -1.0 / 24.0;
    for (int i = 15; i <= 18; i++) wxx[i] = -1.0 / 24.0;
    for (int i = 7; i <= 14; i++) wyy[i] = -1.0 / 24.0;
    for (int i = 11; i <= 18; i++) wzz[i] = -1.0 / 24.0;
    for (int i = 11; i <= 14; i++) wxx[i] = 1.0 / 12.0;
    for (int i = 15; i <= 18; i++) wyy[i] = 1.0 / 12.0;
    for (int i = 7; i <= 10; i++) wzz[i] = 1.0 / 12.0;
    wxy[7] = wxy[10] = 0.25;
    wxy[8] = wxy[9] = -0.25;
    wyz[11] = wyz[14] = 0.25;
    wyz[12] = wyz[13] = -0.25;
    wzx[15] = wzx[18] = 0.25;
    wzx[16] = wzx[17] = -0.25;
    double A = (1.0 - 8.0 * p->B) / 2.0;  /* 2A + 8B = 1 */
    double C = 1.0 - 4.0 * p->D;          /* C + 4D = 1 */
    double Ef = (1.0 - 8.0 * p->F) / 2.0;
    build_gradient(3, A, p->B, t->gx, t->gy, t->gz);
    build_laplacian(3, C, p->D, t->lap);
    build_gradient(3, Ef, p->F, t->fx, t->fy, t->fz);
}

/* ---- lattice helpers ---------------------------------------------------- */

static inline int wrap(int v, int n) { v %= n; return v < 0 ? v + n : v; }

static inline long sidx(const orc_params *p, int x, int y, int z)
{
    return ((long)wrap(z, p->nz) * p->ny + wrap(y, p->ny)) * p->nx + wrap(x, p->nx);
}

static inline long nsites(const orc_params *p) { return (long)p->nx * p->ny * p->nz; }

/* apply a 3x3x3 stencil (paper layout) to a scalar field at (x,y,z) */
static double apply(const orc_params *p, const double s[3][3][3], const double *fld,
                    int x, int y, int z)
{
    double acc = 0.0;
    for (int sl = 0; sl < 3; sl++)
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                double k = s[sl][r][c];
                if (k == 0.0) continue;
                acc += k * fld[sidx(p, x + c - 1, y + 1 - r, z + 1 - sl)];
            }
    return acc;
}

/* ---- thermodynamics: Eq. (p0) and c_s^2 = dp0/drho ------------------------ */

double orc_p0(double a, double b, double T, double rho)
{
    return rho * T / (1.0 - b * rho) - a * rho * rho;
}

double orc_cs2(double a, double b, double T, double rho)
{
    double d = 1.0 - b * rho;
    return T / (d * d) - 2.0 * a * rho;
}

/* ---- per-site equilibrium and forcing ------------------------------------- */

/* Eq. (equilibrium) for i >= 1 and Eq. (feq0) for i = 0.
 * grad = discrete gradient of rho, lap = discrete Laplacian of rho.
 * with_m = 1 adds the kappa d_a rho d_b rho terms (equilibrium scheme). */
static void feq_site_t(const orc_params *p, const tables *t, double rho, const double j[3],
                       const double grad[3], double lap, int with_m, double *feq)
{
    int dim = t->dim;
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double p0 = orc_p0(p->a, p->b, p->T, rho);
    double nu = (p->tau - 0.5) / 3.0;                  /* Eq. (viscous) */
    double lam = p->lambda_on ? nu * (1.0 - 3.0 * orc_cs2(p->a, p->b, p->T, rho)) : 0.0;
    double udg = 0.0;
    for (int g = 0; g < dim; g++) udg += u[g] * grad[g];
    double X[3][3];
    for (int al = 0; al < 3; al++)
        for (int be = 0; be < 3; be++) {
            X[al][be] = rho * u[al] * u[be] +
                        lam * (u[al] * grad[be] + u[be] * grad[al] + (al == be ? udg : 0.0));
        }
    double M[6] = {p->kappa * grad[0] * grad[0], p->kappa * grad[1] * grad[1],
                   p->kappa * grad[2] * grad[2], p->kappa * grad[0] * grad[1],
                   p->kappa * grad[1] * grad[2], p->kappa * grad[2] * grad[0]};
    double sum = 0.0;
    for (int i = 1; i < t->q; i++) {
        const int *e = t->e[i];
        double ej = 0.0, ex = 0.0;
        for (int al = 0; al < dim; al++) ej += e[al] * j[al];
        for (int al = 0; al < dim; al++)
            for (int be = 0; be < dim; be++)
                ex += (e[al] * e[be] - (al == be ? 1.0 / 3.0 : 0.0)) * X[al][be];
        double v = t->w[i] * (ej + 1.5 * ex) + t->wp[i] * p0 - t->wt[i] * p->kappa * rho * lap;
        if (with_m)
            for (int m = 0; m < 6; m++) v += t->wm[m][i] * M[m];
        feq[i] = v;
        sum += v;
    }
    feq[0] = rho - sum;
}

/* Forcing term of Section "Using a forcing method" for i >= 1; the rest
 * term closes the zeroth moment. */
static void force_site_t(const tables *t, const double u[3], const double g[3], double *F)
{
    int dim = t->dim;
    double sum = 0.0;
    for (int i = 1; i < t->q; i++) {
        const int *e = t->e[i];
        double eg = 0.0, ex = 0.0;
        for (int al = 0; al < dim; al++) eg += e[al] * g[al];
        for (int al = 0; al < dim; al++)
            for (int be = 0; be < dim; be++)
                ex += (e[al] * e[be] - (al == be ? 1.0 / 3.0 : 0.0)) *
                      (u[al] * g[be] + u[be] * g[al]);
        F[i] = t->w[i] * (eg + 1.5 * ex);
        sum += F[i];
    }
    F[0] = -sum;
}

/* ---- fields ----------------------------------------------------------------- */

/* Eq. (rho): rho = sum_i f_i, j = sum_i f_i e_i */
static void moments(const orc_params *p, const tables *t, const double *f, double *rho,
                    double *j)
{
    long n = nsites(p);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double r = 0, jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < t->q; i++) {
            double v = f[i * n + s];
            r += v;
            jx += v * t->e[i][0];
            jy += v * t->e[i][1];
            jz += v * t->e[i][2];
        }
        rho[s] = r;
        j[s] = jx;
        j[n + s] = jy;
        j[2 * n + s] = jz;
    }
}

static void stencil_field(const orc_params *p, const double s[3][3][3], const double *in,
                          double *out)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++)
                out[sidx(p, x, y, z)] = apply(p, s, in, x, y, z);
}

/* gradient (3 components, z zero in 2D) and Laplacian of rho */
static void derivatives(const orc_params *p, const tables *t, const double *rho,
                        double *grad, double *lap)
{
    long n = nsites(p);
    stencil_field(p, t->gx, rho, grad);
    stencil_field(p, t->gy, rho, grad + n);
    if (t->dim == 3) stencil_field(p, t->gz, rho, grad + 2 * n);
    else memset(grad + 2 * n, 0, sizeof(double) * n);
    stencil_field(p, t->lap, rho, lap);
}

/* Body force of the forcing scheme: g_a = -d_b (M_ab - delta_ab M_gg / 2)
 * with M_ab = kappa d_a rho d_b rho, derivatives taken with the force
 * stencil.  In 2D this is g_x = -d_x((M_xx - M_yy)/2) - d_y M_xy as printed. */
static void body_force(const orc_params *p, const tables *t, const double *grad, double *g)
{
    long n = nsites(p);
    int dim = t->dim;
    double *T = (double *)malloc(sizeof(double) * n * 9); /* T_ab = M_ab - delta tr/2 */
    double *tmp = (double *)malloc(sizeof(double) * n);
    for (long s = 0; s < n; s++) {
        double d[3] = {grad[s], grad[n + s], grad[2 * n + s]};
        double tr = 0.0;
        for (int g2 = 0; g2 < dim; g2++) tr += p->kappa * d[g2] * d[g2];
        for (int al = 0; al < 3; al++)
            for (int be = 0; be < 3; be++)
                T[(al * 3 + be) * n + s] =
                    p->kappa * d[al] * d[be] - (al == be ? 0.5 * tr : 0.0);
    }
    const double(*fs[3])[3][3] = {t->fx, t->fy, t->fz};
    for (int al = 0; al < 3; al++) {
        for (long s = 0; s < n; s++) g[al * n + s] = 0.0;
        if (al >= dim) continue;
        for (int be = 0; be < dim; be++) {
            stencil_field(p, fs[be], T + (al * 3 + be) * n, tmp);
            for (long s = 0; s < n; s++) g[al * n + s] -= tmp[s];
        }
    }
    free(T);
    free(tmp);
}

/* ---- public entry points ------------------------------------------------------ */

int orc_num_sites(const orc_params *p) { return (int)nsites(p); }

/* Stencils as the 27 coefficients [slice][row][col] (for the Taylor tests). */
void orc_stencils(const orc_params *p, double *gx, double *gy, double *gz, double *lap,
                  double *fx, double *fy, double *fz)
{
    tables t;
    build_tables(p, &t);
    memcpy(gx, t.gx, sizeof(t.gx));
    memcpy(gy, t.gy, sizeof(t.gy));
    memcpy(gz, t.gz, sizeof(t.gz));
    memcpy(lap, t.lap, sizeof(t.lap));
    memcpy(fx, t.fx, sizeof(t.fx));
    memcpy(fy, t.fy, sizeof(t.fy));
    memcpy(fz, t.fz, sizeof(t.fz));
}

/* Velocity set and weight tables: e[q*3], w, wp, wt [q], wm[6*q]. */
void orc_tables(const orc_params *p, int *e, double *w, double *wp, double *wt, double *wm)
{
    tables t;
    build_tables(p, &t);
    for (int i = 0; i < t.q; i++) {
        for (int a = 0; a < 3; a++) e[i * 3 + a] = t.e[i][a];
        w[i] = t.w[i];
        wp[i] = t.wp[i];
        wt[i] = t.wt[i];
        for (int m = 0; m < 6; m++) wm[m * t.q + i] = t.wm[m][i];
    }
}

/* Equilibrium at one site for given moments and derivatives. */
void orc_feq_site(const orc_params *p, double rho, const double *j, const double *grad,
                  double lap, double *feq)
{
    tables t;
    build_tables(p, &t);
    feq_site_t(p, &t, rho, j, grad, lap, p->scheme == 0, feq);
}

/* Forcing term at one site for given u and g. */
void orc_force_site(const orc_params *p, const double *u, const double *g, double *F)
{
    tables t;
    build_tables(p, &t);
    force_site_t(&t, u, g, F);
}

/* Discrete gradient [3][n] and Laplacian [n] of a scalar field. */
void orc_derivatives(const orc_params *p, const double *rho, double *grad, double *lap)
{
    tables t;
    build_tables(p, &t);
    derivatives(p, &t, rho, grad, lap);
}

/* Body force [3][n] of the forcing scheme for a density field. */
void orc_body_force(const orc_params *p, const double *rho, double *g)
{
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double *grad = (double *)malloc(sizeof(double) * 3 * n);
    double *lap = (double *)malloc(sizeof(double) * n);
    derivatives(p, &t, rho, grad, lap);
    body_force(p, &t, grad, g);
    free(grad);
    free(lap);
}

/* Initial populations f_i = f_i^eq(rho0, rho0 u0) of the active scheme
 * (u0 may be NULL for a fluid at rest). */
void orc_init(const orc_params *p, const double *rho0, const double *u0, double *f)
{
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double *grad = (double *)malloc(sizeof(double) * 3 * n);
    double *lap = (double *)malloc(sizeof(double) * n);
    derivatives(p, &t, rho0, grad, lap);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double j[3] = {0, 0, 0};
        if (u0)
            for (int a = 0; a < 3; a++) j[a] = rho0[s] * u0[a * n + s];
        double g[3] = {grad[s], grad[n + s], grad[2 * n + s]};
        double feq[19];
        feq_site_t(p, &t, rho0[s], j, g, lap[s], p->scheme == 0, feq);
        for (int i = 0; i < t.q; i++) f[i * n + s] = feq[i];
    }
    free(grad);
    free(lap);
}

/* One time step, Eq. (latbolt): f_out(r + e_i) = f_i - (f_i - f_i^eq)/tau + F_i. */
static void step_t(const orc_params *p, const tables *t, const double *f, double *fout,
                   double *rho, double *j, double *grad, double *lap, double *g)
{
    long n = nsites(p);
    int force = (p->scheme == 1);
    moments(p, t, f, rho, j);
    derivatives(p, t, rho, grad, lap);
    if (force) body_force(p, t, grad, g);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                long s = sidx(p, x, y, z);
                double jj[3] = {j[s], j[n + s], j[2 * n + s]};
                double gr[3] = {grad[s], grad[n + s], grad[2 * n + s]};
                double feq[19], F[19];
                feq_site_t(p, t, rho[s], jj, gr, lap[s], !force, feq);
                if (force) {
                    double u[3] = {jj[0] / rho[s], jj[1] / rho[s], jj[2] / rho[s]};
                    double gg[3] = {g[s], g[n + s], g[2 * n + s]};
                    force_site_t(t, u, gg, F);
                } else {
                    for (int i = 0; i < t->q; i++) F[i] = 0.0;
                }
                for (int i = 0; i < t->q; i++) {
                    double fi = f[i * n + s];
                    double fstar = fi - (fi - feq[i]) / p->tau + F[i];
                    const int *e = t->e[i];
                    fout[i * n + sidx(p, x + e[0], y + e[1], z + e[2])] = fstar;
                }
            }
}

/* Advance f (in place) by nsteps. Returns 0, or -1 on a bad argument. */
int orc_run(const orc_params *p, double *f, int nsteps)
{
    if (!(p->q == 9 || p->q == 19 || p->q == 15) || nsteps < 0) return -1;
    if (p->q == 9 && p->nz != 1) return -1;
    if (p->q == 15 && p->scheme != 0) return -1; /* equilibrium scheme only */
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double *buf = (double *)malloc(sizeof(double) * n * t.q);
    double *rho = (double *)malloc(sizeof(double) * n);
    double *j = (double *)malloc(sizeof(double) * 3 * n);
    double *grad = (double *)malloc(sizeof(double) * 3 * n);
    double *lap = (double *)malloc(sizeof(double) * n);
    double *g = (double *)malloc(sizeof(double) * 3 * n);
    double *cur = f, *nxt = buf;
    for (int s = 0; s < nsteps; s++) {
        step_t(p, &t, cur, nxt, rho, j, grad, lap, g);
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (cur != f) memcpy(f, cur, sizeof(double) * n * t.q);
    free(buf); free(rho); free(j); free(grad); free(lap); free(g);
    return 0;
}

/* Observables: rho [n] and the velocity [3][n]: u = j/rho for the
 * equilibrium scheme, v = u + g/(2 rho) for the forcing scheme. */
void orc_observe(const orc_params *p, const double *f, double *rho, double *vel)
{
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double *j = (double *)malloc(sizeof(double) * 3 * n);
    moments(p, &t, f, rho, j);
    for (long s = 0; s < n; s++)
        for (int a = 0; a < 3; a++) vel[a * n + s] = j[a * n + s] / rho[s];
    if (p->scheme == 1) {
        double *g = (double *)malloc(sizeof(double) * 3 * n);
        double *grad = (double *)malloc(sizeof(double) * 3 * n);
        double *lap = (double *)malloc(sizeof(double) * n);
        derivatives(p, &t, rho, grad, lap);
        body_force(p, &t, grad, g);
        for (long s = 0; s < n; s++)
            for (int a = 0; a < 3; a++) vel[a * n + s] += g[a * n + s] / (2.0 * rho[s]);
        free(g); free(grad); free(lap);
    }
    free(j);
}

/* ---- site-local evaluation (for sampled checks on large lattices) ---------- */

static double rho_at(const orc_params *p, const tables *t, const double *f, int x, int y, int z)
{
    long n = nsites(p), s = sidx(p, x, y, z);
    double r = 0.0;
    for (int i = 0; i < t->q; i++) r += f[i * n + s];
    return r;
}

static double apply_rho(const orc_params *p, const tables *t, const double s[3][3][3],
                        const double *f, int x, int y, int z)
{
    double acc = 0.0;
    for (int sl = 0; sl < 3; sl++)
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                double k = s[sl][r][c];
                if (k == 0.0) continue;
                acc += k * rho_at(p, t, f, x + c - 1, y + 1 - r, z + 1 - sl);
            }
    return acc;
}

static void grad_at(const orc_params *p, const tables *t, const double *f, int x, int y,
                    int z, double d[3])
{
    d[0] = apply_rho(p, t, t->gx, f, x, y, z);
    d[1] = apply_rho(p, t, t->gy, f, x, y, z);
    d[2] = (t->dim == 3) ? apply_rho(p, t, t->gz, f, x, y, z) : 0.0;
}

/* Post-collision populations f*_i(r) (before streaming) at a list of sites
 * given as (x,y,z) triples; out is [nsite][q].  The post-stream state
 * after the step has f_i(r + e_i) = f*_i(r). */
void orc_collide_sites(const orc_params *p, const double *f, int nsite, const int *xyz,
                       double *out)
{
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    int force = (p->scheme == 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < nsite; k++) {
        int x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
        long s = sidx(p, x, y, z);
        double rho = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < t.q; i++) {
            double v = f[i * n + s];
            rho += v;
            for (int a = 0; a < 3; a++) j[a] += v * t.e[i][a];
        }
        double d[3];
        grad_at(p, &t, f, x, y, z, d);
        double lap = apply_rho(p, &t, t.lap, f, x, y, z);
        double feq[19], F[19] = {0};
        feq_site_t(p, &t, rho, j, d, lap, !force, feq);
        if (force) {
            /* g_a = -sum_b sum_stencil k * T_ab(neighbour) */
            const double(*fs[3])[3][3] = {t.fx, t.fy, t.fz};
            double g[3] = {0, 0, 0};
            for (int sl = 0; sl < 3; sl++)
                for (int r = 0; r < 3; r++)
                    for (int c = 0; c < 3; c++) {
                        int nbx = x + c - 1, nby = y + 1 - r, nbz = z + 1 - sl;
                        int any = 0;
                        for (int be = 0; be < t.dim; be++) any |= (fs[be][sl][r][c] != 0.0);
                        if (!any) continue;
                        double dn[3];
                        grad_at(p, &t, f, nbx, nby, nbz, dn);
                        double tr = 0.0;
                        for (int g2 = 0; g2 < t.dim; g2++) tr += p->kappa * dn[g2] * dn[g2];
                        for (int al = 0; al < t.dim; al++)
                            for (int be = 0; be < t.dim; be++) {
                                double Tab = p->kappa * dn[al] * dn[be] -
                                             (al == be ? 0.5 * tr : 0.0);
                                g[al] -= fs[be][sl][r][c] * Tab;
                            }
                    }
            double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
            force_site_t(&t, u, g, F);
        }
        for (int i = 0; i < t.q; i++) {
            double fi = f[i * n + s];
            out[(long)k * t.q + i] = fi - (fi - feq[i]) / p->tau + F[i];
        }
    }
}

/* Totals: mass = sum rho, momentum = sum_r sum_i f_i e_i (FP64, serial). */
void orc_totals(const orc_params *p, const double *f, double *mass, double *mom)
{
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double m = 0, mx = 0, my = 0, mz = 0;
    for (int i = 0; i < t.q; i++)
        for (long s = 0; s < n; s++) {
            double v = f[i * n + s];
            m += v;
            mx += v * t.e[i][0];
            my += v * t.e[i][1];
            mz += v * t.e[i][2];
        }
    *mass = m;
    mom[0] = mx;
    mom[1] = my;
    mom[2] = mz;
}

/* Thread count of the OpenMP loops (results do not depend on it: every
 * site is computed independently and the totals are serial). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ==== binary fluid (order parameter phi) ====================================
 *
 * The Introduction states that the analysis carries over to other multiphase
 * systems such as binary fluids, without giving that model.  This section
 * takes the symmetric binary free energy
 *     Psi = sum_r [ rho/3 + phi_a phi^2/2 + phi_b phi^4/4 + kappa |d phi|^2/2 ]
 * (an ideal-gas carrier rho with c_s^2 = 1/3, a double-well bulk term in the
 * order parameter phi, phi_a < 0 < phi_b) and applies the paper's tuned
 * equilibrium to it, with phi in the place of rho wherever rho is
 * differentiated:
 *   - f equilibrium: Eq. (equilibrium)/(feq0) with bulk pressure
 *     p0 = rho/3 + phi psi'(phi) - psi(phi) = rho/3 + phi_a phi^2/2
 *     + 3 phi_b phi^4/4, the w^t term -w^t_i kappa phi lap(phi), the w^ab
 *     terms kappa d_a phi d_b phi, and no lambda term (lambda = nu (1 - 3
 *     c_s^2) vanishes for c_s^2 = 1/3, Eq. (viscous));
 *   - a second distribution g_i relaxing (time tau_phi) to an equilibrium
 *     with moments sum g = phi, sum g e_a = phi u_a and sum g e_a e_b =
 *     gamma mu delta_ab + phi u_a u_b, mu = phi_a phi + phi_b phi^3 -
 *     kappa lap(phi); the gamma mu term is carried by the pressure weights
 *     w^p_i (the role p0 plays in the f equilibrium), the velocity terms by
 *     w_i, and g_0 closes the zeroth moment;
 *   - gradients and Laplacians with the same stencils as the liquid-gas
 *     model (Eqs. (xderiv), (laplace), (laplacian3d)).
 * The forcing scheme (base.scheme = 1) carries over the same way: the f
 * equilibrium drops the w^ab terms, and the body force g_a = -d_b (M_ab -
 * delta_ab M_gg / 2), M_ab = kappa d_a phi d_b phi, with the force stencil,
 * enters f through the forcing terms of section "Using a forcing method"
 * (F_i with u = j / rho, F_0 = -sum F_i); the order parameter is advected by
 * the fluid velocity of that scheme, v = u + g / (2 rho), which is also the
 * reported velocity.  Walls are not combined with the forcing scheme.
 */
typedef struct {
    orc_params base;     /* q, extent, kappa, tau, stencils, weights */
    double phi_a, phi_b; /* bulk free energy phi_a phi^2/2 + phi_b phi^4/4 */
    double gamma;        /* mobility coefficient of the mu term */
    double tau_phi;      /* relaxation time of g */
    int wall;            /* 1: walls at both ends of the last axis (see below) */
} orc_bin_params;

/* Walls (not defined by the paper; the forcing section only remarks that
 * boundaries are harder with forcing).  With wall = 1 the last axis (z for
 * D3Q19, y for D2Q9) is bounded by two walls halfway between lattice planes,
 * at -1/2 and n - 1/2: a population streaming into a wall returns to the
 * site it left with its velocity reversed (halfway bounce-back), and the
 * stencils read a site beyond a wall as its mirror image in the fluid (zero
 * normal derivative of phi: a neutral wall).  The other axes stay periodic. */
static long bin_sidx(const orc_bin_params *bp, int x, int y, int z)
{
    const orc_params *p = &bp->base;
    if (bp->wall) {
        if (p->q != 9) {
            if (z < 0) z = -1 - z;
            else if (z >= p->nz) z = 2 * p->nz - 1 - z;
        } else {
            if (y < 0) y = -1 - y;
            else if (y >= p->ny) y = 2 * p->ny - 1 - y;
        }
    }
    return sidx(p, x, y, z);
}

/* 1 if site (x, y, z) lies beyond a wall */
static int bin_beyond(const orc_bin_params *bp, int y, int z)
{
    const orc_params *p = &bp->base;
    if (!bp->wall) return 0;
    return p->q != 9 ? (z < 0 || z >= p->nz) : (y < 0 || y >= p->ny);
}

/* Site index with the bounded axis reflected to any depth: the fluid is
 * continued beyond each wall as its mirror image, so along that axis the
 * continuation has period 2n. */
static void bin_reflect(const orc_bin_params *bp, int *y, int *z)
{
    const orc_params *p = &bp->base;
    if (!bp->wall) return;
    int *w = (p->q != 9) ? z : y;
    const int n = (p->q != 9) ? p->nz : p->ny;
    const int m = ((*w % (2 * n)) + 2 * n) % (2 * n);
    *w = (m < n) ? m : 2 * n - 1 - m;
}

static long bin_ridx(const orc_bin_params *bp, int x, int y, int z)
{
    bin_reflect(bp, &y, &z);
    return sidx(&bp->base, x, y, z);
}

/* Body force of the forcing scheme between walls (the reading of the walls
 * above carried to the force): phi continued beyond a wall as its mirror
 * image, the gradient taken with the gradient stencil at every site the
 * force stencil reaches (ghost planes beyond a wall included),
 * T_ab = kappa d_a phi d_b phi - delta_ab kappa |d phi|^2 / 2 there, and
 * g_a = -sum_b (force stencil along b applied to T_ab). */
static void bin_body_force_walls(const orc_bin_params *bp, const tables *t, const double *phi,
                                 double *g)
{
    const orc_params *p = &bp->base;
    long n = nsites(p);
    const int dim = t->dim;
    const double(*gs[3])[3][3] = {t->gx, t->gy, t->gz};
    const double(*fs[3])[3][3] = {t->fx, t->fy, t->fz};
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                double acc[3] = {0.0, 0.0, 0.0};
                for (int sl = 0; sl < 3; sl++)
                    for (int r = 0; r < 3; r++)
                        for (int c = 0; c < 3; c++) {
                            int used = 0;
                            for (int be = 0; be < dim; be++) used |= fs[be][sl][r][c] != 0.0;
                            if (!used) continue;
                            const int nx_ = x + c - 1, ny_ = y + 1 - r, nz_ = z + 1 - sl;
                            double d[3] = {0.0, 0.0, 0.0};
                            for (int a = 0; a < dim; a++)
                                for (int sl2 = 0; sl2 < 3; sl2++)
                                    for (int r2 = 0; r2 < 3; r2++)
                                        for (int c2 = 0; c2 < 3; c2++) {
                                            const double k = gs[a][sl2][r2][c2];
                                            if (k == 0.0) continue;
                                            d[a] += k * phi[bin_ridx(bp, nx_ + c2 - 1, ny_ + 1 - r2,
                                                                     nz_ + 1 - sl2)];
                                        }
                            double tr = 0.0;
                            for (int a = 0; a < dim; a++) tr += p->kappa * d[a] * d[a];
                            for (int al = 0; al < dim; al++)
                                for (int be = 0; be < dim; be++) {
                                    const double k = fs[be][sl][r][c];
                                    if (k == 0.0) continue;
                                    acc[al] -= k * (p->kappa * d[al] * d[be] - (al == be ? 0.5 * tr : 0.0));
                                }
                        }
                const long s = sidx(p, x, y, z);
                for (int a = 0; a < 3; a++) g[a * n + s] = acc[a];
            }
}

static int opposite(const tables *t, int i)
{
    for (int j = 0; j < t->q; j++)
        if (t->e[j][0] == -t->e[i][0] && t->e[j][1] == -t->e[i][1] && t->e[j][2] == -t->e[i][2])
            return j;
    return -1;
}

/* gradient and Laplacian of phi with the stencils, walls mirrored */
static void bin_derivatives(const orc_bin_params *bp, const tables *t, const double *phi,
                            double *grad, double *lap)
{
    const orc_params *p = &bp->base;
    long n = nsites(p);
    const double(*st[4])[3][3] = {t->gx, t->gy, t->gz, t->lap};
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++) {
                long s = sidx(p, x, y, z);
                double v[4];
                for (int k = 0; k < 4; k++) {
                    double acc = 0.0;
                    for (int sl = 0; sl < 3; sl++)
                        for (int r = 0; r < 3; r++)
                            for (int c = 0; c < 3; c++) {
                                double kc = st[k][sl][r][c];
                                if (kc == 0.0) continue;
                                acc += kc * phi[bin_sidx(bp, x + c - 1, y + 1 - r, z + 1 - sl)];
                            }
                    v[k] = acc;
                }
                grad[s] = v[0];
                grad[n + s] = v[1];
                grad[2 * n + s] = (t->dim == 3) ? v[2] : 0.0;
                lap[s] = v[3];
            }
}

static double bin_p0(const orc_bin_params *bp, double rho, double phi)
{
    double p2 = phi * phi;
    return rho / 3.0 + 0.5 * bp->phi_a * p2 + 0.75 * bp->phi_b * p2 * p2;
}

static double bin_mu(const orc_bin_params *bp, double phi, double lap)
{
    return bp->phi_a * phi + bp->phi_b * phi * phi * phi - bp->base.kappa * lap;
}

/* f equilibrium of the binary fluid at one site: grad, lap of phi */
static void feq_bin_site_t(const orc_bin_params *bp, const tables *t, double rho,
                           const double j[3], double phi, const double grad[3], double lap,
                           double *feq)
{
    const double kappa = bp->base.kappa;
    int dim = t->dim;
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double p0 = bin_p0(bp, rho, phi);
    double M[6] = {kappa * grad[0] * grad[0], kappa * grad[1] * grad[1],
                   kappa * grad[2] * grad[2], kappa * grad[0] * grad[1],
                   kappa * grad[1] * grad[2], kappa * grad[2] * grad[0]};
    const int with_m = bp->base.scheme == 0; /* the forcing scheme moves M into the force */
    double sum = 0.0;
    for (int i = 1; i < t->q; i++) {
        const int *e = t->e[i];
        double ej = 0.0, ex = 0.0;
        for (int al = 0; al < dim; al++) ej += e[al] * j[al];
        for (int al = 0; al < dim; al++)
            for (int be = 0; be < dim; be++)
                ex += (e[al] * e[be] - (al == be ? 1.0 / 3.0 : 0.0)) * rho * u[al] * u[be];
        double v = t->w[i] * (ej + 1.5 * ex) + t->wp[i] * p0 - t->wt[i] * kappa * phi * lap;
        if (with_m)
            for (int m = 0; m < 6; m++) v += t->wm[m][i] * M[m];
        feq[i] = v;
        sum += v;
    }
    feq[0] = rho - sum;
}

/* g equilibrium at one site */
static void geq_bin_site_t(const orc_bin_params *bp, const tables *t, double phi,
                           const double u[3], double mu, double *geq)
{
    int dim = t->dim;
    double sum = 0.0;
    for (int i = 1; i < t->q; i++) {
        const int *e = t->e[i];
        double eu = 0.0, ex = 0.0;
        for (int al = 0; al < dim; al++) eu += e[al] * u[al];
        for (int al = 0; al < dim; al++)
            for (int be = 0; be < dim; be++)
                ex += (e[al] * e[be] - (al == be ? 1.0 / 3.0 : 0.0)) * u[al] * u[be];
        double v = t->wp[i] * bp->gamma * mu + t->w[i] * phi * (eu + 1.5 * ex);
        geq[i] = v;
        sum += v;
    }
    geq[0] = phi - sum;
}

static int bin_valid(const orc_bin_params *bp)
{
    const orc_params *p = &bp->base;
    if (!(p->q == 9 || p->q == 19 || p->q == 15)) return 0;
    if (p->q == 9 && p->nz != 1) return 0;
    if (p->scheme != 0 && p->scheme != 1) return 0;
    if (p->q == 15 && p->scheme != 0) return 0; /* D3Q15: tuned equilibrium only */
    return p->nx > 0 && p->ny > 0 && p->nz > 0;
}

/* phi = sum_i g_i */
static void order_parameter(const orc_params *p, const tables *t, const double *g, double *phi)
{
    long n = nsites(p);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double v = 0.0;
        for (int i = 0; i < t->q; i++) v += g[i * n + s];
        phi[s] = v;
    }
}

/* Initial populations: f = f^eq(rho0, rho0 u0, phi0), g = g^eq(phi0, u0, mu). */
int orc_bin_init(const orc_bin_params *bp, const double *rho0, const double *phi0,
                 const double *u0, double *f, double *g)
{
    if (!bin_valid(bp)) return -1;
    const orc_params *p = &bp->base;
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double *grad = (double *)malloc(sizeof(double) * 3 * n);
    double *lap = (double *)malloc(sizeof(double) * n);
    bin_derivatives(bp, &t, phi0, grad, lap);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double u[3] = {0, 0, 0}, j[3];
        if (u0)
            for (int a = 0; a < 3; a++) u[a] = u0[a * n + s];
        for (int a = 0; a < 3; a++) j[a] = rho0[s] * u[a];
        double d[3] = {grad[s], grad[n + s], grad[2 * n + s]};
        double fe[19], ge[19];
        feq_bin_site_t(bp, &t, rho0[s], j, phi0[s], d, lap[s], fe);
        geq_bin_site_t(bp, &t, phi0[s], u, bin_mu(bp, phi0[s], lap[s]), ge);
        for (int i = 0; i < t.q; i++) {
            f[i * n + s] = fe[i];
            g[i * n + s] = ge[i];
        }
    }
    free(grad);
    free(lap);
    return 0;
}

/* Advance (f, g) in place by nsteps: both distributions collide (BGK, tau
 * and tau_phi) and stream as in Eq. (latbolt). */
int orc_bin_run(const orc_bin_params *bp, double *f, double *g, int nsteps)
{
    if (!bin_valid(bp) || nsteps < 0) return -1;
    const orc_params *p = &bp->base;
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    int q = t.q;
    double *fb = (double *)malloc(sizeof(double) * n * q);
    double *gb = (double *)malloc(sizeof(double) * n * q);
    double *rho = (double *)malloc(sizeof(double) * n);
    double *j = (double *)malloc(sizeof(double) * 3 * n);
    double *phi = (double *)malloc(sizeof(double) * n);
    double *grad = (double *)malloc(sizeof(double) * 3 * n);
    double *lap = (double *)malloc(sizeof(double) * n);
    const int force = p->scheme == 1;
    double *gbody = (double *)malloc(sizeof(double) * 3 * n);
    double *fc = f, *gc = g, *fn = fb, *gn = gb;
    for (int step = 0; step < nsteps; step++) {
        moments(p, &t, fc, rho, j);
        order_parameter(p, &t, gc, phi);
        bin_derivatives(bp, &t, phi, grad, lap);
        if (force && bp->wall) bin_body_force_walls(bp, &t, phi, gbody);
        else if (force) body_force(p, &t, grad, gbody);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < p->nz; z++)
            for (int y = 0; y < p->ny; y++)
                for (int x = 0; x < p->nx; x++) {
                    long s = sidx(p, x, y, z);
                    double jj[3] = {j[s], j[n + s], j[2 * n + s]};
                    double u[3] = {jj[0] / rho[s], jj[1] / rho[s], jj[2] / rho[s]};
                    double d[3] = {grad[s], grad[n + s], grad[2 * n + s]};
                    double fe[19], ge[19], F[19] = {0};
                    double vg[3] = {u[0], u[1], u[2]}; /* advecting velocity of phi */
                    if (force) {
                        double gs[3] = {gbody[s], gbody[n + s], gbody[2 * n + s]};
                        force_site_t(&t, u, gs, F);
                        for (int a = 0; a < 3; a++) vg[a] += gs[a] / (2.0 * rho[s]);
                    }
                    feq_bin_site_t(bp, &t, rho[s], jj, phi[s], d, lap[s], fe);
                    geq_bin_site_t(bp, &t, phi[s], vg, bin_mu(bp, phi[s], lap[s]), ge);
                    for (int i = 0; i < q; i++) {
                        const int *e = t.e[i];
                        /* into a wall: back to this site, reversed */
                        long dst = bin_beyond(bp, y + e[1], z + e[2])
                                       ? (long)opposite(&t, i) * n + s
                                       : i * n + sidx(p, x + e[0], y + e[1], z + e[2]);
                        double fi = fc[i * n + s], gi = gc[i * n + s];
                        fn[dst] = fi - (fi - fe[i]) / p->tau + F[i];
                        gn[dst] = gi - (gi - ge[i]) / bp->tau_phi;
                    }
                }
        double *tf = fc, *tg = gc;
        fc = fn; gc = gn; fn = tf; gn = tg;
    }
    if (fc != f) {
        memcpy(f, fc, sizeof(double) * n * q);
        memcpy(g, gc, sizeof(double) * n * q);
    }
    free(fb); free(gb); free(rho); free(j); free(phi); free(grad); free(lap); free(gbody);
    return 0;
}

/* Observables: rho [n], phi [n], u = j / rho [3][n], mu [n] (any may be NULL). */
int orc_bin_observe(const orc_bin_params *bp, const double *f, const double *g, double *rho,
                    double *phi, double *vel, double *mu)
{
    if (!bin_valid(bp)) return -1;
    const orc_params *p = &bp->base;
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    double *r = (double *)malloc(sizeof(double) * n);
    double *j = (double *)malloc(sizeof(double) * 3 * n);
    double *ph = (double *)malloc(sizeof(double) * n);
    double *grad = (double *)malloc(sizeof(double) * 3 * n);
    double *lap = (double *)malloc(sizeof(double) * n);
    moments(p, &t, f, r, j);
    order_parameter(p, &t, g, ph);
    bin_derivatives(bp, &t, ph, grad, lap);
    double *gbody = (double *)calloc(3 * n, sizeof(double));
    if (p->scheme == 1 && bp->wall) bin_body_force_walls(bp, &t, ph, gbody);
    else if (p->scheme == 1) body_force(p, &t, grad, gbody);
    for (long s = 0; s < n; s++) {
        if (rho) rho[s] = r[s];
        if (phi) phi[s] = ph[s];
        if (vel) /* u, plus g / (2 rho) for the forcing scheme */
            for (int a = 0; a < 3; a++)
                vel[a * n + s] = j[a * n + s] / r[s] + gbody[a * n + s] / (2.0 * r[s]);
        if (mu) mu[s] = bin_mu(bp, ph[s], lap[s]);
    }
    free(gbody);
    free(r); free(j); free(ph); free(grad); free(lap);
    return 0;
}

/* Totals (serial, FP64): mass sum f, order parameter sum g, momentum sum f e. */
int orc_bin_totals(const orc_bin_params *bp, const double *f, const double *g, double *mass,
                   double *phi_total, double *mom)
{
    if (!bin_valid(bp)) return -1;
    orc_totals(&bp->base, f, mass, mom);
    const orc_params *p = &bp->base;
    long n = nsites(p);
    int q = p->q;
    double s = 0.0;
    for (int i = 0; i < q; i++)
        for (long k = 0; k < n; k++) s += g[i * n + k];
    *phi_total = s;
    return 0;
}

/* Equilibria at one site for given moments and derivatives of phi. */
void orc_bin_feq_site(const orc_bin_params *bp, double rho, const double *j, double phi,
                      const double *grad, double lap, double *feq)
{
    tables t;
    build_tables(&bp->base, &t);
    feq_bin_site_t(bp, &t, rho, j, phi, grad, lap, feq);
}

void orc_bin_geq_site(const orc_bin_params *bp, double phi, const double *u, double lap,
                      double *geq)
{
    tables t;
    build_tables(&bp->base, &t);
    geq_bin_site_t(bp, &t, phi, u, bin_mu(bp, phi, lap), geq);
}

/* Post-collision populations f*_i(r), g*_i(r) (before streaming) of the
 * binary fluid at a list of sites (x,y,z triples); fout, gout are
 * [nsite][q].  After the step, f_i(r + e_i) = f*_i(r) and likewise g. */
int orc_bin_collide_sites(const orc_bin_params *bp, const double *f, const double *g, int nsite,
                          const int *xyz, double *fout, double *gout)
{
    if (!bin_valid(bp)) return -1;
    const orc_params *p = &bp->base;
    tables t;
    build_tables(p, &t);
    long n = nsites(p);
    const double(*gs[3])[3][3] = {t.gx, t.gy, t.gz};
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < nsite; k++) {
        int x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
        long s = sidx(p, x, y, z);
        double rho = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < t.q; i++) {
            double v = f[i * n + s];
            rho += v;
            for (int a = 0; a < 3; a++) j[a] += v * t.e[i][a];
        }
        /* phi over the 3x3x3 neighbourhood, then the stencils */
        double d[3] = {0, 0, 0}, lap = 0.0;
        for (int sl = 0; sl < 3; sl++)
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) {
                    double kl = t.lap[sl][r][c];
                    int any = kl != 0.0;
                    for (int a = 0; a < t.dim; a++) any |= gs[a][sl][r][c] != 0.0;
                    if (!any) continue;
                    /* rho_at sums any distribution: here g, giving phi (a site
                     * beyond a wall: its mirror image) */
                    int yy = y + 1 - r, zz = z + 1 - sl;
                    bin_reflect(bp, &yy, &zz);
                    double ph = rho_at(p, &t, g, x + c - 1, yy, zz);
                    for (int a = 0; a < t.dim; a++) d[a] += gs[a][sl][r][c] * ph;
                    lap += kl * ph;
                }
        double phi = rho_at(p, &t, g, x, y, z);
        double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
        double fe[19], ge[19], F[19] = {0};
        double vg[3] = {u[0], u[1], u[2]};
        if (p->scheme == 1) {
            /* g_a = -sum_b sum_stencil k * T_ab(neighbour), the phi gradient at
             * each neighbour from the sums of g around it */
            const double(*fs[3])[3][3] = {t.fx, t.fy, t.fz};
            double gb[3] = {0, 0, 0};
            for (int sl = 0; sl < 3; sl++)
                for (int r = 0; r < 3; r++)
                    for (int c = 0; c < 3; c++) {
                        int any = 0;
                        for (int be = 0; be < t.dim; be++) any |= (fs[be][sl][r][c] != 0.0);
                        if (!any) continue;
                        double dn[3] = {0.0, 0.0, 0.0};
                        if (!bp->wall) {
                            grad_at(p, &t, g, x + c - 1, y + 1 - r, z + 1 - sl, dn);
                        } else { /* gradient of the mirrored phi, ghost sites included */
                            for (int a = 0; a < t.dim; a++)
                                for (int s2 = 0; s2 < 3; s2++)
                                    for (int r2 = 0; r2 < 3; r2++)
                                        for (int c2 = 0; c2 < 3; c2++) {
                                            const double k2 = gs[a][s2][r2][c2];
                                            if (k2 == 0.0) continue;
                                            int yy = y + 1 - r + 1 - r2, zz = z + 1 - sl + 1 - s2;
                                            bin_reflect(bp, &yy, &zz);
                                            dn[a] += k2 * rho_at(p, &t, g, x + c - 1 + c2 - 1, yy, zz);
                                        }
                        }
                        double tr = 0.0;
                        for (int g2 = 0; g2 < t.dim; g2++) tr += p->kappa * dn[g2] * dn[g2];
                        for (int al = 0; al < t.dim; al++)
                            for (int be = 0; be < t.dim; be++)
                                gb[al] -= fs[be][sl][r][c] *
                                          (p->kappa * dn[al] * dn[be] - (al == be ? 0.5 * tr : 0.0));
                    }
            force_site_t(&t, u, gb, F);
            for (int a = 0; a < 3; a++) vg[a] += gb[a] / (2.0 * rho);
        }
        feq_bin_site_t(bp, &t, rho, j, phi, d, lap, fe);
        geq_bin_site_t(bp, &t, phi, vg, bin_mu(bp, phi, lap), ge);
        for (int i = 0; i < t.q; i++) {
            double fi = f[i * n + s], gi = g[i * n + s];
            fout[(long)k * t.q + i] = fi - (fi - fe[i]) / p->tau + F[i];
            gout[(long)k * t.q + i] = gi - (gi - ge[i]) / bp->tau_phi;
        }
    }
    return 0;
}
