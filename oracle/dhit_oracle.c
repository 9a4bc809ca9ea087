/*
 * Plain FP64 CPU oracle for the LBE and DUGKS time steps of
 * Wang, Wang & Guo, "Comparison of the LBE and DUGKS methods for DNS of
 * decaying homogeneous isotropic turbulence" (arXiv 1601.03815).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library: every constant below
 * is written out here from the paper's definitions.
 *
 * Conventions
 *   - lattice units: dx = 1, c = 1, RT = c_s^2 = 1/3 (Sec. IV.A), rho0 given
 *     (the paper sets it to 1);
 *   - periodic n^3 box, cell (x,y,z), x fastest: idx = (z*n + y)*n + x;
 *   - a population field is stored as f[q*ncell + idx], q = 0..18;
 *   - D3Q19 order (the library ABI order): q0 rest; q1..q6 = +x,-x,+y,-y,
 *     +z,-z; q7..q10 = (1,1,0),(-1,1,0),(1,-1,0),(-1,-1,0); q11..q14 the same
 *     sign pattern in (x,z); q15..q18 the same pattern in (y,z).
 *
 * Everything is written for clarity, not speed: one loop per step of the
 * method, in the order the paper states them, with no fusion.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Sec. II.A, D3Q19 velocity set: xi_i in {0, +-e_a, +-e_a +- e_b} c. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

/* Sec. II.A, weights: W0 = 1/3, W1..6 = 1/18, W7..18 = 1/36. */
static double weight(int q)
{
    if (q == 0) return 1.0 / 3.0;
    if (q <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static const double RT = 1.0 / 3.0; /* Sec. IV.A: c_s^2 = RT = 1/3 */

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

static int64_t cell_index(int64_t x, int64_t y, int64_t z, int64_t n)
{
    return (wrap(z, n) * n + wrap(y, n)) * n + wrap(x, n);
}

/* ------------------------------------------------------------------ */
/* Lattice and equilibrium                                             */
/* ------------------------------------------------------------------ */

int oracle_version(void) { return 1; }

/* Export of the velocity set and the weights, so tests can check the
 * isotropy conditions the quadrature of Sec. II.A must satisfy. */
void oracle_lattice(int32_t *c /* [19][3] */, double *w /* [19] */)
{
    for (int q = 0; q < Q; q++) {
        c[3 * q + 0] = CX[q];
        c[3 * q + 1] = CY[q];
        c[3 * q + 2] = CZ[q];
        w[q] = weight(q);
    }
}

/* Discrete incompressible equilibrium, Sec. II.A (discrete equilibrium
 * equation): f_i^eq = W_i [drho + rho0 (xi.u/RT + (xi.u)^2/(2 RT^2)
 * - |u|^2/(2 RT))], with rho0 u = j. */
void oracle_feq(double drho, double jx, double jy, double jz, double rho0,
                double *feq /* [19] */)
{
    double ux = jx / rho0, uy = jy / rho0, uz = jz / rho0;
    double uu = ux * ux + uy * uy + uz * uz;
    for (int q = 0; q < Q; q++) {
        double xu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
        feq[q] = weight(q) * (drho + rho0 * (xu / RT + xu * xu / (2.0 * RT * RT) - uu / (2.0 * RT)));
    }
}

/* Moments of one cell: drho = sum f, rho0 u = j = sum xi f
 * (Sec. II.A macroscopic equations; Sec. II.B, density/momentum). */
static void cell_moments(const double *f, int64_t ncell, int64_t idx,
                         double *drho, double *jx, double *jy, double *jz)
{
    double r = 0, ax = 0, ay = 0, az = 0;
    for (int q = 0; q < Q; q++) {
        double v = f[q * ncell + idx];
        r += v;
        ax += CX[q] * v;
        ay += CY[q] * v;
        az += CZ[q] * v;
    }
    *drho = r; *jx = ax; *jy = ay; *jz = az;
}

/* ------------------------------------------------------------------ */
/* MRT transformation, Sec. II.B                                       */
/* ------------------------------------------------------------------ */

/* M[k][a] from the row formulas of Sec. II.B, a = population index. */
void oracle_mrt_matrix(double *M /* [19][19], row-major */)
{
    for (int a = 0; a < Q; a++) {
        double x = CX[a], y = CY[a], z = CZ[a];
        double s = x * x + y * y + z * z;   /* ||xi||^2 */
        double col[Q];
        col[0] = 1.0;                                   /* drho */
        col[1] = 19.0 * s - 30.0;                       /* e */
        col[2] = (21.0 * s * s - 53.0 * s + 24.0) / 2;  /* epsilon */
        col[3] = x;                                     /* j_x */
        col[4] = (5.0 * s - 9.0) * x;                   /* q_x */
        col[5] = y;                                     /* j_y */
        col[6] = (5.0 * s - 9.0) * y;                   /* q_y */
        col[7] = z;                                     /* j_z */
        col[8] = (5.0 * s - 9.0) * z;                   /* q_z */
        col[9] = 3.0 * x * x - s;                       /* 3 p_xx */
        col[10] = (3.0 * s - 5.0) * (3.0 * x * x - s);  /* 3 pi_xx */
        col[11] = y * y - z * z;                        /* p_ww */
        col[12] = (3.0 * s - 5.0) * (y * y - z * z);    /* pi_ww */
        col[13] = x * y;                                /* p_xy */
        col[14] = y * z;                                /* p_yz */
        col[15] = x * z;                                /* p_xz */
        col[16] = (y * y - z * z) * x;                  /* m_x */
        col[17] = (z * z - x * x) * y;                  /* m_y */
        col[18] = (x * x - y * y) * z;                  /* m_z */
        for (int k = 0; k < Q; k++) M[k * Q + a] = col[k];
    }
}

/* Inverse of M.  The rows of M are mutually orthogonal, so
 * M^-1 = M^T diag(1/|row_k|^2); the norms are computed from M itself. */
void oracle_mrt_inverse(const double *M, double *Minv /* [19][19] */)
{
    for (int k = 0; k < Q; k++) {
        double nrm = 0;
        for (int a = 0; a < Q; a++) nrm += M[k * Q + a] * M[k * Q + a];
        for (int a = 0; a < Q; a++) Minv[a * Q + k] = M[k * Q + a] / nrm;
    }
}

/* Equilibrium moments, Sec. II.B. */
void oracle_mrt_meq(double drho, double jx, double jy, double jz, double rho0,
                    double w_eps, double w_epsj, double w_xx, double *meq /* [19] */)
{
    double jj = jx * jx + jy * jy + jz * jz;
    meq[0] = drho;
    meq[1] = -11.0 * drho + 19.0 / rho0 * jj;
    meq[2] = w_eps * drho + w_epsj / rho0 * jj;
    meq[3] = jx;
    meq[4] = -2.0 / 3.0 * jx;
    meq[5] = jy;
    meq[6] = -2.0 / 3.0 * jy;
    meq[7] = jz;
    meq[8] = -2.0 / 3.0 * jz;
    /* the moment is 3 p_xx with p_xx^eq = [2 jx^2 - (jy^2 + jz^2)] / (3 rho0) */
    meq[9] = 3.0 * (2.0 * jx * jx - (jy * jy + jz * jz)) / (3.0 * rho0);
    meq[10] = w_xx * meq[9];                          /* 3 pi_xx = w_xx * 3 p_xx */
    meq[11] = (jy * jy - jz * jz) / rho0;             /* p_ww */
    meq[12] = w_xx * meq[11];                         /* pi_ww */
    meq[13] = jx * jy / rho0;
    meq[14] = jy * jz / rho0;
    meq[15] = jx * jz / rho0;
    meq[16] = 0.0;
    meq[17] = 0.0;
    meq[18] = 0.0;
}

/* ------------------------------------------------------------------ */
/* LBE: collision and streaming                                        */
/* ------------------------------------------------------------------ */

/* BGK collision in place: f <- f - (f - f^eq)/tau.  Single-relaxation
 * form of the lattice BGK equation built on the equilibrium of Sec. II.A. */
void oracle_collide_bgk(double *f, int32_t n, double tau, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ncell; i++) {
        double r, jx, jy, jz, feq[Q];
        cell_moments(f, ncell, i, &r, &jx, &jy, &jz);
        oracle_feq(r, jx, jy, jz, rho0, feq);
        for (int q = 0; q < Q; q++) {
            double v = f[q * ncell + i];
            f[q * ncell + i] = v - (v - feq[q]) / tau;
        }
    }
}

/* MRT collision in place, Sec. II.B evolution equation (right-hand side):
 * f <- f - M^-1 S (M f - m^eq). */
void oracle_collide_mrt(double *f, int32_t n, const double *s /* [19] */,
                        double w_eps, double w_epsj, double w_xx, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
    double M[Q * Q], Minv[Q * Q];
    oracle_mrt_matrix(M);
    oracle_mrt_inverse(M, Minv);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ncell; i++) {
        double fl[Q], m[Q], meq[Q], dm[Q];
        for (int q = 0; q < Q; q++) fl[q] = f[q * ncell + i];
        for (int k = 0; k < Q; k++) {
            m[k] = 0;
            for (int a = 0; a < Q; a++) m[k] += M[k * Q + a] * fl[a];
        }
        /* conserved moments: drho = m0, j = (m3, m5, m7) */
        oracle_mrt_meq(m[0], m[3], m[5], m[7], rho0, w_eps, w_epsj, w_xx, meq);
        for (int k = 0; k < Q; k++) dm[k] = s[k] * (m[k] - meq[k]);
        for (int a = 0; a < Q; a++) {
            double acc = 0;
            for (int k = 0; k < Q; k++) acc += Minv[a * Q + k] * dm[k];
            f[a * ncell + i] = fl[a] - acc;
        }
    }
}

/* Streaming with periodic wrap, left-hand side of the LBE evolution
 * equation: g_q(x + xi_q) = f_q(x). */
void oracle_stream(const double *f, double *g, int32_t n)
{
    int64_t ncell = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < n; z++)
        for (int64_t y = 0; y < n; y++)
            for (int64_t x = 0; x < n; x++) {
                int64_t src = cell_index(x, y, z, n);
                for (int q = 0; q < Q; q++) {
                    int64_t dst = cell_index(x + CX[q], y + CY[q], z + CZ[q], n);
                    g[q * ncell + dst] = f[q * ncell + src];
                }
            }
}

/* One LBE step in the paper's form (collide, then stream), from the
 * pre-collision state f(t_n) to the pre-collision state f(t_n + 1).
 * method 0 = BGK with tau; method 1 = MRT with s[19] and the w's. */
void oracle_lbe_step(const double *f, double *g, int32_t n, int32_t method,
                     double tau, const double *s, double w_eps, double w_epsj,
                     double w_xx, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
    double *tmp = (double *)malloc(sizeof(double) * Q * ncell);
    memcpy(tmp, f, sizeof(double) * Q * ncell);
    if (method == 0)
        oracle_collide_bgk(tmp, n, tau, rho0);
    else
        oracle_collide_mrt(tmp, n, s, w_eps, w_epsj, w_xx, rho0);
    oracle_stream(tmp, g, n);
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* DUGKS, Sec. II.A                                                    */
/* ------------------------------------------------------------------ */

/* Cell transforms (Sec. II.A, the two relations between f-tilde,
 * f-bar-plus and f-tilde-plus).  From the tracked f~ of every cell:
 *   moments of f~ -> f^eq -> fbp = (2tau-h)/(2tau+dt) f~ + 3h/(2tau+dt) f^eq
 *   ftp = 4/3 fbp - 1/3 f~,  with h = dt/2. */
void oracle_dugks_transform(const double *ft, double *fbp, double *ftp,
                            int32_t n, double tau, double dt, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
    double h = 0.5 * dt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ncell; i++) {
        double r, jx, jy, jz, feq[Q];
        cell_moments(ft, ncell, i, &r, &jx, &jy, &jz);
        oracle_feq(r, jx, jy, jz, rho0, feq);
        for (int q = 0; q < Q; q++) {
            double v = ft[q * ncell + i];
            double bp = (2.0 * tau - h) / (2.0 * tau + dt) * v + 3.0 * h / (2.0 * tau + dt) * feq[q];
            fbp[q * ncell + i] = bp;
            if (ftp) ftp[q * ncell + i] = 4.0 / 3.0 * bp - 1.0 / 3.0 * v;
        }
    }
}

/* Distribution f at the centre of the face between cell L = (x,y,z) and
 * R = L + e_d at t_n + h, for all 19 populations (Sec. II.A):
 *   1. linear interpolation of fbp and of its gradient sigma to the face
 *      (the one-dimensional interpolation formulas applied along the
 *      normal; tangential derivatives are the mean of the central
 *      differences of the two adjacent cells);
 *   2. fbar(x_b, t_n + h) = fbp(x_b) - h xi . sigma;
 *   3. face moments of fbar (all 19 populations) -> f^eq at the face;
 *   4. f = 2tau/(2tau+h) fbar + h/(2tau+h) f^eq. */
static void face_distribution(const double *fbp, int64_t n, int64_t x, int64_t y, int64_t z,
                              int d, double tau, double h, double rho0, double *fb /* [19] */)
{
    const double dx = 1.0;
    int64_t ncell = n * n * n;
    int64_t e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int64_t L = cell_index(x, y, z, n);
    int64_t R = cell_index(x + e[d][0], y + e[d][1], z + e[d][2], n);
    double fbar[Q];
    for (int q = 0; q < Q; q++) {
        double fl = fbp[q * ncell + L], fr = fbp[q * ncell + R];
        double sigma[3];
        for (int t = 0; t < 3; t++) {
            if (t == d) {
                sigma[t] = (fr - fl) / dx;
            } else {
                /* central difference at L and at R, then their mean */
                int64_t Lp = cell_index(x + e[t][0], y + e[t][1], z + e[t][2], n);
                int64_t Lm = cell_index(x - e[t][0], y - e[t][1], z - e[t][2], n);
                int64_t Rp = cell_index(x + e[d][0] + e[t][0], y + e[d][1] + e[t][1], z + e[d][2] + e[t][2], n);
                int64_t Rm = cell_index(x + e[d][0] - e[t][0], y + e[d][1] - e[t][1], z + e[d][2] - e[t][2], n);
                double gL = (fbp[q * ncell + Lp] - fbp[q * ncell + Lm]) / (2.0 * dx);
                double gR = (fbp[q * ncell + Rp] - fbp[q * ncell + Rm]) / (2.0 * dx);
                sigma[t] = 0.5 * (gL + gR);
            }
        }
        double at_face = fl + sigma[d] * (0.5 * dx);   /* x_{j+1/2} - x_j = dx/2 */
        double xs = CX[q] * sigma[0] + CY[q] * sigma[1] + CZ[q] * sigma[2];
        fbar[q] = at_face - h * xs;
    }
    double r = 0, jx = 0, jy = 0, jz = 0, feq[Q];
    for (int q = 0; q < Q; q++) {
        r += fbar[q];
        jx += CX[q] * fbar[q];
        jy += CY[q] * fbar[q];
        jz += CZ[q] * fbar[q];
    }
    oracle_feq(r, jx, jy, jz, rho0, feq);
    for (int q = 0; q < Q; q++)
        fb[q] = 2.0 * tau / (2.0 * tau + h) * fbar[q] + h / (2.0 * tau + h) * feq[q];
}

/* Updated f~ of one cell (Sec. II.A finite-volume update with the
 * midpoint rule for the face flux): f~^{n+1} = f~+ - dt/|V| F, where
 * F = sum over the six faces of (xi . n) f_face * area; |V| = dx^3,
 * area = dx^2. */
static void dugks_cell_update(const double *fbp, const double *ftp, int64_t n,
                              int64_t x, int64_t y, int64_t z, double tau,
                              double dt, double rho0, double *out /* [19] */)
{
    const double dx = 1.0, area = dx * dx, vol = dx * dx * dx;
    double h = 0.5 * dt;
    int64_t ncell = n * n * n;
    int64_t idx = cell_index(x, y, z, n);
    double flux[Q];
    for (int q = 0; q < Q; q++) flux[q] = 0;
    for (int d = 0; d < 3; d++) {
        double fplus[Q], fminus[Q];
        /* face at +d/2: between this cell and its +d neighbour; outward normal +e_d */
        face_distribution(fbp, n, x, y, z, d, tau, h, rho0, fplus);
        /* face at -d/2: between the -d neighbour and this cell; outward normal -e_d */
        face_distribution(fbp, n, x - (d == 0), y - (d == 1), z - (d == 2), d, tau, h, rho0, fminus);
        for (int q = 0; q < Q; q++) {
            double xn = (d == 0) ? CX[q] : (d == 1) ? CY[q] : CZ[q];
            flux[q] += xn * fplus[q] * area - xn * fminus[q] * area;
        }
    }
    for (int q = 0; q < Q; q++) out[q] = ftp[q * ncell + idx] - dt / vol * flux[q];
}

/* One DUGKS step on the whole box: f~(t_n) -> f~(t_n + dt). */
void oracle_dugks_step(const double *ft, double *out, int32_t n, double tau,
                       double dt, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
    double *fbp = (double *)malloc(sizeof(double) * Q * ncell);
    double *ftp = (double *)malloc(sizeof(double) * Q * ncell);
    oracle_dugks_transform(ft, fbp, ftp, n, tau, dt, rho0);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < n; z++)
        for (int64_t y = 0; y < n; y++)
            for (int64_t x = 0; x < n; x++) {
                double o[Q];
                dugks_cell_update(fbp, ftp, n, x, y, z, tau, dt, rho0, o);
                int64_t idx = cell_index(x, y, z, n);
                for (int q = 0; q < Q; q++) out[q * ncell + idx] = o[q];
            }
    free(fbp);
    free(ftp);
}

/* ------------------------------------------------------------------ */
/* DUGKS on a stretched (non-uniform, tensor-product) periodic mesh     */
/* ------------------------------------------------------------------ */

/* Geometry of one axis from its n cell widths w[0..n-1] (periodic):
 * the centre of cell i sits at c_i = w_0/2 + sum_{k<i} (w_k + w_{k+1})/2 and
 * its faces at c_i -/+ w_i/2.  Distances between centres wrap around. */
static double centre_gap(const double *w, int64_t n, int64_t i) /* c_{i+1} - c_i */
{
    return 0.5 * (w[wrap(i, n)] + w[wrap(i + 1, n)]);
}

/* Distribution f at the centre of the face between cell L = (x,y,z) and
 * R = L + e_d at t_n + h on the mesh with widths W[3][n] (Sec. II.A, the
 * one-dimensional interpolation formulas applied along the face normal):
 *   sigma_d = (fbp_R - fbp_L) / (c_R - c_L),
 *   fbp(x_b) = fbp_L + sigma_d (x_b - c_L), x_b - c_L = w_L / 2;
 * tangential derivatives: the central difference of each adjacent cell,
 * (fbp(+e_t) - fbp(-e_t)) / (c_{k+1} - c_{k-1}), interpolated linearly to
 * the face with the same weight as the value (on a uniform mesh: their
 * mean); then fbar = fbp(x_b) - h xi . sigma, face moments, f^eq, and
 * f = 2tau/(2tau+h) fbar + h/(2tau+h) f^eq. */
static void face_distribution_mesh(const double *fbp, int64_t n, const double *W, int64_t x, int64_t y,
                                   int64_t z, int d, double tau, double h, double rho0, double *fb)
{
    int64_t ncell = n * n * n;
    int64_t e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int64_t pos[3] = {x, y, z};
    int64_t L = cell_index(x, y, z, n);
    int64_t R = cell_index(x + e[d][0], y + e[d][1], z + e[d][2], n);
    const double *wd = W + d * n;
    double gap = centre_gap(wd, n, pos[d]);   /* c_R - c_L */
    double half = 0.5 * wd[wrap(pos[d], n)];   /* x_b - c_L */
    double lam = half / gap;                    /* interpolation weight of R */
    double fbar[Q];
    for (int q = 0; q < Q; q++) {
        double fl = fbp[q * ncell + L], fr = fbp[q * ncell + R];
        double sigma[3];
        for (int t = 0; t < 3; t++) {
            if (t == d) {
                sigma[t] = (fr - fl) / gap;
            } else {
                const double *wt = W + t * n;
                int64_t k = pos[t];
                double span = centre_gap(wt, n, k - 1) + centre_gap(wt, n, k); /* c_{k+1} - c_{k-1} */
                int64_t Lp = cell_index(x + e[t][0], y + e[t][1], z + e[t][2], n);
                int64_t Lm = cell_index(x - e[t][0], y - e[t][1], z - e[t][2], n);
                int64_t Rp = cell_index(x + e[d][0] + e[t][0], y + e[d][1] + e[t][1], z + e[d][2] + e[t][2], n);
                int64_t Rm = cell_index(x + e[d][0] - e[t][0], y + e[d][1] - e[t][1], z + e[d][2] - e[t][2], n);
                double gL = (fbp[q * ncell + Lp] - fbp[q * ncell + Lm]) / span;
                double gR = (fbp[q * ncell + Rp] - fbp[q * ncell + Rm]) / span;
                sigma[t] = gL + lam * (gR - gL);
            }
        }
        double at_face = fl + sigma[d] * half;
        double xs = CX[q] * sigma[0] + CY[q] * sigma[1] + CZ[q] * sigma[2];
        fbar[q] = at_face - h * xs;
    }
    double r = 0, jx = 0, jy = 0, jz = 0, feq[Q];
    for (int q = 0; q < Q; q++) {
        r += fbar[q];
        jx += CX[q] * fbar[q];
        jy += CY[q] * fbar[q];
        jz += CZ[q] * fbar[q];
    }
    oracle_feq(r, jx, jy, jz, rho0, feq);
    for (int q = 0; q < Q; q++)
        fb[q] = 2.0 * tau / (2.0 * tau + h) * fbar[q] + h / (2.0 * tau + h) * feq[q];
}

/* One DUGKS step on the stretched mesh W[3][n] (cell widths per axis):
 * f~^{n+1} = f~+ - dt/|V| sum over the six faces of (xi . n) f_face A,
 * |V| = w_x w_y w_z of the cell, A the face's area (product of the two
 * tangential widths). */
void oracle_dugks_step_mesh(const double *ft, double *out, int32_t n, const double *W /* [3][n] */,
                            double tau, double dt, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
    double h = 0.5 * dt;
    double *fbp = (double *)malloc(sizeof(double) * Q * ncell);
    double *ftp = (double *)malloc(sizeof(double) * Q * ncell);
    oracle_dugks_transform(ft, fbp, ftp, n, tau, dt, rho0);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < n; z++)
        for (int64_t y = 0; y < n; y++)
            for (int64_t x = 0; x < n; x++) {
                double w[3] = {W[x], W[n + y], W[2 * n + z]};
                double vol = w[0] * w[1] * w[2];
                double flux[Q];
                for (int q = 0; q < Q; q++) flux[q] = 0;
                for (int d = 0; d < 3; d++) {
                    double area = vol / w[d];
                    double fplus[Q], fminus[Q];
                    face_distribution_mesh(fbp, n, W, x, y, z, d, tau, h, rho0, fplus);
                    face_distribution_mesh(fbp, n, W, x - (d == 0), y - (d == 1), z - (d == 2), d, tau, h, rho0,
                                           fminus);
                    for (int q = 0; q < Q; q++) {
                        double xn = (d == 0) ? CX[q] : (d == 1) ? CY[q] : CZ[q];
                        flux[q] += xn * (fplus[q] - fminus[q]) * area;
                    }
                }
                int64_t idx = cell_index(x, y, z, n);
                for (int q = 0; q < Q; q++) out[q * ncell + idx] = ftp[q * ncell + idx] - dt / vol * flux[q];
            }
    free(fbp);
    free(ftp);
}

/* DUGKS update of selected cells only, for checks at sizes where a whole
 * oracle step is too slow.  The update of a cell reads f-bar-plus only at
 * offsets inside the 3x3x3 cube around it (every face uses L, R and their
 * tangential neighbours), and the cell transform is local, so the cube of
 * f~ around the cell is copied into a 3^3 box and the centre cell of that
 * box is updated; its stencil never reaches the box's wrapped border. */
void oracle_dugks_cells(const double *ft, int32_t n, double tau, double dt, double rho0,
                        const int64_t *cells, int64_t ncells, double *out /* [ncells][19] */)
{
    int64_t ncell = (int64_t)n * n * n;
    const int64_t m = 3, mc = 27;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ncells; s++) {
        int64_t c = cells[s];
        int64_t x = c % n, y = (c / n) % n, z = c / ((int64_t)n * n);
        double lft[Q * 27], lbp[Q * 27], ltp[Q * 27];
        for (int64_t k = 0; k < m; k++)
            for (int64_t j = 0; j < m; j++)
                for (int64_t i = 0; i < m; i++) {
                    int64_t g = cell_index(x + i - 1, y + j - 1, z + k - 1, n);
                    int64_t l = (k * m + j) * m + i;
                    for (int q = 0; q < Q; q++) lft[q * mc + l] = ft[q * ncell + g];
                }
        oracle_dugks_transform(lft, lbp, ltp, (int32_t)m, tau, dt, rho0);
        dugks_cell_update(lbp, ltp, m, 1, 1, 1, tau, dt, rho0, out + s * Q);
    }
}

/* Pull-form LBE of selected cells: the pre-collision populations that
 * stream into each listed cell from the post-collision field fpost
 * (g_q(x) = fpost_q(x - xi_q)), then collided.  Used to check a step of
 * a solver that stores post-collision populations. */
void oracle_lbe_pull_cells(const double *fpost, int32_t n, int32_t method, double tau,
                           const double *s, double w_eps, double w_epsj, double w_xx,
                           double rho0, const int64_t *cells, int64_t ncells,
                           double *out /* [ncells][19] */)
{
    int64_t ncell = (int64_t)n * n * n;
    for (int64_t t = 0; t < ncells; t++) {
        int64_t c = cells[t];
        int64_t x = c % n, y = (c / n) % n, z = c / ((int64_t)n * n);
        double g[Q];
        for (int q = 0; q < Q; q++)
            g[q] = fpost[q * ncell + cell_index(x - CX[q], y - CY[q], z - CZ[q], n)];
        /* collide a one-cell box (n = 1 is a valid single-cell field) */
        if (method == 0)
            oracle_collide_bgk(g, 1, tau, rho0);
        else
            oracle_collide_mrt(g, 1, s, w_eps, w_epsj, w_xx, rho0);
        for (int q = 0; q < Q; q++) out[t * Q + q] = g[q];
    }
}

/* ------------------------------------------------------------------ */
/* Moments and global sums                                             */
/* ------------------------------------------------------------------ */

/* Per-cell drho, j (optional) and the global sums
 * (sum drho, sum jx, sum jy, sum jz, 1/2 sum |u|^2), u = j/rho0.
 * The sums run serially in cell order. */
void oracle_moments(const double *f, int32_t n, double rho0, double *drho /* [ncell] or NULL */,
                    double *j /* [3][ncell] or NULL */, double *sums /* [5] or NULL */)
{
    int64_t ncell = (int64_t)n * n * n;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    for (int64_t i = 0; i < ncell; i++) {
        double r, jx, jy, jz;
        cell_moments(f, ncell, i, &r, &jx, &jy, &jz);
        if (drho) drho[i] = r;
        if (j) {
            j[i] = jx;
            j[ncell + i] = jy;
            j[2 * ncell + i] = jz;
        }
        s0 += r; s1 += jx; s2 += jy; s3 += jz;
        s4 += 0.5 * (jx * jx + jy * jy + jz * jz) / (rho0 * rho0);
    }
    if (sums) {
        sums[0] = s0; sums[1] = s1; sums[2] = s2; sums[3] = s3; sums[4] = s4;
    }
}

/* Equilibrium populations of a velocity field (and optional drho field):
 * f_q = f_q^eq(drho, rho0 u).  Sec. II.A equilibrium; the starting state
 * for BGK-LBE and for DUGKS (where f~ = f when Omega = 0). */
void oracle_init_equilibrium(double *f, int32_t n, const double *u /* [3][ncell] */,
                             const double *drho /* [ncell] or NULL */, double rho0)
{
    int64_t ncell = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ncell; i++) {
        double feq[Q];
        double r = drho ? drho[i] : 0.0;
        oracle_feq(r, rho0 * u[i], rho0 * u[ncell + i], rho0 * u[2 * ncell + i], rho0, feq);
        for (int q = 0; q < Q; q++) f[q * ncell + i] = feq[q];
    }
}

/* MRT equilibrium populations f = M^-1 m^eq(drho, rho0 u): the fixed point
 * of the MRT collision for the given conserved moments. */
void oracle_init_mrt_equilibrium(double *f, int32_t n, const double *u, const double *drho,
                                 double rho0, double w_eps, double w_epsj, double w_xx)
{
    int64_t ncell = (int64_t)n * n * n;
    double M[Q * Q], Minv[Q * Q];
    oracle_mrt_matrix(M);
    oracle_mrt_inverse(M, Minv);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ncell; i++) {
        double meq[Q];
        double r = drho ? drho[i] : 0.0;
        oracle_mrt_meq(r, rho0 * u[i], rho0 * u[ncell + i], rho0 * u[2 * ncell + i], rho0,
                       w_eps, w_epsj, w_xx, meq);
        for (int a = 0; a < Q; a++) {
            double acc = 0;
            for (int k = 0; k < Q; k++) acc += Minv[a * Q + k] * meq[k];
            f[a * ncell + i] = acc;
        }
    }
}
