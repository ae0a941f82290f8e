/*
 * FP64 CPU oracle for one time step of the phase-field discrete unified
 * gas-kinetic scheme (DUGKS) of Yang, Zhong & Zhuo, "A phase-field model for
 * large-density-ratio two-phase flows based on discrete unified gas-kinetic
 * scheme" (arXiv:1810.07802).
 *
 * TEST INFRASTRUCTURE. This library is the correctness reference for the HIP
 * path. Only the test suite, the package smoke check and the CPU-baseline leg
 * of the benchmark may load it. It shares no source with the HIP path, and the
 * product never calls it.
 *
 * It is written for a reader checking it against the paper: plain loops in the
 * paper's order, every array a full field, no fusion and no blocking. All
 * arithmetic is IEEE double; build with -ffp-contract=off.
 *
 * Paper references:
 *   Sec. II.A  free energy, chemical potential, conservative Allen-Cahn,
 *              incompressible NS, density interpolation  (Eqs. 1-10)
 *   Sec. II.B  the two kinetic models: D2Q9 set and weights (Eq. 14),
 *              truncated f equilibrium (Eq. 15), f source (Eq. 16),
 *              g equilibrium (Eq. 17-18), g source (Eq. 19), the DUGKS
 *              integral (Eq. 21-22), tilde auxiliaries (Eq. 23), cell update
 *              (Eq. 24), half-step characteristic (Eq. 25-27), face original
 *              distribution (Eq. 28), bar-plus and tilde-plus from tilde
 *              (Eq. 29-30), cell macros (Eq. 31-33), relaxation times and
 *              viscosity interpolation (Eq. 34-36), stencils and CFL time step
 *              (text before Eq. 37 and Eq. 37).
 *
 * Readings of points the paper leaves open (every one is also listed in the
 * design notes of the repository):
 *   R1  RT = 1/3, so that sqrt(3RT) = 1 and xi_q = e_q; delta_l = 1, so
 *       dt = CFL and h = dt/2 (Eq. 37 with the grid spacing of Sec. III).
 *   R2  kappa = 3 sigma W / (2 Delta^2), beta = 12 sigma / (W Delta^4) with
 *       Delta = phi_H - phi_L; they reduce to Eq. 3 when Delta = 1 and keep the
 *       interface width W and tension sigma for any Delta.
 *   R4  Central reconstruction at a face: the value is the mean of the two
 *       cells, the normal slope their difference, the tangential slope the
 *       mean of the two cells' central differences.
 *   R5  Gradient-type inputs at a face (grad phi, mu_phi, the time derivative
 *       D) are the mean of the two adjacent cells at t_n; algebraic functions
 *       of phi (rho, theta, tau_g, gravity) are re-evaluated from the face phi.
 *   R6  Face macros use the cell formulas of Eq. 32-33 with dt/2 -> h/2.
 *   R7  n = grad phi / sqrt(|grad phi|^2 + eps^2), eps = eps_n |phi_H - phi_L|
 *       (eps_n = 1e-6 by default): the unit normal where |grad phi| >> eps,
 *       zero for a uniform field, and continuous where the gradient vanishes
 *       (at saddle points of phi, and in the flat far field, where the plain
 *       unit vector follows the rounding of a vanishing gradient). eps_n = 0
 *       gives the plain unit normal of Sec. II.A, with n = 0 only where the
 *       gradient is exactly zero.
 *   R8  grad phi: isotropic D2Q9-weighted difference (six non-zero points per
 *       component).
 *   R9  Laplacian: isotropic nine-point stencil.
 *   R10 d_t(phi u) = [(phi u)^n - (phi u)^(n-1)] / dt, zero on the first step.
 *   R11 Initial tilde distributions: psi^eq - (dt/2) S with D = 0.
 *   R12 Viscosity: a uniform nu gives tau_g = nu / RT everywhere; unequal
 *       mu_H, mu_L are interpolated in s reciprocally (1/mu = s/mu_H +
 *       (1-s)/mu_L) or linearly, and tau_g = mu / (rho RT).
 *   R13 s = (phi - phi_L)/Delta is clamped to [0,1] inside rho, mu and tau_g
 *       only; grad rho = rho' grad phi is not clamped.
 *   R15 No-slip walls on the faces y = 0 and y = ny (see wall_face()).
 *   R16 Gravity either rho g or (rho - (rho_H + rho_L)/2) g, plus a constant
 *       body-force density.
 *   R22 Pressure follows Eq. 33 exactly as printed.
 *   Upwind mode (recon = ORC_RECON_UPWIND; the paper names an upwind, limited
 *       reconstruction as the cure for the dissipation of the central one):
 *       a population crossing a face is traced back from the face by h xi
 *       into its upwind cell and evaluated there with the cell's van Leer
 *       limited slopes, VL(a, b) = 2ab / (a + b) if ab > 0, else 0, of the
 *       backward and forward differences (one-sided next to a wall); a
 *       population along the face takes the mean of the two cells and the
 *       mean of their limited tangential slopes.
 */
#include "dugks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocity set in the paper's order and its weights (Eq. 14). */
static const int EX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int EY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
static const double WQ[9] = {4.0 / 9.0,  1.0 / 9.0, 1.0 / 36.0,
                             1.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0};
/* Opposite direction: for q >= 1, ((q + 3) mod 8) + 1. */
static int opp(int q) { return q == 0 ? 0 : ((q + 3) % 8) + 1; }

static const double RT = 1.0 / 3.0;

struct orc_sim {
    int nx, ny, coupled;
    orc_params P;
    /* derived constants */
    double dt, h, Dphi, phibar, kappa, beta, tau_f, drho;
    long step;
    /* state: tilde distributions and the history (phi u)^(n-1) */
    double *f, *g, *hist;
    /* Pass A: cell macros at t_n */
    double *phi, *gpx, *gpy, *lap, *mu, *rho, *ux, *uy, *p, *Dx, *Dy, *theta,
        *taug;
    /* Pass B: bar-plus and tilde-plus at cell centres */
    double *fbp, *gbp, *ftp, *gtp;
    /* Pass C: original distributions at faces.  x-face arrays hold the face
       east of cell (i,j); y-face arrays have ny+1 rows, row jj is the face at
       y = jj (between cell rows jj-1 and jj). */
    double *fxf, *gxf, *fyf, *gyf;
    /* stretched mesh (R27): cell widths and centres, NULL on the unit mesh;
       dl is the smallest width */
    double *mdx, *mdy, *mxc, *myc, dl;
};

/* ---------------------------------------------------------------- helpers */

static int wrapi(int i, int n) { return ((i % n) + n) % n; }

static void derive(orc_sim *s) {
    const orc_params *P = &s->P;
    /* Eq. 37 with sqrt(3RT) = 1 and delta_l the smallest cell width */
    s->dt = s->mdx ? P->cfl * s->dl : P->cfl;
    s->h = 0.5 * s->dt;
    s->Dphi = P->phi_H - P->phi_L;
    s->phibar = 0.5 * (P->phi_H + P->phi_L);
    s->kappa = 1.5 * P->sigma * P->W / (s->Dphi * s->Dphi);          /* R2 */
    s->beta = 12.0 * P->sigma / (P->W * pow(s->Dphi, 4.0));          /* R2 */
    s->tau_f = P->M / RT;                                            /* Eq. 34 */
    s->drho = (P->rho_H - P->rho_L) / s->Dphi;                       /* Eq. 10 */
}

static double s_clamped(const orc_sim *s, double phi) {
    double v = (phi - s->P.phi_L) / s->Dphi;
    if (v < 0.0) v = 0.0;
    if (v > 1.0) v = 1.0;
    return v;
}

/* Eq. 10, with the clamp of R13. */
static double rho_of(const orc_sim *s, double phi) {
    return s->P.rho_L + (s->P.rho_H - s->P.rho_L) * s_clamped(s, phi);
}

/* Eq. 6 */
static double theta_of(const orc_sim *s, double phi) {
    return -4.0 * (phi - s->P.phi_H) * (phi - s->P.phi_L) / (s->P.W * s->Dphi);
}

/* Eq. 34-36: tau_g = mu / (rho RT) with mu interpolated in s (R12, R13), or a
   uniform kinematic viscosity nu = tau_g RT. */
static double taug_of(const orc_sim *s, double phi, double rho) {
    const orc_params *P = &s->P;
    double sv = s_clamped(s, phi);
    double mu;
    if (P->visc_mode == ORC_VISC_UNIFORM_NU) return P->nu / RT;
    if (P->visc_mode == ORC_VISC_RECIPROCAL)
        mu = 1.0 / (sv / P->mu_H + (1.0 - sv) / P->mu_L);
    else
        mu = sv * P->mu_H + (1.0 - sv) * P->mu_L;
    return mu / (rho * RT);
}

/* Body force G (R16). */
static void gravity(const orc_sim *s, double rho, double *Gx, double *Gy) {
    const orc_params *P = &s->P;
    double r = (P->gravity_form == ORC_GRAV_BUOYANCY)
                   ? rho - 0.5 * (P->rho_H + P->rho_L)
                   : rho;
    *Gx = P->Gx + r * P->gx;
    *Gy = P->Gy + r * P->gy;
}

/* Chemical potential, Eq. 4. */
static double chem_pot(const orc_sim *s, double phi, double lap) {
    return 4.0 * s->beta * (phi - s->P.phi_H) * (phi - s->P.phi_L) *
               (phi - s->phibar) -
           s->kappa * lap;
}

/* Prescribed velocity fields of the interface-capturing tests (Sec. III,
   Eqs. 40-43). */
static void presc_vel(const orc_params *P, double x, double y, double t,
                      double *u, double *v) {
    const double pi = 3.14159265358979323846;
    double U0 = P->U0, L0 = P->L0;
    switch (P->vel_kind) {
    case ORC_VEL_UNIFORM: /* Eq. 40 */
        *u = U0;
        *v = U0;
        break;
    case ORC_VEL_ROTATION: /* Eq. 41 */
        *u = -U0 * pi / L0 * (y - 0.5 * L0);
        *v = U0 * pi / L0 * (x - 0.5 * L0);
        break;
    case ORC_VEL_SHEAR: { /* Eq. 42, reversed at half the period */
        double sg = (t < 0.5 * P->T_period) ? 1.0 : -1.0;
        *u = sg * U0 * pi * sin(pi * x / L0) * cos(pi * y / L0);
        *v = -sg * U0 * pi * cos(pi * x / L0) * sin(pi * y / L0);
        break;
    }
    case ORC_VEL_DEFORM: { /* Eq. 43 */
        double c = cos(pi * t / P->T_period);
        *u = -U0 * sin(4.0 * pi * x / L0) * sin(4.0 * pi * y / L0) * c;
        *v = -U0 * cos(4.0 * pi * x / L0) * cos(4.0 * pi * y / L0) * c;
        break;
    }
    default:
        *u = 0.0;
        *v = 0.0;
    }
}

/* ------------------------------------------- equilibria and source terms */

/* Truncated equilibrium of f, Eq. 15 (c_s^2 = RT). */
void orc_feq(double phi, double ux, double uy, double *out) {
    for (int q = 0; q < 9; ++q)
        out[q] = WQ[q] * phi * (1.0 + (EX[q] * ux + EY[q] * uy) / RT);
}

/* Source of f, Eq. 16: w theta xi.n + w xi.D / RT with D = d_t(phi u). */
void orc_sf(double theta, double nx, double ny, double Dx, double Dy,
            double *out) {
    for (int q = 0; q < 9; ++q)
        out[q] = WQ[q] * theta * (EX[q] * nx + EY[q] * ny) +
                 WQ[q] * (EX[q] * Dx + EY[q] * Dy) / RT;
}

/* Gamma_q(u) of Eq. 18. */
static double gamma_q(int q, double ux, double uy) {
    double eu = EX[q] * ux + EY[q] * uy;
    double uu = ux * ux + uy * uy;
    return WQ[q] * (1.0 + eu / RT + eu * eu / (2.0 * RT * RT) - uu / (2.0 * RT));
}

/* Equilibrium of g, Eq. 17. */
void orc_geq(double p, double rho, double ux, double uy, double *out) {
    for (int q = 0; q < 9; ++q) {
        double pre = (q == 0) ? (WQ[q] - 1.0) : WQ[q];
        out[q] = p / RT * pre + rho * (gamma_q(q, ux, uy) - gamma_q(q, 0.0, 0.0));
    }
}

/* Source of g, Eq. 19, with grad(rho RT) = RT grad rho (RT constant). */
void orc_sg(double ux, double uy, double drx, double dry, double Fx,
            double Fy, double *out) {
    for (int q = 0; q < 9; ++q) {
        double cx = EX[q] - ux, cy = EY[q] - uy;
        double gu = gamma_q(q, ux, uy), g0 = gamma_q(q, 0.0, 0.0);
        double ax = (gu - g0) * RT * drx + Fx * gu;
        double ay = (gu - g0) * RT * dry + Fy * gu;
        out[q] = (cx * ax + cy * ay) / RT;
    }
}

/* Eq. 29-30: bar-plus and tilde-plus from the tilde distribution. */
void orc_bar_plus(double tau, double dt, const double *tl, const double *eq,
                  const double *S, double *bp, double *tp) {
    double h = 0.5 * dt, den = 2.0 * tau + dt;
    for (int q = 0; q < 9; ++q) {
        bp[q] = (2.0 * tau - h) / den * tl[q] + 3.0 * h / den * eq[q] +
                3.0 * tau * h / den * S[q];
        tp[q] = 4.0 / 3.0 * bp[q] - 1.0 / 3.0 * tl[q];
    }
}

/* Eq. 28: original distribution at a face from its bar value. */
void orc_face_df(double tau, double h, const double *bar, const double *eq,
                 const double *S, double *out) {
    double den = 2.0 * tau + h;
    for (int q = 0; q < 9; ++q)
        out[q] = 2.0 * tau / den * bar[q] + h / den * eq[q] +
                 tau * h / den * S[q];
}

/* ------------------------------------------------------------- stencils */

/* phi at (i, j) with x periodic and y periodic or mirrored at walls. */
static double phi_at(const orc_sim *s, const double *phi, int i, int j) {
    int nx = s->nx, ny = s->ny;
    i = wrapi(i, nx);
    if (s->P.walls_y) {
        if (j < 0) j = -1 - j;            /* mirror about y = 0   */
        if (j >= ny) j = 2 * ny - 1 - j;  /* mirror about y = ny  */
    } else {
        j = wrapi(j, ny);
    }
    return phi[(size_t)j * nx + i];
}

/* Stretched mesh (R27): widths of cells i and j (x periodic; with walls a
   mirrored ghost row has the width of the row it mirrors), distances between
   neighbouring centres (m: to the previous cell, p: to the next), and the
   first and second derivatives at 0 of the parabola through (-hm, am),
   (0, ac), (hp, ap). */
static double wx(const orc_sim *s, int i) { return s->mdx[wrapi(i, s->nx)]; }
static double wy(const orc_sim *s, int j) {
    int ny = s->ny;
    if (s->P.walls_y) {
        if (j < 0) j = -1 - j;
        if (j >= ny) j = 2 * ny - 1 - j;
    } else {
        j = wrapi(j, ny);
    }
    return s->mdy[j];
}
static double hxm(const orc_sim *s, int i) { return 0.5 * (wx(s, i - 1) + wx(s, i)); }
static double hxp(const orc_sim *s, int i) { return 0.5 * (wx(s, i) + wx(s, i + 1)); }
static double hym(const orc_sim *s, int j) { return 0.5 * (wy(s, j - 1) + wy(s, j)); }
static double hyp(const orc_sim *s, int j) { return 0.5 * (wy(s, j) + wy(s, j + 1)); }
static double d1(double am, double ac, double ap, double hm, double hp) {
    return (hm * hm * (ap - ac) + hp * hp * (ac - am)) / (hm * hp * (hm + hp));
}
static double d2(double am, double ac, double ap, double hm, double hp) {
    return 2.0 * ((ap - ac) / hp - (ac - am) / hm) / (hm + hp);
}
/* cell centres and face positions */
static double xcen(const orc_sim *s, int i) { return s->mdx ? s->mxc[i] : i + 0.5; }
static double ycen(const orc_sim *s, int j) { return s->mdx ? s->myc[j] : j + 0.5; }

/* R27: the stencils of R8 and R9 on a stretched mesh. Each is a weighted sum
   of one-dimensional derivatives on the rows (columns) j-1, j, j+1 (i-1, i,
   i+1), the neighbouring rows weighted by the opposite distance so that the
   sum is centred on the cell: exact on quadratics, and R8, R9 on the unit
   mesh. */
static void stencils_mesh(const orc_sim *s, const double *phi, int i, int j,
                          double *gx, double *gy, double *lap) {
    double xm = hxm(s, i), xp = hxp(s, i), ym = hym(s, j), yp = hyp(s, j);
    double dxr[3], dxxr[3], dyc[3], dyyc[3];
    for (int k = -1; k <= 1; ++k) {
        double m = phi_at(s, phi, i - 1, j + k), c = phi_at(s, phi, i, j + k),
               pp = phi_at(s, phi, i + 1, j + k);
        dxr[k + 1] = d1(m, c, pp, xm, xp);
        dxxr[k + 1] = d2(m, c, pp, xm, xp);
        m = phi_at(s, phi, i + k, j - 1);
        c = phi_at(s, phi, i + k, j);
        pp = phi_at(s, phi, i + k, j + 1);
        dyc[k + 1] = d1(m, c, pp, ym, yp);
        dyyc[k + 1] = d2(m, c, pp, ym, yp);
    }
    *gx = (2.0 / 3.0) * dxr[1] + (1.0 / 3.0) * (ym * dxr[2] + yp * dxr[0]) / (ym + yp);
    *gy = (2.0 / 3.0) * dyc[1] + (1.0 / 3.0) * (xm * dyc[2] + xp * dyc[0]) / (xm + xp);
    *lap = (5.0 / 6.0) * (dxxr[1] + dyyc[1]) +
           (1.0 / 6.0) * (ym * dxxr[2] + yp * dxxr[0]) / (ym + yp) +
           (1.0 / 6.0) * (xm * dyyc[2] + xp * dyyc[0]) / (xm + xp);
}

/* R8: isotropic gradient, d/dx = (1/RT) sum_q w_q e_qx phi(x + e_q), written
   as differences of opposite neighbours so that a uniform field gives an
   exactly zero gradient (and n = 0 by R7):
     d/dx = [4 (phi_E - phi_W) + (phi_NE - phi_NW) + (phi_SE - phi_SW)] / 12.
   R9: isotropic Laplacian, (2/RT) sum_q w_q [phi(x + e_q) - phi(x)]. */
static void stencils(const orc_sim *s, const double *phi, int i, int j,
                     double *gx, double *gy, double *lap) {
    if (s->mdx) {
        stencils_mesh(s, phi, i, j, gx, gy, lap);
        return;
    }
    double c = phi_at(s, phi, i, j);
    double E = phi_at(s, phi, i + 1, j), Wv = phi_at(s, phi, i - 1, j);
    double N = phi_at(s, phi, i, j + 1), S = phi_at(s, phi, i, j - 1);
    double NE = phi_at(s, phi, i + 1, j + 1), NW = phi_at(s, phi, i - 1, j + 1);
    double SE = phi_at(s, phi, i + 1, j - 1), SW = phi_at(s, phi, i - 1, j - 1);
    *gx = (4.0 * (E - Wv) + (NE - NW) + (SE - SW)) / 12.0;
    *gy = (4.0 * (N - S) + (NE - SE) + (NW - SW)) / 12.0;
    double sl = 0.0;
    for (int q = 1; q < 9; ++q)
        sl += WQ[q] * (phi_at(s, phi, i + EX[q], j + EY[q]) - c);
    *lap = 2.0 * sl / RT;
}

void orc_stencils(int nx, int ny, int walls_y, const double *dx, const double *dy,
                  const double *phi, double *gx, double *gy, double *lap) {
    orc_sim tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.nx = nx;
    tmp.ny = ny;
    tmp.P.walls_y = walls_y;
    if ((dx || dy) && orc_set_mesh(&tmp, dx, dy) != 0) return;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            stencils(&tmp, phi, i, j, &gx[c], &gy[c], &lap[c]);
        }
    orc_set_mesh(&tmp, NULL, NULL);
}

/* R7: regularised unit normal (eps in gradient units: over the smallest
   cell width on a stretched mesh, R27). */
static void unit(const orc_sim *s, double gx, double gy, double *nx, double *ny) {
    double eps = s->P.eps_n * fabs(s->Dphi) / (s->mdx ? s->dl : 1.0);
    double m = sqrt(gx * gx + gy * gy + eps * eps);
    *nx = m > 0.0 ? gx / m : 0.0;
    *ny = m > 0.0 ? gy / m : 0.0;
}

/* ------------------------------------------------------ allocation / API */

static double *alloc(size_t n) { return (double *)calloc(n, sizeof(double)); }

orc_sim *orc_create(int nx, int ny, int coupled, const orc_params *P) {
    if (nx < 3 || ny < 3) return NULL;
    if (P->walls_y && (ny < 4 || !coupled)) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    size_t n = (size_t)nx * ny, ny1 = (size_t)nx * (ny + 1);
    s->nx = nx;
    s->ny = ny;
    s->coupled = coupled;
    s->P = *P;
    derive(s);
    s->f = alloc(9 * n);
    s->g = alloc(9 * n);
    s->hist = alloc(2 * n);
    s->phi = alloc(n); s->gpx = alloc(n); s->gpy = alloc(n); s->lap = alloc(n);
    s->mu = alloc(n); s->rho = alloc(n); s->ux = alloc(n); s->uy = alloc(n);
    s->p = alloc(n); s->Dx = alloc(n); s->Dy = alloc(n); s->theta = alloc(n);
    s->taug = alloc(n);
    s->fbp = alloc(9 * n); s->gbp = alloc(9 * n);
    s->ftp = alloc(9 * n); s->gtp = alloc(9 * n);
    s->fxf = alloc(9 * n); s->gxf = alloc(9 * n);
    s->fyf = alloc(9 * ny1); s->gyf = alloc(9 * ny1);
    return s;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    double *arr[] = {s->f,   s->g,   s->hist, s->phi, s->gpx, s->gpy, s->lap,
                     s->mu,  s->rho, s->ux,   s->uy,  s->p,   s->Dx,  s->Dy,
                     s->theta, s->taug, s->fbp, s->gbp, s->ftp, s->gtp,
                     s->fxf, s->gxf, s->fyf, s->gyf};
    for (size_t k = 0; k < sizeof arr / sizeof arr[0]; ++k) free(arr[k]);
    orc_set_mesh(s, NULL, NULL);
    free(s);
}

/* R27: widths dx[nx], dy[ny] of a stretched tensor-product mesh (either may
   be NULL: unit widths on that axis). Both NULL: back to the unit mesh and
   its own code. The time step becomes cfl times the smallest width. */
int orc_set_mesh(orc_sim *s, const double *dx, const double *dy) {
    free(s->mdx); free(s->mdy); free(s->mxc); free(s->myc);
    s->mdx = s->mdy = s->mxc = s->myc = NULL;
    s->dl = 1.0;
    if (dx || dy) {
        int nx = s->nx, ny = s->ny;
        s->mdx = alloc(nx); s->mdy = alloc(ny); s->mxc = alloc(nx); s->myc = alloc(ny);
        double x = 0.0, y = 0.0, lo = HUGE_VAL;
        for (int i = 0; i < nx; ++i) {
            double w = dx ? dx[i] : 1.0;
            if (!(w > 0.0)) return orc_set_mesh(s, NULL, NULL), -1;
            s->mdx[i] = w;
            s->mxc[i] = x + 0.5 * w;
            x += w;
            if (w < lo) lo = w;
        }
        for (int j = 0; j < ny; ++j) {
            double w = dy ? dy[j] : 1.0;
            if (!(w > 0.0)) return orc_set_mesh(s, NULL, NULL), -1;
            s->mdy[j] = w;
            s->myc[j] = y + 0.5 * w;
            y += w;
            if (w < lo) lo = w;
        }
        s->dl = lo;
    }
    derive(s);
    return 0;
}

int orc_set_params(orc_sim *s, const orc_params *P) {
    s->P = *P;
    derive(s);
    return 0;
}

double orc_time(const orc_sim *s) { return s->step * s->dt; }
long orc_step_count(const orc_sim *s) { return s->step; }

void orc_derived(const orc_sim *s, double *out) {
    out[0] = s->dt; out[1] = s->h; out[2] = s->kappa; out[3] = s->beta;
    out[4] = s->tau_f; out[5] = s->drho;
}

/* ---------------------------------------------------------- Pass A: cells */

/* Cell macros at t_n from the tilde distributions (Eq. 31-33, 34, 4, 10). */
static void pass_a(orc_sim *s) {
    int nx = s->nx, ny = s->ny;
    size_t n = (size_t)nx * ny;
    double t = orc_time(s);

#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)n; ++c) {
        double acc = 0.0;
        for (int q = 0; q < 9; ++q) acc += s->f[q * n + c]; /* Eq. 31 */
        s->phi[c] = acc;
    }

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double phi = s->phi[c], gx, gy, lap;
            stencils(s, s->phi, i, j, &gx, &gy, &lap);
            s->gpx[c] = gx;
            s->gpy[c] = gy;
            s->lap[c] = lap;
            s->mu[c] = chem_pot(s, phi, lap);
            s->theta[c] = theta_of(s, phi);
            double rho = rho_of(s, phi);
            s->rho[c] = rho;
            double ux, uy, p = 0.0;
            if (s->coupled) {
                double Gx, Gy;
                gravity(s, rho, &Gx, &Gy);
                double Fx = s->mu[c] * gx + Gx, Fy = s->mu[c] * gy + Gy;
                double mx = 0.0, my = 0.0, m0 = 0.0;
                for (int q = 0; q < 9; ++q) {
                    double gq = s->g[q * n + c];
                    mx += EX[q] * gq;
                    my += EY[q] * gq;
                    if (q != 0) m0 += gq;
                }
                ux = (mx + 0.5 * s->dt * Fx) / rho; /* Eq. 32 */
                uy = (my + 0.5 * s->dt * Fy) / rho;
                double drx = s->drho * gx, dry = s->drho * gy;
                double G0 = gamma_q(0, ux, uy) - gamma_q(0, 0.0, 0.0);
                p = RT / (1.0 - WQ[0]) *
                    (m0 + 0.5 * s->dt * (ux * drx + uy * dry) + rho * G0); /* Eq. 33 */
                s->taug[c] = taug_of(s, phi, rho);
            } else {
                presc_vel(&s->P, xcen(s, i), ycen(s, j), t, &ux, &uy);
                s->taug[c] = 0.0;
            }
            s->ux[c] = ux;
            s->uy[c] = uy;
            s->p[c] = p;
            /* R10: first-order difference of phi u in time */
            s->Dx[c] = (phi * ux - s->hist[c]) / s->dt;
            s->Dy[c] = (phi * uy - s->hist[n + c]) / s->dt;
        }
}

/* ------------------------------------------------ Pass B: bar-plus fields */

static void cell_eq_src(const orc_sim *s, size_t c, double *feq, double *sf,
                        double *geq, double *sg) {
    double nxv, nyv;
    unit(s, s->gpx[c], s->gpy[c], &nxv, &nyv);
    orc_feq(s->phi[c], s->ux[c], s->uy[c], feq);
    orc_sf(s->theta[c], nxv, nyv, s->Dx[c], s->Dy[c], sf);
    if (s->coupled) {
        double Gx, Gy;
        gravity(s, s->rho[c], &Gx, &Gy);
        double Fx = s->mu[c] * s->gpx[c] + Gx, Fy = s->mu[c] * s->gpy[c] + Gy;
        orc_geq(s->p[c], s->rho[c], s->ux[c], s->uy[c], geq);
        orc_sg(s->ux[c], s->uy[c], s->drho * s->gpx[c], s->drho * s->gpy[c],
               Fx, Fy, sg);
    }
}

static void pass_b(orc_sim *s) {
    size_t n = (size_t)s->nx * s->ny;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)n; ++c) {
        double feq[9], sf[9], geq[9], sg[9], tl[9], bp[9], tp[9];
        cell_eq_src(s, c, feq, sf, geq, sg);
        for (int q = 0; q < 9; ++q) tl[q] = s->f[q * n + c];
        orc_bar_plus(s->tau_f, s->dt, tl, feq, sf, bp, tp);
        for (int q = 0; q < 9; ++q) {
            s->fbp[q * n + c] = bp[q];
            s->ftp[q * n + c] = tp[q];
        }
        if (s->coupled) {
            for (int q = 0; q < 9; ++q) tl[q] = s->g[q * n + c];
            orc_bar_plus(s->taug[c], s->dt, tl, geq, sg, bp, tp);
            for (int q = 0; q < 9; ++q) {
                s->gbp[q * n + c] = bp[q];
                s->gtp[q * n + c] = tp[q];
            }
        }
    }
}

/* ------------------------------------------------------- Pass C: faces */

/* R27 on a stretched mesh: slopes are derivatives (differences over the
   centre distances), and the face value and tangential slope interpolate
   linearly to the face position instead of taking the plain mean. */
static double slope_y_mesh(const orc_sim *s, const double *a, int i, int j) {
    int nx = s->nx, ny = s->ny;
    if (s->P.walls_y) {
        if (j == 0) return (a[(size_t)1 * nx + i] - a[i]) / hyp(s, 0);
        if (j == ny - 1)
            return (a[(size_t)(ny - 1) * nx + i] - a[(size_t)(ny - 2) * nx + i]) / hym(s, ny - 1);
    }
    return d1(a[(size_t)wrapi(j - 1, ny) * nx + i], a[(size_t)j * nx + i],
              a[(size_t)wrapi(j + 1, ny) * nx + i], hym(s, j), hyp(s, j));
}
static double slope_x_mesh(const orc_sim *s, const double *a, int i, int j) {
    int nx = s->nx;
    return d1(a[(size_t)j * nx + wrapi(i - 1, nx)], a[(size_t)j * nx + i],
              a[(size_t)j * nx + wrapi(i + 1, nx)], hxm(s, i), hxp(s, i));
}

/* Central slope of a cell field in y (R4); one-sided next to a wall. */
static double slope_y(const orc_sim *s, const double *a, int i, int j) {
    if (s->mdx) return slope_y_mesh(s, a, i, j);
    int nx = s->nx, ny = s->ny;
    if (s->P.walls_y) {
        if (j == 0) return a[(size_t)1 * nx + i] - a[i];
        if (j == ny - 1)
            return a[(size_t)(ny - 1) * nx + i] - a[(size_t)(ny - 2) * nx + i];
    }
    return 0.5 * (a[(size_t)wrapi(j + 1, ny) * nx + i] -
                  a[(size_t)wrapi(j - 1, ny) * nx + i]);
}

/* Central slope of a cell field in x (x is always periodic). */
static double slope_x(const orc_sim *s, const double *a, int i, int j) {
    if (s->mdx) return slope_x_mesh(s, a, i, j);
    int nx = s->nx;
    return 0.5 * (a[(size_t)j * nx + wrapi(i + 1, nx)] -
                  a[(size_t)j * nx + wrapi(i - 1, nx)]);
}

/* Upwind mode: van Leer limited slope of two one-sided differences. */
static double van_leer(double a, double b) {
    return a * b > 0.0 ? 2.0 * a * b / (a + b) : 0.0;
}

/* R27: on a stretched mesh the limited slope is van Leer's of the two
   one-sided slopes (differences over the centre distances), capped at twice
   the smaller one-sided difference over the cell's own width, so that the
   one-dimensional reconstruction anywhere in the cell stays between the
   neighbours. The cap never binds on linear data, nor on the unit mesh. */
static double lim_mesh(double b, double f, double hm, double hp, double w) {
    double s = van_leer(b / hm, f / hp);
    double cap = 2.0 * fmin(fabs(b), fabs(f)) / w;
    return s > cap ? cap : (s < -cap ? -cap : s);
}

/* Limited x and y slopes of a cell field (one-sided next to a wall in y). */
static double lim_x(const orc_sim *s, const double *a, int i, int j) {
    int nx = s->nx;
    size_t c = (size_t)j * nx + i;
    if (s->mdx)
        return lim_mesh(a[c] - a[(size_t)j * nx + wrapi(i - 1, nx)],
                        a[(size_t)j * nx + wrapi(i + 1, nx)] - a[c], hxm(s, i), hxp(s, i),
                        wx(s, i));
    return van_leer(a[c] - a[(size_t)j * nx + wrapi(i - 1, nx)],
                    a[(size_t)j * nx + wrapi(i + 1, nx)] - a[c]);
}
static double lim_y(const orc_sim *s, const double *a, int i, int j) {
    int nx = s->nx, ny = s->ny;
    if (s->mdx) {
        if (s->P.walls_y && (j == 0 || j == ny - 1)) return slope_y_mesh(s, a, i, j);
        size_t c = (size_t)j * nx + i;
        return lim_mesh(a[c] - a[(size_t)wrapi(j - 1, ny) * nx + i],
                        a[(size_t)wrapi(j + 1, ny) * nx + i] - a[c], hym(s, j), hyp(s, j),
                        wy(s, j));
    }
    if (s->P.walls_y) {
        if (j == 0) return a[(size_t)1 * nx + i] - a[i];
        if (j == ny - 1) return a[(size_t)(ny - 1) * nx + i] - a[(size_t)(ny - 2) * nx + i];
    }
    size_t c = (size_t)j * nx + i;
    return van_leer(a[c] - a[(size_t)wrapi(j - 1, ny) * nx + i],
                    a[(size_t)wrapi(j + 1, ny) * nx + i] - a[c]);
}

/* Bar value of population q at the x-face between L = (i,j) and R = (ir,j)
   (upwind mode): x_f - h xi lies in the upwind cell at (1/2 - h e_x, -h e_y)
   from its centre (mirrored for e_x < 0). */
static double upwind_x(const orc_sim *s, const double *a, int q, int i, int ir, int j) {
    int nx = s->nx;
    size_t L = (size_t)j * nx + i, R = (size_t)j * nx + ir;
    double h = s->h;
    if (s->mdx) { /* offsets from the upwind centre: (dL - h, -h e_y) or (h - dR, -h e_y) */
        double dL = 0.5 * wx(s, i), dR = 0.5 * wx(s, ir);
        if (EX[q] > 0)
            return a[L] + (dL - h) * lim_x(s, a, i, j) - h * EY[q] * lim_y(s, a, i, j);
        if (EX[q] < 0)
            return a[R] + (h - dR) * lim_x(s, a, ir, j) - h * EY[q] * lim_y(s, a, ir, j);
        return (dR * (a[L] - h * EY[q] * lim_y(s, a, i, j)) +
                dL * (a[R] - h * EY[q] * lim_y(s, a, ir, j))) / (dL + dR);
    }
    if (EX[q] > 0)
        return a[L] + (0.5 - h) * lim_x(s, a, i, j) - h * EY[q] * lim_y(s, a, i, j);
    if (EX[q] < 0)
        return a[R] - (0.5 - h) * lim_x(s, a, ir, j) - h * EY[q] * lim_y(s, a, ir, j);
    return 0.5 * (a[L] + a[R]) - h * EY[q] * 0.5 * (lim_y(s, a, i, j) + lim_y(s, a, ir, j));
}

/* Same at the y-face between D = (i,jd) and U = (i,ju). */
static double upwind_y(const orc_sim *s, const double *a, int q, int i, int jd, int ju) {
    int nx = s->nx;
    size_t Dn = (size_t)jd * nx + i, Up = (size_t)ju * nx + i;
    double h = s->h;
    if (s->mdx) {
        double dD = 0.5 * wy(s, jd), dU = 0.5 * wy(s, ju);
        if (EY[q] > 0)
            return a[Dn] + (dD - h) * lim_y(s, a, i, jd) - h * EX[q] * lim_x(s, a, i, jd);
        if (EY[q] < 0)
            return a[Up] + (h - dU) * lim_y(s, a, i, ju) - h * EX[q] * lim_x(s, a, i, ju);
        return (dU * (a[Dn] - h * EX[q] * lim_x(s, a, i, jd)) +
                dD * (a[Up] - h * EX[q] * lim_x(s, a, i, ju))) / (dD + dU);
    }
    if (EY[q] > 0)
        return a[Dn] + (0.5 - h) * lim_y(s, a, i, jd) - h * EX[q] * lim_x(s, a, i, jd);
    if (EY[q] < 0)
        return a[Up] - (0.5 - h) * lim_y(s, a, i, ju) - h * EX[q] * lim_x(s, a, i, ju);
    return 0.5 * (a[Dn] + a[Up]) - h * EX[q] * 0.5 * (lim_x(s, a, i, jd) + lim_x(s, a, i, ju));
}

/* Bar value of population q at the x-face between L = (i,j) and R = (ir,j)
   with the central reconstruction of R4: a - h (e_qx d_n + e_qy d_t). */
static double central_x(const orc_sim *s, const double *a, int q, int i, int ir, int j) {
    size_t L = (size_t)j * s->nx + i, R = (size_t)j * s->nx + ir;
    if (s->mdx) {
        double dL = 0.5 * wx(s, i), dR = 0.5 * wx(s, ir), H = dL + dR;
        double af = (dR * a[L] + dL * a[R]) / H, dn = (a[R] - a[L]) / H;
        double dtg = (dR * slope_y(s, a, i, j) + dL * slope_y(s, a, ir, j)) / H;
        return af - s->h * (EX[q] * dn + EY[q] * dtg);
    }
    double avg = 0.5 * (a[L] + a[R]), dn = a[R] - a[L];
    double dtg = 0.5 * (slope_y(s, a, i, j) + slope_y(s, a, ir, j));
    return avg - s->h * (EX[q] * dn + EY[q] * dtg);
}

/* Same at the y-face between D = (i,jd) and U = (i,ju). */
static double central_y(const orc_sim *s, const double *a, int q, int i, int jd, int ju) {
    size_t Dn = (size_t)jd * s->nx + i, Up = (size_t)ju * s->nx + i;
    if (s->mdx) {
        double dD = 0.5 * wy(s, jd), dU = 0.5 * wy(s, ju), H = dD + dU;
        double af = (dU * a[Dn] + dD * a[Up]) / H, dn = (a[Up] - a[Dn]) / H;
        double dtg = (dU * slope_x(s, a, i, jd) + dD * slope_x(s, a, i, ju)) / H;
        return af - s->h * (EY[q] * dn + EX[q] * dtg);
    }
    double avg = 0.5 * (a[Dn] + a[Up]), dn = a[Up] - a[Dn];
    double dtg = 0.5 * (slope_x(s, a, i, jd) + slope_x(s, a, i, ju));
    return avg - s->h * (EY[q] * dn + EX[q] * dtg);
}

/* Face value in the reconstruction the parameters select. */
static double recon_x(const orc_sim *s, const double *a, int q, int i, int ir, int j) {
    return s->P.recon == ORC_RECON_UPWIND ? upwind_x(s, a, q, i, ir, j)
                                          : central_x(s, a, q, i, ir, j);
}
static double recon_y(const orc_sim *s, const double *a, int q, int i, int jd, int ju) {
    return s->P.recon == ORC_RECON_UPWIND ? upwind_y(s, a, q, i, jd, ju)
                                          : central_y(s, a, q, i, jd, ju);
}

/* Bar values of population q on every x-face (east of each cell) and every
   y-face (north of each cell; rows 0 .. ny-2 with walls) for a cell field a,
   in the reconstruction recon selects, with the functions Pass C uses. */
void orc_recon(int nx, int ny, int walls_y, const double *dx, const double *dy, int recon,
               double h, int q, const double *a, double *xface, double *yface) {
    orc_sim tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.nx = nx;
    tmp.ny = ny;
    tmp.P.walls_y = walls_y;
    tmp.P.recon = recon;
    if ((dx || dy) && orc_set_mesh(&tmp, dx, dy) != 0) return;
    tmp.h = h;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            xface[c] = recon_x(&tmp, a, q, i, wrapi(i + 1, nx), j);
            yface[c] = (walls_y && j == ny - 1) ? 0.0 : recon_y(&tmp, a, q, i, j, wrapi(j + 1, ny));
        }
    orc_set_mesh(&tmp, NULL, NULL);
}

/* Face macros and the face original distributions (Eq. 28) from the bar
   distributions at the face (R5, R6). The averaged gradient-type inputs come
   in as arguments. */
typedef struct {
    double gx, gy, mu, Dx, Dy; /* averaged gradient-type inputs (R5) */
    double xf, yf;             /* face position (for prescribed velocity) */
} face_in;

static void face_df(const orc_sim *s, const face_in *in, const double *fb,
                    const double *gb, double *fo, double *go) {
    double phif = 0.0;
    for (int q = 0; q < 9; ++q) phif += fb[q];
    double rhof = rho_of(s, phif), thf = theta_of(s, phif);
    double nxv, nyv;
    unit(s, in->gx, in->gy, &nxv, &nyv);
    double uf, vf;
    double feq[9], sf[9];
    if (s->coupled) {
        double Gx, Gy;
        gravity(s, rhof, &Gx, &Gy);
        double Fx = in->mu * in->gx + Gx, Fy = in->mu * in->gy + Gy;
        double drx = s->drho * in->gx, dry = s->drho * in->gy;
        double mx = 0.0, my = 0.0, m0 = 0.0;
        for (int q = 0; q < 9; ++q) {
            mx += EX[q] * gb[q];
            my += EY[q] * gb[q];
            if (q != 0) m0 += gb[q];
        }
        uf = (mx + 0.5 * s->h * Fx) / rhof;
        vf = (my + 0.5 * s->h * Fy) / rhof;
        double G0 = gamma_q(0, uf, vf) - gamma_q(0, 0.0, 0.0);
        double pf = RT / (1.0 - WQ[0]) *
                    (m0 + 0.5 * s->h * (uf * drx + vf * dry) + rhof * G0);
        double geq[9], sg[9];
        orc_geq(pf, rhof, uf, vf, geq);
        orc_sg(uf, vf, drx, dry, Fx, Fy, sg);
        orc_face_df(taug_of(s, phif, rhof), s->h, gb, geq, sg, go);
    } else {
        presc_vel(&s->P, in->xf, in->yf, orc_time(s) + s->h, &uf, &vf);
    }
    orc_feq(phif, uf, vf, feq);
    orc_sf(thf, nxv, nyv, in->Dx, in->Dy, sf);
    orc_face_df(s->tau_f, s->h, fb, feq, sf, fo);
}

/* R15: no-slip wall on the face below cell row 0 (bottom = 1) or above cell
   row ny-1 (bottom = 0). Outgoing populations are traced back into the
   adjacent cell with a one-sided y slope; their face distributions follow
   Eq. 28 with the face macros of the adjacent cell, zero velocity and zero
   normal components of grad phi and D. Incoming populations bounce back:
   psi_q = psi_opp(q). The mass flux of phi through the wall is then zero. */
static void wall_face(orc_sim *s, int i, int bottom) {
    int nx = s->nx, ny = s->ny;
    size_t n = (size_t)nx * ny;
    int j = bottom ? 0 : ny - 1, jn = bottom ? 1 : ny - 2;
    size_t c = (size_t)j * nx + i, cn = (size_t)jn * nx + i;
    size_t row = bottom ? 0 : (size_t)ny;
    double dyw = bottom ? -0.5 : 0.5; /* wall y minus cell-centre y */
    double sgn = bottom ? 1.0 : -1.0; /* sign of the one-sided difference */
    double idy = 1.0;                 /* 1 / distance to the next centre */
    if (s->mdx) {                     /* R27 */
        dyw = bottom ? -0.5 * wy(s, 0) : 0.5 * wy(s, ny - 1);
        idy = 1.0 / (bottom ? hyp(s, 0) : hym(s, ny - 1));
    }

    double phiw = s->phi[c];
    double rhow = rho_of(s, phiw), thw = theta_of(s, phiw);
    double gxw = s->gpx[c], gyw = 0.0, muw = s->mu[c];
    double Dxw = s->Dx[c], Dyw = 0.0;
    double nxv, nyv;
    unit(s, gxw, gyw, &nxv, &nyv);
    double Gx, Gy;
    gravity(s, rhow, &Gx, &Gy);
    double Fx = muw * gxw + Gx, Fy = muw * gyw + Gy;
    double feq[9], sf[9], geq[9], sg[9];
    orc_feq(phiw, 0.0, 0.0, feq);
    orc_sf(thw, nxv, nyv, Dxw, Dyw, sf);
    orc_geq(s->p[c], rhow, 0.0, 0.0, geq);
    orc_sg(0.0, 0.0, s->drho * gxw, s->drho * gyw, Fx, Fy, sg);
    double tg = taug_of(s, phiw, rhow);

    double fb[9], gb[9], fo[9], go[9];
    for (int q = 0; q < 9; ++q) {
        double dx = -s->h * EX[q], dy = dyw - s->h * EY[q];
        double sxf = slope_x(s, s->fbp + q * n, i, j);
        double syf = sgn * (s->fbp[q * n + cn] - s->fbp[q * n + c]);
        if (s->mdx) syf *= idy;
        fb[q] = s->fbp[q * n + c] + dx * sxf + dy * syf;
        double sxg = slope_x(s, s->gbp + q * n, i, j);
        double syg = sgn * (s->gbp[q * n + cn] - s->gbp[q * n + c]);
        if (s->mdx) syg *= idy;
        gb[q] = s->gbp[q * n + c] + dx * sxg + dy * syg;
    }
    orc_face_df(s->tau_f, s->h, fb, feq, sf, fo);
    orc_face_df(tg, s->h, gb, geq, sg, go);
    for (int q = 0; q < 9; ++q) {
        int out = bottom ? (EY[q] < 0) : (EY[q] > 0);
        int in = bottom ? (EY[q] > 0) : (EY[q] < 0);
        double fv = 0.0, gv = 0.0;
        if (out) {
            fv = fo[q];
            gv = go[q];
        } else if (in) {
            fv = fo[opp(q)];
            gv = go[opp(q)];
        }
        s->fyf[q * (size_t)nx * (ny + 1) + row * nx + i] = fv;
        s->gyf[q * (size_t)nx * (ny + 1) + row * nx + i] = gv;
    }
}

static void pass_c(orc_sim *s) {
    int nx = s->nx, ny = s->ny;
    size_t n = (size_t)nx * ny, n1 = (size_t)nx * (ny + 1);

    /* x-faces: face east of cell (i,j), between L = (i,j) and R = (i+1,j);
       the bar values at the face (Eq. 27) in the selected reconstruction. */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int ir = wrapi(i + 1, nx);
            size_t L = (size_t)j * nx + i, R = (size_t)j * nx + ir;
            double fb[9], gb[9], fo[9], go[9];
            for (int q = 0; q < 9; ++q) {
                fb[q] = recon_x(s, s->fbp + q * n, q, i, ir, j);
                if (s->coupled) gb[q] = recon_x(s, s->gbp + q * n, q, i, ir, j);
            }
            face_in in;
            if (s->mdx) { /* R27: linear interpolation to the face */
                double dL = 0.5 * wx(s, i), dR = 0.5 * wx(s, ir), H = dL + dR;
                in.gx = (dR * s->gpx[L] + dL * s->gpx[R]) / H;
                in.gy = (dR * s->gpy[L] + dL * s->gpy[R]) / H;
                in.mu = (dR * s->mu[L] + dL * s->mu[R]) / H;
                in.Dx = (dR * s->Dx[L] + dL * s->Dx[R]) / H;
                in.Dy = (dR * s->Dy[L] + dL * s->Dy[R]) / H;
                in.xf = xcen(s, i) + dL;
                in.yf = ycen(s, j);
            } else {
                in.gx = 0.5 * (s->gpx[L] + s->gpx[R]);
                in.gy = 0.5 * (s->gpy[L] + s->gpy[R]);
                in.mu = 0.5 * (s->mu[L] + s->mu[R]);
                in.Dx = 0.5 * (s->Dx[L] + s->Dx[R]);
                in.Dy = 0.5 * (s->Dy[L] + s->Dy[R]);
                in.xf = i + 1.0;
                in.yf = j + 0.5;
            }
            face_df(s, &in, fb, gb, fo, go);
            for (int q = 0; q < 9; ++q) {
                s->fxf[q * n + L] = fo[q];
                if (s->coupled) s->gxf[q * n + L] = go[q];
            }
        }

    /* y-faces between D = (i,j) and U = (i,j+1): rows jj = 1 .. ny-1, plus
       jj = ny when y is periodic (U wraps to row 0). */
    int jlast = s->P.walls_y ? ny - 1 : ny;
#pragma omp parallel for schedule(static)
    for (int jj = 1; jj <= jlast; ++jj)
        for (int i = 0; i < nx; ++i) {
            int jd = jj - 1, ju = wrapi(jj, ny);
            size_t Dn = (size_t)jd * nx + i, Up = (size_t)ju * nx + i;
            double fb[9], gb[9], fo[9], go[9];
            for (int q = 0; q < 9; ++q) {
                fb[q] = recon_y(s, s->fbp + q * n, q, i, jd, ju);
                if (s->coupled) gb[q] = recon_y(s, s->gbp + q * n, q, i, jd, ju);
            }
            face_in in;
            if (s->mdx) {
                double dD = 0.5 * wy(s, jd), dU = 0.5 * wy(s, ju), H = dD + dU;
                in.gx = (dU * s->gpx[Dn] + dD * s->gpx[Up]) / H;
                in.gy = (dU * s->gpy[Dn] + dD * s->gpy[Up]) / H;
                in.mu = (dU * s->mu[Dn] + dD * s->mu[Up]) / H;
                in.Dx = (dU * s->Dx[Dn] + dD * s->Dx[Up]) / H;
                in.Dy = (dU * s->Dy[Dn] + dD * s->Dy[Up]) / H;
                in.xf = xcen(s, i);
                in.yf = ycen(s, jd) + dD;
            } else {
                in.gx = 0.5 * (s->gpx[Dn] + s->gpx[Up]);
                in.gy = 0.5 * (s->gpy[Dn] + s->gpy[Up]);
                in.mu = 0.5 * (s->mu[Dn] + s->mu[Up]);
                in.Dx = 0.5 * (s->Dx[Dn] + s->Dx[Up]);
                in.Dy = 0.5 * (s->Dy[Dn] + s->Dy[Up]);
                in.xf = i + 0.5;
                in.yf = (double)jj;
            }
            face_df(s, &in, fb, gb, fo, go);
            for (int q = 0; q < 9; ++q) {
                s->fyf[q * n1 + (size_t)jj * nx + i] = fo[q];
                if (s->coupled) s->gyf[q * n1 + (size_t)jj * nx + i] = go[q];
            }
        }

    if (s->P.walls_y) {
        for (int i = 0; i < nx; ++i) {
            wall_face(s, i, 1);
            wall_face(s, i, 0);
        }
    } else { /* periodic: the face at y = 0 is the face at y = ny */
        for (int q = 0; q < 9; ++q)
            for (int i = 0; i < nx; ++i) {
                s->fyf[q * n1 + i] = s->fyf[q * n1 + (size_t)ny * nx + i];
                if (s->coupled) s->gyf[q * n1 + i] = s->gyf[q * n1 + (size_t)ny * nx + i];
            }
    }
}

/* ------------------------------------------------------ Pass D: update */

/* Eq. 24 with the microflux of Eq. 22 on rectangular cells: the outward
   normals are +-x and +-y; a face's length over the cell's area is 1/dx or
   1/dy (1 on the unit mesh). */
static void pass_d(orc_sim *s) {
    int nx = s->nx, ny = s->ny;
    size_t n = (size_t)nx * ny, n1 = (size_t)nx * (ny + 1);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i, w = (size_t)j * nx + wrapi(i - 1, nx);
            size_t fn = (size_t)(j + 1) * nx + i, fs = (size_t)j * nx + i;
            /* R27: face lengths over the cell area, 1/dx and 1/dy */
            double ax = s->mdx ? 1.0 / wx(s, i) : 1.0, ay = s->mdx ? 1.0 / wy(s, j) : 1.0;
            for (int q = 0; q < 9; ++q) {
                double Jx = EX[q] * (s->fxf[q * n + c] - s->fxf[q * n + w]);
                double Jy = EY[q] * (s->fyf[q * n1 + fn] - s->fyf[q * n1 + fs]);
                double J = s->mdx ? ax * Jx + ay * Jy : Jx + Jy;
                s->f[q * n + c] = s->ftp[q * n + c] - s->dt * J;
                if (s->coupled) {
                    double Jgx = EX[q] * (s->gxf[q * n + c] - s->gxf[q * n + w]);
                    double Jgy = EY[q] * (s->gyf[q * n1 + fn] - s->gyf[q * n1 + fs]);
                    double Jg = s->mdx ? ax * Jgx + ay * Jgy : Jgx + Jgy;
                    s->g[q * n + c] = s->gtp[q * n + c] - s->dt * Jg;
                }
            }
            s->hist[c] = s->phi[c] * s->ux[c];
            s->hist[n + c] = s->phi[c] * s->uy[c];
        }
}

void orc_step(orc_sim *s, int nsteps) {
    for (int k = 0; k < nsteps; ++k) {
        pass_a(s);
        pass_b(s);
        pass_c(s);
        pass_d(s);
        s->step += 1;
    }
}

/* ----------------------------------------------------- init and readout */

/* R11: tilde distributions from the initial macros with D = 0. For the
   interface-only model the velocity is the prescribed field at t = 0 and the
   u, v, p arguments are ignored. */
int orc_init(orc_sim *s, const double *phi0, const double *u0, const double *v0,
             const double *p0) {
    int nx = s->nx, ny = s->ny;
    size_t n = (size_t)nx * ny;
    s->step = 0;
    memcpy(s->phi, phi0, n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double phi = s->phi[c], gx, gy, lap, ux, uy, p = 0.0;
            stencils(s, s->phi, i, j, &gx, &gy, &lap);
            s->gpx[c] = gx;
            s->gpy[c] = gy;
            s->lap[c] = lap;
            s->mu[c] = chem_pot(s, phi, lap);
            s->theta[c] = theta_of(s, phi);
            s->rho[c] = rho_of(s, phi);
            if (s->coupled) {
                ux = u0 ? u0[c] : 0.0;
                uy = v0 ? v0[c] : 0.0;
                p = p0 ? p0[c] : 0.0;
            } else {
                presc_vel(&s->P, xcen(s, i), ycen(s, j), 0.0, &ux, &uy);
            }
            s->ux[c] = ux;
            s->uy[c] = uy;
            s->p[c] = p;
            s->Dx[c] = 0.0;
            s->Dy[c] = 0.0;
            double feq[9], sf[9], geq[9], sg[9];
            cell_eq_src(s, c, feq, sf, geq, sg);
            for (int q = 0; q < 9; ++q) {
                s->f[q * n + c] = feq[q] - 0.5 * s->dt * sf[q];
                s->g[q * n + c] = s->coupled ? geq[q] - 0.5 * s->dt * sg[q] : 0.0;
            }
            s->hist[c] = phi * ux;
            s->hist[n + c] = phi * uy;
        }
    return 0;
}

/* Cell macros of the current state (Pass A). Any output may be NULL. */
void orc_macros(orc_sim *s, double *phi, double *u, double *v, double *p,
                double *rho) {
    size_t n = (size_t)s->nx * s->ny;
    pass_a(s);
    if (phi) memcpy(phi, s->phi, n * sizeof(double));
    if (u) memcpy(u, s->ux, n * sizeof(double));
    if (v) memcpy(v, s->uy, n * sizeof(double));
    if (p) memcpy(p, s->p, n * sizeof(double));
    if (rho) memcpy(rho, s->rho, n * sizeof(double));
}

/* Extra cell fields of Pass A for diagnostics: grad phi, Laplacian, mu_phi. */
void orc_cell_fields(orc_sim *s, double *gx, double *gy, double *lap,
                     double *mu) {
    size_t n = (size_t)s->nx * s->ny;
    pass_a(s);
    if (gx) memcpy(gx, s->gpx, n * sizeof(double));
    if (gy) memcpy(gy, s->gpy, n * sizeof(double));
    if (lap) memcpy(lap, s->lap, n * sizeof(double));
    if (mu) memcpy(mu, s->mu, n * sizeof(double));
}

/* Full state: f (9n), g (9n), hist (2n), and the step counter. */
void orc_get_state(const orc_sim *s, double *f, double *g, double *hist,
                   long *step) {
    size_t n = (size_t)s->nx * s->ny;
    if (f) memcpy(f, s->f, 9 * n * sizeof(double));
    if (g) memcpy(g, s->g, 9 * n * sizeof(double));
    if (hist) memcpy(hist, s->hist, 2 * n * sizeof(double));
    if (step) *step = s->step;
}

void orc_set_state(orc_sim *s, const double *f, const double *g,
                   const double *hist, long step) {
    size_t n = (size_t)s->nx * s->ny;
    if (f) memcpy(s->f, f, 9 * n * sizeof(double));
    if (g) memcpy(s->g, g, 9 * n * sizeof(double));
    if (hist) memcpy(s->hist, hist, 2 * n * sizeof(double));
    s->step = step;
}
