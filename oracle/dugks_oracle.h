/*
 * FP64 CPU oracle of the phase-field DUGKS step (arXiv:1810.07802).
 * TEST INFRASTRUCTURE: used only by the tests, the package smoke check and
 * the CPU-baseline leg of the benchmark. Not part of the product.
 *
 * Fields are row-major [ny][nx] (cell (i,j) at index j*nx + i, centre at
 * (i+1/2, j+1/2)). Distributions are [9][ny][nx] in the paper's velocity order.
 */
#ifndef DUGKS_ORACLE_H
#define DUGKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_VISC_UNIFORM_NU = 0, ORC_VISC_RECIPROCAL = 1, ORC_VISC_LINEAR = 2 };
enum { ORC_GRAV_RHO_G = 0, ORC_GRAV_BUOYANCY = 1 };
enum { ORC_VEL_UNIFORM = 0, ORC_VEL_ROTATION = 1, ORC_VEL_SHEAR = 2, ORC_VEL_DEFORM = 3 };
enum { ORC_RECON_CENTRAL = 0, ORC_RECON_UPWIND = 1 };

typedef struct {
    double phi_H, phi_L;   /* order parameter of the heavy / light phase */
    double rho_H, rho_L;   /* densities */
    double mu_H, mu_L;     /* dynamic viscosities (reciprocal / linear modes) */
    double nu;             /* kinematic viscosity (uniform mode) */
    int visc_mode;         /* ORC_VISC_* */
    double sigma, W, M;    /* surface tension, interface width, mobility */
    double gx, gy;         /* gravitational acceleration */
    int gravity_form;      /* ORC_GRAV_* */
    double Gx, Gy;         /* constant body-force density */
    double cfl;            /* CFL number; dt = cfl */
    int walls_y;           /* 0: periodic in y, 1: no-slip walls at y=0, ny */
    int vel_kind;          /* interface-only model: prescribed velocity */
    double U0, L0, T_period;
    int recon;             /* ORC_RECON_*: face reconstruction of Eq. 27 */
    double eps_n;          /* R7: regularisation of the unit normal, in units of
                              |phi_H - phi_L| / delta_l; 0 = the plain unit normal */
} orc_params;

typedef struct orc_sim orc_sim;

orc_sim *orc_create(int nx, int ny, int coupled, const orc_params *P);
void orc_destroy(orc_sim *s);
int orc_set_params(orc_sim *s, const orc_params *P);
/* Stretched tensor-product mesh: cell widths dx[nx], dy[ny] (> 0; either may
   be NULL for unit widths on that axis; both NULL: the unit mesh). Returns -1
   on a width <= 0. dt becomes cfl times the smallest width. */
int orc_set_mesh(orc_sim *s, const double *dx, const double *dy);
int orc_init(orc_sim *s, const double *phi0, const double *u0,
             const double *v0, const double *p0);
void orc_step(orc_sim *s, int nsteps);
void orc_macros(orc_sim *s, double *phi, double *u, double *v, double *p,
                double *rho);
void orc_cell_fields(orc_sim *s, double *gx, double *gy, double *lap,
                     double *mu);
void orc_get_state(const orc_sim *s, double *f, double *g, double *hist,
                   long *step);
void orc_set_state(orc_sim *s, const double *f, const double *g,
                   const double *hist, long step);
double orc_time(const orc_sim *s);
long orc_step_count(const orc_sim *s);
void orc_derived(const orc_sim *s, double *out6);

/* point functions (for the moment-identity tests) */
void orc_feq(double phi, double ux, double uy, double *out9);
void orc_sf(double theta, double nx, double ny, double Dx, double Dy,
            double *out9);
void orc_geq(double p, double rho, double ux, double uy, double *out9);
void orc_sg(double ux, double uy, double drx, double dry, double Fx,
            double Fy, double *out9);
void orc_bar_plus(double tau, double dt, const double *tl, const double *eq,
                  const double *S, double *bp, double *tp);
void orc_face_df(double tau, double h, const double *bar, const double *eq,
                 const double *S, double *out);
/* Bar values of population q at the faces (Eq. 27, both reconstructions):
   xface[j nx + i] east of cell (i,j), yface[j nx + i] north of it. */
void orc_recon(int nx, int ny, int walls_y, const double *dx, const double *dy, int recon,
               double h, int q, const double *a, double *xface, double *yface);
/* Gradient and Laplacian of phi (R8, R9; R27 when dx or dy is given). */
void orc_stencils(int nx, int ny, int walls_y, const double *dx, const double *dy,
                  const double *phi, double *gx, double *gy, double *lap);

#ifdef __cplusplus
}
#endif
#endif
