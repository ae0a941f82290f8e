/*
 * dugks.h — C ABI of the MI355X (gfx950) implementation of the phase-field
 * discrete unified gas-kinetic scheme of Yang, Zhong & Zhuo,
 * "A phase-field model for large-density-ratio two-phase flows based on
 * discrete unified gas-kinetic scheme" (arXiv:1810.07802).
 *
 * One handle is one uniform 2-D D2Q9 grid of nx x ny unit cells (cell (i,j)
 * centred at (i+1/2, j+1/2), row-major [ny][nx] in every host or device field
 * passed through this ABI), x always periodic, y periodic or bounded by
 * no-slip walls on the faces y = 0 and y = ny. It carries either
 *   - the coupled model: conservative Allen-Cahn kinetic model f for the order
 *     parameter phi plus the incompressible hydrodynamic model g for the
 *     dynamic pressure p and the velocity u (Sec. II.A-II.B), or
 *   - the interface-only model: f alone, advected by a prescribed velocity
 *     field (Sec. III, Eqs. 40-43).
 * The time step is the DUGKS update of Sec. II.B (Eqs. 21-33).
 *
 * Conventions
 *   - Every call returns an int status: DUGKS_OK (0) or a negative DUGKS_E*
 *     code; dugks_last_error() gives a message. Nothing aborts, no C++
 *     exception crosses the ABI.
 *   - The library owns all device memory of a handle. The caller owns every
 *     pointer it passes; the library never keeps one after the call returns.
 *   - Calls on one handle are not thread-safe; distinct handles are
 *     independent. All device work of a handle is ordered on its stream
 *     (default: the null stream; see dugks_set_stream()).
 *   - Time is implicit: t = steps * dt with dt = CFL (grid spacing 1,
 *     sqrt(3RT) = 1; Eq. 37), or CFL times the smallest width on a
 *     stretched mesh (dugks_set_mesh).
 */
#ifndef DUGKS_H
#define DUGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DUGKS_OK 0
#define DUGKS_EINVAL (-1)   /* bad argument or parameter */
#define DUGKS_ENOMEM (-2)   /* device or host allocation failed */
#define DUGKS_EDEVICE (-3)  /* HIP runtime error */
#define DUGKS_ENUMERIC (-4) /* NaN/Inf in the state (sticky; see dugks_sync) */
#define DUGKS_ESTATE (-5)   /* call out of order (e.g. step before init) */
#define DUGKS_EBUSY (-6)    /* pool has no room for the request */

enum { DUGKS_FP32 = 0, DUGKS_FP64 = 1 };
enum { DUGKS_MODEL_AC = 0, DUGKS_MODEL_COUPLED = 1 };
enum { DUGKS_VISC_UNIFORM_NU = 0, DUGKS_VISC_RECIPROCAL = 1, DUGKS_VISC_LINEAR = 2 };
enum { DUGKS_GRAV_RHO_G = 0, DUGKS_GRAV_BUOYANCY = 1 };
enum { DUGKS_BC_PERIODIC = 0, DUGKS_BC_WALLS = 1 };
enum { DUGKS_VEL_UNIFORM = 0, DUGKS_VEL_ROTATION = 1, DUGKS_VEL_SHEAR = 2,
       DUGKS_VEL_DEFORM = 3 };
enum { DUGKS_RECON_CENTRAL = 0, DUGKS_RECON_UPWIND = 1 };

/* Physical and numerical parameters (Sec. II, III, IV of the paper).
 *   phi_H, phi_L   order parameter of the heavy / light phase (Sec. II.A);
 *                  the interface sits at their mean. Must differ.
 *   rho_H, rho_L   densities, interpolated linearly in phi (Eq. 10); > 0.
 *   mu_H, mu_L     dynamic viscosities for visc_mode RECIPROCAL (Eq. 35) or
 *                  LINEAR (Eq. 36); > 0 when used.
 *   nu             kinematic viscosity for visc_mode UNIFORM_NU; > 0.
 *   sigma, W       surface tension (>= 0) and interface width (> 0); they set
 *                  kappa and beta (Eq. 3, generalised so that width and
 *                  tension hold for any phi_H - phi_L).
 *   M_phi          mobility (>= 0); tau_f = M_phi / RT (Eq. 34).
 *   gx, gy         gravitational acceleration; gravity_form RHO_G gives
 *                  G = rho g, BUOYANCY gives G = (rho - (rho_H+rho_L)/2) g.
 *   Gx, Gy         constant body-force density added to G (layered
 *                  Poiseuille flow, Sec. IV.B).
 *   cfl            CFL number in (0, 1]; dt = cfl, h = dt/2.
 *   bc_y           DUGKS_BC_PERIODIC or DUGKS_BC_WALLS (coupled model only;
 *                  needs ny >= 4).
 *   vel_kind, U0, L0, T_period
 *                  prescribed velocity of the interface-only model
 *                  (Eqs. 40-43); ignored by the coupled model.
 *   recon          face reconstruction of the bar distributions (Eq. 27):
 *                  DUGKS_RECON_CENTRAL (0, default) is the central one of the
 *                  paper's runs: mean of the two cells, their difference as
 *                  the normal slope, central differences along the face.
 *                  DUGKS_RECON_UPWIND (1) is the upwind, limited
 *                  reconstruction that Sec. III names against the central
 *                  one's Peclet-number error growth: the population crossing
 *                  a face is evaluated in its upwind cell at the point it
 *                  left from, x_face - h xi, with that cell's van Leer limited
 *                  slopes (2ab/(a+b) of the one-sided differences a, b if
 *                  ab > 0, else 0; one-sided and unlimited next to a wall);
 *                  populations along the face take the mean of both cells.
 *                  Upwind runs on single handles only (EINVAL in batches and
 *                  pools); it needs no device memory beyond the state. It
 *                  runs as a second march like the central one (each
 *                  cell's limited slopes formed once), on the unit mesh and
 *                  on a stretched mesh (see dugks_set_mesh).
 *   eps_n          regularisation of the interface normal of the phase-field
 *                  source (Eq. 16, n of Sec. II.A):
 *                  n = grad phi / sqrt(|grad phi|^2 + eps^2) with
 *                  eps = eps_n |phi_H - phi_L| (over the smallest width on a
 *                  stretched mesh). eps_n = 0 is the plain unit normal (n = 0
 *                  where grad phi = 0 exactly); a small eps_n (1e-6, the
 *                  Python default) keeps n continuous where the gradient
 *                  vanishes. >= 0.
 */
typedef struct dugks_params {
    double phi_H, phi_L;
    double rho_H, rho_L;
    double mu_H, mu_L;
    double nu;
    int visc_mode;
    double sigma, W, M_phi;
    double gx, gy;
    int gravity_form;
    double Gx, Gy;
    double cfl;
    int bc_y;
    int vel_kind;
    double U0, L0, T_period;
    int recon;
    double eps_n;
} dugks_params;

typedef struct dugks_handle dugks_handle;

/* Create a grid of nx x ny cells (nx, ny >= 3) holding `model`
 * (DUGKS_MODEL_*) in `precision` (DUGKS_FP32: distributions and arithmetic in
 * float, density and relaxation-time interpolation in double; DUGKS_FP64: all
 * double). Allocates the two state buffers on the current HIP device.
 * nx * ny may not exceed 2^28 cells in FP32, 2^27 in FP64.
 * Errors: EINVAL (sizes, enums), ENOMEM, EDEVICE. *out is NULL on error. */
int dugks_create(int nx, int ny, int precision, int model, dugks_handle **out);

/* Validate and set parameters. EINVAL on phi_H == phi_L, rho <= 0, a needed
 * viscosity <= 0, M_phi < 0, cfl outside (0,1], W <= 0, sigma < 0, walls with
 * the interface-only model or ny < 4. Resets nothing; takes effect from the
 * next init or step. */
int dugks_set_params(dugks_handle *h, const dugks_params *p);

/* Use `stream` (a hipStream_t, NULL = null stream) for all later work. */
int dugks_set_stream(dugks_handle *h, void *stream);

/* Work decomposition of the step kernel: rows per segment of a 62-column
 * strip (each (strip, segment) tile is one 64-lane wave). 0 = automatic
 * (the shortest segments whose tiles are all resident on the device at
 * once; if those would exceed 64 rows, the shortest that fit eight rounds;
 * for periodic FP32 cases whose one-row tiles outnumber the compute units
 * while two-row tiles do not, two rows, run by the four-wave two-row
 * kernel). Results do not depend on it, bit for bit. A batch uses a case's
 * explicit value, and its own automatic choice for cases left at 0. With
 * the upwind reconstruction or a stretched mesh the value is the segment of
 * the reconstruction march instead (60-column strips; automatic: one round of resident
 * waves, or where that needs more than 64 rows the shortest segments that
 * number at most 32 waves per compute unit). EINVAL outside [0, 4096].
 * dugks_get_tile returns the value in use (-1 for NULL). */
int dugks_set_tile(dugks_handle *h, int seg_rows);
int dugks_get_tile(const dugks_handle *h);

/* Stretched tensor-product mesh (DUGKS is a finite-volume scheme: Eq. 21
 * integrates the microflux over the cell surface and divides by the cell
 * volume; the introduction names this as its advantage over the uniform
 * lattice of the lattice Boltzmann method). dx[nx] and dy[ny] are the cell
 * widths (host arrays of double, copied; finite and > 0; either may be NULL
 * for unit widths on that axis). Both NULL returns to the unit mesh.
 * On a stretched mesh:
 *   - dt = cfl * (smallest width), and the time of dugks_time follows it;
 *   - the update divides the x and y microfluxes by the cell's widths;
 *   - the gradient and Laplacian are weighted sums of the derivatives of the
 *     parabola through three neighbouring centres (exact on quadratics, the
 *     unit-mesh stencils on unit widths);
 *   - the face reconstruction interpolates linearly to the face, with slopes
 *     over the centre distances (both reconstructions; the upwind slopes are
 *     van Leer's of the one-sided slopes, capped at twice the smaller
 *     one-sided difference over the cell width);
 *   - the regularisation of the unit normal is eps_n |phi_H - phi_L| over
 *     the smallest width.
 * The step then runs as the reconstruction march (both reconstructions; the
 * central one forms its parabola slopes where used), which needs no device
 * memory beyond the state and the metrics. Cell centres start at
 * x = 0, y = 0. Takes effect at the next dugks_init_fields (the state is
 * invalidated: ESTATE until then). Not for batches or pool cases (EINVAL).
 * Errors: EINVAL (widths), ENOMEM. */
int dugks_set_mesh(dugks_handle *h, const double *dx, const double *dy);

/* Build the initial state from cell macros: host arrays [ny][nx] of double,
 * copied during the call. u, v, p may be NULL (zero); the interface-only
 * model ignores them and uses the prescribed velocity at t = 0. The tilde
 * distributions start at psi^eq - (dt/2) S with a zero time derivative of
 * phi u (Eqs. 23, 15-19). Resets the step counter. ESTATE before set_params. */
int dugks_init_fields(dugks_handle *h, const double *phi, const double *u,
                      const double *v, const double *p);

/* As dugks_init_fields with device pointers (double, [ny][nx]), read on the
 * handle's stream; asynchronous. */
int dugks_init_fields_device(dugks_handle *h, const double *phi,
                             const double *u, const double *v,
                             const double *p);

/* Enqueue nsteps >= 0 time steps (Sec. II.B: cell macros, bar-plus and
 * tilde-plus auxiliaries, half-step face reconstruction, face macros and face
 * distributions, microflux, cell update). Asynchronous; ESTATE before init.
 * Every step checks each updated cell: a non-finite new phi, phi u or p sets
 * the handle's device flag. A synchronising call that finds the flag set
 * (dugks_sync, dugks_get_macros, dugks_get_diagnostics, dugks_get_state)
 * makes the numeric error sticky; from then on dugks_step returns ENUMERIC
 * without enqueuing anything, until dugks_init_fields or dugks_set_state.
 * On a stream set with dugks_set_stream (not the null stream, and not while
 * the caller captures it), a sequence of 8 or more steps is recorded once in
 * a HIP graph per step count (the last 8 counts are kept, and all are dropped
 * when the step's variant or tiles change) and replayed: the same kernels in
 * the same order, the same results bit for bit. */
int dugks_step(dugks_handle *h, int nsteps);

/* Wait for the handle's stream and read its non-finite flag. EDEVICE on a
 * device error; ENUMERIC when a step since the last init produced a
 * non-finite value (sticky: see dugks_step). */
int dugks_sync(dugks_handle *h);

/* Cell macros of the current state (Eqs. 31-33 and Eq. 10): phi, u, v, p,
 * rho into host arrays [ny][nx] of double; NULL skips a field. Synchronises
 * the handle's stream. For the interface-only model u, v are the prescribed
 * field at the current time and p = 0. A readout: returns OK on a non-finite
 * state too (the values are copied as they are), but makes the numeric error
 * sticky if the flag is set. */
int dugks_get_macros(dugks_handle *h, double *phi, double *u, double *v,
                     double *p, double *rho);

/* As dugks_get_macros into device arrays; asynchronous on the stream. */
int dugks_get_macros_device(dugks_handle *h, double *phi, double *u,
                            double *v, double *p, double *rho);

/* Diagnostics of the current state, accumulated in double on the device in
 * a fixed order: out[0] = sum phi, out[1] = sum rho u, out[2] = sum rho v,
 * out[3] = sum rho |u|^2 / 2, out[4] = max |u|, out[5] = sum rho,
 * out[6] = number of non-finite cells, out[7] = time. Sums are over cells,
 * not weighted by cell area (on a stretched mesh the conserved quantity is
 * the area integral of phi). Synchronises. Returns ENUMERIC (with out
 * filled) when out[6] > 0. */
int dugks_get_diagnostics(dugks_handle *h, double out[8]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): the diagnostics of dugks_get_diagnostics
 * (out_dev[0..6], same order and meaning) written asynchronously on the
 * handle's stream to out_dev, a device array of at least 7 doubles owned by
 * the caller; the time is dugks_time. Allocates nothing: the cell macros are
 * formed inside the reduction, and its per-row partial sums go to a
 * file-scope device array of the library (65536 rows x 7 doubles, one per
 * GPU, held until the process ends). Every call on a GPU shares that array:
 * calls that overlap on one GPU (other streams, other threads) race, and
 * must be ordered by the caller. The sums are accumulated in double in a
 * fixed order (rows, then row order): they agree with dugks_get_diagnostics
 * to rounding; the maximum and the count agree exactly. EINVAL for a grid
 * of more than 65536 rows; ESTATE before init. Does not read or report the
 * non-finite flag (out_dev[6] counts non-finite cells). */
int dugks_get_diagnostics_noalloc(dugks_handle *h, double *out_dev);

/* Steps taken since init and the current time. */
long long dugks_steps_done(const dugks_handle *h);
double dugks_time(const dugks_handle *h);

/* Checkpoint/resume: the state is the tilde distributions, the history
 * (phi u)^(n-1), phi and the step counter. dugks_state_bytes()
 * gives the size of the host buffer; get/set copy it (synchronous). Layout
 * (values of the handle's precision): ny rows, row y first; each row holds
 * the values f0..f8, [g0..g8], hist_x, hist_y of its nx cells in groups of
 * four consecutive values, each group cell-interleaved ([nx][4]; a last
 * partial group of w values is [nx][w]), then phi [nx], and is padded to a
 * multiple of 128 bytes. */
size_t dugks_state_bytes(const dugks_handle *h);
int dugks_get_state(dugks_handle *h, void *host_buf, size_t bytes,
                    long long *steps);
int dugks_set_state(dugks_handle *h, const void *host_buf, size_t bytes,
                    long long steps);

/* Tile autotuner: times probe_steps (1..1000) steps (with a stream set, as
 * one captured graph replayed; on the null stream as direct launches) for
 * each of a few
 * segment lengths (1 and 2 rows, for the lowest latency per step, and for
 * k = 1..8, 12, 16, 20, 24 the shortest segment whose tiles fit k rounds of the
 * device's resident waves) on the handle's current state, keeps the fastest as the
 * handle's tile (dugks_set_tile) and puts the state and step counter back as
 * they were. With the upwind reconstruction or a stretched mesh the tiles are
 * those of the reconstruction march (60-column strips, its own resident
 * waves). Results do not depend on the tile, bit for bit. Synchronous;
 * holds one extra copy of the state on the device while it runs. Outputs
 * (NULL to skip): the chosen seg_rows and its time per step in microseconds.
 * ESTATE before init; on EDEVICE the state is undefined. */
int dugks_autotune(dugks_handle *h, int probe_steps, int *seg_rows,
                   double *us_per_step);

/* Device bytes a handle of this shape holds (both state buffers). A
 * stretched mesh adds 156 (nx + ny) bytes of metrics (13 arrays per axis in
 * double and again in float). */
size_t dugks_footprint_bytes(int nx, int ny, int precision, int model);

/* Message of the last error on h (or of the last failed create when h is
 * NULL). Never NULL. */
const char *dugks_last_error(const dugks_handle *h);

/* Release a handle; NULL is accepted. */
int dugks_destroy(dugks_handle *h);

/* ---------------------------------------------------------------- batches
 * A batch advances several cases of the same precision and model together
 * (independent grids of uneven sizes, e.g. the spinodal runs of Sec. IV.C):
 * work items are the (case, column strip, row segment) tiles of every case,
 * and a step sequence can be recorded once in a HIP graph and replayed. The
 * cases are handles and stay usable on their own (set_params, init,
 * get_macros) between batch calls; the batch works on the batch's stream.
 * With two or more cases they run as two independent chains of launches,
 * one per half of the cells (split between cases): one chain on the batch's
 * stream, the other on a stream the batch owns (default priority), forked
 * from and joined back to the batch's stream within each dugks_batch_step,
 * so that work after the call on the batch's stream sees all cases done. Work items are built at the first
 * dugks_batch_step or dugks_batch_autotune, and again when a case's boundary
 * or explicit tile changes. Every case needs its parameters and state then
 * (ESTATE otherwise); the upwind reconstruction and stretched meshes are
 * refused (EINVAL). */
typedef struct dugks_batch dugks_batch;

/* n cases of nx[k] x ny[k] cells (host arrays, read during the call) in
 * `precision` and `model`, created and owned by the batch (destroyed with
 * it). Set up each case through dugks_batch_case. Errors as dugks_create,
 * naming the case. */
int dugks_batch_create(int n, const int *nx, const int *ny, int precision,
                       int model, dugks_batch **out);

/* Case k of a batch (NULL for a bad index or batch): a handle for
 * dugks_set_params, dugks_init_fields, dugks_get_macros and the other
 * single-case calls. Owned by the batch when it made the case. */
dugks_handle *dugks_batch_case(dugks_batch *b, int k);

/* A batch over existing handles (with parameters set, of one precision and
 * model), which must outlive the batch; the batch does not destroy them. */
int dugks_batch_create_from(int n, dugks_handle *const *cases,
                            dugks_batch **out);

/* Advance every active case by nsteps. use_graph = 1 records the sequence of
 * nsteps launches in a HIP graph on first use (per distinct nsteps) and
 * replays it; it needs a stream set with dugks_batch_set_stream (the null
 * stream cannot be captured: EINVAL). Cases with a step budget
 * (dugks_batch_set_budget) stop when it runs out. Asynchronous on the batch
 * stream. ENUMERIC (nothing enqueued) while a case's numeric error is sticky
 * (see dugks_step); the message names the cases. */
int dugks_batch_step(dugks_batch *b, int nsteps, int use_graph);

/* Limit case k to `steps` more steps (negative = unlimited); takes effect
 * from the next dugks_batch_step. */
int dugks_batch_set_budget(dugks_batch *b, int k, long long steps);

int dugks_batch_set_stream(dugks_batch *b, void *stream);
/* Wait for the batch stream and read every case's non-finite flag: ENUMERIC
 * (naming the cases) when one is set; those cases' numeric errors become
 * sticky. */
int dugks_batch_sync(dugks_batch *b);
int dugks_batch_destroy(dugks_batch *b);

/* Tile autotuner of a batch: for each boundary group (periodic cases, wall
 * cases) in turn, times probe_steps (1..1000) batch steps (with a stream set,
 * as one captured graph replayed, the way dugks_batch_step with use_graph
 * runs them; on the null stream as direct launches) for the same
 * candidate segment lengths as dugks_autotune, computed over the whole group,
 * keeps the fastest for every case of the group, and puts every case's state
 * and the batch's step counter back as they were (results do not depend on
 * the tile, bit for bit). Synchronous; holds one extra copy of every case's
 * state while it runs. Outputs (NULL to skip): the chosen segment length of
 * each group (0 for an empty group). ESTATE if a case has no state; on
 * EDEVICE the states are undefined. */
int dugks_batch_autotune(dugks_batch *b, int probe_steps, int *seg_periodic,
                         int *seg_walls);

/* Message of the last error on b (or of the last failed batch_create when b
 * is NULL). Never NULL. */
const char *dugks_batch_last_error(const dugks_batch *b);

/* ------------------------------------------------------------ serving pool
 * Continuous batching of solve requests (cases) of one precision and model.
 * The pool owns one device arena of hbm_bytes for case states and a table of
 * max_cases slots. A case is admitted while others run if a slot is free and
 * its state (dugks_pool_case_bytes) fits in the arena; otherwise admission
 * returns EBUSY and changes nothing. Every admitted case runs its own number
 * of steps: dugks_pool_step advances all cases that still have steps left,
 * in batched launches, and a case stops at its target. A retired case's
 * memory returns to the arena once the pool's stream has passed the
 * retirement. Results do not depend on the other cases in the pool, bit for
 * bit (the step of a case reads only its own state). Not thread-safe. */
typedef struct dugks_pool dugks_pool;

/* max_cells bounds the cells of one case (it sizes the staging area for
 * init and readout: 5 max_cells doubles). EINVAL, ENOMEM, EDEVICE. */
int dugks_pool_create(size_t hbm_bytes, int max_cases, long long max_cells,
                      int precision, int model, dugks_pool **out);
/* Stream of all pool work (hipStream_t, NULL = null stream). */
int dugks_pool_set_stream(dugks_pool *p, void *stream);
/* Arena bytes a case of this shape takes (two state buffers). */
size_t dugks_pool_case_bytes(int nx, int ny, int precision, int model);
/* Admit a case: parameters as dugks_set_params, initial fields as
 * dugks_init_fields (host [ny][nx] doubles, copied during the call; u, v, p
 * may be NULL), and its number of steps. The initial state is built on the
 * pool's stream. *slot receives the case's slot. EBUSY: no free slot or no
 * room in the arena. EINVAL: bad sizes or parameters. */
int dugks_pool_admit(dugks_pool *p, int nx, int ny, const dugks_params *prm,
                     const double *phi, const double *u, const double *v,
                     const double *pr, long long nsteps, int *slot);
/* Admit an existing handle (the form of the other calls' cases): its
 * parameters and its current state (at its current time) are copied into a
 * new slot, which then runs nsteps steps; the handle itself is left as it
 * is. Waits for the handle's stream. The handle needs a state (ESTATE), the
 * pool's precision and model, and the unit mesh with the central
 * reconstruction (EINVAL); ENUMERIC if its state is non-finite. EBUSY as
 * dugks_pool_admit. */
int dugks_pool_admit_handle(dugks_pool *p, dugks_handle *h, long long nsteps,
                            int *slot);
/* Enqueue nsteps pool steps: every case with steps left advances by
 * min(nsteps, steps left). use_graph: replay a captured HIP graph while the
 * set of running cases does not change; it needs a stream set with
 * dugks_pool_set_stream (the null stream cannot be captured: EINVAL).
 * Asynchronous. A case whose state turns non-finite is not stopped: the
 * caller sees it in dugks_pool_status and retires it. */
int dugks_pool_step(dugks_pool *p, int nsteps, int use_graph);
/* Steps done and steps left of a slot (host bookkeeping, -1 for a free slot). */
long long dugks_pool_steps_done(const dugks_pool *p, int slot);
long long dugks_pool_remaining(const dugks_pool *p, int slot);
/* Cell macros of a slot's current state, as dugks_get_macros (synchronous:
 * waits for the work queued on the pool's stream). ENUMERIC (outputs filled)
 * when the slot's state is non-finite. */
int dugks_pool_get_macros(dugks_pool *p, int slot, double *phi, double *u,
                          double *v, double *pr, double *rho);
/* Free a slot; its arena block is reused once the stream passes this point. */
int dugks_pool_retire(dugks_pool *p, int slot);
/* Free arena bytes (blocks whose retirement the stream has passed). */
size_t dugks_pool_bytes_free(dugks_pool *p);
/* Wait for the pool's stream and read the non-finite flag of every slot
 * (see dugks_pool_status). */
int dugks_pool_sync(dugks_pool *p);
/* Numeric status of a slot as of the last dugks_pool_sync or
 * dugks_pool_get_macros: OK, or ENUMERIC when one of its steps produced a
 * non-finite value (a failed request: only that slot is affected). EINVAL
 * for a free slot. */
int dugks_pool_status(const dugks_pool *p, int slot);
const char *dugks_pool_last_error(const dugks_pool *p);
int dugks_pool_destroy(dugks_pool *p);

#ifdef __cplusplus
}
#endif
#endif /* DUGKS_H */
