/*
 * pp.h -- C ABI of the MI355X variable-density pressure-Poisson solver.
 *
 * The library solves the pressure equation of a fractional-step two-phase
 * flow solver (Kumar & Vanka, arXiv 2104.01636, Section 2.2, step 11):
 *
 *     div( grad(p) / rho ) = div(u_f) / dt
 *
 * on a uniform grid of nx * ny * nz cubic cells of edge h, with no-penetration
 * walls in x and y and periodicity in z (Section 4).  The face coefficient is
 * 1/rho_f with rho_f the linear average of the two neighbouring cells (Section
 * 2.2, the note after the step list): beta_f = 2 / (rho_L + rho_R).  The
 * discrete operator is singular (the constants are its kernel), so the library
 * solves A p = b - mean(b) and returns the zero-mean solution.
 *
 * Conventions for every entry point
 *   - Arrays are float64, contiguous, laid out with flat index
 *     i + nx*(j + ny*k) (x fastest, z = periodic direction slowest).
 *   - "device" pointers point to memory of the GPU the handle was created on;
 *     the caller owns them.  The library never keeps a caller pointer past the
 *     call that receives it.
 *   - Work is ordered on the HIP stream given at creation (NULL = the null
 *     stream).  Calls that return a result to the host synchronise that stream.
 *   - Return value: PP_OK (0) or a negative pp_status; no exception crosses
 *     the boundary.  pp_last_error() returns a message for the last failure.
 *   - A handle is not re-entrant; distinct handles are independent and may be
 *     used from different host threads.
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_handle_s* pp_handle;

typedef enum {
    PP_OK = 0,
    PP_ERR_INVALID = -1,       /* bad argument: sizes, tolerance, null pointer */
    PP_ERR_OOM = -2,           /* device allocation failed */
    PP_ERR_NOT_CONVERGED = -3, /* max_iters reached; p holds the last iterate */
    PP_ERR_HIP = -4,           /* a HIP runtime call failed */
    PP_ERR_NONFINITE = -5,     /* rho not finite or not > 0, or rhs not finite */
    PP_ERR_STATE = -6          /* pp_solve before pp_set_density */
} pp_status;

typedef enum {
    PP_FP64 = 0,        /* every kernel in float64 */
    PP_FP32_REFINED = 1 /* float64 flexible CG (x, r, d, q, the operator and the dots in float64)
                           preconditioned by a float32 multigrid cycle on a float32 copy of r */
} pp_mode;

typedef struct {
    int nx, ny, nz;    /* cells; nx, ny >= 2, nz >= 2 and even (red-black colouring across the periodic seam) */
    double h;          /* cell edge (> 0) */
    int mode;          /* pp_mode */
    double tol;        /* relative residual ||bbar - A p||_2 / ||bbar||_2 to reach (> 0) */
    int max_iters;     /* flexible-CG iterations over all passes; <= 0 selects 1000 */
    int pre_sweeps;    /* red-black Gauss-Seidel sweeps on the finest level; <= 0 selects 1 */
    int post_sweeps;   /* sweeps on level 1 (and, in the multigrid-solver form, on every coarse
                          level); <= 0 selects 2 */
    int flags;         /* PP_FLAG_* bits, 0 for the default solver */
    double omega;      /* SOR factor of the red-black smoother, in [0, 2); <= 0 selects 1 (Gauss-Seidel) */
} pp_config;

/* flags: run multigrid cycles as the solver, x += M (bbar - A x), instead of
 * using them to precondition conjugate gradients -- the paper's own form
 * (red-black SOR relaxation accelerated by multigrid, Section 2.1).  Float64
 * mode only. */
#define PP_FLAG_MG_SOLVER 1
/* flags, with PP_FLAG_MG_SOLVER only: W-cycles instead of V-cycles -- every coarse
 * level (down to the single-launch small-level cycle) is visited twice per visit
 * of the level above, the second time on the residual the first left, e += M (f -
 * K e), and each coarse correction is added once (no over-correction). */
#define PP_FLAG_W_CYCLE 2

typedef struct {
    int iters;              /* flexible-CG iterations over all passes (multigrid-solver form: cycles) */
    int outer_iters;        /* passes started from a freshly computed float64 residual f - A x (1 when
                               the first pass meets the tolerance; 0 when the guess already does) */
    int inner_iters_total;  /* float32 multigrid cycles applied (refined mode; 0 in float64 mode) */
    double rel_residual;    /* ||bbar - A p|| / ||bbar|| in float64 at return (library's own operator) */
    double setup_ms;        /* last pp_set_density, device time */
    double solve_ms;        /* this pp_solve, host wall time */
    size_t device_bytes;    /* device memory held by the handle */
} pp_stats;

/* Device bytes pp_create would allocate for cfg (host only, no GPU needed).
 * Returns 0 for an invalid configuration. */
size_t pp_footprint_bytes(const pp_config* cfg);

/* Create a solver for cfg on the current device, ordered on hip_stream
 * (a hipStream_t, may be NULL).  Allocates the multigrid hierarchy and all
 * workspaces.  *out is set to NULL on failure. */
int pp_create(const pp_config* cfg, void* hip_stream, pp_handle* out);

/* Give the cell densities rho (device, N values, each finite and > 0).  Builds
 * the face coefficients (beta_f = 2/(rho_L + rho_R), zero on walls, periodic in
 * z) and the coarse levels.  rho is copied; the caller may free it afterwards. */
int pp_set_density(pp_handle h, const double* rho);

/* Solve A p = rhs - mean(rhs).  rhs (device, N values) is not modified.
 * p (device, N values) holds the initial guess on entry and the zero-mean
 * solution on return.  st may be NULL.  On PP_ERR_NOT_CONVERGED p holds the
 * last iterate and st is filled. */
int pp_solve(pp_handle h, const double* rhs, double* p, pp_stats* st);

/* y = A x (device, N values each) with the density of the last
 * pp_set_density: the discrete div(beta grad x) of step 11, computed by the
 * same plane-marching kernel, tiles and float64 face coefficients (formed from
 * the density) as the solve's own operator passes. */
int pp_apply(pp_handle h, const double* x, double* y);

/* The two legs of the multigrid cycle on the finest level (red-black SOR
 * relaxation accelerated by multigrid, Section 2.1), run by exactly the
 * kernels the preconditioner uses there, on caller arrays.  They work on the
 * scaled equation K x = f with K = -h^2 A (positive semi-definite: (K x)_c =
 * D_c x_c - sum_f beta_f x_nb(f), D_c = sum_f beta_f).  Arrays are in the
 * preconditioner's precision: float64 for a PP_FP64 handle, float32 for
 * PP_FP32_REFINED.  f, x, z hold N values; rc and e hold the N/8 values of the
 * first coarse level (nx/2 x ny/2 x nz/2, same layout).  The grid must coarsen
 * (nx, ny even, nz divisible by 4, N > 64), else PP_ERR_INVALID; before
 * pp_set_density, PP_ERR_STATE.  Both return after the work is done.
 *
 * pp_presmooth_restrict: x = the pre-smoothing from a zero guess (pre_sweeps
 * red-black sweeps, red first), rc = the residual f - K x summed over the 8
 * children of each coarse cell. */
int pp_presmooth_restrict(pp_handle h, const void* f, void* x, void* rc);

/* pp_prolong_postsmooth: z = x + wc * (P e) with P the injection (each fine
 * cell takes its parent's value), followed by pre_sweeps red-black sweeps of
 * K z = f, black first.  With q (float64 device array of N values, may be
 * NULL) also dots[0] = sum(z) and dots[1] = <z, q> (host array of 2, float64
 * accumulation in a fixed order), the two reductions the Krylov step takes from
 * this pass. */
int pp_prolong_postsmooth(pp_handle h, const void* f, const void* x, const void* e, double wc, void* z, const double* q,
                          double* dots);

/* Release everything the handle holds.  NULL is accepted. */
int pp_destroy(pp_handle h);

/* Message of the last failure on h, or of the last failure of a handle-less
 * call on this thread when h is NULL.  Never NULL. */
const char* pp_last_error(pp_handle h);

/* Mixture density from the gas volume fraction a (Section 2.1,
 * eq. density_viscosity, with the liquid fraction written as 1 - a):
 * rho[c] = rho_l * (1 - a[c]) + rho_g * a[c], rounded exactly as written.
 * a and rho are device arrays of n values; may alias.  hip_stream may be NULL. */
int pp_density_from_fraction(const double* a, double rho_l, double rho_g, double* rho, size_t n, void* hip_stream);

/* Right-hand side of step 11: out = div(u_f) / dt per cell,
 * (((u_e - u_w) + (v_n - v_s)) + (w_t - w_b)) / (h*dt).
 * u, v, w (device, N values each) hold the +x / +y / +z face velocity of every
 * cell; the +x face of i = nx-1 and the +y face of j = ny-1 are walls and their
 * entries are ignored (taken as zero), as are the faces at i = -1/2 and
 * j = -1/2.  The +z face of the last plane joins plane 0. */
int pp_divergence(int nx, int ny, int nz, double h, double dt, const double* u, const double* v, const double* w,
                  double* out, void* hip_stream);

/* Projection of the face velocities (step 12 of Section 2.2, on faces), in
 * place: u_f -= dt * beta_f * (p_R - p_L) / h for every face, beta_f from rho;
 * the wall entries (i = nx-1 of u, j = ny-1 of v) are set to zero.  With p
 * from pp_solve for rhs = div(u)/dt, div(u_new) = dt * (residual of the
 * solve).  rho, p, u, v, w: device, N values each. */
int pp_project(int nx, int ny, int nz, double h, double dt, const double* rho, const double* p, double* u, double* v,
               double* w, void* hip_stream);

/* Step 12 of Section 2.2 in one pass, in place, after the solve:
 *   face velocities  u_f -= dt * beta_f * (p_R - p_L) / h        (as pp_project;
 *                    wall entries i = nx-1 of u and j = ny-1 of v set to zero),
 *   cell velocities  u_c -= dt * (grad p / rho + grad pt / rho)_{f->c},
 * where the face term beta_f ((p_R - p_L) + (pt_R - pt_L)) / h (beta_f =
 * 2/(rho_L + rho_R), zero on the walls, each pressure's term rounded on its own
 * and then added) is averaged to the cell centre from the two faces bounding it
 * along each axis: (g_west + g_east)/2 for uc, likewise vc and wc (the
 * face-to-cell counterpart of the linear averaging in the note after the step
 * list).  pt, the surface-tension pressure of step 6, may be NULL (no
 * surface-tension term).  u, v, w hold the +x/+y/+z face of every cell; uc, vc,
 * wc the cell-centred components.  Device arrays of N values; the call returns
 * after the work on hip_stream (may be NULL) is done. */
int pp_correct_velocity(int nx, int ny, int nz, double h, double dt, const double* rho, const double* p, const double* pt,
                        double* u, double* v, double* w, double* uc, double* vc, double* wc, void* hip_stream);

/* Right-hand side of the surface-tension pressure equation (Section 2.1,
 * eq. ppe_surface_tension with the interface force of eq. jump_condition as
 * its source, applied at faces): out = div(beta f) with the face force
 * f = sigma * (kappa_L + kappa_R)/2 * (a_R - a_L) / h, a the gas fraction and
 * kappa the cell curvature (positive for a bubble).  Solving A p = out with
 * pp_solve gives the pressure that balances f (higher inside the gas); for a
 * constant curvature it is sigma * kappa * (a - mean a).  Device arrays of N
 * values; wall faces carry no force. */
int pp_surface_tension_rhs(int nx, int ny, int nz, double h, double sigma, const double* rho, const double* alpha,
                           const double* kappa, double* out, void* hip_stream);

/* Relative residual of a pressure field on the device:
 *     *rel_out = ||bbar - A p||_2 / ||bbar||_2,   bbar = rhs - mean(rhs),
 * with A the operator of step 11 (face coefficients 2/(rho_L + rho_R), walls
 * in x and y, periodic in z) -- the acceptance measure of a solve, taken on the
 * GPU from the density alone, float64 throughout, sums in a fixed order (bitwise
 * repeatable).  0 when bbar and the residual are both zero, +inf when only bbar
 * is.  rho, rhs, p: device arrays of N values; rel_out: host double.  The
 * call allocates (and frees) a small device buffer for its partial sums, and
 * returns after the work on hip_stream (may be NULL) is done.  Errors:
 * PP_ERR_INVALID (sizes, h <= 0, null pointers, more than 4096 tiles of 64 x 8
 * cells per plane), PP_ERR_NONFINITE (rho not finite or not > 0, rhs not
 * finite), PP_ERR_OOM. */
int pp_rel_residual(int nx, int ny, int nz, double h, const double* rho, const double* rhs, const double* p, double* rel_out,
                    void* hip_stream);

/* pp_rel_residual without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels, result and errors.  Its
 * partial sums live in a fixed static device array of 131136 bytes per GPU
 * (held until the process ends); grids needing more partial sums than it holds
 * (more than 4096 tiles of 64 x 8 cells per plane) are rejected with
 * PP_ERR_INVALID.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (different host threads or streams) race and must be serialised
 * by the caller.  Call it with the device of hip_stream current. */
int pp_rel_residual_noalloc(int nx, int ny, int nz, double h, const double* rho, const double* rhs, const double* p,
                            double* rel_out, void* hip_stream);

/* Device time of the finest-level kernels, measured with HIP events on the
 * handle's stream around each launch.
 *   mode = 1: clear the counters and start timing;
 *   mode = -1: stop timing;
 *   mode = 0: copy up to max_entries entries into out (one per kernel and
 *             precision that ran) and return how many were written.
 * bytes is the algorithmic traffic of all timed launches: every array element
 * the kernel must read or write counted once (neighbour reuse free). */
typedef struct {
    char name[40];
    double total_ms;
    long long launches;
    double bytes;
} pp_kernel_time;
int pp_kernel_timing(pp_handle h, int mode, pp_kernel_time* out, int max_entries);

/* Library version string. */
const char* pp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PP_H */
