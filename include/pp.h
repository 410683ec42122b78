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
 * pp_set_density: the discrete div(beta grad x) of step 11. */
int pp_apply(pp_handle h, const double* x, double* y);

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
