/*
 * ppref.c -- float64 CPU reference for the variable-density pressure solve.
 *
 * TEST INFRASTRUCTURE ONLY.  The library never links or calls this file; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code with the HIP path.  Plain C99 + OpenMP, built with
 * -ffp-contract=off so every expression rounds exactly as written.
 *
 * Problem (Kumar & Vanka, arXiv 2104.01636):
 *   Section 2.2, step 11: div(grad(p)/rho) = div(u_f)/dt on the cells;
 *   face coefficient 1/rho_f with rho_f the linear average of the two cells
 *   (Section 2.2, note after the step list): beta_f = 2/(rho_L + rho_R);
 *   Section 4: walls in x and y (no flux through wall faces), periodic in z;
 *   Section 2.1, eq. density_viscosity: rho from the volume fraction.
 * Layout: flat index i + nx*(j + ny*k); face arrays hold the +x/+y/+z face of
 * each cell; the +z face of the last plane joins plane 0.
 *
 * Solver: conjugate gradients on K p = -h^2 (b - mean b), K = -h^2 A (positive
 * semi-definite, kernel = constants), preconditioned by one symmetric V-cycle
 * (damped Jacobi, omega = 0.8, two sweeps before and after; sum restriction,
 * injection prolongation, coarse operators P^T K P; coarsest level by a dense
 * Cholesky factor of K + (mean diag / n) 1 1^T).  The preconditioner only
 * changes how fast the iteration converges: the result is the unique
 * zero-mean solution, accepted by its residual computed with ppref_apply.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IX(i, j, k) ((size_t)(i) + (size_t)nx * ((size_t)(j) + (size_t)ny * (size_t)(k)))

/* ---------------------------------------------------------------- definitions */

void ppref_density_from_fraction(long n, const double* a, double rho_l, double rho_g, double* rho)
{
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) rho[c] = rho_l * (1.0 - a[c]) + rho_g * a[c];
}

void ppref_face_coefficients(int nx, int ny, int nz, const double* rho, double* bx, double* by, double* bz)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        int kp = (k + 1) % nz;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX(i, j, k);
                bx[c] = (i < nx - 1) ? 2.0 / (rho[c] + rho[IX(i + 1, j, k)]) : 0.0;
                by[c] = (j < ny - 1) ? 2.0 / (rho[c] + rho[IX(i, j + 1, k)]) : 0.0;
                bz[c] = 2.0 / (rho[c] + rho[IX(i, j, kp)]);
            }
    }
}

/* (((u_e - u_w) + (v_n - v_s)) + (w_t - w_b)) / (h*dt); wall faces carry zero. */
void ppref_divergence(int nx, int ny, int nz, double h, double dt, const double* u, const double* v,
                      const double* w, double* out)
{
    double hd = h * dt;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        int km = (k + nz - 1) % nz;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX(i, j, k);
                double ue = (i < nx - 1) ? u[c] : 0.0;
                double uw = (i > 0) ? u[IX(i - 1, j, k)] : 0.0;
                double vn = (j < ny - 1) ? v[c] : 0.0;
                double vs = (j > 0) ? v[IX(i, j - 1, k)] : 0.0;
                double wt = w[c];
                double wb = w[IX(i, j, km)];
                out[c] = (((ue - uw) + (vn - vs)) + (wt - wb)) / hd;
            }
    }
}

/* out = A p = div(beta grad p), flux form with face gradients (p_R - p_L)/h. */
void ppref_apply(int nx, int ny, int nz, double h, const double* rho, const double* p, double* out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        int km = (k + nz - 1) % nz, kp = (k + 1) % nz;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX(i, j, k);
                double fe = 0.0, fw = 0.0, fn = 0.0, fs = 0.0, ft, fb;
                if (i < nx - 1) {
                    size_t e = IX(i + 1, j, k);
                    fe = (2.0 / (rho[c] + rho[e])) * ((p[e] - p[c]) / h);
                }
                if (i > 0) {
                    size_t wv = IX(i - 1, j, k);
                    fw = (2.0 / (rho[wv] + rho[c])) * ((p[c] - p[wv]) / h);
                }
                if (j < ny - 1) {
                    size_t n = IX(i, j + 1, k);
                    fn = (2.0 / (rho[c] + rho[n])) * ((p[n] - p[c]) / h);
                }
                if (j > 0) {
                    size_t s = IX(i, j - 1, k);
                    fs = (2.0 / (rho[s] + rho[c])) * ((p[c] - p[s]) / h);
                }
                {
                    size_t t = IX(i, j, kp), b = IX(i, j, km);
                    ft = (2.0 / (rho[c] + rho[t])) * ((p[t] - p[c]) / h);
                    fb = (2.0 / (rho[b] + rho[c])) * ((p[c] - p[b]) / h);
                }
                out[c] = (((fe - fw) + (fn - fs)) + (ft - fb)) / h;
            }
    }
}

static double mean_of(long n, const double* x)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long c = 0; c < n; ++c) s += x[c];
    return s / (double)n;
}

/* ||bbar - A p|| / ||bbar||, bbar = b - mean(b); scratch is n doubles. */
double ppref_rel_residual(int nx, int ny, int nz, double h, const double* rho, const double* b,
                          const double* p, double* scratch)
{
    long n = (long)nx * ny * nz;
    double mb = mean_of(n, b);
    ppref_apply(nx, ny, nz, h, rho, p, scratch);
    double rr = 0.0, bb = 0.0;
#pragma omp parallel for reduction(+ : rr, bb) schedule(static)
    for (long c = 0; c < n; ++c) {
        double bc = b[c] - mb;
        double r = bc - scratch[c];
        rr += r * r;
        bb += bc * bc;
    }
    return sqrt(rr) / sqrt(bb);
}

/* ---------------------------------------------------------------- multigrid */

typedef struct {
    int nx, ny, nz;
    long n;
    double *wx, *wy, *wz, *d; /* face weights and diagonal of K on this level */
    double *x, *f, *r;        /* correction, right-hand side, residual */
    double* chol;             /* coarsest only: dense Cholesky factor (n x n, lower) */
} level_t;

#define MAXLEV 24
#define DENSE_MAX 1024

typedef struct {
    int nlev;
    level_t L[MAXLEV];
    int nu;       /* sweeps before and after */
    double omega; /* Jacobi damping */
} mg_t;

static void k_apply(const level_t* L, const double* x, double* y)
{
    int nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        int km = (k + nz - 1) % nz, kp = (k + 1) % nz;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX(i, j, k);
                double s = 0.0;
                if (i > 0) s += L->wx[IX(i - 1, j, k)] * x[IX(i - 1, j, k)];
                if (i < nx - 1) s += L->wx[c] * x[IX(i + 1, j, k)];
                if (j > 0) s += L->wy[IX(i, j - 1, k)] * x[IX(i, j - 1, k)];
                if (j < ny - 1) s += L->wy[c] * x[IX(i, j + 1, k)];
                s += L->wz[IX(i, j, km)] * x[IX(i, j, km)];
                s += L->wz[c] * x[IX(i, j, kp)];
                y[c] = L->d[c] * x[c] - s;
            }
    }
}

static void make_diag(level_t* L)
{
    int nx = L->nx, ny = L->ny, nz = L->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        int km = (k + nz - 1) % nz;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX(i, j, k);
                double d = L->wx[c] + L->wy[c] + L->wz[c] + L->wz[IX(i, j, km)];
                if (i > 0) d += L->wx[IX(i - 1, j, k)];
                if (j > 0) d += L->wy[IX(i, j - 1, k)];
                L->d[c] = d;
            }
    }
}

static int level_alloc(level_t* L, int nx, int ny, int nz)
{
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->n = (long)nx * ny * nz;
    size_t b = (size_t)L->n * sizeof(double);
    L->wx = malloc(b); L->wy = malloc(b); L->wz = malloc(b); L->d = malloc(b);
    L->x = malloc(b); L->f = malloc(b); L->r = malloc(b);
    L->chol = NULL;
    return L->wx && L->wy && L->wz && L->d && L->x && L->f && L->r;
}

static void level_free(level_t* L)
{
    free(L->wx); free(L->wy); free(L->wz); free(L->d);
    free(L->x); free(L->f); free(L->r); free(L->chol);
}

/* coarse face weight = sum of the 4 fine faces forming it (K_c = P^T K P) */
static void coarsen(const level_t* F, level_t* C)
{
    int nx = F->nx, ny = F->ny;
    int cnx = C->nx, cny = C->ny, cnz = C->nz;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < cnz; ++K)
        for (int J = 0; J < cny; ++J)
            for (int I = 0; I < cnx; ++I) {
                size_t cc = (size_t)I + (size_t)cnx * ((size_t)J + (size_t)cny * K);
                double sx = 0.0, sy = 0.0, sz = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        sx += F->wx[IX(2 * I + 1, 2 * J + a, 2 * K + b)];
                        sy += F->wy[IX(2 * I + a, 2 * J + 1, 2 * K + b)];
                        sz += F->wz[IX(2 * I + a, 2 * J + b, 2 * K + 1)];
                    }
                C->wx[cc] = sx; C->wy[cc] = sy; C->wz[cc] = sz;
            }
}

static int dense_factor(level_t* L)
{
    long n = L->n;
    double* M = calloc((size_t)n * n, sizeof(double));
    double* e = calloc((size_t)n, sizeof(double));
    double* col = calloc((size_t)n, sizeof(double));
    if (!M || !e || !col) { free(M); free(e); free(col); return 0; }
    double dm = mean_of(n, L->d);
    for (long c = 0; c < n; ++c) {
        e[c] = 1.0;
        k_apply(L, e, col);
        e[c] = 0.0;
        for (long r = 0; r < n; ++r) M[r * n + c] = col[r] + dm / (double)n;
    }
    /* Cholesky, lower triangle in place */
    for (long j = 0; j < n; ++j) {
        double s = M[j * n + j];
        for (long k = 0; k < j; ++k) s -= M[j * n + k] * M[j * n + k];
        if (!(s > 0.0)) { free(M); free(e); free(col); return 0; }
        double ljj = sqrt(s);
        M[j * n + j] = ljj;
        for (long i = j + 1; i < n; ++i) {
            double t = M[i * n + j];
            for (long k = 0; k < j; ++k) t -= M[i * n + k] * M[j * n + k];
            M[i * n + j] = t / ljj;
        }
    }
    free(e); free(col);
    L->chol = M;
    return 1;
}

static void dense_solve(const level_t* L, const double* f, double* x)
{
    long n = L->n;
    const double* M = L->chol;
    for (long i = 0; i < n; ++i) {
        double s = f[i];
        for (long k = 0; k < i; ++k) s -= M[i * n + k] * x[k];
        x[i] = s / M[i * n + i];
    }
    for (long i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (long k = i + 1; k < n; ++k) s -= M[k * n + i] * x[k];
        x[i] = s / M[i * n + i];
    }
}

static void jacobi(const level_t* L, double* x, const double* f, double* tmp, int sweeps, double omega,
                   int zero_start)
{
    long n = L->n;
    for (int s = 0; s < sweeps; ++s) {
        if (zero_start && s == 0) {
#pragma omp parallel for schedule(static)
            for (long c = 0; c < n; ++c) x[c] = omega * f[c] / L->d[c];
            continue;
        }
        k_apply(L, x, tmp);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; ++c) x[c] += omega * (f[c] - tmp[c]) / L->d[c];
    }
}

static void vcycle(mg_t* mg, int l)
{
    level_t* L = &mg->L[l];
    int nx = L->nx, ny = L->ny;
    if (l == mg->nlev - 1) {
        if (L->chol) {
            dense_solve(L, L->f, L->x);
        } else {
            jacobi(L, L->x, L->f, L->r, 40, mg->omega, 1);
            jacobi(L, L->x, L->f, L->r, 40, mg->omega, 0);
        }
        return;
    }
    level_t* C = &mg->L[l + 1];
    jacobi(L, L->x, L->f, L->r, mg->nu, mg->omega, 1);
    k_apply(L, L->x, L->r);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < L->n; ++c) L->r[c] = L->f[c] - L->r[c];
    int cnx = C->nx, cny = C->ny, cnz = C->nz;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < cnz; ++K)
        for (int J = 0; J < cny; ++J)
            for (int I = 0; I < cnx; ++I) {
                double s = 0.0;
                for (int c2 = 0; c2 < 2; ++c2)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) s += L->r[IX(2 * I + a, 2 * J + b, 2 * K + c2)];
                C->f[(size_t)I + (size_t)cnx * ((size_t)J + (size_t)cny * K)] = s;
            }
    vcycle(mg, l + 1);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                L->x[IX(i, j, k)] += C->x[(size_t)(i / 2) + (size_t)cnx * ((size_t)(j / 2) + (size_t)cny * (k / 2))];
    jacobi(L, L->x, L->f, L->r, mg->nu, mg->omega, 0);
}

static void mg_free(mg_t* mg)
{
    for (int l = 0; l < mg->nlev; ++l) level_free(&mg->L[l]);
    mg->nlev = 0;
}

static int mg_build(mg_t* mg, int nx, int ny, int nz, const double* rho)
{
    memset(mg, 0, sizeof(*mg));
    mg->nu = 2;
    mg->omega = 0.8;
    if (!level_alloc(&mg->L[0], nx, ny, nz)) return 0;
    mg->nlev = 1;
    ppref_face_coefficients(nx, ny, nz, rho, mg->L[0].wx, mg->L[0].wy, mg->L[0].wz);
    make_diag(&mg->L[0]);
    while (mg->nlev < MAXLEV) {
        level_t* F = &mg->L[mg->nlev - 1];
        if (F->n <= 512 || (F->nx & 1) || (F->ny & 1) || (F->nz & 1)) break;
        level_t* C = &mg->L[mg->nlev];
        if (!level_alloc(C, F->nx / 2, F->ny / 2, F->nz / 2)) return 0;
        mg->nlev++;
        coarsen(F, C);
        make_diag(C);
    }
    level_t* B = &mg->L[mg->nlev - 1];
    if (B->n <= DENSE_MAX && !dense_factor(B)) return 0;
    return 1;
}

/*
 * Solve A p = b - mean(b), mean(p) = 0.  p holds the initial guess on entry
 * and the solution on return.  Returns the number of PCG iterations, or -1 on
 * allocation failure.  *relres = ||bbar - A p|| / ||bbar|| by ppref_apply.
 */
int ppref_solve(int nx, int ny, int nz, double h, const double* rho, const double* b, double* p,
                double tol, int maxit, double* relres)
{
    long n = (long)nx * ny * nz;
    mg_t mg;
    if (!mg_build(&mg, nx, ny, nz, rho)) { mg_free(&mg); return -1; }
    size_t bytes = (size_t)n * sizeof(double);
    double *f = malloc(bytes), *r = malloc(bytes), *z = malloc(bytes), *d = malloc(bytes), *q = malloc(bytes);
    if (!f || !r || !z || !d || !q) {
        free(f); free(r); free(z); free(d); free(q); mg_free(&mg);
        return -1;
    }
    level_t* L0 = &mg.L[0];
    double mb = mean_of(n, b);
    double h2 = h * h;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) f[c] = -h2 * (b[c] - mb);
    double fn = 0.0;
#pragma omp parallel for reduction(+ : fn) schedule(static)
    for (long c = 0; c < n; ++c) fn += f[c] * f[c];
    fn = sqrt(fn);
    double mp = mean_of(n, p);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) p[c] -= mp;
    int it = 0;
    if (fn == 0.0) {
        memset(p, 0, bytes);
        *relres = 0.0;
        goto done;
    }
    for (;;) { /* restart loop: recompute the true residual */
        k_apply(L0, p, q);
        double rn = 0.0;
#pragma omp parallel for reduction(+ : rn) schedule(static)
        for (long c = 0; c < n; ++c) { r[c] = f[c] - q[c]; rn += r[c] * r[c]; }
        if (sqrt(rn) <= tol * fn || it >= maxit) break;
        double rz_old = 0.0;
        int inner = 0;
        while (it < maxit) {
            memcpy(L0->f, r, bytes);
            vcycle(&mg, 0);
            double mz = mean_of(n, L0->x);
            double rz = 0.0;
#pragma omp parallel for reduction(+ : rz) schedule(static)
            for (long c = 0; c < n; ++c) { z[c] = L0->x[c] - mz; rz += r[c] * z[c]; }
            if (inner) {
                double beta = rz / rz_old;
#pragma omp parallel for schedule(static)
                for (long c = 0; c < n; ++c) d[c] = z[c] + beta * d[c];
            } else { /* first direction of a (re)start: d = z (d holds no earlier direction) */
#pragma omp parallel for schedule(static)
                for (long c = 0; c < n; ++c) d[c] = z[c];
            }
            k_apply(L0, d, q);
            double dq = 0.0;
#pragma omp parallel for reduction(+ : dq) schedule(static)
            for (long c = 0; c < n; ++c) dq += d[c] * q[c];
            double alpha = rz / dq;
            rn = 0.0;
#pragma omp parallel for reduction(+ : rn) schedule(static)
            for (long c = 0; c < n; ++c) {
                p[c] += alpha * d[c];
                r[c] -= alpha * q[c];
                rn += r[c] * r[c];
            }
            rz_old = rz;
            ++it;
            ++inner;
            if (sqrt(rn) <= tol * fn) break;
        }
        if (it >= maxit) break;
    }
    mp = mean_of(n, p);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) p[c] -= mp;
    *relres = ppref_rel_residual(nx, ny, nz, h, rho, b, p, q);
done:
    free(f); free(r); free(z); free(d); free(q);
    mg_free(&mg);
    return it;
}

int ppref_num_threads(void)
{
    return omp_get_max_threads();
}
