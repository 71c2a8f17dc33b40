/*
 * stp_oracle.c -- plain, slow FP64 CPU oracle of the S-TPLS time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this file.  It shares no
 * code, header or table with the HIP library; the two meet only through
 * seeded inputs.
 *
 * What it computes (Fannon et al., "Simplified TPLS as a learning tool for
 * high-performance computational fluid dynamics", arXiv 1511.07800):
 *   - incompressible Navier-Stokes in a channel, periodic in x and y,
 *     no-slip walls at z = 0 and z = lz, driven by a constant mean pressure
 *     gradient G = dp/dx (Sec. 2.1, eqs. for the non-dimensional NS system);
 *   - optional Smagorinsky eddy viscosity with Van Driest damping
 *     (Sec. 2.2, definitions of nu_t, Delta and phi_w);
 *   - MAC staggered finite volumes, centred differences (Sec. 3.1, 3.2);
 *   - projection: predictor u*, Poisson problem for p, correction
 *     (Sec. 3.1, eqs. for u*, the Poisson equation and the correction);
 *   - viscous split: the "convective-like" part d_j(nu_T d_i u_j) and the
 *     convection with third-order Adams-Bashforth, the "diffusive" part
 *     d_j(nu_T d_j u_i) with Crank-Nicolson (Sec. 3.1);
 *   - the Poisson problem solved with Scheduled Relaxation Jacobi: Jacobi
 *     with over-relaxation, a cycle of M sweeps with prescribed weights
 *     omega_k, repeated until convergence (Sec. 3.4, Jacobi-SOR equation).
 *
 * Layout: every field is a flat array with x fastest,
 *   idx(i,j,k) = i + nx*(j + ny*k).
 * u (x-faces, at x = i dx), v (y-faces, at y = j dy): nx*ny*nz values.
 * w (z-faces, at z = k dz, k = 0..nz): nx*ny*(nz+1) values; planes k = 0 and
 * k = nz are the walls and hold 0.  p and nu_T sit at cell centres.
 *
 * Readings of points the paper leaves open (each also listed with the
 * design notes):
 *   - wall ghosts: u and v odd about the wall (no slip), p even (zero normal
 *     gradient, matching w* = 0 on the wall faces);
 *   - Jacobi diagonal: one scalar D = 2/dx^2 + 2/dy^2 + 2/dz^2 for every
 *     cell, wall cells included, so the sweep is weighted Richardson;
 *   - convection in divergence form with arithmetic interpolation;
 *   - nu_T frozen at time level n for both Crank-Nicolson halves;
 *   - Adams-Bashforth start-up: first order, then second, then third;
 *   - edge viscosity: mean of the four surrounding centres, nu on wall edges;
 *   - |S| at centres: diagonal strains at the centre, squared off-diagonal
 *     strains averaged over the four surrounding edges;
 *   - Crank-Nicolson system solved by a stationary iteration to round-off;
 *   - Poisson stop test ||b - L p||_2 <= rtol ||b||_2, checked before the
 *     first cycle and after every full cycle; rtol = 0 runs maxit cycles.
 *
 * Arithmetic: FP64 throughout, built with -O2 -ffp-contract=off.  The loops
 * over z-planes of the stencils (Laplacian, sweep, divergence, correction,
 * eddy viscosity, viscous and explicit terms) may run on OpenMP threads:
 * every value is computed by the same expression as in a serial run, and
 * every reduction (sums, maxima, norms) is a serial loop.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;   /* cells */
    int32_t les;          /* 0: nu_T = nu; 1: Smagorinsky + Van Driest */
    double lx, ly, lz;    /* domain lengths; walls at z = 0 and z = lz */
    double nu;            /* molecular kinematic viscosity */
    double dpdx;          /* G: constant mean pressure gradient */
    double dt;
    double cs;            /* Smagorinsky coefficient C_S */
    double vd_a;          /* Van Driest constant A */
} or_params;

typedef struct {
    int32_t poisson_cycles;
    int32_t cn_sweeps;
    int32_t status;        /* 0 ok, -4 not converged, -5 non-finite */
    int32_t pad;
    double relres0;        /* ||b - L p0|| / ||b|| before the solve */
    double relres;         /* after the solve */
    double bnorm;
    double max_div;        /* max |div u^{n+1}| */
    double u_bulk;         /* mean of u over all x-faces */
    double u_max;          /* max |u| */
    double cfl;            /* max(|u| dt/dx, |v| dt/dy, |w| dt/dz) */
    double u_centre;       /* mean u on the centreline */
    double nut_max;
} or_stats;

/* ---------------------------------------------------------------- grid -- */

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static size_t ix(const or_params* P, int i, int j, int k)
{
    return (size_t)wrap(i, P->nx) + (size_t)P->nx * ((size_t)wrap(j, P->ny) + (size_t)P->ny * (size_t)k);
}

static double hx(const or_params* P) { return P->lx / P->nx; }
static double hy(const or_params* P) { return P->ly / P->ny; }
static double hz(const or_params* P) { return P->lz / P->nz; }

size_t or_ncell(const or_params* P) { return (size_t)P->nx * P->ny * P->nz; }
size_t or_nwface(const or_params* P) { return (size_t)P->nx * P->ny * (P->nz + 1); }

/* velocity accessors with the wall conditions applied:
 * u, v at plane k outside 0..nz-1 are the odd ghosts of the adjacent plane;
 * w at planes 0 and nz is zero. */
static double U(const or_params* P, const double* u, int i, int j, int k)
{
    if (k < 0) return -u[ix(P, i, j, 0)];
    if (k >= P->nz) return -u[ix(P, i, j, P->nz - 1)];
    return u[ix(P, i, j, k)];
}
static double W(const or_params* P, const double* w, int i, int j, int k)
{
    if (k <= 0 || k >= P->nz) return 0.0;
    return w[ix(P, i, j, k)];
}

/* ------------------------------------------------------ Poisson problem -- */

/* L_p p: the discrete Laplacian div(grad p) at cell centres, periodic in x
 * and y, zero normal gradient at the walls (Sec. 3.1, Poisson equation).
 * Planes are independent, so they are spread over OpenMP threads. */
void or_lap_p(const or_params* P, const double* p, double* out)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P);
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const size_t plane = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
            const double* row = p + k * plane + (size_t)j * nx;
            const double* rowm = p + k * plane + (size_t)jm * nx;
            const double* rowp = p + k * plane + (size_t)jp * nx;
            for (int i = 0; i < nx; ++i) {
                const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
                const double c = row[i];
                double s = (row[ip] - c) / (dx * dx) + (row[im] - c) / (dx * dx)
                         + (rowp[i] - c) / (dy * dy) + (rowm[i] - c) / (dy * dy);
                if (k + 1 < nz) s += (row[i + plane] - c) / (dz * dz);
                if (k > 0) s += (row[i - plane] - c) / (dz * dz);
                out[k * plane + (size_t)j * nx + i] = s;
            }
        }
}

double or_diag_d(const or_params* P)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P);
    return 2.0 / (dx * dx) + 2.0 / (dy * dy) + 2.0 / (dz * dz);
}

/* One Jacobi-SOR sweep with weight omega (Sec. 3.4): the Jacobi value
 * p_J = p + (L_p p - b)/D blended as (1 - omega) p + omega p_J, evaluated in
 * the equivalent increment form p + omega (p_J - p) so that large weights
 * do not cancel two large terms.  Not in place; lap is scratch of n values. */
static void srj_sweep_into(const or_params* P, double omega, const double* p, const double* b, double* out,
                           double* lap)
{
    const size_t n = or_ncell(P);
    const double D = or_diag_d(P);
    or_lap_p(P, p, lap);
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; ++c) {
        const double jac_increment = (lap[c] - b[c]) / D;     /* p_J - p */
        out[c] = p[c] + omega * jac_increment;
    }
}

void or_srj_sweep(const or_params* P, double omega, const double* p, const double* b, double* out)
{
    double* lap = (double*)malloc(or_ncell(P) * sizeof(double));
    srj_sweep_into(P, omega, p, b, out, lap);
    free(lap);
}

/* The sweep value at a list of cells only (for sampling very large grids):
 * out[q] = p + (omega/D)(L_p p - b) at cell index cells[q]. */
void or_srj_sweep_at(const or_params* P, double omega, const double* p, const double* b, const int64_t* cells,
                     int64_t count, double* out)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P), D = or_diag_d(P);
    const size_t plane = (size_t)P->nx * P->ny;
    for (int64_t q = 0; q < count; ++q) {
        const size_t c = (size_t)cells[q];
        const int k = (int)(c / plane), j = (int)((c % plane) / P->nx), i = (int)(c % P->nx);
        const double pc = p[c];
        double lap = (p[ix(P, i + 1, j, k)] - pc) / (dx * dx) + (p[ix(P, i - 1, j, k)] - pc) / (dx * dx)
                   + (p[ix(P, i, j + 1, k)] - pc) / (dy * dy) + (p[ix(P, i, j - 1, k)] - pc) / (dy * dy);
        if (k + 1 < P->nz) lap += (p[ix(P, i, j, k + 1)] - pc) / (dz * dz);
        if (k > 0) lap += (p[ix(P, i, j, k - 1)] - pc) / (dz * dz);
        out[q] = pc + omega * ((lap - b[c]) / D);
    }
}

/* r = b - L_p p; returns sum r^2. */
double or_residual(const or_params* P, const double* p, const double* b, double* r)
{
    const size_t n = or_ncell(P);
    or_lap_p(P, p, r);
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) {
        r[c] = b[c] - r[c];
        s += r[c] * r[c];
    }
    return s;
}

static double sumsq(const double* a, size_t n)
{
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += a[c] * a[c];
    return s;
}

static double mean(const double* a, size_t n)
{
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += a[c];
    return s / (double)n;
}

/* The m sweeps of one cycle, in order, alternating between p and the
 * scratch q (each sweep reads one array and writes the other); the cycle's
 * result is left in p. */
static void srj_cycle(const or_params* P, const double* omega, int m, double* p, const double* b, double* q,
                      double* lap)
{
    double* cur = p;
    double* nxt = q;
    for (int s = 0; s < m; ++s) {
        srj_sweep_into(P, omega[s], cur, b, nxt, lap);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != p) memcpy(p, cur, or_ncell(P) * sizeof(double));
}

/* p <- the m sweeps omega[0..m-1] applied in order (one cycle, no residual
 * test), with the scratch arrays allocated once for the whole sequence. */
void or_srj_cycle(const or_params* P, const double* omega, int m, double* p, const double* b)
{
    const size_t n = or_ncell(P);
    double* q = (double*)malloc(n * sizeof(double));
    double* lap = (double*)malloc(n * sizeof(double));
    srj_cycle(P, omega, m, p, b, q, lap);
    free(q);
    free(lap);
}

/* Scheduled Relaxation Jacobi (Sec. 3.4): the M-sweep cycle omega[0..m-1]
 * is applied repeatedly; convergence is tested before the first cycle and
 * after each full cycle.  p holds the initial guess on entry and the
 * solution on exit (mean removed).  Returns 0, -4 (maxit cycles reached
 * without convergence) or -5 (non-finite residual). */
int or_poisson_srj(const or_params* P, const double* b, double* p, const double* omega, int m,
                   double rtol, int maxit, int* cycles_out, double* relres0, double* relres)
{
    const size_t n = or_ncell(P);
    double* r = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    double* lap = (double*)malloc(n * sizeof(double));
    const double bn = sqrt(sumsq(b, n));
    const double floor_b = bn > 1e-300 ? bn : 1e-300;
    int status = 0, cycles = 0;
    double rn = sqrt(or_residual(P, p, b, r));
    *relres0 = rn / floor_b;
    /* one cycle: the m sweeps of the schedule, in order */
#define SRJ_CYCLE() srj_cycle(P, omega, m, p, b, q, lap)
    if (rtol > 0.0) {
        while (!(rn <= rtol * floor_b)) {
            if (!isfinite(rn)) { status = -5; break; }
            if (cycles >= maxit) { status = -4; break; }
            SRJ_CYCLE();
            ++cycles;
            rn = sqrt(or_residual(P, p, b, r));
        }
    } else {
        for (cycles = 0; cycles < maxit; ++cycles) { SRJ_CYCLE(); }
        rn = sqrt(or_residual(P, p, b, r));
        if (!isfinite(rn)) status = -5;
    }
#undef SRJ_CYCLE
    const double pm = mean(p, n);
    for (size_t c = 0; c < n; ++c) p[c] -= pm;
    *relres = rn / floor_b;
    *cycles_out = cycles;
    free(r);
    free(q);
    free(lap);
    return status;
}

/* ------------------------------------------------------ div, grad, proj -- */

/* Discrete divergence of a face field at cell centres. */
void or_divergence(const or_params* P, const double* u, const double* v, const double* w, double* out)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i)
                out[ix(P, i, j, k)] = (u[ix(P, i + 1, j, k)] - u[ix(P, i, j, k)]) / dx
                                    + (v[ix(P, i, j + 1, k)] - v[ix(P, i, j, k)]) / dy
                                    + (W(P, w, i, j, k + 1) - W(P, w, i, j, k)) / dz;
}

/* Correction u^{n+1} = u* - dt grad p^{n+1} (Sec. 3.1) on every face; wall
 * w faces stay 0. */
void or_project(const or_params* P, const double* p, double* u, double* v, double* w)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P), dt = P->dt;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                u[ix(P, i, j, k)] -= dt * (p[ix(P, i, j, k)] - p[ix(P, i - 1, j, k)]) / dx;
                v[ix(P, i, j, k)] -= dt * (p[ix(P, i, j, k)] - p[ix(P, i, j - 1, k)]) / dy;
            }
#pragma omp parallel for schedule(static)
    for (int k = 1; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i)
                w[ix(P, i, j, k)] -= dt * (p[ix(P, i, j, k)] - p[ix(P, i, j, k - 1)]) / dz;
}

/* ------------------------------------------------------------ viscosity -- */

/* Van Driest factor phi_w (Sec. 2.2) with p = q = 1: 1 - exp(-z+/A), where
 * z+ is the distance to the nearer wall in wall units, u_tau / nu per unit
 * length, u_tau = sqrt(lz |G| / 2) (the paper's friction-velocity scale). */
static double van_driest(const or_params* P, double z)
{
    const double utau = sqrt(0.5 * P->lz * fabs(P->dpdx));
    const double dwall = z < P->lz - z ? z : P->lz - z;
    return 1.0 - exp(-dwall * utau / P->nu / P->vd_a);
}

/* nu_T = nu + nu_t at cell centres, nu_t = (C_S Delta phi_w)^2 |S|,
 * Delta = 2 (dx dy dz)^(1/3), |S| = sqrt(2 S_ij S_ij) (Sec. 2.2).
 * Returns max nu_T. */
double or_nut(const or_params* P, const double* u, const double* v, const double* w, double* nut)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P);
    const size_t n = or_ncell(P);
    double mx = P->nu;
    if (!P->les) {
        for (size_t c = 0; c < n; ++c) nut[c] = P->nu;
        return P->nu;
    }
    const double delta = 2.0 * cbrt(dx * dy * dz);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                const double s11 = (u[ix(P, i + 1, j, k)] - u[ix(P, i, j, k)]) / dx;
                const double s22 = (v[ix(P, i, j + 1, k)] - v[ix(P, i, j, k)]) / dy;
                const double s33 = (W(P, w, i, j, k + 1) - W(P, w, i, j, k)) / dz;
                /* off-diagonal strains on the four edges around the centre */
                double a12 = 0.0, a13 = 0.0, a23 = 0.0;
                for (int e = 0; e < 4; ++e) {
                    const int di = e & 1, dj = e >> 1;
                    /* x-y edge at (i+di, j+dj): S12 = (du/dy + dv/dx)/2 */
                    const double s12 = 0.5 * ((U(P, u, i + di, j + dj, k) - U(P, u, i + di, j + dj - 1, k)) / dy
                                            + (v[ix(P, i + di, j + dj, k)] - v[ix(P, i + di - 1, j + dj, k)]) / dx);
                    /* x-z edge at (i+di, k+dj): S13 = (du/dz + dw/dx)/2 */
                    const int kk = k + dj;
                    const double s13 = 0.5 * ((U(P, u, i + di, j, kk) - U(P, u, i + di, j, kk - 1)) / dz
                                            + (W(P, w, i + di, j, kk) - W(P, w, i + di - 1, j, kk)) / dx);
                    /* y-z edge at (j+di, k+dj): S23 = (dv/dz + dw/dy)/2 */
                    const double s23 = 0.5 * ((U(P, v, i, j + di, kk) - U(P, v, i, j + di, kk - 1)) / dz
                                            + (W(P, w, i, j + di, kk) - W(P, w, i, j + di - 1, kk)) / dy);
                    a12 += 0.25 * s12 * s12;
                    a13 += 0.25 * s13 * s13;
                    a23 += 0.25 * s23 * s23;
                }
                const double s2 = 2.0 * (s11 * s11 + s22 * s22 + s33 * s33) + 4.0 * (a12 + a13 + a23);
                const double smag = sqrt(s2);
                const double zc = (k + 0.5) * dz;
                const double l = P->cs * delta * van_driest(P, zc);
                const double val = P->nu + l * l * smag;
                nut[ix(P, i, j, k)] = val;
            }
    for (size_t c = 0; c < n; ++c)
        if (nut[c] > mx) mx = nut[c];
    return mx;
}

/* edge viscosities: mean of the four surrounding centres; nu on wall edges */
static double nu_xy(const or_params* P, const double* nut, int i, int j, int k)
{   /* edge at x = i dx, y = j dy, plane k */
    return 0.25 * (nut[ix(P, i - 1, j - 1, k)] + nut[ix(P, i, j - 1, k)] + nut[ix(P, i - 1, j, k)] + nut[ix(P, i, j, k)]);
}
static double nu_xz(const or_params* P, const double* nut, int i, int j, int k)
{   /* edge at x = i dx, z = k dz, row j */
    if (k <= 0 || k >= P->nz) return P->nu;
    return 0.25 * (nut[ix(P, i - 1, j, k - 1)] + nut[ix(P, i, j, k - 1)] + nut[ix(P, i - 1, j, k)] + nut[ix(P, i, j, k)]);
}
static double nu_yz(const or_params* P, const double* nut, int i, int j, int k)
{   /* edge at y = j dy, z = k dz, column i */
    if (k <= 0 || k >= P->nz) return P->nu;
    return 0.25 * (nut[ix(P, i, j - 1, k - 1)] + nut[ix(P, i, j, k - 1)] + nut[ix(P, i, j - 1, k)] + nut[ix(P, i, j, k)]);
}

/* ----------------------------------------------- momentum: the operators -- */

/* Diffusive part L_nu f = d_j(nu_T d_j f) for component c (0 = u, 1 = v,
 * 2 = w), the term treated with Crank-Nicolson (Sec. 3.1).  For w only the
 * interior planes 1..nz-1 are written; wall planes get 0. */
void or_visc_diff(const or_params* P, int c, const double* nut, const double* f, double* out)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P);
    const int nz = P->nz;
    if (c == 0) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < P->ny; ++j)
                for (int i = 0; i < P->nx; ++i) {
                    const double fc = f[ix(P, i, j, k)];
                    const double tx = nut[ix(P, i, j, k)] * (f[ix(P, i + 1, j, k)] - fc)
                                    - nut[ix(P, i - 1, j, k)] * (fc - f[ix(P, i - 1, j, k)]);
                    const double ty = nu_xy(P, nut, i, j + 1, k) * (f[ix(P, i, j + 1, k)] - fc)
                                    - nu_xy(P, nut, i, j, k) * (fc - f[ix(P, i, j - 1, k)]);
                    const double tz = nu_xz(P, nut, i, j, k + 1) * (U(P, f, i, j, k + 1) - fc)
                                    - nu_xz(P, nut, i, j, k) * (fc - U(P, f, i, j, k - 1));
                    out[ix(P, i, j, k)] = tx / (dx * dx) + ty / (dy * dy) + tz / (dz * dz);
                }
    } else if (c == 1) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < P->ny; ++j)
                for (int i = 0; i < P->nx; ++i) {
                    const double fc = f[ix(P, i, j, k)];
                    const double tx = nu_xy(P, nut, i + 1, j, k) * (f[ix(P, i + 1, j, k)] - fc)
                                    - nu_xy(P, nut, i, j, k) * (fc - f[ix(P, i - 1, j, k)]);
                    const double ty = nut[ix(P, i, j, k)] * (f[ix(P, i, j + 1, k)] - fc)
                                    - nut[ix(P, i, j - 1, k)] * (fc - f[ix(P, i, j - 1, k)]);
                    const double tz = nu_yz(P, nut, i, j, k + 1) * (U(P, f, i, j, k + 1) - fc)
                                    - nu_yz(P, nut, i, j, k) * (fc - U(P, f, i, j, k - 1));
                    out[ix(P, i, j, k)] = tx / (dx * dx) + ty / (dy * dy) + tz / (dz * dz);
                }
    } else {
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                out[ix(P, i, j, 0)] = 0.0;
                out[ix(P, i, j, nz)] = 0.0;
            }
#pragma omp parallel for schedule(static)
        for (int k = 1; k < nz; ++k)
            for (int j = 0; j < P->ny; ++j)
                for (int i = 0; i < P->nx; ++i) {
                    const double fc = f[ix(P, i, j, k)];
                    const double tx = nu_xz(P, nut, i + 1, j, k) * (f[ix(P, i + 1, j, k)] - fc)
                                    - nu_xz(P, nut, i, j, k) * (fc - f[ix(P, i - 1, j, k)]);
                    const double ty = nu_yz(P, nut, i, j + 1, k) * (f[ix(P, i, j + 1, k)] - fc)
                                    - nu_yz(P, nut, i, j, k) * (fc - f[ix(P, i, j - 1, k)]);
                    const double tz = nut[ix(P, i, j, k)] * (W(P, f, i, j, k + 1) - fc)
                                    - nut[ix(P, i, j, k - 1)] * (fc - W(P, f, i, j, k - 1));
                    out[ix(P, i, j, k)] = tx / (dx * dx) + ty / (dy * dy) + tz / (dz * dz);
                }
    }
}

/* Explicit right-hand side E_i = -d_j(u_j u_i) + d_j(nu_T d_i u_j) - G delta_ix
 * (Sec. 3.1: convection and the "convective-like" viscous part, both
 * advanced with Adams-Bashforth; the forcing is the constant -dp/dx).
 * Convection is in divergence form with arithmetic interpolation. */
void or_explicit(const or_params* P, const double* u, const double* v, const double* w, const double* nut,
                 double* eu, double* ev, double* ew)
{
    const double dx = hx(P), dy = hy(P), dz = hz(P);
    const int nz = P->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                /* ---- x-momentum at the x-face (i, j, k) ---- */
                {
                    const double uc = u[ix(P, i, j, k)];
                    const double ue = 0.5 * (uc + u[ix(P, i + 1, j, k)]);        /* at centre i   */
                    const double uw = 0.5 * (u[ix(P, i - 1, j, k)] + uc);        /* at centre i-1 */
                    const double cx = (ue * ue - uw * uw) / dx;
                    const double vn = 0.5 * (v[ix(P, i - 1, j + 1, k)] + v[ix(P, i, j + 1, k)]);
                    const double vs = 0.5 * (v[ix(P, i - 1, j, k)] + v[ix(P, i, j, k)]);
                    const double cy = (vn * 0.5 * (uc + u[ix(P, i, j + 1, k)]) - vs * 0.5 * (u[ix(P, i, j - 1, k)] + uc)) / dy;
                    const double wt = 0.5 * (W(P, w, i - 1, j, k + 1) + W(P, w, i, j, k + 1));
                    const double wb = 0.5 * (W(P, w, i - 1, j, k) + W(P, w, i, j, k));
                    const double cz = (wt * 0.5 * (uc + U(P, u, i, j, k + 1)) - wb * 0.5 * (U(P, u, i, j, k - 1) + uc)) / dz;
                    /* d_x(nu du/dx) + d_y(nu dv/dx) + d_z(nu dw/dx) */
                    const double vx = (nut[ix(P, i, j, k)] * (u[ix(P, i + 1, j, k)] - uc)
                                     - nut[ix(P, i - 1, j, k)] * (uc - u[ix(P, i - 1, j, k)])) / (dx * dx);
                    const double vy = (nu_xy(P, nut, i, j + 1, k) * (v[ix(P, i, j + 1, k)] - v[ix(P, i - 1, j + 1, k)])
                                     - nu_xy(P, nut, i, j, k) * (v[ix(P, i, j, k)] - v[ix(P, i - 1, j, k)])) / (dx * dy);
                    const double vz = (nu_xz(P, nut, i, j, k + 1) * (W(P, w, i, j, k + 1) - W(P, w, i - 1, j, k + 1))
                                     - nu_xz(P, nut, i, j, k) * (W(P, w, i, j, k) - W(P, w, i - 1, j, k))) / (dx * dz);
                    eu[ix(P, i, j, k)] = -(cx + cy + cz) + (vx + vy + vz) - P->dpdx;
                }
                /* ---- y-momentum at the y-face (i, j, k) ---- */
                {
                    const double vc = v[ix(P, i, j, k)];
                    const double ue = 0.5 * (u[ix(P, i + 1, j - 1, k)] + u[ix(P, i + 1, j, k)]);
                    const double uw = 0.5 * (u[ix(P, i, j - 1, k)] + u[ix(P, i, j, k)]);
                    const double cx = (ue * 0.5 * (vc + v[ix(P, i + 1, j, k)]) - uw * 0.5 * (v[ix(P, i - 1, j, k)] + vc)) / dx;
                    const double vn = 0.5 * (vc + v[ix(P, i, j + 1, k)]);
                    const double vs = 0.5 * (v[ix(P, i, j - 1, k)] + vc);
                    const double cy = (vn * vn - vs * vs) / dy;
                    const double wt = 0.5 * (W(P, w, i, j - 1, k + 1) + W(P, w, i, j, k + 1));
                    const double wb = 0.5 * (W(P, w, i, j - 1, k) + W(P, w, i, j, k));
                    const double cz = (wt * 0.5 * (vc + U(P, v, i, j, k + 1)) - wb * 0.5 * (U(P, v, i, j, k - 1) + vc)) / dz;
                    /* d_x(nu du/dy) + d_y(nu dv/dy) + d_z(nu dw/dy) */
                    const double vx = (nu_xy(P, nut, i + 1, j, k) * (u[ix(P, i + 1, j, k)] - u[ix(P, i + 1, j - 1, k)])
                                     - nu_xy(P, nut, i, j, k) * (u[ix(P, i, j, k)] - u[ix(P, i, j - 1, k)])) / (dx * dy);
                    const double vy = (nut[ix(P, i, j, k)] * (v[ix(P, i, j + 1, k)] - vc)
                                     - nut[ix(P, i, j - 1, k)] * (vc - v[ix(P, i, j - 1, k)])) / (dy * dy);
                    const double vz = (nu_yz(P, nut, i, j, k + 1) * (W(P, w, i, j, k + 1) - W(P, w, i, j - 1, k + 1))
                                     - nu_yz(P, nut, i, j, k) * (W(P, w, i, j, k) - W(P, w, i, j - 1, k))) / (dy * dz);
                    ev[ix(P, i, j, k)] = -(cx + cy + cz) + (vx + vy + vz);
                }
            }
    /* ---- z-momentum at the interior z-faces (i, j, k), k = 1..nz-1 ---- */
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            ew[ix(P, i, j, 0)] = 0.0;
            ew[ix(P, i, j, nz)] = 0.0;
        }
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                const double wc = w[ix(P, i, j, k)];
                const double ue = 0.5 * (u[ix(P, i + 1, j, k - 1)] + u[ix(P, i + 1, j, k)]);
                const double uw = 0.5 * (u[ix(P, i, j, k - 1)] + u[ix(P, i, j, k)]);
                const double cx = (ue * 0.5 * (wc + w[ix(P, i + 1, j, k)]) - uw * 0.5 * (w[ix(P, i - 1, j, k)] + wc)) / dx;
                const double vn = 0.5 * (v[ix(P, i, j + 1, k - 1)] + v[ix(P, i, j + 1, k)]);
                const double vs = 0.5 * (v[ix(P, i, j, k - 1)] + v[ix(P, i, j, k)]);
                const double cy = (vn * 0.5 * (wc + w[ix(P, i, j + 1, k)]) - vs * 0.5 * (w[ix(P, i, j - 1, k)] + wc)) / dy;
                const double wt = 0.5 * (wc + W(P, w, i, j, k + 1));
                const double wb = 0.5 * (W(P, w, i, j, k - 1) + wc);
                const double cz = (wt * wt - wb * wb) / dz;
                /* d_x(nu du/dz) + d_y(nu dv/dz) + d_z(nu dw/dz) */
                const double vx = (nu_xz(P, nut, i + 1, j, k) * (u[ix(P, i + 1, j, k)] - u[ix(P, i + 1, j, k - 1)])
                                 - nu_xz(P, nut, i, j, k) * (u[ix(P, i, j, k)] - u[ix(P, i, j, k - 1)])) / (dx * dz);
                const double vy = (nu_yz(P, nut, i, j + 1, k) * (v[ix(P, i, j + 1, k)] - v[ix(P, i, j + 1, k - 1)])
                                 - nu_yz(P, nut, i, j, k) * (v[ix(P, i, j, k)] - v[ix(P, i, j, k - 1)])) / (dy * dz);
                const double vz = (nut[ix(P, i, j, k)] * (W(P, w, i, j, k + 1) - wc)
                                 - nut[ix(P, i, j, k - 1)] * (wc - W(P, w, i, j, k - 1))) / (dz * dz);
                ew[ix(P, i, j, k)] = -(cx + cy + cz) + (vx + vy + vz);
            }
}

/* Crank-Nicolson solve (I - dt/2 L_nu) x = R for component c.  The paper
 * only says the system is solved numerically; here by the stationary
 * iteration x <- x + (R - (I - h L_nu) x) / (1 + h s) with h = dt/2 and the
 * scalar shift s = Lambda/2, where Lambda = 4 nu_max (1/dx^2 + 1/dy^2 +
 * 1/dz^2) bounds the spectrum of -L_nu (Gershgorin).  Its fixed point is the
 * exact solution and it contracts for every dt.  Starts from x = R and stops
 * when an iteration changes no value by more than 1e-15 of max |x| (or after
 * 1000 sweeps).  Returns the number of sweeps. */
int or_cn_solve(const or_params* P, int c, const double* nut, double nut_max, const double* R, double* x)
{
    const size_t n = c == 2 ? or_nwface(P) : or_ncell(P);
    const double dx = hx(P), dy = hy(P), dz = hz(P);
    double* lx = (double*)malloc(n * sizeof(double));
    const double h = 0.5 * P->dt;
    const double lam = 4.0 * nut_max * (1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz));
    const double s = 0.5 * lam;
    memcpy(x, R, n * sizeof(double));
    int sweeps = 0;
    while (sweeps < 1000) {
        or_visc_diff(P, c, nut, x, lx);
        double dmax = 0.0, xmax = 0.0;
        for (size_t q = 0; q < n; ++q) {
            const double res = R[q] - (x[q] - h * lx[q]);
            const double d = res / (1.0 + h * s);
            x[q] += d;
            if (fabs(d) > dmax) dmax = fabs(d);
            if (fabs(x[q]) > xmax) xmax = fabs(x[q]);
        }
        ++sweeps;
        if (dmax <= 1e-15 * xmax) break;
    }
    if (c == 2)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                x[ix(P, i, j, 0)] = 0.0;
                x[ix(P, i, j, P->nz)] = 0.0;
            }
    free(lx);
    return sweeps;
}

/* --------------------------------------------------------- diagnostics -- */

void or_diagnostics(const or_params* P, const double* u, const double* v, const double* w, or_stats* st)
{
    const size_t n = or_ncell(P);
    double* d = (double*)malloc(n * sizeof(double));
    or_divergence(P, u, v, w, d);
    double md = 0.0, su = 0.0, mu = 0.0, cfl = 0.0, sc = 0.0;
    for (size_t c = 0; c < n; ++c) if (fabs(d[c]) > md) md = fabs(d[c]);
    for (size_t c = 0; c < n; ++c) {
        su += u[c];
        if (fabs(u[c]) > mu) mu = fabs(u[c]);
        const double cu = fabs(u[c]) * P->dt / hx(P), cv = fabs(v[c]) * P->dt / hy(P);
        if (cu > cfl) cfl = cu;
        if (cv > cfl) cfl = cv;
    }
    for (size_t c = 0; c < or_nwface(P); ++c) {
        const double cw = fabs(w[c]) * P->dt / hz(P);
        if (cw > cfl) cfl = cw;
    }
    /* centreline z = lz/2: the u plane(s) nearest to it */
    const size_t plane = (size_t)P->nx * P->ny;
    if (P->nz % 2 == 0) {
        for (size_t q = 0; q < plane; ++q)
            sc += 0.5 * (u[(size_t)(P->nz / 2 - 1) * plane + q] + u[(size_t)(P->nz / 2) * plane + q]);
    } else {
        for (size_t q = 0; q < plane; ++q) sc += u[(size_t)(P->nz / 2) * plane + q];
    }
    st->max_div = md;
    st->u_bulk = su / (double)n;
    st->u_max = mu;
    st->cfl = cfl;
    st->u_centre = sc / (double)plane;
    free(d);
}

/* Plane means at every height (Sec. 6: the x-y part of the paper's
 * space-time averages), out[q (nz + 1) + k]:
 *   q = 0 u, 1 v, 2 u^2, 3 v^2, 4 nu_T on the cell planes k < nz (0 at k = nz);
 *   q = 5 w, 6 w^2 on the face planes k = 0..nz;
 *   q = 7 u w on the x-z edges (i dx, k dz): u averaged over the cell planes
 *   k - 1 and k (odd ghosts beyond the walls), w over the columns i - 1, i. */
void or_plane_stats(const or_params* P, const double* u, const double* v, const double* w, const double* nut,
                    double* out)
{
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const double area = (double)nx * ny;
    for (int k = 0; k <= nz; ++k) {
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (k < nz) {
                    const double uc = u[ix(P, i, j, k)], vc = v[ix(P, i, j, k)];
                    s[0] += uc;
                    s[1] += vc;
                    s[2] += uc * uc;
                    s[3] += vc * vc;
                    s[4] += nut[ix(P, i, j, k)];
                }
                const double wc = w[ix(P, i, j, k)];
                s[5] += wc;
                s[6] += wc * wc;
                const double ue = 0.5 * (U(P, u, i, j, k - 1) + U(P, u, i, j, k));
                const double we = 0.5 * (w[ix(P, i - 1, j, k)] + w[ix(P, i, j, k)]);
                s[7] += ue * we;
            }
        for (int q = 0; q < 8; ++q) out[q * (nz + 1) + k] = s[q] / area;
    }
}

/* ----------------------------------------------------------- time step -- */

/* One time step of the projection scheme (Sec. 3.1), in the paper's order:
 * eddy viscosity, explicit terms, Crank-Nicolson predictor u*, divergence,
 * SRJ pressure solve, correction.
 *   u, v, w, p   state at level n on entry, n+1 on exit (p: warm start in)
 *   e_hist       9 arrays: E_u, E_v, E_w for levels n-1 and n-2 on entry
 *                (slot order [n-1 u, v, w, n-2 u, v, w]); shifted on exit
 *   nstep        number of steps already taken (selects the AB start-up)
 *   nut          work/out: nu_T at level n
 *   b            work/out: the Poisson right-hand side div(u*)/dt, mean-free */
int or_step(const or_params* P, double* u, double* v, double* w, double* p, double* const* e_hist,
            int nstep, const double* omega, int m, double rtol, int maxit, double* nut, double* b, or_stats* st)
{
    const size_t n = or_ncell(P), nw = or_nwface(P);
    double* vel[3] = {u, v, w};
    const size_t len[3] = {n, n, nw};
    double* en[3];
    double* R[3];
    double* lu = (double*)malloc(nw * sizeof(double));
    for (int c = 0; c < 3; ++c) {
        en[c] = (double*)malloc(len[c] * sizeof(double));
        R[c] = (double*)malloc(len[c] * sizeof(double));
    }
    memset(st, 0, sizeof(*st));

    /* 1. eddy viscosity at level n */
    st->nut_max = or_nut(P, u, v, w, nut);

    /* 2. explicit terms at level n */
    or_explicit(P, u, v, w, nut, en[0], en[1], en[2]);

    /* 3. Adams-Bashforth weights: AB1, AB2, then AB3 */
    double beta[3] = {1.0, 0.0, 0.0};
    if (nstep == 1) { beta[0] = 1.5; beta[1] = -0.5; }
    if (nstep >= 2) { beta[0] = 23.0 / 12.0; beta[1] = -16.0 / 12.0; beta[2] = 5.0 / 12.0; }

    /* 4. Crank-Nicolson right-hand side and solve, one component at a time */
    int sweeps = 0;
    for (int c = 0; c < 3; ++c) {
        or_visc_diff(P, c, nut, vel[c], lu);
        for (size_t q = 0; q < len[c]; ++q) {
            const double ab = beta[0] * en[c][q] + beta[1] * e_hist[c][q] + beta[2] * e_hist[3 + c][q];
            R[c][q] = vel[c][q] + P->dt * ab + 0.5 * P->dt * lu[q];
        }
        if (c == 2)
            for (size_t q = 0; q < (size_t)P->nx * P->ny; ++q) {
                R[2][q] = 0.0;
                R[2][(size_t)P->nz * P->nx * P->ny + q] = 0.0;
            }
    }
    for (int c = 0; c < 3; ++c) {
        const int s = or_cn_solve(P, c, nut, st->nut_max, R[c], vel[c]);     /* vel[c] := u* */
        if (s > sweeps) sweeps = s;
    }
    st->cn_sweeps = sweeps;

    /* 5. Poisson right-hand side b = div(u*)/dt, mean removed */
    or_divergence(P, u, v, w, b);
    for (size_t q = 0; q < n; ++q) b[q] /= P->dt;
    const double bm = mean(b, n);
    for (size_t q = 0; q < n; ++q) b[q] -= bm;
    st->bnorm = sqrt(sumsq(b, n));

    /* 6. SRJ pressure solve from the warm start in p */
    int cycles = 0;
    const int status = or_poisson_srj(P, b, p, omega, m, rtol, maxit, &cycles, &st->relres0, &st->relres);
    st->poisson_cycles = cycles;
    st->status = status;

    /* 7. correction */
    or_project(P, p, u, v, w);

    /* 8. shift the Adams-Bashforth history: n-2 <- n-1, n-1 <- n */
    for (int c = 0; c < 3; ++c) {
        memcpy(e_hist[3 + c], e_hist[c], len[c] * sizeof(double));
        memcpy(e_hist[c], en[c], len[c] * sizeof(double));
    }

    /* 9. diagnostics */
    or_diagnostics(P, u, v, w, st);

    free(lu);
    for (int c = 0; c < 3; ++c) { free(en[c]); free(R[c]); }
    return status;
}

/* ------------------------------------------------------------ threads -- */

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the plane loops use (for timing the oracle on 1 or all cores);
 * returns the number in effect afterwards.  n <= 0 leaves it unchanged. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
