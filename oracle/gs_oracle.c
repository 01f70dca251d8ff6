/*
 * gs_oracle.c -- plain, slow FP64 CPU oracle for one explicit RK2
 * finite-volume step of the 3D ideal-gas Euler equations on a Cartesian mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark have an independent,
 * obviously correct statement of what the GPU library computes.  The product
 * library neither links, includes nor calls anything here, and nothing here
 * includes anything from the product.
 *
 * Structure (paper, Section 3, Algorithm 1 "Fluid Evolution"): every kernel is
 * its own pass over whole arrays that carry two layers of ghost cells on each
 * side of every axis (the rank-3 remapping with bounds -1:n+2 in Section 3).
 * One step is
 *     TimeStep = ComputeTimeStep(FluidCurrent)
 *     FluidOld = FluidCurrent
 *     Differences -> Reconstruction -> Fluxes -> Update(TimeStep)
 *     FluidCurrent = FluidOld + FluidUpdate;              GhostExchange
 *     Differences -> Reconstruction -> Fluxes -> Update(TimeStep)
 *     FluidCurrent = 0.5 * (FluidOld + FluidCurrent + FluidUpdate);  GhostExchange
 *
 * The paper names the kernels but gives no formulas.  The readings taken
 * where it is silent (all of them shared with the GPU path by specification,
 * never by code):
 *   - ideal gas, p = (gamma-1) (E - rho |v|^2 / 2); conserved fields in the
 *     order (rho, m_x, m_y, m_z, E), primitive (rho, v_x, v_y, v_z, p);
 *   - the differences and the reconstruction act on primitive variables;
 *     difference index ranges as in the paper's listing (Section 3):
 *     dV(i) = V(i) - V(i-1) for i = 0 .. n+2 in the paper's 1-based cells;
 *   - limited slope sigma(i) = minmod(dV(i), dV(i+1)); face states
 *     V_L(i+1/2) = V(i) + sigma(i)/2, V_R(i+1/2) = V(i+1) - sigma(i+1)/2;
 *   - HLL flux with Davis wave-speed estimates from the face states;
 *   - Update = -TimeStep * sum_d (F(i+1/2) - F(i-1/2)) / h_d, accumulated in
 *     the order x, y, z;
 *   - TimeStep = CFL / max over proper cells of sum_d (|v_d| + c) / h_d;
 *   - GhostExchange: outflow copies the edge proper cell into both ghost
 *     layers, periodic wraps.
 *
 * Built with gcc -O2 -fopenmp -ffp-contract=off: IEEE FP64, no contraction,
 * no fast-math.  OpenMP only splits independent outer loops; every output
 * element is computed by exactly one thread, and the one reduction (a max) is
 * exact, so results do not depend on the thread count.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 5 /* number of fields */

/* Mesh of proper cells plus two ghost layers on each side of every axis. */
typedef struct {
    int n[3];        /* proper cells along x, y, z                      */
    double h[3];     /* cell widths                                      */
    double gamma;    /* ratio of specific heats                          */
    ptrdiff_t s[3];  /* element strides of a ghosted field along x, y, z */
    ptrdiff_t nf;    /* elements per field of a ghosted array            */
} Mesh;

static void mesh_init(Mesh* m, int nx, int ny, int nz, double dx, double dy,
                      double dz, double gamma)
{
    m->n[0] = nx; m->n[1] = ny; m->n[2] = nz;
    m->h[0] = dx; m->h[1] = dy; m->h[2] = dz;
    m->gamma = gamma;
    m->s[0] = 1;
    m->s[1] = (ptrdiff_t)(nx + 4);
    m->s[2] = (ptrdiff_t)(nx + 4) * (ny + 4);
    m->nf = (ptrdiff_t)(nx + 4) * (ny + 4) * (nz + 4);
}

/* Offset of cell (i, j, k) in a ghosted field; proper cells are 0..n-1,
 * ghosts -2, -1 and n, n+1. */
static ptrdiff_t at(const Mesh* m, int i, int j, int k)
{
    return (ptrdiff_t)(i + 2) * m->s[0] + (ptrdiff_t)(j + 2) * m->s[1] +
           (ptrdiff_t)(k + 2) * m->s[2];
}

static double* alloc_fields(const Mesh* m)
{
    return (double*)calloc((size_t)NV * (size_t)m->nf, sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Pointwise physics                                                         */
/* ------------------------------------------------------------------------ */

/* Conserved (rho, m, E) -> primitive (rho, v, p) for an ideal gas. */
void ora_c2p(double gamma, const double U[NV], double W[NV])
{
    double rho = U[0];
    double vx = U[1] / rho, vy = U[2] / rho, vz = U[3] / rho;
    double kinetic = 0.5 * (U[1] * vx + U[2] * vy + U[3] * vz);
    W[0] = rho;
    W[1] = vx;
    W[2] = vy;
    W[3] = vz;
    W[4] = (gamma - 1.0) * (U[4] - kinetic);
}

/* Primitive (rho, v, p) -> conserved (rho, m, E) for an ideal gas. */
void ora_p2c(double gamma, const double W[NV], double U[NV])
{
    double rho = W[0];
    double v2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
    U[0] = rho;
    U[1] = rho * W[1];
    U[2] = rho * W[2];
    U[3] = rho * W[3];
    U[4] = W[4] / (gamma - 1.0) + 0.5 * rho * v2;
}

/* minmod(a, b): the smaller-magnitude argument when both have the same
 * strict sign, else 0.  Written with sign tests rather than a*b > 0, which
 * can underflow to 0 for tiny arguments. */
double ora_minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

/* Physical flux of the Euler equations through a face with unit normal
 * along `axis`, for primitive state W with conserved state U. */
static void normal_flux(int axis, const double W[NV], const double U[NV],
                        double F[NV])
{
    double un = W[1 + axis];
    double p = W[4];
    F[0] = U[0] * un;
    F[1] = U[1] * un;
    F[2] = U[2] * un;
    F[3] = U[3] * un;
    F[1 + axis] += p;
    F[4] = (U[4] + p) * un;
}

/* HLL approximate Riemann flux through a face normal to `axis` between the
 * left face state WL and the right face state WR (primitive).  The first half
 * is what the paper calls the Riemann-solver input (Section 4): conserved
 * states, physical fluxes, sound speeds and the Davis estimates of the
 * slowest and fastest signal speeds.  S, if non-NULL, receives (S_L, S_R). */
void ora_hll(double gamma, int axis, const double WL[NV], const double WR[NV],
             double F[NV], double S[2])
{
    double UL[NV], UR[NV], FL[NV], FR[NV];
    ora_p2c(gamma, WL, UL);
    ora_p2c(gamma, WR, UR);
    normal_flux(axis, WL, UL, FL);
    normal_flux(axis, WR, UR, FR);
    double cL = sqrt(gamma * WL[4] / WL[0]);
    double cR = sqrt(gamma * WR[4] / WR[0]);
    double unL = WL[1 + axis], unR = WR[1 + axis];
    double aL = unL - cL, bL = unR - cR;
    double aR = unL + cL, bR = unR + cR;
    double SL = aL < bL ? aL : bL;
    double SR = aR > bR ? aR : bR;
    if (S) { S[0] = SL; S[1] = SR; }

    if (SL >= 0.0) {
        for (int v = 0; v < NV; ++v) F[v] = FL[v];
    } else if (SR <= 0.0) {
        for (int v = 0; v < NV; ++v) F[v] = FR[v];
    } else {
        for (int v = 0; v < NV; ++v)
            F[v] = ((SR * FL[v] - SL * FR[v]) + (SL * SR) * (UR[v] - UL[v])) /
                   (SR - SL);
    }
}

/* Fastest signal rate of a proper cell, sum_d (|v_d| + c) / h_d. */
static double signal_rate(const Mesh* m, const double U[NV])
{
    double W[NV];
    ora_c2p(m->gamma, U, W);
    double c = sqrt(m->gamma * W[4] / W[0]);
    double r = 0.0;
    for (int d = 0; d < 3; ++d) r += (fabs(W[1 + d]) + c) / m->h[d];
    return r;
}

/* ------------------------------------------------------------------------ */
/* Line kernels: one variable along one axis.  V points at proper cell 0;     */
/* element i lives at V[i * st] for i = -2 .. n+1.                            */
/* ------------------------------------------------------------------------ */

/* ComputeDifferences along a line (Section 3 listing):
 * dV(i) = V(i) - V(i-1) for i = -1 .. n+1 (the paper's 0 .. n+2). */
static void differences_line(int n, const double* V, double* dV, ptrdiff_t st)
{
    for (int i = -1; i <= n + 1; ++i)
        dV[i * st] = V[i * st] - V[(i - 1) * st];
}

/* ComputeReconstruction along a line: limited slopes for cells -1 .. n and
 * the two face states of faces i+1/2, i = -1 .. n-1 (stored at index i). */
static void reconstruction_line(int n, const double* V, const double* dV,
                                double* sigma, double* VL, double* VR,
                                ptrdiff_t st)
{
    for (int i = -1; i <= n; ++i)
        sigma[i * st] = ora_minmod(dV[i * st], dV[(i + 1) * st]);
    for (int i = -1; i <= n - 1; ++i) {
        VL[i * st] = V[i * st] + 0.5 * sigma[i * st];
        VR[i * st] = V[(i + 1) * st] - 0.5 * sigma[(i + 1) * st];
    }
}

/* Contiguous-line entry points of the two kernels above, for tests.  Arrays
 * hold n+4 elements, element 0 being ghost -2. */
void ora_differences_line(int n, const double* V, double* dV)
{
    differences_line(n, V + 2, dV + 2, 1);
}

void ora_reconstruction_line(int n, const double* V, const double* dV,
                             double* sigma, double* VL, double* VR)
{
    reconstruction_line(n, V + 2, dV + 2, sigma + 2, VL + 2, VR + 2, 1);
}

/* ------------------------------------------------------------------------ */
/* Mesh-level kernels                                                         */
/* ------------------------------------------------------------------------ */

/* The axes transverse to d, in (x, y, z) order. */
static void transverse(int d, int* t1, int* t2)
{
    *t1 = (d == 0) ? 1 : 0;
    *t2 = (d == 2) ? 1 : 2;
}

/* Proper source index of ghost index g on an axis of n proper cells. */
static int ghost_source(int g, int n, int periodic)
{
    if (periodic) return ((g % n) + n) % n;
    return g < 0 ? 0 : n - 1;
}

/* GhostExchange for the physical boundaries of one subdomain: fills both
 * ghost layers of every axis, axis by axis, so that edges and corners are
 * filled too (the stencil never reads them, but the primitive recovery runs
 * over every cell). */
static void ghost_exchange(const Mesh* m, double* U, int periodic)
{
    for (int d = 0; d < 3; ++d) {
        int t1, t2;
        transverse(d, &t1, &t2);
        /* x over proper (y, z); y over all x, proper z; z over all x, y. */
        int lo1 = (t1 < d) ? -2 : 0, hi1 = (t1 < d) ? m->n[t1] + 2 : m->n[t1];
        int lo2 = (t2 < d) ? -2 : 0, hi2 = (t2 < d) ? m->n[t2] + 2 : m->n[t2];
        const int ghosts[4] = {-2, -1, m->n[d], m->n[d] + 1};
        for (int f = 0; f < NV; ++f) {
            double* Uf = U + (ptrdiff_t)f * m->nf;
#pragma omp parallel for collapse(2) schedule(static)
            for (int b = lo2; b < hi2; ++b)
                for (int a = lo1; a < hi1; ++a) {
                    ptrdiff_t base = (ptrdiff_t)(a + 2) * m->s[t1] +
                                     (ptrdiff_t)(b + 2) * m->s[t2] +
                                     2 * m->s[d];
                    for (int q = 0; q < 4; ++q) {
                        int g = ghosts[q];
                        int src = ghost_source(g, m->n[d], periodic);
                        Uf[base + (ptrdiff_t)g * m->s[d]] =
                            Uf[base + (ptrdiff_t)src * m->s[d]];
                    }
                }
        }
    }
}

/* Primitive recovery on every cell of a ghosted array. */
static void primitives(const Mesh* m, const double* U, double* W)
{
    ptrdiff_t nf = m->nf;
#pragma omp parallel for schedule(static)
    for (ptrdiff_t p = 0; p < nf; ++p) {
        double u[NV], w[NV];
        for (int f = 0; f < NV; ++f) u[f] = U[f * nf + p];
        ora_c2p(m->gamma, u, w);
        for (int f = 0; f < NV; ++f) W[f * nf + p] = w[f];
    }
}

/* Work arrays of one stage: every one a whole ghosted 5-field array, kept
 * separate as in the paper's Section 3 (Differences, Reconstruction, Fluxes,
 * FluidUpdate). */
typedef struct {
    double *W, *dW, *sigma, *WL, *WR, *F, *acc;
} Work;

static int work_alloc(const Mesh* m, Work* w)
{
    w->W = alloc_fields(m);
    w->dW = alloc_fields(m);
    w->sigma = alloc_fields(m);
    w->WL = alloc_fields(m);
    w->WR = alloc_fields(m);
    w->F = alloc_fields(m);
    w->acc = alloc_fields(m);
    return w->W && w->dW && w->sigma && w->WL && w->WR && w->F && w->acc;
}

static void work_free(Work* w)
{
    free(w->W); free(w->dW); free(w->sigma); free(w->WL); free(w->WR);
    free(w->F); free(w->acc);
}

/* One substep's kernels: from FluidCurrent U (ghosts already filled) to
 * FluidUpdate = -dt * div F on the proper cells (stored in w->acc). */
static void compute_update(const Mesh* m, const double* U, double dt, Work* w)
{
    const ptrdiff_t nf = m->nf;
    primitives(m, U, w->W);
    memset(w->acc, 0, sizeof(double) * (size_t)NV * (size_t)nf);

    for (int d = 0; d < 3; ++d) {
        int t1, t2;
        transverse(d, &t1, &t2);
        const int n = m->n[d];
        const ptrdiff_t st = m->s[d];

        /* ComputeDifferences and ComputeReconstruction, per field. */
        for (int f = 0; f < NV; ++f) {
            const double* V = w->W + f * nf;
            double* dV = w->dW + f * nf;
            double* sg = w->sigma + f * nf;
            double* VL = w->WL + f * nf;
            double* VR = w->WR + f * nf;
#pragma omp parallel for collapse(2) schedule(static)
            for (int b = 0; b < m->n[t2]; ++b)
                for (int a = 0; a < m->n[t1]; ++a) {
                    ptrdiff_t base = (ptrdiff_t)(a + 2) * m->s[t1] +
                                     (ptrdiff_t)(b + 2) * m->s[t2] + 2 * st;
                    differences_line(n, V + base, dV + base, st);
                    reconstruction_line(n, V + base, dV + base, sg + base,
                                        VL + base, VR + base, st);
                }
        }

        /* ComputeFluxes: HLL on faces i+1/2, i = -1 .. n-1 (stored at i). */
#pragma omp parallel for collapse(2) schedule(static)
        for (int b = 0; b < m->n[t2]; ++b)
            for (int a = 0; a < m->n[t1]; ++a) {
                ptrdiff_t base = (ptrdiff_t)(a + 2) * m->s[t1] +
                                 (ptrdiff_t)(b + 2) * m->s[t2] + 2 * st;
                for (int i = -1; i <= n - 1; ++i) {
                    ptrdiff_t p = base + (ptrdiff_t)i * st;
                    double wl[NV], wr[NV], fl[NV];
                    for (int f = 0; f < NV; ++f) {
                        wl[f] = w->WL[f * nf + p];
                        wr[f] = w->WR[f * nf + p];
                    }
                    ora_hll(m->gamma, d, wl, wr, fl, NULL);
                    for (int f = 0; f < NV; ++f) w->F[f * nf + p] = fl[f];
                }
            }

        /* ComputeUpdate, part 1: accumulate this axis' flux difference. */
#pragma omp parallel for collapse(2) schedule(static)
        for (int b = 0; b < m->n[t2]; ++b)
            for (int a = 0; a < m->n[t1]; ++a) {
                ptrdiff_t base = (ptrdiff_t)(a + 2) * m->s[t1] +
                                 (ptrdiff_t)(b + 2) * m->s[t2] + 2 * st;
                for (int i = 0; i < n; ++i) {
                    ptrdiff_t p = base + (ptrdiff_t)i * st;
                    for (int f = 0; f < NV; ++f)
                        w->acc[f * nf + p] +=
                            (w->F[f * nf + p] - w->F[f * nf + p - st]) /
                            m->h[d];
                }
            }
    }

    /* ComputeUpdate, part 2: FluidUpdate = -TimeStep * divergence. */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m->n[2]; ++k)
        for (int j = 0; j < m->n[1]; ++j)
            for (int i = 0; i < m->n[0]; ++i) {
                ptrdiff_t p = at(m, i, j, k);
                for (int f = 0; f < NV; ++f)
                    w->acc[f * nf + p] = -dt * w->acc[f * nf + p];
            }
}

/* Copy between the proper cells of a ghosted array and a plain
 * [field][z][y][x] array. */
static void scatter_proper(const Mesh* m, const double* U, double* G)
{
    for (int f = 0; f < NV; ++f)
#pragma omp parallel for schedule(static)
        for (int k = 0; k < m->n[2]; ++k)
            for (int j = 0; j < m->n[1]; ++j)
                for (int i = 0; i < m->n[0]; ++i)
                    G[f * m->nf + at(m, i, j, k)] =
                        U[(((ptrdiff_t)f * m->n[2] + k) * m->n[1] + j) *
                              m->n[0] + i];
}

static void gather_proper(const Mesh* m, const double* G, double* U)
{
    for (int f = 0; f < NV; ++f)
#pragma omp parallel for schedule(static)
        for (int k = 0; k < m->n[2]; ++k)
            for (int j = 0; j < m->n[1]; ++j)
                for (int i = 0; i < m->n[0]; ++i)
                    U[(((ptrdiff_t)f * m->n[2] + k) * m->n[1] + j) * m->n[0] +
                      i] = G[f * m->nf + at(m, i, j, k)];
}

/* ComputeTimeStep on the proper cells of a plain [field][z][y][x] array. */
static double time_step_plain(const Mesh* m, double cfl, const double* U)
{
    const ptrdiff_t ncell = (ptrdiff_t)m->n[0] * m->n[1] * m->n[2];
    double rmax = 0.0;
#pragma omp parallel for reduction(max : rmax) schedule(static)
    for (ptrdiff_t p = 0; p < ncell; ++p) {
        double u[NV];
        for (int f = 0; f < NV; ++f) u[f] = U[f * ncell + p];
        double r = signal_rate(m, u);
        if (r > rmax) rmax = r;
    }
    return cfl / rmax;
}

/* One RK2 step (both substeps of Algorithm 1) on ghosted FluidCurrent G with
 * ghosts already filled.  Old is scratch of the same shape. */
static void rk2_step(const Mesh* m, double* G, double* Old, double dt,
                     int periodic, Work* w)
{
    const ptrdiff_t nf = m->nf;
    memcpy(Old, G, sizeof(double) * (size_t)NV * (size_t)nf); /* FluidOld = FluidCurrent */

    compute_update(m, G, dt, w);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m->n[2]; ++k)
        for (int j = 0; j < m->n[1]; ++j)
            for (int i = 0; i < m->n[0]; ++i) {
                ptrdiff_t p = at(m, i, j, k);
                for (int f = 0; f < NV; ++f)
                    G[f * nf + p] = Old[f * nf + p] + w->acc[f * nf + p];
            }
    ghost_exchange(m, G, periodic);

    compute_update(m, G, dt, w);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m->n[2]; ++k)
        for (int j = 0; j < m->n[1]; ++j)
            for (int i = 0; i < m->n[0]; ++i) {
                ptrdiff_t p = at(m, i, j, k);
                for (int f = 0; f < NV; ++f)
                    G[f * nf + p] =
                        0.5 * ((Old[f * nf + p] + G[f * nf + p]) +
                               w->acc[f * nf + p]);
            }
    ghost_exchange(m, G, periodic);
}

/* ------------------------------------------------------------------------ */
/* Exported mesh-level entry points.  U is a plain array [5][nz][ny][nx]       */
/* (x fastest) of conserved fields.  Return 0 on success, -1 on bad arguments */
/* or allocation failure.                                                     */
/* ------------------------------------------------------------------------ */

static int args_ok(int nx, int ny, int nz, double dx, double dy, double dz,
                   double gamma, int bc)
{
    return nx >= 1 && ny >= 1 && nz >= 1 && dx > 0 && dy > 0 && dz > 0 &&
           gamma > 1.0 && (bc == 0 || bc == 1);
}

double ora_time_step(int nx, int ny, int nz, double dx, double dy, double dz,
                     double gamma, double cfl, const double* U)
{
    Mesh m;
    mesh_init(&m, nx, ny, nz, dx, dy, dz, gamma);
    return time_step_plain(&m, cfl, U);
}

/* Advance up to nsteps RK2 steps in place.  TimeStep is recomputed from
 * FluidCurrent before every step (Algorithm 1); if t_end > 0 the last step is
 * shortened so that the time reaches t_end exactly, and stepping stops there.
 * dts (may be NULL) receives each step's TimeStep.  Returns the number of
 * steps taken, or -1. */
int ora_run(int nx, int ny, int nz, double dx, double dy, double dz,
            double gamma, double cfl, int bc, double* U, int nsteps,
            double t_end, double* dts)
{
    if (!args_ok(nx, ny, nz, dx, dy, dz, gamma, bc) || !(cfl > 0) || nsteps < 0)
        return -1;
    Mesh m;
    mesh_init(&m, nx, ny, nz, dx, dy, dz, gamma);
    Work w;
    double* G = alloc_fields(&m);
    double* Old = alloc_fields(&m);
    if (!G || !Old || !work_alloc(&m, &w)) {
        free(G); free(Old); work_free(&w);
        return -1;
    }
    scatter_proper(&m, U, G);
    ghost_exchange(&m, G, bc == 1);

    double t = 0.0;
    int taken = 0;
    for (int s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && !(t < t_end)) break;
        gather_proper(&m, G, U);
        double dt = time_step_plain(&m, cfl, U);
        if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
        rk2_step(&m, G, Old, dt, bc == 1, &w);
        t += dt;
        if (dts) dts[s] = dt;
        ++taken;
    }
    gather_proper(&m, G, U);
    free(G); free(Old); work_free(&w);
    return taken;
}

/* One RK2 step in place with a given TimeStep. */
int ora_step(int nx, int ny, int nz, double dx, double dy, double dz,
             double gamma, int bc, double* U, double dt)
{
    if (!args_ok(nx, ny, nz, dx, dy, dz, gamma, bc)) return -1;
    Mesh m;
    mesh_init(&m, nx, ny, nz, dx, dy, dz, gamma);
    Work w;
    double* G = alloc_fields(&m);
    double* Old = alloc_fields(&m);
    if (!G || !Old || !work_alloc(&m, &w)) {
        free(G); free(Old); work_free(&w);
        return -1;
    }
    scatter_proper(&m, U, G);
    ghost_exchange(&m, G, bc == 1);
    rk2_step(&m, G, Old, dt, bc == 1, &w);
    gather_proper(&m, G, U);
    free(G); free(Old); work_free(&w);
    return 0;
}

/* One RK2 step of a periodic mesh, evaluated only on the window of
 * wx*wy*wz proper cells whose first cell is (i0, j0, k0) (any integers; the
 * window wraps).  The result equals that window of ora_step's output: the
 * second substep on the window needs the first substep's result two cells
 * around it, which in turn needs FluidCurrent four cells around it, all taken
 * from the periodic full array.  out receives [5][wz][wy][wx]. */
int ora_step_window(int nx, int ny, int nz, double dx, double dy, double dz,
                    double gamma, const double* U, double dt, int i0, int j0,
                    int k0, int wx, int wy, int wz, double* out)
{
    if (!args_ok(nx, ny, nz, dx, dy, dz, gamma, 1) || wx < 1 || wy < 1 ||
        wz < 1)
        return -1;
    const ptrdiff_t ncell = (ptrdiff_t)nx * ny * nz;

    /* Substep 1 runs on a mesh of (w+4) proper cells whose ghosts are the
     * true neighbours, i.e. the window grown by 4 cells on each side. */
    Mesh m1, m2;
    mesh_init(&m1, wx + 4, wy + 4, wz + 4, dx, dy, dz, gamma);
    mesh_init(&m2, wx, wy, wz, dx, dy, dz, gamma);
    Work w1, w2;
    double* G1 = alloc_fields(&m1);
    double* G2 = alloc_fields(&m2);
    double* Old2 = alloc_fields(&m2);
    int ok = G1 && G2 && Old2;
    ok = work_alloc(&m1, &w1) && ok;
    ok = work_alloc(&m2, &w2) && ok;
    if (!ok) {
        free(G1); free(G2); free(Old2); work_free(&w1); work_free(&w2);
        return -1;
    }

    for (int f = 0; f < NV; ++f)
        for (int k = -2; k < wz + 6; ++k)
            for (int j = -2; j < wy + 6; ++j)
                for (int i = -2; i < wx + 6; ++i) {
                    int gi = ghost_source(i0 - 2 + i, nx, 1);
                    int gj = ghost_source(j0 - 2 + j, ny, 1);
                    int gk = ghost_source(k0 - 2 + k, nz, 1);
                    G1[f * m1.nf + at(&m1, i, j, k)] =
                        U[f * ncell + ((ptrdiff_t)gk * ny + gj) * nx + gi];
                }

    /* Substep 1 on the grown window: FluidCurrent = FluidOld + FluidUpdate. */
    compute_update(&m1, G1, dt, &w1);
    for (int f = 0; f < NV; ++f)
        for (int k = -2; k < wz + 2; ++k)
            for (int j = -2; j < wy + 2; ++j)
                for (int i = -2; i < wx + 2; ++i) {
                    ptrdiff_t p1 = f * m1.nf + at(&m1, i + 2, j + 2, k + 2);
                    ptrdiff_t p2 = f * m2.nf + at(&m2, i, j, k);
                    G2[p2] = G1[p1] + w1.acc[p1];
                    Old2[p2] = G1[p1];
                }

    /* Substep 2 on the window, ghosts being substep-1 values of true
     * neighbours. */
    compute_update(&m2, G2, dt, &w2);
    for (int f = 0; f < NV; ++f)
        for (int k = 0; k < wz; ++k)
            for (int j = 0; j < wy; ++j)
                for (int i = 0; i < wx; ++i) {
                    ptrdiff_t p = f * m2.nf + at(&m2, i, j, k);
                    out[(((ptrdiff_t)f * wz + k) * wy + j) * wx + i] =
                        0.5 * ((Old2[p] + G2[p]) + w2.acc[p]);
                }

    free(G1); free(G2); free(Old2); work_free(&w1); work_free(&w2);
    return 0;
}

/* GhostExchange alone, for tests: copies the plain array U [5][nz][ny][nx]
 * into the proper cells of G [5][nz+4][ny+4][nx+4] and fills G's ghost
 * layers for boundary kind bc (0 outflow, 1 periodic). */
int ora_fill_ghosts(int nx, int ny, int nz, int bc, const double* U, double* G)
{
    if (!args_ok(nx, ny, nz, 1.0, 1.0, 1.0, 2.0, bc)) return -1;
    Mesh m;
    mesh_init(&m, nx, ny, nz, 1.0, 1.0, 1.0, 2.0);
    memset(G, 0, sizeof(double) * (size_t)NV * (size_t)m.nf);
    scatter_proper(&m, U, G);
    ghost_exchange(&m, G, bc == 1);
    return 0;
}

/* Number of OpenMP threads the mesh-level entry points use. */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set that number (n >= 1); no effect without OpenMP. */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
