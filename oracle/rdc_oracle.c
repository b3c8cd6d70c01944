/*
 * rdc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of what the
 * Oregonator stepper computes.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product library never links,
 * loads or calls anything here, and this file shares no code with it.
 *
 * What is computed (Stovold, RDCSim, Sec. 2):
 *   Eq. (1), the two-variable Oregonator
 *       du/dt = (1/eps) [ u - u^2 - (f v + phi) (u - q)/(u + q) ] + D_u lap(u)
 *       dv/dt = u - v
 *   integrated by explicit forward Euler with time step dt, the Laplacian
 *   taken by the five-node operator on a square grid of spacing dx.
 *   Stimulation sets u := 1.0 on the stimulated pixels.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - boundary: no-flux, cell-centred: a neighbour outside the grid takes the
 *     value of the edge cell itself;
 *   - five-node weights (1,1,1,1,-4)/dx^2;
 *   - the v update uses u of the same (old) step (plain explicit Euler);
 *   - one fixed order of operations, FP64, no contraction (build with
 *     -ffp-contract=off), IEEE division:
 *         c1  = dt/eps,  c2 = dt*D_u/(dx*dx)
 *         s   = (uW + uE) + (uN + uS)
 *         lap = s - 4*uC
 *         a   = uC - uC*uC
 *         g   = f*vC + phiC
 *         r   = (uC - q)/(uC + q)
 *         Ru  = a - g*r
 *         u'  = (uC + c1*Ru) + c2*lap
 *         v'  = vC + dt*(uC - vC)
 *   - a stimulus disk covers the cells with (x-cx)^2 + (y-cy)^2 <= r^2;
 *   - arrival of a cell = first step index at which u >= theta.
 *
 * Layout: row-major planes of ny rows by nx columns, x fastest, no padding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double eps, f, q, D_u, dt, dx;
} rdco_params;

#define RDCO_NEVER INT32_MAX

/* Threads the OpenMP loops below run on (1 in a serial build). */
int rdco_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Value of u at (x, y), or of the edge cell (xc, yc) when (x, y) is outside
 * the grid: the zero-flux ghost of the cell-centred grid. */
static inline double at_or_edge(const double *u, int64_t nx, int64_t ny,
                                int64_t x, int64_t y, double edge) {
    if (x < 0 || x >= nx || y < 0 || y >= ny) return edge;
    return u[y * nx + x];
}

/* One forward-Euler step of Eq. (1) over the whole grid, old state (u, v)
 * to new state (un, vn).  Both updates read only the old state. */
void rdco_step(int64_t nx, int64_t ny, const rdco_params *p, const double *u,
               const double *v, const double *phi, double *un, double *vn) {
    const double c1 = p->dt / p->eps;
    const double c2 = p->dt * p->D_u / (p->dx * p->dx);
    const double f = p->f, q = p->q, dt = p->dt;
    int64_t y;
#pragma omp parallel for schedule(static) if (nx * ny >= 65536)
    for (y = 0; y < ny; ++y) {
        for (int64_t x = 0; x < nx; ++x) {
            const int64_t c = y * nx + x;
            const double uC = u[c];
            const double vC = v[c];
            const double phiC = phi[c];
            const double uW = at_or_edge(u, nx, ny, x - 1, y, uC);
            const double uE = at_or_edge(u, nx, ny, x + 1, y, uC);
            const double uN = at_or_edge(u, nx, ny, x, y - 1, uC);
            const double uS = at_or_edge(u, nx, ny, x, y + 1, uC);
            const double s = (uW + uE) + (uN + uS);
            const double lap = s - 4.0 * uC;
            const double a = uC - uC * uC;
            const double g = f * vC + phiC;
            const double r = (uC - q) / (uC + q);
            const double Ru = a - g * r;
            un[c] = (uC + c1 * Ru) + c2 * lap;
            vn[c] = vC + dt * (uC - vC);
        }
    }
}

/* Forward-Euler amplification factor of the u-equation at one cell, with v
 * frozen: 1 + dt * dR_u/du, where
 *   dR_u/du = (1/eps) [ 1 - 2u - (f v + phi) * 2q/(u+q)^2 ].
 * Explicit Euler is unstable for this mode where the factor is below -1. */
double rdco_euler_factor(const rdco_params *p, double u, double v, double phi) {
    const double d = u + p->q;
    const double dRdu = (1.0 - 2.0 * u - (p->f * v + phi) * (2.0 * p->q) / (d * d)) / p->eps;
    return 1.0 + p->dt * dRdu;
}

/* Record step index `step` for every cell with u >= theta not yet arrived. */
void rdco_mark_arrival(int64_t nx, int64_t ny, const double *u, int32_t *arrival,
                       double theta, int64_t step) {
    int64_t c;
#pragma omp parallel for schedule(static) if (nx * ny >= 65536)
    for (c = 0; c < nx * ny; ++c)
        if (arrival[c] == RDCO_NEVER && u[c] >= theta) arrival[c] = (int32_t)step;
}

/* Catalytic stimulation: u := 1.0 on every cell of every disk; v is left
 * unchanged.  Cells of a disk that fall outside the grid are skipped.  When
 * `arrival` is given, newly stimulated cells that have not arrived get
 * `step` (the stimulated state has u = 1 >= any threshold <= 1). */
void rdco_stimulate(int64_t nx, int64_t ny, double *u, int32_t k, const int32_t *cx,
                    const int32_t *cy, const int32_t *r, int32_t *arrival,
                    double theta, int64_t step) {
    for (int32_t d = 0; d < k; ++d) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t dx = x - cx[d], dy = y - cy[d];
                if (dx * dx + dy * dy <= (int64_t)r[d] * r[d]) u[y * nx + x] = 1.0;
            }
        }
    }
    if (arrival) rdco_mark_arrival(nx, ny, u, arrival, theta, step);
}

/* Advance (u, v) in place by `nsteps` Euler steps, the first of which takes
 * state index `step0` to `step0 + 1`.
 *   arrival   (nullable): after each step, cells with u >= theta that have not
 *                         arrived get the new state index;
 *   unstable  (nullable): before each step from a state index >= unstable_from,
 *                         cells whose Euler factor is below -1 are flagged 1;
 *                         *first_unstable gets the first such state index
 *                         (left untouched if none).
 * Returns 0, or -1 if scratch memory could not be allocated. */
int rdco_run(int64_t nx, int64_t ny, const rdco_params *p, double *u, double *v,
             const double *phi, int64_t nsteps, int64_t step0, int32_t *arrival,
             double theta, uint8_t *unstable, int64_t unstable_from,
             int64_t *first_unstable) {
    const int64_t n = nx * ny;
    double *un = (double *)malloc(sizeof(double) * (size_t)n);
    double *vn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!un || !vn) {
        free(un);
        free(vn);
        return -1;
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t state = step0 + s;
        if (unstable && state >= unstable_from) {
            int any = 0;
            int64_t c;
#pragma omp parallel for schedule(static) reduction(| : any) if (n >= 65536)
            for (c = 0; c < n; ++c) {
                if (rdco_euler_factor(p, u[c], v[c], phi[c]) < -1.0) {
                    unstable[c] = 1;
                    any = 1;
                }
            }
            if (any && first_unstable && *first_unstable < 0) *first_unstable = state;
        }
        rdco_step(nx, ny, p, u, v, phi, un, vn);
        memcpy(u, un, sizeof(double) * (size_t)n);
        memcpy(v, vn, sizeof(double) * (size_t)n);
        if (arrival) rdco_mark_arrival(nx, ny, u, arrival, theta, state + 1);
    }
    free(un);
    free(vn);
    return 0;
}
