/* Runs the C oracle (oracle/rdc_oracle.c) under AddressSanitizer and UBSan:
 * stimulation at the edges, a run with the arrival and stability trackers,
 * and the same run split in two (the results must match bit for bit). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double eps, f, q, D_u, dt, dx;
} rdco_params;
void rdco_stimulate(int64_t nx, int64_t ny, double *u, int32_t k, const int32_t *cx,
                    const int32_t *cy, const int32_t *r, int32_t *arrival, double theta,
                    int64_t step);
int rdco_run(int64_t nx, int64_t ny, const rdco_params *p, double *u, double *v,
             const double *phi, int64_t nsteps, int64_t step0, int32_t *arrival, double theta,
             uint8_t *unstable, int64_t unstable_from, int64_t *first_unstable);

int main(void) {
    const int64_t nx = 37, ny = 23, n = nx * ny;
    const rdco_params p = {0.022, 1.4, 0.002, 1.0, 0.001, 0.25};
    double *u[2], *v[2], *phi = malloc(sizeof(double) * n);
    int32_t *arr[2];
    uint8_t *uns[2];
    for (int k = 0; k < 2; ++k) {
        u[k] = calloc(n, sizeof(double));
        v[k] = calloc(n, sizeof(double));
        arr[k] = malloc(sizeof(int32_t) * n);
        uns[k] = calloc(n, 1);
        for (int64_t i = 0; i < n; ++i) arr[k][i] = INT32_MAX;
    }
    for (int64_t i = 0; i < n; ++i) phi[i] = 0.04 + 0.04 * (double)(i % 7) / 7.0;
    const int32_t cx[4] = {0, 36, 18, -2}, cy[4] = {0, 22, 11, 5}, r[4] = {3, 4, 2, 3};
    int64_t first[2] = {-1, -1};
    for (int k = 0; k < 2; ++k) rdco_stimulate(nx, ny, u[k], 4, cx, cy, r, arr[k], 0.5, 0);
    int bad = rdco_run(nx, ny, &p, u[0], v[0], phi, 300, 0, arr[0], 0.5, uns[0], 0, &first[0]);
    bad |= rdco_run(nx, ny, &p, u[1], v[1], phi, 137, 0, arr[1], 0.5, uns[1], 0, &first[1]);
    bad |= rdco_run(nx, ny, &p, u[1], v[1], phi, 163, 137, arr[1], 0.5, uns[1], 0, &first[1]);
    int same = memcmp(u[0], u[1], sizeof(double) * n) == 0 &&
               memcmp(v[0], v[1], sizeof(double) * n) == 0 &&
               memcmp(arr[0], arr[1], sizeof(int32_t) * n) == 0 &&
               memcmp(uns[0], uns[1], n) == 0 && first[0] == first[1];
    int finite = 1, arrived = 0;
    for (int64_t i = 0; i < n; ++i) {
        finite &= isfinite(u[0][i]) && isfinite(v[0][i]);
        arrived += arr[0][i] != INT32_MAX;
    }
    printf("same %d finite %d arrived %d\n", same, finite, arrived);
    for (int k = 0; k < 2; ++k) { free(u[k]); free(v[k]); free(arr[k]); free(uns[k]); }
    free(phi);
    if (!bad && same && finite && arrived > 0) printf("ALL OK\n");
    return !(!bad && same && finite && arrived > 0);
}
