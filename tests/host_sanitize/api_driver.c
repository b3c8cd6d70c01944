/* Drives every entry point of include/rdc.h through its argument checks,
 * launch planning and copies, on the host-memory HIP shim (no GPU), so that
 * AddressSanitizer and UBSan see the library's host code.  Prints one line
 * per failed expectation and "ALL OK" at the end if there was none. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rdc.h"

long shim_launches(void);
long shim_bad_launches(void);
long shim_live_allocations(void);
int hipMalloc(void **p, size_t n);
int hipFree(void *p);

static int failures;
#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            ++failures;                                                           \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, \
                    #cond);                                                       \
        }                                                                         \
    } while (0)

static void *dev(size_t n) {
    void *p = NULL;
    hipMalloc(&p, n);
    return p;
}

static rdc_params table1(void) {
    rdc_params p = {0.0243, 1.4, 0.002, 0.45, 0.001, 0.25};
    return p;
}

static void plain_context(void) {
    const int nx = 333, ny = 275;
    const int64_t pitch = 384, plane = pitch * ny;
    rdc_buffers b;
    b.u[0] = dev(plane * 4); b.u[1] = dev(plane * 4);
    b.v[0] = dev(plane * 4); b.v[1] = dev(plane * 4);
    b.phi = dev(plane * 4); b.pitch = pitch;
    rdc_ctx *c = NULL;

    EXPECT(rdc_create(0, ny, RDC_FP32, &b, NULL, &c) == RDC_E_INVAL);
    EXPECT(rdc_create(nx, ny, RDC_FP32, NULL, NULL, &c) == RDC_E_INVAL);
    EXPECT(rdc_create(nx, ny, RDC_FP32, &b, NULL, NULL) == RDC_E_INVAL);
    rdc_buffers bad = b;
    bad.u[1] = bad.u[0];
    EXPECT(rdc_create(nx, ny, RDC_FP32, &bad, NULL, &c) == RDC_E_INVAL);
    bad = b;
    bad.v[0] = (char *)bad.v[0] + 4;
    EXPECT(rdc_create(nx, ny, RDC_FP32, &bad, NULL, &c) == RDC_E_INVAL);
    bad = b;
    bad.pitch = 320;
    EXPECT(rdc_create(nx, ny, RDC_FP32, &bad, NULL, &c) == RDC_E_INVAL);
    EXPECT(strlen(rdc_last_error(NULL)) > 0);
    EXPECT(rdc_create(nx, ny, RDC_FP32, &b, NULL, &c) == RDC_OK && c);

    rdc_params p = table1();
    const double nan = NAN, inf = INFINITY;
    double *fields[] = {&p.eps, &p.eps, &p.f, &p.q, &p.D_u, &p.dt, &p.dx};
    double values[] = {0.0, nan, inf, 0.0, -1.0, 0.0, 0.0};
    for (int i = 0; i < 7; ++i) {
        p = table1();
        *fields[i] = values[i];
        EXPECT(rdc_set_params(c, &p) == RDC_E_INVAL);
    }
    p = table1();
    p.D_u = 1.0;
    p.dt = 0.02;                                    /* dt D_u / dx^2 = 0.32 > 1/4 */
    EXPECT(rdc_set_params(c, &p) == RDC_E_INVAL);
    p = table1();
    EXPECT(rdc_set_params(c, &p) == RDC_OK);

    float *hu = malloc(sizeof(float) * nx * ny), *hv = malloc(sizeof(float) * nx * ny);
    float *ru = malloc(sizeof(float) * nx * ny), *rv = malloc(sizeof(float) * nx * ny);
    for (int i = 0; i < nx * ny; ++i) {
        hu[i] = (float)(i % 97) / 97.0f;
        hv[i] = (float)(i % 31) / 310.0f;
    }
    EXPECT(rdc_set_phi(c, hu, nx, RDC_HOST) == RDC_OK);
    EXPECT(rdc_set_phi(c, hu, nx - 1, RDC_HOST) == RDC_E_INVAL);
    EXPECT(rdc_write(c, hu, hv, nx, RDC_HOST) == RDC_OK);
    EXPECT(rdc_write(c, NULL, hv, nx, RDC_HOST) == RDC_E_INVAL);
    EXPECT(rdc_read(c, ru, rv, nx, RDC_HOST) == RDC_OK);
    EXPECT(memcmp(hu, ru, sizeof(float) * nx * ny) == 0);
    EXPECT(memcmp(hv, rv, sizeof(float) * nx * ny) == 0);
    EXPECT(rdc_read(c, ru, rv, nx - 1, RDC_HOST) == RDC_E_INVAL);

    EXPECT(rdc_set_block(c, 13) == RDC_E_INVAL);
    EXPECT(rdc_set_block(c, -1) == RDC_E_INVAL);
    EXPECT(rdc_set_tile_rows(c, 50) == RDC_E_INVAL);
    EXPECT(rdc_tile_rows_supported(56) == 1 && rdc_tile_rows_supported(57) == 0);
    EXPECT(rdc_step(c, -1) == RDC_E_INVAL);
    long before = shim_launches();
    EXPECT(rdc_step(c, 0) == RDC_OK);
    EXPECT(shim_launches() == before);
    const int rows[] = {48, 56, 64, 80};
    int64_t expect_step = 0;
    for (int T = 1; T <= 12; ++T) {
        for (int r = 0; r < 4; ++r) {
            EXPECT(rdc_set_block(c, T) == RDC_OK);
            EXPECT(rdc_set_tile_rows(c, rows[r]) == RDC_OK);
            before = shim_launches();
            EXPECT(rdc_step(c, 17) == RDC_OK);
            expect_step += 17;
            EXPECT(shim_launches() - before == (17 + T - 1) / T);
        }
    }
    int64_t step = -1;
    EXPECT(rdc_get_step(c, &step) == RDC_OK && step == expect_step);
    EXPECT(rdc_set_step(c, -1) == RDC_E_INVAL);
    EXPECT(rdc_set_step(c, (int64_t)INT32_MAX) == RDC_E_INVAL);
    EXPECT(rdc_set_step(c, expect_step) == RDC_OK);
    EXPECT(rdc_set_step(NULL, 0) == RDC_E_INVAL);
    EXPECT(rdc_set_block(c, 0) == RDC_OK && rdc_set_tile_rows(c, 0) == RDC_OK);
    EXPECT(rdc_step(c, 23) == RDC_OK);

    int32_t cx[100], cy[100], rr[100];
    for (int i = 0; i < 100; ++i) {
        cx[i] = (i * 37) % (nx + 10) - 5;
        cy[i] = (i * 53) % (ny + 10) - 5;
        rr[i] = 8;                                   /* every disk reaches the grid */
    }
    before = shim_launches();
    EXPECT(rdc_stimulate(c, cx, cy, rr, 100) == RDC_OK);
    EXPECT(shim_launches() - before == 2);         /* 64 disks per launch */
    int32_t far_x = nx + 50, far_y = 10, r3 = 3, neg = -1;
    EXPECT(rdc_stimulate(c, &far_x, &far_y, &r3, 1) == RDC_E_INVAL);
    EXPECT(rdc_stimulate(c, cx, cy, &neg, 1) == RDC_E_INVAL);
    EXPECT(rdc_stimulate(c, NULL, cy, rr, 1) == RDC_E_INVAL);
    EXPECT(rdc_stimulate(c, cx, cy, rr, -1) == RDC_E_INVAL);

    int32_t *arr = dev(sizeof(int32_t) * pitch * ny);
    float *tl = dev(sizeof(float) * plane);
    EXPECT(rdc_set_arrival(c, arr, 100, 0.5) == RDC_E_INVAL);
    EXPECT(rdc_set_arrival(c, arr + 1, pitch, 0.5) == RDC_E_INVAL);
    EXPECT(rdc_set_arrival(c, arr, pitch, NAN) == RDC_E_INVAL);
    EXPECT(rdc_set_arrival(c, arr, pitch, 0.5) == RDC_OK);
    EXPECT(rdc_set_timelapse(c, tl, pitch, 0) == RDC_E_INVAL);
    EXPECT(rdc_set_timelapse(c, tl, pitch, 5) == RDC_OK);
    EXPECT(rdc_set_block(c, 8) == RDC_OK);
    EXPECT(rdc_step(c, 30) == RDC_OK);
    EXPECT(rdc_set_arrival(c, NULL, 0, 0.5) == RDC_OK);
    EXPECT(rdc_set_timelapse(c, NULL, 0, 1) == RDC_OK);

    void *cu = NULL, *cv = NULL;
    EXPECT(rdc_current(c, NULL, &cv) == RDC_E_INVAL);
    EXPECT(rdc_current(c, &cu, &cv) == RDC_OK && cu && cv);

    EXPECT(rdc_copy(b.u[1], b.u[0], 64, NULL) == RDC_OK);
    EXPECT(rdc_copy(b.u[1], b.u[0], 60, NULL) == RDC_E_INVAL);
    EXPECT(rdc_copy((char *)b.u[1] + 4, b.u[0], 64, NULL) == RDC_E_INVAL);
    for (int s = 0; s >= -5; --s) EXPECT(rdc_status_string((rdc_status)s) != NULL);
    EXPECT(rdc_set_params(NULL, &p) == RDC_E_INVAL);
    EXPECT(rdc_step(NULL, 1) == RDC_E_INVAL);

    EXPECT(rdc_destroy(c) == RDC_OK);
    EXPECT(rdc_destroy(NULL) == RDC_OK);
    hipFree(arr); hipFree(tl);
    for (int i = 0; i < 2; ++i) { hipFree(b.u[i]); hipFree(b.v[i]); }
    hipFree(b.phi);
    free(hu); free(hv); free(ru); free(rv);
}

static void fp64_context(void) {
    const int nx = 70, ny = 45;
    const int64_t pitch = 128, plane = pitch * ny;
    rdc_buffers b;
    b.u[0] = dev(plane * 8); b.u[1] = dev(plane * 8);
    b.v[0] = dev(plane * 8); b.v[1] = dev(plane * 8);
    b.phi = dev(plane * 8); b.pitch = pitch;
    rdc_ctx *c = NULL;
    EXPECT(rdc_create(nx, ny, RDC_FP64, &b, NULL, &c) == RDC_OK);
    EXPECT(rdc_set_block(c, 9) == RDC_E_INVAL);     /* FP64 tiles take at most 8 steps */
    EXPECT(rdc_set_block(c, 1) == RDC_OK);
    long before = shim_launches();
    EXPECT(rdc_step(c, 5) == RDC_OK);
    EXPECT(shim_launches() - before == 5);
    const int rows[] = {48, 56, 64, 80};
    for (int T = 2; T <= 8; ++T) {
        for (int r = 0; r < 4; ++r) {
            EXPECT(rdc_set_block(c, T) == RDC_OK);
            EXPECT(rdc_set_tile_rows(c, rows[r]) == RDC_OK);
            before = shim_launches();
            EXPECT(rdc_step(c, 19) == RDC_OK);
            EXPECT(shim_launches() - before == (19 + T - 1) / T);
        }
    }
    int32_t x = 0, y = 0, r = 5;
    EXPECT(rdc_stimulate(c, &x, &y, &r, 1) == RDC_OK);
    double *h = calloc((size_t)nx * ny, sizeof(double));
    EXPECT(rdc_read(c, h, h, nx, RDC_HOST) == RDC_OK);
    EXPECT(rdc_destroy(c) == RDC_OK);
    free(h);
    for (int i = 0; i < 2; ++i) { hipFree(b.u[i]); hipFree(b.v[i]); }
    hipFree(b.phi);
}

static void batch(void) {
    rdc_sim_desc s[3];
    const int dims[3][2] = {{100, 70}, {333, 41}, {64, 64}};
    int64_t off = 0;
    for (int i = 0; i < 3; ++i) {
        s[i].nx = dims[i][0];
        s[i].ny = dims[i][1];
        s[i].pitch = (s[i].nx + 63) / 64 * 64;
        s[i].offset = off;
        s[i].params = table1();
        off += s[i].pitch * s[i].ny;
    }
    const int64_t elems = off;
    rdc_buffers pool;
    pool.u[0] = dev(elems * 4); pool.u[1] = dev(elems * 4);
    pool.v[0] = dev(elems * 4); pool.v[1] = dev(elems * 4);
    pool.phi = dev(elems * 4); pool.pitch = 0;
    rdc_batch *bt = NULL;
    rdc_sim_desc bad[3];
    memcpy(bad, s, sizeof s);
    bad[1].offset = bad[0].offset + 64;             /* overlaps simulation 0 */
    EXPECT(rdc_batch_create(3, bad, &pool, elems, NULL, &bt) == RDC_E_INVAL);
    memcpy(bad, s, sizeof s);
    bad[2].pitch = 100;
    EXPECT(rdc_batch_create(3, bad, &pool, elems, NULL, &bt) == RDC_E_INVAL);
    EXPECT(rdc_batch_create(3, s, &pool, elems - 64, NULL, &bt) == RDC_E_INVAL);
    EXPECT(rdc_batch_create(0, s, &pool, elems, NULL, &bt) == RDC_E_INVAL);
    EXPECT(rdc_batch_create(3, s, &pool, elems, NULL, &bt) == RDC_OK && bt);

    float *hu = malloc(sizeof(float) * 333 * 41), *hv = malloc(sizeof(float) * 333 * 41);
    float *ru = malloc(sizeof(float) * 333 * 41), *rv = malloc(sizeof(float) * 333 * 41);
    for (int i = 0; i < 333 * 41; ++i) { hu[i] = (float)(i % 13) * 0.05f; hv[i] = 0.01f; }
    EXPECT(rdc_batch_set_phi(bt, 1, hu, 333, RDC_HOST) == RDC_OK);
    EXPECT(rdc_batch_set_phi(bt, 3, hu, 333, RDC_HOST) == RDC_E_INVAL);
    EXPECT(rdc_batch_write(bt, 1, hu, hv, 333, RDC_HOST) == RDC_OK);
    EXPECT(rdc_batch_read(bt, 1, ru, rv, 333, RDC_HOST) == RDC_OK);
    EXPECT(memcmp(hu, ru, sizeof(float) * 333 * 41) == 0);
    EXPECT(memcmp(hv, rv, sizeof(float) * 333 * 41) == 0);
    int32_t sim[2] = {0, 2}, cx[2] = {5, 63}, cy[2] = {5, 0}, r[2] = {4, 3}, bad_sim = 7;
    EXPECT(rdc_batch_stimulate(bt, sim, cx, cy, r, 2) == RDC_OK);
    EXPECT(rdc_batch_stimulate(bt, &bad_sim, cx, cy, r, 1) == RDC_E_INVAL);
    EXPECT(rdc_batch_set_block(bt, 13, 56) == RDC_E_INVAL);
    EXPECT(rdc_batch_set_block(bt, 12, 48) == RDC_OK);
    EXPECT(rdc_batch_set_block(bt, 6, 48) == RDC_OK);
    /* all three grids fit the whole-grid path by default: one launch for 20 steps */
    EXPECT(rdc_batch_resident_count(bt) == 3);
    long l0 = shim_launches();
    EXPECT(rdc_batch_step(bt, 20) == RDC_OK);
    EXPECT(shim_launches() - l0 == 1);
    l0 = shim_launches();
    EXPECT(rdc_batch_step(bt, 40000) == RDC_OK);    /* split into launches of <= 16384 steps */
    EXPECT(shim_launches() - l0 == 3);
    EXPECT(rdc_batch_step(bt, -1) == RDC_E_INVAL);
    rdc_graph *g = NULL;
    EXPECT(rdc_batch_capture(bt, 1, &g) == RDC_E_INVAL);
    EXPECT(rdc_batch_capture(bt, 10, &g) == RDC_OK && g);
    EXPECT(rdc_graph_launch(g) == RDC_OK);
    /* 100 x 70 only (4096 cells) on the whole-grid path, the others tiled */
    EXPECT(rdc_batch_set_resident(bt, -1) == RDC_E_INVAL);
    EXPECT(rdc_batch_set_resident(bt, 7000) == RDC_OK);
    EXPECT(rdc_batch_resident_count(bt) == 2);       /* 100 x 70 and 64 x 64 */
    EXPECT(rdc_graph_launch(g) == RDC_E_STATE);      /* recorded under the old plan */
    EXPECT(rdc_graph_destroy(g) == RDC_OK);
    l0 = shim_launches();
    EXPECT(rdc_batch_step(bt, 20) == RDC_OK);       /* 1 whole-grid + 4 tiled (T = 6) */
    EXPECT(shim_launches() - l0 == 5);
    EXPECT(rdc_batch_set_resident(bt, 0) == RDC_OK);
    EXPECT(rdc_batch_resident_count(bt) == 0);
    l0 = shim_launches();
    EXPECT(rdc_batch_step(bt, 20) == RDC_OK);
    EXPECT(shim_launches() - l0 == 4);
    EXPECT(rdc_batch_capture(bt, 10, &g) == RDC_OK && g);
    EXPECT(rdc_graph_launch(g) == RDC_OK);
    EXPECT(rdc_graph_destroy(g) == RDC_OK);
    /* row pipelines: 20 steps at T = 6 in 4 launches of 5; a one-step call on the tiles */
    EXPECT(rdc_batch_set_block(bt, 12, RDC_TILE_STREAM) == RDC_E_INVAL);
    EXPECT(rdc_batch_set_block(bt, 6, RDC_TILE_STREAM) == RDC_OK);
    l0 = shim_launches();
    EXPECT(rdc_batch_step(bt, 20) == RDC_OK);
    EXPECT(shim_launches() - l0 == 4);
    l0 = shim_launches();
    EXPECT(rdc_batch_step(bt, 1) == RDC_OK);
    EXPECT(shim_launches() - l0 == 1);
    EXPECT(rdc_batch_capture(bt, 12, &g) == RDC_OK && g);
    EXPECT(rdc_graph_launch(g) == RDC_OK);
    EXPECT(rdc_graph_destroy(g) == RDC_OK);
    EXPECT(rdc_batch_set_block(bt, 6, 48) == RDC_OK);
    EXPECT(rdc_batch_resident_count(NULL) == -1);
    void *cu = NULL, *cv = NULL;
    EXPECT(rdc_batch_current(bt, &cu, &cv) == RDC_OK && cu && cv);
    EXPECT(rdc_batch_last_error(bt) != NULL);
    EXPECT(rdc_batch_destroy(bt) == RDC_OK);
    EXPECT(rdc_batch_destroy(NULL) == RDC_OK);
    free(hu); free(hv); free(ru); free(rv);
    for (int i = 0; i < 2; ++i) { hipFree(pool.u[i]); hipFree(pool.v[i]); }
    hipFree(pool.phi);
}

static void nn(void) {
    const int n = 2, h = 16, w = 64, cin = 32, cout = 64;
    const int64_t px = (int64_t)n * h * w;
    void *x = dev(px * cin * 2), *y = dev(px * cout * 2), *wt = dev(9 * cin * cout * 2);
    float *bias = dev(cout * 4), *wf = dev(9 * cin * cout * 4);
    EXPECT(rdc_nn_conv3x3(x, cin, wt, bias, y, cout, n, h, w, cin, cout, cout, 1, NULL) == RDC_OK);
    EXPECT(rdc_nn_conv3x3(x, cin, wt, NULL, y, cout, n, h, w - 2, cin, cout, cout, 0, NULL) ==
           RDC_E_INVAL);
    EXPECT(rdc_nn_conv3x3(x, cin, wt, NULL, y, cout, n, h, w, cin, 48, 48, 0, NULL) ==
           RDC_E_INVAL);
    EXPECT(rdc_nn_conv3x3((char *)x + 2, cin, wt, NULL, y, cout, n, h, w, cin, cout, cout, 0,
                          NULL) == RDC_E_INVAL);
    EXPECT(strlen(rdc_nn_last_error()) > 0);
    EXPECT(rdc_nn_dgrad_weights(wf, wt, cout, cin, NULL) == RDC_OK);
    const int64_t sf = rdc_nn_wgrad_scratch_floats(n, h, w, cin, cout);
    EXPECT(sf > 9 * cin * cout);
    float *scratch = dev(sf * 4), *grad = dev(9 * cin * cout * 4), *gb = dev(cout * 4);
    EXPECT(rdc_nn_conv3x3_wgrad(x, cin, y, cout, scratch, grad, gb, n, h, w, cin, cout, NULL) ==
           RDC_OK);
    EXPECT(rdc_nn_conv3x3_wgrad(x, cin, y, cout, scratch, grad, gb, n, h, w, 16, cout, NULL) ==
           RDC_E_INVAL);
    /* the variant that allocates nothing: same launches, static workspace */
    const long live = shim_live_allocations();
    EXPECT(rdc_nn_conv3x3_wgrad_noalloc(x, cin, y, cout, grad, gb, n, h, w, cin, cout, NULL) ==
           RDC_OK);
    EXPECT(rdc_nn_conv3x3_wgrad_noalloc(x, cin, y, cout, grad, NULL, n, h, w, cin, cout, NULL) ==
           RDC_OK);
    EXPECT(shim_live_allocations() == live);
    EXPECT(rdc_nn_conv3x3_wgrad_noalloc(x, cin, y, cout, grad, gb, n, h, w, 16, cout, NULL) ==
           RDC_E_INVAL);
    EXPECT(rdc_nn_wgrad_scratch_floats(16, 512, 512, 32, 32) > rdc_nn_wgrad_static_floats());
    EXPECT(rdc_nn_conv3x3_wgrad_noalloc(x, cin, y, cout, grad, gb, 16, 512, 512, 32, 32, NULL) ==
           RDC_E_INVAL);
    EXPECT(rdc_nn_to_bf16(wf, wt, 9 * cin * cout, NULL) == RDC_OK);
    EXPECT(rdc_nn_relu_bwd(y, cout, y, cout, px, cout, NULL) == RDC_OK);
    void *lo = dev(px * cin * 2 / 4);
    EXPECT(rdc_nn_pool2(x, cin, lo, cin, n, h / 2, w / 2, cin, NULL) == RDC_OK);
    EXPECT(rdc_nn_pool2_bwd(lo, cin, x, cin, n, h / 2, w / 2, cin, 1, NULL) == RDC_OK);
    EXPECT(rdc_nn_up2(lo, cin, x, cin, n, h, w, cin, NULL) == RDC_OK);
    EXPECT(rdc_nn_up2_bwd(x, cin, lo, cin, n, h / 2, w / 2, cin, NULL) == RDC_OK);
    const int64_t pitch = w, plane = (int64_t)h * w;
    float *u = dev(n * plane * 4), *v = dev(n * plane * 4), *phi = dev(n * plane * 4);
    float *uo = dev(n * plane * 4), *vo = dev(n * plane * 4);
    EXPECT(rdc_nn_prep(u, v, phi, pitch, plane, x, cin, n, h, w, 1.0f, 4.0f, 5.0f, NULL) ==
           RDC_OK);
    EXPECT(rdc_nn_apply(u, v, phi, y, cout, pitch, plane, uo, vo, n, h, w, 1.0f, 4.0f, 1.4f,
                        0.3f, NULL) == RDC_OK);
    const int32_t nb = rdc_nn_loss_blocks(px);
    EXPECT(nb >= 1);
    float *partial = dev((nb + 1) * 4);
    EXPECT(rdc_nn_loss(u, v, uo, vo, pitch, plane, y, cout, x, cin, n, h, w, 1.0f, 4.0f, 0.5f,
                       4.0f, partial, NULL) == RDC_OK);
    float *m = dev(100 * 4), *vv = dev(100 * 4);
    EXPECT(rdc_nn_adam(wf, grad, m, vv, 100, 1e-3f, 0.9f, 0.999f, 1e-8f, 1.0f, NULL) == RDC_OK);
    EXPECT(rdc_nn_conv3x3_planes(u, v, phi, pitch, plane, 1.0f, 4.0f, 5.0f, wt, bias, y, cout,
                                 n, h, w, cin, cout, cout, NULL) == RDC_OK);
    EXPECT(rdc_nn_conv3x3_planes(u, v, phi, pitch, plane - 1, 1.0f, 4.0f, 5.0f, wt, bias, y,
                                 cout, n, h, w, cin, cout, cout, NULL) == RDC_E_INVAL);
    void *xcat = dev(px * 96 * 2), *xlow = dev(px / 4 * 64 * 2), *w96 = dev(9 * 96 * 32 * 2);
    EXPECT(rdc_nn_conv3x3_up(xcat, 96, xlow, 64, 64, w96, bias, y, 32, n, h, w, 96, 32, 32,
                             NULL) == RDC_OK);
    EXPECT(rdc_nn_conv3x3_up(xcat, 96, xlow, 64, 64, w96, bias, y, 32, n, h - 1, w, 96, 32, 32,
                             NULL) == RDC_E_INVAL);
    hipFree(xcat); hipFree(xlow); hipFree(w96);
    EXPECT(rdc_nn_conv3x3_apply(x, cin, wt, bias, u, v, phi, pitch, plane, uo, vo, n, h, w, cin,
                                1.0f, 4.0f, 1.4f, 0.3f, NULL) == RDC_OK);
    EXPECT(rdc_nn_conv3x3_apply(x, cin, wt, bias, u, v, phi, pitch, plane, uo, vo, n, h, w, cin,
                                1.0f, 4.0f, 0.0f, 0.3f, NULL) == RDC_E_INVAL);
    uint32_t *cnt = dev(4);
    EXPECT(rdc_nn_front_check(u, uo, pitch, w, h, 0.5f, cnt, NULL) == RDC_OK);
    EXPECT(rdc_nn_state_check(u, v, phi, pitch, w, h, -0.002f, 1.5f, 1.4f, 0.3f, cnt, NULL) ==
           RDC_OK);
    void *ptrs[] = {x, y, wt, bias, wf, scratch, grad, gb, lo, u, v, phi, uo, vo, partial, m,
                    vv, cnt};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) hipFree(ptrs[i]);
}

int main(void) {
    plain_context();
    fp64_context();
    batch();
    nn();
    EXPECT(shim_bad_launches() == 0);
    EXPECT(shim_live_allocations() == 0);
    printf("launches %ld\n", shim_launches());
    if (failures == 0) printf("ALL OK\n");
    return failures != 0;
}
