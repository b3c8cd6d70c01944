/*
 * rdc.h -- C ABI of the MI355X (gfx950) Oregonator stepper, librdc.so.
 *
 * The library advances the two-variable Oregonator reaction-diffusion model
 * of Stovold, "RDCSim" (arXiv 1901.06535), Sec. 2, Eq. (1):
 *
 *     du/dt = (1/eps) [ u - u^2 - (f v + phi) (u - q)/(u + q) ] + D_u lap(u)
 *     dv/dt = u - v
 *
 * by explicit forward Euler with time step dt and the five-node Laplacian on
 * a square grid of spacing dx (Sec. 2), with a per-cell excitability map phi
 * (active vs. passive / inhibitive substrate drawn by the user, Sec. 3) and
 * catalytic stimulation that sets u := 1.0 on stimulated pixels (Sec. 2).
 * Where the paper is silent the library takes these readings:
 *   - edges are no-flux, cell-centred: a neighbour outside the grid takes the
 *     value of the edge cell itself;
 *   - both updates of one step read the old state only;
 *   - a stimulus disk (cx, cy, r) covers the cells with
 *     (x - cx)^2 + (y - cy)^2 <= r^2.
 *
 * Conventions for every call:
 *   - Every call returns an rdc_status; nothing throws or aborts across the
 *     ABI.  After a failure rdc_last_error(ctx) holds a message.
 *   - Planes are row-major: ny rows of nx cells, x fastest, rows `pitch`
 *     elements apart.  Device planes handed to rdc_create must use one pitch
 *     that is a multiple of 64 elements, be at least pitch*ny elements long
 *     and start on a 256-byte boundary.  Cells in columns [nx, pitch) are
 *     padding: the library may read them but never gives them meaning.
 *   - Element type is float (RDC_FP32) or double (RDC_FP64) for u, v, phi.
 *   - All device work is queued on the stream given to rdc_create (a
 *     hipStream_t passed as void*; NULL = the legacy default stream).  Calls
 *     that take HOST pointers copy synchronously and have finished with the
 *     pointer when they return; calls on DEVICE pointers are asynchronous on
 *     that stream.  rdc_read and rdc_current always wait for the stream;
 *     they report device errors and the non-finite flag.
 *   - A context is not thread-safe.  Distinct contexts are independent.
 */
#ifndef RDC_H
#define RDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rdc_ctx rdc_ctx; /* opaque, one per grid */

typedef enum {
    RDC_OK = 0,
    RDC_E_INVAL = -1,     /* bad argument: see each call */
    RDC_E_NOMEM = -2,     /* host or device allocation failed */
    RDC_E_DEVICE = -3,    /* a HIP call or kernel launch failed */
    RDC_E_NONFINITE = -4, /* a non-finite u or v was produced (sticky until rdc_write) */
    RDC_E_STATE = -5      /* call not valid in the current state */
} rdc_status;

typedef enum { RDC_FP32 = 0, RDC_FP64 = 1 } rdc_dtype;
typedef enum { RDC_HOST = 0, RDC_DEVICE = 1 } rdc_where;

/* Model and scheme parameters of Eq. (1) and Table 1 (Sec. 2). */
typedef struct {
    double eps; /* time-scale ratio of u and v, > 0 (+inf turns the reaction off) */
    double f;   /* stoichiometric coefficient, finite */
    double q;   /* propagation scaling factor, > 0 */
    double D_u; /* diffusion coefficient of u, >= 0 */
    double dt;  /* forward-Euler time step, > 0 */
    double dx;  /* grid spacing, > 0 */
} rdc_params;

/* Device planes owned by the caller and borrowed by the context for its whole
 * lifetime: two ping-pong copies of u and of v, and phi; one pitch (elements)
 * for all five. */
typedef struct {
    void *u[2];
    void *v[2];
    void *phi;
    int64_t pitch;
} rdc_buffers;

/* Create a context for an nx-by-ny grid (Sec. 2: one simulated reactor).
 * Checks the buffers (non-NULL, 256-byte aligned, pitch a multiple of 64 and
 * >= nx) and binds the current HIP device and `hip_stream`.  Parameters start
 * at Table 1 with phi from the caller's plane; the state is whatever the u[0]
 * and v[0] planes hold; the step counter is 0.
 * Errors: RDC_E_INVAL for nx or ny < 1, ny > 1048560 (the one-step kernel's
 * launch grid), a row of 2 GiB or more (pitch times the element size), a bad
 * buffer or a NULL `out`;
 * RDC_E_NOMEM / RDC_E_DEVICE if the small device status word cannot be made. */
rdc_status rdc_create(int32_t nx, int32_t ny, rdc_dtype dtype, const rdc_buffers *bufs,
                      void *hip_stream, rdc_ctx **out);

/* Release the context (never the caller's planes).  Waits for its stream.
 * NULL is accepted. */
rdc_status rdc_destroy(rdc_ctx *ctx);

/* Set eps, f, q, D_u, dt, dx (Eq. (1), Table 1; Sec. 3 notes they are meant
 * to be user-editable).  Errors, leaving the old values in place:
 * RDC_E_INVAL for eps <= 0 or NaN, non-finite f, q <= 0, D_u < 0, dt <= 0,
 * dx <= 0, or dt*D_u/dx^2 > 1/4 (the explicit-diffusion stability bound of
 * the five-node scheme). */
rdc_status rdc_set_params(rdc_ctx *ctx, const rdc_params *p);

/* Copy the excitability map phi (Sec. 3: active vs. passive substrate) from
 * `phi` (host or device, `pitch` elements per row, ctx dtype) into the
 * context's phi plane.  Errors: RDC_E_INVAL for NULL or pitch < nx. */
rdc_status rdc_set_phi(rdc_ctx *ctx, const void *phi, int64_t pitch, rdc_where where);

/* Replace the state (u, v) by the given planes (ctx dtype, `pitch` elements
 * per row), reset the non-finite flag, keep the step counter.  Used for
 * initial conditions (the medium's state before stimulation, Sec. 2) and to
 * resume from a snapshot (Sec. 3.1) taken by rdc_read.
 * Errors: RDC_E_INVAL for NULL or pitch < nx. */
rdc_status rdc_write(rdc_ctx *ctx, const void *u, const void *v, int64_t pitch,
                     rdc_where where);

/* Catalytic stimulation (Sec. 2): set u := 1.0 on every cell of each of the k
 * disks (host arrays cx[k], cy[k], r[k]; cx is the column), leave v alone.
 * Applied to the current state, between steps; cells outside the grid are
 * skipped.  If an arrival map is set, stimulated cells that have not arrived
 * get the current step index.  Errors: RDC_E_INVAL for k < 0, a NULL array
 * with k > 0, r < 0, or a disk that covers no cell of the grid. */
rdc_status rdc_stimulate(rdc_ctx *ctx, const int32_t *cx, const int32_t *cy,
                         const int32_t *r, int32_t k);

/* Advance the state by n >= 0 forward-Euler steps (Sec. 2; how many steps
 * pass between two renders is the simulation speed, Sec. 2).  Queued
 * asynchronously: the library launches ceil(n/T) kernels of near-equal length,
 * each taking up to T steps on chip (T from rdc_set_block).  Errors: RDC_E_INVAL for n < 0,
 * RDC_E_DEVICE if a launch fails.  Faults and the non-finite flag surface at
 * the next rdc_read or rdc_current. */
rdc_status rdc_step(rdc_ctx *ctx, int64_t n);

/* Snapshot (Sec. 3.1): wait for the stream, then copy the current u and v
 * into the given planes (host or device, `pitch` elements per row; either
 * pointer may be NULL to skip it).  Errors: RDC_E_INVAL for a bad pitch,
 * RDC_E_DEVICE for a device error, RDC_E_NONFINITE if any step produced a
 * non-finite value since the last rdc_write (the copy is still made). */
rdc_status rdc_read(rdc_ctx *ctx, void *u, void *v, int64_t pitch, rdc_where where);

/* Steps per launch: T in 1..12 (FP32) or 1..8 (FP64), or 0 to choose by grid
 * size (the default: 8 from 1024 x 1024 cells on, else 1).  A launch runs T
 * steps on chip between two visits to memory, as the app runs several steps
 * between two rendered frames (Sec. 2).  The result does not depend on T:
 * every variant of one precision computes each cell with the same expression
 * and gives bit-identical results (FP64 ones bit-identical to a plain C
 * evaluation of Eq. (1)).  Errors: RDC_E_INVAL outside 0..12 (FP32) or 0..8
 * (FP64). */
rdc_status rdc_set_block(rdc_ctx *ctx, int32_t T);

/* How launches of several steps are laid out on chip (the result does not
 * depend on it): 0 (auto: LDS tiles of 56 rows), one of the LDS tile heights
 * 48, 56, 64, 80, or RDC_TILE_STREAM: every wave walks a strip of 256
 * (FP32) or 128 (FP64) columns down a segment of rows, carrying all T steps
 * of each row in registers (FP32 T = 2..11, and 12 on grids whose width is
 * a multiple of 4 and at least 256; FP64 T = 2..8; other launches, and those
 * with an arrival map or timelapse attached, use 56-row tiles).  The Python
 * autotuner times the choices on the grid's shape.  Errors: RDC_E_INVAL. */
#define RDC_TILE_STREAM 1
rdc_status rdc_set_tile_rows(rdc_ctx *ctx, int32_t rows);

/* Non-zero if `rows` is a value rdc_set_tile_rows accepts (other than 0). */
int32_t rdc_tile_rows_supported(int32_t rows);

/* Device addresses of the planes that hold the current u and v: a zero-copy
 * view of the state at a step boundary, the device-side form of the
 * snapshot of Sec. 3.1 (valid until the next rdc_step or rdc_write).  Like
 * rdc_read it waits for the stream and reports what the queued work left:
 * RDC_E_DEVICE for a device error, RDC_E_NONFINITE if any step produced a
 * non-finite value since the last rdc_write; the addresses are stored in
 * both cases.  Errors: RDC_E_INVAL for NULL outputs. */
rdc_status rdc_current(rdc_ctx *ctx, void **u_dev, void **v_dev);

/* Attach (or, with NULL, detach) a caller-owned int32 device plane that
 * records for each cell the first step index at which u >= theta (the
 * wave-front arrival time); cells that have not arrived hold INT32_MAX.
 * Attaching initialises the plane from the current state.  `pitch` must be a
 * multiple of 64 and >= nx.  FP32 and FP64 contexts both support it.
 * Errors: RDC_E_INVAL for a bad pitch or alignment. */
rdc_status rdc_set_arrival(rdc_ctx *ctx, int32_t *arrival_dev, int64_t pitch, double theta);

/* Timelapse (Sec. 3.1: u recorded over time at a user-set rate, shown over
 * the static substrate).  Attach (or, with NULL, detach) a caller-owned
 * device plane of the context's precision that holds the maximum of u over
 * the recorded frames: attaching copies the current u into it (the first
 * frame), and after every step that leaves a step index that is a multiple
 * of `rate`, each cell takes max(plane, u).  Fused into the stepping
 * kernels' epilogue (like the arrival map), so no frame is copied out.
 * `pitch` must be a multiple of 64 and >= nx; the plane 256-byte aligned.
 * Errors: RDC_E_INVAL for rate < 1, a bad pitch or alignment. */
rdc_status rdc_set_timelapse(rdc_ctx *ctx, void *timelapse_dev, int64_t pitch, int32_t rate);

/* Number of steps taken since rdc_create.  Errors: RDC_E_INVAL for NULL. */
rdc_status rdc_get_step(const rdc_ctx *ctx, int64_t *step);

/* Set the step counter, to resume a run from a snapshot (Sec. 3.1) taken at
 * that step: arrival times and timelapse frames continue from it.  The state
 * itself comes from rdc_write.  Errors: RDC_E_INVAL for NULL or a step
 * outside 0 .. INT32_MAX - 8. */
rdc_status rdc_set_step(rdc_ctx *ctx, int64_t step);

/* Message of the last failed call on ctx ("" if none); with ctx == NULL the
 * last failure of rdc_create.  The string is owned by the library. */
const char *rdc_last_error(const rdc_ctx *ctx);

/* Device-to-device copy of `nbytes` bytes (a multiple of 16; both pointers
 * 16-byte aligned; regions must not overlap) by a plain streaming kernel
 * queued on `hip_stream`.  It is the measured HBM-bandwidth ceiling that the
 * stepper kernels are compared with.  Errors: RDC_E_INVAL for bad arguments
 * (message via rdc_last_error(NULL)), RDC_E_DEVICE if the launch fails. */
rdc_status rdc_copy(void *dst, const void *src, int64_t nbytes, void *hip_stream);

/* Short name of a status code. */
const char *rdc_status_string(rdc_status s);


/* ------------------------------------------------------------------------
 * Batched simulations: many independent grids, each with its own size,
 * parameters and phi map (parameter sweeps and circuit variants, the paper's
 * reproducibility aim of Sec. 1 and Sec. 5), advanced together: one launch
 * covers every tile of every grid, and small grids run whole in LDS (see
 * rdc_batch_set_resident).  FP32 only; the per-cell update is the same as
 * rdc_step's, so each grid evolves bit-identically to a single context.
 * ------------------------------------------------------------------------ */
typedef struct rdc_batch rdc_batch; /* opaque */
typedef struct rdc_graph rdc_graph; /* opaque: a recorded sequence of launches */

/* One simulation of a batch.  Its planes live inside the batch's pool
 * planes: elements [offset, offset + pitch*ny) of each of u[0], u[1], v[0],
 * v[1] and phi.  pitch and offset are multiples of 64 elements; the regions
 * of different simulations must not overlap. */
typedef struct {
    int32_t nx, ny;
    int64_t pitch;
    int64_t offset;
    rdc_params params; /* Eq. (1) parameters of this simulation (checked as in rdc_set_params) */
} rdc_sim_desc;

/* Create a batch of `count` >= 1 simulations over caller-owned FP32 pool
 * planes of `pool_elems` elements each (pool->pitch is ignored), bound to
 * `hip_stream`.  Copies the descriptors (host array); allocates a small
 * device table and one status word per simulation.  The state of each
 * simulation is whatever its region of u[0], v[0] holds.  Errors:
 * RDC_E_INVAL for count < 1, bad sizes, pitches, offsets, overlaps,
 * misaligned pool planes or bad parameters (message via
 * rdc_last_error(NULL)); RDC_E_NOMEM / RDC_E_DEVICE for device setup. */
rdc_status rdc_batch_create(int32_t count, const rdc_sim_desc *sims, const rdc_buffers *pool,
                            int64_t pool_elems, void *hip_stream, rdc_batch **out);

/* Release the batch (not the pool).  Waits for its stream.  NULL accepted. */
rdc_status rdc_batch_destroy(rdc_batch *b);

/* Steps per launch (1..12, default 8) and tile rows (48, 56 or 64, default
 * 56) of the batched kernel, or rows = RDC_TILE_STREAM with T in 1..11: the
 * tiled grids then run on row pipelines (one wave per strip of a grid and
 * segment of its rows, the segment heights planned over all grids so that
 * every wave's work is about equal; launches of one step take 56-row
 * tiles).  Does not change results.  RDC_E_INVAL outside these values. */
rdc_status rdc_batch_set_block(rdc_batch *b, int32_t T, int32_t rows);

/* Whole-grid path for small grids (same scheme, Sec. 2 Eq. (1)): a grid of
 * at most max_cells cells whose shape fits one workgroup (nx <= 1024 and
 * ceil(ny / floor(1024 / nx)) <= 16 rows per thread; every 128 x 128 grid
 * does) is read once per rdc_batch_step call, advanced through all n steps
 * in LDS and registers by one workgroup (one barrier per step, no HBM
 * traffic in between) and written back once.  These launches run on a
 * second stream of the batch, forked from its stream before the tiled
 * grids' launches and joined into it after (so captures record them too).
 * max_cells = 0 turns the path off; the default is
 * RDC_BATCH_RESIDENT_DEFAULT (128 x 128).  Does not change results.  Waits
 * for the batch's stream; a graph captured before the call refers to the
 * old plan and its rdc_graph_launch returns RDC_E_STATE.  Errors:
 * RDC_E_INVAL for max_cells < 0; RDC_E_NOMEM / RDC_E_DEVICE for the item
 * table. */
#define RDC_BATCH_RESIDENT_DEFAULT 16384
rdc_status rdc_batch_set_resident(rdc_batch *b, int32_t max_cells);

/* Number of grids the whole-grid path takes under the current setting (-1
 * for NULL). */
int32_t rdc_batch_resident_count(const rdc_batch *b);

/* Copy phi of simulation `sim` (ny rows of `pitch` elements, host or
 * device).  Errors: RDC_E_INVAL for a bad index, NULL or pitch < nx. */
rdc_status rdc_batch_set_phi(rdc_batch *b, int32_t sim, const void *phi, int64_t pitch,
                             rdc_where where);

/* Replace the state of simulation `sim` and clear its non-finite flag. */
rdc_status rdc_batch_write(rdc_batch *b, int32_t sim, const void *u, const void *v,
                           int64_t pitch, rdc_where where);

/* Catalytic stimulation (Sec. 2) of k disks: disk j hits simulation sim[j]
 * (host arrays).  Errors as rdc_stimulate, plus a bad simulation index. */
rdc_status rdc_batch_stimulate(rdc_batch *b, const int32_t *sim, const int32_t *cx,
                               const int32_t *cy, const int32_t *r, int32_t k);

/* Advance every simulation by n >= 0 steps (asynchronous, like rdc_step). */
rdc_status rdc_batch_step(rdc_batch *b, int64_t n);

/* Snapshot of simulation `sim` (waits for the stream); RDC_E_NONFINITE if
 * that simulation produced a non-finite value since its last write. */
rdc_status rdc_batch_read(rdc_batch *b, int32_t sim, void *u, void *v, int64_t pitch,
                          rdc_where where);

/* Record the launches of rdc_batch_step(b, n) into a HIP graph instead of
 * running them; rdc_graph_launch then replays all of them as one submission
 * on the batch's stream and advances the batch by n steps each time.  The
 * recording always holds an even number of launches (one launch is split if
 * needed) and is made once from each ping-pong copy of the planes; a replay
 * runs the one that starts from the copy holding the current state, so
 * eager rdc_batch_step calls may come between replays; n must be >= 2.
 * The graph refers to the batch, which must outlive it, and to its launch
 * plan: after rdc_batch_set_resident, rdc_graph_launch returns RDC_E_STATE.
 * Errors: RDC_E_INVAL for n < 2 or NULL; RDC_E_DEVICE if capture fails. */
rdc_status rdc_batch_capture(rdc_batch *b, int64_t n, rdc_graph **out);
rdc_status rdc_graph_launch(rdc_graph *g);
rdc_status rdc_graph_destroy(rdc_graph *g);

/* Device addresses (inside the pool planes) of the u and v planes that hold
 * the batch's current state (valid until the next step).  Errors:
 * RDC_E_INVAL for NULL outputs. */
rdc_status rdc_batch_current(rdc_batch *b, void **u_pool, void **v_pool);

/* Message of the last failed call on b ("" if none). */
const char *rdc_batch_last_error(const rdc_batch *b);

/* ------------------------------------------------------------------------
 * Learned coarse stepper: the kernels a 3x3-convolution U-Net needs to be
 * trained and run on the GPU next to the plain stepper (a surrogate that
 * advances (u, v, phi) by K steps; the plain forward-Euler stepper of Sec. 2
 * stays the reference check and the fallback).  Activations are NHWC bfloat16 stored
 * as 16-bit words, with a pixel stride `ld` (elements) so a layer can read
 * or write a channel slice of a concatenation buffer; weights of a layer are
 * [9][cout][cin] (tap = 3*(dy+1) + (dx+1)), bf16 for the convolution and fp32
 * masters for training.  All calls queue work on `stream` and return at once;
 * argument errors return RDC_E_INVAL with a message in rdc_nn_last_error().
 * ------------------------------------------------------------------------ */

/* 3x3 "same" convolution (zero padding) on the matrix cores: bf16 operands,
 * fp32 accumulation, + bias (fp32, optional: NULL), optional ReLU, bf16
 * output of channels [0, cout_store).  Requires w % 32 == 0, cin % 16 == 0,
 * cout in {32, 64, 96, 128, 192, 256}, ldx % 8 == 0, ldy % 4 == 0, x and w 16-byte
 * aligned, y 8-byte aligned. */
rdc_status rdc_nn_conv3x3(const void *x, int32_t ldx, const void *w, const float *bias, void *y,
                          int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin,
                          int32_t cout, int32_t cout_store, int32_t relu, void *stream);

/* rdc_nn_conv3x3 (bias added, ReLU applied) on a concatenation whose first
 * up_c channels are the nearest 2x upsampling of a half-resolution tensor
 * `xu` (n x h/2 x wd/2 pixels, stride ldu) and whose channels [up_c, cin)
 * are channels [up_c, cin) of x (stride ldx): the decoder step of a U-Net,
 * with the upsampled part read straight from the coarse level instead of
 * being written out first.  Bit-identical to rdc_nn_up2 into channels
 * [0, up_c) of x followed by rdc_nn_conv3x3.  Requires h even, wd % 64 == 0,
 * up_c a multiple of 32 in 32..cin, cout in {32, 64, 128}, ldu % 8 == 0, xu
 * 16-byte aligned; channels [0, up_c) of x are not read. */
rdc_status rdc_nn_conv3x3_up(const void *x, int32_t ldx, const void *xu, int32_t ldu,
                             int32_t up_c, const void *w, const float *bias, void *y,
                             int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin,
                             int32_t cout, int32_t cout_store, void *stream);

/* rdc_nn_conv3x3 (bias added, ReLU applied) whose input is built while it is
 * loaded from the stepper planes u, v, phi (fp32, row pitch `pitch`, image i
 * at i*plane_stride): channels bf16(su u), bf16(sv v), bf16(sp phi), zeros
 * up to cin -- the network's first layer without the input tensor.
 * Bit-identical to rdc_nn_prep followed by rdc_nn_conv3x3.  Requires
 * cin in {16, 32}, cout in {32, 64, 128}, pitch >= wd, plane_stride >=
 * pitch*h. */
rdc_status rdc_nn_conv3x3_planes(const float *u, const float *v, const float *phi,
                                 int64_t pitch, int64_t plane_stride, float su, float sv,
                                 float sp, const void *w, const float *bias, void *y,
                                 int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin,
                                 int32_t cout, int32_t cout_store, void *stream);

/* The network's head and the prediction in one launch: rdc_nn_conv3x3 with
 * 32 output channels, bias, no ReLU, whose outputs are not stored; instead
 * each pixel's first two (bf16-rounded) outputs go through rdc_nn_apply:
 * uo = clamp(u + out0/su, 0, 1), vo = clamp(v + out1/sv, 0, (cmax - phi)/f)
 * on the fp32 planes (row pitch `pitch`, image i at i*plane_stride).
 * Bit-identical to rdc_nn_conv3x3 into a head tensor followed by
 * rdc_nn_apply; uo, vo may alias u, v. */
rdc_status rdc_nn_conv3x3_apply(const void *x, int32_t ldx, const void *w, const float *bias,
                                const float *u, const float *v, const float *phi, int64_t pitch,
                                int64_t plane_stride, float *uo, float *vo, int32_t n, int32_t h,
                                int32_t wd, int32_t cin, float su, float sv, float f, float cmax,
                                void *stream);

/* Weights of the input-gradient convolution: wd[tap][ci][co] =
 * bf16(w[8 - tap][co][ci]); rdc_nn_conv3x3 with them (cin <-> cout, no bias,
 * no ReLU) on the output gradient gives the input gradient. */
rdc_status rdc_nn_dgrad_weights(const float *w, void *wd, int32_t cout, int32_t cin, void *stream);

/* Floats of scratch rdc_nn_conv3x3_wgrad needs for this shape (the weight
 * and bias partials of every pixel chunk). */
int64_t rdc_nn_wgrad_scratch_floats(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout);

/* Weight gradient grad[9][cout][cin] (fp32) = sum over pixels of
 * dy[p][co] * x[p + tap offset][ci], and, when gbias is not NULL, the bias
 * gradient gbias[co] = sum over pixels of dy[p][co].  Deterministic: each
 * chunk of pixels writes its partials to `scratch`, which are then summed in
 * a fixed order.  Requires cin, cout % 32 == 0, w % 32 == 0, ldx and lddy
 * multiples of 8, x and dy 16-byte aligned. */
rdc_status rdc_nn_conv3x3_wgrad(const void *x, int32_t ldx, const void *dy, int32_t lddy,
                                float *scratch, float *grad, float *gbias, int32_t n, int32_t h,
                                int32_t w, int32_t cin, int32_t cout, void *stream);

/* rdc_nn_conv3x3_wgrad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid allocation): the same kernels and results, with the partials in a
 * static device array of the library instead of a caller's `scratch` (one
 * array per GPU, rdc_nn_wgrad_static_floats() floats = 32 MiB, held until
 * the process ends).  Allocates nothing and needs no clearing (every partial
 * a call sums is written by that call first).  Calls on one GPU share the
 * array: calls that overlap in time there (e.g. on two streams) race and give
 * wrong gradients; calls queued on one stream are ordered and safe.
 * Errors: as rdc_nn_conv3x3_wgrad, plus RDC_E_INVAL when the shape needs
 * more than rdc_nn_wgrad_static_floats() floats of workspace
 * (rdc_nn_wgrad_scratch_floats), RDC_E_DEVICE if the array's address cannot
 * be had. */
rdc_status rdc_nn_conv3x3_wgrad_noalloc(const void *x, int32_t ldx, const void *dy, int32_t lddy,
                                        float *grad, float *gbias, int32_t n, int32_t h,
                                        int32_t w, int32_t cin, int32_t cout, void *stream);

/* Floats of workspace the static scratch of rdc_nn_conv3x3_wgrad_noalloc holds. */
int64_t rdc_nn_wgrad_static_floats(void);

/* dst = bf16(src), n elements. */
rdc_status rdc_nn_to_bf16(const float *src, void *dst, int64_t n, void *stream);

/* ReLU adjoint in place: g[p][c] = 0 where y[p][c] <= 0. */
rdc_status rdc_nn_relu_bwd(void *g, int32_t ldg, const void *y, int32_t ldy, int64_t pixels,
                           int32_t c, void *stream);

/* 2x2 average pooling to (ho, wo) and its adjoint (accumulate != 0 adds into gin). */
rdc_status rdc_nn_pool2(const void *in, int32_t ldi, void *out, int32_t ldo, int32_t n, int32_t ho,
                        int32_t wo, int32_t c, void *stream);
rdc_status rdc_nn_pool2_bwd(const void *gout, int32_t ldo, void *gin, int32_t ldi, int32_t n,
                            int32_t ho, int32_t wo, int32_t c, int32_t accumulate, void *stream);

/* Nearest 2x upsampling to (ho, wo) and its adjoint (from (2hi, 2wi) to (hi, wi)). */
rdc_status rdc_nn_up2(const void *in, int32_t ldi, void *out, int32_t ldo, int32_t n, int32_t ho,
                      int32_t wo, int32_t c, void *stream);
rdc_status rdc_nn_up2_bwd(const void *gout, int32_t ldo, void *gin, int32_t ldi, int32_t n,
                          int32_t hi, int32_t wi, int32_t c, void *stream);

/* Network input from stepper planes (fp32, row pitch `pitch`, image i at
 * i*plane_stride): channels (su u, sv v, sp phi), zeros up to c. */
rdc_status rdc_nn_prep(const float *u, const float *v, const float *phi, int64_t pitch,
                       int64_t plane_stride, void *x, int32_t c, int32_t n, int32_t h, int32_t w,
                       float su, float sv, float sp, void *stream);

/* Prediction, projected onto the states the explicit stepper can continue
 * from: uo = clamp(u + head[.,0]/su, 0, 1) (the box 0 <= u <= 1 is invariant
 * under the flow of Eq. (1)) and vo = clamp(v + head[.,1]/sv, 0, (cmax -
 * phi)/f).  With a = dt (f v + phi) / eps, one forward-Euler step from any
 * u >= 0 stays above the pole at u = -q of the reaction term iff a < 8 q
 * (minimum over s = u + q of s - a + 2 a q / s); so cmax = 8 q eps / dt,
 * less a margin for the diffusion term, is the caller's choice.  phi has the
 * layout of u.  uo, vo may alias u, v. */
rdc_status rdc_nn_apply(const float *u, const float *v, const float *phi, const void *head,
                        int32_t ldh, int64_t pitch, int64_t plane_stride, float *uo, float *vo,
                        int32_t n, int32_t h, int32_t w, float su, float sv, float f, float cmax,
                        void *stream);

/* Number of per-block loss partials rdc_nn_loss writes for `pixels` pixels;
 * `partial` must hold one float more (the total). */
int32_t rdc_nn_loss_blocks(int64_t pixels);

/* Front-weighted squared error of the head against the scaled increments
 * (su (ut - u), sv (vt - v)), weight 1 + front_w where u or ut crosses
 * theta, mean over pixels; writes its gradient into g (channels 0, 1; the
 * rest of ldg zero), per-block partial sums into partial[0 .. nb) and the
 * loss (their sum, fixed order) into partial[nb], nb = rdc_nn_loss_blocks. */
rdc_status rdc_nn_loss(const float *u, const float *v, const float *ut, const float *vt,
                       int64_t pitch, int64_t plane_stride, const void *head, int32_t ldh,
                       void *g, int32_t ldg, int32_t n, int32_t h, int32_t w, float su, float sv,
                       float theta, float front_w, float *partial, void *stream);

/* Adam step on fp32 parameters (gradient clipped to +-clip; lr_t includes
 * the bias corrections). */
rdc_status rdc_nn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr_t,
                       float b1, float b2, float eps, float clip, void *stream);

/* Front check between two u planes (fp32, row pitch `pitch`): adds to
 * *count (device) the number of cells where one side is >= theta and no
 * cell of the other side's 3x3 neighbourhood is.  Zero means the fronts agree
 * to within one cell: the coarse stepper's front-error criterion. */
rdc_status rdc_nn_front_check(const float *a, const float *b, int64_t pitch, int32_t nx, int32_t ny,
                              float theta, uint32_t *count, void *stream);

/* State check: adds to *count (device) the number of cells the explicit
 * stepper of Eq. (1) cannot be trusted to continue from: u or v NaN, u
 * outside [ulo, uhi], or f v + phi > cmax.  With ulo = -q (the reaction
 * term's pole) and cmax = 8 q eps / dt (see rdc_nn_apply), zero means one
 * Euler step from every cell stays finite and above the pole. */
rdc_status rdc_nn_state_check(const float *u, const float *v, const float *phi, int64_t pitch,
                              int32_t nx, int32_t ny, float ulo, float uhi, float f, float cmax,
                              uint32_t *count, void *stream);

/* Message of the last failed rdc_nn_* call of this thread. */
const char *rdc_nn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RDC_H */
