/* Host-memory stand-in for the HIP runtime calls librdc's host code makes,
 * so that code (argument checks, launch planning, copies, batch tables,
 * graph recording) can run on a machine without a GPU under AddressSanitizer
 * and UBSan.  "Device" allocations are host allocations, copies are memcpy,
 * kernel launches are recorded (grid, block) and not run.  Types are
 * restated with the HIP C ABI's layout (hipError_t an int-sized enum, dim3
 * three unsigned ints, handles pointers). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef int hipError_t;
typedef struct { unsigned x, y, z; } dim3;
typedef void *hipStream_t;
typedef void *hipGraph_t;
typedef void *hipGraphExec_t;

enum { ok = 0, invalid_value = 1, invalid_config = 9 };

static long n_launch, n_bad_launch, n_alloc, n_free;
static dim3 cfg_grid, cfg_block;
static int capturing;

long shim_launches(void) { return n_launch; }
long shim_bad_launches(void) { return n_bad_launch; }
long shim_live_allocations(void) { return n_alloc - n_free; }

hipError_t hipGetDevice(int *d) { *d = 0; return ok; }
hipError_t hipSetDevice(int d) { return d == 0 ? ok : invalid_value; }
hipError_t hipDeviceGetAttribute(int *v, int attr, int dev) {
    (void)attr; (void)dev;
    *v = 256;                                   /* compute units of the target chip */
    return ok;
}
hipError_t hipMalloc(void **p, size_t n) {
    if (posix_memalign(p, 256, n ? n : 1) != 0) return 2;
    memset(*p, 0, n);
    ++n_alloc;
    return ok;
}
hipError_t hipFree(void *p) {
    if (p) { free(p); ++n_free; }
    return ok;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, int kind) {
    (void)kind;
    memmove(dst, src, n);
    return ok;
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch,
                            size_t width, size_t height, int kind, hipStream_t s) {
    (void)kind; (void)s;
    if (width > dpitch || width > spitch) return invalid_value;
    for (size_t r = 0; r < height; ++r)
        memmove((char *)dst + r * dpitch, (const char *)src + r * spitch, width);
    return ok;
}
hipError_t hipStreamSynchronize(hipStream_t s) { (void)s; return ok; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags) {
    (void)flags;
    *s = malloc(16);
    return ok;
}
hipError_t hipStreamDestroy(hipStream_t s) { free(s); return ok; }
typedef void *hipEvent_t;
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags) {
    (void)flags;
    *e = malloc(16);
    return ok;
}
hipError_t hipEventDestroy(hipEvent_t e) { free(e); return ok; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) { (void)s; return e ? ok : invalid_value; }
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags) {
    (void)s; (void)flags;
    return e ? ok : invalid_value;
}
hipError_t hipStreamBeginCapture(hipStream_t s, int mode) {
    (void)s; (void)mode;
    capturing = 1;
    return ok;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    (void)s;
    capturing = 0;
    *g = malloc(16);
    return ok;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *node, char *log, size_t n) {
    (void)g; (void)node; (void)log; (void)n;
    *e = malloc(16);
    return ok;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) { (void)e; (void)s; return ok; }
hipError_t hipGraphDestroy(hipGraph_t g) { free(g); return ok; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); return ok; }
hipError_t hipGetLastError(void) { return ok; }
const char *hipGetErrorString(hipError_t e) { return e == ok ? "no error" : "shim error"; }

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shmem, hipStream_t s) {
    (void)shmem; (void)s;
    cfg_grid = g;
    cfg_block = b;
    return ok;
}
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *shmem, hipStream_t *s) {
    *g = cfg_grid;
    *b = cfg_block;
    *shmem = 0;
    *s = NULL;
    return ok;
}
hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **args, size_t shmem,
                           hipStream_t s) {
    (void)f; (void)args; (void)shmem; (void)s;
    ++n_launch;
    const uint64_t threads = (uint64_t)b.x * b.y * b.z;
    if (g.x == 0 || g.y == 0 || g.z == 0 || threads == 0 || threads > 1024 ||
        g.y > 65535 || g.z > 65535) {
        ++n_bad_launch;
        fprintf(stderr, "bad launch: grid %u %u %u block %u %u %u\n", g.x, g.y, g.z, b.x, b.y,
                b.z);
        return invalid_config;
    }
    return ok;
}

static char shim_module;
void **__hipRegisterFatBinary(const void *data) { (void)data; return (void **)&shim_module; }
void __hipRegisterFunction(void **m, const void *h, char *d, const char *n, unsigned t, void *a,
                           void *b, void *c, void *e, int *w) {
    (void)m; (void)h; (void)d; (void)n; (void)t; (void)a; (void)b; (void)c; (void)e; (void)w;
}
void __hipUnregisterFatBinary(void **m) { (void)m; }
/* A __device__ variable: its host shadow stands in for the device copy. */
void __hipRegisterVar(void **m, void *var, char *host_var, char *dev_var, int ext, size_t size,
                      int constant, int global) {
    (void)m; (void)var; (void)host_var; (void)dev_var; (void)ext; (void)size; (void)constant;
    (void)global;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
    *p = (void *)symbol;
    return ok;
}
