// Host-only stand-in for the HIP runtime, for CPU tests of the library's host
// logic.  It takes the soname and symbol versions of the real runtime so that
// libfic.so binds to it through LD_LIBRARY_PATH.  Device memory is host
// memory, copies are memcpy, events are inert, and kernel launches are not
// run: each one is checked for a legal grid and handed to a hook that the
// test installs (kernel name, grid, block, argument pointers).
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

extern "C" {
typedef void (*mock_hook_t)(const char *name, unsigned grid, unsigned block, void **args);

static dim3 g_grid, g_block;
static size_t g_shm;
static hipStream_t g_stream;
static std::map<const void *, std::string> *g_names;
static mock_hook_t g_hook;
static long g_launches, g_captured, g_replays;
static int g_capturing;

void mock_set_hook(mock_hook_t h) { g_hook = h; }
long mock_launches() { return g_launches; }

void **__hipRegisterFatBinary(const void *) {
    static void *handle[4];
    return handle;
}
void __hipRegisterFunction(void **, const void *host_fn, char *device_fn, const char *, unsigned int, void *,
                           void *, dim3 *, dim3 *, int *) {
    if (!g_names) g_names = new std::map<const void *, std::string>();
    (*g_names)[host_fn] = device_fn;
}
void __hipUnregisterFatBinary(void **) {}
// A __device__ variable: the host shadow the runtime registers stands in for
// the device copy (device memory is host memory here).
static std::map<const void *, size_t> *g_vars;
void __hipRegisterVar(void **, void *var, char *, char *, int, size_t size, int, int) {
    if (!g_vars) g_vars = new std::map<const void *, size_t>();
    (*g_vars)[var] = size;
}
hipError_t hipGetSymbolAddress(void **dev, const void *symbol) {
    if (!g_vars || !g_vars->count(symbol)) return hipErrorInvalidSymbol;
    *dev = const_cast<void *>(symbol);
    return hipSuccess;
}
// Calls that allocate memory or runtime objects, counted for the tests of the
// allocation-free entry point.
static long g_allocs;
long mock_allocs() { return g_allocs; }
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, hipStream_t st) {
    g_grid = grid;
    g_block = block;
    g_shm = shm;
    g_stream = st;
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shm, hipStream_t *st) {
    *grid = g_grid;
    *block = g_block;
    *shm = g_shm;
    *st = g_stream;
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void *f, dim3 grid, dim3 block, void **args, size_t, hipStream_t) {
    const char *name = (g_names && g_names->count(f)) ? (*g_names)[f].c_str() : "?";
    if (grid.x == 0 || grid.x > 0x7fffffffu || grid.y != 1 || grid.z != 1 || block.x == 0 || block.x > 1024) {
        fprintf(stderr, "illegal launch of %s: grid %u block %u\n", name, grid.x, block.x);
        abort();
    }
    ++g_launches;
    if (g_capturing) ++g_captured;
    if (g_hook) g_hook(name, grid.x, block.x, args);
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
    ++g_allocs;
    *e = (hipEvent_t)malloc(16);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    ++g_allocs;
    *e = (hipEvent_t)malloc(16);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    free(e);
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 0.f;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipFree(void *p) {
    ++g_allocs;
    free(p);
    return hipSuccess;
}
hipError_t hipGetDeviceCount(int *n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *p, int) {
    memset(p, 0, sizeof(*p));
    strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
    p->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipHostFree(void *p) {
    ++g_allocs;
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) {
    ++g_allocs;
    *p = malloc(n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipMalloc(void **p, size_t n) {
    ++g_allocs;
    *p = aligned_alloc(256, (n + 255) / 256 * 256 + 256);
    if (*p) memset(*p, 0xA5, n);  // device memory starts as garbage
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
    memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
// Resident workgroups per CU of any kernel: persistent grids then hold 512.
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t) {
    *n = 2;
    return hipSuccess;
}

// Streams and graphs: launches during a capture are checked like any other
// and counted as captured; a graph launch only counts a replay.
long mock_captured() { return g_captured; }
long mock_replays() { return g_replays; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    ++g_allocs;
    *s = (hipStream_t)malloc(16);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    free(s);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
    if (g_capturing) return hipErrorInvalidValue;
    g_capturing = 1;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    if (!g_capturing) return hipErrorInvalidValue;
    g_capturing = 0;
    *g = (hipGraph_t)malloc(16);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, hipGraphNode_t *, char *, size_t) {
    *e = (hipGraphExec_t)malloc(16);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) {
    ++g_replays;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    free(e);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    free(g);
    return hipSuccess;
}
}
