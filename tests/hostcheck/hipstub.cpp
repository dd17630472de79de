// Stand-in HIP runtime for a CPU run of the library's host logic under ASan:
// "device" memory is host memory, kernels are not run, events/graphs are
// tracked objects so a use after destroy or a double destroy is caught.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <vector>
#include <mutex>
#include <hip/hip_runtime_api.h>

static std::mutex mu;
static std::set<void*> live_events, live_graphs, live_execs;
static void die(const char* m, void* p) { std::fprintf(stderr, "STUB ERROR: %s %p\n", m, p); std::abort(); }
struct Graph { std::vector<void*> nodes; };

extern "C" {
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memmove(d, s, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { *p = std::calloc(1, n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void*) { std::memset(a, 0, sizeof *a); a->type = hipMemoryTypeDevice; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int d) { if (d != 0) die("set device", nullptr); return hipSuccess; }
// the library's static device arrays: one host block stands in for each symbol
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    static std::vector<char> block(2u << 20);
    if (!sym) die("null symbol", nullptr);
    *p = block.data(); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { std::lock_guard<std::mutex> l(mu); *e = (hipEvent_t) new int(1); live_events.insert(*e); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { std::lock_guard<std::mutex> l(mu); if (!live_events.erase(e)) die("event destroy", e); delete (int*)e; return hipSuccess; }
static void chk_ev(hipEvent_t e) { std::lock_guard<std::mutex> l(mu); if (e && !live_events.count(e)) die("dead event", e); }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { chk_ev(e); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t e) { chk_ev(e); return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) { chk_ev(a); chk_ev(b); *ms = 0.01f; return hipSuccess; }
hipError_t hipExtLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t, hipStream_t, hipEvent_t e0, hipEvent_t e1, int) {
    chk_ev(e0); chk_ev(e1); if (!f || !args || g.x == 0 || b.x == 0 || b.x > 1024) die("bad launch", (void*)f); return hipSuccess; }
hipError_t hipLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t, hipStream_t) {
    if (!f || g.x == 0 || b.x == 0 || b.x > 1024) die("bad launch", (void*)f); (void)args; return hipSuccess; }
hipError_t hipGraphCreate(hipGraph_t* g, unsigned) { std::lock_guard<std::mutex> l(mu); *g = (hipGraph_t) new Graph(); live_graphs.insert(*g); return hipSuccess; }
hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t* deps, size_t nd, const hipKernelNodeParams* p) {
    std::lock_guard<std::mutex> l(mu);
    if (!live_graphs.count(g)) die("dead graph", g);
    Graph* G = (Graph*)g;
    for (size_t i = 0; i < nd; ++i) { bool ok = false; for (void* x : G->nodes) ok |= x == (void*)deps[i]; if (!ok) die("foreign dep", deps[i]); }
    if (!p->func || p->gridDim.x == 0 || p->blockDim.x == 0) die("bad node", (void*)p->func);
    void* node = new int(0); G->nodes.push_back(node); *n = (hipGraphNode_t)node; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    std::lock_guard<std::mutex> l(mu); if (!live_graphs.count(g)) die("dead graph", g); *e = (hipGraphExec_t) new int(2); live_execs.insert(*e); return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) { std::lock_guard<std::mutex> l(mu); if (!live_execs.count(e)) die("dead exec", e); return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { std::lock_guard<std::mutex> l(mu); if (!live_execs.erase(e)) die("exec destroy", e); delete (int*)e; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { std::lock_guard<std::mutex> l(mu); if (!live_graphs.erase(g)) die("graph destroy", g);
    Graph* G = (Graph*)g; for (void* x : G->nodes) delete (int*)x; delete G; return hipSuccess; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
void** __hipRegisterFatBinary(const void*) { static void* h = nullptr; return &h; }
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*, void*, void*, int*) {}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, void*, char*, const char*, int, size_t, int, int) {}
hipError_t __hipPushCallConfiguration(dim3, dim3, size_t, hipStream_t) { return hipSuccess; }
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* s, hipStream_t* st) { *g = dim3(1); *b = dim3(1); *s = 0; *st = nullptr; return hipSuccess; }
}
