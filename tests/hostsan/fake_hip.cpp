// CPU stand-in for the HIP runtime and the kernel launchers, so that the host
// code of the library (aqc_host.cpp) runs under AddressSanitizer or
// ThreadSanitizer without a GPU.  "Device" memory is zeroed host memory, kernels do nothing (reductions
// return 1, diagonal ranges [-1, 3]), and every allocation, stream, event and
// graph is tracked: a free or use of an unknown handle aborts, and ranges a
// launcher is given must lie inside the allocation they start in.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
// the stand-in is used from several host threads: one lock for all of it (the
// real runtime is thread-safe, so only the library's own state can race)
static std::recursive_mutex g_mu;
#define FAKE_LOCK std::lock_guard<std::recursive_mutex> fake_lock_(g_mu)
#include "../../paper_1311_3938_amd/csrc/aqc_internal.h"

static std::map<void*, size_t> g_dev, g_host;
static std::set<void*> g_obj;
// the stream each event was last recorded on, and the events whose stream has
// since been destroyed: the library never waits on or queries those
static std::map<void*, void*> g_ev_stream;
static std::set<void*> g_ev_orphan;
static void die(const char* what, void* p) { FAKE_LOCK;
  fprintf(stderr, "fake_hip: %s %p\n", what, p);
  abort();
}
static void* newobj() { FAKE_LOCK;
  void* p = malloc(64);
  g_obj.insert(p);
  return p;
}
static void delobj(void* p, const char* what) { FAKE_LOCK;
  if (!p) return;
  if (!g_obj.erase(p)) die(what, p);
  free(p);
}
struct FakeGraph {
  void* dst = nullptr;
  const void* src = nullptr;
  size_t n = 0;
};
static std::set<void*> g_graphs, g_execs;

extern "C" {
hipError_t hipDeviceGetAttribute(int* pi, hipDeviceAttribute_t, int) { FAKE_LOCK; *pi = 160 * 1024; return hipSuccess; }
hipError_t hipDeviceSynchronize(void) { FAKE_LOCK; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { FAKE_LOCK; *e = (hipEvent_t)newobj(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { FAKE_LOCK; *e = (hipEvent_t)newobj(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { FAKE_LOCK;
  g_ev_stream.erase((void*)e);
  g_ev_orphan.erase((void*)e);
  delobj((void*)e, "event destroy");
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { FAKE_LOCK; *ms = 1.0f; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) { FAKE_LOCK;
  if (!g_obj.count((void*)e)) die("event record", (void*)e);
  if (s && !g_obj.count((void*)s)) die("event record on unknown stream", (void*)s);
  g_ev_stream[(void*)e] = (void*)s;
  g_ev_orphan.erase((void*)e);
  return hipSuccess;
}
static void live_event(hipEvent_t e, const char* what) {
  if (!g_obj.count((void*)e)) die(what, (void*)e);
  if (g_ev_orphan.count((void*)e)) die("event used after the stream it was recorded on was destroyed", (void*)e);
}
hipError_t hipEventQuery(hipEvent_t e) { FAKE_LOCK; live_event(e, "event query"); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t e) { FAKE_LOCK; live_event(e, "event sync"); return hipSuccess; }
hipError_t hipGetLastError(void) { FAKE_LOCK; return hipSuccess; }
hipError_t hipFree(void* p) { FAKE_LOCK;
  if (!p) return hipSuccess;
  auto it = g_dev.find(p);
  if (it == g_dev.end()) die("hipFree of unknown pointer", p);
  g_dev.erase(it);
  free(p);
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int* c) { FAKE_LOCK; *c = 1; return hipSuccess; }
hipError_t hipGetDevice(int* d) { FAKE_LOCK; *d = 0; return hipSuccess; }
const char* hipGetErrorString(hipError_t) { FAKE_LOCK; return "fake error"; }
hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t* nd, hipGraph_t g, const hipGraphNode_t*, size_t, void* dst,
                                   const void* src, size_t count, hipMemcpyKind) {
  FAKE_LOCK;
  if (!g_graphs.count((void*)g)) die("graph add", (void*)g);
  auto* fg = (FakeGraph*)g;
  fg->dst = dst; fg->src = src; fg->n = count;
  *nd = (hipGraphNode_t)g;
  return hipSuccess;
}
hipError_t hipGraphCreate(hipGraph_t* g, unsigned) { FAKE_LOCK; auto* f = new FakeGraph(); g_graphs.insert(f); *g = (hipGraph_t)f; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { FAKE_LOCK; if (!g) return hipSuccess; if (!g_graphs.erase((void*)g)) die("graph destroy", (void*)g); delete (FakeGraph*)g; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, hipGraphNode_t*, char*, size_t) { FAKE_LOCK;
  if (!g_graphs.count((void*)g)) die("instantiate", (void*)g);
  auto* f = new FakeGraph(*(FakeGraph*)g);
  g_execs.insert(f);
  *ex = (hipGraphExec_t)f;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) { FAKE_LOCK; if (!g_execs.erase((void*)ex)) die("exec destroy", (void*)ex); delete (FakeGraph*)ex; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t) { FAKE_LOCK;
  if (!g_execs.count((void*)ex)) die("graph launch", (void*)ex);
  auto* f = (FakeGraph*)ex;
  if (f->n) memcpy(f->dst, f->src, f->n);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) { FAKE_LOCK;
  if (!p) return hipSuccess;
  if (!g_host.erase(p)) die("hipHostFree of unknown pointer", p);
  free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { FAKE_LOCK; *p = calloc(1, n ? n : 1); g_host[*p] = n; return hipSuccess; }
// hipMalloc fails once after this many more successful calls (-1: never)
static long g_malloc_fail = -1;
hipError_t hipMalloc(void** p, size_t n) { FAKE_LOCK;
  if (g_malloc_fail == 0) {
    g_malloc_fail = -1;
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  if (g_malloc_fail > 0) --g_malloc_fail;
  *p = calloc(1, n ? n : 1); g_dev[*p] = n; return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { FAKE_LOCK; memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { FAKE_LOCK; memcpy(d, s, n); return hipSuccess; }
hipError_t hipSetDevice(int) { FAKE_LOCK; return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { FAKE_LOCK; *s = (hipStream_t)newobj(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { FAKE_LOCK;
  for (auto& kv : g_ev_stream)
    if (kv.second == (void*)s) g_ev_orphan.insert(kv.first);
  delobj((void*)s, "stream destroy");
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) { FAKE_LOCK; if (s && !g_obj.count((void*)s)) die("stream sync", (void*)s); return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { FAKE_LOCK; live_event(e, "wait event"); return hipSuccess; }
}

// every byte range a launcher is handed must lie in a live allocation
static void need(const void* p, size_t n, const char* what) { FAKE_LOCK;
  if (!p || !n) return;
  // pointers from outside the fake runtime (host tensors) are not checked
  auto it = g_dev.upper_bound((void*)p);
  if (it == g_dev.begin()) return;
  --it;
  const char* b = (const char*)it->first;
  if ((const char*)p >= b + it->second) return;
  if ((const char*)p + n > b + it->second) die(what, (void*)p);
}

namespace aqc {
hipError_t launch_regpass(const RegPassArgs&, int, hipStream_t) { FAKE_LOCK; return hipSuccess; }
int64_t regpass_blocks(int n, int wb, int) { FAKE_LOCK; return (int64_t)1 << (n > 12 ? n - 12 : 0); }
hipError_t launch_regpass_batch(const RegPassArgs* a, const int2* m, int64_t nb, int, int, hipStream_t) { FAKE_LOCK;
  need(m, nb * sizeof(int2), "regpass batch map");
  return hipSuccess;
}
hipError_t launch_pass_batch(const PassArgs*, const int2* m, int64_t nb, int, int, int, hipStream_t) { FAKE_LOCK;
  need(m, nb * sizeof(int2), "pass batch map");
  return hipSuccess;
}
hipError_t launch_pass(const PassArgs&, int, int64_t, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t add_regpass_batch_node(hipGraph_t g, hipGraphNode_t* nd, hipGraphNode_t, const RegPassArgs*,
                                  const int2* m, int64_t nb, int, int) {
  FAKE_LOCK;
  need(m, nb * sizeof(int2), "regpass node map");
  *nd = (hipGraphNode_t)g;
  return hipSuccess;
}
hipError_t add_pass_batch_node(hipGraph_t g, hipGraphNode_t* nd, hipGraphNode_t, const PassArgs*, const int2* m,
                               int64_t nb, int, int, int) {
  FAKE_LOCK;
  need(m, nb * sizeof(int2), "pass node map");
  *nd = (hipGraphNode_t)g;
  return hipSuccess;
}
// the library's fixed scratch array: one block for the process, never freed
// (not counted among the live handles)
hipError_t scratch_address(void** p) { FAKE_LOCK;
  static void* s = calloc(1, kScratchBytes);
  *p = s;
  return hipSuccess;
}
hipError_t launch_resident(const ResidentSolve* solves, int count, int, int, hipStream_t) { FAKE_LOCK;
  need(solves, (size_t)count * sizeof(ResidentSolve), "resident descriptors");
  return hipSuccess;
}
size_t pass_lds_bytes(int tb, int dtype) { FAKE_LOCK; return ((size_t)1 << tb) * (dtype == 0 ? 8 : 16); }
hipError_t prepare_kernels() { FAKE_LOCK; return hipSuccess; }
hipError_t launch_reduce_sum(const double* parts, int64_t nb, int nk, double* out, hipStream_t) { FAKE_LOCK;
  need(parts, nb * nk * sizeof(double), "reduce parts");
  for (int k = 0; k < nk; ++k) out[k] = 1.0;
  return hipSuccess;
}
hipError_t launch_norm2(const void*, int, int64_t N, double* parts, int64_t* nb, hipStream_t) { FAKE_LOCK;
  *nb = N > 4096 ? N / 4096 : 1;
  need(parts, *nb * sizeof(double), "norm2 parts");
  return hipSuccess;
}
hipError_t launch_overlap(const void*, const void*, int, int64_t N, double* parts, int64_t* nb, hipStream_t) { FAKE_LOCK;
  *nb = N > 4096 ? N / 4096 : 1;
  need(parts, 2 * *nb * sizeof(double), "overlap parts");
  return hipSuccess;
}
hipError_t launch_gather_mass(const void*, int, const int64_t*, int64_t m, double* parts, int64_t* nb, hipStream_t) { FAKE_LOCK;
  *nb = m > 256 ? m / 256 : 1;
  need(parts, *nb * sizeof(double), "gather parts");
  return hipSuccess;
}
hipError_t launch_diag_minmax(const PassArgs&, int64_t nb, double* parts, hipStream_t) { FAKE_LOCK;
  need(parts, 2 * nb * sizeof(double), "minmax parts");
  for (int64_t i = 0; i < nb; ++i) { parts[i] = -1.0; parts[nb + i] = 3.0; }
  return hipSuccess;
}
hipError_t launch_diag_mass(const PassArgs&, int, int64_t nb, double, double* parts, hipStream_t) { FAKE_LOCK;
  need(parts, nb * sizeof(double), "mass parts");
  return hipSuccess;
}
hipError_t launch_scale(void*, int, int64_t, double, double, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_copy(void*, const void*, int, int64_t, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_zero(void* d, size_t n, hipStream_t) { FAKE_LOCK; need(d, n, "zero"); memset(d, 0, n); return hipSuccess; }
int64_t sector_blocks(int64_t dim) { FAKE_LOCK; return (dim + 1023) / 1024; }
hipError_t launch_sector_matvec(const SectorArgs& a, int, hipStream_t) { FAKE_LOCK;
  if (a.s.dstore > 0) need(a.s.dtab, (size_t)a.s.dstore * (size_t)a.s.dim * sizeof(double), "sector diagonal parts");
  return hipSuccess;
}
hipError_t launch_sector_dtab(const SectorArgs& a, double* out, hipStream_t) { FAKE_LOCK;
  need(out, (size_t)a.s.dim * sizeof(double), "sector diagonal part");
  return hipSuccess;
}
hipError_t launch_sector_diag(const SectorArgs&, int, double, const void*, int, double*, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_sector_expand(const SectorDev&, const void*, void*, int, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_fill(void*, int, int64_t, double, double, hipStream_t) { FAKE_LOCK; return hipSuccess; }
int64_t lz_blocks(int64_t N) { FAKE_LOCK; return (N + 1023) / 1024; }
hipError_t launch_multidot(const void*, int64_t, int64_t, int, const void*, int, double*, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_multiaxpy(const void*, int64_t, int64_t, int, const double*, void*, int, double*, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_scale_copy(void*, const void*, int, int64_t, double, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_basis_transform(void*, int64_t, int64_t, int, int, const double*, int, hipStream_t) { FAKE_LOCK; return hipSuccess; }
hipError_t launch_random_fill(void*, int, int64_t, uint64_t, hipStream_t) { FAKE_LOCK; return hipSuccess; }
}  // namespace aqc

// the next hipMalloc after k successful ones fails (k < 0: none fails)
extern "C" void fake_hip_fail_malloc_after(long k) { FAKE_LOCK; g_malloc_fail = k; }

// handles still alive (allocations, streams, events, graphs)
extern "C" long fake_hip_live() { FAKE_LOCK;
  return (long)(g_dev.size() + g_host.size() + g_obj.size() + g_graphs.size() + g_execs.size());
}
