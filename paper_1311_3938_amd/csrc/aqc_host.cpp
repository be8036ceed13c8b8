// Host runtime of the C ABI in include/aqc.h: Hamiltonian compiler, tile-pass
// planner, split diagonal tables, integrator driver and reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <numeric>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/aqc.h"
#include "aqc_internal.h"

using namespace aqc;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static aqc_status fail(aqc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(AQC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define STCHK(expr)                 \
  do {                              \
    aqc_status s_ = (expr);         \
    if (s_ != AQC_OK) return s_;    \
  } while (0)

extern "C" const char* aqc_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* aqc_version(void) { return "aqc 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// largest dynamic LDS a workgroup may use (set by aqc_create)
static std::atomic<size_t> g_lds_max{0};

struct aqc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t lds_max = 0;
  double* parts = nullptr;      // per-block partial sums
  size_t parts_cap = 0;         // doubles
  double* dres = nullptr;       // device results [64]
  double* hres = nullptr;       // pinned host results [64]
  int64_t* didx = nullptr;      // device index list for basis-list fidelity
  size_t didx_cap = 0;
  // instrumentation: event pairs around tile-pass launches
  bool prof_on = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[2] = {0, 0};
  int64_t prof_n[2] = {0, 0};
  double prof_bytes[2] = {0, 0};  // algorithmic bytes of the timed launches
  // device address of this device's fixed scratch array (aqc_energy_noalloc)
  void* scratch = nullptr;
  // lifetime: one reference for the caller that created the context and one
  // per batch created on it; the memory goes with the last one.  closed is set
  // by aqc_destroy (the caller's release); a batch then refuses further work
  std::atomic<int> refs{1};
  std::atomic<bool> closed{false};
};

// Device address of the fixed scratch array, looked up once per device (each
// GPU holds its own copy of the array at its own address).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

static aqc_status scratch_for_device(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(AQC_ENOTSUP, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    // the caller has made `device` current
    HIPCHK(scratch_address(&p));
    if (!p) return fail(AQC_EDEVICE, "scratch array has no device address");
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// Device buffers of Hamiltonian tables.  Freeing device memory waits for
// every stream of the device, so a finished solve that frees its Hamiltonian
// would stall the solves running beside it.  Table buffers of released
// Hamiltonians and replaced plans are kept per device instead, and handed out
// again once every stream the library launches on has passed an event
// recorded at the release (no launch queued before it can still read them);
// otherwise a fresh buffer is allocated.  The cache holds at most
// kTabCacheBytes per device; aqc_trim empties it.
// ---------------------------------------------------------------------------
struct TabEv {
  hipStream_t s;
  hipEvent_t e;
};
struct TabBuf {
  void* p = nullptr;
  size_t cap = 0;
  std::vector<TabEv> ev;   // recorded at the release, one per stream
};
constexpr size_t kTabCacheBytes = size_t(1) << 30;
static std::mutex g_tab_mu;
static std::vector<TabBuf> g_tab_free[kMaxDevices];      // released, maybe still read
static std::map<void*, size_t> g_tab_size[kMaxDevices];  // buffers handed out
static size_t g_tab_cached[kMaxDevices] = {};
static std::map<hipStream_t, int> g_tab_streams[kMaxDevices];  // streams launched on

static void tab_stream_add(int dev, hipStream_t s) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_tab_mu);
  ++g_tab_streams[dev][s];
}

// The caller has synchronized `s`: every event recorded on it has completed.
// Its last user gone, the stream may be destroyed next, so the kept buffers
// drop their events on it (no event outlives the stream it was recorded on).
static void tab_stream_remove(int dev, hipStream_t s) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tab_streams[dev].find(s);
  if (it == g_tab_streams[dev].end() || --it->second > 0) return;
  g_tab_streams[dev].erase(it);
  for (TabBuf& b : g_tab_free[dev]) {
    auto keep = b.ev.begin();
    for (auto e = b.ev.begin(); e != b.ev.end(); ++e) {
      if (e->s == s)
        hipEventDestroy(e->e);
      else
        *keep++ = *e;
    }
    b.ev.erase(keep, b.ev.end());
  }
}

// Every launch queued before the release has ended.  A query that reports
// anything but success or not-ready counts as not ready, and the error it
// leaves behind is consumed here rather than by the next launch check.
static bool tab_ready(const TabBuf& b) {
  for (const TabEv& e : b.ev) {
    const hipError_t r = hipEventQuery(e.e);
    if (r == hipSuccess) continue;
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// `bytes` of device memory on the current device (the caller has set it)
static aqc_status tab_alloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(AQC_ENOTSUP, "device index above 63");
  {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto& fl = g_tab_free[dev];
    int best = -1;
    for (int i = 0; i < (int)fl.size(); ++i) {
      const size_t c = fl[i].cap;
      if (c < bytes || c > 2 * bytes + 65536) continue;
      if (best >= 0 && c >= fl[best].cap) continue;
      if (!tab_ready(fl[i])) continue;
      best = i;
    }
    if (best >= 0) {
      TabBuf b = fl[best];
      fl.erase(fl.begin() + best);
      for (const TabEv& e : b.ev) hipEventDestroy(e.e);
      g_tab_cached[dev] -= b.cap;
      g_tab_size[dev][b.p] = b.cap;
      *p = b.p;
      return AQC_OK;
    }
  }
  HIPCHK(hipMalloc(p, bytes));
  std::lock_guard<std::mutex> lk(g_tab_mu);
  g_tab_size[dev][*p] = bytes;
  return AQC_OK;
}

// Releases a buffer of tab_alloc on device `dev` (null: nothing).
static void tab_release(int dev, void* p) {
  if (!p || dev < 0 || dev >= kMaxDevices) return;
  std::unique_lock<std::mutex> lk(g_tab_mu);
  auto it = g_tab_size[dev].find(p);
  const size_t cap = it != g_tab_size[dev].end() ? it->second : 0;
  if (it != g_tab_size[dev].end()) g_tab_size[dev].erase(it);
  if (cap == 0 || g_tab_cached[dev] + cap > kTabCacheBytes) {
    lk.unlock();
    hipSetDevice(dev);
    hipFree(p);   // waits for the device
    return;
  }
  TabBuf b;
  b.p = p;
  b.cap = cap;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(dev);
  bool ok = true;
  for (const auto& kv : g_tab_streams[dev]) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      ok = false;
      break;
    }
    b.ev.push_back({kv.first, e});
    if (hipEventRecord(e, kv.first) != hipSuccess) {
      ok = false;
      break;
    }
  }
  if (!ok) {
    // no proof that the queued launches are done with it: free instead
    (void)hipGetLastError();
    lk.unlock();
    for (const TabEv& e : b.ev) hipEventDestroy(e.e);
    hipFree(p);   // waits for the device
    hipSetDevice(cur);
    return;
  }
  hipSetDevice(cur);
  g_tab_cached[dev] += cap;
  g_tab_free[dev].push_back(std::move(b));
}

extern "C" aqc_status aqc_trim(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(AQC_EINVAL, "aqc_trim: bad device index");
  std::vector<TabBuf> fl;
  {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    fl.swap(g_tab_free[device]);
    g_tab_cached[device] = 0;
  }
  if (fl.empty()) return AQC_OK;
  HIPCHK(hipSetDevice(device));
  for (TabBuf& b : fl) {
    for (const TabEv& e : b.ev) {
      hipEventSynchronize(e.e);
      hipEventDestroy(e.e);
    }
    HIPCHK(hipFree(b.p));
  }
  return AQC_OK;
}

static aqc_status prof_drain(aqc_ctx* c) {
  if (c->prof_pending.empty()) return AQC_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (auto& r : c->prof_pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    c->prof_ms[r.kind] += ms;
    c->prof_n[r.kind] += 1;
    c->prof_pool.push_back(r.a);
    c->prof_pool.push_back(r.b);
  }
  c->prof_pending.clear();
  return AQC_OK;
}

static aqc_status prof_event(aqc_ctx* c, hipEvent_t* e) {
  if (!c->prof_pool.empty()) {
    *e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return AQC_OK;
  }
  HIPCHK(hipEventCreate(e));
  return AQC_OK;
}

extern "C" aqc_status aqc_profile_enable(aqc_ctx* c, int on) {
  if (!c) return fail(AQC_EINVAL, "aqc_profile_enable: ctx is NULL");
  c->prof_on = on != 0;
  return AQC_OK;
}

extern "C" aqc_status aqc_profile_reset(aqc_ctx* c) {
  if (!c) return fail(AQC_EINVAL, "aqc_profile_reset: ctx is NULL");
  STCHK(prof_drain(c));
  c->prof_ms[0] = c->prof_ms[1] = 0.0;
  c->prof_n[0] = c->prof_n[1] = 0;
  c->prof_bytes[0] = c->prof_bytes[1] = 0.0;
  return AQC_OK;
}

extern "C" aqc_status aqc_profile_read(aqc_ctx* c, int kind, double* ms, int64_t* n,
                                       double* bytes) {
  if (!c || !ms || !n || !bytes) return fail(AQC_EINVAL, "aqc_profile_read: NULL argument");
  if (kind != AQC_PROF_HIGH_PASS && kind != AQC_PROF_LAST_PASS)
    return fail(AQC_EINVAL, "aqc_profile_read: unknown kind");
  STCHK(prof_drain(c));
  *ms = c->prof_ms[kind];
  *n = c->prof_n[kind];
  *bytes = c->prof_bytes[kind];
  return AQC_OK;
}

static aqc_status ensure_parts(aqc_ctx* c, size_t n) {
  if (n <= c->parts_cap) return AQC_OK;
  if (c->parts) {
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipFree(c->parts));
    c->parts = nullptr;
  }
  size_t cap = std::max<size_t>(n, 1 << 16);
  HIPCHK(hipMalloc(&c->parts, cap * sizeof(double)));
  c->parts_cap = cap;
  return AQC_OK;
}

extern "C" aqc_status aqc_create(int device, void* stream, aqc_ctx** out) {
  if (!out) return fail(AQC_EINVAL, "aqc_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AQC_EINVAL, "aqc_create: bad device index");
  HIPCHK(hipSetDevice(device));
  // an error return below destroys the context made so far
  struct CtxFree {
    void operator()(aqc_ctx* p) const { aqc_destroy(p); }
  };
  std::unique_ptr<aqc_ctx, CtxFree> c(new aqc_ctx());
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  tab_stream_add(device, c->stream);
  int lds = 0;
  HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
  c->lds_max = (size_t)lds;
  g_lds_max.store((size_t)lds, std::memory_order_relaxed);
  HIPCHK(prepare_kernels());
  STCHK(scratch_for_device(device, &c->scratch));
  HIPCHK(hipMalloc(&c->dres, 64 * sizeof(double)));
  HIPCHK(hipHostMalloc(&c->hres, 64 * sizeof(double), hipHostMallocDefault));
  STCHK(ensure_parts(c.get(), 1 << 16));
  *out = c.release();
  return AQC_OK;
}

// Drops one reference; the last one frees the context's buffers and memory.
static void ctx_release(aqc_ctx* c) {
  if (c->refs.fetch_sub(1, std::memory_order_acq_rel) != 1) return;
  hipSetDevice(c->device);
  if (c->parts) hipFree(c->parts);
  if (c->dres) hipFree(c->dres);
  if (c->hres) hipHostFree(c->hres);
  if (c->didx) hipFree(c->didx);
  for (hipEvent_t e : c->prof_pool) hipEventDestroy(e);
  delete c;
}

extern "C" aqc_status aqc_destroy(aqc_ctx* c) {
  if (!c) return AQC_OK;
  if (c->closed.exchange(true)) return fail(AQC_EINVAL, "aqc_destroy: context already destroyed");
  hipSetDevice(c->device);
  // everything queued on the borrowed stream (the batches' work there too)
  // ends here; a batch still alive never touches that stream again
  hipStreamSynchronize(c->stream);
  prof_drain(c);
  tab_stream_remove(c->device, c->stream);
  ctx_release(c);
  return AQC_OK;
}

extern "C" aqc_status aqc_set_stream(aqc_ctx* c, void* stream) {
  if (!c) return fail(AQC_EINVAL, "aqc_set_stream: ctx is NULL");
  // work queued on the old stream may read tables released later, which are
  // reused once the streams in use have passed the release: finish it first
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipStreamSynchronize(c->stream));
  tab_stream_add(c->device, reinterpret_cast<hipStream_t>(stream));
  tab_stream_remove(c->device, c->stream);
  c->stream = reinterpret_cast<hipStream_t>(stream);
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// schedules (time dependence of the coefficients, end of Sec. II.A)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Hamiltonian
// ---------------------------------------------------------------------------
struct HTerm {
  uint64_t x, z;
  double w;
  int sid;
};

struct Pass {
  int kind = 0;              // 0: LDS tile pass, 1: register hypercube pass
  int hb = 0;                // kind 1: hypercube bits [hb, hb + RB + wb)
  int wb = 0;                // kind 1: bits spanned by the waves of a workgroup
  int bit_group[16] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  int tb = 0, lbits = 0;
  uint64_t hmask = 0, cmask = 0;
  bool final_pass = false;
  bool stream = false;       // last pass: some groups flip bits outside the tile
  std::vector<int> groups;   // indices into Ham::groups
  DevGroup* dgroups = nullptr;
  DevTerm* dterms = nullptr;
  int ng = 0, nterms = 0;
};

struct Plan {
  bool built = false;
  bool has_stream = false;   // the last pass reads partners outside its tile
  int tbf = 0;               // last pass tile bits
  std::vector<Pass> passes;  // high passes first, last pass last
  // split diagonal tables for tile bits tbf
  DiagDev dg{};
  double* dCT = nullptr;
  double* dLT = nullptr;
  double* dTAB64 = nullptr;
  DevTerm* dres = nullptr;
};

struct GroupH {
  uint64_t x;
  std::vector<HTerm> terms;
  bool plain;
};

struct aqc_ham {
  int n = 0;
  int device = 0;
  std::vector<aqc_sched> scheds;
  aqc_path path{};
  std::vector<HTerm> terms;      // merged
  std::vector<HTerm> diag;       // x == 0, z != 0
  std::vector<HTerm> ident;      // x == 0, z == 0
  std::vector<GroupH> groups;    // x != 0
  Plan plans[2];
  // tile passes only (no register passes, no stream groups), per dtype: the
  // plan of the batch engine's resident solves, built when first needed
  Plan tplans[2];
  // tiling chosen for this Hamiltonian (aqc_ham_set_tiling), per dtype
  bool tiling_set[2] = {false, false};
  int tiling[2][4] = {{0, 0, 0, 1}, {0, 0, 0, 1}};  // tbf, tbh, lh, register passes
  // diagonal minimum and maximum per schedule (spectral enclosure)
  bool have_minmax = false;
  std::vector<double> dmin, dmax;  // per schedule
  // amplitudes of a state: 2^n, or C(n, w) for a Hamming-weight sector
  int64_t dim = 0;
  int sector_w = -1;             // weight of a sector (aqc_sector_create), else -1
  SectorDev sd{};                // a sector's device tables
  std::vector<void*> sec_bufs;   // and their allocations
  // plans and the diagonal range are built on first use when not built
  // eagerly; this lock makes that safe from several host threads
  std::recursive_mutex mu;
};

// plans of both dtypes are built with the Hamiltonian up to this size (the
// tables are small there); larger ones are built on first use
constexpr int kEagerPlanMaxN = 26;

// Releases a plan's table buffers (they are reused only after every stream
// the library launches on has passed this point).
static void free_plan(Plan& p, int dev) {
  for (auto& ps : p.passes) {
    tab_release(dev, ps.dgroups);
    tab_release(dev, ps.dterms);
  }
  p.passes.clear();
  tab_release(dev, p.dCT);
  tab_release(dev, p.dLT);
  tab_release(dev, p.dTAB64);
  tab_release(dev, p.dres);
  p = Plan();
}

extern "C" aqc_status aqc_ham_free(aqc_ham* h) {
  if (!h) return AQC_OK;
  free_plan(h->plans[0], h->device);
  free_plan(h->plans[1], h->device);
  free_plan(h->tplans[0], h->device);
  free_plan(h->tplans[1], h->device);
  for (void* b : h->sec_bufs) tab_release(h->device, b);
  delete h;
  return AQC_OK;
}

// owner of a Hamiltonian under construction: an error return releases its
// device tables with it
struct HamFree {
  void operator()(aqc_ham* h) const { aqc_ham_free(h); }
};
using HamPtr = std::unique_ptr<aqc_ham, HamFree>;

static int popc(uint64_t v) { return __builtin_popcountll(v); }
static aqc_status build_plan(aqc_ham* h, int dtype, hipStream_t s);

extern "C" aqc_status aqc_build_hamiltonian(aqc_ctx* ctx, int n, int64_t n_terms,
                                            const uint64_t* xm, const uint64_t* zm,
                                            const double* w, const int32_t* sid, int n_sched,
                                            const aqc_sched* scheds, const aqc_path* path,
                                            aqc_ham** out) {
  if (!out) return fail(AQC_EINVAL, "aqc_build_hamiltonian: out is NULL");
  *out = nullptr;
  if (!ctx) return fail(AQC_EINVAL, "aqc_build_hamiltonian: ctx is NULL");
  if (n < 1) return fail(AQC_EINVAL, "aqc_build_hamiltonian: n_qubits < 1");
  if (n > 34) return fail(AQC_ENOTSUP, "aqc_build_hamiltonian: n_qubits > 34");
  if (n_terms < 0) return fail(AQC_EINVAL, "aqc_build_hamiltonian: n_terms < 0");
  if (n_terms > 0 && (!xm || !zm || !w || !sid))
    return fail(AQC_EINVAL, "aqc_build_hamiltonian: NULL term array");
  if (n_sched < 1 || n_sched > kMaxSched || !scheds)
    return fail(AQC_EINVAL, "aqc_build_hamiltonian: need 1..32 schedules");
  if (!path || !(path->T > 0.0) || !std::isfinite(path->T) ||
      (path->kind != AQC_PATH_LINEAR && path->kind != AQC_PATH_SIN2))
    return fail(AQC_EINVAL, "aqc_build_hamiltonian: bad path");
  for (int s = 0; s < n_sched; ++s) {
    const aqc_sched& sc = scheds[s];
    if (sc.kind < 0 || sc.kind > 3) return fail(AQC_EINVAL, "aqc_build_hamiltonian: bad schedule kind");
    if (sc.kind == AQC_SCHED_PWL_S) {
      if (sc.degree < 0 || sc.degree > 3) return fail(AQC_EINVAL, "aqc_build_hamiltonian: 1..4 knots");
      for (int d = 0; d < 2 * (sc.degree + 1); ++d)
        if (!std::isfinite(sc.coef[d])) return fail(AQC_EINVAL, "aqc_build_hamiltonian: non-finite knot");
      for (int d = 0; d < sc.degree; ++d)
        if (sc.coef[2 * d + 2] < sc.coef[2 * d])
          return fail(AQC_EINVAL, "aqc_build_hamiltonian: knots must not decrease in s");
    }
    if (sc.kind == AQC_SCHED_POLY_S) {
      if (sc.degree < 0 || sc.degree > 7) return fail(AQC_EINVAL, "aqc_build_hamiltonian: poly degree");
      for (int d = 0; d <= sc.degree; ++d)
        if (!std::isfinite(sc.coef[d])) return fail(AQC_EINVAL, "aqc_build_hamiltonian: non-finite coef");
      if (std::isnan(sc.s_lo) || std::isnan(sc.s_hi))
        return fail(AQC_EINVAL, "aqc_build_hamiltonian: NaN window");
    }
    if (sc.kind == AQC_SCHED_TRIG_T &&
        !(std::isfinite(sc.amp) && std::isfinite(sc.omega) && std::isfinite(sc.phase)))
      return fail(AQC_EINVAL, "aqc_build_hamiltonian: non-finite trig schedule");
  }
  const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
  std::map<std::tuple<uint64_t, uint64_t, int>, double> merged;
  for (int64_t l = 0; l < n_terms; ++l) {
    if ((xm[l] & ~full) || (zm[l] & ~full))
      return fail(AQC_EINVAL, "aqc_build_hamiltonian: mask outside the n qubits (term " +
                                  std::to_string(l) + ")");
    if (!std::isfinite(w[l])) return fail(AQC_EINVAL, "aqc_build_hamiltonian: non-finite weight");
    if (sid[l] < 0 || sid[l] >= n_sched)
      return fail(AQC_EINVAL, "aqc_build_hamiltonian: sched_id out of range");
    merged[std::make_tuple(xm[l], zm[l], (int)sid[l])] += w[l];
  }
  HamPtr h(new aqc_ham());
  h->n = n;
  h->dim = (int64_t)1 << n;
  h->device = ctx->device;
  h->scheds.assign(scheds, scheds + n_sched);
  h->path = *path;
  std::map<uint64_t, size_t> gidx;
  for (auto& kv : merged) {
    HTerm t{std::get<0>(kv.first), std::get<1>(kv.first), kv.second, std::get<2>(kv.first)};
    if (t.w == 0.0) continue;
    h->terms.push_back(t);
    if (t.x == 0) {
      if (t.z == 0) h->ident.push_back(t);
      else h->diag.push_back(t);
    } else {
      auto it = gidx.find(t.x);
      if (it == gidx.end()) {
        gidx[t.x] = h->groups.size();
        h->groups.push_back(GroupH{t.x, {}, true});
        it = gidx.find(t.x);
      }
      GroupH& g = h->groups[it->second];
      g.terms.push_back(t);
      if (t.z != 0) g.plain = false;
    }
  }
  if (n <= kEagerPlanMaxN) {
    HIPCHK(hipSetDevice(ctx->device));
    for (int d = 0; d < 2; ++d) {
      // a Hamiltonian the default tiling cannot hold is still returned: the
      // error then comes from the first use (or aqc_ham_set_tiling fixes it)
      if (build_plan(h.get(), d, ctx->stream) != AQC_OK) {
        free_plan(h->plans[d], h->device);
        g_last_error.clear();
      }
    }
  }
  *out = h.release();
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// planner
// ---------------------------------------------------------------------------
struct Tiling {
  int tbf, tbh, lh;
};

// wide register passes when they give at least 2^this many workgroups
constexpr int kWideMinLogBlocks = 8;
// flip patterns above the last tile that no register pass takes are applied
// by the last pass from memory (1) or by tile high passes (0)
constexpr int kStreamDefault = 0;

static Tiling default_tiling(int dtype) {
  // last pass: 2^13 (c64) / 2^12 (c128) amplitudes = 64 KiB of LDS, so two
  // workgroups share a CU; high passes use the same tile with 128-byte chunks.
  return dtype == 0 ? Tiling{13, 13, 4} : Tiling{12, 12, 3};
}

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

static aqc_status upload(void** dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) {
    *dst = nullptr;
    return AQC_OK;
  }
  STCHK(tab_alloc(dst, bytes));
  HIPCHK(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return AQC_OK;
}

static uint64_t pext_host(uint64_t v, uint64_t mask) {
  uint64_t r = 0;
  int k = 0;
  for (int b = 0; b < 64; ++b)
    if (mask >> b & 1ull) r |= ((v >> b) & 1ull) << (k++);
  return r;
}

static aqc_status build_pass_tables(Pass& ps, const aqc_ham* h, int dtype, hipStream_t s) {
  std::vector<DevGroup> dg;
  std::vector<DevTerm> dt;
  const uint64_t tmask = ((1ull << ps.lbits) - 1ull) | ps.hmask;
  const int slots = dtype == AQC_C64 ? kFastSlotsC64 : kFastSlotsC128;
  int nfast = 0;
  for (int gi : ps.groups) {
    const GroupH& g = h->groups[gi];
    DevGroup d{};
    d.x = g.x;
    d.xl = (uint32_t)pext_host(g.x, tmask);
    d.t0 = (int)dt.size();
    d.nt = (int)g.terms.size();
    d.plain = g.plain ? 1 : 0;
    d.fslot = -1;
    bool inside = popc(g.x) <= 2;
    for (const HTerm& t : g.terms) {
      dt.push_back(DevTerm{t.z, t.w, t.sid, popc(t.x & t.z) & 3});
      inside = inside && !(t.z & ~g.x);
    }
    if (!g.plain && inside && nfast < slots) {
      d.fslot = nfast++;
      const int bi = __builtin_ctzll(g.x), bj = 63 - __builtin_clzll(g.x);
      d.bij = bi | (bj << 8);
      if (!(g.x & ~tmask)) {
        // the bits' positions in tile-local coordinates (the tile's bits in order)
        const int li = popc(tmask & ((1ull << bi) - 1ull)), lj = popc(tmask & ((1ull << bj) - 1ull));
        d.lij = li | (lj << 8);
      }
    }
    dg.push_back(d);
  }
  ps.ng = (int)dg.size();
  ps.nterms = (int)dt.size();
  STCHK(upload((void**)&ps.dgroups, dg.data(), dg.size() * sizeof(DevGroup), s));
  STCHK(upload((void**)&ps.dterms, dt.data(), dt.size() * sizeof(DevTerm), s));
  return AQC_OK;
}

// Split the diagonal terms for tile bits tb: see DiagDev.
static aqc_status build_diag_tables(Plan& p, const aqc_ham* h, hipStream_t s) {
  const int n = h->n, tb = p.tbf;
  const uint64_t lomask = (1ull << tb) - 1ull;
  const int64_t nhi = (int64_t)1 << (n - tb);
  const int64_t ntile = (int64_t)1 << tb;
  std::vector<int> sd, ts;
  std::vector<HTerm> ct_terms, lt_terms, tab_terms, res;
  auto slot = [](std::vector<int>& v, int sid, int cap) -> int {
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] == sid) return (int)i;
    if ((int)v.size() >= cap) return -1;
    v.push_back(sid);
    return (int)v.size() - 1;
  };
  for (const HTerm& t : h->diag) {
    const uint64_t u = t.z & lomask;
    const uint64_t zh = t.z >> tb;
    const int pu = popc(u);
    if (pu <= 1) {
      if (slot(sd, t.sid, kMaxDiagSched) < 0) {
        res.push_back(t);
        continue;
      }
      (pu == 0 ? ct_terms : lt_terms).push_back(t);
    } else if (zh == 0) {
      if (slot(ts, t.sid, kMaxTabSched) < 0) {
        res.push_back(t);
        continue;
      }
      tab_terms.push_back(t);
    } else {
      res.push_back(t);
    }
  }
  const int nsd = (int)sd.size(), ntab = (int)ts.size();
  std::vector<double> CT((size_t)std::max(nsd, 1) * nhi, 0.0);
  std::vector<double> LT((size_t)std::max(nsd, 1) * nhi * tb, 0.0);
  std::vector<double> TAB((size_t)std::max(ntab, 1) * ntile, 0.0);
  auto sidx = [&](const std::vector<int>& v, int sid) {
    return (int)(std::find(v.begin(), v.end(), sid) - v.begin());
  };
  for (const HTerm& t : ct_terms) {
    const int k = sidx(sd, t.sid);
    const uint64_t zh = t.z >> tb;
    for (int64_t hi = 0; hi < nhi; ++hi)
      CT[(size_t)k * nhi + hi] += (popc((uint64_t)hi & zh) & 1) ? -t.w : t.w;
  }
  for (const HTerm& t : lt_terms) {
    const int k = sidx(sd, t.sid);
    const uint64_t zh = t.z >> tb;
    const int i = __builtin_ctzll(t.z & lomask);
    for (int64_t hi = 0; hi < nhi; ++hi)
      LT[((size_t)k * nhi + hi) * tb + i] += (popc((uint64_t)hi & zh) & 1) ? -t.w : t.w;
  }
  for (const HTerm& t : tab_terms) {
    const int k = sidx(ts, t.sid);
    const uint64_t u = t.z & lomask;
    for (int64_t lo = 0; lo < ntile; ++lo)
      TAB[(size_t)k * ntile + lo] += (popc((uint64_t)lo & u) & 1) ? -t.w : t.w;
  }
  std::vector<DevTerm> dres;
  for (const HTerm& t : res) dres.push_back(DevTerm{t.z, t.w, t.sid, 0});
  STCHK(upload((void**)&p.dCT, CT.data(), CT.size() * sizeof(double), s));
  STCHK(upload((void**)&p.dLT, LT.data(), LT.size() * sizeof(double), s));
  STCHK(upload((void**)&p.dTAB64, TAB.data(), TAB.size() * sizeof(double), s));
  STCHK(upload((void**)&p.dres, dres.data(), dres.size() * sizeof(DevTerm), s));
  DiagDev& d = p.dg;
  d = DiagDev{};
  d.nsd = nsd;
  for (int i = 0; i < nsd; ++i) d.sd_sid[i] = sd[i];
  d.ntab = ntab;
  for (int i = 0; i < ntab; ++i) d.tab_sid[i] = ts[i];
  d.nres = (int)dres.size();
  d.CT = p.dCT;
  d.LT = p.dLT;
  d.TAB64 = p.dTAB64;
  d.res = p.dres;
  return AQC_OK;
}

// Pass layout (host only): the last pass tiles the low tbf bits; every other
// flip pattern goes to a high pass whose tile is [0, lh) plus at most tbh - lh
// further bits.
// force_reg >= 0 overrides the register-pass mode (used to weigh the
// library's choice against a layout without register passes).
static aqc_status layout_passes(const aqc_ham* h, int dtype, std::vector<Pass>& out, int* tbf_out,
                                bool tiles_only = false, int force_reg = -1) {
  Tiling tl = default_tiling(dtype);
  tl.tbf = env_int(dtype == 0 ? "AQC_TBF_C64" : "AQC_TBF_C128", tl.tbf);
  tl.tbh = env_int(dtype == 0 ? "AQC_TBH_C64" : "AQC_TBH_C128", tl.tbh);
  tl.lh = env_int(dtype == 0 ? "AQC_LH_C64" : "AQC_LH_C128", tl.lh);
  int use_reg = env_int("AQC_REGPASS", 1);
  if (use_reg < 0 || use_reg > 3) use_reg = 1;
  bool use_stream = env_int("AQC_STREAM", kStreamDefault) != 0;
  if (h->tiling_set[dtype]) {
    tl.tbf = h->tiling[dtype][0];
    tl.tbh = h->tiling[dtype][1];
    tl.lh = h->tiling[dtype][2];
    use_reg = h->tiling[dtype][3] & 3;
    use_stream = (h->tiling[dtype][3] & 4) != 0;
  }
  if (tiles_only) {
    use_reg = 0;
    use_stream = false;
  }
  if (force_reg >= 0) use_reg = force_reg;
  const int maxtb = dtype == 0 ? 14 : 13;
  if (tl.tbf < 1 || tl.tbf > maxtb || tl.tbh < 2 || tl.tbh > maxtb || tl.lh < 1 || tl.lh >= tl.tbh)
    return fail(AQC_EINVAL, "tiling parameters out of range");
  const size_t lds_max = g_lds_max.load(std::memory_order_relaxed);
  if (lds_max > 0) {
    while (tl.tbf > 1 && pass_lds_bytes(tl.tbf, dtype) > lds_max) --tl.tbf;
    while (tl.tbh > tl.lh + 1 && pass_lds_bytes(tl.tbh, dtype) > lds_max) --tl.tbh;
  }
  const int n = h->n;
  const uint64_t full = (1ull << n) - 1ull;
  const int tbf = std::min(n, tl.tbf);
  const int lh = std::min(tl.lh, tbf);
  const int tbh = std::min(n, tl.tbh);
  const int cap = std::max(0, tbh - lh);  // high bits per pass
  const uint64_t fmask = (1ull << tbf) - 1ull;
  const uint64_t lowh = (1ull << lh) - 1ull;

  Pass last;
  last.final_pass = true;
  last.tb = tbf;
  last.lbits = tbf;
  last.hmask = 0;
  last.cmask = full & ~fmask;
  std::vector<int> rest;
  int lterms = 0;
  for (size_t gi = 0; gi < h->groups.size(); ++gi) {
    const GroupH& g = h->groups[gi];
    if ((g.x & ~fmask) == 0 && (int)last.groups.size() < kMaxPassGroups &&
        lterms + (int)g.terms.size() <= kMaxPassTerms) {
      last.groups.push_back((int)gi);
      lterms += (int)g.terms.size();
    } else {
      rest.push_back((int)gi);
    }
  }
  // single-qubit flips with real coefficients above the last pass's tile go to
  // register hypercube passes over contiguous ranges of RB (+ kWaveBits) bits.
  // use_reg: 0 none, 1 wide passes when the state is large enough to give
  // every CU several workgroups, else narrow; 2 narrow only; 3 wide only.
  std::vector<Pass> regp;
  const int rb = dtype == 0 ? kRegBitsC64 : kRegBitsC128;
  int wb = 0;
  if (use_reg == 3 || (use_reg == 1 && n - 6 - rb - kWaveBits >= kWideMinLogBlocks)) wb = kWaveBits;
  if (wb && n - 6 - rb - wb < 1) wb = 0;
  const int width = rb + wb;
  if (use_reg && n - 6 - rb >= 2) {
    std::map<int, int> single;  // bit -> group
    std::vector<int> keep;
    for (int gi : rest) {
      const GroupH& g = h->groups[gi];
      const int b = __builtin_ctzll(g.x);
      if (popc(g.x) == 1 && g.plain && b >= 6) single[b] = gi;
      else keep.push_back(gi);
    }
    while (!single.empty()) {
      const int b0 = single.begin()->first;
      const int hb = std::max(6, std::min(b0, n - width));
      Pass ps;
      ps.kind = 1;
      ps.hb = hb;
      ps.wb = wb;
      for (int b = 0; b < width; ++b) {
        auto it = single.find(hb + b);
        if (it != single.end()) {
          ps.bit_group[b] = it->second;
          ps.groups.push_back(it->second);
          single.erase(it);
        }
      }
      ps.tb = width;
      regp.push_back(ps);
    }
    rest.swap(keep);
  }
  // stream groups: the remaining flip patterns are applied by the last pass,
  // which reads their partners from the source vector directly
  if (use_stream) {
    std::vector<int> keep;
    for (int gi : rest) {
      const GroupH& g = h->groups[gi];
      if ((int)last.groups.size() < kMaxPassGroups && lterms + (int)g.terms.size() <= kMaxPassTerms) {
        last.groups.push_back(gi);
        lterms += (int)g.terms.size();
        last.stream = true;
      } else {
        keep.push_back(gi);
      }
    }
    rest.swap(keep);
  }
  std::sort(rest.begin(), rest.end(), [&](int a, int b) {
    const uint64_t xa = h->groups[a].x, xb = h->groups[b].x;
    const int ha = 63 - __builtin_clzll(xa), hb = 63 - __builtin_clzll(xb);
    if (ha != hb) return ha < hb;
    return xa < xb;
  });
  std::vector<Pass> high;
  std::vector<int> hterms;
  for (int gi : rest) {
    const GroupH& g = h->groups[gi];
    if ((int)g.terms.size() > kMaxPassTerms)
      return fail(AQC_ENOTSUP, "a flip pattern has more terms than a pass holds");
    const uint64_t need = g.x & ~lowh;
    if (popc(need) > cap)
      return fail(AQC_ENOTSUP, "a flip pattern spans more bits than a high-pass tile holds");
    bool placed = false;
    for (size_t p2 = 0; p2 < high.size() && !placed; ++p2) {
      Pass& ps = high[p2];
      if (popc(ps.hmask | need) <= cap && (int)ps.groups.size() < kMaxPassGroups &&
          hterms[p2] + (int)g.terms.size() <= kMaxPassTerms) {
        ps.hmask |= need;
        ps.groups.push_back(gi);
        hterms[p2] += (int)g.terms.size();
        placed = true;
      }
    }
    if (!placed) {
      Pass ps;
      ps.final_pass = false;
      ps.lbits = lh;
      ps.hmask = need;
      ps.groups.push_back(gi);
      high.push_back(ps);
      hterms.push_back((int)g.terms.size());
    }
  }
  // fill every high tile to its full width with unused bits, lowest first
  for (Pass& ps : high) {
    for (int b = lh; b < n && popc(ps.hmask) < cap; ++b)
      if (!(ps.hmask >> b & 1ull)) ps.hmask |= 1ull << b;
    ps.tb = lh + popc(ps.hmask);
    ps.cmask = full & ~(lowh | ps.hmask);
  }
  out.clear();
  // highest hypercube first: the first register pass only writes the partial
  // product, the later ones also read it, and a pass with two input streams
  // loses less to long strides when its rows lie closer together (n = 30:
  // the two passes 1-3 % faster on average in this order)
  std::reverse(regp.begin(), regp.end());
  for (Pass& ps : regp) out.push_back(ps);
  for (Pass& ps : high) out.push_back(ps);
  out.push_back(last);
  *tbf_out = tbf;
  // the library's choice of register passes: a layout without them wins when
  // the tile high passes can take the single-qubit flips with fewer passes in
  // all (each pass streams the state once; with pair flips above the tile,
  // high passes are needed anyway and often have room for the single flips).
  // Not with stream groups, which would take the single flips as re-reads.
  if (use_reg == 1 && !use_stream && !regp.empty()) {
    std::vector<Pass> alt;
    int tbf_alt = 0;
    const std::string err = g_last_error;   // a layout that cannot be built is only not taken
    if (layout_passes(h, dtype, alt, &tbf_alt, tiles_only, 0) == AQC_OK && alt.size() < out.size()) {
      out.swap(alt);
      *tbf_out = tbf_alt;
    }
    g_last_error = err;
  }
  return AQC_OK;
}

static aqc_status build_plan_into(aqc_ham* h, Plan& p, int dtype, hipStream_t s, bool tiles_only) {
  std::lock_guard<std::recursive_mutex> lk(h->mu);
  if (p.built) return AQC_OK;
  if (h->sector_w >= 0) {
    // one kernel per product; it reads partners anywhere in its source, so
    // y^p is double-buffered like a last pass with stream groups
    p.passes.assign(1, Pass());
    p.passes[0].final_pass = true;
    p.has_stream = true;
    p.built = true;
    return AQC_OK;
  }
  HIPCHK(hipSetDevice(h->device));
  std::vector<Pass> passes;
  int tbf = 0;
  STCHK(layout_passes(h, dtype, passes, &tbf, tiles_only));
  p.tbf = tbf;
  p.passes = passes;
  p.has_stream = false;
  for (const Pass& ps : p.passes) p.has_stream = p.has_stream || ps.stream;
  for (Pass& ps : p.passes)
    if (ps.kind == 0) STCHK(build_pass_tables(ps, h, dtype, s));
  STCHK(build_diag_tables(p, h, s));
  p.built = true;
  return AQC_OK;
}

static aqc_status build_plan(aqc_ham* h, int dtype, hipStream_t s) {
  return build_plan_into(h, h->plans[dtype], dtype, s, false);
}

// ---------------------------------------------------------------------------
// pass execution
// ---------------------------------------------------------------------------
struct Coefs {
  double f[kMaxSched];
  double ident;  // identity terms at t
};

static Coefs coefs_at(const aqc_ham* h, double t) {
  Coefs c{};
  for (size_t s = 0; s < h->scheds.size(); ++s) c.f[s] = sched_value(h->scheds[s], h->path, t);
  c.ident = 0.0;
  for (const HTerm& it : h->ident) c.ident += it.w * c.f[it.sid];
  return c;
}

static void fill_common(PassArgs& a, const aqc_ham* h, const Plan& p, const Pass& ps,
                        const Coefs& c, double shift) {
  std::memset(&a, 0, sizeof(a));
  a.n = h->n;
  a.tb = ps.tb;
  a.lbits = ps.lbits;
  a.final_pass = ps.final_pass ? 1 : 0;
  a.hmask = ps.hmask;
  a.cmask = ps.cmask;
  a.groups = ps.dgroups;
  a.terms = ps.dterms;
  a.ng = ps.ng;
  a.nterms = ps.nterms;
  for (int i = 0; i < kMaxSched; ++i) a.f[i] = c.f[i];
  a.dconst = c.ident - shift;
  a.dg = p.dg;
}

// coefficient of each bit's single-qubit flip in a register pass
static void fill_reg_coefs(RegPassArgs& ra, const aqc_ham* h, const Pass& ps, const Coefs& c) {
  for (int b = 0; b < 12; ++b) {
    double cb = 0.0;
    if (b < ps.tb && ps.bit_group[b] >= 0)
      for (const HTerm& t : h->groups[ps.bit_group[b]].terms) cb += t.w * c.f[t.sid];
    ra.cb[b] = cb;
  }
}

// (H(t) - shift) u, with the last pass's epilogue `epi`.  hbuf: one vector when
// the plan has high passes.
static aqc_status run_sector_matvec(aqc_ctx* ctx, const aqc_ham* h, int dtype, double t,
                                    double shift, const void* u, const EpiDesc& epi);

static aqc_status run_matvec(aqc_ctx* ctx, const aqc_ham* h, int dtype, double t, double shift,
                             const void* u, void* hbuf, const EpiDesc& epi) {
  if (h->sector_w >= 0) return run_sector_matvec(ctx, h, dtype, t, shift, u, epi);
  const Plan& p = h->plans[dtype];
  const Coefs c = coefs_at(h, t);
  const int np = (int)p.passes.size();
  if (np > 1 && !hbuf) return fail(AQC_ENOMEM, "workspace for the partial product missing");
  for (int k = 0; k < np; ++k) {
    const Pass& ps = p.passes[k];
    if (ps.kind == 1) {
      RegPassArgs ra;
      std::memset(&ra, 0, sizeof(ra));
      ra.n = h->n;
      ra.hb = ps.hb;
      ra.wb = ps.wb;
      ra.src = u;
      ra.acc_in = k > 0 ? hbuf : nullptr;
      ra.acc_out = hbuf;
      fill_reg_coefs(ra, h, ps, c);
      if (ctx->prof_on) {
        aqc_ctx::Rec r;
        r.kind = AQC_PROF_HIGH_PASS;
        STCHK(prof_event(ctx, &r.a));
        STCHK(prof_event(ctx, &r.b));
        HIPCHK(hipEventRecord(r.a, ctx->stream));
        HIPCHK(launch_regpass(ra, dtype, ctx->stream));
        HIPCHK(hipEventRecord(r.b, ctx->stream));
        ctx->prof_pending.push_back(r);
        ctx->prof_bytes[r.kind] += (double)(2 + (ra.acc_in ? 1 : 0)) * (double)((size_t)1 << h->n) *
                                   (dtype == 0 ? 8.0 : 16.0);
        if (ctx->prof_pending.size() >= 4096) STCHK(prof_drain(ctx));
      } else {
        HIPCHK(launch_regpass(ra, dtype, ctx->stream));
      }
      continue;
    }
    PassArgs a;
    fill_common(a, h, p, ps, c, shift);
    a.src = u;
    if (!ps.final_pass) {
      a.acc_in = k > 0 ? hbuf : nullptr;
      a.acc_out = hbuf;
    } else {
      a.acc_in = np > 1 ? hbuf : nullptr;
      a.epi = epi;
    }
    const int64_t nb = (int64_t)1 << (h->n - ps.tb);
    if (ctx->prof_on) {
      aqc_ctx::Rec r;
      r.kind = ps.final_pass ? AQC_PROF_LAST_PASS : AQC_PROF_HIGH_PASS;
      STCHK(prof_event(ctx, &r.a));
      STCHK(prof_event(ctx, &r.b));
      HIPCHK(hipEventRecord(r.a, ctx->stream));
      HIPCHK(launch_pass(a, dtype, nb, ctx->stream));
      HIPCHK(hipEventRecord(r.b, ctx->stream));
      ctx->prof_pending.push_back(r);
      // algorithmic traffic: the tile source once, each streamed input and
      // output once, the partial product in and out
      int nvec = 1 + (a.acc_in ? 1 : 0) + (a.acc_out ? 1 : 0);
      int nlo = 0;
      if (ps.final_pass) {
        for (int i = 0; i < 4; ++i) nvec += a.epi.in[i] ? 1 : 0;
        for (int i = 0; i < 3; ++i) nvec += a.epi.out[i] ? 1 : 0;
        if (a.epi.comp) nlo = (a.epi.comp_flags & 8) ? 2 : 1;  // y_lo read (and written)
      }
      ctx->prof_bytes[r.kind] += ((double)nvec * (dtype == 0 ? 8.0 : 16.0) + 4.0 * nlo) *
                                 (double)((size_t)1 << h->n);
      if (ctx->prof_pending.size() >= 4096) STCHK(prof_drain(ctx));
    } else {
      HIPCHK(launch_pass(a, dtype, nb, ctx->stream));
    }
  }
  return AQC_OK;
}

static int64_t last_nblocks(const aqc_ham* h, int dtype) {
  if (h->sector_w >= 0) return sector_blocks(h->dim);
  return (int64_t)1 << (h->n - h->plans[dtype].tbf);
}

static aqc_status read_results(aqc_ctx* ctx, int k, double* out) {
  HIPCHK(hipMemcpyAsync(ctx->hres, ctx->dres, k * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < k; ++i) out[i] = ctx->hres[i];
  return AQC_OK;
}

static EpiDesc epi_zero() {
  EpiDesc e;
  std::memset(&e, 0, sizeof(e));
  return e;
}

static aqc_status check_common(aqc_ctx* ctx, const aqc_ham* h, int dtype) {
  if (!ctx) return fail(AQC_EINVAL, "ctx is NULL");
  if (!h) return fail(AQC_EINVAL, "ham is NULL");
  if (dtype != AQC_C64 && dtype != AQC_C128) return fail(AQC_ENOTSUP, "dtype must be C64 or C128");
  if (h->device != ctx->device) return fail(AQC_EINVAL, "ham built for another device");
  HIPCHK(hipSetDevice(ctx->device));
  return build_plan(const_cast<aqc_ham*>(h), dtype, ctx->stream);
}

static size_t vec_bytes(const aqc_ham* h, int dtype) {
  return (size_t)h->dim * (dtype == AQC_C64 ? 8 : 16);
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

extern "C" aqc_status aqc_ham_info(const aqc_ham* h, aqc_ham_info_t* out) {
  if (!h || !out) return fail(AQC_EINVAL, "aqc_ham_info: NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->n_qubits = h->n;
  out->n_terms = (int)h->terms.size();
  out->n_diag_terms = (int)(h->diag.size() + h->ident.size());
  out->n_groups = (int)h->groups.size();
  for (int d = 0; d < 2; ++d) {
    out->n_passes[d] = h->plans[d].built ? (int)h->plans[d].passes.size() : 0;
    out->tile_bits[d] = h->plans[d].built ? h->plans[d].tbf : 0;
  }
  out->spec_lo = NAN;
  out->spec_hi = NAN;
  return AQC_OK;
}

extern "C" aqc_status aqc_ham_set_tiling(aqc_ham* h, int dtype, int tbf, int tbh, int lh,
                                         int options) {
  if (!h) return fail(AQC_EINVAL, "aqc_ham_set_tiling: ham is NULL");
  if (h->sector_w >= 0) return fail(AQC_EINVAL, "aqc_ham_set_tiling: a sector has no tile plan");
  if (dtype != AQC_C64 && dtype != AQC_C128) return fail(AQC_ENOTSUP, "aqc_ham_set_tiling: dtype");
  const int maxtb = dtype == 0 ? 14 : 13;
  if (tbf < 1 || tbf > maxtb || tbh < 2 || tbh > maxtb || lh < 1 || lh >= tbh)
    return fail(AQC_EINVAL, "aqc_ham_set_tiling: tile bits out of range");
  if (options < 0 || options > 7)
    return fail(AQC_EINVAL, "aqc_ham_set_tiling: options is 0..7");
  std::lock_guard<std::recursive_mutex> lk(h->mu);
  // check the layout before replacing the plan
  const bool old_set = h->tiling_set[dtype];
  int old[4];
  std::memcpy(old, h->tiling[dtype], sizeof(old));
  h->tiling_set[dtype] = true;
  h->tiling[dtype][0] = tbf;
  h->tiling[dtype][1] = tbh;
  h->tiling[dtype][2] = lh;
  h->tiling[dtype][3] = options;
  std::vector<Pass> passes;
  int tb_out = 0;
  const aqc_status st = layout_passes(h, dtype, passes, &tb_out);
  if (st != AQC_OK) {
    h->tiling_set[dtype] = old_set;
    std::memcpy(h->tiling[dtype], old, sizeof(old));
    return st;
  }
  // the old plan's tables may still be read by queued launches: they are
  // released, not freed (see tab_release)
  if (h->plans[dtype].built) free_plan(h->plans[dtype], h->device);
  if (h->tplans[dtype].built) free_plan(h->tplans[dtype], h->device);
  if (h->n <= kEagerPlanMaxN) {
    // rebuilt now, as aqc_build_hamiltonian does, so that later calls need
    // no allocation (uploads on the null stream, into buffers that no queued
    // launch reads)
    HIPCHK(hipSetDevice(h->device));
    STCHK(build_plan(h, dtype, nullptr));
  }
  return AQC_OK;
}

// Number of passes of the plan and whether its last pass has stream groups
// (from the built plan, else from a layout computed on the host).
static aqc_status plan_shape(const aqc_ham* h, int dtype, size_t* np, bool* stream) {
  if (h->sector_w >= 0) {
    *np = 1;
    *stream = true;
    return AQC_OK;
  }
  const Plan& p = h->plans[dtype];
  if (p.built) {
    *np = p.passes.size();
    *stream = p.has_stream;
    return AQC_OK;
  }
  std::vector<Pass> passes;
  int tbf = 0;
  STCHK(layout_passes(h, dtype, passes, &tbf));
  *np = passes.size();
  *stream = false;
  for (const Pass& ps : passes) *stream = *stream || ps.stream;
  return AQC_OK;
}

extern "C" size_t aqc_apply_workspace_bytes(const aqc_ham* h, int dtype) {
  if (!h || (dtype != 0 && dtype != 1)) return 0;
  size_t np = 0;
  bool stream = false;
  if (plan_shape(h, dtype, &np, &stream) != AQC_OK) return 0;
  return np > 1 ? vec_bytes(h, dtype) : 0;
}

extern "C" aqc_status aqc_apply(aqc_ctx* ctx, const aqc_ham* h, double t, const void* in,
                                void* out, int dtype, void* ws, size_t ws_bytes) {
  STCHK(check_common(ctx, h, dtype));
  if (!in || !out) return fail(AQC_EINVAL, "aqc_apply: NULL state pointer");
  if (in == out) return fail(AQC_EINVAL, "aqc_apply: psi_in and psi_out must differ");
  if (!aligned16(in) || !aligned16(out)) return fail(AQC_EINVAL, "aqc_apply: pointers must be 16-byte aligned");
  if (!std::isfinite(t)) return fail(AQC_EINVAL, "aqc_apply: t not finite");
  const Plan& p = h->plans[dtype];
  void* hbuf = nullptr;
  if (p.passes.size() > 1) {
    if (!ws || ws_bytes < vec_bytes(h, dtype)) return fail(AQC_ENOMEM, "aqc_apply: workspace too small");
    hbuf = ws;
  }
  EpiDesc e = epi_zero();
  e.out[0] = out;
  e.scale[0] = 1.0;
  e.br[0] = 1.0;
  return run_matvec(ctx, h, dtype, t, 0.0, in, hbuf, e);
}

extern "C" aqc_status aqc_energy(aqc_ctx* ctx, const aqc_ham* h, double t, const void* psi,
                                 int dtype, void* ws, size_t ws_bytes, double* out) {
  STCHK(check_common(ctx, h, dtype));
  if (!psi || !out) return fail(AQC_EINVAL, "aqc_energy: NULL pointer");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "aqc_energy: psi must be 16-byte aligned");
  const Plan& p = h->plans[dtype];
  void* hbuf = nullptr;
  if (p.passes.size() > 1) {
    if (!ws || ws_bytes < vec_bytes(h, dtype)) return fail(AQC_ENOMEM, "aqc_energy: workspace too small");
    hbuf = ws;
  }
  const int64_t nb = last_nblocks(h, dtype);
  STCHK(ensure_parts(ctx, 3 * (size_t)nb));
  EpiDesc e = epi_zero();
  e.red = ctx->parts;
  e.red_flags = 4;
  STCHK(run_matvec(ctx, h, dtype, t, 0.0, psi, hbuf, e));
  HIPCHK(launch_reduce_sum(ctx->parts + 2 * nb, nb, 1, ctx->dres, ctx->stream));
  return read_results(ctx, 1, out);
}

// The energy of aqc_energy with no allocation and no caller workspace: the
// partial product and the reduction partials live in the device's fixed
// scratch array.  The plan must exist already (it is built with the
// Hamiltonian for n <= 26); nothing in the scratch needs clearing, since the
// first high pass writes the whole partial product and every workgroup of the
// last pass writes its partial sum.
extern "C" aqc_status aqc_energy_noalloc(aqc_ctx* ctx, const aqc_ham* h, double t, const void* psi,
                                         int dtype, double* out) {
  if (!ctx || !h || !psi || !out) return fail(AQC_EINVAL, "aqc_energy_noalloc: NULL argument");
  if (dtype != AQC_C64 && dtype != AQC_C128) return fail(AQC_ENOTSUP, "aqc_energy_noalloc: dtype");
  if (h->device != ctx->device) return fail(AQC_EINVAL, "aqc_energy_noalloc: ham built for another device");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "aqc_energy_noalloc: psi must be 16-byte aligned");
  if (!std::isfinite(t)) return fail(AQC_EINVAL, "aqc_energy_noalloc: t not finite");
  if (!ctx->scratch) return fail(AQC_EDEVICE, "aqc_energy_noalloc: no scratch address for this device");
  const Plan& p = h->plans[dtype];
  if (!p.built)
    return fail(AQC_EINVAL, "aqc_energy_noalloc: the Hamiltonian's plan for this dtype is not built "
                            "(it is built with the Hamiltonian up to 26 qubits; otherwise call "
                            "aqc_apply or aqc_energy once first)");
  const size_t vneed = p.passes.size() > 1 ? vec_bytes(h, dtype) : 0;
  const int64_t nb = last_nblocks(h, dtype);
  const size_t pneed = 3 * (size_t)nb * sizeof(double);
  if (vneed > kScratchVecBytes || pneed > kScratchPartBytes)
    return fail(AQC_ENOMEM, "aqc_energy_noalloc: needs " + std::to_string(vneed) +
                                " bytes for the partial product and " + std::to_string(pneed) +
                                " for the partials; the fixed scratch holds " +
                                std::to_string(kScratchVecBytes) + " and " +
                                std::to_string(kScratchPartBytes) + " (use aqc_energy)");
  HIPCHK(hipSetDevice(ctx->device));
  char* base = reinterpret_cast<char*>(ctx->scratch);
  void* hbuf = vneed ? base : nullptr;
  double* parts = reinterpret_cast<double*>(base + kScratchVecBytes);
  EpiDesc e = epi_zero();
  e.red = parts;
  e.red_flags = 4;
  // event timing would create events; it is skipped for this call
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  const aqc_status st = run_matvec(ctx, h, dtype, t, 0.0, psi, hbuf, e);
  ctx->prof_on = prof;
  STCHK(st);
  HIPCHK(launch_reduce_sum(parts + 2 * nb, nb, 1, ctx->dres, ctx->stream));
  return read_results(ctx, 1, out);
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
static aqc_status check_state(aqc_ctx* ctx, const void* psi, int dtype, int n) {
  if (!ctx) return fail(AQC_EINVAL, "ctx is NULL");
  if (!psi) return fail(AQC_EINVAL, "state pointer is NULL");
  if (dtype != 0 && dtype != 1) return fail(AQC_ENOTSUP, "dtype must be C64 or C128");
  if (n < 1 || n > 34) return fail(AQC_EINVAL, "n_qubits outside 1..34");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "state must be 16-byte aligned");
  HIPCHK(hipSetDevice(ctx->device));
  return AQC_OK;
}

static aqc_status norm2_len(aqc_ctx* ctx, const void* psi, int dtype, int64_t len, double* out) {
  STCHK(ensure_parts(ctx, 16384));
  int64_t nb = 0;
  HIPCHK(launch_norm2(psi, dtype, len, ctx->parts, &nb, ctx->stream));
  HIPCHK(launch_reduce_sum(ctx->parts, nb, 1, ctx->dres, ctx->stream));
  return read_results(ctx, 1, out);
}

extern "C" aqc_status aqc_norm2(aqc_ctx* ctx, const void* psi, int dtype, int n, double* out) {
  STCHK(check_state(ctx, psi, dtype, n));
  if (!out) return fail(AQC_EINVAL, "aqc_norm2: out is NULL");
  return norm2_len(ctx, psi, dtype, (int64_t)1 << n, out);
}

static aqc_status check_len(aqc_ctx* ctx, const void* psi, int dtype, int64_t len) {
  if (!ctx) return fail(AQC_EINVAL, "ctx is NULL");
  if (!psi) return fail(AQC_EINVAL, "state pointer is NULL");
  if (dtype != 0 && dtype != 1) return fail(AQC_ENOTSUP, "dtype must be C64 or C128");
  if (len < 1) return fail(AQC_EINVAL, "length < 1");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "state must be 16-byte aligned");
  HIPCHK(hipSetDevice(ctx->device));
  return AQC_OK;
}

extern "C" aqc_status aqc_norm2_len(aqc_ctx* ctx, const void* psi, int dtype, int64_t len,
                                    double* out) {
  STCHK(check_len(ctx, psi, dtype, len));
  if (!out) return fail(AQC_EINVAL, "aqc_norm2_len: out is NULL");
  return norm2_len(ctx, psi, dtype, len, out);
}

static aqc_status overlap_len(aqc_ctx* ctx, const void* phi, const void* psi, int dtype, int64_t len,
                              double* re, double* im);

extern "C" aqc_status aqc_overlap_len(aqc_ctx* ctx, const void* phi, const void* psi, int dtype,
                                      int64_t len, double* re, double* im) {
  STCHK(check_len(ctx, psi, dtype, len));
  STCHK(check_len(ctx, phi, dtype, len));
  if (!re || !im) return fail(AQC_EINVAL, "aqc_overlap_len: NULL output");
  return overlap_len(ctx, phi, psi, dtype, len, re, im);
}

extern "C" aqc_status aqc_overlap(aqc_ctx* ctx, const void* phi, const void* psi, int dtype, int n,
                                  double* re, double* im) {
  STCHK(check_state(ctx, psi, dtype, n));
  STCHK(check_state(ctx, phi, dtype, n));
  if (!re || !im) return fail(AQC_EINVAL, "aqc_overlap: NULL output");
  return overlap_len(ctx, phi, psi, dtype, (int64_t)1 << n, re, im);
}

static aqc_status overlap_len(aqc_ctx* ctx, const void* phi, const void* psi, int dtype, int64_t len,
                              double* re, double* im) {
  STCHK(ensure_parts(ctx, 2 * 16384));
  int64_t nb = 0;
  HIPCHK(launch_overlap(phi, psi, dtype, len, ctx->parts, &nb, ctx->stream));
  HIPCHK(launch_reduce_sum(ctx->parts, nb, 2, ctx->dres, ctx->stream));
  double r[2];
  STCHK(read_results(ctx, 2, r));
  *re = r[0];
  *im = r[1];
  return AQC_OK;
}

extern "C" aqc_status aqc_fidelity(aqc_ctx* ctx, const void* psi, int dtype, int n, int kind,
                                   const void* target, int64_t len, double* out) {
  STCHK(check_state(ctx, psi, dtype, n));
  if (!out || !target) return fail(AQC_EINVAL, "aqc_fidelity: NULL argument");
  if (kind == AQC_TARGET_STATE) {
    double re, im;
    STCHK(aqc_overlap(ctx, target, psi, dtype, n, &re, &im));
    *out = re * re + im * im;
    return AQC_OK;
  }
  if (kind != AQC_TARGET_BASIS_LIST) return fail(AQC_EINVAL, "aqc_fidelity: unknown target kind");
  if (len < 0) return fail(AQC_EINVAL, "aqc_fidelity: negative list length");
  const int64_t* li = reinterpret_cast<const int64_t*>(target);
  std::vector<int64_t> idx(li, li + len);
  std::sort(idx.begin(), idx.end());
  idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
  for (int64_t v : idx)
    if (v < 0 || v >= ((int64_t)1 << n)) return fail(AQC_EINVAL, "aqc_fidelity: basis index out of range");
  if (idx.empty()) {
    *out = 0.0;
    return AQC_OK;
  }
  if (idx.size() > ctx->didx_cap) {
    if (ctx->didx) {
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipFree(ctx->didx));
    }
    ctx->didx = nullptr;
    HIPCHK(hipMalloc(&ctx->didx, idx.size() * sizeof(int64_t)));
    ctx->didx_cap = idx.size();
  }
  HIPCHK(hipMemcpyAsync(ctx->didx, idx.data(), idx.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                        ctx->stream));
  STCHK(ensure_parts(ctx, 16384));
  int64_t nb = 0;
  HIPCHK(launch_gather_mass(psi, dtype, ctx->didx, (int64_t)idx.size(), ctx->parts, &nb, ctx->stream));
  HIPCHK(launch_reduce_sum(ctx->parts, nb, 1, ctx->dres, ctx->stream));
  return read_results(ctx, 1, out);
}

// diagonal of H(t) restricted to schedule weights f (float64 tables)
static void diag_args(PassArgs& a, const aqc_ham* h, const Plan& p, const double* f, double dconst) {
  std::memset(&a, 0, sizeof(a));
  a.n = h->n;
  a.tb = p.tbf;
  a.lbits = p.tbf;
  a.final_pass = 1;
  for (int i = 0; i < kMaxSched; ++i) a.f[i] = f[i];
  a.dconst = dconst;
  a.dg = p.dg;
}

static aqc_status sector_diag_minmax(aqc_ctx* ctx, const aqc_ham* h, const double* f,
                                     double dconst, double* mn, double* mx);

static aqc_status diag_minmax(aqc_ctx* ctx, const aqc_ham* h, const Plan& p, const double* f,
                              double dconst, double* mn, double* mx) {
  if (h->sector_w >= 0) return sector_diag_minmax(ctx, h, f, dconst, mn, mx);
  PassArgs a;
  diag_args(a, h, p, f, dconst);
  const int64_t nb = (int64_t)1 << (h->n - p.tbf);
  STCHK(ensure_parts(ctx, 2 * (size_t)nb));
  HIPCHK(launch_diag_minmax(a, nb, ctx->parts, ctx->stream));
  std::vector<double> host(2 * nb);
  HIPCHK(hipMemcpyAsync(host.data(), ctx->parts, 2 * nb * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double a0 = INFINITY, b0 = -INFINITY;
  for (int64_t i = 0; i < nb; ++i) {
    a0 = std::min(a0, host[i]);
    b0 = std::max(b0, host[nb + i]);
  }
  *mn = a0;
  *mx = b0;
  return AQC_OK;
}

// the arguments of a sector kernel for schedule values f and constant dconst
static SectorArgs sector_args(const aqc_ham* h, const double* f, double dconst) {
  SectorArgs a;
  std::memset(&a, 0, sizeof(a));
  a.s = h->sd;
  for (int i = 0; i < kMaxSched; ++i) a.f[i] = f[i];
  a.dconst = dconst;
  for (int k = 0; k < h->sd.dstore; ++k) a.dstore_f[k] = f[h->sd.dstore_sid[k]];
  return a;
}

extern "C" aqc_status aqc_ground_mass(aqc_ctx* ctx, const aqc_ham* h, double t, const void* psi,
                                      int dtype, double rel_tol, double* mass, double* e_min) {
  STCHK(check_common(ctx, h, dtype));
  if (!psi || !mass || !e_min) return fail(AQC_EINVAL, "aqc_ground_mass: NULL argument");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "aqc_ground_mass: psi must be 16-byte aligned");
  if (!(rel_tol >= 0.0)) return fail(AQC_EINVAL, "aqc_ground_mass: rel_tol < 0");
  // float64 tables of the same geometry as this dtype's last pass
  const Plan& p = h->plans[dtype];
  const Coefs c = coefs_at(h, t);
  double mn, mx;
  STCHK(diag_minmax(ctx, h, p, c.f, c.ident, &mn, &mx));
  const double thr = mn + rel_tol * std::max(1.0, std::fabs(mn));
  if (h->sector_w >= 0) {
    const SectorArgs sa = sector_args(h, c.f, c.ident);
    const int64_t nb = sector_blocks(h->dim);
    STCHK(ensure_parts(ctx, (size_t)nb));
    HIPCHK(launch_sector_diag(sa, 1, thr, psi, dtype, ctx->parts, ctx->stream));
    HIPCHK(launch_reduce_sum(ctx->parts, nb, 1, ctx->dres, ctx->stream));
    STCHK(read_results(ctx, 1, mass));
    *e_min = mn;
    return AQC_OK;
  }
  PassArgs a;
  diag_args(a, h, p, c.f, c.ident);
  a.src = psi;
  const int64_t nb = (int64_t)1 << (h->n - p.tbf);
  STCHK(ensure_parts(ctx, (size_t)nb));
  HIPCHK(launch_diag_mass(a, dtype, nb, thr, ctx->parts, ctx->stream));
  HIPCHK(launch_reduce_sum(ctx->parts, nb, 1, ctx->dres, ctx->stream));
  STCHK(read_results(ctx, 1, mass));
  *e_min = mn;
  return AQC_OK;
}

static aqc_status ensure_minmax(aqc_ctx* ctx, aqc_ham* h) {
  std::lock_guard<std::recursive_mutex> lk(h->mu);
  if (h->have_minmax) return AQC_OK;
  STCHK(build_plan(h, 1, ctx->stream));
  const Plan& p = h->plans[1];
  const int ns = (int)h->scheds.size();
  h->dmin.assign(ns, 0.0);
  h->dmax.assign(ns, 0.0);
  for (int s = 0; s < ns; ++s) {
    bool any = false;
    for (const HTerm& t : h->diag) any |= (t.sid == s);
    double idc = 0.0;
    for (const HTerm& t : h->ident)
      if (t.sid == s) idc += t.w;
    if (!any) {
      h->dmin[s] = h->dmax[s] = idc;
      continue;
    }
    double f[kMaxSched] = {0};
    f[s] = 1.0;
    double mn, mx;
    STCHK(diag_minmax(ctx, h, p, f, idc, &mn, &mx));
    h->dmin[s] = mn;
    h->dmax[s] = mx;
  }
  h->have_minmax = true;
  return AQC_OK;
}

static void enclosure_at(const aqc_ham* h, double t, double* lo, double* hi) {
  const Coefs c = coefs_at(h, t);
  double a = 0.0, b = 0.0;
  for (size_t s = 0; s < h->scheds.size(); ++s) {
    const double f = c.f[s];
    if (f >= 0) {
      a += f * h->dmin[s];
      b += f * h->dmax[s];
    } else {
      a += f * h->dmax[s];
      b += f * h->dmin[s];
    }
  }
  double off = 0.0;
  for (const GroupH& g : h->groups)
    for (const HTerm& t : g.terms) off += std::fabs(t.w * c.f[t.sid]);
  *lo = a - off;
  *hi = b + off;
}

extern "C" aqc_status aqc_spectral_bounds(aqc_ctx* ctx, const aqc_ham* hc, double t0, double t1,
                                          double* lo, double* hi) {
  if (!ctx || !hc || !lo || !hi) return fail(AQC_EINVAL, "aqc_spectral_bounds: NULL argument");
  aqc_ham* h = const_cast<aqc_ham*>(hc);
  HIPCHK(hipSetDevice(ctx->device));
  STCHK(ensure_minmax(ctx, h));
  double a = INFINITY, b = -INFINITY;
  const int K = 256;
  for (int k = 0; k <= K; ++k) {
    const double t = t0 + (t1 - t0) * k / K;
    double l, u;
    enclosure_at(h, t, &l, &u);
    a = std::min(a, l);
    b = std::max(b, u);
  }
  *lo = a;
  *hi = b;
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// Hamming-weight sectors (Sec. III.A.2-3)
// ---------------------------------------------------------------------------
static uint64_t binom64(int p, int k) {
  if (k < 0 || p < 0 || k > p) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(p - k + i) / (uint64_t)i;
  return r;
}

// Does the flip group g map every basis state of one weight to states of the
// same weight?  Its flips change two bits i, j; the weight is kept when they
// differ, and where they are equal the group's coefficient must vanish, for
// each schedule separately (the schedules are independent functions of t).
static aqc_status check_group_keeps_weight(const GroupH& g, int n_sched) {
  if (popc(g.x) != 2)
    return fail(AQC_EINVAL, "aqc_sector_create: a term flips other than two bits, so it changes "
                            "the Hamming weight");
  uint64_t u = 0;
  double wsum = 0.0;
  for (const HTerm& t : g.terms) {
    u |= t.z;
    wsum += std::fabs(t.w);
  }
  u &= ~g.x;
  if (popc(u) > 16) return fail(AQC_ENOTSUP, "aqc_sector_create: a pair term's Z string is too long to check");
  for (int s = 0; s < n_sched; ++s) {
    for (int both = 0; both < 2; ++both) {
      uint64_t sub = 0;
      do {
        const uint64_t y = sub | (both ? g.x : 0ull);
        const uint64_t src = y ^ g.x;
        double cr = 0.0, ci = 0.0;
        for (const HTerm& t : g.terms) {
          if (t.sid != s) continue;
          double m = (popc(src & t.z) & 1) ? -t.w : t.w;
          switch (popc(t.x & t.z) & 3) {
            case 0: cr += m; break;
            case 1: ci += m; break;
            case 2: cr -= m; break;
            default: ci -= m; break;
          }
        }
        if (std::hypot(cr, ci) > 1e-12 * std::max(1.0, wsum))
          return fail(AQC_EINVAL, "aqc_sector_create: a pair term connects states of different "
                                  "Hamming weight");
        sub = (sub - u) & u;  // next subset of u
      } while (sub != 0);
    }
  }
  return AQC_OK;
}

template <typename T>
static aqc_status sector_upload(aqc_ham* h, const std::vector<T>& v, const T** dst) {
  *dst = nullptr;
  if (v.empty()) return AQC_OK;
  void* d = nullptr;
  STCHK(tab_alloc(&d, v.size() * sizeof(T)));
  h->sec_bufs.push_back(d);
  HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = reinterpret_cast<const T*>(d);
  return AQC_OK;
}

extern "C" aqc_status aqc_sector_create(aqc_ctx* ctx, const aqc_ham* src, int weight, aqc_ham** out) {
  if (!ctx || !src || !out) return fail(AQC_EINVAL, "aqc_sector_create: NULL argument");
  *out = nullptr;
  if (src->sector_w >= 0) return fail(AQC_EINVAL, "aqc_sector_create: already a sector");
  if (src->device != ctx->device) return fail(AQC_EINVAL, "aqc_sector_create: ham built for another device");
  const int n = src->n;
  if (n > kSecMaxN) return fail(AQC_ENOTSUP, "aqc_sector_create: at most 34 qubits");
  if (weight < 0 || weight > n) return fail(AQC_EINVAL, "aqc_sector_create: weight outside 0..n");
  for (const GroupH& g : src->groups) STCHK(check_group_keeps_weight(g, (int)src->scheds.size()));
  HIPCHK(hipSetDevice(ctx->device));
  HamPtr h(new aqc_ham());
  h->n = n;
  h->device = src->device;
  h->scheds = src->scheds;
  h->path = src->path;
  h->terms = src->terms;
  h->diag = src->diag;
  h->ident = src->ident;
  h->groups = src->groups;
  h->sector_w = weight;
  h->dim = (int64_t)binom64(n, weight);
  SectorDev& sd = h->sd;
  sd.n = n;
  sd.w = weight;
  sd.zero_bits = weight > n - weight ? 1 : 0;
  sd.nch = (n + kSecChunkBits - 1) / kSecChunkBits;
  sd.dim = h->dim;
  std::vector<uint32_t> binom(kSecBinom * kSecBinom, 0u);
  for (int p = 0; p < kSecBinom; ++p)
    for (int k = 0; k < kSecBinom; ++k) binom[p * kSecBinom + k] = (uint32_t)binom64(p, k);
  // Rank part of chunk c holding the pattern `pat` when `cnt` 1-bits lie
  // below it: the sum over its set bits b (local order j) of
  // C(6c + b, cnt + j + 1), the combinatorial number system's terms of those
  // bits.  A weight-w state has between max(0, w - (n - 6c)) and min(6c, w)
  // 1-bits below chunk c; the rows cover that range and one spare row on each
  // side (a partner's count is one more or one less; lanes whose bits agree
  // read the spare rows and discard the result).
  const int CB = kSecChunkBits, CW = 1 << kSecChunkBits;
  std::vector<uint32_t> rtab;
  for (int c = 0; c < sd.nch; ++c) {
    const int lo = std::max(0, weight - (n - CB * c)), hi = std::min(CB * c, weight);
    const size_t off = rtab.size();
    sd.cbase[c] = (int32_t)off - (lo - 1) * CW;
    rtab.resize(off + (size_t)(hi - lo + 3) * CW, 0u);
    for (int cnt = lo; cnt <= hi; ++cnt)
      for (int pat = 0; pat < CW; ++pat) {
        if (cnt + popc((uint64_t)pat) > weight) continue;
        uint64_t v = 0;
        int j = 0;
        bool valid = true;
        for (int b = 0; b < CB; ++b) {
          if (!((pat >> b) & 1)) continue;
          if (CB * c + b >= n) valid = false;
          v += binom64(CB * c + b, cnt + j + 1);
          ++j;
        }
        if (valid && v <= 0xFFFFFFFFull) rtab[off + (size_t)(cnt - lo + 1) * CW + pat] = (uint32_t)v;
      }
  }
  sd.rwords = (int32_t)rtab.size();
  std::vector<SecHop> hops;
  std::vector<DevTerm> hterms;
  for (const GroupH& g : src->groups) {
    SecHop hp{};
    hp.x = g.x;
    hp.t0 = (int32_t)hterms.size();
    hp.nt = (int32_t)g.terms.size();
    hp.bi = __builtin_ctzll(g.x);
    hp.bj = 63 - __builtin_clzll(g.x);
    hp.fast = 1;
    for (const HTerm& t : g.terms) {
      hterms.push_back(DevTerm{t.z, t.w, t.sid, popc(t.x & t.z) & 3});
      if (t.z & ~g.x) hp.fast = 0;
    }
    hops.push_back(hp);
  }
  // runs of hops with the same chunk pair share their per-state work in k_sector
  auto chunk = [](int b) { return b / kSecChunkBits; };
  std::stable_sort(hops.begin(), hops.end(), [&](const SecHop& a, const SecHop& b) {
    return std::make_tuple(chunk(a.bi), chunk(a.bj), a.bi, a.bj) < std::make_tuple(chunk(b.bi), chunk(b.bj), b.bi, b.bj);
  });
  for (size_t k = 0; k < hops.size();) {
    size_t e = k + 1;
    while (e < hops.size() && chunk(hops[e].bi) == chunk(hops[k].bi) && chunk(hops[e].bj) == chunk(hops[k].bj)) ++e;
    hops[k].group = (int32_t)(e - k);
    for (size_t j = k + 1; j < e; ++j) hops[j].group = 0;
    k = e;
  }
  if (hterms.size() > (size_t)kSecMaxHopTerms)
    return fail(AQC_ENOTSUP, "aqc_sector_create: more than 1024 pair terms");
  if (hops.size() > (size_t)kSecMaxHops)
    return fail(AQC_ENOTSUP, "aqc_sector_create: more than 600 flip pairs");
  std::map<uint64_t, std::vector<HTerm>> bymask;
  std::vector<DevTerm> res;
  for (const HTerm& t : src->diag) {
    if (popc(t.z) <= 2) bymask[t.z].push_back(t);
    else res.push_back(DevTerm{t.z, t.w, t.sid, 0});
  }
  std::vector<SecMask> masks;
  std::vector<DevTerm> mterms;
  for (auto& kv : bymask) {
    const uint64_t z = kv.first;
    const int p = __builtin_ctzll(z);
    const uint64_t rest = z & (z - 1);
    SecMask m{p, rest ? __builtin_ctzll(rest) : -1, (int32_t)mterms.size(), (int32_t)kv.second.size()};
    for (const HTerm& t : kv.second) mterms.push_back(DevTerm{t.z, t.w, t.sid, 0});
    masks.push_back(m);
  }
  sd.nhops = (int)hops.size();
  sd.nhterms = (int)hterms.size();
  sd.nmasks = (int)masks.size();
  sd.nres = (int)res.size();
  STCHK(sector_upload(h.get(), binom, &sd.binom));
  STCHK(sector_upload(h.get(), rtab, &sd.rtab));
  STCHK(sector_upload(h.get(), hops, &sd.hops));
  STCHK(sector_upload(h.get(), hterms, &sd.hterms));
  STCHK(sector_upload(h.get(), masks, &sd.masks));
  STCHK(sector_upload(h.get(), mterms, &sd.mterms));
  STCHK(sector_upload(h.get(), res, &sd.res));
  // the diagonal is linear in the schedule values: with few schedules it is
  // kept per state, one part per schedule (each the diagonal with that
  // schedule at 1 and the others at 0), so that a product reads it instead
  // of summing the terms again
  std::vector<int> dsid;
  for (const HTerm& t : src->diag)
    if (std::find(dsid.begin(), dsid.end(), t.sid) == dsid.end()) dsid.push_back(t.sid);
  std::sort(dsid.begin(), dsid.end());
  sd.dstore = -1;
  sd.dtab = nullptr;
  if (dsid.size() <= (size_t)kSecDiagStore &&
      (double)dsid.size() * (double)h->dim * sizeof(double) <= (double)kSecDiagStoreBytes) {
    sd.dstore = (int32_t)dsid.size();
    for (size_t k = 0; k < dsid.size(); ++k) sd.dstore_sid[k] = dsid[k];
    if (!dsid.empty()) {
      void* d = nullptr;
      STCHK(tab_alloc(&d, dsid.size() * (size_t)h->dim * sizeof(double)));
      h->sec_bufs.push_back(d);
      double* dt = reinterpret_cast<double*>(d);
      for (size_t k = 0; k < dsid.size(); ++k) {
        SectorArgs a;
        std::memset(&a, 0, sizeof(a));
        a.s = sd;
        a.f[dsid[k]] = 1.0;
        HIPCHK(launch_sector_dtab(a, dt + k * (size_t)h->dim, ctx->stream));
      }
      HIPCHK(hipStreamSynchronize(ctx->stream));
      sd.dtab = dt;
    }
  }
  // a sector's plan is one kernel per product and needs no tables
  STCHK(build_plan(h.get(), 0, ctx->stream));
  STCHK(build_plan(h.get(), 1, ctx->stream));
  *out = h.release();
  return AQC_OK;
}

extern "C" int64_t aqc_ham_dim(const aqc_ham* h) { return h ? h->dim : 0; }

extern "C" int aqc_ham_sector_weight(const aqc_ham* h) { return h ? h->sector_w : -1; }

static aqc_status run_sector_matvec(aqc_ctx* ctx, const aqc_ham* h, int dtype, double t,
                                    double shift, const void* u, const EpiDesc& epi) {
  const Coefs c = coefs_at(h, t);
  SectorArgs a = sector_args(h, c.f, c.ident - shift);
  a.src = u;
  a.epi = epi;
  if (ctx->prof_on) {
    aqc_ctx::Rec r;
    r.kind = AQC_PROF_LAST_PASS;
    STCHK(prof_event(ctx, &r.a));
    STCHK(prof_event(ctx, &r.b));
    HIPCHK(hipEventRecord(r.a, ctx->stream));
    HIPCHK(launch_sector_matvec(a, dtype, ctx->stream));
    HIPCHK(hipEventRecord(r.b, ctx->stream));
    ctx->prof_pending.push_back(r);
    int nvec = 1;
    for (int i = 0; i < 4; ++i) nvec += epi.in[i] ? 1 : 0;
    for (int i = 0; i < 3; ++i) nvec += epi.out[i] ? 1 : 0;
    const int nlo = epi.comp ? ((epi.comp_flags & 8) ? 2 : 1) : 0;
    const int ndiag = std::max(0, (int)h->sd.dstore);   // stored diagonal parts, float64
    ctx->prof_bytes[r.kind] +=
        ((double)nvec * (dtype == 0 ? 8.0 : 16.0) + 4.0 * nlo + 8.0 * ndiag) * (double)h->dim;
    if (ctx->prof_pending.size() >= 4096) STCHK(prof_drain(ctx));
    return AQC_OK;
  }
  HIPCHK(launch_sector_matvec(a, dtype, ctx->stream));
  return AQC_OK;
}

static aqc_status sector_diag_minmax(aqc_ctx* ctx, const aqc_ham* h, const double* f,
                                     double dconst, double* mn, double* mx) {
  const SectorArgs a = sector_args(h, f, dconst);
  const int64_t nb = sector_blocks(h->dim);
  STCHK(ensure_parts(ctx, 2 * (size_t)nb));
  HIPCHK(launch_sector_diag(a, 0, 0.0, nullptr, 1, ctx->parts, ctx->stream));
  std::vector<double> host(2 * nb);
  HIPCHK(hipMemcpyAsync(host.data(), ctx->parts, 2 * nb * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double a0 = INFINITY, b0 = -INFINITY;
  for (int64_t i = 0; i < nb; ++i) {
    a0 = std::min(a0, host[i]);
    b0 = std::max(b0, host[nb + i]);
  }
  *mn = a0;
  *mx = b0;
  return AQC_OK;
}

extern "C" aqc_status aqc_sector_expand(aqc_ctx* ctx, const aqc_ham* sector, const void* psi_s,
                                        void* psi_full, int dtype) {
  if (!ctx || !sector || !psi_s || !psi_full) return fail(AQC_EINVAL, "aqc_sector_expand: NULL argument");
  if (sector->sector_w < 0) return fail(AQC_EINVAL, "aqc_sector_expand: not a sector");
  if (dtype != AQC_C64 && dtype != AQC_C128) return fail(AQC_ENOTSUP, "aqc_sector_expand: dtype");
  if (!aligned16(psi_s) || !aligned16(psi_full)) return fail(AQC_EINVAL, "aqc_sector_expand: alignment");
  if (psi_s == psi_full) return fail(AQC_EINVAL, "aqc_sector_expand: the two states must differ");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t full_bytes = ((size_t)1 << sector->n) * (dtype == AQC_C64 ? 8 : 16);
  HIPCHK(launch_zero(psi_full, full_bytes, ctx->stream));
  HIPCHK(launch_sector_expand(sector->sd, psi_s, psi_full, dtype, ctx->stream));
  return AQC_OK;
}

extern "C" aqc_status aqc_sector_dicke(aqc_ctx* ctx, const aqc_ham* sector, void* psi, int dtype) {
  if (!ctx || !sector || !psi) return fail(AQC_EINVAL, "aqc_sector_dicke: NULL argument");
  if (sector->sector_w < 0) return fail(AQC_EINVAL, "aqc_sector_dicke: not a sector");
  if (dtype != AQC_C64 && dtype != AQC_C128) return fail(AQC_ENOTSUP, "aqc_sector_dicke: dtype");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "aqc_sector_dicke: alignment");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_fill(psi, dtype, sector->dim, 1.0 / std::sqrt((double)sector->dim), 0.0, ctx->stream));
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// Lowest eigenvalues of H(t) (Sec. IV.B): thick-restart Lanczos with full
// reorthogonalisation.  The product, the dot products and the updates run on
// the device; the projected matrix (at most 48 x 48) is diagonalised here.
// ---------------------------------------------------------------------------
using cd = std::complex<double>;

// Cyclic Jacobi for a Hermitian matrix (row-major, n x n): each step makes
// a_pq real with a phase on column q, then zeroes it with a plane rotation.
// Eigenvalues ascending into w, eigenvectors as the columns of Z.
static void hermitian_jacobi(int n, std::vector<cd> A, std::vector<double>& w, std::vector<cd>& Z) {
  Z.assign((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  for (int i = 0; i < n; ++i) A[(size_t)i * n + i] = cd(A[(size_t)i * n + i].real(), 0.0);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p) {
      diag += std::norm(A[(size_t)p * n + p]);
      for (int q = p + 1; q < n; ++q) off += std::norm(A[(size_t)p * n + q]);
    }
    if (off <= 1e-32 * std::max(diag, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd apq = A[(size_t)p * n + q];
        const double r = std::abs(apq);
        if (r == 0.0) continue;
        const cd ph = apq / r;  // e^{i phi}
        const double app = A[(size_t)p * n + p].real(), aqq = A[(size_t)q * n + q].real();
        const double theta = (aqq - app) / (2.0 * r);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // U = diag(1, e^{-i phi}) [[c, s], [-s, c]] on (p, q)
        const cd upp = c, upq = s, uqp = -s * std::conj(ph), uqq = c * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // A <- A U
          const cd akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = akp * upp + akq * uqp;
          A[(size_t)k * n + q] = akp * upq + akq * uqq;
        }
        for (int k = 0; k < n; ++k) {  // A <- U^H A
          const cd apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = std::conj(upp) * apk + std::conj(uqp) * aqk;
          A[(size_t)q * n + k] = std::conj(upq) * apk + std::conj(uqq) * aqk;
        }
        A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
        A[(size_t)p * n + p] = A[(size_t)p * n + p].real();
        A[(size_t)q * n + q] = A[(size_t)q * n + q].real();
        for (int k = 0; k < n; ++k) {  // Z <- Z U
          const cd zkp = Z[(size_t)k * n + p], zkq = Z[(size_t)k * n + q];
          Z[(size_t)k * n + p] = zkp * upp + zkq * uqp;
          Z[(size_t)k * n + q] = zkp * upq + zkq * uqq;
        }
      }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    return A[(size_t)a * n + a].real() < A[(size_t)b * n + b].real();
  });
  w.resize(n);
  std::vector<cd> Zs((size_t)n * n);
  for (int i = 0; i < n; ++i) {
    w[i] = A[(size_t)idx[i] * n + idx[i]].real();
    for (int k = 0; k < n; ++k) Zs[(size_t)k * n + i] = Z[(size_t)k * n + idx[i]];
  }
  Z.swap(Zs);
}

extern "C" aqc_status aqc_hermitian_eigh(int n, const double* a, double* w, double* z) {
  if (n < 1 || n > 512 || !a || !w) return fail(AQC_EINVAL, "aqc_hermitian_eigh: bad argument");
  std::vector<cd> A((size_t)n * n);
  for (size_t i = 0; i < A.size(); ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
  std::vector<double> ev;
  std::vector<cd> Z;
  hermitian_jacobi(n, A, ev, Z);
  for (int i = 0; i < n; ++i) w[i] = ev[i];
  if (z)
    for (size_t i = 0; i < Z.size(); ++i) {
      z[2 * i] = Z[i].real();
      z[2 * i + 1] = Z[i].imag();
    }
  return AQC_OK;
}

namespace {
struct LzLayout {
  size_t vb, v, w, hbuf, coef, ymat, total;
};
LzLayout lz_layout(const aqc_ham* h, int dtype, int m) {
  LzLayout L{};
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  L.vb = al(vec_bytes(h, dtype));
  size_t np = 1;
  bool stream = false;
  plan_shape(h, dtype, &np, &stream);
  size_t off = 0;
  L.v = off;
  off += (size_t)m * L.vb;
  L.w = off;
  off += L.vb;
  L.hbuf = np > 1 ? off : (size_t)-1;
  if (np > 1) off += L.vb;
  L.coef = off;
  off += al(3 * 2 * kLzMaxBasis * sizeof(double));
  L.ymat = off;
  off += al(2 * kLzMaxBasis * kLzMaxKeep * sizeof(double));
  L.total = off;
  return L;
}
}  // namespace

extern "C" size_t aqc_lowest_eigs_workspace_bytes(const aqc_ham* h, int dtype, int max_basis) {
  if (!h || (dtype != 0 && dtype != 1) || max_basis < 3 || max_basis > kLzMaxBasis) return 0;
  return lz_layout(h, dtype, max_basis).total;
}

extern "C" aqc_status aqc_lowest_eigs(aqc_ctx* ctx, const aqc_ham* h, double t, int dtype, int n_eig,
                                      int max_basis, int max_matvecs, double tol, const void* start,
                                      void* ws, size_t ws_bytes, double* evals, double* resid,
                                      int* matvecs, void* ground_out) {
  STCHK(check_common(ctx, h, dtype));
  if (!evals || !resid || !matvecs) return fail(AQC_EINVAL, "aqc_lowest_eigs: NULL output");
  const int m = max_basis;
  if (n_eig < 1 || n_eig > 8 || m < n_eig + 2 || m > kLzMaxBasis)
    return fail(AQC_EINVAL, "aqc_lowest_eigs: need 1 <= n_eig <= 8 and n_eig + 2 <= max_basis <= 48");
  if (!(tol > 0.0) || !std::isfinite(t) || max_matvecs < m)
    return fail(AQC_EINVAL, "aqc_lowest_eigs: need tol > 0, finite t, max_matvecs >= max_basis");
  if (!ws || !aligned16(ws) || (start && !aligned16(start)) || (ground_out && !aligned16(ground_out)))
    return fail(AQC_EINVAL, "aqc_lowest_eigs: workspace/start must be 16-byte aligned device memory");
  const LzLayout L = lz_layout(h, dtype, m);
  if (ws_bytes < L.total) return fail(AQC_ENOMEM, "aqc_lowest_eigs: workspace too small");
  const int64_t N = h->dim;
  if (N < m) return fail(AQC_EINVAL, "aqc_lowest_eigs: max_basis exceeds the dimension");
  char* base = reinterpret_cast<char*>(ws);
  // basis vectors vb bytes apart (16-byte aligned); N amplitudes used in each
  auto V = [&](int j) { return (void*)(base + L.v + (size_t)j * L.vb); };
  void* w = base + L.w;
  void* hbuf = L.hbuf == (size_t)-1 ? nullptr : base + L.hbuf;
  double* coef = reinterpret_cast<double*>(base + L.coef);  // c1[2m], c2[2m], norm
  double* ymat = reinterpret_cast<double*>(base + L.ymat);
  const int64_t nb = lz_blocks(N);
  STCHK(ensure_parts(ctx, (size_t)2 * m * nb + 16));
  hipStream_t s = ctx->stream;
  const int64_t stride = (int64_t)(L.vb / (dtype == 0 ? 8 : 16));  // amplitudes between basis vectors

  // first vector: the given start or a fixed pseudo-random state, normalised
  if (start) HIPCHK(launch_copy(V(0), start, dtype, N, s));
  else HIPCHK(launch_random_fill(V(0), dtype, N, 0x5EEDull, s));
  double n0;
  STCHK(norm2_len(ctx, V(0), dtype, N, &n0));
  if (!(n0 > 0.0) || !std::isfinite(n0)) return fail(AQC_EINVAL, "aqc_lowest_eigs: zero or non-finite start");
  HIPCHK(launch_scale_copy(V(0), V(0), dtype, N, 1.0 / std::sqrt(n0), s));

  std::vector<cd> T((size_t)m * m, cd(0.0, 0.0));
  std::vector<double> host(4 * kLzMaxBasis + 2);
  int keep = 0, nmv = 0;
  const int kk = std::min(m - 2, std::max(n_eig + 4, 2 * n_eig));
  std::vector<double> theta;
  std::vector<cd> Y;
  double beta = 0.0;
  int m_eff = m;
  bool converged = false;
  while (true) {
    m_eff = m;
    bool invariant = false;
    for (int j = keep; j < m; ++j) {
      EpiDesc e = epi_zero();
      e.out[0] = w;
      e.scale[0] = 1.0;
      e.br[0] = 1.0;
      STCHK(run_matvec(ctx, h, dtype, t, 0.0, V(j), hbuf, e));
      ++nmv;
      // classical Gram-Schmidt twice against V_0..V_j
      for (int pass = 0; pass < 2; ++pass) {
        double* c = coef + pass * 2 * kLzMaxBasis;
        HIPCHK(launch_multidot(V(0), stride, N, j + 1, w, dtype, ctx->parts, s));
        HIPCHK(launch_reduce_sum(ctx->parts, nb, 2 * (j + 1), c, s));
        HIPCHK(launch_multiaxpy(V(0), stride, N, j + 1, c, w, dtype, ctx->parts, s));
      }
      HIPCHK(launch_reduce_sum(ctx->parts, nb, 1, coef + 4 * kLzMaxBasis, s));
      HIPCHK(hipMemcpyAsync(host.data(), coef, (4 * kLzMaxBasis + 1) * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i <= j; ++i) {
        const cd ci(host[2 * i] + host[2 * kLzMaxBasis + 2 * i],
                    host[2 * i + 1] + host[2 * kLzMaxBasis + 2 * i + 1]);
        T[(size_t)i * m + j] = ci;
        T[(size_t)j * m + i] = std::conj(ci);
      }
      T[(size_t)j * m + j] = cd(T[(size_t)j * m + j].real(), 0.0);
      beta = std::sqrt(std::max(host[4 * kLzMaxBasis], 0.0));
      double tnorm = 0.0;
      for (int i = 0; i <= j; ++i) tnorm = std::max(tnorm, std::abs(T[(size_t)i * m + i]));
      if (beta <= 1e-13 * std::max(1.0, tnorm)) {
        // the Krylov space is exhausted: an invariant subspace
        m_eff = j + 1;
        invariant = true;
        break;
      }
      if (j + 1 < m) HIPCHK(launch_scale_copy(V(j + 1), w, dtype, N, 1.0 / beta, s));
    }
    std::vector<cd> Tm((size_t)m_eff * m_eff);
    for (int i = 0; i < m_eff; ++i)
      for (int k = 0; k < m_eff; ++k) Tm[(size_t)i * m_eff + k] = T[(size_t)i * m + k];
    hermitian_jacobi(m_eff, Tm, theta, Y);
    const int ne = std::min(n_eig, m_eff);
    converged = true;
    for (int i = 0; i < ne; ++i) {
      const double r = invariant ? 0.0 : beta * std::abs(Y[(size_t)(m_eff - 1) * m_eff + i]);
      resid[i] = r;
      evals[i] = theta[i];
      if (r > tol * std::max(1.0, std::fabs(theta[i]))) converged = false;
    }
    for (int i = ne; i < n_eig; ++i) {
      evals[i] = NAN;
      resid[i] = NAN;
    }
    if (converged || invariant || nmv >= max_matvecs) break;
    // thick restart: keep the kk lowest Ritz vectors, continue from the residual
    std::vector<double> yh((size_t)2 * m * kk);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < kk; ++i) {
        yh[2 * ((size_t)j * kk + i)] = Y[(size_t)j * m + i].real();
        yh[2 * ((size_t)j * kk + i) + 1] = Y[(size_t)j * m + i].imag();
      }
    HIPCHK(hipMemcpyAsync(ymat, yh.data(), yh.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(launch_basis_transform(V(0), stride, N, m, kk, ymat, dtype, s));
    HIPCHK(launch_scale_copy(V(kk), w, dtype, N, 1.0 / beta, s));
    HIPCHK(hipStreamSynchronize(s));  // yh is freed at the end of this scope
    std::fill(T.begin(), T.end(), cd(0.0, 0.0));
    for (int i = 0; i < kk; ++i) T[(size_t)i * m + i] = theta[i];
    keep = kk;
  }
  *matvecs = nmv;
  if (ground_out) {
    // the lowest Ritz vector sum_j V_j Y[j][0], normalised by construction
    std::vector<double> y0((size_t)2 * m_eff);
    for (int j = 0; j < m_eff; ++j) {
      y0[2 * j] = Y[(size_t)j * m_eff].real();
      y0[2 * j + 1] = Y[(size_t)j * m_eff].imag();
    }
    HIPCHK(hipMemcpyAsync(ymat, y0.data(), y0.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(launch_basis_transform(V(0), stride, N, m_eff, 1, ymat, dtype, s));
    HIPCHK(launch_copy(ground_out, V(0), dtype, N, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (!converged && nmv >= max_matvecs)
    return fail(AQC_EUNSTABLE, "aqc_lowest_eigs: not converged within max_matvecs (values are the "
                               "last Ritz values)");
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// time evolution (Sec. II.B)
// ---------------------------------------------------------------------------
namespace {

constexpr double kMilne = 19.0 / 270.0;

struct Evolver {
  aqc_ctx* ctx;
  const aqc_ham* h;
  int dtype;
  double shift;
  int64_t N;
  size_t vb;
  int method;
  SolveVecs v;
  void* ckpt;        // adaptive: state at the window start
  void* ckpt_lo;     // adaptive: low part at the window start
  int64_t nb_last;
  aqc_evolve_stats* st;
  int check_every;
  double norm_tol;
  int64_t steps_since_check = 0;
  double* errbuf;    // device, per-step Milne sums of a window

  aqc_status norm_check(double t_now, int64_t k_global) {
    HIPCHK(launch_reduce_sum(ctx->parts, nb_last, 1, ctx->dres, ctx->stream));
    double val;
    STCHK(read_results(ctx, 1, &val));
    if (!std::isfinite(val) || std::fabs(val - st->norm2_initial) > norm_tol) {
      st->status_step = (int32_t)k_global;
      st->t_reached = t_now;
      char buf[160];
      snprintf(buf, sizeof buf, "norm guard: |psi|^2 = %.6g at t = %.6g (initial %.6g)", val, t_now,
               st->norm2_initial);
      return fail(AQC_EUNSTABLE, buf);
    }
    return AQC_OK;
  }

  // Take `nsteps` more steps of the segment `sg`; the Milne sums of its pc4
  // steps go to errbuf[0..] when want_err (count in *nerr).
  aqc_status advance(SegStepper& sg, int64_t nsteps, bool more_after, bool want_err, int* nerr) {
    sg.k_end = sg.k + nsteps;
    sg.more_after = more_after;
    int ne = 0;
    while (sg.k < sg.k_end) {
      MatvecStage m = sg.next(v);
      bool chk = false;
      if (m.ends_step && check_every > 0) chk = ((steps_since_check + 1) % check_every) == 0;
      if (chk) m.e.red_flags |= 1;
      if (m.pc4 && want_err) m.e.red_flags |= 2;
      if (m.e.red_flags) m.e.red = ctx->parts;
      STCHK(run_matvec(ctx, h, dtype, m.t, shift, m.src, v.hbuf, m.e));
      st->matvecs += 1;
      if (m.pc4 && want_err) {
        HIPCHK(launch_reduce_sum(ctx->parts + nb_last, nb_last, 1, errbuf + ne, ctx->stream));
        ++ne;
      }
      sg.advance();
      if (m.ends_step) {
        ++steps_since_check;
        st->steps += 1;
        if (chk) STCHK(norm_check(sg.ts + (double)sg.k * sg.h, st->steps));
      }
    }
    if (nerr) *nerr = ne;
    return AQC_OK;
  }
};

// Bytes of the low part of a compensated complex64 state: a bfloat16 pair per
// amplitude, rounded up to keep what follows aligned.
static size_t comp_bytes(const aqc_ham* h) {
  return ((size_t)h->dim * 4 + 255) & ~(size_t)255;
}

// Lay out the solve vectors in a workspace: y^p, four history vectors (pc4) or
// one accumulator (rk4), the partial product when the plan has high passes,
// the second y^p buffer when the last pass has stream groups, and the low part
// of a compensated complex64 state.  Advances *w.
aqc_status carve_workspace(const aqc_ham* h, int dtype, int method, bool compensated, void* psi,
                           char** w, SolveVecs* v, const Plan* plan = nullptr) {
  const Plan& pl = plan ? *plan : h->plans[dtype];
  const size_t vb = vec_bytes(h, dtype);
  v->y = psi;
  v->yp = *w;
  *w += vb;
  if (method == AQC_METHOD_RK4) {
    v->B[0] = *w;
    *w += vb;
    v->B[1] = v->B[2] = v->B[3] = nullptr;
  } else {
    for (int i = 0; i < 4; ++i) {
      v->B[i] = *w;
      *w += vb;
    }
  }
  v->hbuf = nullptr;
  if (pl.passes.size() > 1) {
    v->hbuf = *w;
    *w += vb;
  }
  v->yp2 = nullptr;
  if (pl.has_stream) {
    v->yp2 = *w;
    *w += vb;
  }
  v->ycomp = nullptr;
  if (dtype == AQC_C64 && compensated) {
    v->ycomp = *w;
    *w += comp_bytes(h);
  }
  return AQC_OK;
}

}  // namespace

extern "C" size_t aqc_evolve_workspace_bytes(const aqc_ham* h, int dtype, const aqc_evolve_opts* o) {
  if (!h || (dtype != 0 && dtype != 1)) return 0;
  const size_t vb = vec_bytes(h, dtype);
  const int method = o ? o->method : AQC_METHOD_PC4;
  size_t nv = method == AQC_METHOD_RK4 ? 2 : 5;
  size_t np = 0;
  bool stream = false;
  if (plan_shape(h, dtype, &np, &stream) != AQC_OK) return 0;
  if (np > 1) nv += 1;
  if (stream) nv += 1;
  const bool adaptive = o && o->n_steps == 0 && o->n_replay <= 0 && method == AQC_METHOD_PC4;
  const bool comp = dtype == AQC_C64 && (!o || o->compensated != 0);
  if (adaptive) nv += 1;
  return nv * vb + (comp ? (adaptive ? 2 : 1) * comp_bytes(h) : 0) + 256;
}

extern "C" aqc_status aqc_evolve(aqc_ctx* ctx, const aqc_ham* h, void* psi, int dtype, double t0,
                                 double t1, const aqc_evolve_opts* o, void* ws, size_t ws_bytes,
                                 aqc_evolve_stats* stats) {
  STCHK(check_common(ctx, h, dtype));
  if (!psi || !o || !stats) return fail(AQC_EINVAL, "aqc_evolve: NULL argument");
  if (!aligned16(psi)) return fail(AQC_EINVAL, "aqc_evolve: psi must be 16-byte aligned");
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0))
    return fail(AQC_EINVAL, "aqc_evolve: need finite t0 <= t1");
  if (o->method != AQC_METHOD_PC4 && o->method != AQC_METHOD_RK4)
    return fail(AQC_EINVAL, "aqc_evolve: unknown method");
  if (o->n_steps < 0) return fail(AQC_EINVAL, "aqc_evolve: n_steps < 0");
  const bool replay = o->n_replay > 0;
  if (replay && (!o->replay || o->method != AQC_METHOD_PC4))
    return fail(AQC_EINVAL, "aqc_evolve: replay needs a segment list and method PC4");
  const bool adaptive = o->n_steps == 0 && !replay;
  if (adaptive && o->method != AQC_METHOD_PC4)
    return fail(AQC_EINVAL, "aqc_evolve: adaptive stepping uses PC4");
  if (adaptive && (!(o->atol > 0.0) || !(o->h0 > 0.0) || o->window < 1))
    return fail(AQC_EINVAL, "aqc_evolve: adaptive stepping needs atol > 0, h0 > 0, window >= 1");
  const size_t need = aqc_evolve_workspace_bytes(h, dtype, o);
  if (!ws || ws_bytes < need)
    return fail(AQC_ENOMEM, "aqc_evolve: workspace needs " + std::to_string(need) + " bytes");
  if (!aligned16(ws)) return fail(AQC_EINVAL, "aqc_evolve: workspace must be 16-byte aligned");
  aqc_pc4_carry* cy = o->carry;
  const bool resume = cy && cy->valid;
  if (cy) {
    if (o->method != AQC_METHOD_PC4 || adaptive || replay)
      return fail(AQC_EINVAL, "aqc_evolve: a carry needs fixed-step pc4");
    if (resume) {
      const double hh = (t1 - t0) / o->n_steps;
      const double tnow = cy->t_start + (double)cy->k * cy->h;
      if (cy->ham != h || cy->psi != psi || cy->workspace != ws || cy->dtype != dtype ||
          !(std::fabs(hh - cy->h) <= 1e-12 * std::fabs(cy->h)) ||
          !(std::fabs(t0 - tnow) <= 1e-9 * std::max(1.0, std::fabs(tnow))) || cy->sub < 0 ||
          cy->sub > 4 || cy->k < 1)
        return fail(AQC_EINVAL, "aqc_evolve: the call does not continue its carry's chain "
                                "(same Hamiltonian, state, workspace, dtype and step; t0 = previous t1)");
    }
  }

  std::memset(stats, 0, sizeof(*stats));
  stats->status_step = -1;
  stats->t_reached = t0;
  aqc_ham* hm = const_cast<aqc_ham*>(h);
  // shift and stability guard
  double lo = 0, hi = 0;
  const bool need_enc = (o->shift_mode == AQC_SHIFT_CENTER && !resume) || o->stab_limit > 0.0;
  if (need_enc) STCHK(aqc_spectral_bounds(ctx, hm, t0, t1, &lo, &hi));
  double shift = resume ? cy->shift : o->shift_mode == AQC_SHIFT_CENTER ? 0.5 * (lo + hi) : o->shift;
  if (!std::isfinite(shift)) return fail(AQC_EINVAL, "aqc_evolve: shift not finite");
  stats->shift_used = shift;
  stats->rho = need_enc ? std::max(hi - shift, shift - lo) : NAN;

  Evolver ev;
  ev.ctx = ctx;
  ev.h = h;
  ev.dtype = dtype;
  ev.shift = shift;
  ev.N = h->dim;
  ev.vb = vec_bytes(h, dtype);
  ev.method = o->method;
  char* w = reinterpret_cast<char*>(ws);
  STCHK(carve_workspace(h, dtype, o->method, o->compensated != 0, psi, &w, &ev.v));
  ev.ckpt = nullptr;
  ev.ckpt_lo = nullptr;
  const bool comp = ev.v.ycomp != nullptr;
  // a continued chain keeps the low part of its state
  if (comp && !resume) HIPCHK(launch_zero(ev.v.ycomp, comp_bytes(h), ctx->stream));
  if (adaptive) {
    ev.ckpt = w;
    w += ev.vb;
    if (comp) {
      ev.ckpt_lo = w;
      w += comp_bytes(h);
    }
  }
  ev.nb_last = last_nblocks(h, dtype);
  ev.st = stats;
  ev.check_every = o->check_every;
  ev.norm_tol = o->norm_tol > 0 ? o->norm_tol : 1e-3;
  STCHK(ensure_parts(ctx, 3 * (size_t)ev.nb_last + 64));
  ev.errbuf = ctx->dres + 8;  // up to 56 per-step estimates per window
  if (adaptive && o->window > 56) return fail(AQC_EINVAL, "aqc_evolve: window must be <= 56");

  STCHK(norm2_len(ctx, psi, dtype, h->dim, &stats->norm2_initial));
  std::vector<double> segs;  // recorded (t_s, h, k)
  auto record = [&](const SegStepper& s) {
    if (s.k <= 0) return;
    segs.push_back(s.ts);
    segs.push_back(s.h);
    segs.push_back((double)s.k);
  };
  auto new_seg = [&](double ts, double hh) {
    SegStepper sg;
    sg.method = o->method;
    sg.ts = ts;
    sg.h = hh;
    sg.dbl = ev.v.yp2 != nullptr;
    return sg;
  };
  auto guard = [&](double hh) -> aqc_status {
    if (o->method == AQC_METHOD_PC4 && o->stab_limit > 0.0 && hh * stats->rho > o->stab_limit) {
      char buf[200];
      snprintf(buf, sizeof buf,
               "stability guard: h*rho = %.4g exceeds %.4g (h = %.4g, rho = %.4g after shift %.4g)",
               hh * stats->rho, o->stab_limit, hh, stats->rho, shift);
      return fail(AQC_EUNSTABLE, buf);
    }
    return AQC_OK;
  };

  aqc_status rc = AQC_OK;
  if (cy) {
    // a chain of fixed-step pc4 calls: continue the grid and the history; the
    // last step of every call forms the prediction for the next one
    SegStepper sg = new_seg(t0, (t1 - t0) / o->n_steps);
    if (resume) {
      sg.ts = cy->t_start;
      sg.h = cy->h;
      sg.k = cy->k;
      sg.sub = cy->sub;
      sg.ypc = cy->ypc;
    }
    STCHK(guard(sg.h));
    rc = ev.advance(sg, o->n_steps, true, false, nullptr);
    stats->h_last = sg.h;
    record(sg);
    if (rc == AQC_OK) {
      if (!resume) {
        cy->t_ref = t0;
        cy->shift = shift;
        cy->ham = h;
        cy->psi = psi;
        cy->workspace = ws;
        cy->dtype = dtype;
      }
      cy->valid = 1;
      cy->t_start = sg.ts;
      cy->h = sg.h;
      cy->k = sg.k;
      cy->sub = sg.sub;
      cy->ypc = sg.ypc;
      const double ph = -cy->shift * (t1 - cy->t_ref);
      cy->phase_re = std::cos(ph);
      cy->phase_im = std::sin(ph);
    } else {
      cy->valid = 0;
    }
  } else if (!adaptive) {
    std::vector<std::tuple<double, double, int64_t>> list;
    if (replay) {
      for (int i = 0; i < o->n_replay; ++i) {
        const double* r = o->replay + 3 * i;
        if (!(r[1] > 0) || !(r[2] >= 1) || !std::isfinite(r[0]))
          return fail(AQC_EINVAL, "aqc_evolve: bad replay segment");
        list.emplace_back(r[0], r[1], (int64_t)r[2]);
      }
    } else {
      list.emplace_back(t0, (t1 - t0) / o->n_steps, (int64_t)o->n_steps);
    }
    for (auto& s3 : list) STCHK(guard(std::get<1>(s3)));
    for (size_t i = 0; i < list.size() && rc == AQC_OK; ++i) {
      SegStepper sg = new_seg(std::get<0>(list[i]), std::get<1>(list[i]));
      rc = ev.advance(sg, std::get<2>(list[i]), false, false, nullptr);
      stats->h_last = sg.h;
      record(sg);
      stats->t_reached = sg.ts + (double)sg.k * sg.h;
    }
  } else {
    // adaptive predictor-corrector (windows of W steps, Milne estimates); the
    // step never grows past the stability guard
    const int W = o->window;
    double hmax = o->hmax > 0 ? o->hmax : INFINITY;
    if (o->stab_limit > 0.0 && stats->rho > 0.0) hmax = std::min(hmax, o->stab_limit / stats->rho);
    SegStepper sg = new_seg(t0, std::min(o->h0, hmax));
    int windows_at_h = 0;
    // halving stops at this floor: an error estimate that never falls below
    // atol (atol under the rounding floor of the dtype) ends the run instead
    // of shrinking the step without bound
    const double h_floor = std::max(o->hmin, 1e-12 * (t1 - t0));
    int rejections_in_row = 0;
    // the estimate of a step is formed from y^p and the new y in the state's
    // precision, so it cannot resolve errors below this floor; a tiny step's
    // estimate is pure rounding (or exactly zero) and the controller would
    // creep along at that step, so an atol below the floor is refused, and the
    // step only grows when the estimate is clearly above the floor
    const double unit = dtype == AQC_C64 ? 0x1p-24 : 0x1p-53;
    const double est_floor = 4.0 * kMilne * unit * std::sqrt(stats->norm2_initial);
    if (o->atol < est_floor) {
      char buf[200];
      snprintf(buf, sizeof buf,
               "adaptive step: atol %.3g is below the precision floor %.3g of the error estimate "
               "for this dtype", o->atol, est_floor);
      return fail(AQC_EUNSTABLE, buf);
    }
    const double grow_below = std::max(o->atol / 64.0, 8.0 * est_floor);
    while (rc == AQC_OK) {
      const double t_now = sg.ts + (double)sg.k * sg.h;
      const double left = t1 - t_now;
      if (left <= 0.0) break;
      const bool fin = left <= W * sg.h * (1.0 + 1e-12);
      int64_t nsteps = W;
      if (fin) {
        nsteps = std::max<int64_t>(1, (int64_t)std::ceil(left / sg.h - 1e-9));
        const double hf = left / (double)nsteps;
        if (hf != sg.h) {
          record(sg);
          sg = new_seg(t_now, hf);
          windows_at_h = 0;
        }
      }
      rc = guard(sg.h);
      if (rc != AQC_OK) break;
      HIPCHK(launch_copy(ev.ckpt, ev.v.y, dtype, ev.N, ctx->stream));
      if (ev.ckpt_lo) HIPCHK(hipMemcpyAsync(ev.ckpt_lo, ev.v.ycomp, (size_t)ev.N * 4, hipMemcpyDeviceToDevice, ctx->stream));
      const SegStepper before = sg;
      const int64_t steps_before = stats->steps;
      int ne = 0;
      rc = ev.advance(sg, nsteps, !fin, true, &ne);
      if (rc != AQC_OK) break;
      double emax = 0.0;
      if (ne > 0) {
        std::vector<double> tmp(8 + ne);
        STCHK(read_results(ctx, 8 + ne, tmp.data()));
        for (int i = 0; i < ne; ++i) emax = std::max(emax, kMilne * std::sqrt(tmp[8 + i]));
      }
      if (emax > o->atol) {
        if (sg.h / 2.0 < h_floor || ++rejections_in_row > 60) {
          stats->t_reached = before.ts + (double)before.k * before.h;
          HIPCHK(launch_copy(ev.v.y, ev.ckpt, dtype, ev.N, ctx->stream));
          if (ev.ckpt_lo) HIPCHK(hipMemcpyAsync(ev.v.ycomp, ev.ckpt_lo, (size_t)ev.N * 4, hipMemcpyDeviceToDevice, ctx->stream));
          char buf[200];
          snprintf(buf, sizeof buf,
                   "adaptive step: error estimate %.3g stays above atol %.3g down to h = %.3g "
                   "(atol below the precision floor?)", emax, o->atol, sg.h);
          rc = fail(AQC_EUNSTABLE, buf);
          break;
        }
        stats->rejected += (stats->steps - steps_before);
        stats->steps = steps_before;
        HIPCHK(launch_copy(ev.v.y, ev.ckpt, dtype, ev.N, ctx->stream));
        if (ev.ckpt_lo) HIPCHK(hipMemcpyAsync(ev.v.ycomp, ev.ckpt_lo, (size_t)ev.N * 4, hipMemcpyDeviceToDevice, ctx->stream));
        record(before);
        sg = new_seg(before.ts + (double)before.k * before.h, before.h / 2.0);
        windows_at_h = 0;
        continue;
      }
      stats->max_err = std::max(stats->max_err, emax);
      rejections_in_row = 0;
      ++windows_at_h;
      if (fin) {
        record(sg);
        stats->t_reached = sg.ts + (double)sg.k * sg.h;
        stats->h_last = sg.h;
        break;
      }
      if (emax < grow_below && windows_at_h >= 2 && 2.0 * sg.h <= hmax) {
        record(sg);
        sg = new_seg(sg.ts + (double)sg.k * sg.h, 2.0 * sg.h);
        windows_at_h = 0;
      }
      stats->h_last = sg.h;
      stats->t_reached = sg.ts + (double)sg.k * sg.h;
    }
  }
  stats->n_segments = (int32_t)(segs.size() / 3);
  if (o->record && o->record_cap > 0) {
    const size_t m = std::min<size_t>(segs.size(), (size_t)o->record_cap * 3);
    std::memcpy(o->record, segs.data(), m * sizeof(double));
  }
  if (rc != AQC_OK) return rc;
  if (shift != 0.0 && !cy) {
    const double ph = -shift * (t1 - t0);
    HIPCHK(launch_scale(psi, dtype, ev.N, std::cos(ph), std::sin(ph), ctx->stream));
  }
  STCHK(norm2_len(ctx, psi, dtype, h->dim, &stats->norm2_final));
  stats->t_reached = t1;
  return AQC_OK;
}

// ---------------------------------------------------------------------------
// batch engine: many fixed-step predictor-corrector solves advanced together
// ---------------------------------------------------------------------------
struct aqc_batch {
  aqc_ctx* ctx = nullptr;
  int dtype = 0;
  int capacity = 0;
  struct Slot {
    bool used = false, done = false, reported = false;
    const aqc_ham* h = nullptr;
    SolveVecs v{};
    SegStepper sg;
    double t0 = 0, t1 = 0, shift = 0;
    int64_t matvecs = 0;
    int nreg = 0, nwide = 0, nlds = 0;  // high passes of each kind in the slot's plan
    bool resident = false;              // run by one workgroup of a resident launch
    int64_t n_steps = 0;
  };
  std::vector<Slot> slots;
  // launch levels: register passes 0..R-1 (narrow, then wide), tile high
  // passes 0..L-1, then the last pass
  struct Level {
    int kind = 0;   // 1 narrow / 3 wide register pass, 0 tile high pass, 2 last pass
    int idx = 0;    // which pass of that kind in each slot's plan
    int max_tb = 0;
    std::vector<int> part;     // participating slots, in argument order
    std::vector<int2> map;     // block -> (participant, local block)
    int2* dmap = nullptr;      // this level's part of dmaps
    size_t arg_off = 0;        // byte offset of this level's arguments
  };
  std::vector<Level> levels;
  // the block maps of all levels, kept across rebuilds and only ever grown:
  // freeing device memory waits for every stream of the device, and a batch
  // rebuilds at every admission and retirement
  int2* dmaps = nullptr;
  size_t dmaps_cap = 0;        // int2 elements
  bool dirty = true;
  size_t args_bytes = 0;
  char* hargs[2] = {nullptr, nullptr};  // pinned
  size_t hargs_cap = 0;
  char* dargs = nullptr;
  size_t dargs_cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_pending[2] = {false, false};
  int cur = 0;
  // graphs: one executable per (pinned buffer, ticks per launch)
  bool use_graph = false;
  hipStream_t bs = nullptr;  // private stream for capture
  hipEvent_t sync_ev = nullptr;
  std::map<std::pair<int, int>, hipGraphExec_t> gexec;
  int64_t ticks = 0;
  // resident solves: admitted with n <= resident_max_n, launched together at
  // the next step (one workgroup each) on their own stream
  int resident_max_n = 0;
  hipStream_t rs = nullptr;
  hipEvent_t rs_ev = nullptr;        // orders rs after the context stream
  std::vector<int> res_pending;      // admitted, not launched yet
  struct ResLaunch {
    hipEvent_t done = nullptr;
    ResidentSolve* d = nullptr;      // device copy of the solves' descriptors
    std::vector<ResidentSolve> host; // the host copy it was made from
    std::vector<int> slots;
  };
  std::vector<ResLaunch> res_launches;
};

// ticks per launch group: arguments of up to this many ticks go up in one copy
// and (with graphs) run as one graph
constexpr int kBatchGroup = 32;
// largest solve a batch runs as a resident solve (one workgroup per solve)
constexpr int kResidentMaxN = 20;

// launch level of a pass: 0 tile high pass, 1 narrow register pass, 2 last
// pass, 3 wide register pass
static int level_kind(const Pass& ps) {
  if (ps.final_pass) return 2;
  if (ps.kind == 1) return ps.wb ? 3 : 1;
  return 0;
}

static bool is_reg_level(int kind) { return kind == 1 || kind == 3; }


static void batch_drop_graphs(aqc_batch* b) {
  for (auto& kv : b->gexec) hipGraphExecDestroy(kv.second);
  b->gexec.clear();
}

extern "C" aqc_status aqc_batch_create(aqc_ctx* ctx, int dtype, int capacity, aqc_batch** out) {
  if (!out) return fail(AQC_EINVAL, "aqc_batch_create: out is NULL");
  *out = nullptr;
  if (!ctx) return fail(AQC_EINVAL, "aqc_batch_create: ctx is NULL");
  if (ctx->closed.load()) return fail(AQC_EINVAL, "aqc_batch_create: context destroyed");
  if (dtype != AQC_C64 && dtype != AQC_C128) return fail(AQC_ENOTSUP, "aqc_batch_create: dtype");
  if (capacity < 1 || capacity > 65536) return fail(AQC_EINVAL, "aqc_batch_create: capacity 1..65536");
  HIPCHK(hipSetDevice(ctx->device));
  std::unique_ptr<aqc_batch> b(new aqc_batch());
  b->ctx = ctx;
  b->dtype = dtype;
  b->capacity = capacity;
  b->slots.resize(capacity);
  HIPCHK(hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&b->sync_ev, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&b->rs, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&b->rs_ev, hipEventDisableTiming));
  tab_stream_add(ctx->device, b->bs);
  tab_stream_add(ctx->device, b->rs);
  ctx->refs.fetch_add(1, std::memory_order_relaxed);  // released by aqc_batch_destroy
  *out = b.release();
  return AQC_OK;
}

// The batch's context was destroyed by its creator: no further work.
static aqc_status batch_ctx_live(const aqc_batch* b, const char* who) {
  if (b->ctx->closed.load()) return fail(AQC_EINVAL, std::string(who) + ": the batch's context was destroyed");
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_destroy(aqc_batch* b) {
  if (!b) return AQC_OK;
  hipSetDevice(b->ctx->device);
  hipStreamSynchronize(b->bs);
  if (b->rs) hipStreamSynchronize(b->rs);
  // the context stream is borrowed: once the context is destroyed it may be
  // gone, and aqc_destroy has already waited for it
  if (!b->ctx->closed.load()) hipStreamSynchronize(b->ctx->stream);
  for (auto& L : b->res_launches) {
    if (L.d) hipFree(L.d);
    if (L.done) hipEventDestroy(L.done);
  }
  if (b->rs_ev) hipEventDestroy(b->rs_ev);
  tab_stream_remove(b->ctx->device, b->bs);
  tab_stream_remove(b->ctx->device, b->rs);
  if (b->rs) hipStreamDestroy(b->rs);
  batch_drop_graphs(b);
  if (b->dmaps) hipFree(b->dmaps);
  for (int i = 0; i < 2; ++i) {
    if (b->hargs[i]) hipHostFree(b->hargs[i]);
    if (b->ev[i]) hipEventDestroy(b->ev[i]);
  }
  if (b->dargs) hipFree(b->dargs);
  if (b->sync_ev) hipEventDestroy(b->sync_ev);
  if (b->bs) hipStreamDestroy(b->bs);
  aqc_ctx* ctx = b->ctx;
  delete b;
  ctx_release(ctx);
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_set_graph(aqc_batch* b, int on) {
  if (!b) return fail(AQC_EINVAL, "aqc_batch_set_graph: NULL batch");
  b->use_graph = on != 0;
  batch_drop_graphs(b);
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_set_resident(aqc_batch* b, int max_n) {
  if (!b) return fail(AQC_EINVAL, "aqc_batch_set_resident: NULL batch");
  if (max_n < 0 || max_n > kResidentMaxN)
    return fail(AQC_EINVAL, "aqc_batch_set_resident: max_n is 0.." + std::to_string(kResidentMaxN));
  b->resident_max_n = max_n;
  return AQC_OK;
}

extern "C" size_t aqc_batch_workspace_bytes(const aqc_ham* h, int dtype) {
  aqc_evolve_opts o;
  std::memset(&o, 0, sizeof(o));
  o.method = AQC_METHOD_PC4;
  o.n_steps = 1;
  o.compensated = 1;
  return aqc_evolve_workspace_bytes(h, dtype, &o);
}

extern "C" aqc_status aqc_batch_admit(aqc_batch* b, const aqc_ham* h, void* psi, void* ws,
                                      size_t ws_bytes, double t0, double t1, int64_t n_steps,
                                      double shift, int* slot) {
  if (!b || !slot) return fail(AQC_EINVAL, "aqc_batch_admit: NULL argument");
  *slot = -1;
  STCHK(batch_ctx_live(b, "aqc_batch_admit"));
  STCHK(check_common(b->ctx, h, b->dtype));
  if (h->sector_w >= 0) return fail(AQC_ENOTSUP, "aqc_batch_admit: sectors are solved with aqc_evolve");
  if (!psi || !ws) return fail(AQC_EINVAL, "aqc_batch_admit: NULL state or workspace");
  if (!aligned16(psi) || !aligned16(ws)) return fail(AQC_EINVAL, "aqc_batch_admit: 16-byte alignment");
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 > t0) || n_steps < 1 || !std::isfinite(shift))
    return fail(AQC_EINVAL, "aqc_batch_admit: need t0 < t1, n_steps >= 1, finite shift");
  if (ws_bytes < aqc_batch_workspace_bytes(h, b->dtype))
    return fail(AQC_ENOMEM, "aqc_batch_admit: workspace too small");
  int s = -1;
  for (int i = 0; i < b->capacity; ++i)
    if (!b->slots[i].used) {
      s = i;
      break;
    }
  if (s < 0) return fail(AQC_EBUSY, "aqc_batch_admit: no free slot");
  // a resident solve runs the tile-pass plan of the Hamiltonian, with at most
  // kResMaxPass passes whose tiles fit the workgroup's LDS
  bool resident = false;
  if (b->resident_max_n > 0 && h->n <= b->resident_max_n) {
    aqc_ham* hm = const_cast<aqc_ham*>(h);
    if (build_plan_into(hm, hm->tplans[b->dtype], b->dtype, b->ctx->stream, true) == AQC_OK) {
      const Plan& tp = h->tplans[b->dtype];
      int max_tb = 0;
      for (const Pass& ps : tp.passes) max_tb = std::max(max_tb, ps.tb);
      resident = (int)tp.passes.size() <= kResMaxPass && !tp.has_stream &&
                 pass_lds_bytes(max_tb, b->dtype) + 4096 <= b->ctx->lds_max;
    } else {
      g_last_error.clear();
    }
  }
  aqc_batch::Slot& sl = b->slots[s];
  sl = aqc_batch::Slot();
  sl.used = true;
  sl.h = h;
  sl.resident = resident;
  sl.n_steps = n_steps;
  char* w = reinterpret_cast<char*>(ws);
  STCHK(carve_workspace(h, b->dtype, AQC_METHOD_PC4, true, psi, &w, &sl.v,
                        resident ? &h->tplans[b->dtype] : nullptr));
  if (sl.v.ycomp) HIPCHK(launch_zero(sl.v.ycomp, comp_bytes(h), b->ctx->stream));
  sl.sg.method = AQC_METHOD_PC4;
  sl.sg.ts = t0;
  sl.sg.h = (t1 - t0) / (double)n_steps;
  sl.sg.k_end = n_steps;
  sl.sg.more_after = false;
  sl.sg.dbl = sl.v.yp2 != nullptr;
  sl.t0 = t0;
  sl.t1 = t1;
  sl.shift = shift;
  if (resident) {
    b->res_pending.push_back(s);
    *slot = s;
    return AQC_OK;
  }
  for (const Pass& ps : h->plans[b->dtype].passes) {
    if (ps.final_pass) continue;
    const int k = level_kind(ps);
    if (k == 1) ++sl.nreg;
    else if (k == 3) ++sl.nwide;
    else ++sl.nlds;
  }
  b->dirty = true;
  *slot = s;
  return AQC_OK;
}

// Rebuild the launch levels and their block maps for the active slots.
static aqc_status batch_rebuild(aqc_batch* b) {
  // the previous launches read the block maps (and their host copies)
  if (b->dmaps) {
    HIPCHK(hipStreamSynchronize(b->ctx->stream));
    HIPCHK(hipStreamSynchronize(b->bs));
  }
  b->levels.clear();
  batch_drop_graphs(b);
  int maxr = 0, maxw = 0, maxl = 0;
  for (auto& sl : b->slots)
    if (sl.used && !sl.done && !sl.resident) {
      maxr = std::max(maxr, sl.nreg);
      maxw = std::max(maxw, sl.nwide);
      maxl = std::max(maxl, sl.nlds);
    }
  auto add_level = [&](int kind, int idx) {
    aqc_batch::Level L;
    L.kind = kind;
    L.idx = idx;
    for (int s = 0; s < b->capacity; ++s) {
      const auto& sl = b->slots[s];
      if (!sl.used || sl.done || sl.resident) continue;
      const Plan& p = sl.h->plans[b->dtype];
      // find the pass of this kind and index
      int seen = 0;
      const Pass* found = nullptr;
      for (const Pass& ps : p.passes) {
        if (level_kind(ps) != kind) continue;
        if (seen++ == idx) {
          found = &ps;
          break;
        }
      }
      if (!found) continue;
      const int pi = (int)L.part.size();
      L.part.push_back(s);
      int64_t nb;
      if (kind == 1 || kind == 3) {
        nb = regpass_blocks(sl.h->n, found->wb, b->dtype);
      } else {
        nb = (int64_t)1 << (sl.h->n - found->tb);
        L.max_tb = std::max(L.max_tb, found->tb);
      }
      for (int64_t q = 0; q < nb; ++q) L.map.push_back(int2{pi, (int)q});
    }
    if (!L.part.empty()) b->levels.push_back(std::move(L));
  };
  // a plan's register passes all have one width, so each slot still runs its
  // passes in plan order
  for (int r = 0; r < maxr; ++r) add_level(1, r);
  for (int r = 0; r < maxw; ++r) add_level(3, r);
  for (int l = 0; l < maxl; ++l) add_level(0, l);
  add_level(2, 0);
  size_t off = 0, moff = 0;
  for (auto& L : b->levels) {
    L.arg_off = off;
    off += L.part.size() * (is_reg_level(L.kind) ? sizeof(RegPassArgs) : sizeof(PassArgs));
    off = (off + 255) & ~(size_t)255;
    if (L.map.size() >= (size_t)INT32_MAX) return fail(AQC_ENOTSUP, "batch too large");
    moff += (L.map.size() + 31) & ~(size_t)31;   // 256-byte aligned parts
  }
  if (moff > b->dmaps_cap) {
    // (nothing reads the old maps any more: see above)
    if (b->dmaps) HIPCHK(hipFree(b->dmaps));
    b->dmaps = nullptr;
    b->dmaps_cap = 0;
    const size_t cap = moff + moff / 2;
    HIPCHK(hipMalloc(&b->dmaps, cap * sizeof(int2)));
    b->dmaps_cap = cap;
  }
  moff = 0;
  for (auto& L : b->levels) {
    L.dmap = b->dmaps + moff;
    moff += (L.map.size() + 31) & ~(size_t)31;
    // ordered before the batch's launches; L.map outlives the copy (the next
    // rebuild synchronises the stream first)
    HIPCHK(hipMemcpyAsync(L.dmap, L.map.data(), L.map.size() * sizeof(int2), hipMemcpyHostToDevice,
                          b->bs));
  }
  b->args_bytes = off;
  const size_t group_bytes = off * kBatchGroup;
  if (group_bytes > b->hargs_cap) {
    HIPCHK(hipStreamSynchronize(b->ctx->stream));
    HIPCHK(hipStreamSynchronize(b->bs));
    for (int i = 0; i < 2; ++i) {
      if (b->hargs[i]) HIPCHK(hipHostFree(b->hargs[i]));
      HIPCHK(hipHostMalloc(&b->hargs[i], group_bytes, hipHostMallocDefault));
      b->ev_pending[i] = false;
    }
    b->hargs_cap = group_bytes;
  }
  if (group_bytes > b->dargs_cap) {
    HIPCHK(hipStreamSynchronize(b->ctx->stream));
    HIPCHK(hipStreamSynchronize(b->bs));
    if (b->dargs) HIPCHK(hipFree(b->dargs));
    HIPCHK(hipMalloc(&b->dargs, group_bytes));
    b->dargs_cap = group_bytes;
  }
  b->dirty = false;
  return AQC_OK;
}

// Fill this tick's arguments of every level into the pinned buffer `buf`.
static void batch_fill_args(aqc_batch* b, char* buf) {
  // stage and coefficients of every active slot (one H|psi> each this tick)
  std::vector<MatvecStage> stage(b->capacity);
  std::vector<Coefs> coef(b->capacity);
  for (int s = 0; s < b->capacity; ++s) {
    auto& sl = b->slots[s];
    if (!sl.used || sl.done || sl.resident) continue;
    stage[s] = sl.sg.next(sl.v);
    coef[s] = coefs_at(sl.h, stage[s].t);
  }
  for (auto& L : b->levels) {
    for (size_t pi = 0; pi < L.part.size(); ++pi) {
      const int sidx = L.part[pi];
      aqc_batch::Slot& sl = b->slots[sidx];
      const aqc_ham* h = sl.h;
      const Plan& p = h->plans[b->dtype];
      const MatvecStage& m = stage[sidx];
      const Coefs& c = coef[sidx];
      // locate the pass and its position in the plan
      int seen = 0, kpos = -1;
      for (int k = 0; k < (int)p.passes.size(); ++k) {
        if (level_kind(p.passes[k]) != L.kind) continue;
        if (seen++ == L.idx) {
          kpos = k;
          break;
        }
      }
      const Pass& ps = p.passes[kpos];
      const int np = (int)p.passes.size();
      if (is_reg_level(L.kind)) {
        RegPassArgs* ra = reinterpret_cast<RegPassArgs*>(buf + L.arg_off) + pi;
        std::memset(ra, 0, sizeof(*ra));
        ra->n = h->n;
        ra->hb = ps.hb;
        ra->wb = ps.wb;
        ra->src = m.src;
        ra->acc_in = kpos > 0 ? sl.v.hbuf : nullptr;
        ra->acc_out = sl.v.hbuf;
        fill_reg_coefs(*ra, h, ps, c);
      } else {
        PassArgs* a = reinterpret_cast<PassArgs*>(buf + L.arg_off) + pi;
        fill_common(*a, h, p, ps, c, sl.shift);
        a->src = m.src;
        if (!ps.final_pass) {
          a->acc_in = kpos > 0 ? sl.v.hbuf : nullptr;
          a->acc_out = sl.v.hbuf;
        } else {
          a->acc_in = np > 1 ? sl.v.hbuf : nullptr;
          a->epi = m.e;
        }
      }
    }
  }
}

// The same work as a graph: a copy node, then one kernel node per level and
// tick in launch order.  Built node by node rather than by stream capture,
// so threads that drive other batches (or torch) need not pause meanwhile.
static aqc_status batch_build_graph(aqc_batch* b, const char* hbuf, int G, hipGraphExec_t* out) {
  hipGraph_t gr = nullptr;
  HIPCHK(hipGraphCreate(&gr, 0));
  struct Guard {
    hipGraph_t g;
    ~Guard() { hipGraphDestroy(g); }
  } guard{gr};
  hipGraphNode_t prev = nullptr, nd = nullptr;
  HIPCHK(hipGraphAddMemcpyNode1D(&nd, gr, nullptr, 0, b->dargs, hbuf, b->args_bytes * (size_t)G,
                                 hipMemcpyHostToDevice));
  prev = nd;
  for (int g = 0; g < G; ++g) {
    const char* dbase = b->dargs + b->args_bytes * (size_t)g;
    for (auto& L : b->levels) {
      const int64_t nb = (int64_t)L.map.size();
      if (is_reg_level(L.kind))
        HIPCHK(add_regpass_batch_node(gr, &nd, prev, reinterpret_cast<const RegPassArgs*>(dbase + L.arg_off),
                                      L.dmap, nb, L.kind == 3 ? kWaveBits : 0, b->dtype));
      else
        HIPCHK(add_pass_batch_node(gr, &nd, prev, reinterpret_cast<const PassArgs*>(dbase + L.arg_off), L.dmap,
                                   nb, L.kind == 2 ? 1 : 0, L.max_tb, b->dtype));
      prev = nd;
    }
  }
  HIPCHK(hipGraphInstantiate(out, gr, nullptr, nullptr, 0));
  return AQC_OK;
}

// Copy G ticks of arguments and launch every level of each tick in order.
static aqc_status batch_launch_group(aqc_batch* b, hipStream_t s, const char* hbuf, int G) {
  HIPCHK(hipMemcpyAsync(b->dargs, hbuf, b->args_bytes * (size_t)G, hipMemcpyHostToDevice, s));
  for (int g = 0; g < G; ++g) {
    const char* dbase = b->dargs + b->args_bytes * (size_t)g;
    for (auto& L : b->levels) {
      const int64_t nb = (int64_t)L.map.size();
      if (is_reg_level(L.kind))
        HIPCHK(launch_regpass_batch(reinterpret_cast<const RegPassArgs*>(dbase + L.arg_off), L.dmap,
                                    nb, L.kind == 3 ? kWaveBits : 0, b->dtype, s));
      else
        HIPCHK(launch_pass_batch(reinterpret_cast<const PassArgs*>(dbase + L.arg_off), L.dmap, nb,
                                 L.kind == 2 ? 1 : 0, L.max_tb, b->dtype, s));
    }
  }
  return AQC_OK;
}

// Launch the resident solves admitted since the last step: one workgroup
// each, on the batch's resident stream, after the context stream's work so
// far (the callers' initial states and the zeroed low parts).
static aqc_status batch_launch_resident(aqc_batch* b) {
  if (b->res_pending.empty()) return AQC_OK;
  std::vector<ResidentSolve> host(b->res_pending.size());
  int max_tb = 1;
  for (size_t i = 0; i < b->res_pending.size(); ++i) {
    const aqc_batch::Slot& sl = b->slots[b->res_pending[i]];
    const aqc_ham* h = sl.h;
    const Plan& tp = h->tplans[b->dtype];
    ResidentSolve& r = host[i];
    std::memset(&r, 0, sizeof(r));
    r.n = h->n;
    r.npass = (int)tp.passes.size();
    r.nsched = (int)h->scheds.size();
    r.dbl = 0;
    r.path = h->path;
    r.shift = sl.shift;
    r.t0 = sl.t0;
    r.t1 = sl.t1;
    r.h = (sl.t1 - sl.t0) / (double)sl.n_steps;
    r.K = sl.n_steps;
    for (const HTerm& it : h->ident) r.ident_w[it.sid] += it.w;
    for (int q = 0; q < r.nsched; ++q) r.sched[q] = h->scheds[q];
    r.v = sl.v;
    const Coefs zero{};
    for (int p = 0; p < r.npass; ++p) {
      const Pass& ps = tp.passes[p];
      fill_common(r.pass[p].pa, h, tp, ps, zero, sl.shift);
      r.pass[p].nblocks = (int64_t)1 << (h->n - ps.tb);
      max_tb = std::max(max_tb, ps.tb);
    }
  }
  aqc_batch::ResLaunch L;
  const size_t bytes = host.size() * sizeof(ResidentSolve);
  HIPCHK(hipMalloc(&L.d, bytes));
  HIPCHK(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
  L.slots = b->res_pending;
  b->res_pending.clear();
  HIPCHK(hipEventRecord(b->rs_ev, b->ctx->stream));
  HIPCHK(hipStreamWaitEvent(b->rs, b->rs_ev, 0));
  // the transfer reads the host descriptors: they live in the launch record
  // until the launch has finished
  L.host = std::move(host);
  HIPCHK(hipMemcpyAsync(L.d, L.host.data(), bytes, hipMemcpyHostToDevice, b->rs));
  HIPCHK(launch_resident(L.d, (int)L.host.size(), max_tb, b->dtype, b->rs));
  HIPCHK(hipEventRecord(L.done, b->rs));
  b->res_launches.push_back(std::move(L));
  return AQC_OK;
}

// Mark the solves of finished resident launches done (wait: block until the
// oldest launch has finished first).
static aqc_status batch_check_resident(aqc_batch* b, bool wait) {
  if (wait && !b->res_launches.empty()) HIPCHK(hipEventSynchronize(b->res_launches.front().done));
  for (size_t i = 0; i < b->res_launches.size();) {
    aqc_batch::ResLaunch& L = b->res_launches[i];
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    HIPCHK(q);
    for (int sidx : L.slots) {
      aqc_batch::Slot& sl = b->slots[sidx];
      sl.done = true;
      sl.sg.k = sl.n_steps;
      sl.matvecs = pc4_matvecs(sl.n_steps);
    }
    HIPCHK(hipFree(L.d));
    HIPCHK(hipEventDestroy(L.done));
    b->res_launches.erase(b->res_launches.begin() + (long)i);
  }
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_step(aqc_batch* b, int ticks, int* n_active) {
  if (!b) return fail(AQC_EINVAL, "aqc_batch_step: NULL batch");
  STCHK(batch_ctx_live(b, "aqc_batch_step"));
  HIPCHK(hipSetDevice(b->ctx->device));
  aqc_ctx* ctx = b->ctx;
  // order the private stream after the context stream's earlier work
  STCHK(batch_launch_resident(b));
  HIPCHK(hipEventRecord(b->sync_ev, ctx->stream));
  HIPCHK(hipStreamWaitEvent(b->bs, b->sync_ev, 0));
  const hipStream_t s = b->bs;
  int t = 0;
  bool ticked = false;
  while (t < ticks) {
    bool any = false;
    for (auto& sl : b->slots) any |= (sl.used && !sl.done && !sl.resident);
    if (!any) break;
    ticked = true;
    if (b->dirty) STCHK(batch_rebuild(b));
    // ticks in this group: no solve may finish inside it
    int64_t G = std::min<int64_t>(ticks - t, kBatchGroup);
    for (auto& sl : b->slots)
      if (sl.used && !sl.done && !sl.resident)
        G = std::min<int64_t>(G, pc4_matvecs(sl.sg.k_end) - sl.matvecs);
    if (G < 1) G = 1;
    const int c = b->cur;
    if (b->ev_pending[c]) HIPCHK(hipEventSynchronize(b->ev[c]));
    for (int g = 0; g < (int)G; ++g) {
      batch_fill_args(b, b->hargs[c] + b->args_bytes * (size_t)g);
      for (auto& sl : b->slots)
        if (sl.used && !sl.done && !sl.resident) {
          sl.sg.advance();
          ++sl.matvecs;
        }
    }
    if (b->use_graph) {
      auto key = std::make_pair(c, (int)G);
      auto it = b->gexec.find(key);
      if (it == b->gexec.end()) {
        hipGraphExec_t ex = nullptr;
        STCHK(batch_build_graph(b, b->hargs[c], (int)G, &ex));
        it = b->gexec.emplace(key, ex).first;
      }
      HIPCHK(hipGraphLaunch(it->second, s));
    } else {
      STCHK(batch_launch_group(b, s, b->hargs[c], (int)G));
    }
    HIPCHK(hipEventRecord(b->ev[c], s));
    b->ev_pending[c] = true;
    b->cur ^= 1;
    b->ticks += G;
    t += (int)G;
    for (auto& sl : b->slots) {
      if (!sl.used || sl.done || sl.resident) continue;
      if (sl.sg.k >= sl.sg.k_end) {
        sl.done = true;
        b->dirty = true;
        if (sl.shift != 0.0) {
          const double ph = -sl.shift * (sl.t1 - sl.t0);
          HIPCHK(launch_scale(sl.v.y, b->dtype, (int64_t)1 << sl.h->n, std::cos(ph), std::sin(ph), s));
        }
      }
    }
  }
  // the context stream continues after this step's work
  HIPCHK(hipEventRecord(b->sync_ev, s));
  HIPCHK(hipStreamWaitEvent(ctx->stream, b->sync_ev, 0));
  // resident solves: when there was nothing to tick, wait for the oldest
  // resident launch rather than return at once (callers loop on step)
  STCHK(batch_check_resident(b, !ticked));
  int na = 0;
  for (auto& sl : b->slots) na += (sl.used && !sl.done) ? 1 : 0;
  if (n_active) *n_active = na;
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_poll(aqc_batch* b, int* slots, int cap, int* n_done) {
  if (!b || !n_done || (cap > 0 && !slots)) return fail(AQC_EINVAL, "aqc_batch_poll: NULL argument");
  STCHK(batch_ctx_live(b, "aqc_batch_poll"));
  HIPCHK(hipSetDevice(b->ctx->device));
  STCHK(batch_check_resident(b, false));
  int n = 0;
  for (int s = 0; s < b->capacity; ++s) {
    auto& sl = b->slots[s];
    if (sl.used && sl.done && !sl.reported) {
      if (n < cap) {
        slots[n] = s;
        sl.reported = true;
      }
      ++n;
    }
  }
  *n_done = std::min(n, cap);
  if (*n_done > 0) HIPCHK(hipStreamSynchronize(b->bs));
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_retire(aqc_batch* b, int slot, aqc_evolve_stats* st) {
  if (!b || slot < 0 || slot >= b->capacity) return fail(AQC_EINVAL, "aqc_batch_retire: bad slot");
  auto& sl = b->slots[slot];
  if (!sl.used) return fail(AQC_EINVAL, "aqc_batch_retire: slot not in use");
  if (!sl.done) return fail(AQC_EBUSY, "aqc_batch_retire: solve not finished");
  STCHK(batch_ctx_live(b, "aqc_batch_retire"));
  HIPCHK(hipStreamSynchronize(b->bs));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->steps = sl.sg.k;
    st->matvecs = sl.matvecs;
    st->n_segments = 1;
    st->status_step = -1;
    st->t_reached = sl.t1;
    st->h_last = sl.sg.h;
    st->shift_used = sl.shift;
    st->rho = NAN;
  }
  sl = aqc_batch::Slot();
  return AQC_OK;
}

extern "C" aqc_status aqc_batch_info(const aqc_batch* b, int* active, int* finished, int64_t* ticks) {
  if (!b) return fail(AQC_EINVAL, "aqc_batch_info: NULL batch");
  int a = 0, f = 0;
  for (auto& sl : b->slots) {
    a += (sl.used && !sl.done) ? 1 : 0;
    f += (sl.used && sl.done) ? 1 : 0;
  }
  if (active) *active = a;
  if (finished) *finished = f;
  if (ticks) *ticks = b->ticks;
  return AQC_OK;
}
