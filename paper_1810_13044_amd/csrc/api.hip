// The C ABI of libslk: argument validation, graph handles and the SLK-BO host loop
// (Algorithm 1: outer mode updates around inner z-updates).
#include "common.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace slk {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

slk_status fail(slk_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

bool scratch_sync_alloc() {
  static const bool v = [] {
    const char* e = getenv("SLK_SCRATCH_MALLOC");
    return e && e[0] == '1';
  }();
  return v;
}

// Per-device stream-ordered pool for the calls' temporary buffers (and the served form's graphs).
// Freed blocks stay in the pool up to kPoolKeepBytes, so that the next call on the device reuses
// them instead of mapping fresh memory (the default pool returns everything at each synchronise).
namespace {
constexpr uint64_t kPoolKeepBytes = 4ull << 30;
constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pools[kMaxDevices] = {};
}  // namespace

hipError_t work_pool(hipMemPool_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (!g_pools[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    e = hipMemPoolCreate(&pool, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = kPoolKeepBytes;
    e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(pool);
      return e;
    }
    g_pools[dev] = pool;
  }
  *out = g_pools[dev];
  return hipSuccess;
}

struct Arena {
  int device = 0;
  std::vector<std::pair<char*, size_t>> chunks;  // (base, bytes)
  size_t ci = 0, off = 0;                        // carving position
  size_t demand = 0;                             // bytes carved by the current call
};

namespace {
constexpr size_t kArenaAlign = 256;
constexpr size_t kArenaMinChunk = 64ull << 20;
std::mutex g_arena_mu;
std::vector<Arena*> g_arenas_idle[kMaxDevices];
}  // namespace

Arena* arena_acquire() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    dev = 0;
  }
  Arena* a = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    if (!g_arenas_idle[dev].empty()) {
      a = g_arenas_idle[dev].back();
      g_arenas_idle[dev].pop_back();
    }
  }
  if (!a) {
    a = new Arena;
    a->device = dev;
  }
  a->ci = 0;
  a->off = 0;
  a->demand = 0;
  return a;
}

hipError_t arena_carve(Arena* a, size_t bytes, void** out) {
  bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
  a->demand += bytes;
  for (; a->ci < a->chunks.size(); ++a->ci, a->off = 0) {
    const auto& c = a->chunks[a->ci];
    if (a->off + bytes <= c.second) {
      *out = c.first + a->off;
      a->off += bytes;
      return hipSuccess;
    }
  }
  void* p = nullptr;
  const size_t cap = std::max(bytes, kArenaMinChunk);
  const hipError_t e = hipMalloc(&p, cap);
  if (e != hipSuccess) return e;
  a->chunks.push_back({static_cast<char*>(p), cap});
  a->ci = a->chunks.size() - 1;
  a->off = bytes;
  *out = p;
  return hipSuccess;
}

// The caller has synchronised the stream the memory was used on.  A call that needed more than
// one chunk leaves the arena with one chunk of its whole demand, so the next call carves from a
// single block.
void arena_release(Arena* a) {
  if (a->chunks.size() > 1) {
    for (auto& c : a->chunks) (void)hipFree(c.first);
    a->chunks.clear();
    void* p = nullptr;
    if (hipMalloc(&p, a->demand) == hipSuccess) a->chunks.push_back({static_cast<char*>(p), a->demand});
    else (void)hipGetLastError();
  }
  std::lock_guard<std::mutex> lk(g_arena_mu);
  g_arenas_idle[a->device].push_back(a);
}

// Frees the idle arenas of one device (those of calls in progress stay).
void arena_trim(int dev) {
  std::vector<Arena*> idle;
  {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    idle.swap(g_arenas_idle[dev]);
  }
  for (Arena* a : idle) {
    for (auto& c : a->chunks) (void)hipFree(c.first);
    delete a;
  }
}

hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
  hipMemPool_t pool = nullptr;
  const hipError_t e = work_pool(&pool);
  if (e != hipSuccess) return e;
  return hipMallocFromPoolAsync(p, bytes, pool, s);
}

slk_status pinned(void** out, size_t bytes) {
  thread_local void* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipHostMalloc(&buf, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      buf = nullptr;
      return fail(SLK_ERR_OUT_OF_MEMORY, "pinned host buffer");
    }
    cap = bytes;
  }
  *out = buf;
  return SLK_OK;
}

// per-kernel timing ---------------------------------------------------------------------------
namespace {
struct TimerPair {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::map<std::string, std::pair<int64_t, double>> g_tacc;
std::vector<TimerPair> g_tpend;
std::vector<hipEvent_t> g_tpool;

hipEvent_t take_event() {
  if (!g_tpool.empty()) {
    hipEvent_t e = g_tpool.back();
    g_tpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}
}  // namespace

bool timing_on() { return g_timing; }

int timer_start(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_tmu);
  TimerPair t{name, take_event(), take_event()};
  if (!t.a || !t.b) return -1;
  (void)hipEventRecord(t.a, s);
  g_tpend.push_back(t);
  return (int)g_tpend.size() - 1;
}

void timer_stop(int slot, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (slot >= 0 && slot < (int)g_tpend.size()) (void)hipEventRecord(g_tpend[slot].b, s);
}

void timing_flush() {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& t : g_tpend) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      auto& acc = g_tacc[t.name];
      acc.first += 1;
      acc.second += ms;
    }
    (void)hipGetLastError();
    g_tpool.push_back(t.a);
    g_tpool.push_back(t.b);
  }
  g_tpend.clear();
}

void timing_retag_tail(const char* name, int count, const char* to) {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto it = g_tpend.rbegin(); it != g_tpend.rend() && count > 0; ++it)
    if (it->name == name) {
      it->name = to;
      --count;
    }
}

// Host-visible mirror of the z-update loop state (two slots, alternating by pass) and one event
// per slot, per device and thread.  The pass reduction stores the state there, so the host loop
// watches the z-updates without a copy on the stream.
// The results of one outer iteration, written by its kernels straight into host-mapped memory:
// the host reads them after one synchronise, with no copies on the stream.
struct OuterHost {
  double eout[2];        // unary sums: FP32 path, FP64 recheck
  long long cut;
  double bound;          // relaxed bound at the final pass's input
  int32_t modes_next[256];
};

struct Watch {
  IterState* host = nullptr;
  IterState* dev = nullptr;
  OuterHost* oh_host = nullptr;
  OuterHost* oh_dev = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
};

slk_status watch_for_device(Watch** out) {
  thread_local std::map<int, Watch> per_dev;
  int dev = 0;
  SLK_HIP(hipGetDevice(&dev));
  Watch& w = per_dev[dev];
  if (!w.host) {
    // two IterState slots, then the OuterHost block (IterState's size keeps it 8-byte aligned)
    void* h = nullptr;
    if (hipHostMalloc(&h, 2 * sizeof(IterState) + sizeof(OuterHost), hipHostMallocCoherent | hipHostMallocMapped) !=
        hipSuccess) {
      (void)hipGetLastError();
      return fail(SLK_ERR_OUT_OF_MEMORY, "pinned loop-state mirror");
    }
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(h);
      return fail(SLK_ERR_DEVICE, "device address of the loop-state mirror");
    }
    for (auto& e : w.ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SLK_ERR_DEVICE, "loop-state event");
      }
    w.host = (IterState*)h;
    w.dev = (IterState*)d;
    w.oh_host = reinterpret_cast<OuterHost*>(w.host + 2);
    w.oh_dev = reinterpret_cast<OuterHost*>(w.dev + 2);
  }
  *out = &w;
  return SLK_OK;
}

// kernels local to this file ----------------------------------------------------------------
namespace {

__global__ void init_state_kernel(IterState* st, double tol, int check, int cap, int last_pass) {
  st->pass = 0;
  st->done = 0;
  st->numeric = 0;
  st->tol = tol;
  st->check = check;
  st->trace_cap = cap;
  st->last_bound = 0.0;
  st->rel = 0.0;
  st->rel_prev = 0.0;
  st->last_pass = last_pass;
  st->emit_pass = -1;
}

__global__ void check_indices_kernel(const int32_t* __restrict__ v, int64_t count, int64_t n, int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    if (v[i] < 0 || v[i] >= n) atomicOr(bad, 1);
}

__global__ void check_row_ptr_kernel(const int32_t* __restrict__ rp, int64_t n, int64_t nnz, int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (rp[i + 1] < rp[i]) atomicOr(bad, 1);
    if (i == 0 && rp[0] != 0) atomicOr(bad, 1);
    if (i == n - 1 && rp[n] != nnz) atomicOr(bad, 1);
  }
}

__global__ void check_labels_kernel(const int32_t* __restrict__ v, int64_t n, int L, int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (v[i] < 0 || v[i] >= L) atomicOr(bad, 1);
}

__global__ void check_finite_kernel(const float* __restrict__ v, int64_t count, int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) atomicOr(bad, 1);
}

__global__ void divide_kernel(double* v, double by) { *v = *v / by; }

slk_status device_flag(hipStream_t s, const char* what, int (*launch)(int32_t*, hipStream_t, const void*),
                       const void* ctx) {
  Scratch sc(s);
  int32_t* bad;
  SLK_TRY(sc.get(&bad, 1));
  SLK_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  launch(bad, s, ctx);
  SLK_LAUNCHED(what);
  int32_t h = 0;
  SLK_HIP(hipMemcpyAsync(&h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  if (h) return fail(SLK_ERR_INVALID_ARG, std::string("invalid device data: ") + what);
  return SLK_OK;
}

struct IdxCtx {
  const int32_t* v;
  int64_t count, n;
};
struct RpCtx {
  const int32_t* rp;
  int64_t n, nnz;
};
struct LabCtx {
  const int32_t* v;
  int64_t n;
  int L;
};
struct FinCtx {
  const float* v;
  int64_t count;
};

inline unsigned grid_for(int64_t count) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 4096)); }

slk_status check_indices(const int32_t* v, int64_t count, int64_t n, hipStream_t s, const char* what) {
  IdxCtx c{v, count, n};
  return device_flag(
      s, what,
      [](int32_t* bad, hipStream_t st, const void* p) {
        auto* c = static_cast<const IdxCtx*>(p);
        hipLaunchKernelGGL(check_indices_kernel, dim3(grid_for(c->count)), dim3(256), 0, st, c->v, c->count, c->n, bad);
        return 0;
      },
      &c);
}

slk_status check_finite(const float* v, int64_t count, hipStream_t s) {
  FinCtx c{v, count};
  return device_flag(
      s, "points must be finite",
      [](int32_t* bad, hipStream_t st, const void* p) {
        auto* c = static_cast<const FinCtx*>(p);
        hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(c->count)), dim3(256), 0, st, c->v, c->count, bad);
        return 0;
      },
      &c);
}

slk_status check_labels(const int32_t* v, int64_t n, int L, hipStream_t s) {
  LabCtx c{v, n, L};
  return device_flag(
      s, "labels must lie in [0, L)",
      [](int32_t* bad, hipStream_t st, const void* p) {
        auto* c = static_cast<const LabCtx*>(p);
        hipLaunchKernelGGL(check_labels_kernel, dim3(grid_for(c->n)), dim3(256), 0, st, c->v, c->n, c->L, bad);
        return 0;
      },
      &c);
}

slk_status check_row_ptr(const int32_t* rp, int64_t n, int64_t nnz, hipStream_t s) {
  RpCtx c{rp, n, nnz};
  return device_flag(
      s, "row_ptr must start at 0, be non-decreasing and end at nnz",
      [](int32_t* bad, hipStream_t st, const void* p) {
        auto* c = static_cast<const RpCtx*>(p);
        hipLaunchKernelGGL(check_row_ptr_kernel, dim3(grid_for(c->n)), dim3(256), 0, st, c->rp, c->n, c->nnz, bad);
        return 0;
      },
      &c);
}

// ------------------------------------------------------------------------------------------
// graph helpers
// ------------------------------------------------------------------------------------------
thread_local bool t_graph_pool = false;

}  // namespace

void set_graph_pool(bool on) { t_graph_pool = on; }
bool graph_pool() { return t_graph_pool; }

hipError_t graph_alloc(void** p, size_t bytes, hipStream_t s) {
  return t_graph_pool ? pool_alloc(p, bytes, s) : hipMalloc(p, bytes);
}

void graph_free(void* p, bool pooled, hipStream_t s) {
  if (!p) return;
  if (pooled) (void)hipFreeAsync(p, s);
  else (void)hipFree(p);
}

namespace {

// Releases the arrays; pooled arrays are freed in the order of stream s.
void free_graph(slk_graph* g, hipStream_t s) {
  if (!g) return;
  const bool pl = g->pooled != 0;
  for (void* p : {(void*)g->row_ptr, (void*)g->col_idx, (void*)g->knn_idx, (void*)g->knn_d2, (void*)g->perm,
                  (void*)g->iperm, (void*)g->heavy})
    graph_free(p, pl, s);
  delete g;
}


struct GraphGuard {
  slk_graph* g;
  hipStream_t s;
  ~GraphGuard() { free_graph(g, s); }
  slk_graph* release() {
    slk_graph* r = g;
    g = nullptr;
    return r;
  }
};

// The rows of degree > kHeavyDeg (internal numbering), largest degree first, ties by row, from a
// host copy of row_ptr.
slk_status heavy_from(slk_graph* g, const std::vector<int32_t>& rp, hipStream_t s) {
  graph_free(g->heavy, g->pooled, s);
  g->heavy = nullptr;
  g->n_heavy = 0;
  const int64_t n = g->n;
  std::vector<int32_t> h;
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] - rp[i] > kHeavyDeg) h.push_back((int32_t)i);
  std::stable_sort(h.begin(), h.end(), [&](int32_t u, int32_t v) { return rp[u + 1] - rp[u] > rp[v + 1] - rp[v]; });
  if (h.empty()) return SLK_OK;
  SLK_HIP(graph_alloc((void**)&g->heavy, sizeof(int32_t) * h.size(), s));
  SLK_HIP(hipMemcpyAsync(g->heavy, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s));
  SLK_HIP(hipStreamSynchronize(s));
  g->n_heavy = (int64_t)h.size();
  return SLK_OK;
}

slk_status build_heavy(slk_graph* g, hipStream_t s) {
  std::vector<int32_t> rp(g->n + 1);
  SLK_HIP(hipMemcpyAsync(rp.data(), g->row_ptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  return heavy_from(g, rp, s);
}

// Breadth-first order of the graph, component by component (roots in increasing index
// order), neighbours visited in CSR order.  Points that are neighbours end up close in the
// internal numbering, so a z-update's neighbour reads stay within a narrow window of Z.
// The queue is visited in an order unrelated to the row numbering, so each row costs two cache
// misses (its row_ptr entry and the start of its columns); both are prefetched from queue entries
// further ahead (kPfRow and kPfCol rows), which halves the walk over a million shuffled rows.
// The host buffers are left uninitialised: the copies overwrite them.
slk_status bfs_reorder(slk_graph* g, hipStream_t s) {
  constexpr int64_t kPfRow = 32, kPfCol = 16;
  const int64_t n = g->n;
  std::unique_ptr<int32_t[]> rp(new int32_t[n + 1]), ci(new int32_t[std::max<int64_t>(g->nnz, 1)]);
  SLK_HIP(hipMemcpyAsync(rp.get(), g->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
  if (g->nnz) SLK_HIP(hipMemcpyAsync(ci.get(), g->col_idx, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  std::unique_ptr<int32_t[]> order(new int32_t[std::max<int64_t>(n, 1)]);
  std::vector<uint8_t> seen(n, 0);
  int64_t tail = 0;
  for (int64_t root = 0; root < n; ++root) {
    if (seen[root]) continue;
    int64_t head = tail;
    order[tail++] = (int32_t)root;
    seen[root] = 1;
    while (head < tail) {
      if (head + kPfRow < tail) __builtin_prefetch(&rp[order[head + kPfRow]]);
      if (head + kPfCol < tail) __builtin_prefetch(&ci[rp[order[head + kPfCol]]]);
      const int32_t v = order[head++];
      for (int32_t j = rp[v], e = rp[v + 1]; j < e; ++j) {
        const int32_t u = ci[j];
        if (!seen[u]) {
          seen[u] = 1;
          order[tail++] = u;
        }
      }
    }
  }
  std::unique_ptr<int32_t[]> inv(new int32_t[std::max<int64_t>(n, 1)]);
  for (int64_t i = 0; i < n; ++i) inv[order[i]] = (int32_t)i;
  SLK_HIP(graph_alloc((void**)&g->perm, sizeof(int32_t) * n, s));
  SLK_HIP(graph_alloc((void**)&g->iperm, sizeof(int32_t) * n, s));
  SLK_HIP(hipMemcpyAsync(g->perm, order.get(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  SLK_HIP(hipMemcpyAsync(g->iperm, inv.get(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  int32_t *nrp = nullptr, *nci = nullptr;
  SLK_HIP(graph_alloc((void**)&nrp, sizeof(int32_t) * (n + 1), s));
  if (graph_alloc((void**)&nci, sizeof(int32_t) * (g->nnz + kColPad), s) != hipSuccess) {
    (void)hipGetLastError();
    graph_free(nrp, g->pooled, s);
    return fail(SLK_ERR_OUT_OF_MEMORY, "relabelled CSR");
  }
  SLK_HIP(hipMemsetAsync(nci + g->nnz, 0, sizeof(int32_t) * kColPad, s));
  slk_status st = relabel_csr(n, g->row_ptr, g->col_idx, g->perm, g->iperm, nrp, nci, s);
  if (st == SLK_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(SLK_ERR_DEVICE, "relabel");
  if (st != SLK_OK) {
    graph_free(nrp, g->pooled, s);
    graph_free(nci, g->pooled, s);
    return st;
  }
  graph_free(g->row_ptr, g->pooled, s);
  graph_free(g->col_idx, g->pooled, s);
  g->row_ptr = nrp;
  g->col_idx = nci;
  g->reordered = 1;
  return SLK_OK;
}

// CSR, degree statistics, sigma^2 and the optional permutation for a graph whose kNN lists are
// set.  The entry count, sigma^2's sum, the degree range and row_ptr come back in one readback.
slk_status finish_from_knn(slk_graph* g, int32_t reorder, hipStream_t s) {
  struct Stats {
    double d2sum;
    int32_t nnz, mn, mx, pad;
  };
  Scratch sc(s);
  Stats* st;
  SLK_TRY(sc.get(&st, 1));
  SLK_HIP(hipMemsetAsync(st, 0, sizeof(Stats), s));
  SLK_TRY(build_csr(g->n, g->k, g->knn_idx, &g->row_ptr, &g->col_idx, &st->nnz, s));
  if (g->knn_d2) SLK_TRY(sum_f64(g->knn_d2, g->n * g->k, &st->d2sum, s));
  SLK_TRY(launch_degree_minmax(g->row_ptr, g->n, &st->mn, s));
  std::vector<int32_t> rp(reorder ? 0 : g->n + 1);  // the reordered graph reads its own row_ptr
  Stats h{};
  if (!reorder)
    SLK_HIP(hipMemcpyAsync(rp.data(), g->row_ptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipMemcpyAsync(&h, st, sizeof(Stats), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  g->nnz = h.nnz;
  if (g->knn_d2) g->sigma2 = h.d2sum / ((double)g->n * (double)g->k);
  g->min_degree = h.mn;
  g->max_degree = h.mx;
  if (reorder) {
    SLK_TRY(bfs_reorder(g, s));
    SLK_TRY(build_heavy(g, s));
  } else {
    SLK_TRY(heavy_from(g, rp, s));
  }
  return SLK_OK;
}

// ------------------------------------------------------------------------------------------
// the z-update loop for fixed modes
// ------------------------------------------------------------------------------------------
struct Work {
  uint32_t* col_off = nullptr;  // float4 path: CSR columns as byte offsets of Z rows
  float* A = nullptr;
  float* Z[2] = {nullptr, nullptr};
  int32_t* labels_int = nullptr;
  double* partial = nullptr;
  double* partial2 = nullptr;
  float* cand_v = nullptr;
  int32_t* cand_i = nullptr;
  IterState* state = nullptr;
  IterState* state2 = nullptr;
  double* bound = nullptr;
  int32_t* modes = nullptr;
  int32_t* modes_next = nullptr;
  int32_t* moved = nullptr;     // L flags: modes_next[l] != modes[l]
  const float* mvec = nullptr;  // SLK-MS: L x d mode vectors used in place of the points at `modes`
  double* epart_un = nullptr;
  double* epart_un64 = nullptr;
  long long* epart_cut = nullptr;
  double* eout = nullptr;
  long long* eout_cut = nullptr;
  double* trace = nullptr;
  int grid = 0, egrid = 0;
};

// Column byte offsets for the float4 z-update (L <= 64), computed once per call.
slk_status prepare_col_off(const slk_graph* g, int32_t L, Scratch& sc, uint32_t** out) {
  *out = nullptr;
  if (L > 64) return SLK_OK;
  SLK_TRY(sc.get(out, g->nnz + kColPad));
  return launch_col_offsets(g->col_idx, g->nnz, g->n, L, *out, sc.stream);
}




slk_status alloc_work(Scratch& sc, const slk_graph* g, int32_t L, int trace_cap, Work& w) {
  const int64_t n = g->n;
  const int ldz = ldz_for(L);
  w.grid = iter_grid(n, L, heavy_rows_for(g, L), tune_wave_steps(n, L));
  w.egrid = energy_grid(n, g->n_heavy);
  SLK_TRY(sc.get(&w.A, n * ldz));
  SLK_TRY(sc.get(&w.Z[0], n * ldz));
  SLK_TRY(sc.get(&w.Z[1], n * ldz));
  SLK_TRY(sc.get(&w.labels_int, n));
  SLK_TRY(sc.get(&w.partial, w.grid));
  SLK_TRY(sc.get(&w.partial2, w.grid));
  SLK_TRY(sc.get(&w.cand_v, (int64_t)w.grid * L));
  SLK_TRY(sc.get(&w.cand_i, (int64_t)w.grid * L));
  SLK_TRY(sc.get(&w.state, 1));
  SLK_TRY(sc.get(&w.state2, 1));
  SLK_TRY(sc.get(&w.bound, 1));
  SLK_TRY(sc.get(&w.modes, L));
  SLK_TRY(sc.get(&w.modes_next, L));
  SLK_TRY(sc.get(&w.moved, L));
  SLK_TRY(sc.get(&w.epart_un, w.egrid));
  SLK_TRY(sc.get(&w.epart_un64, w.egrid));
  SLK_TRY(sc.get(&w.epart_cut, w.egrid));
  SLK_TRY(sc.get(&w.eout, 2));
  SLK_TRY(sc.get(&w.eout_cut, 1));
  SLK_TRY(sc.get(&w.trace, std::max(trace_cap, 1)));
  return SLK_OK;
}

struct OuterOut {
  int passes = 0;
  int converged = 0;
  double energy = 0, energy64 = 0, bound = 0;
  long long cut = 0;
  int32_t modes_next[256] = {};  // the byproduct modes (also in Work::modes_next on the device)
  int final_pass = 0;            // 1 if the separate final pass ran
};

IterArgs make_iter(const slk_graph* g, const Work& w, int64_t n, int32_t L, const slk_params& p) {
  IterArgs a{};
  a.row_ptr = g->row_ptr;
  a.col_idx = g->col_idx;
  a.col_off = w.col_off;
  a.A = w.A;
  a.n = n;
  a.L = L;
  a.ldz = ldz_for(L);
  a.lam_eff = (float)(p.pairwise_scale * p.lambda);
  a.half_lam_eff = (float)(0.5 * p.pairwise_scale * p.lambda);
  a.delta = (float)p.delta;
  a.partial = w.partial;
  a.state = w.state;
  a.trace = w.trace;
  a.bound_out = nullptr;
  a.mirror = nullptr;
  a.wsteps = tune_wave_steps(n, L);
  set_heavy(a, g, L);
  return a;
}

// One outer iteration with the modes in w.modes.  Device outputs: w.labels_int, w.modes_next,
// w.trace, and Z of the last z-update in w.Z[o->passes & 1] (internal order; the final pass
// recomputes that z-update for the labels and modes, with the same result, so the caller's Z and
// labels are scattered from there once, after the last outer iteration).  Host outputs in *o;
// with energy_always = false the energy, cut and their o-> fields are left stale when a mode
// moved (the caller then runs another outer iteration and never reports them).
slk_status run_outer(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const slk_params& p,
                     double sigma2, int trace_cap, int want_fp64, bool energy_always, hipStream_t s, Work& w,
                     OuterOut* o) {
  {
    KernelTimer kt("unary_kernel", s);
    SLK_TRY(launch_unary(x, n, d, g->perm, w.modes, L, ldz_for(L), sigma2, unary_mode(p.prec), w.A, w.Z[0], s,
                         nullptr, w.mvec));
  }
  const int check = p.fixed_inner > 0 ? 0 : 1;
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, s, w.state, p.bound_tol, check, trace_cap,
                     (check ? p.max_inner : p.fixed_inner) - 1);
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, s, w.state2, 0.0, 0, 0, -1);
  SLK_LAUNCHED("init_state_kernel");
  IterArgs a = make_iter(g, w, n, L, p);
  IterState hs{};
  int launched = 0;
  Watch* wt = nullptr;
  SLK_TRY(watch_for_device(&wt));
  // For 8 < L <= 64 the z-update that the device expects to end the loop (the last pass allowed,
  // or the relative change of the bound predicted below the tolerance from the two passes
  // before) also leaves the labels and byproduct-mode candidates of its input, which is what the
  // final pass computes from it, and records its index in the state; the bound of every pass
  // goes to the host-mapped results.  The final pass then runs only if the pass that ended the
  // loop was not that one.  (For L <= 8 the extra registers would cost the z-update a wave per
  // SIMD.)
  const bool emit = L > 8 && L <= 64 && p.final_pass == 0;
  FinalArgs fe{};
  if (emit) {
    a.bound_out = &wt->oh_dev->bound;
    fe.perm = g->perm;
    fe.labels_int = w.labels_int;
    fe.cand_v = w.cand_v;
    fe.cand_i = w.cand_i;
  }
  auto launch_pass = [&]() -> slk_status {
    if (!emit) return launch_iter(a, w.grid, s);
    fe.it = a;
    return launch_iter_emit(fe, w.grid, s);
  };
  if (!check) {
    for (; launched < p.fixed_inner; ++launched) {
      a.Zin = w.Z[launched & 1];
      a.Zout = w.Z[(launched + 1) & 1];
      SLK_TRY(launch_pass());
    }
    SLK_HIP(hipMemcpyAsync(&hs, w.state, sizeof(IterState), hipMemcpyDeviceToHost, s));
    SLK_HIP(hipStreamSynchronize(s));
    if (timing_on()) timing_flush();
  } else {
    // One pass ahead: pass k+1 is queued before the host looks at the state after pass k, so
    // the device never waits for the host; once the bound has settled, the one pass already
    // queued returns at once.
    auto enqueue = [&](int k) -> slk_status {
      a.Zin = w.Z[k & 1];
      a.Zout = w.Z[(k + 1) & 1];
      a.mirror = wt->dev + (k & 1);
      SLK_TRY(launch_pass());
      SLK_HIP(hipEventRecord(wt->ev[k & 1], s));
      return SLK_OK;
    };
    SLK_TRY(enqueue(0));
    launched = 1;
    int last = 0;
    for (int k = 0; k < launched; ++k) {
      if (launched < p.max_inner) {
        SLK_TRY(enqueue(launched));
        ++launched;
      }
      SLK_HIP(hipEventSynchronize(wt->ev[k & 1]));
      last = k;
      const volatile IterState* m = wt->host + (k & 1);
      if (m->done) break;
    }
    // The state after pass `last` is the final one: either it is done, and the passes queued
    // after it are no-ops that leave the state alone, or it is the last pass launched.
    memcpy(&hs, (const void*)(wt->host + (last & 1)), sizeof(IterState));
    if (timing_on()) timing_retag_tail("iter_kernel", launched - hs.pass, "iter_kernel_after_stop");
  }
  if (hs.numeric) return fail(SLK_ERR_NUMERIC, "relaxed bound is not finite");
  const int passes = hs.pass;
  if (passes < 1) return fail(SLK_ERR_INVALID_ARG, "at least one z-update is needed");
  o->passes = passes;
  o->converged = check ? hs.done : 1;
  o->final_pass = !emit || hs.emit_pass != passes - 1;
  if (o->final_pass) {
    // final pass on the input of the last z-update: its labels, modes candidates and bound
    FinalArgs f{};
    f.it = a;
    f.it.Zin = w.Z[(passes - 1) & 1];
    f.it.Zout = nullptr;
    f.it.state = w.state2;
    f.it.partial = w.partial2;
    f.it.trace = nullptr;
    f.it.bound_out = &wt->oh_dev->bound;
    f.it.mirror = nullptr;
    f.perm = g->perm;
    f.z_user = nullptr;
    f.labels_int = w.labels_int;
    f.labels_user = nullptr;
    f.cand_v = w.cand_v;
    f.cand_i = w.cand_i;
    SLK_TRY(launch_final(f, w.grid, s));
  }
  {
    KernelTimer kt("mode_reduce_kernel", s);
    SLK_TRY(launch_mode_reduce(w.cand_v, w.cand_i, w.grid, L, w.modes_next, s, wt->oh_dev->modes_next,
                               energy_always ? nullptr : w.modes, energy_always ? nullptr : w.moved));
  }
  EnergyArgs e{};
  set_heavy(e, g);
  e.row_ptr = g->row_ptr;
  e.col_idx = g->col_idx;
  e.labels_int = w.labels_int;
  e.A = w.A;
  e.x = want_fp64 ? x : nullptr;
  e.perm = g->perm;
  e.modes = w.modes;
  e.mvec = w.mvec;
  e.n = n;
  e.d = d;
  e.L = L;
  e.ldz = ldz_for(L);
  e.inv2s2 = 1.0 / (2.0 * sigma2);
  e.part_un = w.epart_un;
  e.part_un64 = w.epart_un64;
  e.part_cut = w.epart_cut;
  e.out = wt->oh_dev->eout;
  e.out_cut = &wt->oh_dev->cut;
  e.moved = energy_always ? nullptr : w.moved;
  SLK_TRY(launch_energy(e, w.egrid, s));
  SLK_HIP(hipStreamSynchronize(s));
  if (timing_on()) timing_flush();
  const volatile OuterHost* oh = wt->oh_host;
  const long long cut = oh->cut;
  o->cut = cut;
  o->energy = -oh->eout[0] + p.lambda * (double)cut;
  o->energy64 = want_fp64 ? -oh->eout[1] + p.lambda * (double)cut : o->energy;
  o->bound = oh->bound;
  for (int l = 0; l < L; ++l) o->modes_next[l] = oh->modes_next[l];
  return SLK_OK;
}



slk_status check_problem(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const int32_t* modes_host) {
  SLK_TRY(check_points(x, n, d));
  if (!g) return fail(SLK_ERR_INVALID_ARG, "graph is NULL");
  if (g->n != n) return fail(SLK_ERR_INVALID_ARG, "graph was built for a different n");
  if (L < 1 || L > 256 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(256, n)");
  if ((uint64_t)n * (uint64_t)ldz_for(L) * 4ull >= (1ull << 32))
    return fail(SLK_ERR_INVALID_ARG, "n * L (rounded up to a multiple of 4) must be < 2^30");
  if (!modes_host) return fail(SLK_ERR_INVALID_ARG, "modes is NULL");
  for (int l = 0; l < L; ++l)
    if (modes_host[l] < 0 || modes_host[l] >= n) return fail(SLK_ERR_INVALID_ARG, "mode index out of range");
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev != g->device)
    return fail(SLK_ERR_INVALID_ARG, "graph lives on another device");
  return SLK_OK;
}


}  // namespace

// Shared with the served form.
slk_status check_points(const float* x, int64_t n, int32_t d) {
  if (!x) return fail(SLK_ERR_INVALID_ARG, "x is NULL");
  if (n < 2 || n >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "n must satisfy 2 <= n < 2^31");
  if (d < 1) return fail(SLK_ERR_INVALID_ARG, "d must be >= 1");
  return SLK_OK;
}

slk_status check_params(const slk_params* p) {
  if (!p) return fail(SLK_ERR_INVALID_ARG, "params is NULL");
  if (!(p->lambda >= 0.0) || !isfinite(p->lambda)) return fail(SLK_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  if (!(p->delta >= 0.0) || !isfinite(p->delta)) return fail(SLK_ERR_INVALID_ARG, "delta must be finite and >= 0");
  if (!isfinite(p->sigma2)) return fail(SLK_ERR_INVALID_ARG, "sigma2 must be finite");
  if (!(p->bound_tol >= 0.0)) return fail(SLK_ERR_INVALID_ARG, "bound_tol must be >= 0");
  if (p->max_outer < 1) return fail(SLK_ERR_INVALID_ARG, "max_outer must be >= 1");
  if (p->max_inner < 1) return fail(SLK_ERR_INVALID_ARG, "max_inner must be >= 1");
  if (p->fixed_inner < 0) return fail(SLK_ERR_INVALID_ARG, "fixed_inner must be >= 0");
  if (p->pairwise_scale != 1 && p->pairwise_scale != 2) return fail(SLK_ERR_INVALID_ARG, "pairwise_scale must be 1 or 2");
  if (p->prec != SLK_PREC_FP32 && p->prec != SLK_PREC_BF16 && p->prec != SLK_PREC_BF16X) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  if (p->final_pass != 0 && p->final_pass != 1) return fail(SLK_ERR_INVALID_ARG, "final_pass must be 0 or 1");
  return SLK_OK;
}

double pick_sigma2(const slk_params& p, const slk_graph* g) { return p.sigma2 > 0.0 ? p.sigma2 : g->sigma2; }

int64_t heavy_rows_for(const slk_graph* g, int32_t L) { return L <= 64 ? g->n_heavy : 0; }

void set_heavy(IterArgs& a, const slk_graph* g, int32_t L) {
  const int64_t nh = heavy_rows_for(g, L);
  a.heavy = nh ? g->heavy : nullptr;
  a.n_heavy = (int32_t)nh;
  a.hblocks = heavy_blocks(nh);
  a.heavy_deg = nh ? kHeavyDeg : INT32_MAX;
}

void set_heavy(EnergyArgs& e, const slk_graph* g) {
  e.heavy = g->n_heavy ? g->heavy : nullptr;
  e.n_heavy = (int32_t)g->n_heavy;
  e.hblocks = heavy_blocks(g->n_heavy);
  e.heavy_deg = g->n_heavy ? kHeavyDeg : INT32_MAX;
}

void destroy_graph_on(slk_graph* g, hipStream_t s) { free_graph(g, s); }

slk_status check_knn_item(const float* x, int64_t n, int32_t d, const slk_knn_opts& o) {
  SLK_TRY(check_points(x, n, d));
  if (o.k < 1 || o.k > 64 || o.k >= n) return fail(SLK_ERR_INVALID_ARG, "k must satisfy 1 <= k <= 64 and k < n");
  if (o.prec != SLK_PREC_FP32 && o.prec != SLK_PREC_BF16 && o.prec != SLK_PREC_BF16X)
    return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  if (o.method < SLK_KNN_AUTO || o.method > SLK_KNN_MFMA) return fail(SLK_ERR_INVALID_ARG, "unknown kNN method");
  if (o.candidates < 0) return fail(SLK_ERR_INVALID_ARG, "candidates must be >= 0");
  if ((int64_t)n * 2 * o.k >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "n * 2k exceeds the CSR index range");
  return SLK_OK;
}

bool knn_takes_exact(int64_t n, int32_t d, const slk_knn_opts& o) {
  return o.method == SLK_KNN_EXACT || (o.method == SLK_KNN_AUTO && (double)n * (double)n * (double)d <= 4.0e9);
}


}  // namespace slk

using namespace slk;

// ============================================================================================
// exported functions
// ============================================================================================
extern "C" {

const char* slk_last_error(void) { return g_err.c_str(); }

const char* slk_version(void) { return "libslk 0.1 (gfx950)"; }

slk_status slk_pool_trim(void) {
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) arena_trim(dev);
  hipMemPool_t pool = nullptr;
  if (work_pool(&pool) != hipSuccess || hipMemPoolTrimTo(pool, 0) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SLK_ERR_DEVICE, "slk_pool_trim: the device's memory pool");
  }
  return SLK_OK;
}

slk_status slk_timing_enable(int32_t on) {
  timing_flush();
  std::lock_guard<std::mutex> lk(g_tmu);
  g_tacc.clear();
  g_timing = on != 0;
  return SLK_OK;
}

slk_status slk_timing_read(const char* kernel, int64_t* launches_host, double* total_ms_host) {
  if (!kernel || !launches_host || !total_ms_host) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  timing_flush();  // launches still pending are waited for and counted
  std::lock_guard<std::mutex> lk(g_tmu);
  auto it = g_tacc.find(kernel);
  *launches_host = it == g_tacc.end() ? 0 : it->second.first;
  *total_ms_host = it == g_tacc.end() ? 0.0 : it->second.second;
  return SLK_OK;
}

slk_status slk_knn_opts_default(slk_knn_opts* o) {
  if (!o) return fail(SLK_ERR_INVALID_ARG, "opts is NULL");
  o->k = 10;
  o->reorder = 0;
  o->candidates = 0;
  o->method = SLK_KNN_AUTO;
  o->prec = SLK_PREC_FP32;
  return SLK_OK;
}

slk_status slk_params_default(slk_params* p) {
  if (!p) return fail(SLK_ERR_INVALID_ARG, "params is NULL");
  memset(p, 0, sizeof(*p));
  p->lambda = 1.0;
  p->sigma2 = 0.0;
  p->delta = 0.0;
  p->bound_tol = 1e-8;
  p->max_outer = 20;
  p->max_inner = 1000;
  p->fixed_inner = 0;
  p->pairwise_scale = 1;
  p->prec = SLK_PREC_FP32;
  p->final_pass = 0;
  return SLK_OK;
}

slk_status slk_build_knn(const float* x, int64_t n, int32_t d, const slk_knn_opts* opts, void* stream,
                         slk_graph** g_out) {
  if (!g_out) return fail(SLK_ERR_INVALID_ARG, "g_out is NULL");
  *g_out = nullptr;
  SLK_TRY(check_points(x, n, d));
  slk_knn_opts o;
  if (opts) o = *opts;
  else slk_knn_opts_default(&o);
  if (o.k < 1 || o.k > 64 || o.k >= n) return fail(SLK_ERR_INVALID_ARG, "k must satisfy 1 <= k <= 64 and k < n");
  if (o.prec != SLK_PREC_FP32 && o.prec != SLK_PREC_BF16 && o.prec != SLK_PREC_BF16X) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  if (o.method < SLK_KNN_AUTO || o.method > SLK_KNN_MFMA) return fail(SLK_ERR_INVALID_ARG, "unknown kNN method");
  if (o.candidates < 0) return fail(SLK_ERR_INVALID_ARG, "candidates must be >= 0");
  if ((int64_t)n * 2 * o.k >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "n * 2k exceeds the CSR index range");
  hipStream_t s = (hipStream_t)stream;
  SLK_TRY(check_finite(x, n * (int64_t)d, s));
  GraphGuard gg{new slk_graph(), s};
  slk_graph* g = gg.g;
  g->pooled = graph_pool();
  SLK_HIP(hipGetDevice(&g->device));
  g->n = n;
  g->k = o.k;
  SLK_HIP(graph_alloc((void**)&g->knn_idx, sizeof(int32_t) * n * o.k, s));
  SLK_HIP(graph_alloc((void**)&g->knn_d2, sizeof(double) * n * o.k, s));
  const int bf16 = o.prec == SLK_PREC_BF16;
  int method = o.method;
  if (method == SLK_KNN_AUTO) method = knn_takes_exact(n, d, o) ? SLK_KNN_EXACT : SLK_KNN_MFMA;
  if (method == SLK_KNN_EXACT) {
    SLK_TRY(knn_exact(x, n, d, o.k, bf16, nullptr, n, g->knn_idx, g->knn_d2, s));
    g->rows_certified = 0;
    g->rows_fallback = n;
  } else {
    int cand = o.candidates > 0 ? o.candidates : std::max(2 * o.k, 32);
    cand = std::min(std::max(cand, o.k), 256);
    SLK_TRY(knn_mfma(x, n, d, o.k, cand, bf16, g->knn_idx, g->knn_d2, &g->rows_certified, &g->rows_fallback, s,
                     nullptr, 0, /*split_ok=*/!g->pooled));
  }
  SLK_TRY(finish_from_knn(g, o.reorder, s));
  *g_out = gg.release();
  return SLK_OK;
}

slk_status slk_build_knn_batched(const slk_knn_item* items, int32_t count, void* stream, slk_graph** graphs_out) {
  if (!items || !graphs_out || count < 0) return fail(SLK_ERR_INVALID_ARG, "NULL argument or negative count");
  for (int i = 0; i < count; ++i) graphs_out[i] = nullptr;
  for (int i = 0; i < count; ++i) {
    if (items[i].reserved != 0) return fail(SLK_ERR_INVALID_ARG, "reserved must be 0");
    SLK_TRY(check_knn_item(items[i].x, items[i].n, items[i].d, items[i].opts));
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<slk_graph*> made(count, nullptr);
  auto fail_all = [&](slk_status st) {
    for (slk_graph* g : made) free_graph(g, s);
    return st;
  };
  std::vector<KnnExactJob> ex;
  std::vector<int> ex_item;
  for (int i = 0; i < count; ++i) {
    const slk_knn_item& it = items[i];
    const slk_knn_opts& o = it.opts;
    if (!knn_takes_exact(it.n, it.d, o)) {
      const slk_status st = slk_build_knn(it.x, it.n, it.d, &o, stream, &made[i]);
      if (st != SLK_OK) return fail_all(st);
      continue;
    }
    slk_status st = check_finite(it.x, it.n * (int64_t)it.d, s);
    if (st != SLK_OK) return fail_all(st);
    slk_graph* g = new slk_graph();
    made[i] = g;
    g->pooled = graph_pool();
    if (hipGetDevice(&g->device) != hipSuccess) return fail_all(fail(SLK_ERR_DEVICE, "hipGetDevice"));
    g->n = it.n;
    g->k = o.k;
    if (graph_alloc((void**)&g->knn_idx, sizeof(int32_t) * it.n * o.k, s) != hipSuccess ||
        graph_alloc((void**)&g->knn_d2, sizeof(double) * it.n * o.k, s) != hipSuccess) {
      (void)hipGetLastError();
      return fail_all(fail(SLK_ERR_OUT_OF_MEMORY, "kNN lists"));
    }
    g->rows_certified = 0;
    g->rows_fallback = it.n;
    ex.push_back(KnnExactJob{it.x, it.n, it.d, o.k, o.prec == SLK_PREC_BF16 ? 1 : 0, g->knn_idx, g->knn_d2});
    ex_item.push_back(i);
  }
  slk_status st = knn_exact_group(ex.data(), (int)ex.size(), s);
  if (st != SLK_OK) return fail_all(st);
  for (size_t e = 0; e < ex_item.size(); ++e) {
    const int i = ex_item[e];
    st = finish_from_knn(made[i], items[i].opts.reorder, s);
    if (st != SLK_OK) return fail_all(st);
  }
  SLK_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) graphs_out[i] = made[i];
  return SLK_OK;
}

slk_status slk_graph_from_knn(int64_t n, int32_t k, const int32_t* knn_idx, const double* knn_d2, int32_t reorder,
                              void* stream, slk_graph** g_out) {
  if (!g_out) return fail(SLK_ERR_INVALID_ARG, "g_out is NULL");
  *g_out = nullptr;
  if (n < 2 || n >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "n must satisfy 2 <= n < 2^31");
  if (k < 1 || k > 64 || k >= n) return fail(SLK_ERR_INVALID_ARG, "k must satisfy 1 <= k <= 64 and k < n");
  if (!knn_idx) return fail(SLK_ERR_INVALID_ARG, "knn_idx is NULL");
  if ((int64_t)n * 2 * k >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "n * 2k exceeds the CSR index range");
  hipStream_t s = (hipStream_t)stream;
  SLK_TRY(check_indices(knn_idx, n * (int64_t)k, n, s, "kNN indices must lie in [0, n)"));
  GraphGuard gg{new slk_graph(), s};
  slk_graph* g = gg.g;
  g->pooled = graph_pool();
  SLK_HIP(hipGetDevice(&g->device));
  g->n = n;
  g->k = k;
  SLK_HIP(graph_alloc((void**)&g->knn_idx, sizeof(int32_t) * n * k, s));
  SLK_HIP(hipMemcpyAsync(g->knn_idx, knn_idx, sizeof(int32_t) * n * k, hipMemcpyDeviceToDevice, s));
  if (knn_d2) {
    SLK_HIP(graph_alloc((void**)&g->knn_d2, sizeof(double) * n * k, s));
    SLK_HIP(hipMemcpyAsync(g->knn_d2, knn_d2, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
  }
  SLK_TRY(finish_from_knn(g, reorder, s));
  *g_out = gg.release();
  return SLK_OK;
}

slk_status slk_graph_from_csr(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              double sigma2_hint, int32_t reorder, void* stream, slk_graph** g_out) {
  if (!g_out) return fail(SLK_ERR_INVALID_ARG, "g_out is NULL");
  *g_out = nullptr;
  if (n < 2 || n >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "n must satisfy 2 <= n < 2^31");
  if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "nnz must satisfy 0 <= nnz < 2^31");
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(SLK_ERR_INVALID_ARG, "CSR array is NULL");
  if (!isfinite(sigma2_hint)) return fail(SLK_ERR_INVALID_ARG, "sigma2_hint must be finite");
  hipStream_t s = (hipStream_t)stream;
  SLK_TRY(check_row_ptr(row_ptr, n, nnz, s));
  if (nnz > 0) SLK_TRY(check_indices(col_idx, nnz, n, s, "CSR columns must lie in [0, n)"));
  GraphGuard gg{new slk_graph(), s};
  slk_graph* g = gg.g;
  g->pooled = graph_pool();
  SLK_HIP(hipGetDevice(&g->device));
  g->n = n;
  g->k = 0;
  g->nnz = nnz;
  g->sigma2 = sigma2_hint > 0 ? sigma2_hint : 0.0;
  SLK_HIP(graph_alloc((void**)&g->row_ptr, sizeof(int32_t) * (n + 1), s));
  SLK_HIP(graph_alloc((void**)&g->col_idx, sizeof(int32_t) * (nnz + kColPad), s));
  SLK_HIP(hipMemsetAsync(g->col_idx + nnz, 0, sizeof(int32_t) * kColPad, s));
  SLK_HIP(hipMemcpyAsync(g->row_ptr, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  if (nnz) SLK_HIP(hipMemcpyAsync(g->col_idx, col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
  if (reorder) SLK_TRY(bfs_reorder(g, s));
  SLK_TRY(build_heavy(g, s));
  int32_t mn, mx;
  SLK_TRY(degree_stats(g->row_ptr, n, &mn, &mx, s));
  g->min_degree = mn;
  g->max_degree = mx;
  *g_out = gg.release();
  return SLK_OK;
}

slk_status slk_graph_info(const slk_graph* g, slk_graph_info_t* info) {
  if (!g || !info) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  info->n = g->n;
  info->k = g->k;
  info->reordered = g->reordered;
  info->nnz = g->nnz;
  info->max_degree = g->max_degree;
  info->min_degree = g->min_degree;
  info->sigma2 = g->sigma2;
  info->rows_certified = g->rows_certified;
  info->rows_fallback = g->rows_fallback;
  return SLK_OK;
}

slk_status slk_graph_export(const slk_graph* g, int32_t* row_ptr, int32_t* col_idx, int32_t* knn_idx, double* knn_d2,
                            int32_t* perm, void* stream) {
  if (!g) return fail(SLK_ERR_INVALID_ARG, "graph is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = g->n;
  if ((knn_idx || knn_d2) && !g->knn_idx) return fail(SLK_ERR_INVALID_ARG, "graph has no kNN lists");
  if (knn_d2 && !g->knn_d2) return fail(SLK_ERR_INVALID_ARG, "graph has no kNN distances");
  if (knn_idx) SLK_HIP(hipMemcpyAsync(knn_idx, g->knn_idx, sizeof(int32_t) * n * g->k, hipMemcpyDeviceToDevice, s));
  if (knn_d2) SLK_HIP(hipMemcpyAsync(knn_d2, g->knn_d2, sizeof(double) * n * g->k, hipMemcpyDeviceToDevice, s));
  if (perm) {
    if (g->perm) {
      SLK_HIP(hipMemcpyAsync(perm, g->perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    } else {
      std::vector<int32_t> id(n);
      for (int64_t i = 0; i < n; ++i) id[i] = (int32_t)i;
      SLK_HIP(hipMemcpyAsync(perm, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
      SLK_HIP(hipStreamSynchronize(s));
    }
  }
  if (row_ptr || col_idx) {
    if (!g->perm) {
      if (row_ptr) SLK_HIP(hipMemcpyAsync(row_ptr, g->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
      if (col_idx && g->nnz)
        SLK_HIP(hipMemcpyAsync(col_idx, g->col_idx, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice, s));
    } else {
      // back to the original numbering: new row p is internal row iperm[p]
      Scratch sc(s);
      int32_t *rp, *ci;
      SLK_TRY(sc.get(&rp, n + 1));
      SLK_TRY(sc.get(&ci, g->nnz));
      SLK_TRY(relabel_csr(n, g->row_ptr, g->col_idx, g->iperm, g->perm, rp, ci, s));
      if (row_ptr) SLK_HIP(hipMemcpyAsync(row_ptr, rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
      if (col_idx && g->nnz) SLK_HIP(hipMemcpyAsync(col_idx, ci, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice, s));
      SLK_HIP(hipStreamSynchronize(s));
    }
  }
  SLK_HIP(hipStreamSynchronize(s));
  return SLK_OK;
}

void slk_graph_destroy(slk_graph* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  const bool pl = g->pooled != 0;
  free_graph(g, nullptr);
  if (pl) (void)hipStreamSynchronize(nullptr);
}

slk_status slk_unary(const float* x, int64_t n, int32_t d, int32_t L, const int32_t* modes_host, double sigma2,
                     slk_precision prec, void* stream, float* a_out, float* z0_out) {
  SLK_TRY(check_points(x, n, d));
  if (L < 1 || L > 256 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(256, n)");
  if (!modes_host) return fail(SLK_ERR_INVALID_ARG, "modes is NULL");
  for (int l = 0; l < L; ++l)
    if (modes_host[l] < 0 || modes_host[l] >= n) return fail(SLK_ERR_INVALID_ARG, "mode index out of range");
  if (!(sigma2 > 0.0) || !isfinite(sigma2)) return fail(SLK_ERR_INVALID_ARG, "sigma2 must be > 0");
  if (prec != SLK_PREC_FP32 && prec != SLK_PREC_BF16 && prec != SLK_PREC_BF16X) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  int32_t* md;
  SLK_TRY(sc.get(&md, L));
  SLK_HIP(hipMemcpyAsync(md, modes_host, sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
  SLK_TRY(launch_unary(x, n, d, nullptr, md, L, L, sigma2, unary_mode(prec), a_out, z0_out, s));
  SLK_HIP(hipStreamSynchronize(s));
  return SLK_OK;
}

slk_status slk_inner_step(const slk_graph* g, int32_t L, const float* a, const float* z_in, double lambda,
                          double delta, int32_t pairwise_scale, void* stream, float* z_out, double* bound_host) {
  if (!g || !a || !z_in) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  if (L < 1 || L > 256 || L > g->n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(256, n)");
  if ((uint64_t)g->n * (uint64_t)ldz_for(L) * 4ull >= (1ull << 32))
    return fail(SLK_ERR_INVALID_ARG, "n * L (rounded up to a multiple of 4) must be < 2^30");
  if (!(lambda >= 0.0) || !isfinite(lambda) || !(delta >= 0.0) || !isfinite(delta))
    return fail(SLK_ERR_INVALID_ARG, "lambda and delta must be finite and >= 0");
  if (pairwise_scale != 1 && pairwise_scale != 2) return fail(SLK_ERR_INVALID_ARG, "pairwise_scale must be 1 or 2");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = g->n;
  Scratch sc(s);
  slk_params p;
  slk_params_default(&p);
  p.lambda = lambda;
  p.delta = delta;
  p.pairwise_scale = pairwise_scale;
  Work w;
  w.grid = iter_grid(n, L, heavy_rows_for(g, L), tune_wave_steps(n, L));
  SLK_TRY(sc.get(&w.partial, w.grid));
  SLK_TRY(sc.get(&w.state, 1));
  SLK_TRY(sc.get(&w.bound, 1));
  SLK_TRY(prepare_col_off(g, L, sc, &w.col_off));
  const int ldz = ldz_for(L);
  const bool relayout = g->perm || ldz != L;
  const float* A = a;
  const float* Zi = z_in;
  float* Zo = z_out;
  if (relayout) {
    float *ta, *tz, *to;
    SLK_TRY(sc.get(&ta, n * ldz));
    SLK_TRY(sc.get(&tz, n * ldz));
    SLK_TRY(sc.get(&to, n * ldz));
    SLK_TRY(launch_gather_rows(a, g->perm, n, L, ldz, ta, s));
    SLK_TRY(launch_gather_rows(z_in, g->perm, n, L, ldz, tz, s));
    A = ta;
    Zi = tz;
    Zo = z_out ? to : nullptr;
  }
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, s, w.state, 0.0, 0, 0, -1);
  SLK_LAUNCHED("init_state_kernel");
  IterArgs ia = make_iter(g, w, n, L, p);
  ia.A = A;
  ia.Zin = Zi;
  ia.Zout = Zo;
  ia.trace = nullptr;
  ia.bound_out = w.bound;
  SLK_TRY(launch_iter(ia, w.grid, s));
  if (relayout && z_out) SLK_TRY(launch_scatter_rows(Zo, g->perm, n, L, ldz, z_out, s));
  if (bound_host) {
    SLK_HIP(hipMemcpyAsync(bound_host, w.bound, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  SLK_HIP(hipStreamSynchronize(s));
  if (timing_on()) timing_flush();
  return SLK_OK;
}

static slk_status assign_or_fit(bool fit, const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L,
                                const int32_t* modes_host, const slk_params* pp, void* stream, float* z_out,
                                int32_t* labels_out, int32_t* modes_next_host, double* trace_host, int32_t trace_cap,
                                slk_result* res) {
  SLK_TRY(check_problem(x, n, d, g, L, modes_host));
  SLK_TRY(check_params(pp));
  if (!z_out) return fail(SLK_ERR_INVALID_ARG, "z_out is NULL");
  const slk_params p = *pp;
  const double sigma2 = pick_sigma2(p, g);
  if (!(sigma2 > 0.0)) return fail(SLK_ERR_INVALID_ARG, "sigma2 unknown: pass params.sigma2 > 0");
  if (trace_cap < 0) return fail(SLK_ERR_INVALID_ARG, "trace_cap must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const int cap = std::max(trace_cap, std::max(p.max_inner, p.fixed_inner));
  Scratch sc(s, true);  // the call synchronises before it returns
  Work w;
  SLK_TRY(alloc_work(sc, g, L, cap, w));
  SLK_TRY(prepare_col_off(g, L, sc, &w.col_off));
  std::vector<int32_t> cur(modes_host, modes_host + L), nxt(L);
  SLK_HIP(hipMemcpyAsync(w.modes, cur.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
  slk_result r{};
  OuterOut o;
  const int outer_cap = fit ? p.max_outer : 1;
  for (int t = 0; t < outer_cap; ++t) {
    SLK_TRY(run_outer(x, n, d, g, L, p, sigma2, cap, 1, !fit || t + 1 == outer_cap, s, w, &o));
    nxt.assign(o.modes_next, o.modes_next + L);
    r.outer_iters = t + 1;
    r.inner_iters_total += o.passes;
    r.inner_iters_last = o.passes;
    r.final_passes += o.final_pass;
    r.energy = o.energy;
    r.energy_fp64 = o.energy64;
    r.bound = o.bound;
    r.cut = o.cut;
    if (!fit) {
      r.converged = o.converged;
      break;
    }
    if (nxt == cur) {
      r.converged = 1;
      break;
    }
    // out of outer iterations: w.modes keeps the modes that produced the last labels
    if (t + 1 == outer_cap) break;
    cur = nxt;
    std::swap(w.modes, w.modes_next);  // the next outer iteration runs on the byproduct modes
  }
  SLK_TRY(launch_scatter_rows(w.Z[o.passes & 1], g->perm, n, L, ldz_for(L), z_out, s));
  if (labels_out) SLK_TRY(launch_labels_to_user(w.labels_int, g->perm, n, labels_out, s));
  // r.energy_fp64 is the FP64 recheck of the last outer iteration's energy: its energy pass also
  // recomputed the unary term from X in FP64 at the last labels and the modes that produced them
  // (the only energy pass of a fit that is not skipped, see run_outer)
  if (trace_host && trace_cap > 0) {
    const int m = std::min(trace_cap, std::min(o.passes, cap));
    SLK_HIP(hipMemcpyAsync(trace_host, w.trace, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  }
  SLK_HIP(hipStreamSynchronize(s));
  if (modes_next_host) memcpy(modes_next_host, nxt.data(), sizeof(int32_t) * L);
  std::vector<int32_t> u(nxt);
  std::sort(u.begin(), u.end());
  r.n_distinct_modes = (int32_t)(std::unique(u.begin(), u.end()) - u.begin());
  if (res) *res = r;
  return SLK_OK;
}

slk_status slk_assign(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const int32_t* modes_host,
                      const slk_params* p, void* stream, float* z_out, int32_t* labels_out, int32_t* modes_next_host,
                      double* bound_trace_host, int32_t trace_cap, slk_result* res_host) {
  return assign_or_fit(false, x, n, d, g, L, modes_host, p, stream, z_out, labels_out, modes_next_host,
                       bound_trace_host, trace_cap, res_host);
}

slk_status slk_fit(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const int32_t* init_modes_host,
                   const slk_params* p, void* stream, float* z_out, int32_t* labels_out, int32_t* modes_out_host,
                   slk_result* res_host) {
  if (!modes_out_host) return fail(SLK_ERR_INVALID_ARG, "modes_out_host is NULL");
  return assign_or_fit(true, x, n, d, g, L, init_modes_host, p, stream, z_out, labels_out, modes_out_host, nullptr, 0,
                       res_host);
}

slk_status slk_fit_ms(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const float* init_modes,
                      const slk_params* pp, double ms_tol, int32_t ms_max_iter, void* stream, float* z_out,
                      int32_t* labels_out, float* modes_out, float* modes_used_out, int32_t* ms_steps_host,
                      slk_result* res) {
  SLK_TRY(check_points(x, n, d));
  if (!g) return fail(SLK_ERR_INVALID_ARG, "graph is NULL");
  if (g->n != n) return fail(SLK_ERR_INVALID_ARG, "graph was built for a different n");
  if (L < 1 || L > 64 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(64, n)");
  if (!init_modes || !z_out || !modes_out) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  if (!(ms_tol >= 0.0) || ms_max_iter < 1) return fail(SLK_ERR_INVALID_ARG, "need ms_tol >= 0 and ms_max_iter >= 1");
  SLK_TRY(check_params(pp));
  const slk_params p = *pp;
  const double sigma2 = pick_sigma2(p, g);
  if (!(sigma2 > 0.0)) return fail(SLK_ERR_INVALID_ARG, "sigma2 unknown: pass params.sigma2 > 0");
  hipStream_t s = (hipStream_t)stream;
  const int cap = std::max(p.max_inner, p.fixed_inner);
  Scratch sc(s, true);  // the call synchronises before it returns
  Work w;
  SLK_TRY(alloc_work(sc, g, L, cap, w));
  SLK_TRY(prepare_col_off(g, L, sc, &w.col_off));
  // mode vectors: cur (used by the outer iteration) and nxt (after its mean-shift)
  float *cur, *nxt;
  SLK_TRY(sc.get(&cur, (size_t)L * d));
  SLK_TRY(sc.get(&nxt, (size_t)L * d));
  SLK_HIP(hipMemcpyAsync(cur, init_modes, sizeof(float) * L * d, hipMemcpyDeviceToDevice, s));
  slk_result r{};
  OuterOut o;
  const int umode = unary_mode(p.prec);
  const double lim = ms_tol * std::sqrt(sigma2);
  int32_t ms_steps = 0;
  SLK_HIP(hipMemsetAsync(w.modes, 0, sizeof(int32_t) * L, s));  // unused: the modes are the vectors
  for (int t = 0; t < p.max_outer; ++t) {
    w.mvec = cur;
    SLK_TRY(run_outer(x, n, d, g, L, p, sigma2, cap, 0, true, s, w, &o));
    r.outer_iters = t + 1;
    r.inner_iters_total += o.passes;
    r.inner_iters_last = o.passes;
    r.final_passes += o.final_pass;
    r.energy = o.energy;
    r.energy_fp64 = o.energy64;
    r.bound = o.bound;
    r.cut = o.cut;
    // Eq. (9) with the relaxed assignment of the last z-update (internal order)
    SLK_HIP(hipMemcpyAsync(nxt, cur, sizeof(float) * L * d, hipMemcpyDeviceToDevice, s));
    int32_t its = 0;
    SLK_TRY(mean_shift_loop(x, n, d, g->perm, w.Z[o.passes & 1], L, ldz_for(L), nxt, sigma2, ms_tol, ms_max_iter, umode,
                            s, &its, nullptr));
    ms_steps += its;
    // how far the modes moved over the whole update
    double move = 0.0;
    {
      std::vector<float> a((size_t)L * d), b((size_t)L * d);
      SLK_HIP(hipMemcpyAsync(a.data(), cur, sizeof(float) * L * d, hipMemcpyDeviceToHost, s));
      SLK_HIP(hipMemcpyAsync(b.data(), nxt, sizeof(float) * L * d, hipMemcpyDeviceToHost, s));
      SLK_HIP(hipStreamSynchronize(s));
      for (int l = 0; l < L; ++l) {
        double m2 = 0.0;
        for (int c = 0; c < d; ++c) {
          const double t2 = (double)b[(size_t)l * d + c] - (double)a[(size_t)l * d + c];
          m2 += t2 * t2;
        }
        move = std::max(move, std::sqrt(m2));
      }
    }
    if (move <= lim) {
      r.converged = 1;
      break;
    }
    if (t + 1 == p.max_outer) break;
    std::swap(cur, nxt);
  }
  SLK_TRY(launch_scatter_rows(w.Z[o.passes & 1], g->perm, n, L, ldz_for(L), z_out, s));
  if (labels_out) SLK_TRY(launch_labels_to_user(w.labels_int, g->perm, n, labels_out, s));
  // FP64 recheck of the final energy at the last labels and the modes that produced them
  {
    EnergyArgs e{};
    set_heavy(e, g);
    e.row_ptr = g->row_ptr;
    e.col_idx = g->col_idx;
    e.labels_int = w.labels_int;
    e.A = w.A;
    e.x = x;
    e.perm = g->perm;
    e.modes = w.modes;
    e.mvec = cur;
    e.n = n;
    e.d = d;
    e.L = L;
    e.ldz = ldz_for(L);
    e.inv2s2 = 1.0 / (2.0 * sigma2);
    e.part_un = w.epart_un;
    e.part_un64 = w.epart_un64;
    e.part_cut = w.epart_cut;
    e.out = w.eout;
    e.out_cut = w.eout_cut;
    SLK_TRY(launch_energy(e, w.egrid, s));
    double eo[2];
    SLK_HIP(hipMemcpyAsync(eo, w.eout, sizeof(eo), hipMemcpyDeviceToHost, s));
    SLK_HIP(hipStreamSynchronize(s));
    r.energy_fp64 = -eo[1] + p.lambda * (double)r.cut;
  }
  SLK_HIP(hipMemcpyAsync(modes_out, nxt, sizeof(float) * L * d, hipMemcpyDeviceToDevice, s));
  if (modes_used_out) SLK_HIP(hipMemcpyAsync(modes_used_out, cur, sizeof(float) * L * d, hipMemcpyDeviceToDevice, s));
  SLK_HIP(hipStreamSynchronize(s));
  r.n_distinct_modes = L;
  if (ms_steps_host) *ms_steps_host = ms_steps;
  if (res) *res = r;
  return SLK_OK;
}

slk_status slk_energy(const float* x, int64_t n, int32_t d, const slk_graph* g, int32_t L, const int32_t* labels,
                      const float* z, const int32_t* modes_host, double lambda, double sigma2, double delta,
                      void* stream, slk_energy_out* out) {
  SLK_TRY(check_problem(x, n, d, g, L, modes_host));
  if (!labels || !out) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  if (!(lambda >= 0.0) || !isfinite(lambda) || !(delta >= 0.0) || !isfinite(delta))
    return fail(SLK_ERR_INVALID_ARG, "lambda and delta must be finite and >= 0");
  const double s2 = sigma2 > 0 ? sigma2 : g->sigma2;
  if (!(s2 > 0.0)) return fail(SLK_ERR_INVALID_ARG, "sigma2 unknown: pass sigma2 > 0");
  hipStream_t s = (hipStream_t)stream;
  SLK_TRY(check_labels(labels, n, L, s));
  Scratch sc(s, true);  // the call synchronises before it returns
  Work w;
  SLK_TRY(alloc_work(sc, g, L, 1, w));
  if (z) SLK_TRY(prepare_col_off(g, L, sc, &w.col_off));
  SLK_HIP(hipMemcpyAsync(w.modes, modes_host, sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
  SLK_TRY(launch_unary(x, n, d, g->perm, w.modes, L, ldz_for(L), s2, 0, w.A, nullptr, s));
  SLK_TRY(launch_to_internal_labels(labels, g->iperm, n, w.labels_int, s));
  EnergyArgs e{};
  set_heavy(e, g);
  e.row_ptr = g->row_ptr;
  e.col_idx = g->col_idx;
  e.labels_int = w.labels_int;
  e.A = w.A;
  e.x = x;
  e.perm = g->perm;
  e.modes = w.modes;
  e.n = n;
  e.d = d;
  e.L = L;
  e.ldz = ldz_for(L);
  e.inv2s2 = 1.0 / (2.0 * s2);
  e.part_un = w.epart_un;
  e.part_un64 = w.epart_un64;
  e.part_cut = w.epart_cut;
  e.out = w.eout;
  e.out_cut = w.eout_cut;
  SLK_TRY(launch_energy(e, w.egrid, s));
  double bnd = 0.0;
  if (z) {
    slk_params p;
    slk_params_default(&p);
    p.lambda = lambda;
    p.delta = delta;
    const float* Zi = z;
    if (g->perm || ldz_for(L) != L) {
      SLK_TRY(launch_gather_rows(z, g->perm, n, L, ldz_for(L), w.Z[0], s));
      Zi = w.Z[0];
    }
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, s, w.state, 0.0, 0, 0, -1);
    SLK_LAUNCHED("init_state_kernel");
    IterArgs ia = make_iter(g, w, n, L, p);
    ia.Zin = Zi;
    ia.Zout = nullptr;
    ia.trace = nullptr;
    ia.bound_out = w.bound;
    SLK_TRY(launch_iter(ia, w.grid, s));
    SLK_HIP(hipMemcpyAsync(&bnd, w.bound, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  double eo[2];
  long long cut;
  SLK_HIP(hipMemcpyAsync(eo, w.eout, sizeof(eo), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipMemcpyAsync(&cut, w.eout_cut, sizeof(cut), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  out->energy = -eo[0] + lambda * (double)cut;
  out->energy_fp64 = -eo[1] + lambda * (double)cut;
  out->bound = bnd;
  out->cut = cut;
  return SLK_OK;
}

}  // extern "C"
