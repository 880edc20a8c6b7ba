// The served and batched form: many SLK-BO fits (Algorithm 1) advanced together on one GPU.
// This is an extension; the paper fits one problem at a time.
//
// Every resident job moves through a small state machine:
//   unary    a = k(x, m), Z^0 = softmax(a), loop state reset        (Eq. (6a), Algorithm 1)
//   inner    z-updates until the bound settles or the pass cap      (Eq. (8))
//   final    labels, byproduct modes, energy                        (Eq. (11), Eq. (1))
//            -> unary again with the new modes, or
//   recheck  FP64 energy at the last labels; outputs delivered
// A step launches, for each kernel, ONE packed launch over every job in the phase that needs it
// (launch_*_packed: each job keeps the work-groups, tiles and reduction order of its own
// launch), then copies every job's small device state (its Slot) back to the host in one copy
// and synchronises.  Queued jobs are admitted between steps when a slot is free and their
// estimated footprint fits the memory budget.  An admitted job's graph is built by a worker
// thread on its own stream while the resident jobs keep stepping (the builds overlap the
// iterations on the device); the job joins the steps once its graph is ready.
#include "common.h"

#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace slk {
namespace {

constexpr int kMaxL = 64;

// Per-job device state, copied back to the host after every step.
struct Slot {
  IterState st;               // inner loop
  IterState st2;              // final pass (bound only)
  double bound;               // relaxed bound of the last z-update's input
  double eout[2];             // unary sums: FP32 path, FP64 recheck
  long long cut;
  int32_t modes[2][kMaxL];    // current and next modes, alternating
};

// Loop-state reset (and, on admission, the initial modes) for one job.
struct InitJob {
  IterState* st;
  IterState* st2;
  double tol;
  int32_t check;
  int32_t L;                  // > 0: copy `modes` to `dst`
  int32_t* dst;
  int32_t modes[kMaxL];
};

__global__ void init_jobs_kernel(const InitJob* __restrict__ jobs, int count) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const InitJob& j = jobs[i];
  if (threadIdx.x == 0) {
    j.st->pass = 0;
    j.st->done = 0;
    j.st->numeric = 0;
    j.st->tol = j.tol;
    j.st->check = j.check;
    j.st->trace_cap = 0;
    j.st->last_bound = 0.0;
    j.st->rel = 0.0;
    j.st->rel_prev = 0.0;
    j.st->last_pass = -1;
    j.st->emit_pass = -1;
    j.st2->pass = 0;
    j.st2->done = 0;
    j.st2->numeric = 0;
    j.st2->tol = 0.0;
    j.st2->check = 0;
    j.st2->trace_cap = 0;
    j.st2->last_bound = 0.0;
    j.st2->rel = 0.0;
    j.st2->rel_prev = 0.0;
    j.st2->last_pass = -1;
    j.st2->emit_pass = -1;
  }
  for (int l = threadIdx.x; l < j.L; l += blockDim.x) j.dst[l] = j.modes[l];
}

enum class Phase { kUnary, kInner, kFinal, kRecheck };

struct Job {
  int64_t ticket = 0;
  slk_job spec{};
  std::vector<int32_t> cur_modes, next_modes;  // host copies
  slk_graph* g = nullptr;
  double sigma2 = 0.0;
  int L = 0, ldz = 0, G = 0, grid = 0, egrid = 0, ugrid = 0, wsteps = 0;
  size_t footprint = 0;
  void* mem = nullptr;
  float* A = nullptr;
  float* Z[2] = {nullptr, nullptr};
  uint32_t* col_off = nullptr;
  int32_t* labels_int = nullptr;
  double* partial = nullptr;
  double* partial2 = nullptr;
  float* cand_v = nullptr;
  int32_t* cand_i = nullptr;
  double* epart_un = nullptr;
  double* epart_un64 = nullptr;
  long long* epart_cut = nullptr;
  int slot = -1;
  int cur = 0;           // row of Slot::modes holding the current modes
  bool fresh = true;     // modes not yet on the device
  Phase phase = Phase::kUnary;
  int launched = 0;      // z-updates queued in this outer iteration
  int passes = 0;        // z-updates that ran in the last finished inner loop
  int limit = 0;         // fixed_inner, else max_inner
  slk_status build_status = SLK_OK;
  slk_result r{};
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device bytes a job may need while resident: graph, kNN transients, work buffers.
size_t job_footprint(const slk_job& j) {
  const size_t n = (size_t)j.n, d = (size_t)j.d, k = (size_t)std::max(j.knn.k, 1), L = (size_t)j.L;
  const size_t ldz = (size_t)ldz_for(j.L);
  const size_t nnz = 2 * k * n + kColPad;
  const size_t graph = 4 * (n + 1) + 4 * nnz + 12 * n * k + 12 * n;
  const size_t knn = 4 * n * d + 8 * n * 64 + 16 * n;
  const size_t grid = (size_t)iter_grid(j.n, j.L, j.n, 1) + 8;   // the largest grid any tile shape takes
  const size_t work = 12 * n * ldz + 4 * nnz + 4 * n + 16 * grid + 8 * L * grid + 24 * grid;
  return graph + knn + work + (1u << 20);
}

}  // namespace
}  // namespace slk

using namespace slk;

struct slk_server {
  slk_server_opts o{};
  hipStream_t s = nullptr;
  int device = 0;
  int64_t next_ticket = 0;
  size_t budget = 0, used = 0;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::vector<int> free_slots;
  Slot* slots_dev = nullptr;
  Slot* slots_host = nullptr;   // pinned
  std::vector<int64_t> finished;
  char* tab_dev = nullptr;
  char* tab_host = nullptr;     // pinned
  size_t tab_cap = 0;
  // graph builds: worker threads, each with its own stream (default priority)
  std::vector<std::thread> builders;
  std::vector<hipStream_t> bss;
  std::mutex mu;
  std::condition_variable cv_todo, cv_built;
  std::deque<Job*> to_build;    // admitted, graph not built yet
  std::deque<Job*> built;       // graph built (or failed: build_status)
  int building = 0;             // handed to the builder and not taken back yet
  bool stop = false;
  std::atomic<int64_t> grouped_builds{0};   // shared launches of the exact kNN search
  // captured step shapes: signature -> executable graph; shapes seen once wait for a second time
  struct Captured {
    std::vector<int64_t> sig;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  std::vector<Captured> graphs;
  std::vector<std::vector<int64_t>> seen;   // shapes seen once (bounded, oldest dropped)
  uint64_t clock = 0;
  int64_t steps = 0, graph_launches = 0, graph_captures = 0;
};

namespace slk {
namespace {

// Host staging of the per-step argument tables; one copy to the device per step.
struct Tables {
  size_t off = 0;
  template <class T>
  size_t reserve(size_t count) {
    off = align_up(off, 256);
    const size_t at = off;
    off += sizeof(T) * std::max<size_t>(count, 1);
    return at;
  }
};

void deliver(slk_server* sv, Job* j, slk_status st) {
  if (st == SLK_OK) {
    if (j->spec.modes_out_host) memcpy(j->spec.modes_out_host, j->next_modes.data(), sizeof(int32_t) * j->L);
    std::vector<int32_t> u(j->next_modes);
    std::sort(u.begin(), u.end());
    j->r.n_distinct_modes = (int32_t)(std::unique(u.begin(), u.end()) - u.begin());
    if (j->spec.result_host) *j->spec.result_host = j->r;
  }
  if (j->spec.status_host) *j->spec.status_host = st;
  sv->finished.push_back(j->ticket);
}

void release(slk_server* sv, Job* j) {
  if (j->mem) (void)hipFreeAsync(j->mem, sv->s);
  if (j->g) destroy_graph_on(j->g, sv->s);
  if (j->slot >= 0) sv->free_slots.push_back(j->slot);
  sv->used -= std::min(sv->used, j->footprint);
  delete j;
}

// A worker: builds the graphs of admitted jobs on its own stream and hands each job back
// complete (its stream synchronised) with the build's status.  A job whose graph takes the exact
// search is built together with the other such jobs waiting at that moment (up to kGroupMax):
// their searches share one launch (slk_build_knn_batched); graphs identical to single builds.
constexpr size_t kGroupMax = 32;
constexpr size_t kGraphsMax = 64;   // captured step shapes kept (least recently used dropped)
constexpr size_t kSeenMax = 256;    // shapes seen once, remembered

bool exact_build(const Job* j) { return knn_takes_exact(j->spec.n, j->spec.d, j->spec.knn); }

void builder_loop(slk_server* sv, int w) {
  (void)hipSetDevice(sv->device);
  set_graph_pool(true);   // graphs freed stream-ordered when their jobs finish
  const hipStream_t bs = sv->bss[w];
  for (;;) {
    std::vector<Job*> group;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_todo.wait(lk, [&] { return sv->stop || !sv->to_build.empty(); });
      if (sv->stop) return;
      group.push_back(sv->to_build.front());
      sv->to_build.pop_front();
      if (exact_build(group[0])) {
        for (auto it = sv->to_build.begin(); it != sv->to_build.end() && group.size() < kGroupMax;) {
          if (exact_build(*it)) {
            group.push_back(*it);
            it = sv->to_build.erase(it);
          } else {
            ++it;
          }
        }
      }
    }
    auto build_one = [&](Job* j) {
      const slk_job& sp = j->spec;
      slk_status st = slk_build_knn(sp.x, sp.n, sp.d, &sp.knn, bs, &j->g);
      if (st == SLK_OK && hipStreamSynchronize(bs) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(SLK_ERR_DEVICE, "graph build");
      }
      j->build_status = st;
    };
    if (group.size() == 1) {
      build_one(group[0]);
    } else {
      std::vector<slk_knn_item> items(group.size());
      std::vector<slk_graph*> gs(group.size(), nullptr);
      for (size_t i = 0; i < group.size(); ++i) {
        const slk_job& sp = group[i]->spec;
        items[i] = slk_knn_item{sp.x, sp.n, sp.d, 0, sp.knn};
      }
      if (slk_build_knn_batched(items.data(), (int32_t)items.size(), bs, gs.data()) == SLK_OK) {
        for (size_t i = 0; i < group.size(); ++i) {
          group[i]->g = gs[i];
          group[i]->build_status = SLK_OK;
        }
        ++sv->grouped_builds;
      } else {
        // one of them failed: build each alone, so that every job gets its own status
        for (Job* j : group) build_one(j);
      }
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (Job* j : group) sv->built.push_back(j);
    }
    sv->cv_built.notify_all();
  }
}

// Buffers and slot state of a job whose graph is built.  On failure the job is delivered with
// the error and released; the server carries on.
slk_status admit(slk_server* sv, Job* j) {
  hipStream_t s = sv->s;
  const slk_job& sp = j->spec;
  if (j->build_status != SLK_OK) return j->build_status;
  j->sigma2 = pick_sigma2(sp.params, j->g);
  if (!(j->sigma2 > 0.0)) return fail(SLK_ERR_INVALID_ARG, "sigma2 unknown: pass params.sigma2 > 0");
  const int64_t n = sp.n;
  j->ldz = ldz_for(j->L);
  j->G = groups4(j->L);
  j->wsteps = tune_wave_steps(n, j->L);
  j->grid = iter_grid(n, j->L, heavy_rows_for(j->g, j->L), j->wsteps);
  j->egrid = energy_grid(n, j->g->n_heavy);
  const size_t nz = (size_t)j->g->nnz + kColPad;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t at = off;
    off += std::max<size_t>(bytes, 1);
    return at;
  };
  const size_t oA = carve(4 * n * j->ldz), oZ0 = carve(4 * n * j->ldz), oZ1 = carve(4 * n * j->ldz);
  const size_t oC = carve(4 * nz), oLab = carve(4 * n), oP = carve(8 * (size_t)j->grid),
               oP2 = carve(8 * (size_t)j->grid), oCV = carve(4 * (size_t)j->L * j->grid),
               oCI = carve(4 * (size_t)j->L * j->grid), oE1 = carve(8 * (size_t)j->egrid),
               oE2 = carve(8 * (size_t)j->egrid), oE3 = carve(8 * (size_t)j->egrid);
  if (hipMallocAsync(&j->mem, off, s) != hipSuccess) {
    (void)hipGetLastError();
    j->mem = nullptr;
    return fail(SLK_ERR_OUT_OF_MEMORY, "job work buffers");
  }
  char* b = (char*)j->mem;
  j->A = (float*)(b + oA);
  j->Z[0] = (float*)(b + oZ0);
  j->Z[1] = (float*)(b + oZ1);
  j->col_off = (uint32_t*)(b + oC);
  j->labels_int = (int32_t*)(b + oLab);
  j->partial = (double*)(b + oP);
  j->partial2 = (double*)(b + oP2);
  j->cand_v = (float*)(b + oCV);
  j->cand_i = (int32_t*)(b + oCI);
  j->epart_un = (double*)(b + oE1);
  j->epart_un64 = (double*)(b + oE2);
  j->epart_cut = (long long*)(b + oE3);
  SLK_TRY(launch_col_offsets(j->g->col_idx, j->g->nnz, n, j->L, j->col_off, s));
  j->phase = Phase::kUnary;
  j->fresh = true;
  j->limit = sp.params.fixed_inner > 0 ? sp.params.fixed_inner : sp.params.max_inner;
  return SLK_OK;
}

IterArgs job_iter(const Job* j, const Slot* slot_dev) {
  const slk_params& p = j->spec.params;
  IterArgs a{};
  a.row_ptr = j->g->row_ptr;
  a.col_idx = j->g->col_idx;
  a.col_off = j->col_off;
  a.A = j->A;
  a.n = j->spec.n;
  a.L = j->L;
  a.ldz = j->ldz;
  a.lam_eff = (float)(p.pairwise_scale * p.lambda);
  a.half_lam_eff = (float)(0.5 * p.pairwise_scale * p.lambda);
  a.delta = (float)p.delta;
  a.partial = j->partial;
  a.state = const_cast<IterState*>(&slot_dev->st);
  a.trace = nullptr;
  a.bound_out = nullptr;
  a.mirror = nullptr;
  a.wsteps = j->wsteps;
  set_heavy(a, j->g, j->L);
  return a;
}

EnergyArgs job_energy(const Job* j, Slot* slot_dev, bool fp64) {
  EnergyArgs e{};
  set_heavy(e, j->g);
  e.row_ptr = j->g->row_ptr;
  e.col_idx = j->g->col_idx;
  e.labels_int = j->labels_int;
  e.A = j->A;
  e.x = fp64 ? j->spec.x : nullptr;
  e.perm = j->g->perm;
  e.modes = slot_dev->modes[j->cur];
  e.n = j->spec.n;
  e.d = j->spec.d;
  e.L = j->L;
  e.ldz = j->ldz;
  e.inv2s2 = 1.0 / (2.0 * j->sigma2);
  e.part_un = j->epart_un;
  e.part_un64 = j->epart_un64;
  e.part_cut = j->epart_cut;
  e.out = slot_dev->eout;
  e.out_cut = &slot_dev->cut;
  return e;
}

void drop_graphs(slk_server* sv) {
  for (auto& c : sv->graphs) (void)hipGraphExecDestroy(c.exec);
  sv->graphs.clear();
  sv->seen.clear();
}

slk_status grow_tables(slk_server* sv, size_t need) {
  if (need <= sv->tab_cap) return SLK_OK;
  drop_graphs(sv);   // captured launches hold addresses in the old table block
  size_t cap = std::max<size_t>(need, 2 * sv->tab_cap);
  cap = align_up(cap, 1 << 16);
  (void)hipFree(sv->tab_dev);
  (void)hipHostFree(sv->tab_host);
  sv->tab_dev = nullptr;
  sv->tab_host = nullptr;
  sv->tab_cap = 0;
  SLK_HIP(hipMalloc(&sv->tab_dev, cap));
  SLK_HIP(hipHostMalloc(&sv->tab_host, cap, hipHostMallocDefault));
  sv->tab_cap = cap;
  return SLK_OK;
}

slk_status server_step(slk_server* sv) {
  hipStream_t s = sv->s;
  // ---- admission: a free slot and room in the budget send a queued job to the builder
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    while (!sv->queue.empty() && !sv->free_slots.empty()) {
      Job* j = sv->queue.front();
      if (sv->used + j->footprint > sv->budget && (!sv->active.empty() || sv->building > 0)) break;
      sv->queue.pop_front();
      sv->used += j->footprint;
      j->slot = sv->free_slots.back();
      sv->free_slots.pop_back();
      sv->to_build.push_back(j);
      ++sv->building;
    }
  }
  sv->cv_todo.notify_all();
  // ---- jobs whose graphs are ready join; with nothing resident, wait for the next one
  std::deque<Job*> ready;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->active.empty() && sv->built.empty() && sv->building > 0)
      sv->cv_built.wait(lk, [&] { return !sv->built.empty(); });
    ready.swap(sv->built);
    sv->building -= (int)ready.size();
  }
  for (Job* j : ready) {
    const slk_status st = admit(sv, j);
    if (st != SLK_OK) {
      deliver(sv, j, st);
      release(sv, j);
      if (st == SLK_ERR_DEVICE) return st;
      continue;
    }
    sv->active.push_back(j);
  }
  if (sv->active.empty()) return SLK_OK;

  // ---- who does what in this step
  std::vector<Job*> fin, rec, una, inn;
  for (Job* j : sv->active) {
    if (j->phase == Phase::kFinal) fin.push_back(j);
    else if (j->phase == Phase::kRecheck) rec.push_back(j);
    else if (j->phase == Phase::kUnary) una.push_back(j);
  }
  for (Job* j : una) {
    j->phase = Phase::kInner;
    j->launched = 0;
  }
  for (Job* j : sv->active)
    if (j->phase == Phase::kInner) inn.push_back(j);
  const int P = sv->o.passes_per_step;
  std::vector<int> npass(inn.size());
  int maxp = 0;
  for (size_t i = 0; i < inn.size(); ++i) {
    npass[i] = std::max(0, std::min(P, inn[i]->limit - inn[i]->launched));
    maxp = std::max(maxp, npass[i]);
  }

  // ---- argument tables
  const int Gs[5] = {1, 2, 4, 8, 16};
  Tables t;
  struct GroupAt {
    size_t args = 0, start = 0;
    int count = 0, blocks = 0;
  };
  // final: per G class
  GroupAt fin_g[5];
  for (int gi = 0; gi < 5; ++gi) {
    int c = 0;
    for (Job* j : fin) c += j->G == Gs[gi];
    fin_g[gi].count = c;
    if (c) {
      fin_g[gi].args = t.reserve<FinalArgs>(c);
      fin_g[gi].start = t.reserve<int32_t>(c + 1);
    }
  }
  const size_t fin_red = t.reserve<ReduceJob>(fin.size());
  const size_t mode_args = t.reserve<ModeJob>(fin.size()), mode_start = t.reserve<int32_t>(fin.size() + 1);
  const size_t nen = fin.size() + rec.size();
  const size_t en_args = t.reserve<EnergyArgs>(nen), en_start = t.reserve<int32_t>(nen + 1);
  const size_t un_args = t.reserve<UnaryArgs>(una.size()), un_start = t.reserve<int32_t>(una.size() + 1);
  const size_t init_args = t.reserve<InitJob>(una.size());
  std::vector<GroupAt> it_g((size_t)maxp * 5);
  std::vector<size_t> it_red(maxp);
  std::vector<int> it_nred(maxp);
  for (int p = 0; p < maxp; ++p) {
    int nr = 0;
    for (int gi = 0; gi < 5; ++gi) {
      int c = 0;
      for (size_t i = 0; i < inn.size(); ++i) c += (p < npass[i] && inn[i]->G == Gs[gi]);
      GroupAt& ga = it_g[(size_t)p * 5 + gi];
      ga.count = c;
      nr += c;
      if (c) {
        ga.args = t.reserve<IterArgs>(c);
        ga.start = t.reserve<int32_t>(c + 1);
      }
    }
    it_nred[p] = nr;
    it_red[p] = t.reserve<ReduceJob>(nr);
  }
  SLK_TRY(grow_tables(sv, t.off));
  char* H = sv->tab_host;
  char* D = sv->tab_dev;
  Slot* SD = sv->slots_dev;

  for (int gi = 0; gi < 5; ++gi) {
    GroupAt& ga = fin_g[gi];
    if (!ga.count) continue;
    FinalArgs* fa = (FinalArgs*)(H + ga.args);
    int32_t* st = (int32_t*)(H + ga.start);
    int k = 0, b = 0;
    for (Job* j : fin) {
      if (j->G != Gs[gi]) continue;
      FinalArgs f{};
      f.it = job_iter(j, SD + j->slot);
      f.it.Zin = j->Z[(j->passes - 1) & 1];
      f.it.Zout = nullptr;
      f.it.state = &SD[j->slot].st2;
      f.it.partial = j->partial2;
      f.it.bound_out = &SD[j->slot].bound;
      f.perm = j->g->perm;
      f.z_user = j->spec.z_out;
      f.labels_int = j->labels_int;
      f.labels_user = j->spec.labels_out;
      f.cand_v = j->cand_v;
      f.cand_i = j->cand_i;
      f.grid = j->grid;
      fa[k] = f;
      st[k++] = b;
      b += j->grid;
    }
    st[k] = b;
    ga.blocks = b;
  }
  {
    ReduceJob* rj = (ReduceJob*)(H + fin_red);
    ModeJob* mj = (ModeJob*)(H + mode_args);
    int32_t* ms = (int32_t*)(H + mode_start);
    int b = 0;
    for (size_t i = 0; i < fin.size(); ++i) {
      Job* j = fin[i];
      rj[i] = ReduceJob{j->partial2, j->grid, &SD[j->slot].st2, nullptr, &SD[j->slot].bound};
      mj[i] = ModeJob{j->cand_v, j->cand_i, j->grid, SD[j->slot].modes[j->cur ^ 1]};
      ms[i] = b;
      b += j->L;
    }
    ms[fin.size()] = b;
  }
  int en_blocks = 0, mode_blocks = 0;
  for (Job* j : fin) mode_blocks += j->L;
  {
    EnergyArgs* ea = (EnergyArgs*)(H + en_args);
    int32_t* es = (int32_t*)(H + en_start);
    size_t k = 0;
    for (Job* j : fin) {
      ea[k] = job_energy(j, SD + j->slot, false);
      es[k++] = en_blocks;
      en_blocks += j->egrid;
    }
    for (Job* j : rec) {
      ea[k] = job_energy(j, SD + j->slot, true);
      es[k++] = en_blocks;
      en_blocks += j->egrid;
    }
    es[k] = en_blocks;
  }
  int un_blocks = 0;
  size_t un_lds = 0;
  {
    UnaryArgs* ua = (UnaryArgs*)(H + un_args);
    int32_t* us = (int32_t*)(H + un_start);
    InitJob* ij = (InitJob*)(H + init_args);
    for (size_t i = 0; i < una.size(); ++i) {
      Job* j = una[i];
      const slk_params& p = j->spec.params;
      ua[i] = unary_args(j->spec.x, j->spec.n, j->spec.d, j->g->perm, SD[j->slot].modes[j->cur], j->L, j->ldz, j->sigma2,
                         unary_mode(p.prec), j->A, j->Z[0]);
      us[i] = un_blocks;
      un_blocks += unary_grid(ua[i]);
      un_lds = std::max(un_lds, unary_lds(ua[i]));
      InitJob in{};
      in.st = &SD[j->slot].st;
      in.st2 = &SD[j->slot].st2;
      in.tol = p.bound_tol;
      in.check = p.fixed_inner > 0 ? 0 : 1;
      in.L = j->fresh ? j->L : 0;
      in.dst = SD[j->slot].modes[j->cur];
      if (j->fresh) memcpy(in.modes, j->cur_modes.data(), sizeof(int32_t) * j->L);
      ij[i] = in;
      j->fresh = false;
    }
    us[una.size()] = un_blocks;
  }
  for (int p = 0; p < maxp; ++p) {
    ReduceJob* rj = (ReduceJob*)(H + it_red[p]);
    int nr = 0;
    for (int gi = 0; gi < 5; ++gi) {
      GroupAt& ga = it_g[(size_t)p * 5 + gi];
      if (!ga.count) continue;
      IterArgs* ia = (IterArgs*)(H + ga.args);
      int32_t* st = (int32_t*)(H + ga.start);
      int k = 0, b = 0;
      for (size_t i = 0; i < inn.size(); ++i) {
        Job* j = inn[i];
        if (p >= npass[i] || j->G != Gs[gi]) continue;
        const int pass = j->launched + p;
        IterArgs a = job_iter(j, SD + j->slot);
        a.Zin = j->Z[pass & 1];
        a.Zout = j->Z[(pass + 1) & 1];
        ia[k] = a;
        st[k++] = b;
        b += j->grid;
        rj[nr++] = ReduceJob{j->partial, j->grid, &SD[j->slot].st, nullptr, nullptr};
      }
      st[k] = b;
      ga.blocks = b;
    }
  }

  // ---- launches (stream order: final, energies, unary + reset, z-updates), between the copy of
  // the argument tables and the copy of the slots.  The kernels' arguments are addresses in the
  // table block, counts and grid sizes: two steps with equal signatures launch identical
  // sequences, so a captured graph of one replays the other.
  std::vector<int64_t> sig;
  auto note = [&](int64_t kind, int64_t a, int64_t b, int64_t c, int64_t d) {
    sig.push_back(kind);
    sig.push_back(a);
    sig.push_back(b);
    sig.push_back(c);
    sig.push_back(d);
  };
  for (int gi = 0; gi < 5; ++gi)
    if (fin_g[gi].count) note(1, gi, (int64_t)fin_g[gi].args, fin_g[gi].count, fin_g[gi].blocks);
  if (!fin.empty()) note(2, (int64_t)fin_red, (int64_t)mode_args, (int64_t)fin.size(), mode_blocks);
  if (nen) note(3, (int64_t)en_args, (int64_t)en_start, (int64_t)nen, en_blocks);
  if (!una.empty()) note(4, (int64_t)init_args, (int64_t)una.size(), un_blocks, (int64_t)un_lds);
  for (int p = 0; p < maxp; ++p) {
    for (int gi = 0; gi < 5; ++gi) {
      const GroupAt& ga = it_g[(size_t)p * 5 + gi];
      if (ga.count) note(5, gi, (int64_t)ga.args, ga.count, ga.blocks);
    }
    note(6, p, (int64_t)it_red[p], it_nred[p], 0);
  }
  auto issue = [&]() -> slk_status {
    for (int gi = 0; gi < 5; ++gi) {
      const GroupAt& ga = fin_g[gi];
      if (ga.count)
        SLK_TRY(launch_final_packed(Gs[gi], (const FinalArgs*)(D + ga.args), (const int32_t*)(D + ga.start), ga.count,
                                    ga.blocks, s));
    }
    if (!fin.empty()) {
      SLK_TRY(launch_reduce_packed((const ReduceJob*)(D + fin_red), (int)fin.size(), s));
      SLK_TRY(launch_mode_reduce_packed((const ModeJob*)(D + mode_args), (const int32_t*)(D + mode_start),
                                        (int)fin.size(), mode_blocks, s));
    }
    if (nen) SLK_TRY(launch_energy_packed((const EnergyArgs*)(D + en_args), (const int32_t*)(D + en_start), (int)nen,
                                          en_blocks, s));
    if (!una.empty()) {
      hipLaunchKernelGGL(init_jobs_kernel, dim3((unsigned)una.size()), dim3(64), 0, s, (const InitJob*)(D + init_args),
                         (int)una.size());
      SLK_LAUNCHED("init_jobs_kernel");
      SLK_TRY(launch_unary_packed((const UnaryArgs*)(D + un_args), (const int32_t*)(D + un_start), (int)una.size(),
                                  un_blocks, un_lds, s));
    }
    for (int p = 0; p < maxp; ++p) {
      for (int gi = 0; gi < 5; ++gi) {
        const GroupAt& ga = it_g[(size_t)p * 5 + gi];
        if (ga.count)
          SLK_TRY(launch_iter_packed(Gs[gi], (const IterArgs*)(D + ga.args), (const int32_t*)(D + ga.start),
                                     ga.count, ga.blocks, s));
      }
      SLK_TRY(launch_reduce_packed((const ReduceJob*)(D + it_red[p]), it_nred[p], s));
    }
    return SLK_OK;
  };
  SLK_HIP(hipMemcpyAsync(D, H, t.off, hipMemcpyHostToDevice, s));
  ++sv->steps;
  bool ran = false;
  // the null stream cannot be captured: a server created on it launches every step directly
  if (sv->o.graph_replay && s != nullptr) {
    ++sv->clock;
    for (auto& c : sv->graphs) {
      if (c.sig == sig) {
        SLK_HIP(hipGraphLaunch(c.exec, s));
        c.used = sv->clock;
        ++sv->graph_launches;
        ran = true;
        break;
      }
    }
    if (!ran) {
      auto it = std::find(sv->seen.begin(), sv->seen.end(), sig);
      if (it == sv->seen.end()) {
        if (sv->seen.size() >= kSeenMax) sv->seen.erase(sv->seen.begin());
        sv->seen.push_back(sig);
      } else {
        sv->seen.erase(it);
        // second occurrence of this shape: capture it
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
        slk_status ist = SLK_OK;
        if (ok) {
          ist = issue();
          ok = hipStreamEndCapture(s, &graph) == hipSuccess && ist == SLK_OK;
        }
        if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (ok) {
          if (sv->graphs.size() >= kGraphsMax) {
            auto lru = std::min_element(sv->graphs.begin(), sv->graphs.end(),
                                        [](const auto& a, const auto& b) { return a.used < b.used; });
            (void)hipGraphExecDestroy(lru->exec);
            sv->graphs.erase(lru);
          }
          sv->graphs.push_back({sig, exec, sv->clock});
          ++sv->graph_captures;
          SLK_HIP(hipGraphLaunch(exec, s));
          ++sv->graph_launches;
          ran = true;
        } else if (exec) {
          (void)hipGraphExecDestroy(exec);
        }
      }
    }
  }
  if (!ran) SLK_TRY(issue());
  SLK_HIP(hipMemcpyAsync(sv->slots_host, sv->slots_dev, sizeof(Slot) * sv->o.max_jobs, hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));

  // ---- advance every job on what its slot says
  std::vector<Job*> keep;
  for (Job* j : sv->active) {
    const Slot& sl = sv->slots_host[j->slot];
    const slk_params& p = j->spec.params;
    bool done = false;
    slk_status st = SLK_OK;
    if (j->phase == Phase::kRecheck) {
      j->r.energy_fp64 = -sl.eout[1] + p.lambda * (double)j->r.cut;
      done = true;
    } else if (j->phase == Phase::kFinal) {
      j->r.outer_iters += 1;
      j->r.final_passes += 1;  // the served form always runs the final pass
      j->r.inner_iters_total += j->passes;
      j->r.inner_iters_last = j->passes;
      j->r.cut = sl.cut;
      j->r.energy = -sl.eout[0] + p.lambda * (double)sl.cut;
      j->r.energy_fp64 = j->r.energy;
      j->r.bound = sl.bound;
      j->next_modes.assign(sl.modes[j->cur ^ 1], sl.modes[j->cur ^ 1] + j->L);
      if (j->next_modes == j->cur_modes) {
        j->r.converged = 1;
        j->phase = Phase::kRecheck;
      } else if (j->r.outer_iters >= p.max_outer) {
        j->phase = Phase::kRecheck;
      } else {
        j->cur ^= 1;
        j->cur_modes = j->next_modes;
        j->phase = Phase::kUnary;
      }
    } else if (j->phase == Phase::kInner) {
      for (size_t i = 0; i < inn.size(); ++i)
        if (inn[i] == j) j->launched += npass[i];
      if (sl.st.numeric) {
        st = fail(SLK_ERR_NUMERIC, "relaxed bound is not finite");
        done = true;
      } else if ((p.fixed_inner == 0 && sl.st.done) || j->launched >= j->limit) {
        j->passes = sl.st.pass;
        if (j->passes < 1) {
          st = fail(SLK_ERR_INVALID_ARG, "at least one z-update is needed");
          done = true;
        } else {
          j->phase = Phase::kFinal;
        }
      }
    }
    if (done) {
      deliver(sv, j, st);
      release(sv, j);
    } else {
      keep.push_back(j);
    }
  }
  sv->active.swap(keep);
  return SLK_OK;
}

slk_status check_job(const slk_job* j) {
  if (!j) return fail(SLK_ERR_INVALID_ARG, "job is NULL");
  SLK_TRY(check_points(j->x, j->n, j->d));
  if (j->L < 1 || j->L > j->n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= n");
  if (j->L > kMaxL) return fail(SLK_ERR_UNSUPPORTED, "the served form takes L <= 64; use slk_fit");
  if ((uint64_t)j->n * (uint64_t)ldz_for(j->L) * 4ull >= (1ull << 32))
    return fail(SLK_ERR_INVALID_ARG, "n * L (rounded up to a multiple of 4) must be < 2^30");
  if (!j->init_modes_host) return fail(SLK_ERR_INVALID_ARG, "init_modes_host is NULL");
  std::vector<int32_t> m(j->init_modes_host, j->init_modes_host + j->L);
  for (int32_t v : m)
    if (v < 0 || v >= j->n) return fail(SLK_ERR_INVALID_ARG, "mode index out of range");
  std::sort(m.begin(), m.end());
  if (std::adjacent_find(m.begin(), m.end()) != m.end()) return fail(SLK_ERR_INVALID_ARG, "modes must be distinct");
  SLK_TRY(check_params(&j->params));
  if (j->knn.k < 1 || j->knn.k > 64 || j->knn.k >= j->n) return fail(SLK_ERR_INVALID_ARG, "k must satisfy 1 <= k <= 64, k < n");
  if (!j->z_out) return fail(SLK_ERR_INVALID_ARG, "z_out is NULL");
  return SLK_OK;
}

}  // namespace
}  // namespace slk

extern "C" {

slk_status slk_server_opts_default(slk_server_opts* o) {
  if (!o) return fail(SLK_ERR_INVALID_ARG, "opts is NULL");
  o->max_jobs = 64;
  o->passes_per_step = 4;
  o->memory_budget = 0;
  o->builders = 3;
  o->graph_replay = 1;
  return SLK_OK;
}

slk_status slk_server_create(const slk_server_opts* opts, void* stream, slk_server** out) {
  if (!out) return fail(SLK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  slk_server_opts o;
  slk_server_opts_default(&o);
  if (opts) o = *opts;
  if (o.max_jobs < 1 || o.max_jobs > 1024) return fail(SLK_ERR_INVALID_ARG, "max_jobs must be in [1, 1024]");
  if (o.passes_per_step < 1) return fail(SLK_ERR_INVALID_ARG, "passes_per_step must be >= 1");
  if (o.memory_budget < 0) return fail(SLK_ERR_INVALID_ARG, "memory_budget must be >= 0");
  if (o.builders < 1 || o.builders > 8) return fail(SLK_ERR_INVALID_ARG, "builders must be in [1, 8]");
  if (o.graph_replay != 0 && o.graph_replay != 1) return fail(SLK_ERR_INVALID_ARG, "graph_replay must be 0 or 1");
  slk_server* sv = new slk_server();
  sv->o = o;
  sv->s = (hipStream_t)stream;
  auto bail = [&](slk_status st) {
    slk_server_destroy(sv);
    return st;
  };
  if (hipGetDevice(&sv->device) != hipSuccess) return bail(fail(SLK_ERR_DEVICE, "hipGetDevice"));
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return bail(fail(SLK_ERR_DEVICE, "hipMemGetInfo"));
  sv->budget = o.memory_budget > 0 ? (size_t)o.memory_budget : (size_t)(0.8 * (double)fr);
  if (hipMalloc(&sv->slots_dev, sizeof(Slot) * o.max_jobs) != hipSuccess)
    return bail(fail(SLK_ERR_OUT_OF_MEMORY, "server slots"));
  if (hipHostMalloc(&sv->slots_host, sizeof(Slot) * o.max_jobs, hipHostMallocDefault) != hipSuccess)
    return bail(fail(SLK_ERR_OUT_OF_MEMORY, "server slot mirror"));
  for (int i = o.max_jobs - 1; i >= 0; --i) sv->free_slots.push_back(i);
  for (int w = 0; w < o.builders; ++w) {
    hipStream_t bs = nullptr;
    if (hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(SLK_ERR_DEVICE, "builder stream"));
    sv->bss.push_back(bs);
  }
  for (int w = 0; w < o.builders; ++w) sv->builders.emplace_back(builder_loop, sv, w);
  *out = sv;
  return SLK_OK;
}

slk_status slk_server_submit(slk_server* sv, const slk_job* job, int64_t* ticket_host) {
  if (!sv) return fail(SLK_ERR_INVALID_ARG, "server is NULL");
  SLK_TRY(check_job(job));
  Job* j = new Job();
  j->ticket = sv->next_ticket++;
  j->spec = *job;
  j->L = job->L;
  j->cur_modes.assign(job->init_modes_host, job->init_modes_host + job->L);
  j->next_modes = j->cur_modes;
  j->footprint = job_footprint(*job);
  sv->queue.push_back(j);
  if (ticket_host) *ticket_host = j->ticket;
  return SLK_OK;
}

slk_status slk_server_step(slk_server* sv, int64_t* done_host, int32_t cap, int32_t* n_done_host,
                           int32_t* n_active_host, int32_t* n_queued_host) {
  if (!sv) return fail(SLK_ERR_INVALID_ARG, "server is NULL");
  if (cap < 0) return fail(SLK_ERR_INVALID_ARG, "cap must be >= 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != sv->device)
    return fail(SLK_ERR_INVALID_ARG, "the server lives on another device");
  SLK_TRY(server_step(sv));
  const int32_t nd = done_host ? (int32_t)std::min<size_t>(sv->finished.size(), (size_t)cap) : 0;
  for (int32_t i = 0; i < nd; ++i) done_host[i] = sv->finished[i];
  sv->finished.erase(sv->finished.begin(), sv->finished.begin() + nd);
  if (n_done_host) *n_done_host = nd;
  if (n_active_host) *n_active_host = (int32_t)sv->active.size();
  if (n_queued_host) {
    std::lock_guard<std::mutex> lk(sv->mu);
    *n_queued_host = (int32_t)(sv->queue.size() + sv->building);
  }
  return SLK_OK;
}

void slk_server_destroy(slk_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_todo.notify_all();
  for (auto& t : sv->builders)
    if (t.joinable()) t.join();
  for (Job* j : sv->to_build) delete j;
  for (Job* j : sv->built) {
    if (j->g) destroy_graph_on(j->g, sv->s);
    delete j;
  }
  for (hipStream_t bs : sv->bss) (void)hipStreamDestroy(bs);
  for (Job* j : sv->active) {
    if (j->mem) (void)hipFreeAsync(j->mem, sv->s);
    if (j->g) destroy_graph_on(j->g, sv->s);
    delete j;
  }
  for (Job* j : sv->queue) delete j;
  (void)hipStreamSynchronize(sv->s);
  drop_graphs(sv);
  (void)hipFree(sv->slots_dev);
  (void)hipHostFree(sv->slots_host);
  (void)hipFree(sv->tab_dev);
  (void)hipHostFree(sv->tab_host);
  delete sv;
}

slk_status slk_server_stats(const slk_server* sv, slk_server_stats_t* out) {
  if (!sv || !out) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  out->steps = sv->steps;
  out->graph_launches = sv->graph_launches;
  out->graph_captures = sv->graph_captures;
  out->grouped_builds = sv->grouped_builds.load();
  return SLK_OK;
}

slk_status slk_fit_batched(const slk_job* jobs, int32_t n_jobs, const slk_server_opts* opts, void* stream) {
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(SLK_ERR_INVALID_ARG, "jobs is NULL");
  for (int32_t i = 0; i < n_jobs; ++i) SLK_TRY(check_job(jobs + i));
  slk_server* sv = nullptr;
  SLK_TRY(slk_server_create(opts, stream, &sv));
  slk_status st = SLK_OK;
  for (int32_t i = 0; i < n_jobs && st == SLK_OK; ++i) st = slk_server_submit(sv, jobs + i, nullptr);
  int32_t active = 1, queued = 1;
  while (st == SLK_OK && (active > 0 || queued > 0))
    st = slk_server_step(sv, nullptr, 0, nullptr, &active, &queued);
  slk_server_destroy(sv);
  return st;
}

}  // extern "C"
