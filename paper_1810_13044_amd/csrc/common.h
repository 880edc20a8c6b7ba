// Internal declarations shared by the libslk translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/slk.h"

namespace slk {

// Rounds a float to the nearest bfloat16 (ties to even) and returns it widened back to float.
// bfloat16 keeps the top 16 bits of the IEEE single format; NaN stays NaN.
__host__ __device__ __forceinline__ float bf16_round(float v) {
  uint32_t b;
  __builtin_memcpy(&b, &v, 4);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return v;
  b += 0x7fffu + ((b >> 16) & 1u);
  b &= 0xffff0000u;
  float r;
  __builtin_memcpy(&r, &b, 4);
  return r;
}

// Buffer loads for kernels that stream rows: a load at or past the end of the resource returns
// zeros without a memory access, so loads near the end of an array need no per-lane branch (a
// branch around a load makes the compiler wait for every load in flight where the paths join).
typedef unsigned int slk_vu4 __attribute__((ext_vector_type(4)));

// Resource over the first `rows` (clamped to [0, cap]) rows of `row_bytes` bytes at p.  Both are
// the same in every lane; the first lane's values are taken so that the descriptor sits in scalar
// registers (a descriptor the compiler cannot prove uniform is applied lane group by lane group in
// a loop).  Plain comparisons: the min/max templates lower 64-bit integers through FP64.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* p, int64_t rows, int cap, int row_bytes) {
  const int r = rows <= 0 ? 0 : (rows >= cap ? cap : (int)rows);
  const int nb = __builtin_amdgcn_readfirstlane(r * row_bytes);
  const uint64_t a = (uint64_t)(uintptr_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  void* base = (void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nb, 0x00020000);
}

// voff: the lane's byte offset; soff: a byte offset common to the wave (kept in a scalar register)
__device__ __forceinline__ uint4 bload16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const slk_vu4 v = __builtin_bit_cast(slk_vu4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float bloadf(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ int bloadi(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------
void set_error(const std::string& msg);
slk_status fail(slk_status s, const std::string& msg);

#define SLK_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      (void)hipGetLastError();                                                               \
      return ::slk::fail(e_ == hipErrorOutOfMemory ? SLK_ERR_OUT_OF_MEMORY : SLK_ERR_DEVICE,   \
                         std::string(#call) + ": " + hipGetErrorString(e_));                 \
    }                                                                                        \
  } while (0)

#define SLK_LAUNCHED(name)                                                                   \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess)                                                                    \
      return ::slk::fail(SLK_ERR_DEVICE, std::string("launch ") + (name) + ": " +            \
                                             hipGetErrorString(e_));                         \
  } while (0)

#define SLK_TRY(expr)                     \
  do {                                    \
    slk_status s_ = (expr);               \
    if (s_ != SLK_OK) return s_;          \
  } while (0)

// ------------------------------------------------------------------------------------
// stream-ordered device buffers owned by one call
// ------------------------------------------------------------------------------------
bool scratch_sync_alloc();
// Stream-ordered allocation from the library's pool on the current device (freed blocks are
// kept for reuse by later calls up to a fixed size; hipFreeAsync returns a block to it).
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s);
hipError_t work_pool(hipMemPool_t* out);
// Work memory that outlives the calls: a block per concurrent user, taken at the start of a
// call and handed back at its end, grown (and consolidated into one allocation) when a call
// needs more.  Allocating and freeing a fit's buffers on the stream costs milliseconds of host
// time per call; carving them from a kept block costs nothing.
struct Arena;
Arena* arena_acquire();
hipError_t arena_carve(Arena* a, size_t bytes, void** out);
void arena_release(Arena* a);

// Temporary device buffers of one call.  Default: stream-ordered allocations from the pool,
// freed stream-ordered when the Scratch goes out of scope.  Cached (for calls that
// synchronise their stream before returning): carved from an arena; the destructor
// synchronises the stream (so that nothing in flight still uses the memory, error paths
// included) before the arena goes back.
struct Scratch {
  hipStream_t stream;
  void* ptrs[32];
  int n = 0;
  Arena* arena = nullptr;
  explicit Scratch(hipStream_t s, bool cached = false) : stream(s), arena(cached ? arena_acquire() : nullptr) {}
  bool sync_alloc = scratch_sync_alloc();
  ~Scratch() {
    if (arena) {
      (void)hipStreamSynchronize(stream);
      arena_release(arena);
      return;
    }
    for (int i = 0; i < n; ++i) {
      if (sync_alloc) (void)hipFree(ptrs[i]);
      else (void)hipFreeAsync(ptrs[i], stream);
    }
  }
  template <class T>
  slk_status get(T** out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    if (n >= 32) return fail(SLK_ERR_INVALID_ARG, "internal: too many scratch buffers");
    void* p = nullptr;
    hipError_t e = arena ? arena_carve(arena, count * sizeof(T), &p)
                   : sync_alloc ? hipMalloc(&p, count * sizeof(T)) : pool_alloc(&p, count * sizeof(T), stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SLK_ERR_OUT_OF_MEMORY, std::string("device allocation: ") + hipGetErrorString(e));
    }
    ptrs[n++] = p;
    *out = static_cast<T*>(p);
    return SLK_OK;
  }
};

// pinned host staging buffer, one per thread, grown on demand
slk_status pinned(void** out, size_t bytes);

// Opt-in per-kernel timing with HIP events recorded on the launch stream (slk_timing_enable).
// KernelTimer brackets one launch; timing_flush() accumulates the finished pairs and must be
// called only after the stream has been synchronised.
bool timing_on();
int timer_start(const char* name, hipStream_t s);
void timer_stop(int slot, hipStream_t s);
void timing_flush();
// Moves the last `count` pending pairs named `name` to the bucket `to` (z-updates queued after
// the loop settled, which return at once).
void timing_retag_tail(const char* name, int count, const char* to);
struct KernelTimer {
  int slot;
  hipStream_t s;
  KernelTimer(const char* name, hipStream_t st) : slot(timing_on() ? timer_start(name, st) : -1), s(st) {}
  ~KernelTimer() {
    if (slot >= 0) timer_stop(slot, s);
  }
};

}  // namespace slk

// ------------------------------------------------------------------------------------
// the graph handle
// ------------------------------------------------------------------------------------
struct slk_graph {
  int64_t n = 0;
  int32_t k = 0;
  int64_t nnz = 0;
  int32_t max_degree = 0, min_degree = 0;
  double sigma2 = 0.0;
  int32_t reordered = 0;
  int64_t rows_certified = 0, rows_fallback = 0;
  int device = 0;
  // device arrays (hipMalloc, owned)
  int32_t* row_ptr = nullptr;   // n+1, internal order
  int32_t* col_idx = nullptr;   // nnz, internal indices, sorted per row
  int32_t* knn_idx = nullptr;   // n*k, original order and indices (may be null)
  double* knn_d2 = nullptr;     // n*k (may be null)
  int32_t* perm = nullptr;      // n: internal row -> original index (null = identity)
  int32_t* iperm = nullptr;     // n: original index -> internal row (null = identity)
  int32_t* heavy = nullptr;     // internal rows of degree > kHeavyDeg, by degree descending
  int64_t n_heavy = 0;
  int32_t pooled = 0;           // arrays from the stream-ordered pool (graphs built for the served form)
};

namespace slk {

// ------------------------------------------------------------------------------------
// kernels and launchers (defined in iter.hip / graph.hip)
// ------------------------------------------------------------------------------------

// Device-side state of one z-update loop.
struct IterState {
  int32_t pass;        // index of the next z-update
  int32_t done;        // 1 once the bound settled (later passes are no-ops)
  int32_t numeric;     // 1 if the bound became non-finite
  double tol;
  int32_t check;       // 1: test convergence; 0: fixed pass count
  int32_t trace_cap;
  double last_bound;
  double rel;          // relative change of the bound in the last pass (0 before two passes)
  double rel_prev;     // the same, one pass earlier
  int32_t last_pass;   // index of the last pass allowed (-1: no z-update writes labels)
  int32_t emit_pass;   // the pass that wrote labels and mode candidates (-1: none yet)
};

// Internal row stride of A and Z: L rounded up to a multiple of 4 (float4 rows) when L <= 64.
inline int ldz_for(int L) { return L <= 64 ? ((L + 3) / 4) * 4 : L; }
// Zero entries kept after the last CSR column so clamped index loads never leave the array.
constexpr int kColPad = 16;
// Rows of more than kHeavyDeg neighbours (the hubs of a kNN graph) are updated by a whole
// workgroup each, at the front of the grid; the row-per-group path skips them.
constexpr int kHeavyDeg = 128;
// Work-groups given to heavy rows: one per row, rounded up to a multiple of the 8 XCDs so the
// tiles behind them keep their XCD placement.
inline int heavy_blocks(int64_t n_heavy) { return (int)(8 * ((n_heavy + 7) / 8)); }

struct IterArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const uint32_t* col_off;  // float4 path (L <= 64): col_idx * row bytes, + kColPad dead entries
  const float* A;        // n x L (internal order)
  const float* Zin;      // n x L
  float* Zout;           // n x L (may be null: bound only)
  int64_t n;
  int32_t L;
  int32_t ldz;           // row stride of A, Zin, Zout (floats)
  float lam_eff;         // pairwise_scale * lambda
  float half_lam_eff;    // pairwise_scale * lambda / 2
  float delta;
  double* partial;       // one double per block
  IterState* state;      // may be null: no convergence bookkeeping
  double* trace;         // bound per pass (device, trace_cap entries) or null
  double* bound_out;     // if non-null, the last block writes the pass's bound here
  IterState* mirror;     // if non-null, host-visible copy of *state stored after the pass
  const int32_t* heavy;  // rows handled by the first hblocks work-groups (float4 path only)
  int32_t n_heavy;
  int32_t hblocks;       // heavy_blocks(n_heavy), or 0
  int32_t heavy_deg;     // rows above this degree belong to the heavy work-groups
  const int32_t* zperm;  // scalar path only: rows of A, Zin, Zout are in the caller's order, row
                         // zperm[r] holding internal row r (null = the internal order itself)
  int32_t wsteps;        // float4 path: row batches per wave in a tile (tune_wave_steps; 0 = 4)
};

struct FinalArgs {
  IterArgs it;
  const int32_t* perm;   // internal -> original (null = identity)
  float* z_user;         // n x L output in original order (null = none)
  int32_t* labels_int;   // n labels, internal order
  int32_t* labels_user;  // n labels, original order (null = none)
  float* cand_v;         // grid x L best log-odds per block
  int32_t* cand_i;       // grid x L original index of that candidate
  int32_t grid;          // work-groups of this pass (the candidate arrays' row length)
};

// How the unary term forms its distances: FP32 direct differences of the points as given, of the
// points rounded to bf16 (SLK_PREC_BF16), or the bf16 split contraction on MFMA (SLK_PREC_BF16X).
constexpr int32_t kUnaryFp32 = 0, kUnaryRounded = 1, kUnaryMfma = 2;
inline int32_t unary_mode(int32_t prec) {
  return prec == SLK_PREC_BF16 ? kUnaryRounded : prec == SLK_PREC_BF16X ? kUnaryMfma : kUnaryFp32;
}

struct UnaryArgs {
  const float* x;        // n x d, original order
  int64_t n;
  int32_t d, L, ldz, R;  // R rows per work-group
  const int32_t* perm;   // internal -> original (null = identity)
  const int32_t* modes;  // L original indices (device)
  float inv2s2;
  int32_t bf16;          // kUnaryFp32, kUnaryRounded or kUnaryMfma
  float* A;              // n x ldz, internal order (may be null)
  float* Z0;             // n x ldz (may be null)
  const float* xm;       // points the mode indices refer to (null = x)
  const float* mvec;     // L x d mode vectors (SLK-MS; null = the points at `modes`)
};

// One job of a packed pass reduction (one work-group per job).
struct ReduceJob {
  const double* partial;
  int32_t nparts;
  IterState* state;
  double* trace;
  double* bound_out;
};

// One job of a packed mode reduction (one work-group per cluster).
struct ModeJob {
  const float* cand_v;
  const int32_t* cand_i;
  int32_t grid;
  int32_t* modes;
};

// xm: the points the mode indices refer to (null = x; the out-of-sample queries use the fit's x)
slk_status launch_unary(const float* x, int64_t n, int32_t d, const int32_t* perm, const int32_t* modes_dev,
                        int32_t L, int32_t ldz, double sigma2, int32_t umode, float* A, float* Z0, hipStream_t s,
                        const float* xm = nullptr, const float* mvec = nullptr);
UnaryArgs unary_args(const float* x, int64_t n, int32_t d, const int32_t* perm, const int32_t* modes_dev, int32_t L,
                     int32_t ldz, double sigma2, int32_t bf16, float* A, float* Z0);
int unary_grid(const UnaryArgs& u);
size_t unary_lds(const UnaryArgs& u);
int groups4(int L);

// Index of the job owning block b: start[j] <= b < start[j + 1] (start has njobs + 1 entries).
__device__ __forceinline__ inline int job_of(const int32_t* __restrict__ start, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Packed launches: one launch covers several jobs; `start` (device, njobs + 1 entries) holds the
// first work-group of each job and the total, `jobs` (device) the per-job arguments.  Every job
// gets exactly the work-groups, tiles and reduction order of its own unpacked launch, so its
// results are bit-identical to running it alone.
slk_status launch_unary_packed(const UnaryArgs* jobs, const int32_t* start, int njobs, int blocks, size_t lds,
                               hipStream_t s);
slk_status launch_iter_packed(int G, const IterArgs* jobs, const int32_t* start, int njobs, int blocks, hipStream_t s);
slk_status launch_final_packed(int G, const FinalArgs* jobs, const int32_t* start, int njobs, int blocks,
                               hipStream_t s);
slk_status launch_reduce_packed(const ReduceJob* jobs, int njobs, hipStream_t s);
slk_status launch_mode_reduce_packed(const ModeJob* jobs, const int32_t* start, int njobs, int blocks, hipStream_t s);
int iter_grid(int64_t n, int32_t L, int64_t n_heavy, int32_t wsteps);
// Tile shapes from the autotuned table (tune.hip): row batches per wave of the float4 z-update and
// final pass for a problem of n rows and L clusters; queries per work-group of the exact kNN.
int32_t tune_wave_steps(int64_t n, int32_t L);
int32_t tune_knn_width(int64_t n, int32_t d, int64_t n_rows);
slk_status launch_iter(const IterArgs& a, int grid, hipStream_t s);
// The row-per-lane-group z-update for any L (no heavy-row split, no col_off), on rows of stride
// a.ldz, optionally in the caller's order (a.zperm), and its pass reduction.
int64_t iter_rows_per_group(int32_t L);
int iter_grid_rows(int64_t n, int32_t L);
slk_status launch_iter_rows(const IterArgs& a, int grid, hipStream_t s);
slk_status launch_final(const FinalArgs& a, int grid, hipStream_t s);
// The z-update (L <= 64) that also writes the labels and byproduct-mode candidates of its input,
// as launch_final would from the same input, and its pass reduction.
slk_status launch_iter_emit(const FinalArgs& f, int grid, hipStream_t s);
// modes_out: L int32 on the device; mirror (may be null): a second copy, e.g. host-mapped memory;
// cur and moved (both null or both set): moved[l] = (modes_out[l] != cur[l]).
slk_status launch_mode_reduce(const float* cand_v, const int32_t* cand_i, int grid, int32_t L, int32_t* modes_out,
                              hipStream_t s, int32_t* mirror = nullptr, const int32_t* cur = nullptr,
                              int32_t* moved = nullptr);
struct EnergyArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* labels_int;  // internal order
  const float* A;             // internal order (FP32 unary)
  const float* x;             // original order points (for the FP64 recheck), may be null
  const int32_t* perm;        // internal -> original
  const int32_t* modes;       // L original indices (device)
  const float* mvec;          // L x d mode vectors (SLK-MS; null = the points at `modes`)
  int64_t n;
  int32_t d, L, ldz;
  double inv2s2;
  double* part_un;            // grid doubles
  double* part_un64;          // grid doubles
  long long* part_cut;        // grid counts
  double* out;                // [0] unary32, [1] unary64 (written by the reduce kernel)
  long long* out_cut;
  const int32_t* heavy;       // rows handled by the first hblocks work-groups
  int32_t n_heavy;
  int32_t hblocks;
  int32_t heavy_deg;
  // L flags from the mode reduction (launch_energy only): if any mode moved, another outer
  // iteration follows and this energy is never reported, so both kernels return at once.
  // Null: always compute.
  const int32_t* moved;
};
// Grids include the heavy-row work-groups in front (n_heavy = 0: none).
int energy_grid(int64_t n, int64_t n_heavy);
slk_status launch_energy(const EnergyArgs& a, int grid, hipStream_t s);
slk_status launch_energy_packed(const EnergyArgs* jobs, const int32_t* start, int njobs, int blocks, hipStream_t s);
// SLK-MS: mean-shift of the modes m (L x d, in place) for the assignment Z (internal order,
// stride ldz) until no mode moves by more than tol * sigma or max_iter steps (meanshift.hip).
slk_status mean_shift_loop(const float* x, int64_t n, int32_t d, const int32_t* perm, const float* Z, int32_t L,
                           int32_t ldz, float* m, double sigma2, double tol, int32_t max_iter, int32_t umode,
                           hipStream_t s, int32_t* iters, double* last_shift);

// One problem of a grouped exact kNN search (all rows of x are queries, the point itself excluded).
struct KnnExactJob {
  const float* x;
  int64_t n;
  int32_t d, k, bf16;
  int32_t* out_idx;   // n x k
  double* out_d2;     // n x k
};
// The exact search of several problems in one launch (graph.hip); lists identical to knn_exact's.
slk_status knn_exact_group(const KnnExactJob* jobs_host, int njobs, hipStream_t s);

// The kNN method AUTO resolves to: the exact search when n^2 d <= 4e9 (api.hip).
bool knn_takes_exact(int64_t n, int32_t d, const slk_knn_opts& o);
// 1 if the MFMA candidate search over n_keys keys tests whole key tiles before merging (long scans)
bool knn_long_scan(int64_t n_keys);

// argument checks and per-graph settings shared by the C ABI and the served form (api.hip)
slk_status check_points(const float* x, int64_t n, int32_t d);
slk_status check_params(const slk_params* p);
double pick_sigma2(const slk_params& p, const slk_graph* g);
int64_t heavy_rows_for(const slk_graph* g, int32_t L);
void set_heavy(IterArgs& a, const slk_graph* g, int32_t L);
void set_heavy(EnergyArgs& e, const slk_graph* g);

// caller layout (stride L, original order) <-> internal layout (stride ldz, internal order)
slk_status launch_gather_rows(const float* src, const int32_t* perm, int64_t n, int32_t L, int32_t ldz, float* dst,
                              hipStream_t s);
slk_status launch_scatter_rows(const float* src, const int32_t* perm, int64_t n, int32_t L, int32_t ldz, float* dst,
                               hipStream_t s);
slk_status launch_col_offsets(const int32_t* col_idx, int64_t nnz, int64_t n, int32_t L, uint32_t* out, hipStream_t s);
slk_status launch_to_internal_labels(const int32_t* labels_user, const int32_t* iperm, int64_t n, int32_t* out,
                                     hipStream_t s);
slk_status launch_labels_to_user(const int32_t* labels_int, const int32_t* perm, int64_t n, int32_t* out,
                                 hipStream_t s);

// graph construction
// k nearest points of x for each query: rows of x (rows[] or all n_rows, the point itself
// excluded) or, if y is given, the n_rows rows of y (nothing excluded).
slk_status knn_exact(const float* x, int64_t n, int32_t d, int32_t k, int32_t bf16, const int32_t* rows,
                     int64_t n_rows, int32_t* out_idx, double* out_d2, hipStream_t s, const float* y = nullptr);
// With split_ok, small query sets (d <= 128) take the split candidate search, which lowers one
// search's latency on an otherwise idle device; the served form's graph builders, whose searches
// run beside other work, pass false (the split search's extra work-groups cost throughput there).
slk_status knn_mfma(const float* x, int64_t n, int32_t d, int32_t k, int32_t cand, int32_t bf16,
                    int32_t* out_idx, double* out_d2, int64_t* n_certified, int64_t* n_fallback, hipStream_t s,
                    const float* y = nullptr, int64_t m = 0, bool split_ok = true);
// Graph arrays.  A thread that enables the pooled mode (the served form's graph builders)
// allocates them from the stream-ordered pool; such a graph is released with destroy_graph_on,
// stream-ordered, without the device-wide synchronisation that freeing plain allocations implies.
void set_graph_pool(bool on);
bool graph_pool();
hipError_t graph_alloc(void** p, size_t bytes, hipStream_t s);
void graph_free(void* p, bool pooled, hipStream_t s);
void destroy_graph_on(slk_graph* g, hipStream_t s);

// Centred bf16 split of the points for MFMA Gram products (knn_mfma.hip): y = x - mean (FP64;
// bf16 points: y = bf16(x), no centring), xh = bf16(y), xl = bf16(y - xh), dp columns (zero
// padded), nrm = ||y||^2; mean receives the d column means (unused with bf16 points).
slk_status split_points(const float* x, int64_t n, int32_t d, int32_t dp, int32_t bf16, double* mean, uint16_t* xh,
                        uint16_t* xl, float* nrm, hipStream_t s);
slk_status build_csr(int64_t n, int32_t k, const int32_t* knn_idx, int32_t** row_ptr, int32_t** col_idx,
                     int32_t* nnz_dev, hipStream_t s);
slk_status sum_f64(const double* v, int64_t count, double* out_dev, hipStream_t s);
slk_status exclusive_scan_i32(const int32_t* in, int64_t count, int32_t* out, hipStream_t s);
slk_status sort_rows(const int32_t* row_ptr, int64_t n, int32_t* col_idx, hipStream_t s);
slk_status relabel_csr(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* perm,
                       const int32_t* iperm, int32_t* new_row_ptr, int32_t* new_col_idx, hipStream_t s);
slk_status degree_stats(const int32_t* row_ptr, int64_t n, int32_t* mn, int32_t* mx, hipStream_t s);
// min and max row length into mm_dev[0], mm_dev[1] (stream-ordered, no readback)
slk_status launch_degree_minmax(const int32_t* row_ptr, int64_t n, int32_t* mm_dev, hipStream_t s);

}  // namespace slk
