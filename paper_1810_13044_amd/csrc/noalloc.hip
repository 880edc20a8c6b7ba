// One z-update (Eqs. (6b), (8)) for callers that cannot allocate device memory.
//
// The z-update's only buffers besides the caller's arrays are the per-work-group partial sums
// of the relaxed bound and the pass state; here they live in `scratch`, a fixed array in device
// memory that every device the library runs on holds for the life of the process.  Host code
// reaches it through the device address hipGetSymbolAddress returns for the current device
// (kept per device), never through the array's name.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace slk {
namespace {

constexpr size_t kScratchBytes = 2u << 20;  // 2 MiB per device
constexpr size_t kStateBytes = 256;         // IterState at the start, partials after it
constexpr size_t kMaxParts = (kScratchBytes - kStateBytes) / sizeof(double);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

__global__ void noalloc_init_state(IterState* st) {
  st->pass = 0;
  st->done = 0;
  st->numeric = 0;
  st->tol = 0.0;
  st->check = 0;
  st->trace_cap = 0;
  st->last_bound = 0.0;
  st->rel = 0.0;
  st->rel_prev = 0.0;
  st->last_pass = -1;
  st->emit_pass = -1;
}

// Device address of this device's scratch array (looked up once per device).
slk_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SLK_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SLK_ERR_UNSUPPORTED, "device index beyond the library's table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(SLK_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SLK_OK;
}

}  // namespace
}  // namespace slk

using namespace slk;

extern "C" {

int64_t slk_inner_step_noalloc_max_rows(int32_t L) {
  if (L < 1 || L > 256) return 0;
  // the grid is a multiple of 8 work-groups of iter_rows_per_group(L) rows, one partial each;
  // n * L < 2^30 holds for every call
  const int64_t by_parts = iter_rows_per_group(L) * (int64_t)(kMaxParts / 8 * 8);
  return std::min<int64_t>(by_parts, ((int64_t)1 << 30) / L - 1);
}

slk_status slk_inner_step_noalloc(const slk_graph* g, int32_t L, const float* a, const float* z_in, double lambda,
                                  double delta, int32_t pairwise_scale, void* stream, float* z_out,
                                  double* bound_dev) {
  if (!g || !a || !z_in) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  const int64_t n = g->n;
  if (L < 1 || L > 256 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(256, n)");
  if ((uint64_t)n * (uint64_t)L * 4ull >= (1ull << 32))
    return fail(SLK_ERR_INVALID_ARG, "n * L must be < 2^30");
  if (!(lambda >= 0.0) || !std::isfinite(lambda) || !(delta >= 0.0) || !std::isfinite(delta))
    return fail(SLK_ERR_INVALID_ARG, "lambda and delta must be finite and >= 0");
  if (pairwise_scale != 1 && pairwise_scale != 2) return fail(SLK_ERR_INVALID_ARG, "pairwise_scale must be 1 or 2");
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev != g->device)
    return fail(SLK_ERR_INVALID_ARG, "graph lives on another device");
  if (n > slk_inner_step_noalloc_max_rows(L))
    return fail(SLK_ERR_INVALID_ARG, "n exceeds the allocation-free limit for this L (slk_inner_step_noalloc_max_rows)");
  const int grid = iter_grid_rows(n, L);
  void* base = nullptr;
  SLK_TRY(scratch_address(&base));
  hipStream_t s = (hipStream_t)stream;
  IterState* st = reinterpret_cast<IterState*>(base);
  double* partial = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kStateBytes);
  hipLaunchKernelGGL(noalloc_init_state, dim3(1), dim3(1), 0, s, st);
  SLK_LAUNCHED("noalloc_init_state");
  IterArgs ia{};
  ia.row_ptr = g->row_ptr;
  ia.col_idx = g->col_idx;
  ia.col_off = nullptr;
  ia.A = a;
  ia.Zin = z_in;
  ia.Zout = z_out;
  ia.n = n;
  ia.L = L;
  ia.ldz = L;
  ia.lam_eff = (float)(pairwise_scale * lambda);
  ia.half_lam_eff = (float)(0.5 * pairwise_scale * lambda);
  ia.delta = (float)delta;
  ia.partial = partial;
  ia.state = st;
  ia.trace = nullptr;
  ia.bound_out = bound_dev;
  ia.mirror = nullptr;
  ia.heavy = nullptr;
  ia.n_heavy = 0;
  ia.hblocks = 0;
  ia.heavy_deg = INT32_MAX;
  ia.zperm = g->perm;
  return launch_iter_rows(ia, grid, s);
}

}  // extern "C"
