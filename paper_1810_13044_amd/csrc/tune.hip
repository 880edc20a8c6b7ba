// Tile shapes chosen by the project's autotuner (tune.py measures the candidates on the GPU and
// writes tune_table.h).  Both the single fits and the served form look shapes up here, so a job's
// tiles - and with them the order of its bound's partial sums - are the same wherever it runs.
#include "common.h"
#include "tune_table.h"

#include <atomic>

namespace slk {
namespace {

constexpr int kQBWide = 8, kQBNarrow = 4;
constexpr double kQBNarrowKeyBytes = 4.0 * 1024 * 1024;  // one XCD's L2
constexpr int64_t kQBNarrowMaxRows = 8 * 512;            // below two wide blocks per CU

std::atomic<int32_t> g_ws_override{0};

}  // namespace

int32_t tune_wave_steps(int64_t n, int32_t L) {
  const int32_t o = g_ws_override.load(std::memory_order_relaxed);
  if (o > 0) return o;
  const int32_t g = groups4(L);
  for (const TuneZEntry& e : kTuneZ)
    if (e.g == g && n <= e.n_max) return e.wave_steps;
  return 4;
}

// 4 queries per work-group while the points fit in one XCD's L2 or the query rows are few (the
// extra blocks hide the latency of key reads that hit L2), else 8 (half the key reads); the
// result does not depend on the width.
int32_t tune_knn_width(int64_t n, int32_t d, int64_t n_rows) {
  return ((double)n * d * sizeof(float) <= kQBNarrowKeyBytes || n_rows < kQBNarrowMaxRows) ? kQBNarrow : kQBWide;
}

}  // namespace slk

using namespace slk;

extern "C" {

slk_status slk_tune_lookup(int64_t n, int32_t d, int32_t L, slk_tune_params* out) {
  if (!out) return fail(SLK_ERR_INVALID_ARG, "out is NULL");
  if (n < 2 || d < 1 || L < 1 || L > 256) return fail(SLK_ERR_INVALID_ARG, "need n >= 2, d >= 1, 1 <= L <= 256");
  out->wave_steps = L <= 64 ? tune_wave_steps(n, L) : 4;
  out->knn_exact_width = tune_knn_width(n, d, n);
  slk_knn_opts o;
  slk_knn_opts_default(&o);
  out->knn_exact = knn_takes_exact(n, d, o) ? 1 : 0;
  out->knn_long_scan = knn_long_scan(n) ? 1 : 0;
  return SLK_OK;
}

slk_status slk_tune_override(int32_t wave_steps) {
  if (wave_steps != 0 && wave_steps != 1 && wave_steps != 2 && wave_steps != 4 && wave_steps != 8)
    return fail(SLK_ERR_INVALID_ARG, "wave_steps must be 0 (table), 1, 2, 4 or 8");
  g_ws_override.store(wave_steps, std::memory_order_relaxed);
  return SLK_OK;
}

const char* slk_tune_source(void) { return kTuneSource; }

}  // extern "C"
