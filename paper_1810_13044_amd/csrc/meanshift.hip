// SLK-MS mode update (Eq. (9), the SLK-MS branch of Algorithm 1): for every cluster l,
//   m_l <- sum_p w_pl x_p / sum_p w_pl,   w_pl = z_pl k(x_p, m_l),
// iterated until no mode moves by more than tol * sigma in one step.
//
// One step: the kernel values k(x_p, m_l) come from the unary kernel (with mode vectors);
// ms_partial_kernel forms w = z * k and, per work-group of 1,024 rows and 128 coordinates, the
// partial sums sum_p w_pl x_pc and sum_p w_pl in FP32.  The first is the contraction W^T X of a
// 64 x 1,024 by 1,024 x 128 block, done on v_mfma_f32_32x32x2_f32 (FP32 products and
// accumulation; each wave owns two 32 x 32 cluster-by-coordinate tiles), rows staged through LDS
// 32 at a time with the next 32 loaded into registers meanwhile.  ms_num_kernel and ms_den_kernel
// add the partials in FP64 in a fixed order, divide, and give each mode's squared displacement.
#include "common.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace slk {
namespace {

constexpr int kBlock = 256;
constexpr int kRowsPer = 1024;   // rows per partial work-group
constexpr int kSub = 32;         // rows staged per LDS round
constexpr int kCw = 128;         // coordinates per work-group
constexpr int kLmax = 64;

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__global__ __launch_bounds__(kBlock) void ms_partial_kernel(const float* __restrict__ x, int64_t n, int d,
                                                            const int32_t* __restrict__ perm,
                                                            const float* __restrict__ Z, const float* __restrict__ A,
                                                            int L, int ldz, int bf16, float* __restrict__ part_num,
                                                            float* __restrict__ part_den) {
  // rows padded by 32 floats: the two half-waves read consecutive rows in different banks
  __shared__ float ws[kSub][kLmax + 32];
  __shared__ float xs[kSub][kCw + 32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, col = lane & 31;
  // wave w: clusters 32 (w / 2) .. +31, coordinates 64 (w % 2) .. +63 as two 32-wide tiles
  const int lb = wave >> 1, cb = (wave & 1) * 64;
  const int64_t rb = blockIdx.x;
  const int c0 = blockIdx.y * kCw;
  const int64_t r0 = rb * kRowsPer;
  f32x16 acc[2];
  acc[0] = f32x16{};
  acc[1] = f32x16{};
  float den = 0.f;
  // the next round's weights and coordinates are loaded into registers while this round
  // computes: thread tid moves weights (tid / 64 + 4 k, tid % 64) and coordinates
  // (tid / 128 + 2 k, tid % 128)
  constexpr int kWk = kSub * kLmax / kBlock, kXk = kSub * kCw / kBlock;
  float wv[kWk], xv[kXk];
  const int wl = tid % kLmax, wr = tid / kLmax;
  const int xc = tid % kCw, xr = tid / kCw;
  auto load = [&](int s0) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < kWk; ++k) {
      const int64_t row = r0 + s0 + wr + (kBlock / kLmax) * k;
      wv[k] = (row < n && wl < L) ? Z[row * ldz + wl] * A[row * ldz + wl] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kXk; ++k) {
      const int64_t row = r0 + s0 + xr + (kBlock / kCw) * k;
      float v = 0.f;
      if (row < n && c0 + xc < d) {
        const int64_t gr = perm ? perm[row] : row;
        v = x[gr * d + c0 + xc];
      }
      xv[k] = v;
    }
  };
  load(0);
  for (int s0 = 0; s0 < kRowsPer; s0 += kSub) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kWk; ++k) ws[wr + (kBlock / kLmax) * k][wl] = wv[k];
#pragma unroll
    for (int k = 0; k < kXk; ++k) xs[xr + (kBlock / kCw) * k][xc] = bf16 ? bf16_round(xv[k]) : xv[k];
    __syncthreads();
    if (s0 + kSub < kRowsPer && r0 + s0 + kSub < n) load(s0 + kSub);
    // A[l][k] = w of row k, B[k][c] = x of row k: lane t supplies row 2 s + t / 32
#pragma unroll 4
    for (int s2 = 0; s2 < kSub / 2; ++s2) {
      const int r = 2 * s2 + g;
      const float a = ws[r][32 * lb + col];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xs[r][cb + col], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xs[r][cb + 32 + col], acc[1], 0, 0, 0);
    }
    if (tid < kLmax)
      for (int r = 0; r < kSub; ++r) den += ws[r][tid];
    if (r0 + s0 + kSub >= n) break;
  }
  // C layout: lane t holds coordinate t % 32 of the tile, clusters 8 (r / 4) + 4 (t / 32) + r % 4
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int c = c0 + cb + 32 * j + col;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int l = 32 * lb + 8 * (r >> 2) + 4 * g + (r & 3);
      if (l < L && c < d) part_num[(rb * L + l) * d + c] = acc[j][r];
    }
  }
  if (blockIdx.y == 0 && tid < L) part_den[rb * L + tid] = den;
}

// den[l] = fixed-order FP64 sum of the partial denominators (one work-group per cluster)
__global__ __launch_bounds__(kBlock) void ms_den_kernel(const float* __restrict__ part_den, int nrb, int L,
                                                        double* __restrict__ den) {
  __shared__ double red[kBlock];
  const int l = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < nrb; b += kBlock) s += (double)part_den[(int64_t)b * L + l];
  red[tid] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) den[l] = red[0];
}

// New mode coordinates: one work-group per (cluster, 64 coordinates), four row-block groups
// summed separately and then in a fixed order; a cluster with no weight keeps its mode.
__global__ __launch_bounds__(kBlock) void ms_num_kernel(const float* __restrict__ part_num, int nrb, int L, int d,
                                                        const double* __restrict__ den,
                                                        const float* __restrict__ m_old, float* __restrict__ m_new) {
  __shared__ double red[4][64];
  const int l = blockIdx.x, tid = threadIdx.x;
  const int cl = tid & 63, grp = tid >> 6;
  const int c = blockIdx.y * 64 + cl;
  double s = 0.0;
  if (c < d)
    for (int b = grp; b < nrb; b += 4) s += (double)part_num[((int64_t)b * L + l) * d + c];
  red[grp][cl] = s;
  __syncthreads();
  if (grp == 0 && c < d) {
    const double num = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
    const double dl = den[l];
    m_new[(int64_t)l * d + c] = dl > 0.0 ? (float)(num / dl) : m_old[(int64_t)l * d + c];
  }
}

// squared displacement of every mode (FP64), one work-group per cluster
__global__ __launch_bounds__(kBlock) void ms_shift_kernel(const float* __restrict__ m_old,
                                                          const float* __restrict__ m_new, int d,
                                                          double* __restrict__ shift2) {
  __shared__ double red[kBlock];
  const int l = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int c = tid; c < d; c += kBlock) {
    const double t = (double)m_new[(int64_t)l * d + c] - (double)m_old[(int64_t)l * d + c];
    s += t * t;
  }
  red[tid] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) shift2[l] = red[0];
}

}  // namespace

// One mean-shift step of all modes for the assignment Z (internal order, stride ldz) and the
// kernel values A at m_old (same layout); writes m_new and each mode's squared displacement.
// pn (nrb L d floats), pd (nrb L floats) and den (L doubles) are workspace, nrb = ceil(n / 1024).
slk_status launch_ms_step(const float* x, int64_t n, int32_t d, const int32_t* perm, const float* Z, const float* A,
                          int32_t L, int32_t ldz, int32_t bf16, const float* m_old, float* m_new, double* shift2,
                          float* pn, float* pd, double* den, hipStream_t s) {
  if (L > kLmax) return fail(SLK_ERR_UNSUPPORTED, "mean-shift modes take L <= 64");
  const int nrb = (int)((n + kRowsPer - 1) / kRowsPer);
  const int ncw = (d + kCw - 1) / kCw;
  {
    KernelTimer kt("ms_partial_kernel", s);
    hipLaunchKernelGGL(ms_partial_kernel, dim3((unsigned)nrb, (unsigned)ncw), dim3(kBlock), 0, s, x, n, d, perm, Z,
                       A, L, ldz, bf16, pn, pd);
    SLK_LAUNCHED("ms_partial_kernel");
  }
  hipLaunchKernelGGL(ms_den_kernel, dim3((unsigned)L), dim3(kBlock), 0, s, pd, nrb, L, den);
  SLK_LAUNCHED("ms_den_kernel");
  hipLaunchKernelGGL(ms_num_kernel, dim3((unsigned)L, (unsigned)((d + 63) / 64)), dim3(kBlock), 0, s, pn, nrb, L, d,
                     den, m_old, m_new);
  SLK_LAUNCHED("ms_num_kernel");
  hipLaunchKernelGGL(ms_shift_kernel, dim3((unsigned)L), dim3(kBlock), 0, s, m_old, m_new, d, shift2);
  SLK_LAUNCHED("ms_shift_kernel");
  return SLK_OK;
}

// Mean-shift iterated from m (L x d, updated in place) until no mode moves by more than tol * sigma
// or max_iter steps; Z and the workspace as above.  *iters receives the steps taken.
slk_status mean_shift_loop(const float* x, int64_t n, int32_t d, const int32_t* perm, const float* Z, int32_t L,
                           int32_t ldz, float* m, double sigma2, double tol, int32_t max_iter, int32_t umode,
                           hipStream_t s, int32_t* iters, double* last_shift) {
  if (L > kLmax) return fail(SLK_ERR_UNSUPPORTED, "mean-shift modes take L <= 64");
  Scratch sc(s);
  float *A, *m2, *pn, *pd;
  double *sh, *den;
  const int64_t nrb = (n + kRowsPer - 1) / kRowsPer;
  SLK_TRY(sc.get(&A, (size_t)n * ldz));
  SLK_TRY(sc.get(&m2, (size_t)L * d));
  SLK_TRY(sc.get(&sh, L));
  SLK_TRY(sc.get(&pn, (size_t)nrb * L * d));
  SLK_TRY(sc.get(&pd, (size_t)nrb * L));
  SLK_TRY(sc.get(&den, L));
  std::vector<double> h(L);
  float* cur = m;
  float* nxt = m2;
  int it = 0;
  double shift = 0.0;
  for (it = 1; it <= max_iter; ++it) {
    SLK_TRY(launch_unary(x, n, d, perm, nullptr, L, ldz, sigma2, umode, A, nullptr, s, nullptr, cur));
    SLK_TRY(launch_ms_step(x, n, d, perm, Z, A, L, ldz, umode == kUnaryRounded, cur, nxt, sh, pn, pd, den, s));
    SLK_HIP(hipMemcpyAsync(h.data(), sh, sizeof(double) * L, hipMemcpyDeviceToHost, s));
    SLK_HIP(hipStreamSynchronize(s));
    shift = std::sqrt(*std::max_element(h.begin(), h.end()));
    std::swap(cur, nxt);
    if (shift <= tol * std::sqrt(sigma2)) break;
  }
  if (it > max_iter) it = max_iter;
  if (cur != m) SLK_HIP(hipMemcpyAsync(m, cur, sizeof(float) * L * d, hipMemcpyDeviceToDevice, s));
  SLK_HIP(hipStreamSynchronize(s));
  *iters = it;
  if (last_shift) *last_shift = shift;
  return SLK_OK;
}

}  // namespace slk

using namespace slk;

extern "C" slk_status slk_mean_shift(const float* x, int64_t n, int32_t d, const float* z, int32_t L,
                                     const float* modes_in, double sigma2, double tol, int32_t max_iter,
                                     slk_precision prec, void* stream, float* modes_out, int32_t* iters_host) {
  SLK_TRY(check_points(x, n, d));
  if (!z || !modes_in || !modes_out) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  if (L < 1 || L > 64 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(64, n)");
  if (!(sigma2 > 0.0) || !isfinite(sigma2)) return fail(SLK_ERR_INVALID_ARG, "sigma2 must be finite and > 0");
  if (!(tol >= 0.0) || max_iter < 1) return fail(SLK_ERR_INVALID_ARG, "need tol >= 0 and max_iter >= 1");
  if (prec != SLK_PREC_FP32 && prec != SLK_PREC_BF16 && prec != SLK_PREC_BF16X) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  if (modes_out != modes_in)
    SLK_HIP(hipMemcpyAsync(modes_out, modes_in, sizeof(float) * L * d, hipMemcpyDeviceToDevice, s));
  int32_t it = 0;
  SLK_TRY(mean_shift_loop(x, n, d, nullptr, z, L, L, modes_out, sigma2, tol, max_iter, unary_mode(prec), s, &it,
                          nullptr));
  if (iters_host) *iters_host = it;
  return SLK_OK;
}
