// Out-of-sample assignment.  Section 1 notes that the explicit assignment variables of the model
// give a direct out-of-sample extension; this is that extension for the bound optimizer's update:
// a query y takes the z-update of Eq. (8) once, with its unary term (Eq. (6a)) to the fitted
// modes and its pairwise term (Eq. (6b)) over its k nearest fitted points, whose assignments stay
// fixed:
//   a_yl = k(y, m_l),   b_y = sum_{q in N(y)} z_q,   z_y = softmax(a_y + lambda b_y),
// with the label the arg-max of the logits (ties to the smaller l).
#include "common.h"

#include <float.h>
#include <math.h>

#include <algorithm>
#include <vector>

namespace slk {
namespace {

constexpr int kBlock = 256;

// One wave per query; lane l holds clusters l, l + 64, ... (L <= 256).
__global__ __launch_bounds__(kBlock) void predict_kernel(const float* __restrict__ a, const float* __restrict__ z,
                                                         const int32_t* __restrict__ nn, int64_t m, int k, int L,
                                                         float lam, float* __restrict__ z_out,
                                                         int32_t* __restrict__ labels_out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= m) return;
  constexpr int E = 4;
  float s[E];
  float mx = -INFINITY;
  float best = -INFINITY;
  int bi = INT32_MAX;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int l = lane + 64 * e;
    if (l < L) {
      float b = 0.f;
      for (int j = 0; j < k; ++j) b += z[(int64_t)nn[row * k + j] * L + l];
      s[e] = a[row * L + l] + lam * b;
      mx = fmaxf(mx, s[e]);
      if (s[e] > best) {
        best = s[e];
        bi = l;
      }
    } else {
      s[e] = -INFINITY;
    }
  }
  // row maximum and first arg-max across the wave
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off));
    const float ov = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  float sum = 0.f;
#pragma unroll
  for (int e = 0; e < E; ++e) sum += (lane + 64 * e < L) ? expf(s[e] - mx) : 0.f;
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int l = lane + 64 * e;
    if (l < L) z_out[row * L + l] = expf(s[e] - mx) / sum;
  }
  if (labels_out && lane == 0) labels_out[row] = bi;
}

}  // namespace
}  // namespace slk

using namespace slk;

extern "C" slk_status slk_predict(const float* x, int64_t n, int32_t d, const float* z, int32_t L,
                                  const int32_t* modes_host, const float* y, int64_t m, int32_t k, double lambda,
                                  double sigma2, slk_knn_method method, slk_precision prec, void* stream,
                                  float* z_out, int32_t* labels_out, int32_t* knn_idx_out) {
  SLK_TRY(check_points(x, n, d));
  if (!z || !y || !z_out || !modes_host) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  if (m < 1 || m >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "m must satisfy 1 <= m < 2^31");
  if (L < 1 || L > 256 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(256, n)");
  if (k < 1 || k > 64 || k > n) return fail(SLK_ERR_INVALID_ARG, "k must satisfy 1 <= k <= min(64, n)");
  if (!(lambda >= 0.0) || !isfinite(lambda)) return fail(SLK_ERR_INVALID_ARG, "lambda must be finite and >= 0");
  if (!(sigma2 > 0.0) || !isfinite(sigma2)) return fail(SLK_ERR_INVALID_ARG, "sigma2 must be finite and > 0");
  if (method < SLK_KNN_AUTO || method > SLK_KNN_MFMA) return fail(SLK_ERR_INVALID_ARG, "unknown kNN method");
  if (prec != SLK_PREC_FP32 && prec != SLK_PREC_BF16 && prec != SLK_PREC_BF16X) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  for (int l = 0; l < L; ++l)
    if (modes_host[l] < 0 || modes_host[l] >= n) return fail(SLK_ERR_INVALID_ARG, "mode index out of range");
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  int32_t *nn, *modes;
  double* d2;
  float* a;
  SLK_TRY(sc.get(&nn, m * k));
  SLK_TRY(sc.get(&d2, m * k));
  SLK_TRY(sc.get(&a, m * L));
  SLK_TRY(sc.get(&modes, L));
  const int bf16 = prec == SLK_PREC_BF16;
  int meth = method;
  if (meth == SLK_KNN_AUTO) meth = ((double)m * (double)n * (double)d <= 4.0e9) ? SLK_KNN_EXACT : SLK_KNN_MFMA;
  if (meth == SLK_KNN_EXACT) {
    SLK_TRY(knn_exact(x, n, d, k, bf16, nullptr, m, nn, d2, s, y));
  } else {
    int64_t cert = 0, fb = 0;
    SLK_TRY(knn_mfma(x, n, d, k, std::max(2 * k, 32), bf16, nn, d2, &cert, &fb, s, y, m));
  }
  std::vector<int32_t> mh(modes_host, modes_host + L);
  SLK_HIP(hipMemcpyAsync(modes, mh.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
  SLK_TRY(launch_unary(y, m, d, nullptr, modes, L, L, sigma2, unary_mode(prec), a, nullptr, s, x));
  hipLaunchKernelGGL(predict_kernel, dim3((unsigned)((m + 3) / 4)), dim3(kBlock), 0, s, a, z, nn, m, k, L,
                     (float)lambda, z_out, labels_out);
  SLK_LAUNCHED("predict_kernel");
  if (knn_idx_out) SLK_HIP(hipMemcpyAsync(knn_idx_out, nn, sizeof(int32_t) * m * k, hipMemcpyDeviceToDevice, s));
  SLK_HIP(hipStreamSynchronize(s));
  return SLK_OK;
}
