// K-means++ seeding (named in Section 4.2 for the initial centres; the sampling rule is that of
// Arthur and Vassilvitskii, 2007) and, as its by-product, the nearest-seed assignment.
//
// The caller passes the uniforms u_0 .. u_{L-1} in [0, 1).  Centre 0 is the point floor(u_0 n);
// centre r >= 1 is the smallest p whose prefix sum of D^2 (in point order) exceeds u_r * sum D^2,
// where D^2(p) is the squared distance from x_p to the nearest centre chosen so far; if
// sum D^2 = 0 every point sits on a centre and centre r is floor(u_r n).
//
// Per round, on the device and with no host round trip:
//   kpp_dist_kernel    D^2(p) <- min(D^2(p), ||x_p - c_r||^2) with the distance a fixed-order FP64
//                      sum over the coordinates (no FMA; the same value as the exact kNN), the
//                      nearest centre's number kept for the assignment (strictly nearer only, so
//                      ties go to the earlier centre), and per-work-group FP64 sums of D^2.
//   kpp_select_kernel  one work-group scans the work-group sums, finds the one holding the target
//                      and scans its points.  The prefix sums are formed in a different order
//                      from a plain left-to-right sum; the choice can differ from such a sum only
//                      when the target lies within a few ulps of a prefix boundary.
// The pass reads x once per round: n d 4 bytes plus 16 n bytes of D^2, HBM-bound.
#include "common.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace slk {
namespace {

constexpr int kRows = 256;   // points per work-group, one per thread
constexpr int kCc = 32;      // coordinates staged per round trip through LDS
constexpr int kSel = 1024;   // threads of the selection work-group

__device__ __forceinline__ double sq_step(double acc, double a, double b) {
#pragma clang fp contract(off)
  const double t = a - b;
  const double t2 = t * t;
  return acc + t2;
}

__global__ __launch_bounds__(kRows) void kpp_dist_kernel(const float* __restrict__ x, int64_t n, int d, int bf16,
                                                         const int32_t* __restrict__ centres, int r,
                                                         double* __restrict__ D2, int32_t* __restrict__ lab,
                                                         double* __restrict__ part) {
  __shared__ float xs[kRows][kCc + 1];
  __shared__ float cs[kCc];
  __shared__ double red[kRows];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  const int64_t row = r0 + tid;
  const int64_t c = centres[r];
  double acc = 0.0;
  for (int c0 = 0; c0 < d; c0 += kCc) {
    const int cw = min(kCc, d - c0);
    // all loads of the chunk in flight before the first LDS store
    // thread tid moves coordinate tid % 32 of rows tid / 32 + 8 k; all loads of the chunk are in
    // flight before the first LDS store
    constexpr int kStep = kRows / kCc;
    const int rr0 = tid / kCc, j = tid % kCc;
    const float* src = x + (r0 + rr0) * d + c0 + j;
    const int64_t stride = (int64_t)kStep * d;
    float v[kCc];
#pragma unroll
    for (int k = 0; k < kCc; ++k)
      v[k] = (r0 + rr0 + kStep * k < n && j < cw) ? src[k * stride] : 0.f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCc; ++k) xs[rr0 + kStep * k][j] = bf16 ? bf16_round(v[k]) : v[k];
    if (tid < kCc) {
      float v = tid < cw ? x[c * d + c0 + tid] : 0.f;
      if (bf16) v = bf16_round(v);
      cs[tid] = v;
    }
    __syncthreads();
    for (int j = 0; j < cw; ++j) acc = sq_step(acc, (double)xs[tid][j], (double)cs[j]);
  }
  double v = 0.0;
  if (row < n) {
    double cur = r == 0 ? INFINITY : D2[row];
    if (acc < cur) {
      cur = acc;
      if (lab) lab[row] = r;
    }
    D2[row] = cur;
    v = cur;
  }
  red[tid] = v;
  __syncthreads();
  for (int w = kRows / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

// Centre r from the D^2 after centre r - 1; writes centres[r].  The owner thread of the crossing
// (in a scan over the per-thread sums of the block sums) finds the block; the block's points are
// then scanned by the whole work-group.
__global__ __launch_bounds__(kSel) void kpp_select_kernel(const double* __restrict__ part, int nb,
                                                          const double* __restrict__ D2, int64_t n,
                                                          const double* __restrict__ u, int r,
                                                          int32_t* __restrict__ centres) {
  __shared__ double sc[kSel];
  __shared__ int s_bb, s_walk, s_first, s_last, s_lastb;
  __shared__ double s_pre;
  const int tid = threadIdx.x;
  const int per = (nb + kSel - 1) / kSel;
  const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += part[b];
  if (tid == 0) {
    s_bb = -1;
    s_walk = 1;
    s_first = INT32_MAX;
    s_last = -1;
    s_lastb = -1;
  }
  sc[tid] = s;
  __syncthreads();
  // inclusive scan of the per-thread sums (fixed order)
  for (int off = 1; off < kSel; off <<= 1) {
    const double t = tid >= off ? sc[tid - off] : 0.0;
    __syncthreads();
    sc[tid] += t;
    __syncthreads();
  }
  const double total = sc[kSel - 1];
  const double target = u[r] * total;
  const double before = tid == 0 ? 0.0 : sc[tid - 1];
  if (total > 0.0 && sc[tid] > target && before <= target) {
    // this thread's blocks hold the crossing
    double pre = before;
    int bb = -1;
    for (int b = b0; b < b1; ++b) {
      if (pre + part[b] > target) {
        bb = b;
        break;
      }
      pre += part[b];
    }
    if (bb < 0) {  // rounding between the scan and this walk: the last block with weight
      s_walk = 0;
      for (int b = b1 - 1; b >= b0; --b)
        if (part[b] > 0.0) {
          bb = b;
          break;
        }
    }
    s_bb = bb;
    s_pre = pre;
  }
  // the target at the very top (rounding of the scan): the last block with weight
  if (total > 0.0) {
    for (int b = b1 - 1; b >= b0; --b)
      if (part[b] > 0.0) {
        atomicMax(&s_lastb, b);
        break;
      }
  }
  __syncthreads();
  const int walk = s_bb >= 0 ? s_walk : 0;
  const int bb = s_bb >= 0 ? s_bb : s_lastb;
  if (total > 0.0 && bb >= 0) {
    // inclusive scan of the block's D^2 (threads 0 .. kRows - 1), then the first crossing
    const int64_t p = (int64_t)bb * kRows + tid;
    const double v = (tid < kRows && p < n) ? D2[p] : 0.0;
    __syncthreads();
    sc[tid] = v;
    __syncthreads();
    for (int off = 1; off < kRows; off <<= 1) {
      const double t = (tid < kRows && tid >= off) ? sc[tid - off] : 0.0;
      __syncthreads();
      if (tid < kRows) sc[tid] += t;
      __syncthreads();
    }
    if (tid < kRows && v > 0.0) {
      atomicMax(&s_last, tid);
      if (walk && s_pre + sc[tid] > target) atomicMin(&s_first, tid);
    }
  }
  __syncthreads();
  if (tid == 0) {
    long long pk;
    if (total > 0.0 && bb >= 0) {
      const int off = s_first != INT32_MAX ? s_first : s_last;
      pk = (long long)bb * kRows + off;
    } else {
      pk = min<long long>((long long)floor(u[r] * (double)n), n - 1);
    }
    centres[r] = (int32_t)pk;
  }
}

}  // namespace
}  // namespace slk

using namespace slk;

extern "C" slk_status slk_kmeanspp(const float* x, int64_t n, int32_t d, int32_t L, const double* u_host,
                                   slk_precision prec, void* stream, int32_t* centres_out_host, int32_t* labels_out,
                                   double* d2_out) {
  SLK_TRY(check_points(x, n, d));
  if (L < 1 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= n");
  if (!u_host || !centres_out_host) return fail(SLK_ERR_INVALID_ARG, "NULL argument");
  for (int r = 0; r < L; ++r)
    if (!(u_host[r] >= 0.0 && u_host[r] < 1.0)) return fail(SLK_ERR_INVALID_ARG, "uniforms must lie in [0, 1)");
  if (prec != SLK_PREC_FP32 && prec != SLK_PREC_BF16) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  const int nb = (int)((n + kRows - 1) / kRows);
  double *D2 = d2_out, *part, *u;
  int32_t* cent;
  if (!D2) SLK_TRY(sc.get(&D2, n));
  SLK_TRY(sc.get(&part, nb));
  SLK_TRY(sc.get(&u, L));
  SLK_TRY(sc.get(&cent, L));
  std::vector<double> uh(u_host, u_host + L);
  const int32_t c0 = (int32_t)std::min<int64_t>((int64_t)std::floor(uh[0] * (double)n), n - 1);
  SLK_HIP(hipMemcpyAsync(u, uh.data(), sizeof(double) * L, hipMemcpyHostToDevice, s));
  SLK_HIP(hipMemcpyAsync(cent, &c0, sizeof(int32_t), hipMemcpyHostToDevice, s));
  const int bf16 = prec == SLK_PREC_BF16;
  for (int r = 0; r < L; ++r) {
    {
      KernelTimer kt("kpp_dist_kernel", s);
      hipLaunchKernelGGL(kpp_dist_kernel, dim3((unsigned)nb), dim3(kRows), 0, s, x, n, d, bf16, cent, r, D2,
                         labels_out, part);
      SLK_LAUNCHED("kpp_dist_kernel");
    }
    if (r + 1 < L) {
      KernelTimer kt("kpp_select_kernel", s);
      hipLaunchKernelGGL(kpp_select_kernel, dim3(1), dim3(kSel), 0, s, part, nb, D2, n, u, r + 1, cent);
      SLK_LAUNCHED("kpp_select_kernel");
    }
  }
  SLK_HIP(hipMemcpyAsync(centres_out_host, cent, sizeof(int32_t) * L, hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  return SLK_OK;
}
