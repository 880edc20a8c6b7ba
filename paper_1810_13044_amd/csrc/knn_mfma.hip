// Exact kNN (Section 4.2) at scale: candidates from a bf16 MFMA Gram matrix, exact FP64 re-rank,
// and a certificate that the exact top-k lies among the candidates.
//
//   1. centre_split: y = x - mean(x) in FP64, split y = h + l with h = bf16(y), l = bf16(y - h)
//      (|y - h - l| <= ~2^-16 |y|); row norms n_p = ||y_p||^2 in FP64.  With bf16 points
//      (SLK_PREC_BF16) the points are bf16(x) themselves: h = bf16(x), l = 0, no centring.
//   2. cand_kernel: G~ = h_p.h_q + h_p.l_q + l_p.h_q on v_mfma_f32_32x32x16_bf16 with FP32
//      accumulation (a fresh accumulator per 32 coordinates, then summed).  For every pair a
//      rigorous lower bound of the squared distance is formed,
//          lb_pq = (1 - c) (n_p + n_q) - 2 G~   <=  ||x_p - x_q||^2,
//      where c bounds the split residual, the FP32 accumulation and the final roundings (times a
//      safety factor 2).  Each query row keeps the C smallest lb (C = candidates) in LDS; a
//      key tile is merged only when one of its bounds beats the row's current C-th bound.
//   3. rerank_kernel: exact FP64 distances of the C candidates (fixed coordinate order, no FMA,
//      identical to the exact kernel), sorted by (distance, index).  The first k are exact if the
//      k-th exact distance is below tau_p, the C-th candidate bound: every other point q has
//      ||x_p - x_q||^2 >= lb_pq >= tau_p.  Rows that fail are recomputed by the exact kernel.
#include "common.h"

#include <float.h>
#include <math.h>

#include <algorithm>
#include <vector>

namespace slk {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kBlock = 256;
constexpr int kTile = 64;      // queries per block and keys per step
constexpr int kDK = 32;        // coordinates per staged chunk
constexpr int kPad = 8;        // bf16 padding per LDS row (16 bytes)
constexpr int kRow = kDK + kPad;
constexpr int kMaxCand = 64;

__device__ __forceinline__ uint16_t bf16_bits(float v) {
  const float r = bf16_round(v);
  uint32_t b;
  __builtin_memcpy(&b, &r, 4);
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ double sqdist_step(double acc, double a, double b) {
#pragma clang fp contract(off)
  const double t = a - b;
  const double t2 = t * t;
  return acc + t2;
}

// (v, i) < (v', i') lexicographically
__device__ __forceinline__ bool lex_less(float v0, int i0, float v1, int i1) { return v0 < v1 || (v0 == v1 && i0 < i1); }
__device__ __forceinline__ bool lex_less_d(double v0, int i0, double v1, int i1) {
  return v0 < v1 || (v0 == v1 && i0 < i1);
}

// ------------------------------------------------------------------------------------------
// 1. column means, centring and the bf16 split
// ------------------------------------------------------------------------------------------
constexpr int kMeanRows = 2048;

__global__ __launch_bounds__(kBlock) void colsum_kernel(const float* __restrict__ x, int64_t n, int d,
                                                        double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.y * kMeanRows;
  const int64_t r1 = min<int64_t>(n, r0 + kMeanRows);
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < d; j += gridDim.x * kBlock) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)x[r * d + j];
    part[(int64_t)blockIdx.y * d + j] = s;
  }
}

__global__ __launch_bounds__(kBlock) void colmean_kernel(const double* __restrict__ part, int nparts, int64_t n, int d,
                                                         double* __restrict__ mean) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * d + j];
  mean[j] = s / (double)n;
}

// one wave per row: h, l (bf16 bits, Dp columns, zero padded) and the FP64 norm of y
__global__ __launch_bounds__(kBlock) void split_kernel(const float* __restrict__ x, int64_t n, int d, int dp,
                                                       const double* __restrict__ mean, int bf16,
                                                       uint16_t* __restrict__ xh, uint16_t* __restrict__ xl,
                                                       float* __restrict__ nrm) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < dp; j += 64) {
    uint16_t hb = 0, lb = 0;
    if (j < d) {
      const float xv = x[row * d + j];
      double y;
      if (bf16) {
        y = (double)bf16_round(xv);
        hb = bf16_bits((float)y);
      } else {
        y = (double)xv - mean[j];
        const float h = bf16_round((float)y);
        hb = bf16_bits(h);
        lb = bf16_bits((float)(y - (double)h));
      }
      s += y * y;
    }
    xh[row * dp + j] = hb;
    xl[row * dp + j] = lb;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) nrm[row] = (float)s;
}

// ------------------------------------------------------------------------------------------
// 2. candidate search on MFMA
// ------------------------------------------------------------------------------------------
// 128-element bitonic sort across a wave, two (value, index) pairs per lane at positions
// lane and lane + 64; ascending.
__device__ __forceinline__ void wave_sort128(float (&v)[2], int (&ix)[2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride == 64) {
        // partners are the two halves held by the same lane; size == 128: ascending
        if (lex_less(v[1], ix[1], v[0], ix[0])) {
          const float tv = v[0];
          const int ti = ix[0];
          v[0] = v[1];
          ix[0] = ix[1];
          v[1] = tv;
          ix[1] = ti;
        }
      } else {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int e = lane + 64 * s;
          const float ov = __shfl_xor(v[s], stride);
          const int oi = __shfl_xor(ix[s], stride);
          const bool lower = (e & stride) == 0;
          const bool asc = (e & size) == 0;
          const bool other_smaller = lex_less(ov, oi, v[s], ix[s]);
          // the lower position of an ascending pair keeps the smaller element
          const bool take_other = (lower == asc) ? other_smaller : !other_smaller;
          if (take_other) {
            v[s] = ov;
            ix[s] = oi;
          }
        }
      }
    }
  }
}

struct CandSmem {
  union {
    struct {
      uint16_t qh[kTile * kRow], ql[kTile * kRow], kh[kTile * kRow], kl[kTile * kRow];
    } st;
    float S[kTile][kTile + 1];
  } u;
  float lv[kTile][kMaxCand];
  int li[kTile][kMaxCand];
  float tau[kTile];
  float nq[kTile];
  float nk[kTile];
  int any;
};

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  bf16x8 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void cand_kernel(const uint16_t* __restrict__ xh, const uint16_t* __restrict__ xl,
                                                      const float* __restrict__ nrm, int64_t n, int dp, int C,
                                                      float c1, int32_t* __restrict__ cand, float* __restrict__ tau_out) {
  __shared__ CandSmem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // 32-row half, 32-key half
  const int64_t q0 = (int64_t)blockIdx.x * kTile;
  for (int e = tid; e < kTile * kMaxCand; e += kBlock) {
    sm.lv[e / kMaxCand][e % kMaxCand] = INFINITY;
    sm.li[e / kMaxCand][e % kMaxCand] = INT32_MAX;
  }
  if (tid < kTile) {
    sm.tau[tid] = INFINITY;
    sm.nq[tid] = (q0 + tid < n) ? nrm[q0 + tid] : 0.f;
  }
  // staging: 64 rows x 32 bf16 = 256 x 16 bytes per array, one 16-byte piece per thread
  const int srow = tid >> 2, spiece = (tid & 3) * 8;
  __syncthreads();

  for (int64_t k0 = 0; k0 < n; k0 += kTile) {
    f32x16 tot = {};
    for (int c0 = 0; c0 < dp; c0 += kDK) {
      __syncthreads();
      {
        const int64_t qr = q0 + srow, kr = k0 + srow;
        uint4 zh = {0, 0, 0, 0}, a = zh, b = zh, cc = zh, dd = zh;
        if (qr < n) {
          a = *reinterpret_cast<const uint4*>(xh + qr * dp + c0 + spiece);
          if (SPLIT) b = *reinterpret_cast<const uint4*>(xl + qr * dp + c0 + spiece);
        }
        if (kr < n) {
          cc = *reinterpret_cast<const uint4*>(xh + kr * dp + c0 + spiece);
          if (SPLIT) dd = *reinterpret_cast<const uint4*>(xl + kr * dp + c0 + spiece);
        }
        *reinterpret_cast<uint4*>(&sm.u.st.qh[srow * kRow + spiece]) = a;
        *reinterpret_cast<uint4*>(&sm.u.st.kh[srow * kRow + spiece]) = cc;
        if (SPLIT) {
          *reinterpret_cast<uint4*>(&sm.u.st.ql[srow * kRow + spiece]) = b;
          *reinterpret_cast<uint4*>(&sm.u.st.kl[srow * kRow + spiece]) = dd;
        }
        if (c0 == 0 && tid < kTile) sm.nk[tid] = (k0 + tid < n) ? nrm[k0 + tid] : 0.f;
      }
      __syncthreads();
      f32x16 part = {};
#pragma unroll
      for (int ks = 0; ks < kDK; ks += 16) {
        const int ar = (32 * wr + (lane & 31)) * kRow + ks + 8 * (lane >> 5);
        const int br = (32 * wc + (lane & 31)) * kRow + ks + 8 * (lane >> 5);
        const bf16x8 ah = load8(&sm.u.st.qh[ar]);
        const bf16x8 bh = load8(&sm.u.st.kh[br]);
        part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, part, 0, 0, 0);
        if (SPLIT) {
          const bf16x8 al = load8(&sm.u.st.ql[ar]);
          const bf16x8 bl = load8(&sm.u.st.kl[br]);
          part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, part, 0, 0, 0);
          part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, part, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[r] += part[r];
    }
    // lower bounds and the filter against each row's current C-th bound
    const int kc = 32 * wc + (lane & 31);
    const int64_t key = k0 + kc;
    const float nkv = sm.nk[kc];
    float lbv[16];
    bool pass = false;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int qi = 32 * wr + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int64_t qrow = q0 + qi;
      float lb = c1 * (sm.nq[qi] + nkv) - 2.0f * tot[r];
      if (key >= n || key == qrow || qrow >= n) lb = INFINITY;
      lbv[r] = lb;
      pass |= lb < sm.tau[qi];
    }
    if (tid == 0) sm.any = 0;
    __syncthreads();
    if (__ballot(pass) != 0ull && lane == 0) sm.any = 1;
    __syncthreads();
    if (!sm.any) continue;
    // merge path: bounds to LDS (aliases the staging buffers, all reads of which are done)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int qi = 32 * wr + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      sm.u.S[qi][kc] = lbv[r];
    }
    __syncthreads();
    for (int qi = wave; qi < kTile; qi += 4) {
      const float t = sm.tau[qi];
      const float v = sm.u.S[qi][lane];
      const bool p = v < t;
      if (__ballot(p) == 0ull) continue;
      float vv[2];
      int ii[2];
      vv[0] = lane < C ? sm.lv[qi][lane] : INFINITY;
      ii[0] = lane < C ? sm.li[qi][lane] : INT32_MAX;
      vv[1] = p ? v : INFINITY;
      ii[1] = p ? (int)(k0 + lane) : INT32_MAX;
      wave_sort128(vv, ii);
      if (lane < C) {
        sm.lv[qi][lane] = vv[0];
        sm.li[qi][lane] = ii[0];
      }
      const float nt = __shfl(vv[0], C - 1);
      if (lane == 0) sm.tau[qi] = nt;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int e = tid; e < kTile * C; e += kBlock) {
    const int qi = e / C, j = e % C;
    if (q0 + qi < n) cand[(q0 + qi) * C + j] = sm.li[qi][j];
  }
  if (tid < kTile && q0 + tid < n) tau_out[q0 + tid] = sm.tau[tid];
}

// ------------------------------------------------------------------------------------------
// 3. exact FP64 re-rank of the candidates, certificate, fallback list
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void rerank_kernel(const float* __restrict__ x, int64_t n, int d, int k, int C,
                                                        int bf16, const int32_t* __restrict__ cand,
                                                        const float* __restrict__ tau, int32_t* __restrict__ out_idx,
                                                        double* __restrict__ out_d2, int32_t* __restrict__ fb_rows,
                                                        int32_t* __restrict__ fb_count,
                                                        unsigned long long* __restrict__ certified) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  int q = lane < C ? cand[row * C + lane] : INT32_MAX;
  double dist = INFINITY;
  if (q >= 0 && q < n) {
    const float* xp = x + row * d;
    const float* xq = x + (int64_t)q * d;
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
      float a = xp[j], b = xq[j];
      if (bf16) {
        a = bf16_round(a);
        b = bf16_round(b);
      }
      acc = sqdist_step(acc, (double)a, (double)b);
    }
    dist = acc;
  } else {
    q = INT32_MAX;
  }
  // bitonic sort of 64 (distance, index) pairs across the wave, ascending
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const double od = __shfl_xor(dist, stride);
      const int oq = __shfl_xor(q, stride);
      const bool lower = (lane & stride) == 0;
      const bool asc = (lane & size) == 0;
      const bool other_smaller = lex_less_d(od, oq, dist, q);
      if ((lower == asc) ? other_smaller : !other_smaller) {
        dist = od;
        q = oq;
      }
    }
  }
  if (lane < k) {
    out_idx[row * k + lane] = q;
    out_d2[row * k + lane] = dist;
  }
  const double dk = __shfl(dist, k - 1);
  const bool ok = dk < (double)tau[row];
  if (lane == 0) {
    if (ok) atomicAdd(certified, 1ull);
    else fb_rows[atomicAdd(fb_count, 1)] = (int32_t)row;
  }
}

}  // namespace

slk_status knn_mfma(const float* x, int64_t n, int32_t d, int32_t k, int32_t cand, int32_t bf16, int32_t* out_idx,
                    double* out_d2, int64_t* n_certified, int64_t* n_fallback, hipStream_t s) {
  const int C = std::min(std::max(cand, k), kMaxCand);
  const int dp = ((d + kDK - 1) / kDK) * kDK;
  Scratch sc(s);
  uint16_t *xh, *xl;
  float *nrm, *tau;
  double *mean, *part;
  int32_t *cidx, *fb_rows, *fb_count;
  unsigned long long* certified;
  const int nparts = (int)((n + kMeanRows - 1) / kMeanRows);
  SLK_TRY(sc.get(&xh, (size_t)n * dp));
  SLK_TRY(sc.get(&xl, (size_t)n * dp));
  SLK_TRY(sc.get(&nrm, n));
  SLK_TRY(sc.get(&tau, n));
  SLK_TRY(sc.get(&mean, d));
  SLK_TRY(sc.get(&part, (size_t)nparts * d));
  SLK_TRY(sc.get(&cidx, (size_t)n * C));
  SLK_TRY(sc.get(&fb_rows, n));
  SLK_TRY(sc.get(&fb_count, 1));
  SLK_TRY(sc.get(&certified, 1));
  SLK_HIP(hipMemsetAsync(fb_count, 0, sizeof(int32_t), s));
  SLK_HIP(hipMemsetAsync(certified, 0, sizeof(unsigned long long), s));
  if (!bf16) {
    hipLaunchKernelGGL(colsum_kernel, dim3((d + kBlock - 1) / kBlock, nparts), dim3(kBlock), 0, s, x, n, d, part);
    SLK_LAUNCHED("colsum_kernel");
    hipLaunchKernelGGL(colmean_kernel, dim3((d + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part, nparts, n, d, mean);
    SLK_LAUNCHED("colmean_kernel");
  }
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kBlock), 0, s, x, n, d, dp, mean, bf16, xh, xl,
                     nrm);
  SLK_LAUNCHED("split_kernel");
  // error constant of the lower bound (see the file comment): split residual + FP32
  // accumulation (32-term chunks, then dp/32 chunk sums) + final roundings, times 2
  const double u = std::ldexp(1.0, -24);
  const double terms = bf16 ? kDK : 3 * kDK;
  const double cG = (bf16 ? 0.0 : 3.05 * std::ldexp(1.0, -16)) + 1.01 * (terms + dp / kDK + 2) * u;
  const double c = 2.0 * (cG + 8 * u);
  const float c1 = (float)(1.0 - c);
  const unsigned grid = (unsigned)((n + kTile - 1) / kTile);
  {
    KernelTimer kt("cand_kernel", s);
    if (bf16)
      hipLaunchKernelGGL(cand_kernel<false>, dim3(grid), dim3(kBlock), 0, s, xh, xl, nrm, n, dp, C, c1, cidx, tau);
    else
      hipLaunchKernelGGL(cand_kernel<true>, dim3(grid), dim3(kBlock), 0, s, xh, xl, nrm, n, dp, C, c1, cidx, tau);
    SLK_LAUNCHED("cand_kernel");
  }
  {
    KernelTimer kt("rerank_kernel", s);
    hipLaunchKernelGGL(rerank_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kBlock), 0, s, x, n, d, k, C, bf16, cidx,
                       tau, out_idx, out_d2, fb_rows, fb_count, certified);
    SLK_LAUNCHED("rerank_kernel");
  }
  int32_t h_fb = 0;
  unsigned long long h_cert = 0;
  SLK_HIP(hipMemcpyAsync(&h_fb, fb_count, sizeof(h_fb), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipMemcpyAsync(&h_cert, certified, sizeof(h_cert), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  if (timing_on()) timing_flush();
  if (h_fb > 0) SLK_TRY(knn_exact(x, n, d, k, bf16, fb_rows, h_fb, out_idx, out_d2, s));
  SLK_HIP(hipStreamSynchronize(s));
  *n_certified = (int64_t)h_cert;
  *n_fallback = h_fb;
  return SLK_OK;
}

}  // namespace slk
