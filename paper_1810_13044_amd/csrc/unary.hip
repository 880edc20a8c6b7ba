// Unary affinities and the initial assignment (Eq. (6a) with the Gaussian kernel of Section 4.2,
// and the initialisation of Algorithm 1):
//   a_pl = exp(-||x_p - m_l||^2 / (2 sigma^2)),   z^0_p = softmax(a_p).
//
// A work-group owns R = 64 rows (32 when L > 128) in the internal order, gathered from the
// caller's order through the permutation.  Coordinates go through LDS 32 at a time, transposed
// (coordinate-major), with 16-byte loads when d is a multiple of 4; each thread computes a 4 x 4
// tile (4 rows x 4 modes) with FP32 direct differences, two 16-byte LDS reads and 16 multiply-adds
// per coordinate.  The squared distance is summed chunk by chunk (32 terms, then the chunk
// sums), which keeps the FP32 error small and avoids the cancellation of |x|^2 + |m|^2 - 2 x.m.
// The row softmax runs on 16 lanes per row with butterfly reductions.
#include "common.h"

#include <float.h>
#include <math.h>

namespace slk {
namespace {

constexpr int kBlock = 256;
constexpr int kUT = 4;       // rows and modes per thread tile
constexpr int kUTiles = 2;   // tiles per thread

template <int DC, bool VEC>
__device__ __forceinline__ void unary_block(const UnaryArgs& u, int64_t bid) {
  const float* __restrict__ x = u.x;
  const int64_t n = u.n;
  const int d = u.d, L = u.L, ldz = u.ldz, R = u.R, bf16 = u.bf16 == kUnaryRounded;
  const int32_t* __restrict__ perm = u.perm;
  const int32_t* __restrict__ modes = u.modes;
  const float inv2s2 = u.inv2s2;
  float* __restrict__ A = u.A;
  float* __restrict__ Z0 = u.Z0;
  const float* __restrict__ xm = u.xm ? u.xm : u.x;
  const float* __restrict__ mvec = u.mvec;
  extern __shared__ float sm[];
  const int MG = (L + kUT - 1) / kUT;
  const int RS = R + 4, MS = MG * kUT + 4;  // padded strides (multiples of 4 floats)
  float* xs = sm;                 // DC x RS, coordinate-major
  float* ms = xs + DC * RS;       // DC x MS
  float* as = sm;                 // R x L, written after the last chunk: shares the staging space
  const int tid = threadIdx.x;
  const int64_t row0 = bid * R;
  const int nr = (int)min<int64_t>(R, n - row0);
  const int ntiles = (R / kUT) * MG;
  float acc[kUTiles][kUT][kUT];
#pragma unroll
  for (int t = 0; t < kUTiles; ++t)
#pragma unroll
    for (int i = 0; i < kUT; ++i)
#pragma unroll
      for (int k = 0; k < kUT; ++k) acc[t][i][k] = 0.f;

  for (int c0 = 0; c0 < d; c0 += DC) {
    const int dc = min(DC, d - c0);
    if constexpr (VEC) {
      // 16-byte pieces: row r, coordinates 4 q .. 4 q + 3 of the chunk (dc is a multiple of 4)
      constexpr int Q = DC / 4;
      for (int e = tid; e < R * Q; e += kBlock) {
        const int r = e / Q, q = e % Q;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < nr && 4 * q < dc) {
          const int64_t gr = perm ? perm[row0 + r] : row0 + r;
          v = *reinterpret_cast<const float4*>(x + gr * d + c0 + 4 * q);
        }
        if (bf16) {
          v.x = bf16_round(v.x);
          v.y = bf16_round(v.y);
          v.z = bf16_round(v.z);
          v.w = bf16_round(v.w);
        }
        xs[(4 * q + 0) * RS + r] = v.x;
        xs[(4 * q + 1) * RS + r] = v.y;
        xs[(4 * q + 2) * RS + r] = v.z;
        xs[(4 * q + 3) * RS + r] = v.w;
      }
      for (int e = tid; e < MG * kUT * Q; e += kBlock) {
        const int l = e / Q, q = e % Q;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (l < L && 4 * q < dc)
          v = *reinterpret_cast<const float4*>((mvec ? mvec + (int64_t)l * d : xm + (int64_t)modes[l] * d) + c0 + 4 * q);
        if (bf16 && !mvec) {  // mode vectors are computed in FP32 and used as they are
          v.x = bf16_round(v.x);
          v.y = bf16_round(v.y);
          v.z = bf16_round(v.z);
          v.w = bf16_round(v.w);
        }
        ms[(4 * q + 0) * MS + l] = v.x;
        ms[(4 * q + 1) * MS + l] = v.y;
        ms[(4 * q + 2) * MS + l] = v.z;
        ms[(4 * q + 3) * MS + l] = v.w;
      }
    } else {
      for (int e = tid; e < R * DC; e += kBlock) {
        const int r = e / DC, j = e % DC;
        float v = 0.f;
        if (r < nr && j < dc) {
          const int64_t gr = perm ? perm[row0 + r] : row0 + r;
          v = x[gr * d + c0 + j];
          if (bf16) v = bf16_round(v);
        }
        xs[j * RS + r] = v;
      }
      for (int e = tid; e < MG * kUT * DC; e += kBlock) {
        const int l = e / DC, j = e % DC;
        float v = 0.f;
        if (l < L && j < dc) {
          v = mvec ? mvec[(int64_t)l * d + c0 + j] : xm[(int64_t)modes[l] * d + c0 + j];
          if (bf16 && !mvec) v = bf16_round(v);
        }
        ms[j * MS + l] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kUTiles; ++t) {
      const int tile = tid + t * kBlock;
      if (tile < ntiles) {
        const int rg = tile / MG, mg = tile % MG;
        float part[kUT][kUT];
#pragma unroll
        for (int i = 0; i < kUT; ++i)
#pragma unroll
          for (int k = 0; k < kUT; ++k) part[i][k] = 0.f;
#pragma unroll 8
        for (int j = 0; j < DC; ++j) {
          const float4 xv = *reinterpret_cast<const float4*>(xs + j * RS + rg * kUT);
          const float4 mv = *reinterpret_cast<const float4*>(ms + j * MS + mg * kUT);
          const float xa[4] = {xv.x, xv.y, xv.z, xv.w};
          const float ma[4] = {mv.x, mv.y, mv.z, mv.w};
#pragma unroll
          for (int i = 0; i < kUT; ++i)
#pragma unroll
            for (int k = 0; k < kUT; ++k) {
              const float df = xa[i] - ma[k];
              part[i][k] = fmaf(df, df, part[i][k]);
            }
        }
#pragma unroll
        for (int i = 0; i < kUT; ++i)
#pragma unroll
          for (int k = 0; k < kUT; ++k) acc[t][i][k] += part[i][k];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < kUTiles; ++t) {
    const int tile = tid + t * kBlock;
    if (tile < ntiles) {
      const int rg = tile / MG, mg = tile % MG;
#pragma unroll
      for (int i = 0; i < kUT; ++i)
#pragma unroll
        for (int k = 0; k < kUT; ++k) {
          const int l = mg * kUT + k;
          if (l < L) as[(rg * kUT + i) * L + l] = expf(-acc[t][i][k] * inv2s2);
        }
    }
  }
  __syncthreads();
  // row softmax of a_p gives z^0_p: 16 lanes per row, 16 rows per block pass
  const int g = tid >> 4, j = tid & 15;
  for (int r = g; r < nr; r += kBlock / 16) {
    float m = -FLT_MAX;
    for (int l = j; l < L; l += 16) m = fmaxf(m, as[r * L + l]);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 16));
    float s = 0.f;
    for (int l = j; l < L; l += 16) s += expf(as[r * L + l] - m);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    const int64_t row = row0 + r;
    for (int l = j; l < ldz; l += 16) {
      const float a = l < L ? as[r * L + l] : 0.f;
      if (A) A[row * ldz + l] = a;
      if (Z0) Z0[row * ldz + l] = l < L ? expf(a - m) / s : 0.f;
    }
  }
}

template <int DC, bool VEC>
__global__ __launch_bounds__(kBlock) void unary_kernel(UnaryArgs u) {
  unary_block<DC, VEC>(u, blockIdx.x);
}

// ------------------------------------------------------------------------------------------
// BF16-X: the distance contraction on MFMA (u.bf16 == kUnaryMfma)
// ------------------------------------------------------------------------------------------
// ||x_p - m_l||^2 = ||y_p||^2 + ||w_l||^2 - 2 y_p.w_l with y = x - c, w = m - c for a reference
// point c: the first row of the wave's tile of 32 rows.  With the locality order a tile's rows are
// neighbours, so |y| is of the order of the within-cluster spread rather than of |x|, and the
// cancellation of the expansion stays small.  y and w are split into three bf16 terms
// (h = bf16(v), m = bf16(v - h), l = bf16(v - h - m), each conversion rounding to nearest even;
// |v - h - m - l| <= 2^-27 |v|), and y.w = h.h + h.m + m.h + h.l + l.h + m.m on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (the dropped products and the residuals are at
// most 3 * 2^-27 |y_j| |w_j| per coordinate, below the accumulation's own rounding).  The norms
// are FP32 sums of y^2 and w^2.
// A wave owns 32 rows and all modes (padded to T tiles of 32): for each 16 coordinates every
// lane loads the 8 it feeds to the MFMA (row col of the tile and mode 32 t + col, coordinates
// 8 half .. 8 half + 7), centres and splits them in registers; no LDS, no barrier.  The row
// softmax runs on the accumulators: for row 8 (r / 4) + 4 half + r % 4 the 32 lanes of one half
// hold modes 32 t + col, reduced with butterfly shuffles.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kXRows = 128;   // rows per work-group (32 per wave)

// v = h + m + l (+ residual), three bf16 vectors; returns sum v^2
__device__ __forceinline__ float split8(const float (&v)[8], bf16x8& h, bf16x8& m, bf16x8& l) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float x = v[i];
    h[i] = (__bf16)x;
    const float r1 = x - (float)h[i];
    m[i] = (__bf16)r1;
    l[i] = (__bf16)(r1 - (float)m[i]);
    s += x * x;
  }
  return s;
}

// 8 coordinates k0 .. k0 + 7 of a row (zeros past d)
template <bool VEC>
__device__ __forceinline__ void load8(const float* __restrict__ row, int k0, int d, float (&v)[8]) {
  if (VEC && k0 + 8 <= d) {
    const float4 a = *reinterpret_cast<const float4*>(row + k0);
    const float4 b = *reinterpret_cast<const float4*>(row + k0 + 4);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = b.x;
    v[5] = b.y;
    v[6] = b.z;
    v[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = k0 + i < d ? row[k0 + i] : 0.f;
  }
}

template <int T, bool VEC>
__device__ __forceinline__ void unary_mfma_block(const UnaryArgs& u, int64_t bid) {
  const int64_t n = u.n;
  const int d = u.d, L = u.L, ldz = u.ldz;
  const int32_t* __restrict__ perm = u.perm;
  const float* __restrict__ xm = u.xm ? u.xm : u.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
  const int64_t t0 = bid * kXRows + 32 * wave;  // the wave's first row (internal order)
  if (t0 >= n) return;                          // the whole wave leaves together
  const int nr = (int)min<int64_t>(32, n - t0);
  const float* cref = u.x + (perm ? perm[t0] : t0) * (int64_t)d;
  const float* xr = u.x + (perm ? perm[t0 + min(col, nr - 1)] : t0 + min(col, nr - 1)) * (int64_t)d;
  const float* mr[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int l = 32 * t + col;
    mr[t] = l < L ? (u.mvec ? u.mvec + (int64_t)l * d : xm + (int64_t)u.modes[l] * d) : nullptr;
  }
  f32x16 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = f32x16{};
  float ny = 0.f, nw[T];
#pragma unroll
  for (int t = 0; t < T; ++t) nw[t] = 0.f;
  // the trip count is the same for both halves (every lane takes part in every MFMA); the
  // coordinates past d load as zeros
  for (int k = 0; k < d; k += 16) {
    const int k0 = k + 8 * half;
    float c[8], v[8];
    load8<VEC>(cref, k0, d, c);
    load8<VEC>(xr, k0, d, v);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = col < nr ? v[i] - c[i] : 0.f;
    bf16x8 ah, am, al;
    ny += split8(v, ah, am, al);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      float w[8];
      if (mr[t]) {
        load8<VEC>(mr[t], k0, d, w);
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] -= c[i];
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = 0.f;
      }
      bf16x8 bh, bm, bl;
      nw[t] += split8(w, bh, bm, bl);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc[t], 0, 0, 0);
    }
  }
  // the two halves hold coordinates 16 s + 0..7 and 16 s + 8..15: add the partner's share
  ny += __shfl_xor(ny, 32);
#pragma unroll
  for (int t = 0; t < T; ++t) nw[t] += __shfl_xor(nw[t], 32);
  // accumulator entry r of lane (half, col): row 8 (r / 4) + 4 half + r % 4, mode 32 t + col
  float a[T][16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r >> 2) + 4 * half + (r & 3);
    const float nyr = __shfl(ny, row);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float d2 = fmaxf(nyr + nw[t] - 2.f * acc[t][r], 0.f);
      a[t][r] = 32 * t + col < L ? expf(-d2 * u.inv2s2) : -INFINITY;
    }
  }
  // row softmax: max and sum over the modes of each row (registers, then the 32 lanes of a half)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float m = a[0][r];
#pragma unroll
    for (int t = 1; t < T; ++t) m = fmaxf(m, a[t][r]);
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 32));
    float e[T], sum = 0.f;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      e[t] = 32 * t + col < L ? expf(a[t][r] - m) : 0.f;
      sum += e[t];
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 32);
    const int row = 8 * (r >> 2) + 4 * half + (r & 3);
    if (row < nr) {
      const int64_t orow = t0 + row;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int l = 32 * t + col;
        if (l < ldz) {
          const bool ok = l < L;
          if (u.A) u.A[orow * ldz + l] = ok ? a[t][r] : 0.f;
          if (u.Z0) u.Z0[orow * ldz + l] = ok ? e[t] / sum : 0.f;
        }
      }
    }
  }
}

template <int T, bool VEC>
__global__ __launch_bounds__(kBlock) void unary_mfma_kernel(UnaryArgs u) {
  unary_mfma_block<T, VEC>(u, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void unary_packed(const UnaryArgs* __restrict__ jobs,
                                                       const int32_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const UnaryArgs& u = jobs[j];
  // 16-byte staging when the job's rows allow it (d % 4 == 0, x 16-byte aligned)
  const bool vec = (u.d & 3) == 0 && ((uintptr_t)u.x & 15) == 0 && ((uintptr_t)(u.xm ? u.xm : u.x) & 15) == 0 &&
                   ((uintptr_t)u.mvec & 15) == 0;
  const int64_t b = (int64_t)blockIdx.x - start[j];
  if (u.bf16 == kUnaryMfma) {
    if (vec) unary_mfma_block<2, true>(u, b);
    else unary_mfma_block<2, false>(u, b);
  } else if (vec) {
    unary_block<32, true>(u, b);
  } else {
    unary_block<32, false>(u, b);
  }
}

}  // namespace

UnaryArgs unary_args(const float* x, int64_t n, int32_t d, const int32_t* perm, const int32_t* modes_dev, int32_t L,
                     int32_t ldz, double sigma2, int32_t bf16, float* A, float* Z0) {
  UnaryArgs u{};
  u.x = x;
  u.n = n;
  u.d = d;
  u.L = L;
  u.ldz = ldz;
  u.R = bf16 == kUnaryMfma ? kXRows : L <= 128 ? 64 : 32;
  u.perm = perm;
  u.modes = modes_dev;
  u.inv2s2 = (float)(1.0 / (2.0 * sigma2));
  u.bf16 = bf16;
  u.A = A;
  u.Z0 = Z0;
  return u;
}

int unary_grid(const UnaryArgs& u) { return (int)((u.n + u.R - 1) / u.R); }

size_t unary_lds(const UnaryArgs& u) {
  if (u.bf16 == kUnaryMfma) return 0;
  const int DC = u.L <= 128 ? 32 : 16;
  const int MG = (u.L + kUT - 1) / kUT;
  const size_t staging = (size_t)DC * (u.R + 4) + (size_t)DC * (MG * kUT + 4);
  return sizeof(float) * std::max(staging, (size_t)u.R * u.L);
}

// 16-byte loads need d % 4 == 0 (rows then start on 16-byte boundaries of a 16-byte aligned x).
static bool vec_ok(const UnaryArgs& u) {
  return (u.d & 3) == 0 && ((uintptr_t)u.x & 15) == 0 && ((uintptr_t)(u.xm ? u.xm : u.x) & 15) == 0 &&
         ((uintptr_t)u.mvec & 15) == 0;
}

slk_status launch_unary(const float* x, int64_t n, int32_t d, const int32_t* perm, const int32_t* modes_dev, int32_t L,
                        int32_t ldz, double sigma2, int32_t bf16, float* A, float* Z0, hipStream_t s,
                        const float* xm, const float* mvec) {
  UnaryArgs u = unary_args(x, n, d, perm, modes_dev, L, ldz, sigma2, bf16, A, Z0);
  u.xm = xm;
  u.mvec = mvec;
  const size_t lds = unary_lds(u);
  const dim3 grid((unsigned)unary_grid(u));
  const bool vec = vec_ok(u);
  if (bf16 == kUnaryMfma) {
#define SLK_UNARY_MFMA(T_)                                                                         \
  do {                                                                                             \
    if (vec) hipLaunchKernelGGL((unary_mfma_kernel<T_, true>), grid, dim3(kBlock), 0, s, u);       \
    else hipLaunchKernelGGL((unary_mfma_kernel<T_, false>), grid, dim3(kBlock), 0, s, u);          \
  } while (0)
    if (L <= 32) SLK_UNARY_MFMA(1);
    else if (L <= 64) SLK_UNARY_MFMA(2);
    else if (L <= 128) SLK_UNARY_MFMA(4);
    else SLK_UNARY_MFMA(8);
#undef SLK_UNARY_MFMA
  } else if (L <= 128) {
    if (vec) hipLaunchKernelGGL((unary_kernel<32, true>), grid, dim3(kBlock), lds, s, u);
    else hipLaunchKernelGGL((unary_kernel<32, false>), grid, dim3(kBlock), lds, s, u);
  } else {
    if (vec) hipLaunchKernelGGL((unary_kernel<16, true>), grid, dim3(kBlock), lds, s, u);
    else hipLaunchKernelGGL((unary_kernel<16, false>), grid, dim3(kBlock), lds, s, u);
  }
  SLK_LAUNCHED("unary_kernel");
  return SLK_OK;
}

// Packed jobs all have L <= 64, so DC = 32 and R = 64 for every one.
slk_status launch_unary_packed(const UnaryArgs* jobs, const int32_t* start, int njobs, int blocks, size_t lds,
                               hipStream_t s) {
  hipLaunchKernelGGL(unary_packed, dim3((unsigned)blocks), dim3(kBlock), lds, s, jobs, start, njobs);
  SLK_LAUNCHED("unary_packed");
  return SLK_OK;
}

}  // namespace slk
