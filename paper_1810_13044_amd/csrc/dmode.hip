// Exact modes by their definition.  Eq. (1) takes each mode as the data point of largest
// z-weighted kernel density, and Eq. (10) adds a proximity term to the previous mode:
//   P[y, l] = sum_p z_pl k(x_p, x_y)  (+ k(x_y, x_{prev_l}) for Eq. (10)),   m_l = argmax_y P[y, l],
// over every point y, ties to the smaller index (Section 4.2: the start modes of SLK-BO follow
// Eq. (1) from the initial assignment).  This is a dense n x n x L kernel sum, done as two chained
// contractions on v_mfma_f32_32x32x16_bf16, an attention forward pass without normalisation:
//   S^T = X_tile Y^T              points x candidates; centred points split into bf16 hi + lo
//                                 (hi.hi + lo.hi + hi.lo, FP32 accumulation)
//   K^T = exp2(min(kscale (n_p + n_y - 2 S^T), 0)),   kscale = -log2(e) / (2 sigma^2)   (FP32,
//                                 v_exp_f32; bf16 conversions on v_cvt_pk_bf16_f32)
//   O^T += Z_tile^T K^T           clusters x candidates; K and Z split into bf16 hi + lo
// The accumulator of the first product holds, in lane t, candidate t % 32 and the points
// 8 (r / 4) + 4 (t / 32) + r % 4 of a 32-point block; that is the B-operand layout of the second
// product once its k index runs over the points in that order.  Z is staged in LDS in the same
// order, so the kernel values never leave registers.
//
// A work-group owns 128 candidates (32 per wave, their operands in registers for d <= 128);
// points stream past in tiles of 64, one 32-coordinate chunk at a time through a ring of three
// LDS buffers with one barrier per chunk.  The density of each candidate is summed in the MFMA
// accumulator over 16 tiles at a time, then added to a running FP32 total.  Each work-group
// writes per-cluster (best value, index) candidates; dm_reduce_kernel picks the maximum.
#include "common.h"

#include <math.h>

#include <algorithm>
#include <type_traits>
#include <vector>

namespace slk {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kBlock = 256;
constexpr int kQT = 128;        // candidates per work-group
constexpr int kPT = 64;         // points per tile
constexpr int kDK = 32;         // coordinates per staged chunk
constexpr int kRow = kDK + 8;   // bf16 per LDS row (16 bytes of padding)
constexpr int kFlush = 16;      // tiles summed in the MFMA accumulator before the running total
constexpr int kStage = kPT * kRow;

__device__ __forceinline__ bf16x8 gload8(const uint16_t* __restrict__ p) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, u);
}

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// RES: candidate operands resident for dp = 32 RES (1..4), 0 = reloaded per chunk.
// SPLIT: points carry a lo slice (FP32 points); LB: 32-cluster blocks; HARD: Z from labels.
template <int RES, bool SPLIT, int LB, bool HARD>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void dmode_kernel(
    const uint16_t* __restrict__ xh, const uint16_t* __restrict__ xl, const float* __restrict__ nrm, int64_t n,
    int dp, const float* __restrict__ z, const int32_t* __restrict__ lab, int L, float kscale,
    const float* __restrict__ prox, float* __restrict__ dens_out, float* __restrict__ cand_v,
    int32_t* __restrict__ cand_i, int grid) {
  // LDS: point ring [3][hi, lo][64][kRow] bf16 (at the end: per-wave best (value, index) per
  //      cluster) | Z^T operands [hi, lo][LB][4][64 lanes][8] bf16 | point norms [64] |
  //      running density totals [wave][16 LB][64 lanes] FP32
  __shared__ __attribute__((aligned(16))) uint16_t xst[3 * 2 * kStage];
  constexpr int kZ = LB * 4 * 64 * 8;
  __shared__ __attribute__((aligned(16))) uint16_t zst[(HARD ? 1 : 2) * kZ];
  __shared__ __attribute__((aligned(16))) float nst[kPT];
  __shared__ __attribute__((aligned(16))) int labs[kPT];
  __shared__ float tots[4 * 16 * LB * 64];
  static_assert(sizeof(float) * 4 * 64 * 2 <= sizeof(uint16_t) * 3 * 2 * kStage, "best lists fit in the ring");
  float(*wbv)[64] = reinterpret_cast<float(*)[64]>(xst);
  int(*wbi)[64] = reinterpret_cast<int(*)[64]>(xst + 4 * 64 * 2);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, col = lane & 31;
  const int64_t q0 = (int64_t)blockIdx.x * kQT + 32 * wave;
  const int nch = dp / kDK;
  const int64_t ntile = (n + kPT - 1) / kPT;
  const int64_t steps = ntile * nch;

  // candidate operands: row q0 + col, coordinates 16 s + 8 g .. + 7 of each chunk
  const int64_t yrow = min<int64_t>(q0 + col, n - 1);
  const uint16_t* yph = xh + yrow * dp + 8 * g;
  const uint16_t* ypl = xl + yrow * dp + 8 * g;
  const float kny = kscale * nrm[yrow];   // kscale n_y
  const float m2k = -2.f * kscale;
  constexpr int NA = RES > 0 ? RES : 1;
  bf16x8 bh[NA][2], bl[NA][2];
  if constexpr (RES > 0) {
#pragma unroll
    for (int c = 0; c < RES; ++c)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        bh[c][s2] = gload8(yph + kDK * c + 16 * s2);
        bl[c][s2] = SPLIT ? gload8(ypl + kDK * c + 16 * s2) : bh[c][s2];
      }
  }

  // staging of the point chunks: thread tid moves point spt (below), 8 coordinates at (tid % 4) * 8
  // point rows of a wave's lanes: 4 (l / 4 % 4) + l / 16, so that the lanes an LDS write serves at
  // once cover rows 4 apart, whose 80-byte rows fall on distinct banks (as in the kNN staging)
  const int spt = 16 * (tid >> 6) + 4 * ((tid >> 2) & 3) + ((tid >> 4) & 3), spiece = (tid & 3) * 8;
  const int svoff = 2 * (spt * dp + spiece);   // this thread's byte offset inside a tile of points
  uint4 ph = make_uint4(0, 0, 0, 0), pl = ph;
  // step positions (tile, chunk) and ring slots advance by counters: no divisions in the loop.
  // Every global load of the loop is a buffer load with no branch around it (zeros past the last
  // point), so the compiler waits only for the loads a step needs.
  auto fetch = [&](int64_t t, int c) __attribute__((always_inline)) {
    const int64_t p0 = t * kPT;
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(xh + p0 * dp, n - p0, kPT, 2 * dp);
    const __amdgpu_buffer_rsrc_t rl = rsrc_of(xl + p0 * dp, n - p0, kPT, 2 * dp);
    const int soff = __builtin_amdgcn_readfirstlane(2 * kDK * c);
    ph = bload16(rh, svoff, soff);
    pl = SPLIT ? bload16(rl, svoff, soff) : ph;
  };
  // RES == 0: the candidate operands of the next chunk are loaded one step ahead
  bf16x8 nbh[2], nbl[2];
  auto yfetch = [&](int c) __attribute__((always_inline)) {
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      nbh[s2] = gload8(yph + kDK * c + 16 * s2);
      nbl[s2] = SPLIT ? gload8(ypl + kDK * c + 16 * s2) : nbh[s2];
    }
  };
  auto stash = [&](int slot) __attribute__((always_inline)) {
    uint16_t* b = xst + slot * 2 * kStage;
    *reinterpret_cast<uint4*>(b + spt * kRow + spiece) = ph;
    if (SPLIT) *reinterpret_cast<uint4*>(b + kStage + spt * kRow + spiece) = pl;
  };

  // Z and norms of a tile.  The Z^T operand of the second product is LB x 4 x 64 slots of 8 bf16
  // (slot s = ((lb 4 + kc) 64 + lane): cluster 32 lb + lane % 32, points 16 kc + 8 (e / 4) +
  // 4 (lane / 32) + e % 4); each thread builds whole slots and writes them as 16 bytes.
  // Hard labels: thread tid < 64 loads the label of point tid of the next tile one step ahead,
  // stores it in `labs` at the tile's second chunk (after a barrier), and the slots read it from
  // there when the tile's Z is stashed (after the next barrier).
  constexpr int SPT = LB * 4 * 64 / kBlock;   // slots per thread
  // the next tile's raw values (labels, Z, norms), turned into operands where they are stashed;
  // every wave loads the tile's labels and norms (point tid % 64), wave 0 stashes them
  float zv[SPT][8];
  int lraw = 0;
  float nraw = 0.f;
  bool pok = false;   // point tid % 64 of the fetched tile exists
  auto zfetch = [&](int64_t t) __attribute__((always_inline)) {
    const int64_t p0 = t * kPT;
    if constexpr (HARD) {
      lraw = bloadi(rsrc_of(lab + p0, n - p0, kPT, 4), 4 * (tid & 63), 0);
    } else {
      const __amdgpu_buffer_rsrc_t rz = rsrc_of(z + p0 * L, n - p0, kPT, 4 * L);
#pragma unroll
      for (int i = 0; i < SPT; ++i) {
        const int sl = tid + kBlock * i;
        const int sln = sl & 63, kc = (sl >> 6) & 3, lb2 = sl >> 8;
        const int l = 32 * lb2 + (sln & 31), gg = sln >> 5;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int pl = 16 * kc + 8 * (e >> 2) + 4 * gg + (e & 3);
          // clusters past L read cluster L - 1 here and are zeroed where stashed
          zv[i][e] = bloadf(rz, 4 * (pl * L + min(l, L - 1)), 0);
        }
      }
    }
    nraw = bloadf(rsrc_of(nrm + p0, n - p0, kPT, 4), 4 * (tid & 63), 0);
    pok = p0 + (tid & 63) < n;
  };
  auto lstash = [&]() __attribute__((always_inline)) {
    if (HARD && tid < kPT) labs[tid] = pok ? lraw : -1;
  };
  auto zstash = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int sl = tid + kBlock * i;
      const int l = 32 * (sl >> 8) + (sl & 31);
      bf16x8 hi, lo;
      int lv[8];
      if constexpr (HARD) {
        const int kc = (sl >> 6) & 3, gg = (sl >> 5) & 1;
        const int4 a0 = *reinterpret_cast<const int4*>(labs + 16 * kc + 4 * gg);
        const int4 a1 = *reinterpret_cast<const int4*>(labs + 16 * kc + 8 + 4 * gg);
        lv[0] = a0.x; lv[1] = a0.y; lv[2] = a0.z; lv[3] = a0.w;
        lv[4] = a1.x; lv[5] = a1.y; lv[6] = a1.z; lv[7] = a1.w;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (HARD) {
          hi[e] = lv[e] == l ? (__bf16)1.0f : (__bf16)0.0f;
        } else {
          const float zz = l < L ? zv[i][e] : 0.f;
          hi[e] = (__bf16)zz;
          lo[e] = (__bf16)(zz - (float)hi[e]);
        }
      }
      *reinterpret_cast<bf16x8*>(zst + sl * 8) = hi;
      if constexpr (!HARD) *reinterpret_cast<bf16x8*>(zst + kZ + sl * 8) = lo;
    }
    if (tid < kPT) nst[tid] = pok ? kscale * nraw : -INFINITY;
  };

  f32x16 acc[2];
  f32x16 opart[LB];
  float* tw = tots + wave * 16 * LB * 64 + lane;   // this lane's totals, stride 64
#pragma unroll
  for (int lb = 0; lb < LB; ++lb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      opart[lb][r] = 0.f;
      tw[(16 * lb + r) * 64] = 0.f;
    }

  auto epilogue = [&](int64_t t) __attribute__((always_inline)) {
    // kernel values, split into bf16 hi + lo, packed as the B operands of the second product
    bf16x8 kh[2][2], kl[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      // kscale-scaled norms of this lane's points: rows 32 j + 8 q + 4 g + 0..3
      float nk[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = *reinterpret_cast<const float4*>(nst + 32 * j + 8 * q + 4 * g);
        nk[4 * q + 0] = v.x + kny;
        nk[4 * q + 1] = v.y + kny;
        nk[4 * q + 2] = v.z + kny;
        nk[4 * q + 3] = v.w + kny;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int r = 8 * h + e;
          // kscale * d^2 with d^2 = n_p + n_y - 2 S, clamped at d^2 >= 0 (kscale < 0)
          const float ex = fminf(fmaf(acc[j][r], m2k, nk[r]), 0.f);
          const float kv = __builtin_amdgcn_exp2f(ex);
          kh[j][h][e] = (__bf16)kv;
          kl[j][h][e] = (__bf16)(kv - (float)kh[j][h][e]);
        }
      }
    }
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int o = ((lb * 4 + kc) * 64 + lane) * 8;
        const bf16x8 za = *reinterpret_cast<const bf16x8*>(zst + o);
        opart[lb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, kh[kc >> 1][kc & 1], opart[lb], 0, 0, 0);
        opart[lb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(za, kl[kc >> 1][kc & 1], opart[lb], 0, 0, 0);
        if constexpr (!HARD) {
          const bf16x8 zb = *reinterpret_cast<const bf16x8*>(zst + kZ + o);
          opart[lb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(zb, kh[kc >> 1][kc & 1], opart[lb], 0, 0, 0);
        }
      }
    if ((t + 1) % kFlush == 0 || t + 1 == ntile) {
#pragma unroll
      for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          tw[(16 * lb + r) * 64] += opart[lb][r];
          opart[lb][r] = 0.f;
        }
    }
  };

  auto advance = [&](int64_t& tt, int& cc) __attribute__((always_inline)) {
    if (++cc == nch) {
      cc = 0;
      ++tt;
    }
  };
  // prologue: chunk 0 staged, chunk 1 and tile 0's Z in flight
  int64_t tf = 0;   // position of the next fetch
  int cf = 0;
  if constexpr (RES == 0) yfetch(0);
  fetch(tf, cf);
  zfetch(0);
  lstash();
  stash(0);
  advance(tf, cf);
  fetch(tf, cf);   // zeros past the last step
  int64_t t = 0;    // position of this step
  int c = 0;
  int slot = 0;     // ring slot of this step
  for (int64_t i = 0; i < steps; ++i) {
    __syncthreads();
    if (c == 0) {
      zstash();
    } else if (c == 1) {
      lstash();
    }
    // (past the last step: zeros into a ring slot nobody reads again)
    const int nslot = slot == 2 ? 0 : slot + 1;
    stash(nslot);
    bf16x8 cbh[2], cbl[2];
    if constexpr (RES == 0) {
      cbh[0] = nbh[0];
      cbh[1] = nbh[1];
      cbl[0] = nbl[0];
      cbl[1] = nbl[1];
      yfetch(c + 1 == nch ? 0 : c + 1);
    }
    advance(tf, cf);
    fetch(tf, cf);
    // the next tile's Z after this step's other loads, so that waiting for those (at the next
    // stash) is not a wait for these as well (past the last tile: zeros, never stashed)
    if (c == 0) zfetch(t + 1);
    if (c == 0) {
      acc[0] = f32x16{};
      acc[1] = f32x16{};
    }
    const uint16_t* b = xst + slot * 2 * kStage;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      bf16x8 yb, yl;
      if constexpr (RES > 0) {
        static_for<RES>([&](auto cc) __attribute__((always_inline)) {
          constexpr int C = decltype(cc)::value;
          if (c == C) {
            yb = bh[C][s2];
            yl = bl[C][s2];
          }
        });
      } else {
        yb = cbh[s2];
        yl = cbl[s2];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int o = (32 * j + col) * kRow + 16 * s2 + 8 * g;
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(b + o);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, yb, acc[j], 0, 0, 0);
        if constexpr (SPLIT) {
          const bf16x8 al = *reinterpret_cast<const bf16x8*>(b + kStage + o);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, yb, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, yl, acc[j], 0, 0, 0);
        }
      }
    }
    if (c == nch - 1) epilogue(t);
    slot = nslot;
    advance(t, c);
  }

  // per cluster: the best candidate of this wave, then of the work-group (the lists reuse the
  // point ring once every wave is past its last chunk)
  __syncthreads();
  const int64_t y = q0 + col;
#pragma unroll
  for (int lb = 0; lb < LB; ++lb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int l = 32 * lb + 8 * (r >> 2) + 4 * g + (r & 3);
      float v = tw[(16 * lb + r) * 64];
      const bool ok = y < n && l < L;
      if (ok && prox) v += prox[y * L + l];
      if (ok && dens_out) dens_out[y * L + l] = v;
      if (!ok) v = -INFINITY;
      int idx = ok ? (int)y : INT32_MAX;
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(idx, off);
        if (ov > v || (ov == v && oi < idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (col == 0) {
        wbv[wave][l] = v;
        wbi[wave][l] = idx;
      }
    }
  __syncthreads();
  if (tid < L) {
    float v = wbv[0][tid];
    int idx = wbi[0][tid];
    for (int w = 1; w < 4; ++w) {
      const float ov = wbv[w][tid];
      const int oi = wbi[w][tid];
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    cand_v[(int64_t)tid * grid + blockIdx.x] = v;
    cand_i[(int64_t)tid * grid + blockIdx.x] = idx;
  }
}

// one work-group per cluster: the largest value over the work-group candidates (ties to the
// smaller index)
__global__ __launch_bounds__(kBlock) void dm_reduce_kernel(const float* __restrict__ cv, const int32_t* __restrict__ ci,
                                                           int grid, int32_t* __restrict__ modes,
                                                           float* __restrict__ best) {
  __shared__ float sv[kBlock];
  __shared__ int si[kBlock];
  const int l = blockIdx.x, tid = threadIdx.x;
  float v = -INFINITY;
  int i = INT32_MAX;
  for (int b = tid; b < grid; b += kBlock) {
    const float ov = cv[(int64_t)l * grid + b];
    const int oi = ci[(int64_t)l * grid + b];
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  sv[tid] = v;
  si[tid] = i;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w && (sv[tid + w] > sv[tid] || (sv[tid + w] == sv[tid] && si[tid + w] < si[tid]))) {
      sv[tid] = sv[tid + w];
      si[tid] = si[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    modes[l] = si[0];
    best[l] = sv[0];
  }
}

// flag[l] = 1 if some point carries weight in cluster l (every writer stores the same value)
__global__ __launch_bounds__(kBlock) void dm_weight_kernel(const float* __restrict__ z, const int32_t* __restrict__ lab,
                                                           int64_t n, int L, int32_t* __restrict__ flag) {
  const int64_t total = lab ? n : n * L;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    if (lab) {
      const int l = lab[e];
      if (l >= 0 && l < L) flag[l] = 1;
    } else if (z[e] > 0.f) {
      flag[e % L] = 1;
    }
  }
}

template <int RES, bool SPLIT, int LB, bool HARD>
void launch_dmode(unsigned grid, hipStream_t s, const uint16_t* xh, const uint16_t* xl, const float* nrm, int64_t n,
                  int dp, const float* z, const int32_t* lab, int L, float kscale, const float* prox, float* dens,
                  float* cv, int32_t* ci) {
  hipLaunchKernelGGL((dmode_kernel<RES, SPLIT, LB, HARD>), dim3(grid), dim3(kBlock), 0, s, xh, xl, nrm, n, dp, z, lab,
                     L, kscale, prox, dens, cv, ci, (int)grid);
}

template <int RES, bool SPLIT>
slk_status dispatch_lb(int LB, bool hard, unsigned grid, hipStream_t s, const uint16_t* xh, const uint16_t* xl,
                       const float* nrm, int64_t n, int dp, const float* z, const int32_t* lab, int L, float kscale,
                       const float* prox, float* dens, float* cv, int32_t* ci) {
  if (LB == 1) {
    if (hard) launch_dmode<RES, SPLIT, 1, true>(grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
    else launch_dmode<RES, SPLIT, 1, false>(grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
  } else {
    if (hard) launch_dmode<RES, SPLIT, 2, true>(grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
    else launch_dmode<RES, SPLIT, 2, false>(grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
  }
  SLK_LAUNCHED("dmode_kernel");
  return SLK_OK;
}

template <bool SPLIT>
slk_status dispatch_res(int res, int LB, bool hard, unsigned grid, hipStream_t s, const uint16_t* xh,
                        const uint16_t* xl, const float* nrm, int64_t n, int dp, const float* z, const int32_t* lab,
                        int L, float kscale, const float* prox, float* dens, float* cv, int32_t* ci) {
  switch (res) {
    case 2: return dispatch_lb<2, SPLIT>(LB, hard, grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
    case 3: return dispatch_lb<3, SPLIT>(LB, hard, grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
    case 4: return dispatch_lb<4, SPLIT>(LB, hard, grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
    default: return dispatch_lb<0, SPLIT>(LB, hard, grid, s, xh, xl, nrm, n, dp, z, lab, L, kscale, prox, dens, cv, ci);
  }
}

}  // namespace
}  // namespace slk

using namespace slk;

extern "C" slk_status slk_dense_modes(const float* x, int64_t n, int32_t d, int32_t L, const float* z,
                                      const int32_t* labels, double sigma2, const int32_t* prev_host,
                                      const int32_t* keep_host, slk_precision prec, void* stream,
                                      int32_t* modes_out_host, float* best_out_host, float* dens_out) {
  SLK_TRY(check_points(x, n, d));
  if (L < 1 || L > 64 || L > n) return fail(SLK_ERR_INVALID_ARG, "L must satisfy 1 <= L <= min(64, n)");
  if ((z == nullptr) == (labels == nullptr)) return fail(SLK_ERR_INVALID_ARG, "pass exactly one of z and labels");
  if (!modes_out_host) return fail(SLK_ERR_INVALID_ARG, "modes_out_host is NULL");
  if (!(sigma2 > 0.0) || !isfinite(sigma2)) return fail(SLK_ERR_INVALID_ARG, "sigma2 must be finite and > 0");
  if (prec != SLK_PREC_FP32 && prec != SLK_PREC_BF16) return fail(SLK_ERR_INVALID_ARG, "unknown precision");
  if ((uint64_t)n * (uint64_t)L >= (1ull << 31)) return fail(SLK_ERR_INVALID_ARG, "n * L must be < 2^31");
  for (int l = 0; l < L; ++l) {
    if (prev_host && (prev_host[l] < 0 || prev_host[l] >= n)) return fail(SLK_ERR_INVALID_ARG, "prev out of range");
    if (keep_host && (keep_host[l] < 0 || keep_host[l] >= n)) return fail(SLK_ERR_INVALID_ARG, "keep out of range");
  }
  hipStream_t s = (hipStream_t)stream;
  const int bf16 = prec == SLK_PREC_BF16;
  // at least two chunks per tile (the Z stage is single-buffered across one barrier)
  const int dp = std::max(2 * kDK, ((d + kDK - 1) / kDK) * kDK);
  const unsigned grid = (unsigned)((n + kQT - 1) / kQT);
  Scratch sc(s);
  uint16_t *xh, *xl;
  float *nrm, *cv, *best, *prox = nullptr;
  double* mean;
  int32_t *ci, *modes, *flag, *prev_dev = nullptr;
  SLK_TRY(sc.get(&xh, (size_t)n * dp));
  SLK_TRY(sc.get(&xl, (size_t)n * dp));
  SLK_TRY(sc.get(&nrm, n));
  SLK_TRY(sc.get(&mean, d));
  SLK_TRY(sc.get(&cv, (size_t)grid * L));
  SLK_TRY(sc.get(&ci, (size_t)grid * L));
  SLK_TRY(sc.get(&modes, L));
  SLK_TRY(sc.get(&best, L));
  SLK_TRY(sc.get(&flag, L));
  SLK_TRY(split_points(x, n, d, dp, bf16, mean, xh, xl, nrm, s));
  std::vector<int32_t> ph;
  if (prev_host) {
    ph.assign(prev_host, prev_host + L);
    SLK_TRY(sc.get(&prev_dev, L));
    SLK_TRY(sc.get(&prox, (size_t)n * L));
    SLK_HIP(hipMemcpyAsync(prev_dev, ph.data(), sizeof(int32_t) * L, hipMemcpyHostToDevice, s));
    // proximity term k(x_y, x_{prev_l}): the unary kernel with the previous modes
    SLK_TRY(launch_unary(x, n, d, nullptr, prev_dev, L, L, sigma2, bf16, prox, nullptr, s));
  }
  const float kscale = (float)(-M_LOG2E / (2.0 * sigma2));
  const int res = dp <= 4 * kDK ? dp / kDK : 0;
  const int LB = L > 32 ? 2 : 1;
  const bool hard = labels != nullptr;
  {
    KernelTimer kt("dmode_kernel", s);
    if (bf16)
      SLK_TRY(dispatch_res<false>(res, LB, hard, grid, s, xh, xl, nrm, n, dp, z, labels, L, kscale, prox, dens_out,
                                  cv, ci));
    else
      SLK_TRY(dispatch_res<true>(res, LB, hard, grid, s, xh, xl, nrm, n, dp, z, labels, L, kscale, prox, dens_out, cv,
                                 ci));
  }
  hipLaunchKernelGGL(dm_reduce_kernel, dim3((unsigned)L), dim3(kBlock), 0, s, cv, ci, (int)grid, modes, best);
  SLK_LAUNCHED("dm_reduce_kernel");
  SLK_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t) * L, s));
  const int64_t total = labels ? n : n * L;
  const unsigned wgrid = (unsigned)std::min<int64_t>(1024, (total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(dm_weight_kernel, dim3(wgrid), dim3(kBlock), 0, s, z, labels, n, L, flag);
  SLK_LAUNCHED("dm_weight_kernel");
  std::vector<int32_t> mh(L), fh(L);
  std::vector<float> bh(L);
  SLK_HIP(hipMemcpyAsync(mh.data(), modes, sizeof(int32_t) * L, hipMemcpyDeviceToHost, s));
  SLK_HIP(hipMemcpyAsync(bh.data(), best, sizeof(float) * L, hipMemcpyDeviceToHost, s));
  SLK_HIP(hipMemcpyAsync(fh.data(), flag, sizeof(int32_t) * L, hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  for (int l = 0; l < L; ++l) {
    if (!fh[l]) {  // no weight: keep the given mode
      const int32_t* k = keep_host ? keep_host : prev_host;
      if (!k) return fail(SLK_ERR_INVALID_ARG, "a cluster has no weight and there is no mode to keep");
      mh[l] = k[l];
    }
    modes_out_host[l] = mh[l];
    if (best_out_host) best_out_host[l] = bh[l];
  }
  return SLK_OK;
}
