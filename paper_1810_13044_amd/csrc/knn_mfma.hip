// Exact kNN (Section 4.2) at scale: candidates from a bf16 MFMA Gram matrix, exact FP64 re-rank,
// and a certificate that the exact top-k lies among the candidates.
//
//   1. centre_split: y = x - mean(x) in FP64, split y = h + l with h = bf16(y), l = bf16(y - h)
//      (|y - h - l| <= ~2^-16 |y|); row norms n_p = ||y_p||^2 in FP64.  With bf16 points
//      (SLK_PREC_BF16) the points are bf16(x) themselves: h = bf16(x), l = 0, no centring.
//   2. cand_kernel: G~ = h_p.h_q + h_p.l_q + l_p.h_q on v_mfma_f32_32x32x16_bf16 with FP32
//      accumulation (one accumulator for d <= 128; above, a fresh one per 32 coordinates, then
//      summed).  For every pair a
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
#include <type_traits>
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
// Column sums over blocks of rows (at most kMeanParts blocks, at least kMeanMinRows rows each),
// then the block sums in order.  Each sum runs in row order; its loads are issued 8 at a time so
// that they are in flight together (one dependent load per row had left a 50k-point build with
// 25 work-groups waiting on memory for 0.6 ms).
constexpr int kMeanParts = 1024;
constexpr int64_t kMeanMinRows = 256;
inline int64_t mean_rows(int64_t n) { return std::max<int64_t>(kMeanMinRows, (n + kMeanParts - 1) / kMeanParts); }
inline int mean_parts(int64_t n) { return (int)((n + mean_rows(n) - 1) / mean_rows(n)); }

__global__ __launch_bounds__(kBlock) void colsum_kernel(const float* __restrict__ x, int64_t n, int d, int64_t rows,
                                                        double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.y * rows;
  const int64_t r1 = min<int64_t>(n, r0 + rows);
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < d; j += gridDim.x * kBlock) {
    double s = 0.0;
    int64_t r = r0;
    for (; r + 8 <= r1; r += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = x[(r + u) * d + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; r < r1; ++r) s += (double)x[r * d + j];
    part[(int64_t)blockIdx.y * d + j] = s;
  }
}

__global__ __launch_bounds__(kBlock) void colmean_kernel(const double* __restrict__ part, int nparts, int64_t n, int d,
                                                         double* __restrict__ mean) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  int b = 0;
  for (; b + 8 <= nparts; b += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u) * d + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < nparts; ++b) s += part[(int64_t)b * d + j];
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
// The value of lane (lane ^ stride): DPP within a row for strides 1 and 2 (quad permutations) and
// 4 and 8 (the row shifted up or down, chosen per lane); the LDS crossbar (__shfl_xor) beyond.
// stride is a constant wherever this is inlined into an unrolled loop.
__device__ __forceinline__ int xor_lane(int x, int stride) {
  if (stride == 1) return __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  if (stride == 2) return __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  if (stride == 4) {
    const int up = __builtin_amdgcn_update_dpp(x, x, 0x104, 0xf, 0xf, false);  // row_shl:4, lane + 4
    const int dn = __builtin_amdgcn_update_dpp(x, x, 0x114, 0xf, 0xf, false);  // row_shr:4, lane - 4
    return (threadIdx.x & 4) ? dn : up;
  }
  if (stride == 8) {
    const int up = __builtin_amdgcn_update_dpp(x, x, 0x108, 0xf, 0xf, false);  // row_shl:8, lane + 8
    const int dn = __builtin_amdgcn_update_dpp(x, x, 0x118, 0xf, 0xf, false);  // row_shr:8, lane - 8
    return (threadIdx.x & 8) ? dn : up;
  }
  return __shfl_xor(x, stride);
}

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
          const float ov = __builtin_bit_cast(float, xor_lane(__builtin_bit_cast(int, v[s]), stride));
          const int oi = xor_lane(ix[s], stride);
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

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  bf16x8 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

__device__ __forceinline__ bf16x8 gload8(const uint16_t* __restrict__ p) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, u);
}

// Key rows, key norms and query norms reach the scan through buffer loads (rsrc_of, common.h):
// with no branch around a load the compiler can count the loads in flight and wait only for the
// oldest ones; a branch around a load had made it drain every load (and so the two-stage
// prefetch) at each step.

// Candidate search.  A work-group owns kQT = 128 query rows, 32 per wave; keys stream past in
// tiles of kKT = 64, one 32-coordinate chunk at a time through an LDS stage (one barrier per
// chunk).  For d <= 128 a stage holds two tiles (128 keys) and a wave multiplies its 32 rows by
// them as four 32 x 32 MFMA tiles, 24 MFMAs between barriers with the bf16 split; above, one tile
// per stage.  The query operands (bf16 hi and lo slices) stay in registers for the whole scan
// when d <= 32 RES, else they are loaded with each chunk.  Each wave keeps the C best lower
// bounds of each of its rows, sorted by (bound, index), in its own part of LDS, so candidate
// merges need no barrier: a row with a few new candidates inserts them one by one, a row with
// many merges them with a 128-wide bitonic sort.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

constexpr int kQT = 128;
constexpr int kKT = 64;
// More new candidates than this (of a row in a tile) go through the 128-wide bitonic merge; fewer
// are inserted one by one.  Measured with the inserts on DPP shifts (64 = always insert, a tile
// holding 64 keys): always inserting is fastest for d <= 96 and for the long-scan form; for the
// row-by-row form at 97 <= d <= 128 it was slower (300,000 x 128: 93 -> 108 ms), 16 stays there;
// above d = 128, 32.
template <int RES, bool FAST>
constexpr int bulk_above() { return RES == 0 ? 32 : (RES == 4 && !FAST) ? 16 : 64; }

// Insert (v, key) into the sorted list of one row held in registers: lane i < C holds entry i
// (cv, ci), lanes from C on hold (+inf, INT32_MAX).  A run of inserts reads the list from LDS once
// and writes it back once (list_load, list_store): an LDS round trip per insert had made the
// inserts the bulk of a short scan.
// Lane i gets lane i - 1's value (lane 0 its own): the DPP whole-wave shift (wave_shr:1), one
// VALU operation; __shfl_up went through the LDS crossbar (ds_bpermute) and its latency.
__device__ __forceinline__ int wave_shr1(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x138, 0xf, 0xf, false); }

__device__ __forceinline__ void list_insert(float& cv, int& ci, int C, float v, int key) {
  const int lane = threadIdx.x & 63;
  // (cv, ci) < (v, key), without branches
  const bool before = (lane < C) & ((cv < v) | ((cv == v) & (ci < key)));
  const int pos = __popcll(__ballot(before));
  const float pv = __builtin_bit_cast(float, wave_shr1(__builtin_bit_cast(int, cv)));
  const int pi = wave_shr1(ci);
  const bool move = (pos < C) & (lane < C) & (lane >= pos);
  cv = move ? (lane == pos ? v : pv) : cv;
  ci = move ? (lane == pos ? key : pi) : ci;
}

__device__ __forceinline__ void list_load(const float* lv, const int* li, int C, float& cv, int& ci) {
  const int lane = threadIdx.x & 63;
  cv = lane < C ? lv[lane] : INFINITY;
  ci = lane < C ? li[lane] : INT32_MAX;
}

// writes the list back and returns its C-th bound
__device__ __forceinline__ float list_store(float* lv, int* li, int C, float cv, int ci) {
  const int lane = threadIdx.x & 63;
  if (lane < C) {
    lv[lane] = cv;
    li[lane] = ci;
  }
  return __shfl(cv, C - 1);
}

// Two waves per SIMD (at most 256 registers per lane): the scan is latency-bound below that.
template <int RES>
constexpr int cand_tiles() { return RES > 0 ? 2 : 1; }   // 64-key tiles per LDS stage
template <int RES>
constexpr int cand_ring() { return RES > 0 ? 2 : 3; }    // LDS stages in the ring

template <bool SPLIT, int RES, bool FAST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void cand_kernel(
    const uint16_t* __restrict__ xh, const uint16_t* __restrict__ xl, const float* __restrict__ nrm, int64_t n, int dp,
    int C, float c1, int32_t* __restrict__ cand, float* __restrict__ tau_out, const uint16_t* __restrict__ qh,
    const uint16_t* __restrict__ ql, const float* __restrict__ qn, int64_t nq, int self) {
  constexpr int P = cand_tiles<RES>();       // tiles per stage
  constexpr int NJ = 2 * P;                  // 32-key MFMA column tiles per stage
  constexpr int RING = cand_ring<RES>();
  extern __shared__ unsigned char smraw[];
  // key stage ring: [RING][hi/lo][key][kRow] bf16, then the candidate lists [wave][row][C]
  uint16_t* kst = reinterpret_cast<uint16_t*>(smraw);
  constexpr int kStage = P * kKT * kRow;  // bf16 per array
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  float* lvw = reinterpret_cast<float*>(smraw + sizeof(uint16_t) * 2 * RING * kStage) + wave * 32 * C;
  int* liw = reinterpret_cast<int*>(smraw + sizeof(uint16_t) * 2 * RING * kStage + sizeof(float) * 4 * 32 * C) +
             wave * 32 * C;
  const int64_t q0 = (int64_t)blockIdx.x * kQT + 32 * wave;
  const int nch = RES > 0 ? RES : dp / kDK;
  for (int e = lane; e < 32 * C; e += 64) {
    lvw[e] = INFINITY;
    liw[e] = INT32_MAX;
  }
  // this lane's rows (accumulator r): 8 (r / 4) + 4 half + r % 4; qv = c1 |y_q|^2, tau = C-th bound
  float qv[16], tau[16];
  {
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(qn + q0, nq - q0, 32, 4);   // zero past the last query
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      qv[r] = __fmul_rn(c1, bloadf(rq, 4 * (4 * half), 4 * (8 * (r >> 2) + (r & 3))));
      tau[r] = INFINITY;
    }
  }
  // query operands: row q0 + col, coordinates 16 s + 8 half .. + 7 of each chunk
  const int64_t arow = min<int64_t>(q0 + col, nq - 1);
  const uint16_t* aph = qh + arow * dp + 8 * half;
  const uint16_t* apl = ql + arow * dp + 8 * half;
  constexpr int NA = RES > 0 ? RES : 1;
  bf16x8 ah[NA][2], al[NA][2];
  if constexpr (RES > 0) {
#pragma unroll
    for (int c = 0; c < RES; ++c)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        ah[c][s2] = gload8(aph + kDK * c + 16 * s2);
        al[c][s2] = SPLIT ? gload8(apl + kDK * c + 16 * s2) : ah[c][s2];
      }
  }
  // staging: thread tid moves keys skey + 64 t (t < P), 8 coordinates at (tid % 4) * 8, hi and
  // lo, through two register slots (loads in flight two chunks ahead) into the LDS ring
  // key rows of a wave's lanes: 4 (l / 4 % 4) + l / 16 (the four pieces of a row in four adjacent
  // lanes), so that the 8 (or 16) lanes an LDS write serves at once cover rows 4 (or 12) apart,
  // whose 80-byte rows fall on distinct banks; rows in order had every write two-way conflicted
  const int skey = 16 * (tid >> 6) + 4 * ((tid >> 2) & 3) + ((tid >> 4) & 3), spiece = (tid & 3) * 8;
  const int svoff = 2 * (skey * dp + spiece);   // this thread's byte offset inside a key stage
  const int64_t nkt = (n + kKT - 1) / kKT;
  const int64_t nst = (nkt + P - 1) / P;   // stages of keys
  const int64_t steps = nst * nch;
  uint4 ph[2][P], pl[2][P];
  bf16x8 sah[2][2], sal[2][2];  // query operands in flight (RES == 0)
  // positions (stage st, chunk c) and ring slots are passed in: no divisions by the runtime
  // chunk count in the loop
  auto fetch = [&](auto slot_c, int64_t st, int c) __attribute__((always_inline)) {
    constexpr int SL = decltype(slot_c)::value;
    // the stage's key rows; past the last key (or past the last stage) the loads return zeros
    const int64_t r0 = st * (P * kKT);
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(xh + r0 * dp, n - r0, P * kKT, 2 * dp);
    const __amdgpu_buffer_rsrc_t rl = rsrc_of(xl + r0 * dp, n - r0, P * kKT, 2 * dp);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const int soff = __builtin_amdgcn_readfirstlane(2 * (kKT * t * dp + kDK * c));
      ph[SL][t] = bload16(rh, svoff, soff);
      pl[SL][t] = SPLIT ? bload16(rl, svoff, soff) : ph[SL][t];
    }
    if constexpr (RES == 0) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        sah[SL][s2] = gload8(aph + kDK * c + 16 * s2);
        sal[SL][s2] = SPLIT ? gload8(apl + kDK * c + 16 * s2) : sah[SL][s2];
      }
    }
  };
  auto stash = [&](auto slot_c, int ring) __attribute__((always_inline)) {
    constexpr int SL = decltype(slot_c)::value;
    uint16_t* b = kst + ring * 2 * kStage;
#pragma unroll
    for (int t = 0; t < P; ++t) {
      *reinterpret_cast<uint4*>(b + (kKT * t + skey) * kRow + spiece) = ph[SL][t];
      if (SPLIT) *reinterpret_cast<uint4*>(b + kStage + (kKT * t + skey) * kRow + spiece) = pl[SL][t];
    }
    if constexpr (RES == 0) {
      ah[0][0] = sah[SL][0];
      ah[0][1] = sah[SL][1];
      al[0][0] = sal[SL][0];
      al[0][1] = sal[SL][1];
    }
  };
  f32x16 tot[NJ], part[NJ];
  float nk[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) nk[j] = 0.f;
  // Merge of row r (accumulator entry r of this lane; one row per lane half) with the tile's
  // bounds lb (keys k0 + 32 j + col): the candidates below the row's C-th bound tr enter its list;
  // returns the row's new C-th bound (for this lane's half).
  auto merge_row = [&](int r, int64_t k0, const float (&lb)[2], float tr) __attribute__((always_inline)) {
    const uint64_t m0 = __ballot(lb[0] < tr), m1 = __ballot(lb[1] < tr);
    if ((m0 | m1) == 0ull) return tr;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t b0 = (uint32_t)(m0 >> (32 * h)), b1 = (uint32_t)(m1 >> (32 * h));
      const int cnt = __popc(b0) + __popc(b1);
      if (cnt == 0) continue;
      const int rho = 8 * (r >> 2) + 4 * h + (r & 3);
      float* lv = lvw + rho * C;
      int* li = liw + rho * C;
      float nt;
      if (cnt <= bulk_above<RES, FAST>()) {
        float cv;
        int ci;
        list_load(lv, li, C, cv, ci);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          uint32_t bb = j == 0 ? b0 : b1;
          while (bb) {
            const int bit = __builtin_ctz(bb);
            bb &= bb - 1;
            const float v =
                __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, lb[j]), 32 * h + bit));
            list_insert(cv, ci, C, v, (int)(k0 + 32 * j + bit));
          }
        }
        nt = list_store(lv, li, C, cv, ci);
      } else {
        // the row's 64 bounds of this tile: lanes 0-31 keys k0 .. k0+31, lanes 32-63 the rest
        const int src = 32 * h + col;
        const float v0 = __shfl(lb[0], src), v1 = __shfl(lb[1], src);
        float vv[2];
        int ii[2];
        vv[0] = lane < C ? lv[lane] : INFINITY;
        ii[0] = lane < C ? li[lane] : INT32_MAX;
        vv[1] = half == 0 ? v0 : v1;
        ii[1] = vv[1] == INFINITY ? INT32_MAX : (int)(k0 + lane);
        wave_sort128(vv, ii);
        if (lane < C) {
          lv[lane] = vv[0];
          li[lane] = ii[0];
        }
        nt = __shfl(vv[0], C - 1);
      }
      if (half == h) tr = nt;
    }
    return tr;
  };
  // lower bounds of tile kt (column tiles j0, j0 + 1 of the stage); rows with a bound below their
  // C-th bound merge (wave-local)
  auto epilogue = [&](int64_t kt, auto j0_c) __attribute__((always_inline)) {
    constexpr int j0 = decltype(j0_c)::value;
    const int64_t k0 = kt * kKT;
    // only the last tile has keys past n, only the tiles holding this wave's rows hold a self
    // pair, only the last work-group has rows past n: other tiles need no masking
    const bool clean = k0 + kKT <= n && (!self || k0 >= q0 + 32 || k0 + kKT <= q0) && q0 + 32 <= nq;
    const float nkc[2] = {__fmul_rn(c1, nk[j0]), __fmul_rn(c1, nk[j0 + 1])};
    auto bounds = [&](int r, float t0, float t1, float qr, float (&lb)[2]) __attribute__((always_inline)) {
      const int64_t q = q0 + 8 * (r >> 2) + 4 * half + (r & 3);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        lb[j] = __fmaf_rn(-2.0f, j == 0 ? t0 : t1, __fadd_rn(qr, nkc[j]));
        if (!clean) {
          const int64_t key = k0 + 32 * j + col;
          if (key >= n || (self && key == q) || q >= nq) lb[j] = INFINITY;
        }
      }
    };
    if constexpr (FAST) {
      // Long scans: rows (bit r) with a bound below their C-th bound in this tile first.  Late in
      // a long scan most tiles improve no row, and this test is a few register operations per
      // row; the merge then visits only the rows found, picking their values out of the register
      // arrays by comparisons (static indices only, so the arrays stay in registers).
      uint32_t rows = 0xffffu;
      if (clean) {
        rows = 0u;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const bool hit = __fmaf_rn(-2.0f, tot[j0][r], __fadd_rn(qv[r], nkc[0])) < tau[r] ||
                           __fmaf_rn(-2.0f, tot[j0 + 1][r], __fadd_rn(qv[r], nkc[1])) < tau[r];
          rows |= __ballot(hit) != 0ull ? (1u << r) : 0u;
        }
      }
      while (rows) {
        const int r = __builtin_ctz(rows);
        rows &= rows - 1;
        float t0 = tot[j0][0], t1 = tot[j0 + 1][0], qr = qv[0], tr = tau[0];
#pragma unroll
        for (int u = 1; u < 16; ++u) {
          t0 = r == u ? tot[j0][u] : t0;
          t1 = r == u ? tot[j0 + 1][u] : t1;
          qr = r == u ? qv[u] : qr;
          tr = r == u ? tau[u] : tr;
        }
        float lb[2];
        bounds(r, t0, t1, qr, lb);
        tr = merge_row(r, k0, lb, tr);
#pragma unroll
        for (int u = 0; u < 16; ++u) tau[u] = r == u ? tr : tau[u];
      }
    } else {
      // short scans, where most tiles improve some row: every row in turn
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float lb[2];
        bounds(r, tot[j0][r], tot[j0 + 1][r], qv[r], lb);
        tau[r] = merge_row(r, k0, lb, tau[r]);
      }
    }
  };
  // step i: loads for step i + 2 go out, chunk i is multiplied from the ring, step i + 1's
  // registers land in the ring, one barrier
  auto step = [&](auto slot_c, int64_t i, int64_t st, int c, int ring, int64_t st2, int c2, auto ai_c)
                  __attribute__((always_inline)) {
    constexpr int ai = decltype(ai_c)::value;
    constexpr int SL = decltype(slot_c)::value;
    if (c == 0) {
      // the stage's key norms (zero past the last key); scaled by c1 where the bounds are formed
      const int64_t r0 = st * (P * kKT);
      const __amdgpu_buffer_rsrc_t rn = rsrc_of(nrm + r0, n - r0, P * kKT, 4);
#pragma unroll
      for (int j = 0; j < NJ; ++j) nk[j] = bloadf(rn, 4 * col, 4 * 32 * j);
    }
    fetch(slot_c, st2, c2);
    const uint16_t* b = kst + ring * 2 * kStage;
    // d <= 128 (RES > 0): one accumulator over all coordinates; else a fresh one per chunk,
    // added to the total (the error constant of the bound follows the same structure)
    f32x16* acc = RES > 0 ? tot : part;
    if (RES == 0 || c == 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[j] = f32x16{};
    }
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int o = (32 * j + col) * kRow + 16 * s2 + 8 * half;
        const bf16x8 bh = load8(b + o);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ai][s2], bh, acc[j], 0, 0, 0);
        if (SPLIT) {
          const bf16x8 bl = load8(b + kStage + o);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ai][s2], bl, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ai][s2], bh, acc[j], 0, 0, 0);
        }
      }
    }
    if constexpr (RES == 0) {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[j][r] = c == 0 ? part[j][r] : tot[j][r] + part[j][r];
    }
    if (c == nch - 1) {
      epilogue(st * P, std::integral_constant<int, 0>{});
      if constexpr (P == 2) {
        if (st * P + 1 < nkt) epilogue(st * P + 1, std::integral_constant<int, 2>{});
      }
    }
    // (past the last step this moves zeros into a ring slot nobody reads again)
    stash(std::integral_constant<int, 1 - SL>{}, ring + 1 == RING ? 0 : ring + 1);
    __syncthreads();
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  fetch(S0{}, 0, 0);
  stash(S0{}, 0);
  fetch(S1{}, nch > 1 ? 0 : 1, nch > 1 ? 1 : 0);
  __syncthreads();
  if constexpr (RES > 0) {
    // two stages per iteration, so every step's register slot, query chunk and the chunk two
    // steps ahead are static; an odd last stage leaves the loop between the two (no branch
    // around a step, whose loads the compiler could then not count)
    for (int64_t s0 = 0;; s0 += 2) {
      static_for<0, RES>([&](auto tc) __attribute__((always_inline)) {
        constexpr int u = decltype(tc)::value;   // step within the pair of stages
        constexpr int c = u, t2 = (u + 2) / RES, c2 = (u + 2) % RES;
        const int64_t i = s0 * RES + c;
        step(std::integral_constant<int, u & 1>{}, i, s0, c, (int)(i % RING), s0 + t2, c2,
             std::integral_constant<int, c>{});
      });
      if (s0 + 1 >= nst) break;
      static_for<RES, 2 * RES>([&](auto tc) __attribute__((always_inline)) {
        constexpr int u = decltype(tc)::value;
        constexpr int c = u - RES, t2 = (u + 2) / RES, c2 = (u + 2) % RES;
        const int64_t i = (s0 + 1) * RES + c;
        step(std::integral_constant<int, u & 1>{}, i, s0 + 1, c, (int)(i % RING), s0 + t2, c2,
             std::integral_constant<int, c>{});
      });
      if (s0 + 2 >= nst) break;
    }
  } else {
    int64_t st = 0, st2 = 0;
    int c = 0, c2 = 0, ring = 0;
    auto advance = [&](int64_t& tt, int& cc) __attribute__((always_inline)) {
      if (++cc == nch) {
        cc = 0;
        ++tt;
      }
    };
    advance(st2, c2);
    advance(st2, c2);   // two steps ahead
    for (int64_t i = 0;; i += 2) {
      step(S0{}, i, st, c, ring, st2, c2, S0{});
      advance(st, c);
      advance(st2, c2);
      ring = ring + 1 == RING ? 0 : ring + 1;
      if (i + 1 >= steps) break;
      step(S1{}, i + 1, st, c, ring, st2, c2, S0{});
      advance(st, c);
      advance(st2, c2);
      ring = ring + 1 == RING ? 0 : ring + 1;
      if (i + 2 >= steps) break;
    }
  }
  for (int e = lane; e < 32 * C; e += 64) {
    const int rho = e / C, j = e % C;
    const int64_t q = q0 + rho;
    if (q < nq) cand[q * C + j] = liw[e];
  }
  if (lane < 32 && q0 + lane < nq) tau_out[q0 + lane] = lvw[lane * C + C - 1];
}

// Candidate search for small query sets (d <= 128), where cand_kernel's grid of one work-group
// per 128 queries would leave most CUs idle: a work-group owns 64 query rows and streams the same
// two-tile stages, but every row's keys are split between two waves - waves 0 and 1 take rows
// 0-31 and 32-63 against the first tile of each stage, waves 2 and 3 the same rows against the
// second - so the grid has twice the work-groups.  Each wave keeps its own C best bounds per row;
// the two waves of a row prune with the smaller of their two C-th bounds (shared through LDS: a
// bound above either list's C-th cannot be among the union's C best, and a stale value is only
// larger) and merge their lists at the end.  The candidate lists and bounds are those of
// cand_kernel.
constexpr int kQS = 64;   // query rows per work-group of the split search
constexpr int64_t kSplitBelow = 256;   // split while cand_kernel would have fewer work-groups (one per CU)
// Key counts from which the plain search tests all rows of a tile before merging (the FAST
// epilogue of cand_kernel).  Measured against merging row by row (ms, row by row -> tile test):
// 1,000,000 keys (d = 128) 900 -> 825, 400,000 keys 116 -> 97 (d = 64), 134 -> 119 (d = 96),
// 510 -> 509 (d = 200); but 300,000 keys 95 -> 108 (d = 128), 68 -> 73 (d = 32), 270,000 keys
// (d = 64) 66 -> 75: in shorter scans most tiles still improve some row.
constexpr int64_t kFastKeys = 3 << 17;   // 393,216

template <bool SPLIT, int RES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void cand_split_kernel(
    const uint16_t* __restrict__ xh, const uint16_t* __restrict__ xl, const float* __restrict__ nrm, int64_t n, int dp,
    int C, float c1, int32_t* __restrict__ cand, float* __restrict__ tau_out, const uint16_t* __restrict__ qh,
    const uint16_t* __restrict__ ql, const float* __restrict__ qn, int64_t nq, int self) {
  static_assert(RES > 0, "the split search keeps the query operands in registers (d <= 128)");
  constexpr int P = 2;                      // tiles per stage, one per key half
  constexpr int RING = 2;
  extern __shared__ unsigned char smraw[];
  uint16_t* kst = reinterpret_cast<uint16_t*>(smraw);
  constexpr int kStage = P * kKT * kRow;  // bf16 per array
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int rh = wave & 1, kh = wave >> 1;   // row half of the work-group, key half of the stage
  float* lvw = reinterpret_cast<float*>(smraw + sizeof(uint16_t) * 2 * RING * kStage) + wave * 32 * C;
  int* liw = reinterpret_cast<int*>(smraw + sizeof(uint16_t) * 2 * RING * kStage + sizeof(float) * 4 * 32 * C) +
             wave * 32 * C;
  __shared__ float tshare[2][kQS];   // [key half][row]: that wave's C-th bound of the row
  const int64_t q0 = (int64_t)blockIdx.x * kQS + 32 * rh;
  constexpr int nch = RES;
  for (int e = lane; e < 32 * C; e += 64) {
    lvw[e] = INFINITY;
    liw[e] = INT32_MAX;
  }
  if (lane < 32) tshare[kh][32 * rh + lane] = INFINITY;
  float qv[16], tau[16];
  {
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(qn + q0, nq - q0, 32, 4);   // zero past the last query
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      qv[r] = __fmul_rn(c1, bloadf(rq, 4 * (4 * half), 4 * (8 * (r >> 2) + (r & 3))));
      tau[r] = INFINITY;
    }
  }
  const int64_t arow = min<int64_t>(q0 + col, nq - 1);
  const uint16_t* aph = qh + arow * dp + 8 * half;
  const uint16_t* apl = ql + arow * dp + 8 * half;
  bf16x8 ah[RES][2], al[RES][2];
#pragma unroll
  for (int c = 0; c < RES; ++c)
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      ah[c][s2] = gload8(aph + kDK * c + 16 * s2);
      al[c][s2] = SPLIT ? gload8(apl + kDK * c + 16 * s2) : ah[c][s2];
    }
  // key rows of a wave's lanes: 4 (l / 4 % 4) + l / 16 (the four pieces of a row in four adjacent
  // lanes), so that the 8 (or 16) lanes an LDS write serves at once cover rows 4 (or 12) apart,
  // whose 80-byte rows fall on distinct banks; rows in order had every write two-way conflicted
  const int skey = 16 * (tid >> 6) + 4 * ((tid >> 2) & 3) + ((tid >> 4) & 3), spiece = (tid & 3) * 8;
  const int svoff = 2 * (skey * dp + spiece);   // this thread's byte offset inside a key stage
  const int64_t nkt = (n + kKT - 1) / kKT;
  const int64_t nst = (nkt + P - 1) / P;
  const int64_t steps = nst * nch;
  uint4 ph[2][P], pl[2][P];
  auto fetch = [&](auto slot_c, int64_t st, int c) __attribute__((always_inline)) {
    constexpr int SL = decltype(slot_c)::value;
    const int64_t r0 = st * (P * kKT);
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(xh + r0 * dp, n - r0, P * kKT, 2 * dp);
    const __amdgpu_buffer_rsrc_t rl = rsrc_of(xl + r0 * dp, n - r0, P * kKT, 2 * dp);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const int soff = __builtin_amdgcn_readfirstlane(2 * (kKT * t * dp + kDK * c));
      ph[SL][t] = bload16(rh, svoff, soff);
      pl[SL][t] = SPLIT ? bload16(rl, svoff, soff) : ph[SL][t];
    }
  };
  auto stash = [&](auto slot_c, int ring) __attribute__((always_inline)) {
    constexpr int SL = decltype(slot_c)::value;
    uint16_t* b = kst + ring * 2 * kStage;
#pragma unroll
    for (int t = 0; t < P; ++t) {
      *reinterpret_cast<uint4*>(b + (kKT * t + skey) * kRow + spiece) = ph[SL][t];
      if (SPLIT) *reinterpret_cast<uint4*>(b + kStage + (kKT * t + skey) * kRow + spiece) = pl[SL][t];
    }
  };
  f32x16 tot[2];
  float nk[2] = {0.f, 0.f};
  // lower bounds of tile kt against this wave's rows; a row merges where a bound is below the
  // smaller of its two waves' C-th bounds
  auto epilogue = [&](int64_t kt) __attribute__((always_inline)) {
    const int64_t k0 = kt * kKT;
    const bool clean = k0 + kKT <= n && (!self || k0 >= q0 + 32 || k0 + kKT <= q0) && q0 + 32 <= nq;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int rrow = 8 * (r >> 2) + 4 * half + (r & 3);
      const int64_t q = q0 + rrow;
      const float thr = fminf(tau[r], tshare[1 - kh][32 * rh + rrow]);
      float lb[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        lb[j] = qv[r] + __fmul_rn(c1, nk[j]) - 2.0f * tot[j][r];
        if (!clean) {
          const int64_t key = k0 + 32 * j + col;
          if (key >= n || (self && key == q) || q >= nq) lb[j] = INFINITY;
        }
      }
      const uint64_t m0 = __ballot(lb[0] < thr), m1 = __ballot(lb[1] < thr);
      if ((m0 | m1) == 0ull) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t b0 = (uint32_t)(m0 >> (32 * h)), b1 = (uint32_t)(m1 >> (32 * h));
        const int cnt = __popc(b0) + __popc(b1);
        if (cnt == 0) continue;
        const int rho = 8 * (r >> 2) + 4 * h + (r & 3);
        float* lv = lvw + rho * C;
        int* li = liw + rho * C;
        float nt;
        if (cnt <= bulk_above<RES, false>()) {
          float cv;
          int ci;
          list_load(lv, li, C, cv, ci);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            uint32_t bb = j == 0 ? b0 : b1;
            while (bb) {
              const int bit = __builtin_ctz(bb);
              bb &= bb - 1;
              const float v =
                  __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, lb[j]), 32 * h + bit));
              list_insert(cv, ci, C, v, (int)(k0 + 32 * j + bit));
            }
          }
          nt = list_store(lv, li, C, cv, ci);
        } else {
          const int src = 32 * h + col;
          const float v0 = __shfl(lb[0], src), v1 = __shfl(lb[1], src);
          float vv[2];
          int ii[2];
          vv[0] = lane < C ? lv[lane] : INFINITY;
          ii[0] = lane < C ? li[lane] : INT32_MAX;
          vv[1] = half == 0 ? v0 : v1;
          ii[1] = vv[1] == INFINITY ? INT32_MAX : (int)(k0 + lane);
          wave_sort128(vv, ii);
          if (lane < C) {
            lv[lane] = vv[0];
            li[lane] = ii[0];
          }
          nt = __shfl(vv[0], C - 1);
        }
        if (half == h) tau[r] = nt;
        if (lane == 0) tshare[kh][32 * rh + rho] = nt;
      }
    }
  };
  auto step = [&](auto slot_c, int64_t i, int64_t st, int c, int ring, int64_t st2, int c2, auto ai_c)
                  __attribute__((always_inline)) {
    constexpr int ai = decltype(ai_c)::value;
    constexpr int SL = decltype(slot_c)::value;
    if (c == 0) {
      const int64_t r0 = st * (P * kKT);
      const __amdgpu_buffer_rsrc_t rn = rsrc_of(nrm + r0, n - r0, P * kKT, 4);
#pragma unroll
      for (int j = 0; j < 2; ++j) nk[j] = bloadf(rn, 4 * col, __builtin_amdgcn_readfirstlane(4 * (kKT * kh + 32 * j)));
    }
    fetch(slot_c, st2, c2);
    const uint16_t* b = kst + ring * 2 * kStage + kKT * kh * kRow;
    if (c == 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j) tot[j] = f32x16{};
    }
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int o = (32 * j + col) * kRow + 16 * s2 + 8 * half;
        const bf16x8 bh = load8(b + o);
        tot[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ai][s2], bh, tot[j], 0, 0, 0);
        if (SPLIT) {
          const bf16x8 bl = load8(b + kStage + o);
          tot[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ai][s2], bl, tot[j], 0, 0, 0);
          tot[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ai][s2], bh, tot[j], 0, 0, 0);
        }
      }
    }
    if (c == nch - 1 && st * P + kh < nkt) epilogue(st * P + kh);
    stash(std::integral_constant<int, 1 - SL>{}, ring + 1 == RING ? 0 : ring + 1);
    __syncthreads();
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  fetch(S0{}, 0, 0);
  stash(S0{}, 0);
  fetch(S1{}, nch > 1 ? 0 : 1, nch > 1 ? 1 : 0);
  __syncthreads();
  for (int64_t s0 = 0;; s0 += 2) {
    static_for<0, RES>([&](auto tc) __attribute__((always_inline)) {
      constexpr int u = decltype(tc)::value;
      constexpr int c = u, t2 = (u + 2) / RES, c2 = (u + 2) % RES;
      const int64_t i = s0 * RES + c;
      step(std::integral_constant<int, u & 1>{}, i, s0, c, (int)(i % RING), s0 + t2, c2,
           std::integral_constant<int, c>{});
    });
    if (s0 + 1 >= nst) break;
    static_for<RES, 2 * RES>([&](auto tc) __attribute__((always_inline)) {
      constexpr int u = decltype(tc)::value;
      constexpr int c = u - RES, t2 = (u + 2) / RES, c2 = (u + 2) % RES;
      const int64_t i = (s0 + 1) * RES + c;
      step(std::integral_constant<int, u & 1>{}, i, s0 + 1, c, (int)(i % RING), s0 + t2, c2,
           std::integral_constant<int, c>{});
    });
    if (s0 + 2 >= nst) break;
  }
  // merge the two waves' lists of each row: waves 0 and 1 take rows 0-15 of their row half,
  // waves 2 and 3 rows 16-31 (the last barrier of the scan made every list visible)
  const int pw = (wave & 1);   // the row half's first wave; its partner is pw + 2
  const float* lva = reinterpret_cast<const float*>(smraw + sizeof(uint16_t) * 2 * RING * kStage) + pw * 32 * C;
  const float* lvb = lva + 2 * 32 * C;
  const int* lia = reinterpret_cast<const int*>(smraw + sizeof(uint16_t) * 2 * RING * kStage +
                                                sizeof(float) * 4 * 32 * C) + pw * 32 * C;
  const int* lib = lia + 2 * 32 * C;
  for (int rho = 16 * kh; rho < 16 * kh + 16; ++rho) {
    const int64_t q = q0 + rho;
    float vv[2];
    int ii[2];
    vv[0] = lane < C ? lva[rho * C + lane] : INFINITY;
    ii[0] = lane < C ? lia[rho * C + lane] : INT32_MAX;
    vv[1] = lane < C ? lvb[rho * C + lane] : INFINITY;
    ii[1] = lane < C ? lib[rho * C + lane] : INT32_MAX;
    wave_sort128(vv, ii);
    if (q < nq && lane < C) cand[q * C + lane] = ii[0];
    const float last = __shfl(vv[0], C - 1);
    if (q < nq && lane == 0) tau_out[q] = last;
  }
}

// ------------------------------------------------------------------------------------------
// 3. exact FP64 re-rank of the candidates, certificate, fallback list
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void rerank_kernel(const float* __restrict__ x, int64_t n, int d, int k, int C,
                                                        int bf16, const int32_t* __restrict__ cand,
                                                        const float* __restrict__ tau, int32_t* __restrict__ out_idx,
                                                        double* __restrict__ out_d2, int32_t* __restrict__ fb_rows,
                                                        int32_t* __restrict__ fb_count,
                                                        unsigned long long* __restrict__ certified,
                                                        const float* __restrict__ yq, int64_t nq) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= nq) return;
  int q = lane < C ? cand[row * C + lane] : INT32_MAX;
  double dist = INFINITY;
  if (q >= 0 && q < n) {
    const float* xp = yq + row * d;
    const float* xq = x + (int64_t)q * d;
    // coordinates in order; the loads of 8 at a time are issued together
    double acc = 0.0;
    int j = 0;
    for (; j + 8 <= d; j += 8) {
      float a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = xp[j + u];
        b[u] = xq[j + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (bf16) {
          a[u] = bf16_round(a[u]);
          b[u] = bf16_round(b[u]);
        }
        acc = sqdist_step(acc, (double)a[u], (double)b[u]);
      }
    }
    for (; j < d; ++j) {
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

bool knn_long_scan(int64_t n_keys) { return n_keys >= kFastKeys; }

slk_status split_points(const float* x, int64_t n, int32_t d, int32_t dp, int32_t bf16, double* mean, uint16_t* xh,
                        uint16_t* xl, float* nrm, hipStream_t s) {
  if (!bf16) {
    Scratch sc(s);
    double* part;
    const int nparts = mean_parts(n);
    SLK_TRY(sc.get(&part, (size_t)nparts * d));
    hipLaunchKernelGGL(colsum_kernel, dim3((d + kBlock - 1) / kBlock, nparts), dim3(kBlock), 0, s, x, n, d,
                       mean_rows(n), part);
    SLK_LAUNCHED("colsum_kernel");
    hipLaunchKernelGGL(colmean_kernel, dim3((d + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part, nparts, n, d, mean);
    SLK_LAUNCHED("colmean_kernel");
  }
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kBlock), 0, s, x, n, d, dp, mean, bf16, xh, xl,
                     nrm);
  SLK_LAUNCHED("split_kernel");
  return SLK_OK;
}

slk_status knn_mfma(const float* x, int64_t n, int32_t d, int32_t k, int32_t cand, int32_t bf16, int32_t* out_idx,
                    double* out_d2, int64_t* n_certified, int64_t* n_fallback, hipStream_t s, const float* y,
                    int64_t m, bool split_ok) {
  // queries: the points themselves (each excluded from its own list) or the m rows of y
  const bool self = y == nullptr;
  const float* qx = self ? x : y;
  const int64_t nq = self ? n : m;
  const int C = std::min(std::max(cand, k), kMaxCand);
  const int dp = ((d + kDK - 1) / kDK) * kDK;
  Scratch sc(s);
  uint16_t *xh, *xl, *qh, *ql;
  float *nrm, *qn, *tau;
  double *mean, *part;
  int32_t *cidx, *fb_rows, *fb_count;
  unsigned long long* certified;
  const int nparts = mean_parts(n);
  SLK_TRY(sc.get(&xh, (size_t)n * dp));
  SLK_TRY(sc.get(&xl, (size_t)n * dp));
  SLK_TRY(sc.get(&nrm, n));
  if (self) {
    qh = xh;
    ql = xl;
    qn = nrm;
  } else {
    SLK_TRY(sc.get(&qh, (size_t)nq * dp));
    SLK_TRY(sc.get(&ql, (size_t)nq * dp));
    SLK_TRY(sc.get(&qn, nq));
  }
  SLK_TRY(sc.get(&tau, nq));
  SLK_TRY(sc.get(&mean, d));
  SLK_TRY(sc.get(&part, (size_t)nparts * d));
  SLK_TRY(sc.get(&cidx, (size_t)nq * C));
  SLK_TRY(sc.get(&fb_rows, nq));
  SLK_TRY(sc.get(&fb_count, 1));
  SLK_TRY(sc.get(&certified, 1));
  SLK_HIP(hipMemsetAsync(fb_count, 0, sizeof(int32_t), s));
  SLK_HIP(hipMemsetAsync(certified, 0, sizeof(unsigned long long), s));
  if (!bf16) {
    hipLaunchKernelGGL(colsum_kernel, dim3((d + kBlock - 1) / kBlock, nparts), dim3(kBlock), 0, s, x, n, d,
                       mean_rows(n), part);
    SLK_LAUNCHED("colsum_kernel");
    hipLaunchKernelGGL(colmean_kernel, dim3((d + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part, nparts, n, d, mean);
    SLK_LAUNCHED("colmean_kernel");
  }
  // the queries are centred with the points' mean (distances do not depend on the centre)
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kBlock), 0, s, x, n, d, dp, mean, bf16, xh, xl,
                     nrm);
  SLK_LAUNCHED("split_kernel");
  if (!self) {
    hipLaunchKernelGGL(split_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(kBlock), 0, s, qx, nq, d, dp, mean, bf16, qh,
                       ql, qn);
    SLK_LAUNCHED("split_kernel");
  }
  // error constant of the lower bound (see the file comment): split residual + FP32
  // accumulation + final roundings, times 2.  For d <= 128 the products of all coordinates go
  // into one accumulator (3 d terms, d with bf16 points); above, 32-coordinate chunks (3 * 32
  // terms) are summed in d / 32 more additions.
  const double u = std::ldexp(1.0, -24);
  const int mul = bf16 ? 1 : 3;
  const double terms = dp <= 4 * kDK ? (double)mul * dp : (double)mul * kDK + dp / kDK;
  const double cG = (bf16 ? 0.0 : 3.05 * std::ldexp(1.0, -16)) + 1.01 * (terms + 2) * u;
  const double c = 2.0 * (cG + 8 * u);
  const float c1 = (float)(1.0 - c);
  // the split search when the plain one's grid would leave CUs idle (d <= 128 only)
  const bool split_search = split_ok && dp <= 4 * kDK && (nq + kQT - 1) / kQT < kSplitBelow;
  const unsigned grid = (unsigned)(split_search ? (nq + kQS - 1) / kQS : (nq + kQT - 1) / kQT);
  const int res = dp <= 4 * kDK ? dp / kDK : 0;
  // the ring of key stages (hi and lo), then the candidate lists
  const int tiles = res > 0 ? cand_tiles<1>() : cand_tiles<0>(), ring = res > 0 ? cand_ring<1>() : cand_ring<0>();
  const size_t lds = sizeof(uint16_t) * 2 * ring * tiles * kKT * kRow + (sizeof(float) + sizeof(int)) * (size_t)kQT * C;
  const int selfi = self ? 1 : 0;
  {
    KernelTimer kt("cand_kernel", s);
#define SLK_CAND(SPL, R)                                                                                          \
  if (R > 0 && split_search)                                                                                    \
    hipLaunchKernelGGL((cand_split_kernel<SPL, (R > 0 ? R : 1)>), dim3(grid), dim3(kBlock), lds, s, xh, xl, nrm, n, \
                       dp, C, c1, cidx, tau, qh, ql, qn, nq, selfi);                                              \
  else if (knn_long_scan(n))                                                                                    \
    hipLaunchKernelGGL((cand_kernel<SPL, R, true>), dim3(grid), dim3(kBlock), lds, s, xh, xl, nrm, n, dp, C, c1,   \
                       cidx, tau, qh, ql, qn, nq, selfi);                                                       \
  else                                                                                                          \
    hipLaunchKernelGGL((cand_kernel<SPL, R, false>), dim3(grid), dim3(kBlock), lds, s, xh, xl, nrm, n, dp, C, c1, cidx,   \
                       tau, qh, ql, qn, nq, selfi)
#define SLK_CAND_RES(SPL)                  \
    switch (res) {                         \
      case 1: SLK_CAND(SPL, 1); break;     \
      case 2: SLK_CAND(SPL, 2); break;     \
      case 3: SLK_CAND(SPL, 3); break;     \
      case 4: SLK_CAND(SPL, 4); break;     \
      default: SLK_CAND(SPL, 0); break;    \
    }
    if (bf16) {
      SLK_CAND_RES(false)
    } else {
      SLK_CAND_RES(true)
    }
#undef SLK_CAND_RES
#undef SLK_CAND
    SLK_LAUNCHED("cand_kernel");
  }
  {
    KernelTimer kt("rerank_kernel", s);
    hipLaunchKernelGGL(rerank_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(kBlock), 0, s, x, n, d, k, C, bf16, cidx,
                       tau, out_idx, out_d2, fb_rows, fb_count, certified, qx, nq);
    SLK_LAUNCHED("rerank_kernel");
  }
  int32_t h_fb = 0;
  unsigned long long h_cert = 0;
  SLK_HIP(hipMemcpyAsync(&h_fb, fb_count, sizeof(h_fb), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipMemcpyAsync(&h_cert, certified, sizeof(h_cert), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  if (timing_on()) timing_flush();
  if (h_fb > 0) SLK_TRY(knn_exact(x, n, d, k, bf16, fb_rows, h_fb, out_idx, out_d2, s, self ? nullptr : qx));
  SLK_HIP(hipStreamSynchronize(s));
  *n_certified = (int64_t)h_cert;
  *n_fallback = h_fb;
  return SLK_OK;
}

}  // namespace slk
