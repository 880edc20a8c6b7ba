// Kernels of the SLK-BO iteration for CDNA4 (gfx950, wave64).
//
//   iter_kernel    b_p = sum_q w_pq z_q (+ delta z_p), z_p' = softmax(a_p + lambda b_p) and the
//                  per-point relaxed-bound terms of the input Z            (Eqs. (6b), (8), (2)/(5))
//   final_kernel   the same logits once more for the last input, hard labels, the result Z in
//                  the caller's order, and per-block log-odds candidates for the modes  (Eq. (11))
//   mode_reduce    column arg-max over the per-block candidates
//   energy_kernel  E = -sum_p a_{p,l_p} + lambda * cut (Eq. (1) with Eq. (3)), FP32 unary term and
//                  an FP64 recheck recomputed from X
//
// Rows of the assignment matrix map onto groups of S lanes of a wavefront (S = next power of two
// >= L, at most 64; 64/S rows per wave); lane l of a group owns cluster l (and l + 64 e for L > 64).
// Neighbour indices of a row are loaded S at a time with one coalesced load and broadcast inside
// the group; every neighbour row z_q is then one coalesced S-lane load.  Row maxima and sums are
// butterfly reductions inside the group.  All reductions have a fixed order: results are
// bit-reproducible.
#include "common.h"

#include <float.h>
#include <math.h>

#include <type_traits>

namespace slk {

namespace {

constexpr int kBlock = 256;  // 4 waves

template <int S>
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
  for (int off = S / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, S));
  return v;
}

template <int S>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int off = S / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, S);
  return v;
}

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long load_agent(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float load_agent(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}




// ------------------------------------------------------------------------------------------
// one z-update: fused SpMM + softmax + bound terms
// ------------------------------------------------------------------------------------------
template <int S, int E>
struct RowOut {
  float s[E];    // logits a + lambda b (-inf on padding lanes)
  float e[E];    // exp(s - max)
  float z[E];    // softmax
  float m;       // row max
  float sum;     // sum of e
  float r;       // bound term of the input row (group-uniform)
};

// Neighbour extent and first index chunk of a row.  A wave walks its rows with a two-deep
// prefetch: while row r is gathered, the index chunk of row r + stride and the extent of
// row r + 2 stride are already in flight, so a row costs about one memory round trip.
struct Cursor {
  int32_t beg, end;  // CSR extent
  int myq;           // column index of neighbour beg + l0 (if l0 < min(S, end - beg))
};

template <int S>
__device__ __forceinline__ void load_extent(const IterArgs& a, int64_t row, Cursor& c) {
  c.beg = 0;
  c.end = 0;
  if (row < a.n) {
    c.beg = a.row_ptr[row];
    c.end = a.row_ptr[row + 1];
  }
}

// Row of A / Z holding internal row r (the caller's order when zperm is given).
__device__ __forceinline__ uint32_t zrow(const IterArgs& a, int64_t r) {
  return a.zperm ? (uint32_t)a.zperm[r] : (uint32_t)r;
}

template <int S>
__device__ __forceinline__ void load_chunk(const IterArgs& a, int l0, Cursor& c) {
  const int cnt = min(S, c.end - c.beg);
  c.myq = (l0 < cnt) ? (int)zrow(a, a.col_idx[c.beg + l0]) : 0;
}

// Computes one row inside its S-lane group.  All lanes of the group must call it together.
// `cur` holds the row's extent and first index chunk; `nxt` holds the extent of the next
// row of this group and receives its first index chunk; `nxt2` receives the extent of the
// row after that.
template <int S, int E>
__device__ __forceinline__ void row_update(const IterArgs& a, int64_t row, int l0, const Cursor& cur, Cursor& nxt,
                                           int64_t row2, Cursor& nxt2, RowOut<S, E>& o) {
  constexpr int CH = S < 16 ? S : 16;  // neighbour rows gathered per round
  const int L = a.L;
  // element offsets fit in 32 bits (n * ldz < 2^32 is checked on the host): one VGPR per address
  const uint32_t uL = (uint32_t)a.ldz;
  const uint32_t roff = zrow(a, row < a.n ? row : 0) * uL;
  float zp[E], av[E], b[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int l = l0 + S * e;
    const bool ok = l < L;
    av[e] = ok ? a.A[roff + l] : 0.f;
    zp[e] = ok ? a.Zin[roff + l] : 0.f;
    b[e] = 0.f;
  }
  // gathers are unconditional loads from always-valid addresses (clamped cluster index, row 0
  // for empty neighbour slots); dead slots are dropped by a group-uniform select, so no
  // branch sits between the loads
  uint32_t lc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) lc[e] = (uint32_t)min(l0 + S * e, L - 1);
  bool prefetched = false;
  for (int32_t c = cur.beg; c < cur.end; c += S) {
    const int cnt = min(S, cur.end - c);
    const int myq = (c == cur.beg) ? cur.myq : ((l0 < cnt) ? (int)zrow(a, a.col_idx[c + l0]) : 0);
    for (int t0 = 0; t0 < cnt; t0 += CH) {
      float v[CH][E];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        uint32_t q;
        if constexpr (S == 64)
          q = (uint32_t)__builtin_amdgcn_readlane(myq, t0 + i);  // one row per wave: scalar index
        else
          q = (uint32_t)__shfl(myq, t0 + i, S);
        const uint32_t qoff = q * uL;
#pragma unroll
        for (int e = 0; e < E; ++e) v[i][e] = a.Zin[qoff + lc[e]];
      }
      if (!prefetched) {
        load_chunk<S>(a, l0, nxt);
        load_extent<S>(a, row2, nxt2);
        prefetched = true;
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const bool live = t0 + i < cnt;
#pragma unroll
        for (int e = 0; e < E; ++e) b[e] += live ? v[i][e] : 0.f;
      }
    }
  }
  if (!prefetched) {
    load_chunk<S>(a, l0, nxt);
    load_extent<S>(a, row2, nxt2);
  }
  float m = -FLT_MAX, term = 0.f;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int l = l0 + S * e;
    if (a.delta != 0.f) b[e] += a.delta * zp[e];
    const bool ok = l < L;
    o.s[e] = ok ? av[e] + a.lam_eff * b[e] : -INFINITY;
    m = fmaxf(m, o.s[e]);
    if (ok) {
      const float zl = zp[e] > 0.f ? zp[e] * logf(zp[e]) : 0.f;
      term += zl - zp[e] * av[e] - a.half_lam_eff * zp[e] * b[e];
    }
  }
  m = group_max<S>(m);
  float sum = 0.f;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    o.e[e] = (l0 + S * e < L) ? expf(o.s[e] - m) : 0.f;
    sum += o.e[e];
  }
  sum = group_sum<S>(sum);
#pragma unroll
  for (int e = 0; e < E; ++e) o.z[e] = o.e[e] / sum;
  o.m = m;
  o.sum = sum;
  o.r = group_sum<S>(term);
}

// Row walk of one group: rows first, first + stride, ... (< last) with the two-deep
// prefetch; body(row, out) consumes each computed row.
template <int S, int E, class F>
__device__ __forceinline__ void row_loop(const IterArgs& a, int64_t first, int64_t stride, int64_t last, int l0,
                                         F&& body) {
  Cursor cur, nxt, nxt2;
  const IterArgs& aa = a;
  load_extent<S>(aa, first < last ? first : a.n, cur);
  load_chunk<S>(aa, l0, cur);
  load_extent<S>(aa, first + stride < last ? first + stride : a.n, nxt);
  for (int64_t row = first; row < last; row += stride) {
    RowOut<S, E> o;
    const int64_t r2 = row + 2 * stride;
    row_update<S, E>(a, row, l0, cur, nxt, r2 < last ? r2 : a.n, nxt2, o);
    body(row, o);
    cur = nxt;
    nxt = nxt2;
  }
}

// Fixed-order block sum of the per-group bound partials (group leaders hold them), written to
// partial[bid]; pass_reduce_kernel then sums the blocks in a fixed order.
template <int G>
__device__ __forceinline__ void block_partial(double* partial, int64_t bid, double acc, int g, int l0) {
  __shared__ double red[4 * G];
  const int tid = threadIdx.x, wave = tid >> 6;
  if (l0 == 0) red[wave * G + g] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < 4 * G; ++i) s += red[i];
    partial[bid] = s;
  }
}

// Fixed-order sum of the bound partials of one z-update, then the loop bookkeeping: bound
// trace, convergence test (relative change of the bound), pass counter.  A no-op once the
// loop is done, like the z-updates queued after it.  Each thread sums a strided slice with
// kRedUnroll independent accumulators (so the loads are all in flight together), then the
// block combines the slices in a fixed tree.  Run by a whole block of NT threads.
constexpr int kRedBlock = 1024;
constexpr int kRedUnroll = 8;
template <int NT>
__device__ __forceinline__ void reduce_pass(const double* __restrict__ partial, int nparts, IterState* st,
                                            double* trace, double* bound_out, IterState* mirror) {
  if (st->done) return;
  __shared__ double red[NT];
  const int tid = threadIdx.x;
  double acc[kRedUnroll];
#pragma unroll
  for (int u = 0; u < kRedUnroll; ++u) acc[u] = 0.0;
  for (int i0 = tid; i0 < nparts; i0 += NT * kRedUnroll) {
#pragma unroll
    for (int u = 0; u < kRedUnroll; ++u) {
      const int i = i0 + u * NT;
      if (i < nparts) acc[u] += load_agent(partial + i);
    }
  }
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < kRedUnroll; ++u) v += acc[u];
  red[tid] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const double R = red[0];
    const int pass = st->pass;
    if (trace && pass < st->trace_cap) trace[pass] = R;
    if (bound_out) *bound_out = R;
    if (!isfinite(R)) {
      st->numeric = 1;
      st->done = 1;
    } else if (st->check && pass >= 1 && fabs(R - st->last_bound) <= st->tol * fabs(st->last_bound)) {
      st->done = 1;
    }
    st->rel_prev = st->rel;
    st->rel = pass >= 1 ? fabs(R - st->last_bound) / fabs(st->last_bound) : 0.0;
    st->last_bound = R;
    st->pass = pass + 1;
    if (mirror) *mirror = *st;
  }
}

// Contiguous work tiles handed out in XCD order.  Workgroups are dispatched to the 8 XCDs
// round-robin (block b runs on XCD b % 8), so physical block b is given logical tile
// (b % 8) * ceil(T / 8) + b / 8: each XCD walks its own contiguous range of tiles in
// dispatch order, and the rows in flight on one XCD - and the neighbour rows they gather -
// stay inside a narrow window its L2 can hold.  The physical grid is 8 * ceil(T / 8).
__device__ __forceinline__ int64_t xcd_tile(int64_t ntiles, int64_t bid) {
  const int64_t gx = (ntiles + 7) >> 3;
  const int64_t x = bid & 7, k = bid >> 3;
  const int64_t t = x * gx + k;
  return (k < gx && t < ntiles) ? t : -1;
}

// Tiles: each wave handles kWaveSteps row groups (scalar kernels) or row batches (float4
// kernels) of one contiguous tile.
constexpr int kWaveSteps = 4;

template <int S, int E>
__global__ __launch_bounds__(kBlock) void iter_kernel(IterArgs a) {
  if (a.state->done) return;
  constexpr int G = 64 / S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / S, l0 = lane % S;
  constexpr int64_t kTileRows = 4 * G * kWaveSteps;
  const int64_t tile = xcd_tile((a.n + kTileRows - 1) / kTileRows, blockIdx.x);
  double acc = 0.0;
  if (tile >= 0) {
    const int64_t base = tile * kTileRows;
    row_loop<S, E>(a, base + wave * G + g, 4 * G, min(a.n, base + kTileRows), l0,
                   [&](int64_t row, const RowOut<S, E>& o) {
                     if (a.Zout) {
                       const uint32_t roff = zrow(a, row) * (uint32_t)a.ldz;
#pragma unroll
                       for (int e = 0; e < E; ++e) {
                         const int l = l0 + S * e;
                         if (l < a.L) a.Zout[roff + l] = o.z[e];
                       }
                     }
                     acc += (double)o.r;
                   });
  }
  block_partial<G>(a.partial, blockIdx.x, acc, g, l0);
}

// final pass: labels, log-odds candidates, output Z in the caller's order
template <int S, int E>
__global__ __launch_bounds__(kBlock) void final_kernel(FinalArgs f) {
  const IterArgs& a = f.it;
  constexpr int G = 64 / S;
  const int L = a.L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / S, l0 = lane % S;
  float bv[E];
  int bi[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    bv[e] = -INFINITY;
    bi[e] = INT32_MAX;
  }
  double acc = 0.0;
  constexpr int64_t kTileRows = 4 * G * kWaveSteps;
  const int64_t tile = xcd_tile((a.n + kTileRows - 1) / kTileRows, blockIdx.x);
  const int64_t base = tile * kTileRows;
  const int64_t first = tile >= 0 ? base + wave * G + g : a.n;
  const int64_t last = tile >= 0 ? min(a.n, base + kTileRows) : a.n;
  row_loop<S, E>(a, first, 4 * G, last, l0, [&](int64_t row, const RowOut<S, E>& o) {
    acc += (double)o.r;
    const int64_t orow = f.perm ? f.perm[row] : row;
    // first arg-max of the logits (ties to the smaller l)
    float tv = -INFINITY;
    int ti = INT32_MAX;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int l = l0 + S * e;
      if (l < L && (o.s[e] > tv)) {
        tv = o.s[e];
        ti = l;
      }
    }
#pragma unroll
    for (int off = S / 2; off > 0; off >>= 1) {
      const float ov = __shfl_xor(tv, off, S);
      const int oi = __shfl_xor(ti, off, S);
      if (ov > tv || (ov == tv && oi < ti)) {
        tv = ov;
        ti = oi;
      }
    }
    const int jt = ti < L ? ti : 0;  // a valid index whatever the logits (see final_row)
    // second largest logit (over j != jt) and the sums needed by the log-odds
    float m2 = -INFINITY, T = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int l = l0 + S * e;
      if (l < L && l != jt) {
        m2 = fmaxf(m2, o.s[e]);
        T += o.e[e];
      }
    }
    m2 = group_max<S>(m2);
    T = group_sum<S>(T);
    float S2 = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int l = l0 + S * e;
      if (l < L && l != jt) S2 += expf(o.s[e] - m2);
    }
    S2 = group_sum<S>(S2);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int l = l0 + S * e;
      if (l >= L) continue;
      float v;
      if (L == 1) {
        v = INFINITY;
      } else if (l == jt) {
        v = (o.m - m2) - logf(S2);      // log z/(1-z) for the top entry, no underflow
      } else {
        const float ub = o.s[e] - o.m;  // v <= ub (see final_row)
        v = ub < bv[e] ? -INFINITY : ub - log1pf(T - o.e[e]);
      }
      if (v > bv[e] || (v == bv[e] && (int)orow < bi[e])) {
        bv[e] = v;
        bi[e] = (int)orow;
      }
      if (f.z_user) f.z_user[orow * L + l] = o.z[e];
    }
    if (l0 == 0) {
      f.labels_int[row] = jt;
      if (f.labels_user) f.labels_user[orow] = jt;
    }
  });
  // combine the candidates of the groups of this wave (same l0 in every group)
#pragma unroll
  for (int off = S; off < 64; off <<= 1) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float ov = __shfl_xor(bv[e], off);
      const int oi = __shfl_xor(bi[e], off);
      if (ov > bv[e] || (ov == bv[e] && oi < bi[e])) {
        bv[e] = ov;
        bi[e] = oi;
      }
    }
  }
  __shared__ float cv[4][64 * E];
  __shared__ int ci[4][64 * E];
  if (g == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cv[wave][l0 + S * e] = bv[e];
      ci[wave][l0 + S * e] = bi[e];
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < L; l += kBlock) {
    float v = cv[0][l];
    int i = ci[0][l];
    for (int w = 1; w < 4; ++w) {
      if (cv[w][l] > v || (cv[w][l] == v && ci[w][l] < i)) {
        v = cv[w][l];
        i = ci[w][l];
      }
    }
    f.cand_v[(int64_t)l * gridDim.x + blockIdx.x] = v;
    f.cand_i[(int64_t)l * gridDim.x + blockIdx.x] = i;
  }
  block_partial<G>(a.partial, blockIdx.x, acc, g, l0);
}

// ------------------------------------------------------------------------------------------
// z-update and final pass on float4 rows (L <= 64)
// ------------------------------------------------------------------------------------------
// A row of A / Z (ldz = 4 ceil(L/4) floats) is held by G = next power of two >= ldz/4 lanes,
// four clusters per lane, so a wave carries 64/G rows at once and every gather instruction
// fetches one 16-byte slice of a neighbour row for each of them.  Row reductions run inside
// the G-lane group with DPP (quad permutes and row mirrors), never through LDS.
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16 lanes

template <int G>
__device__ __forceinline__ float gsum4(float v) {
  if constexpr (G >= 2) v += dppf<kDppXor1>(v);
  if constexpr (G >= 4) v += dppf<kDppXor2>(v);
  if constexpr (G >= 8) v += dppf<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dppf<kDppMirror>(v);
  return v;
}
template <int G>
__device__ __forceinline__ float gmax4(float v) {
  if constexpr (G >= 2) v = fmaxf(v, dppf<kDppXor1>(v));
  if constexpr (G >= 4) v = fmaxf(v, dppf<kDppXor2>(v));
  if constexpr (G >= 8) v = fmaxf(v, dppf<kDppHalfMirror>(v));
  if constexpr (G >= 16) v = fmaxf(v, dppf<kDppMirror>(v));
  return v;
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(float& v, int& i) {
  const float ov = dppf<CTRL>(v);
  const int oi = dppi<CTRL>(i);
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
template <int G>
__device__ __forceinline__ void gargmax4(float& v, int& i) {
  if constexpr (G >= 2) argmax_step<kDppXor1>(v, i);
  if constexpr (G >= 4) argmax_step<kDppXor2>(v, i);
  if constexpr (G >= 8) argmax_step<kDppHalfMirror>(v, i);
  if constexpr (G >= 16) argmax_step<kDppMirror>(v, i);
}

__device__ __forceinline__ float f4(const float4& v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }

typedef float vf4 __attribute__((ext_vector_type(4)));  // native vector for the non-temporal builtins
typedef float vf2 __attribute__((ext_vector_type(2)));

struct Row4 {
  float s[4], e[4], z[4];
  float m, sum, r;
};

// Broadcast of lane K of each G-lane group to the whole group, without LDS: quad permutes for
// G = 2 and 4, row_newbcast for G = 16 (one DPP row), an LDS permute only for G = 8.
template <int G, int K>
__device__ __forceinline__ uint32_t group_bcast(uint32_t v) {
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G == 2) {
    return (uint32_t)dppi<K | (K << 2) | ((2 + K) << 4) | ((2 + K) << 6)>((int)v);
  } else if constexpr (G == 4) {
    return (uint32_t)dppi<K * 0x55>((int)v);
  } else if constexpr (G == 16) {
    return (uint32_t)dppi<0x150 + K>((int)v);  // row_newbcast:K
  } else {
    return (uint32_t)__shfl((int)v, K, G);
  }
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}


// Buffer resource over an array of `bytes` bytes (< 2^32): loads at offsets >= bytes return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float4 load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  // bit-cast the whole vector: casting its elements one by one mis-lowers to a 4-byte load
  const vf4 v = __builtin_bit_cast(vf4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
  return make_float4(v.x, v.y, v.z, v.w);
}

constexpr int kCH = 16;  // neighbour slots per round (one index register per lane for G = 16)
constexpr int kHalf = kCH / 2;

// Byte offset of neighbour slot t of a row (CSR entries beg..beg+deg), or `dead` (= n * row
// bytes, past the end of Z) when t >= deg.
__device__ __forceinline__ uint32_t neighbour_offset(const IterArgs& a, int32_t beg, int deg, int t, uint32_t dead) {
  const int tc = min(t, max(deg - 1, 0));
  const uint32_t q = (uint32_t)__builtin_nontemporal_load(&a.col_off[beg + tc]);
  return t < deg ? q : dead;
}

// One batch of 64/G rows (one per group), row extent beg..end of this group's row.
// Per round the lanes of a group load the byte offsets of kCH neighbour slots (lane j holds
// slots t0 + j + G u) and broadcast them slot by slot; Z rows are fetched with 32-bit buffer
// offsets.  A round is issued in two halves of kHalf slots, the second only if some row of the
// wave still has neighbours there, so rows of degree 17..24 cost 24 slots, not 32.  The dead
// offset lies past the end of Z: empty slots read zeros and need no masking.
// Sum of the Z rows of the CSR entries beg .. beg+cnt-1 (this lane's 16-byte slice of them).
// Per round the lanes of a group load the byte offsets of kCH neighbour slots (lane j holds
// slots t0 + j + G u) and broadcast them slot by slot; Z rows are fetched with 32-bit buffer
// offsets.  A round is issued in two halves of kHalf slots, the second only if some group of
// the wave still has neighbours there, so 17..24 neighbours cost 24 slots, not 32.  The dead
// offset lies past the end of Z: empty slots read zeros and need no masking.
template <int G>
__device__ __forceinline__ float4 gather_sum(const IterArgs& a, __amdgpu_buffer_rsrc_t zr, int j, uint32_t jc16,
                                             int32_t beg, int cnt, uint32_t dead) {
  constexpr int U = kCH / G;   // offset registers per lane and round
  float bx = 0.f, by = 0.f, bz = 0.f, bw = 0.f;
  // the offsets of round t0 + kCH are loaded while round t0's rows are in flight
  uint32_t off[U];
#pragma unroll
  for (int u = 0; u < U; ++u) off[u] = neighbour_offset(a, beg, cnt, j + G * u, dead);
  for (int t0 = 0; __ballot(t0 < cnt) != 0ull; t0 += kCH) {
    float4 v[kCH];
    auto gather_lo = [&](auto ic) {
      constexpr int i = decltype(ic)::value;
      v[i] = load4(zr, group_bcast<G, i % G>(off[i / G]) + jc16);
    };
    auto gather_hi = [&](auto ic) {
      constexpr int i = decltype(ic)::value + kHalf;
      v[i] = load4(zr, group_bcast<G, i % G>(off[i / G]) + jc16);
    };
    static_for<0, kHalf>(gather_lo);
    const bool hi = __ballot(t0 + kHalf < cnt) != 0ull;
    if (hi) static_for<0, kHalf>(gather_hi);
    if (__ballot(t0 + kCH < cnt) != 0ull) {
#pragma unroll
      for (int u = 0; u < U; ++u) off[u] = neighbour_offset(a, beg, cnt, t0 + kCH + j + G * u, dead);
    }
#pragma unroll
    for (int i = 0; i < kHalf; ++i) {
      bx += v[i].x;
      by += v[i].y;
      bz += v[i].z;
      bw += v[i].w;
    }
    if (hi) {
#pragma unroll
      for (int i = kHalf; i < kCH; ++i) {
        bx += v[i].x;
        by += v[i].y;
        bz += v[i].z;
        bw += v[i].w;
      }
    }
  }
  return make_float4(bx, by, bz, bw);
}

// Logits s = a + lambda b (+ delta z), the softmax of the row and its bound term, from the
// neighbour sum b; av and zp are this lane's slices of the row of A and Z^i.
template <int G>
__device__ __forceinline__ void row_finish(const IterArgs& a, float4 av, float4 zp, float4 b, int j, Row4& o) {
  const int L = a.L;
  const float bb[4] = {b.x, b.y, b.z, b.w};
  float m = -FLT_MAX, term = 0.f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool ok = 4 * j + e < L;
    const float z0 = f4(zp, e), a0 = f4(av, e);
    float b0 = bb[e];
    if (a.delta != 0.f) b0 += a.delta * z0;
    o.s[e] = ok ? a0 + a.lam_eff * b0 : -INFINITY;
    m = fmaxf(m, o.s[e]);
    if (ok) {
      const float zl = z0 > 0.f ? z0 * __logf(z0) : 0.f;
      term += zl - z0 * a0 - a.half_lam_eff * z0 * b0;
    }
  }
  m = gmax4<G>(m);
  float sum = 0.f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    o.e[e] = (4 * j + e < L) ? __expf(o.s[e] - m) : 0.f;
    sum += o.e[e];
  }
  sum = gsum4<G>(sum);
  const float inv = 1.0f / sum;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.z[e] = o.e[e] * inv;
  o.m = m;
  o.sum = sum;
  o.r = gsum4<G>(term);
}

struct RowGeom {
  uint32_t L4, rb, jc16, dead;
  __amdgpu_buffer_rsrc_t zr;
};

__device__ __forceinline__ RowGeom row_geom(const IterArgs& a, int j) {
  RowGeom r;
  r.L4 = (uint32_t)(a.ldz >> 2);
  r.rb = r.L4 * 16u;                                  // row bytes
  r.jc16 = min((uint32_t)j, r.L4 - 1) * 16u;
  r.dead = (uint32_t)a.n * r.rb;
  r.zr = buffer_of(a.Zin, r.dead);
  return r;
}

__device__ __forceinline__ float4 row_slice_A(const IterArgs& a, const RowGeom& r, uint32_t rowc) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(a.A) + (rowc * r.L4 + (r.jc16 >> 4)));
  return make_float4(v.x, v.y, v.z, v.w);
}

// One batch of 64/G rows (one per group), row extent beg..end of this group's row; a row
// with valid = false gathers nothing.
template <int G>
__device__ __forceinline__ void row4_update(const IterArgs& a, uint32_t rowc, bool valid, int j, int32_t beg,
                                            int32_t end, Row4& o) {
  const RowGeom r = row_geom(a, j);
  const float4 av = row_slice_A(a, r, rowc);
  const float4 zp = load4(r.zr, rowc * r.rb + r.jc16);
  const float4 b = gather_sum<G>(a, r.zr, j, r.jc16, beg, valid ? end - beg : 0, r.dead);
  row_finish<G>(a, av, zp, b, j, o);
}

// Heavy row hb of the block (a.heavy[hb]; none when hb >= n_heavy).  Every group of the block
// sums a contiguous share of the row's neighbours; the shares are added in group order through
// LDS and wave 0 finishes the row - each of its groups computes the same row, group 0's copy is
// the one stored.  Must be reached by the whole block.
template <int G>
__device__ __forceinline__ bool heavy_row(const IterArgs& a, int hb, int wave, int g, int j, uint32_t& rowc, Row4& o) {
  constexpr int RW = 64 / G, NG = 4 * RW;
  const bool valid = hb < a.n_heavy;
  rowc = valid ? (uint32_t)a.heavy[hb] : 0u;
  const int32_t beg = a.row_ptr[rowc], end = a.row_ptr[rowc + 1];
  const int deg = valid ? end - beg : 0;
  const int share = (deg + NG - 1) / NG;
  const int gid = wave * RW + g;
  const int s0 = min(deg, gid * share), s1 = min(deg, s0 + share);
  const RowGeom r = row_geom(a, j);
  const float4 part = gather_sum<G>(a, r.zr, j, r.jc16, beg + s0, s1 - s0, r.dead);
  __shared__ float4 hsum[kBlock];
  hsum[threadIdx.x] = part;
  __syncthreads();
  if (wave == 0) {
    float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
    // a short unroll: a full one holds every group's share in registers at once
#pragma unroll 4
    for (int q = 0; q < NG; ++q) {
      const float4 v = hsum[q * G + j];
      b.x += v.x;
      b.y += v.y;
      b.z += v.z;
      b.w += v.w;
    }
    const float4 av = row_slice_A(a, r, rowc);
    const float4 zp = load4(r.zr, rowc * r.rb + r.jc16);
    row_finish<G>(a, av, zp, b, j, o);
  }
  return valid;
}

template <int G>
__device__ __forceinline__ void final_row(const FinalArgs& f, int64_t row, bool valid, bool store, int j, const Row4& o,
                                          float (&bv)[4], int (&bi)[4], double& acc);
template <int G>
__device__ __forceinline__ void block_candidates(const FinalArgs& f, int bid, float (&bv)[4], int (&bi)[4], int g, int j,
                                                 int wave);

// One work-group of the z-update.  With EMIT it also produces what the final pass would produce
// from the same input (labels in f->labels_int, the work-group's byproduct-mode candidates in
// f->cand_v / f->cand_i), with the same per-row arithmetic: the pass that ends the loop then
// leaves them behind and no separate final pass is needed.
template <int G, bool EMIT>
__device__ __forceinline__ void iter4_body(const IterArgs& a, const FinalArgs* f, int bid) {
  if (a.state->done) return;
  constexpr int RW = 64 / G;  // rows per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / G, j = lane % G;
  const uint32_t L4 = (uint32_t)(a.ldz >> 2);
  float4* __restrict__ O4 = reinterpret_cast<float4*>(a.Zout);
  double acc = 0.0, unused = 0.0;
  float bv[4];
  int bi[4];
  if constexpr (EMIT) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bv[e] = -INFINITY;
      bi[e] = INT32_MAX;
    }
  }
  if (bid < a.hblocks) {
    uint32_t rowc;
    Row4 o;
    const bool valid = heavy_row<G>(a, bid, wave, g, j, rowc, o);
    if (valid && wave == 0 && g == 0) {
      if (O4 && (uint32_t)j < L4)
        __builtin_nontemporal_store(vf4{o.z[0], o.z[1], o.z[2], o.z[3]}, reinterpret_cast<vf4*>(O4) + (rowc * L4 + j));
      if (j == 0) acc = (double)o.r;
    }
    // every group of wave 0 holds the same row: all offer the same candidates, group 0 stores
    if constexpr (EMIT) {
      if (wave == 0) final_row<G>(*f, rowc, valid, g == 0, j, o, bv, bi, unused);
      block_candidates<G>(*f, bid, bv, bi, g, j, wave);
    }
    block_partial<RW>(a.partial, bid, acc, g, j);
    return;
  }
  const int64_t nbatch = (a.n + RW - 1) / RW;
  const int64_t TB = 4 * (a.wsteps > 0 ? a.wsteps : kWaveSteps);  // batches per tile
  const int64_t tile = xcd_tile((nbatch + TB - 1) / TB, (int64_t)bid - a.hblocks);
  // a block without a tile (grid padding) walks nothing: b0 = bstop = 0
  const int64_t b0 = tile >= 0 ? tile * TB + wave : 0;
  const int64_t bstop = tile >= 0 ? min(nbatch, (tile + 1) * TB) : 0;
  // the row extent of batch b + 4 is loaded while batch b is computed
  auto clamp_row = [&](int64_t row) { return (uint32_t)(row >= 0 && row < a.n ? row : a.n - 1); };
  int32_t nbeg = 0, nend = 0;
  if (b0 < bstop) {
    const uint32_t r0 = clamp_row(b0 * RW + g);
    nbeg = a.row_ptr[r0];
    nend = a.row_ptr[r0 + 1];
  }
  for (int64_t b = b0; b < bstop; b += 4) {
    const int64_t row = b * RW + g;
    const uint32_t rowc = clamp_row(row);
    const int32_t beg = nbeg, end = nend;
    if (b + 4 < bstop) {
      const uint32_t r1 = clamp_row((b + 4) * RW + g);
      nbeg = a.row_ptr[r1];
      nend = a.row_ptr[r1 + 1];
    }
    // heavy rows belong to the work-groups in front of the grid
    const bool valid = row >= 0 && row < a.n && end - beg <= a.heavy_deg;
    Row4 o;
    row4_update<G>(a, rowc, valid, j, beg, end, o);
    if (valid) {
      if (O4 && (uint32_t)j < L4)
        __builtin_nontemporal_store(vf4{o.z[0], o.z[1], o.z[2], o.z[3]}, reinterpret_cast<vf4*>(O4) + (rowc * L4 + j));
      if (j == 0) acc += (double)o.r;
    }
    if constexpr (EMIT) final_row<G>(*f, row, valid, true, j, o, bv, bi, unused);
  }
  if constexpr (EMIT) block_candidates<G>(*f, bid, bv, bi, g, j, wave);
  block_partial<RW>(a.partial, bid, acc, g, j);
}

template <int G>
__global__ __launch_bounds__(kBlock) void iter4_kernel(IterArgs a) {
  iter4_body<G, false>(a, nullptr, blockIdx.x);
}

// Whether the z-update about to run (index st->pass) is expected to end the loop: it is the last
// pass allowed, or, testing convergence, the relative change of the bound predicted for it from
// the two passes before (geometric decay, ratio at most 1) is within twice the tolerance.  Every
// work-group reads the same state, so all take the same branch.
__device__ __forceinline__ bool expect_last_pass(const IterState* st) {
  const int k = st->pass;
  if (k >= st->last_pass) return true;
  if (!st->check || k < 2) return false;
  const double r1 = st->rel, r0 = st->rel_prev;
  const double pred = r0 > 0.0 ? r1 * fmin(r1 / r0, 1.0) : r1;
  return pred <= 2.0 * st->tol;
}

// The z-update that writes the labels and byproduct-mode candidates of its input when it expects
// to end the loop (work-group 0 records the pass in st->emit_pass), and is the plain z-update
// otherwise.  Four waves per SIMD (at most 128 registers) where that needs no spills, as for the
// plain z-update; the host uses this form for L > 8 only.
template <int G>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(G >= 4 ? 4 : 1))) void iter4_emit_kernel(
    FinalArgs f) {
  IterState* st = f.it.state;
  if (st->done) return;
  if (expect_last_pass(st)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->emit_pass = st->pass;
    iter4_body<G, true>(f.it, &f, blockIdx.x);
  } else {
    iter4_body<G, false>(f.it, nullptr, blockIdx.x);
  }
}

template <int G>
__global__ __launch_bounds__(kBlock) void iter4_packed(const IterArgs* __restrict__ jobs,
                                                       const int32_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  iter4_body<G, false>(jobs[j], nullptr, blockIdx.x - start[j]);
}

// Labels, byproduct-mode candidates and caller-order outputs of one finished row.  `valid`
// rows update the candidates and the bound sum; `store` rows also write labels and z_user.
template <int G>
__device__ __forceinline__ void final_row(const FinalArgs& f, int64_t row, bool valid, bool store, int j, const Row4& o,
                                          float (&bv)[4], int (&bi)[4], double& acc) {
  const int L = f.it.L;
  // first arg-max of the logits (ties to the smaller l)
  float tv = -INFINITY;
  int ti = INT32_MAX;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (4 * j + e < L && o.s[e] > tv) {
      tv = o.s[e];
      ti = 4 * j + e;
    }
  gargmax4<G>(tv, ti);
  // every logit is finite when the bound of the pass was (the loop stops on a non-finite bound),
  // so ti < L; the clamp keeps the label a valid index regardless
  const int jt = ti < L ? ti : 0;
  float m2 = -INFINITY, T = 0.f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = 4 * j + e;
    if (l < L && l != jt) {
      m2 = fmaxf(m2, o.s[e]);
      T += o.e[e];
    }
  }
  m2 = gmax4<G>(m2);
  T = gsum4<G>(T);
  float S2 = 0.f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = 4 * j + e;
    if (l < L && l != jt) S2 += expf(o.s[e] - m2);
  }
  S2 = gsum4<G>(S2);
  if (!valid) return;
  if (store) acc += (j == 0) ? (double)o.r : 0.0;
  const int64_t orow = f.perm ? f.perm[row] : row;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = 4 * j + e;
    if (l >= L) continue;
    float v;
    if (L == 1) {
      v = INFINITY;
    } else if (l == jt) {
      v = (o.m - m2) - logf(S2);      // log z/(1-z) for the top entry, no underflow
    } else {
      // T >= e exactly (a rounded sum of nonnegative terms is at least each term), so the log1p
      // is >= 0 and v <= s - m: an entry below this lane's best candidate cannot win or tie
      const float ub = o.s[e] - o.m;
      v = ub < bv[e] ? -INFINITY : ub - log1pf(T - o.e[e]);
    }
    if (v > bv[e] || (v == bv[e] && (int)orow < bi[e])) {
      bv[e] = v;
      bi[e] = (int)orow;
    }
    if (store && f.z_user) f.z_user[orow * L + l] = o.z[e];
  }
  if (store && j == 0) {
    f.labels_int[row] = jt;
    if (f.labels_user) f.labels_user[orow] = jt;
  }
}

// The work-group's best byproduct-mode candidate per cluster (largest log-odds, ties to the
// smaller index) from the lanes' candidates, to cand_v / cand_i[l * grid + bid].  Reached by the
// whole work-group.
template <int G>
__device__ __forceinline__ void block_candidates(const FinalArgs& f, int bid, float (&bv)[4], int (&bi)[4], int g, int j,
                                                 int wave) {
  // combine the candidates of the groups of this wave (same j in every group)
#pragma unroll
  for (int off = G; off < 64; off <<= 1) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float ov = __shfl_xor(bv[e], off);
      const int oi = __shfl_xor(bi[e], off);
      if (ov > bv[e] || (ov == bv[e] && oi < bi[e])) {
        bv[e] = ov;
        bi[e] = oi;
      }
    }
  }
  __shared__ float cv[4][64];
  __shared__ int ci[4][64];
  if (g == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (4 * j + e < 64) {
        cv[wave][4 * j + e] = bv[e];
        ci[wave][4 * j + e] = bi[e];
      }
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < f.it.L; l += kBlock) {
    float v = cv[0][l];
    int i = ci[0][l];
    for (int w = 1; w < 4; ++w) {
      if (cv[w][l] > v || (cv[w][l] == v && ci[w][l] < i)) {
        v = cv[w][l];
        i = ci[w][l];
      }
    }
    f.cand_v[(int64_t)l * f.grid + bid] = v;
    f.cand_i[(int64_t)l * f.grid + bid] = i;
  }
}

template <int G>
__device__ __forceinline__ void final4_block(const FinalArgs& f, int bid) {
  const IterArgs& a = f.it;
  constexpr int RW = 64 / G;
  const int L = a.L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / G, j = lane % G;
  float bv[4];
  int bi[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    bv[e] = -INFINITY;
    bi[e] = INT32_MAX;
  }
  double acc = 0.0;
  if (bid < a.hblocks) {
    uint32_t rowc;
    Row4 o;
    const bool valid = heavy_row<G>(a, bid, wave, g, j, rowc, o);
    // every group of wave 0 holds the same row: all offer the same candidates, group 0 stores
    if (wave == 0) final_row<G>(f, rowc, valid, g == 0, j, o, bv, bi, acc);
  } else {
    const int64_t nbatch = (a.n + RW - 1) / RW;
    const int64_t TB = 4 * (a.wsteps > 0 ? a.wsteps : kWaveSteps);  // batches per tile
    const int64_t tile = xcd_tile((nbatch + TB - 1) / TB, (int64_t)bid - a.hblocks);
    // a block without a tile (grid padding) walks nothing
    const int64_t b0 = tile >= 0 ? tile * TB + wave : 0;
    const int64_t bstop = tile >= 0 ? min(nbatch, (tile + 1) * TB) : 0;
    for (int64_t b = b0; b < bstop; b += 4) {
      const int64_t row = b * RW + g;
      const uint32_t rowc = (uint32_t)(row >= 0 && row < a.n ? row : a.n - 1);
      const int32_t beg = a.row_ptr[rowc], end = a.row_ptr[rowc + 1];
      const bool valid = row >= 0 && row < a.n && end - beg <= a.heavy_deg;
      Row4 o;
      row4_update<G>(a, rowc, valid, j, beg, end, o);
      final_row<G>(f, row, valid, true, j, o, bv, bi, acc);
    }
  }
  block_candidates<G>(f, bid, bv, bi, g, j, wave);
  block_partial<RW>(a.partial, bid, acc, g, j);
}

template <int G>
__global__ __launch_bounds__(kBlock) void final4_kernel(FinalArgs f) {
  final4_block<G>(f, blockIdx.x);
}

template <int G>
__global__ __launch_bounds__(kBlock) void final4_packed(const FinalArgs* __restrict__ jobs,
                                                        const int32_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  final4_block<G>(jobs[j], blockIdx.x - start[j]);
}

__device__ __forceinline__ void mode_reduce_block(const float* __restrict__ cv, const int32_t* __restrict__ ci, int grid,
                                                  int32_t* __restrict__ modes, int l, int32_t* mirror = nullptr,
                                                  const int32_t* cur = nullptr, int32_t* moved = nullptr) {
  const int tid = threadIdx.x;
  float v = -INFINITY;
  int i = INT32_MAX;
  const float* __restrict__ cvl = cv + (int64_t)l * grid;
  const int32_t* __restrict__ cil = ci + (int64_t)l * grid;
  // candidates tid, tid + kBlock, ... in that order; their loads are issued 8 at a time
  int b = tid;
  for (; b + 7 * kBlock < grid; b += 8 * kBlock) {
    float ov[8];
    int oi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      ov[u] = cvl[b + u * kBlock];
      oi[u] = cil[b + u * kBlock];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (ov[u] > v || (ov[u] == v && oi[u] < i)) {
        v = ov[u];
        i = oi[u];
      }
  }
  for (; b < grid; b += kBlock) {
    const float ov = cvl[b];
    const int oi = cil[b];
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  __shared__ float sv[kBlock];
  __shared__ int si[kBlock];
  sv[tid] = v;
  si[tid] = i;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      if (sv[tid + w] > sv[tid] || (sv[tid + w] == sv[tid] && si[tid + w] < si[tid])) {
        sv[tid] = sv[tid + w];
        si[tid] = si[tid + w];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int32_t m = si[0] == INT32_MAX ? 0 : si[0];
    modes[l] = m;
    if (mirror) mirror[l] = m;
    if (moved) moved[l] = m != cur[l];
  }
}

__global__ __launch_bounds__(kBlock) void mode_reduce_kernel(const float* __restrict__ cv, const int32_t* __restrict__ ci,
                                                             int grid, int L, int32_t* __restrict__ modes,
                                                             int32_t* mirror, const int32_t* cur, int32_t* moved) {
  mode_reduce_block(cv, ci, grid, modes, blockIdx.x, mirror, cur, moved);
}

// one block per (job, cluster): start[j] = first block of job j, L_j blocks each
__global__ __launch_bounds__(kBlock) void mode_reduce_packed(const ModeJob* __restrict__ jobs,
                                                             const int32_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const ModeJob m = jobs[j];
  mode_reduce_block(m.cand_v, m.cand_i, m.grid, m.modes, blockIdx.x - start[j]);
}

// ------------------------------------------------------------------------------------------
// energy: FP32 unary term, exact cut count and an FP64 recheck of the unary term
// ------------------------------------------------------------------------------------------
// 16 lanes per row, 4 rows per wave, contiguous XCD-ordered tiles.
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double gsum16d(double v) {
  v += dppd<kDppXor1>(v);
  v += dppd<kDppXor2>(v);
  v += dppd<kDppHalfMirror>(v);
  v += dppd<kDppMirror>(v);
  return v;
}
__device__ __forceinline__ int gsum16i(int v) {
  v += dppi<kDppXor1>(v);
  v += dppi<kDppXor2>(v);
  v += dppi<kDppHalfMirror>(v);
  v += dppi<kDppMirror>(v);
  return v;
}

// FP64 recheck of the unary term of one row (16 lanes; the caller sums them).
__device__ __forceinline__ double unary64_part(const EnergyArgs& e, int64_t rowc, int lab, int j) {
  const int64_t orow = e.perm ? e.perm[rowc] : rowc;
  const float* xp = e.x + orow * e.d;
  const float* mp = e.mvec ? e.mvec + (int64_t)lab * e.d : e.x + (int64_t)e.modes[lab] * e.d;
  double d64 = 0.0;
  for (int k = j; k < e.d; k += 16) {
    const double t = (double)xp[k] - (double)mp[k];
    d64 += t * t;
  }
  return d64;
}

__device__ __forceinline__ void energy_block(const EnergyArgs& e, int bid) {
  constexpr int G = 16, RW = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tid = threadIdx.x;
  const int g = lane / G, j = lane % G;
  if (bid < e.hblocks) {
    // one heavy row: the block counts its cut edges, wave 0 rechecks its unary term
    const int hb = bid;
    const bool valid = hb < e.n_heavy;
    const int64_t rowc = valid ? e.heavy[hb] : 0;
    const int lab = e.labels_int[rowc];
    const int32_t beg = e.row_ptr[rowc], end = valid ? e.row_ptr[rowc + 1] : beg;
    int c = 0;
    for (int32_t t = beg + tid; t < end; t += kBlock) c += (e.labels_int[e.col_idx[t]] != lab);
    __shared__ int hc[kBlock];
    hc[tid] = c;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (tid < w) hc[tid] += hc[tid + w];
      __syncthreads();
    }
    double d64 = 0.0;
    if (e.x && wave == 0) d64 = gsum16d(unary64_part(e, rowc, lab, j));
    if (tid == 0) {
      e.part_un[bid] = valid ? (double)e.A[rowc * e.ldz + lab] : 0.0;
      e.part_un64[bid] = valid && e.x ? exp(-d64 * e.inv2s2) : 0.0;
      e.part_cut[bid] = hc[0];
    }
    return;
  }
  double un = 0.0, un64 = 0.0;
  long long cut = 0;
  const int64_t nbatch = (e.n + RW - 1) / RW;
  const int64_t tile = xcd_tile((nbatch + 4 * kWaveSteps - 1) / (4 * kWaveSteps), (int64_t)bid - e.hblocks);
  // a block without a tile (grid padding) walks nothing
  const int64_t b0 = tile >= 0 ? tile * 4 * kWaveSteps + wave : 0;
  const int64_t bstop = tile >= 0 ? min(nbatch, (tile + 1) * 4 * kWaveSteps) : 0;
  // d = 64 or 128 with 16-byte rows: the FP64 recheck's coordinates are loaded as float4 before
  // the cut's dependent gathers, so both are in flight together
  const bool x4 = e.x && (e.d == 64 || e.d == 128) && (((uintptr_t)e.x | (uintptr_t)e.mvec) & 15) == 0;
  for (int64_t b = b0; b < bstop; b += 4) {
    const int64_t row = b * RW + g;
    const int64_t rowc = row >= 0 && row < e.n ? row : e.n - 1;
    const int lab = e.labels_int[rowc];
    const int32_t beg = e.row_ptr[rowc], end0 = e.row_ptr[rowc + 1];
    // heavy rows belong to the work-groups in front of the grid
    const bool valid = row >= 0 && row < e.n && end0 - beg <= e.heavy_deg;
    const int32_t end = valid ? end0 : beg;
    float4 xv[2], mv[2];
    if (x4) {
      const int64_t orow = e.perm ? e.perm[rowc] : rowc;
      const float4* xp = reinterpret_cast<const float4*>(e.x + orow * e.d);
      const float4* mp = reinterpret_cast<const float4*>(e.mvec ? e.mvec + (int64_t)lab * e.d
                                                                 : e.x + (int64_t)e.modes[lab] * e.d);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int q = j + 16 * i;  // float4 index: coordinates 4 q .. 4 q + 3
        xv[i] = q < e.d / 4 ? xp[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        mv[i] = q < e.d / 4 ? mp[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    int c = 0;
    for (int32_t t = beg + j; t < end; t += G) c += (e.labels_int[e.col_idx[t]] != lab);
    c = gsum16i(c);
    double d64 = 0.0;
    if (x4) {
      double p = 0.0;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double t0 = (double)xv[i].x - (double)mv[i].x, t1 = (double)xv[i].y - (double)mv[i].y;
        const double t2 = (double)xv[i].z - (double)mv[i].z, t3 = (double)xv[i].w - (double)mv[i].w;
        p += t0 * t0;
        p += t1 * t1;
        p += t2 * t2;
        p += t3 * t3;
      }
      d64 = gsum16d(p);
    } else if (e.x) {
      d64 = gsum16d(unary64_part(e, rowc, lab, j));
    }
    if (valid && j == 0) {
      un += (double)e.A[rowc * e.ldz + lab];
      cut += c;
      if (e.x) un64 += exp(-d64 * e.inv2s2);
    }
  }
  // lanes 0, 16, 32, 48 hold the sums of their groups; fixed-order block sums
  __shared__ double s_un[16], s_un64[16];
  __shared__ long long s_cut[16];
  if (j == 0) {
    s_un[wave * RW + g] = un;
    s_un64[wave * RW + g] = un64;
    s_cut[wave * RW + g] = cut;
  }
  __syncthreads();
  if (tid == 0) {
    double a0 = 0, a1 = 0;
    long long c0 = 0;
    for (int w = 0; w < 16; ++w) {
      a0 += s_un[w];
      a1 += s_un64[w];
      c0 += s_cut[w];
    }
    e.part_un[bid] = a0;
    e.part_un64[bid] = a1;
    e.part_cut[bid] = c0;
  }
}

// True when a mode moved (the energy of this outer iteration is not needed).
__device__ __forceinline__ bool energy_skipped(const int32_t* moved, int L) {
  if (!moved) return false;
  for (int l = 0; l < L; ++l)
    if (moved[l]) return true;
  return false;
}

__global__ __launch_bounds__(kBlock) void energy_kernel(EnergyArgs e) {
  if (energy_skipped(e.moved, e.L)) return;
  energy_block(e, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void energy_packed(const EnergyArgs* __restrict__ jobs,
                                                        const int32_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  energy_block(jobs[j], blockIdx.x - start[j]);
}

// Fixed-order sums of the energy block partials (one block).
__device__ __forceinline__ void energy_reduce_block(const double* __restrict__ p_un, const double* __restrict__ p_un64,
                                                    const long long* __restrict__ p_cut, int nparts, double* out,
                                                    long long* out_cut) {
  __shared__ double r0[kBlock], r1[kBlock];
  __shared__ long long r2[kBlock];
  const int tid = threadIdx.x;
  double a0 = 0, a1 = 0;
  long long c0 = 0;
  // partials tid, tid + kBlock, ... in that order; their loads are issued 4 at a time
  int i = tid;
  for (; i + 3 * kBlock < nparts; i += 4 * kBlock) {
    double u0[4], u1[4];
    long long uc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      u0[u] = p_un[i + u * kBlock];
      u1[u] = p_un64[i + u * kBlock];
      uc[u] = p_cut[i + u * kBlock];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0 += u0[u];
      a1 += u1[u];
      c0 += uc[u];
    }
  }
  for (; i < nparts; i += kBlock) {
    a0 += p_un[i];
    a1 += p_un64[i];
    c0 += p_cut[i];
  }
  r0[tid] = a0;
  r1[tid] = a1;
  r2[tid] = c0;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      r0[tid] += r0[tid + w];
      r1[tid] += r1[tid + w];
      r2[tid] += r2[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
    *out_cut = r2[0];
  }
}

__global__ __launch_bounds__(kBlock) void energy_reduce_kernel(const double* __restrict__ p_un,
                                                               const double* __restrict__ p_un64,
                                                               const long long* __restrict__ p_cut, int nparts,
                                                               double* out, long long* out_cut,
                                                               const int32_t* moved, int L) {
  if (energy_skipped(moved, L)) return;
  energy_reduce_block(p_un, p_un64, p_cut, nparts, out, out_cut);
}

// one block per job
__global__ __launch_bounds__(kBlock) void energy_reduce_packed(const EnergyArgs* __restrict__ jobs,
                                                               const int32_t* __restrict__ start, int njobs) {
  const EnergyArgs& e = jobs[blockIdx.x];
  energy_reduce_block(e.part_un, e.part_un64, e.part_cut, start[blockIdx.x + 1] - start[blockIdx.x], e.out, e.out_cut);
}

__global__ __launch_bounds__(kRedBlock) void pass_reduce_kernel(const double* __restrict__ partial, int nparts,
                                                                IterState* st, double* trace, double* bound_out,
                                                                IterState* mirror) {
  reduce_pass<kRedBlock>(partial, nparts, st, trace, bound_out, mirror);
}

// one block per job
__global__ __launch_bounds__(kRedBlock) void pass_reduce_packed(const ReduceJob* __restrict__ jobs) {
  const ReduceJob r = jobs[blockIdx.x];
  reduce_pass<kRedBlock>(r.partial, r.nparts, r.state, r.trace, r.bound_out, nullptr);
}

__global__ void gather_rows_kernel(const float* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int L,
                                   int ldz, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * ldz) return;
  const int64_t r = i / ldz, l = i % ldz;
  const int64_t sr = perm ? perm[r] : r;
  dst[i] = l < L ? src[sr * L + l] : 0.f;
}

__global__ void scatter_rows_kernel(const float* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int L,
                                    int ldz, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * L) return;
  const int64_t r = i / L, l = i % L;
  const int64_t dr = perm ? perm[r] : r;
  dst[dr * L + l] = src[r * ldz + l];
}

// Internal rows of 4-float slices (ldz = 4 * L4) to the caller's layout: one thread per slice,
// 16-byte loads; two 8-byte stores where the destination row starts 8-byte aligned (L or the
// row index even) and the slice is whole, else one store per entry.
__global__ void scatter_rows4_kernel(const float* __restrict__ src, const int32_t* __restrict__ perm, uint32_t n,
                                     int L, uint32_t L4, float* __restrict__ dst) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * L4) return;
  const uint32_t r = i / L4, j = i - r * L4;
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(src) + i);
  const int64_t dr = perm ? perm[r] : r;
  float* d = dst + dr * L + 4 * j;
  const int l0 = 4 * (int)j;
  if (l0 + 3 < L && ((dr * L) & 1) == 0) {
    __builtin_nontemporal_store(vf2{v.x, v.y}, reinterpret_cast<vf2*>(d));
    __builtin_nontemporal_store(vf2{v.z, v.w}, reinterpret_cast<vf2*>(d + 2));
  } else {
    if (l0 < L) d[0] = v.x;
    if (l0 + 1 < L) d[1] = v.y;
    if (l0 + 2 < L) d[2] = v.z;
    if (l0 + 3 < L) d[3] = v.w;
  }
}

// Neighbour columns as byte offsets of Z rows (row bytes rb); the padding entries after the
// last column get the dead offset n * rb.
__global__ void col_offsets_kernel(const int32_t* __restrict__ col_idx, int64_t nnz, uint32_t rb, uint32_t dead,
                                   uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) out[i] = (uint32_t)col_idx[i] * rb;
  else if (i < nnz + kColPad) out[i] = dead;
}

// out[p[i]] = in[i]: labels from one order to the other (p = iperm: caller's -> internal;
// p = perm: internal -> caller's)
__global__ void permute_labels_kernel(const int32_t* __restrict__ in, const int32_t* __restrict__ p, int64_t n,
                                      int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[p ? p[i] : i] = in[i];
}

inline int lanes_for(int L) {
  if (L <= 4) return 4;
  if (L <= 8) return 8;
  if (L <= 16) return 16;
  if (L <= 32) return 32;
  return 64;
}

}  // namespace

int groups4(int L) {
  const int l4 = (ldz_for(L) + 3) / 4;
  return l4 <= 1 ? 1 : l4 <= 2 ? 2 : l4 <= 4 ? 4 : l4 <= 8 ? 8 : 16;
}

inline int64_t tile_grid(int64_t ntiles) { return 8 * ((std::max<int64_t>(ntiles, 1) + 7) / 8); }

int iter_grid(int64_t n, int32_t L, int64_t n_heavy, int32_t wsteps) {
  if (L <= 64) {
    const int64_t RW = 64 / groups4(L);
    const int64_t nbatch = (n + RW - 1) / RW;
    const int64_t TB = 4 * (wsteps > 0 ? wsteps : kWaveSteps);
    return heavy_blocks(n_heavy) + (int)tile_grid((nbatch + TB - 1) / TB);
  }
  const int64_t rows = 4 * (64 / lanes_for(L)) * kWaveSteps;
  return (int)tile_grid((n + rows - 1) / rows);
}

#define SLK_DISPATCH_G(G, KERNEL, ...)                                         \
  do {                                                                         \
    if (G == 1) hipLaunchKernelGGL((KERNEL<1>), __VA_ARGS__);                  \
    else if (G == 2) hipLaunchKernelGGL((KERNEL<2>), __VA_ARGS__);             \
    else if (G == 4) hipLaunchKernelGGL((KERNEL<4>), __VA_ARGS__);             \
    else if (G == 8) hipLaunchKernelGGL((KERNEL<8>), __VA_ARGS__);             \
    else hipLaunchKernelGGL((KERNEL<16>), __VA_ARGS__);                        \
  } while (0)

slk_status launch_iter_packed(int G, const IterArgs* jobs, const int32_t* start, int njobs, int blocks, hipStream_t s) {
  SLK_DISPATCH_G(G, iter4_packed, dim3((unsigned)blocks), dim3(kBlock), 0, s, jobs, start, njobs);
  SLK_LAUNCHED("iter4_packed");
  return SLK_OK;
}

slk_status launch_final_packed(int G, const FinalArgs* jobs, const int32_t* start, int njobs, int blocks,
                               hipStream_t s) {
  SLK_DISPATCH_G(G, final4_packed, dim3((unsigned)blocks), dim3(kBlock), 0, s, jobs, start, njobs);
  SLK_LAUNCHED("final4_packed");
  return SLK_OK;
}

slk_status launch_reduce_packed(const ReduceJob* jobs, int njobs, hipStream_t s) {
  hipLaunchKernelGGL(pass_reduce_packed, dim3((unsigned)njobs), dim3(kRedBlock), 0, s, jobs);
  SLK_LAUNCHED("pass_reduce_packed");
  return SLK_OK;
}

slk_status launch_mode_reduce_packed(const ModeJob* jobs, const int32_t* start, int njobs, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(mode_reduce_packed, dim3((unsigned)blocks), dim3(kBlock), 0, s, jobs, start, njobs);
  SLK_LAUNCHED("mode_reduce_packed");
  return SLK_OK;
}

// energy partials per job, then one reduction work-group per job (start gives each job's count)
slk_status launch_energy_packed(const EnergyArgs* jobs, const int32_t* start, int njobs, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(energy_packed, dim3((unsigned)blocks), dim3(kBlock), 0, s, jobs, start, njobs);
  SLK_LAUNCHED("energy_packed");
  hipLaunchKernelGGL(energy_reduce_packed, dim3((unsigned)njobs), dim3(kBlock), 0, s, jobs, start, njobs);
  SLK_LAUNCHED("energy_reduce_packed");
  return SLK_OK;
}

#define SLK_DISPATCH_LANES(L, KERNEL, ...)                                                   \
  do {                                                                                       \
    const int S_ = lanes_for(L);                                                             \
    if (L > 64) {                                                                            \
      const int E_ = (L + 63) / 64;                                                          \
      if (E_ == 2) hipLaunchKernelGGL((KERNEL<64, 2>), __VA_ARGS__);                         \
      else if (E_ == 3) hipLaunchKernelGGL((KERNEL<64, 3>), __VA_ARGS__);                    \
      else hipLaunchKernelGGL((KERNEL<64, 4>), __VA_ARGS__);                                 \
    } else if (S_ == 4) hipLaunchKernelGGL((KERNEL<4, 1>), __VA_ARGS__);                     \
    else if (S_ == 8) hipLaunchKernelGGL((KERNEL<8, 1>), __VA_ARGS__);                       \
    else if (S_ == 16) hipLaunchKernelGGL((KERNEL<16, 1>), __VA_ARGS__);                     \
    else if (S_ == 32) hipLaunchKernelGGL((KERNEL<32, 1>), __VA_ARGS__);                     \
    else hipLaunchKernelGGL((KERNEL<64, 1>), __VA_ARGS__);                                   \
  } while (0)

#define SLK_DISPATCH_G4(L, KERNEL, ...)                                        \
  do {                                                                         \
    const int G_ = groups4(L);                                                 \
    if (G_ == 1) hipLaunchKernelGGL((KERNEL<1>), __VA_ARGS__);                 \
    else if (G_ == 2) hipLaunchKernelGGL((KERNEL<2>), __VA_ARGS__);            \
    else if (G_ == 4) hipLaunchKernelGGL((KERNEL<4>), __VA_ARGS__);            \
    else if (G_ == 8) hipLaunchKernelGGL((KERNEL<8>), __VA_ARGS__);            \
    else hipLaunchKernelGGL((KERNEL<16>), __VA_ARGS__);                        \
  } while (0)

slk_status launch_iter(const IterArgs& a, int grid, hipStream_t s) {
  {
    KernelTimer kt("iter_kernel", s);
    if (a.L <= 64) SLK_DISPATCH_G4(a.L, iter4_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    else SLK_DISPATCH_LANES(a.L, iter_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    SLK_LAUNCHED("iter_kernel");
  }
  hipLaunchKernelGGL(pass_reduce_kernel, dim3(1), dim3(kRedBlock), 0, s, a.partial, grid, a.state, a.trace, a.bound_out,
                     a.mirror);
  SLK_LAUNCHED("pass_reduce_kernel");
  return SLK_OK;
}

int64_t iter_rows_per_group(int32_t L) { return 4 * (64 / lanes_for(L)) * kWaveSteps; }

int iter_grid_rows(int64_t n, int32_t L) {
  const int64_t rows = iter_rows_per_group(L);
  return (int)tile_grid((n + rows - 1) / rows);
}

slk_status launch_iter_rows(const IterArgs& a, int grid, hipStream_t s) {
  SLK_DISPATCH_LANES(a.L, iter_kernel, dim3(grid), dim3(kBlock), 0, s, a);
  SLK_LAUNCHED("iter_kernel");
  hipLaunchKernelGGL(pass_reduce_kernel, dim3(1), dim3(kRedBlock), 0, s, a.partial, grid, a.state, a.trace, a.bound_out,
                     a.mirror);
  SLK_LAUNCHED("pass_reduce_kernel");
  return SLK_OK;
}

slk_status launch_iter_emit(const FinalArgs& f0, int grid, hipStream_t s) {
  FinalArgs f = f0;
  f.grid = grid;
  const IterArgs& a = f.it;
  {
    KernelTimer kt("iter_kernel", s);
    SLK_DISPATCH_G4(a.L, iter4_emit_kernel, dim3(grid), dim3(kBlock), 0, s, f);
    SLK_LAUNCHED("iter_kernel");
  }
  hipLaunchKernelGGL(pass_reduce_kernel, dim3(1), dim3(kRedBlock), 0, s, a.partial, grid, a.state, a.trace, a.bound_out,
                     a.mirror);
  SLK_LAUNCHED("pass_reduce_kernel");
  return SLK_OK;
}

slk_status launch_final(const FinalArgs& f0, int grid, hipStream_t s) {
  FinalArgs f = f0;
  f.grid = grid;
  {
    KernelTimer kt("final_kernel", s);
    if (f.it.L <= 64) SLK_DISPATCH_G4(f.it.L, final4_kernel, dim3(grid), dim3(kBlock), 0, s, f);
    else SLK_DISPATCH_LANES(f.it.L, final_kernel, dim3(grid), dim3(kBlock), 0, s, f);
    SLK_LAUNCHED("final_kernel");
  }
  hipLaunchKernelGGL(pass_reduce_kernel, dim3(1), dim3(kRedBlock), 0, s, f.it.partial, grid, f.it.state, f.it.trace,
                     f.it.bound_out, f.it.mirror);
  SLK_LAUNCHED("pass_reduce_kernel");
  return SLK_OK;
}

slk_status launch_mode_reduce(const float* cand_v, const int32_t* cand_i, int grid, int32_t L, int32_t* modes_out,
                              hipStream_t s, int32_t* mirror, const int32_t* cur, int32_t* moved) {
  hipLaunchKernelGGL(mode_reduce_kernel, dim3(L), dim3(kBlock), 0, s, cand_v, cand_i, grid, L, modes_out, mirror, cur,
                     moved);
  SLK_LAUNCHED("mode_reduce_kernel");
  return SLK_OK;
}

int energy_grid(int64_t n, int64_t n_heavy) {
  const int64_t nbatch = (n + 3) / 4;
  return heavy_blocks(n_heavy) + (int)tile_grid((nbatch + 4 * kWaveSteps - 1) / (4 * kWaveSteps));
}

slk_status launch_energy(const EnergyArgs& a, int grid, hipStream_t s) {
  {
    KernelTimer kt("energy_kernel", s);
    hipLaunchKernelGGL(energy_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    SLK_LAUNCHED("energy_kernel");
  }
  hipLaunchKernelGGL(energy_reduce_kernel, dim3(1), dim3(kBlock), 0, s, a.part_un, a.part_un64, a.part_cut, grid, a.out,
                     a.out_cut, a.moved, a.L);
  SLK_LAUNCHED("energy_reduce_kernel");
  return SLK_OK;
}

slk_status launch_gather_rows(const float* src, const int32_t* perm, int64_t n, int32_t L, int32_t ldz, float* dst,
                              hipStream_t s) {
  const int64_t tot = n * ldz;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, perm, n, L, ldz,
                     dst);
  SLK_LAUNCHED("gather_rows_kernel");
  return SLK_OK;
}

slk_status launch_scatter_rows(const float* src, const int32_t* perm, int64_t n, int32_t L, int32_t ldz, float* dst,
                               hipStream_t s) {
  if (ldz == ldz_for(L) && ldz % 4 == 0 && n * (ldz / 4) < (int64_t)INT32_MAX) {
    const uint32_t L4 = (uint32_t)(ldz / 4);
    const int64_t slices = n * L4;
    hipLaunchKernelGGL(scatter_rows4_kernel, dim3((unsigned)((slices + 255) / 256)), dim3(256), 0, s, src, perm,
                       (uint32_t)n, L, L4, dst);
    SLK_LAUNCHED("scatter_rows4_kernel");
    return SLK_OK;
  }
  const int64_t tot = n * L;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, perm, n, L, ldz,
                     dst);
  SLK_LAUNCHED("scatter_rows_kernel");
  return SLK_OK;
}

slk_status launch_col_offsets(const int32_t* col_idx, int64_t nnz, int64_t n, int32_t L, uint32_t* out, hipStream_t s) {
  const uint32_t rb = (uint32_t)ldz_for(L) * 4u;
  const int64_t tot = nnz + kColPad;
  hipLaunchKernelGGL(col_offsets_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, col_idx, nnz, rb,
                     (uint32_t)n * rb, out);
  SLK_LAUNCHED("col_offsets_kernel");
  return SLK_OK;
}

slk_status launch_to_internal_labels(const int32_t* labels_user, const int32_t* iperm, int64_t n, int32_t* out,
                                     hipStream_t s) {
  hipLaunchKernelGGL(permute_labels_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, labels_user, iperm, n,
                     out);
  SLK_LAUNCHED("permute_labels_kernel");
  return SLK_OK;
}

slk_status launch_labels_to_user(const int32_t* labels_int, const int32_t* perm, int64_t n, int32_t* out,
                                 hipStream_t s) {
  return launch_to_internal_labels(labels_int, perm, n, out, s);
}

}  // namespace slk
