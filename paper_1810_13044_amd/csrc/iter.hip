// Kernels of the SLK-BO iteration for CDNA4 (gfx950, wave64).
//
//   unary_kernel   a_pl = k(x_p, m_l) and z^0_p = softmax(a_p)            (Eq. (6a), Algorithm 1)
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
// unary affinities
// ------------------------------------------------------------------------------------------
constexpr int kUDcMax = 64;  // coordinates per LDS chunk (32 when L > 128)
constexpr int kUPairs = 8;   // (row, cluster) pairs per thread

__global__ __launch_bounds__(kBlock) void unary_kernel(const float* __restrict__ x, int64_t n, int d,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ modes, int L, int R,
                                                       int kUDc, float inv2s2, int bf16, float* __restrict__ A,
                                                       float* __restrict__ Z0) {
  extern __shared__ float sm[];
  float* xs = sm;                         // R x (kUDc+1)
  float* ms = xs + R * (kUDc + 1);        // L x (kUDc+1)
  float* as = ms + L * (kUDc + 1);        // R x L
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int nr = (int)min<int64_t>(R, n - row0);
  const int npairs = R * L;
  float acc[kUPairs];
#pragma unroll
  for (int k = 0; k < kUPairs; ++k) acc[k] = 0.f;

  for (int c0 = 0; c0 < d; c0 += kUDc) {
    const int dc = min(kUDc, d - c0);
    for (int e = tid; e < R * kUDc; e += kBlock) {
      const int r = e / kUDc, j = e % kUDc;
      float v = 0.f;
      if (r < nr && j < dc) {
        const int64_t gr = perm ? perm[row0 + r] : row0 + r;
        v = x[gr * d + c0 + j];
        if (bf16) v = bf16_round(v);
      }
      xs[r * (kUDc + 1) + j] = v;
    }
    for (int e = tid; e < L * kUDc; e += kBlock) {
      const int l = e / kUDc, j = e % kUDc;
      float v = 0.f;
      if (j < dc) {
        v = x[(int64_t)modes[l] * d + c0 + j];
        if (bf16) v = bf16_round(v);
      }
      ms[l * (kUDc + 1) + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kUPairs; ++k) {
      const int pr = tid + k * kBlock;
      if (pr < npairs) {
        const int r = pr / L, l = pr % L;
        const float* xr = xs + r * (kUDc + 1);
        const float* mr = ms + l * (kUDc + 1);
        float part = 0.f;  // one chunk summed on its own, then added: two-level summation
        for (int j = 0; j < dc; ++j) {
          const float t = xr[j] - mr[j];
          part = fmaf(t, t, part);
        }
        acc[k] += part;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kUPairs; ++k) {
    const int pr = tid + k * kBlock;
    if (pr < npairs) as[pr] = expf(-acc[k] * inv2s2);
  }
  __syncthreads();
  // row softmax of a_p gives z^0_p; one wave per row
  const int wave = tid >> 6, lane = tid & 63;
  for (int r = wave; r < nr; r += kBlock / 64) {
    float m = -FLT_MAX;
    for (int l = lane; l < L; l += 64) m = fmaxf(m, as[r * L + l]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    float s = 0.f;
    for (int l = lane; l < L; l += 64) s += expf(as[r * L + l] - m);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const int64_t row = row0 + r;
    for (int l = lane; l < L; l += 64) {
      const float a = as[r * L + l];
      if (A) A[row * L + l] = a;
      if (Z0) Z0[row * L + l] = expf(a - m) / s;
    }
  }
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

// Computes one row inside its S-lane group.  All lanes of the group must call it together.
template <int S, int E>
__device__ __forceinline__ void row_update(const IterArgs& a, int64_t row, int l0, RowOut<S, E>& o) {
  const int L = a.L;
  float zp[E], av[E], b[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int l = l0 + S * e;
    const bool ok = l < L;
    av[e] = ok ? a.A[row * L + l] : 0.f;
    zp[e] = ok ? a.Zin[row * L + l] : 0.f;
    b[e] = 0.f;
  }
  const int32_t beg = a.row_ptr[row], end = a.row_ptr[row + 1];
  for (int32_t c = beg; c < end; c += S) {
    const int cnt = min(S, end - c);
    const int myq = (l0 < cnt) ? a.col_idx[c + l0] : 0;
    int t = 0;
    for (; t + 4 <= cnt; t += 4) {
      const int64_t q0 = __shfl(myq, t, S), q1 = __shfl(myq, t + 1, S);
      const int64_t q2 = __shfl(myq, t + 2, S), q3 = __shfl(myq, t + 3, S);
      float v0[E], v1[E], v2[E], v3[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int l = l0 + S * e;
        const bool ok = l < L;
        v0[e] = ok ? a.Zin[q0 * L + l] : 0.f;
        v1[e] = ok ? a.Zin[q1 * L + l] : 0.f;
        v2[e] = ok ? a.Zin[q2 * L + l] : 0.f;
        v3[e] = ok ? a.Zin[q3 * L + l] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        b[e] += v0[e];
        b[e] += v1[e];
        b[e] += v2[e];
        b[e] += v3[e];
      }
    }
    for (; t < cnt; ++t) {
      const int64_t q = __shfl(myq, t, S);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int l = l0 + S * e;
        b[e] += (l < L) ? a.Zin[q * L + l] : 0.f;
      }
    }
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

// Block-level fixed-order reduction of per-group bound partials, then the grid-level
// "last block finishes" reduction with the convergence test.
template <int G>
__device__ __forceinline__ void finish_pass(const IterArgs& a, double acc, int g, int l0) {
  __shared__ double red[4 * G];
  __shared__ double red2[kBlock];
  __shared__ int is_last;
  const int tid = threadIdx.x, wave = tid >> 6;
  if (l0 == 0) red[wave * G + g] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < 4 * G; ++i) s += red[i];
    a.partial[blockIdx.x] = s;
    __threadfence();
    const unsigned prev = atomicAdd(&a.state->arrive, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double v = 0.0;
  for (int i = tid; i < (int)gridDim.x; i += kBlock) v += load_agent(a.partial + i);
  red2[tid] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) red2[tid] += red2[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    IterState* st = a.state;
    const double R = red2[0];
    const int pass = st->pass;
    if (a.trace && pass < st->trace_cap) a.trace[pass] = R;
    if (a.bound_out) *a.bound_out = R;
    if (!isfinite(R)) {
      st->numeric = 1;
      st->done = 1;
    } else if (st->check && pass >= 1 && fabs(R - st->last_bound) <= st->tol * fabs(st->last_bound)) {
      st->done = 1;
    }
    st->last_bound = R;
    st->pass = pass + 1;
    st->arrive = 0u;
    __threadfence();
  }
}

template <int S, int E>
__global__ __launch_bounds__(kBlock) void iter_kernel(IterArgs a) {
  if (a.state->done) return;
  constexpr int G = 64 / S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / S, l0 = lane % S;
  const int64_t stride = (int64_t)gridDim.x * 4 * G;
  double acc = 0.0;
  for (int64_t row = ((int64_t)blockIdx.x * 4 + wave) * G + g; row < a.n; row += stride) {
    RowOut<S, E> o;
    row_update<S, E>(a, row, l0, o);
    if (a.Zout) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int l = l0 + S * e;
        if (l < a.L) a.Zout[row * a.L + l] = o.z[e];
      }
    }
    acc += (double)o.r;
  }
  finish_pass<G>(a, acc, g, l0);
}

// final pass: labels, log-odds candidates, output Z in the caller's order
template <int S, int E>
__global__ __launch_bounds__(kBlock) void final_kernel(FinalArgs f) {
  const IterArgs& a = f.it;
  constexpr int G = 64 / S;
  const int L = a.L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / S, l0 = lane % S;
  const int64_t stride = (int64_t)gridDim.x * 4 * G;
  float bv[E];
  int bi[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    bv[e] = -INFINITY;
    bi[e] = INT32_MAX;
  }
  double acc = 0.0;
  for (int64_t row = ((int64_t)blockIdx.x * 4 + wave) * G + g; row < a.n; row += stride) {
    RowOut<S, E> o;
    row_update<S, E>(a, row, l0, o);
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
    const int jt = ti;
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
        v = (o.s[e] - o.m) - log1pf(T - o.e[e]);
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
  }
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
    f.cand_v[(int64_t)blockIdx.x * L + l] = v;
    f.cand_i[(int64_t)blockIdx.x * L + l] = i;
  }
  finish_pass<G>(a, acc, g, l0);
}

__global__ __launch_bounds__(kBlock) void mode_reduce_kernel(const float* __restrict__ cv, const int32_t* __restrict__ ci,
                                                             int grid, int L, int32_t* __restrict__ modes) {
  const int l = blockIdx.x, tid = threadIdx.x;
  float v = -INFINITY;
  int i = INT32_MAX;
  for (int b = tid; b < grid; b += kBlock) {
    const float ov = cv[(int64_t)b * L + l];
    const int oi = ci[(int64_t)b * L + l];
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
  if (tid == 0) modes[l] = si[0] == INT32_MAX ? 0 : si[0];
}

// ------------------------------------------------------------------------------------------
// energy: FP32 unary term, exact cut count and an FP64 recheck of the unary term
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void energy_kernel(EnergyArgs e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tid = threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 4;
  double un = 0.0, un64 = 0.0;
  long long cut = 0;
  for (int64_t row = (int64_t)blockIdx.x * 4 + wave; row < e.n; row += stride) {
    const int lab = e.labels_int[row];
    const int32_t beg = e.row_ptr[row], end = e.row_ptr[row + 1];
    int c = 0;
    for (int32_t j = beg + lane; j < end; j += 64) c += (e.labels_int[e.col_idx[j]] != lab);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (e.x) {
      const int64_t orow = e.perm ? e.perm[row] : row;
      const float* xp = e.x + orow * e.d;
      const float* mp = e.x + (int64_t)e.modes[lab] * e.d;
      double s = 0.0;
      for (int j = lane; j < e.d; j += 64) {
        const double t = (double)xp[j] - (double)mp[j];
        s += t * t;
      }
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      if (lane == 0) un64 += exp(-s * e.inv2s2);
    }
    if (lane == 0) {
      un += (double)e.A[row * e.L + lab];
      cut += c;
    }
  }
  __shared__ double s_un[4], s_un64[4];
  __shared__ long long s_cut[4];
  __shared__ int is_last;
  if (lane == 0) {
    s_un[wave] = un;
    s_un64[wave] = un64;
    s_cut[wave] = cut;
  }
  __syncthreads();
  if (tid == 0) {
    double a0 = 0, a1 = 0;
    long long c0 = 0;
    for (int w = 0; w < 4; ++w) {
      a0 += s_un[w];
      a1 += s_un64[w];
      c0 += s_cut[w];
    }
    e.part_un[blockIdx.x] = a0;
    e.part_un64[blockIdx.x] = a1;
    e.part_cut[blockIdx.x] = c0;
    __threadfence();
    is_last = (atomicAdd(e.arrive, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  __shared__ double r0[kBlock], r1[kBlock];
  __shared__ long long r2[kBlock];
  double a0 = 0, a1 = 0;
  long long c0 = 0;
  for (int i = tid; i < (int)gridDim.x; i += kBlock) {
    a0 += load_agent(e.part_un + i);
    a1 += load_agent(e.part_un64 + i);
    c0 += load_agent(e.part_cut + i);
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
    e.out[0] = r0[0];
    e.out[1] = r1[0];
    *e.out_cut = r2[0];
    *e.arrive = 0u;
  }
}

__global__ void gather_rows_kernel(const float* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int L,
                                   float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * L) return;
  const int64_t r = i / L, l = i % L;
  dst[i] = src[(int64_t)perm[r] * L + l];
}

__global__ void scatter_rows_kernel(const float* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int L,
                                    float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * L) return;
  const int64_t r = i / L, l = i % L;
  dst[(int64_t)perm[r] * L + l] = src[i];
}

__global__ void labels_to_internal_kernel(const int32_t* __restrict__ lu, const int32_t* __restrict__ iperm,
                                          int64_t n, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[iperm ? iperm[i] : i] = lu[i];
}

inline int lanes_for(int L) {
  if (L <= 4) return 4;
  if (L <= 8) return 8;
  if (L <= 16) return 16;
  if (L <= 32) return 32;
  return 64;
}

}  // namespace

int iter_grid(int64_t n, int32_t L) {
  const int S = lanes_for(L);
  const int64_t rows_per_block = 4 * (64 / S);
  const int64_t need = (n + rows_per_block - 1) / rows_per_block;
  // enough blocks to fill 256 CUs several times over; rows beyond are grid-strided
  return (int)std::max<int64_t>(1, std::min<int64_t>(need, 256 * 16));
}

slk_status launch_unary(const float* x, int64_t n, int32_t d, const int32_t* perm, const int32_t* modes_dev, int32_t L,
                        double sigma2, int32_t bf16, float* A, float* Z0, hipStream_t s) {
  const int R = std::max(1, std::min(32, (kUPairs * kBlock) / L));
  const int dcw = L > 128 ? kUDcMax / 2 : kUDcMax;
  const size_t lds = sizeof(float) * ((size_t)R * (dcw + 1) + (size_t)L * (dcw + 1) + (size_t)R * L);
  const int64_t grid = (n + R - 1) / R;
  const float inv2s2 = (float)(1.0 / (2.0 * sigma2));
  hipLaunchKernelGGL(unary_kernel, dim3((unsigned)grid), dim3(kBlock), lds, s, x, n, d, perm, modes_dev, L, R, dcw,
                     inv2s2, bf16, A, Z0);
  SLK_LAUNCHED("unary_kernel");
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

slk_status launch_iter(const IterArgs& a, int grid, hipStream_t s) {
  SLK_DISPATCH_LANES(a.L, iter_kernel, dim3(grid), dim3(kBlock), 0, s, a);
  SLK_LAUNCHED("iter_kernel");
  return SLK_OK;
}

slk_status launch_final(const FinalArgs& f, int grid, hipStream_t s) {
  SLK_DISPATCH_LANES(f.it.L, final_kernel, dim3(grid), dim3(kBlock), 0, s, f);
  SLK_LAUNCHED("final_kernel");
  return SLK_OK;
}

slk_status launch_mode_reduce(const float* cand_v, const int32_t* cand_i, int grid, int32_t L, int32_t* modes_out,
                              hipStream_t s) {
  hipLaunchKernelGGL(mode_reduce_kernel, dim3(L), dim3(kBlock), 0, s, cand_v, cand_i, grid, L, modes_out);
  SLK_LAUNCHED("mode_reduce_kernel");
  return SLK_OK;
}

int energy_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, 256 * 8)); }

slk_status launch_energy(const EnergyArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(grid), dim3(kBlock), 0, s, a);
  SLK_LAUNCHED("energy_kernel");
  return SLK_OK;
}

slk_status launch_gather_rows(const float* src, const int32_t* perm, int64_t n, int32_t L, float* dst, hipStream_t s) {
  const int64_t tot = n * L;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, perm, n, L, dst);
  SLK_LAUNCHED("gather_rows_kernel");
  return SLK_OK;
}

slk_status launch_scatter_rows(const float* src, const int32_t* perm, int64_t n, int32_t L, float* dst,
                               hipStream_t s) {
  const int64_t tot = n * L;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, perm, n, L, dst);
  SLK_LAUNCHED("scatter_rows_kernel");
  return SLK_OK;
}

slk_status launch_to_internal_labels(const int32_t* labels_user, const int32_t* iperm, int64_t n, int32_t* out,
                                     hipStream_t s) {
  hipLaunchKernelGGL(labels_to_internal_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, labels_user, iperm,
                     n, out);
  SLK_LAUNCHED("labels_to_internal_kernel");
  return SLK_OK;
}

}  // namespace slk
