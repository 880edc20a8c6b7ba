// Construction of the kNN affinity of Section 4.2 on the GPU.
//
//   knn_exact_kernel  every distance in FP64 with the fixed coordinate order (no fused
//                     multiply-add), top-k by (distance, index) per query row
//   CSR build         OR-symmetrisation of the kNN lists: count, scan, scatter, per-row
//                     sort, de-duplication and compaction
//   relabel           applies a locality permutation to the CSR
//   sum_f64           fixed-order FP64 sum (sigma^2 from the kNN squared distances)
#include "common.h"

#include <type_traits>

#include <float.h>
#include <math.h>

#include <algorithm>
#include <vector>

namespace slk {

namespace {

constexpr int kBlock = 256;


// One step of the reference distance: acc + (a - b)^2 with the subtraction, the square and
// the addition each rounded to FP64 (never fused into a multiply-add).
__device__ __forceinline__ double sqdist_step(double acc, double a, double b) {
#pragma clang fp contract(off)
  const double t = a - b;
  const double t2 = t * t;
  return acc + t2;
}

// (d, q) < (d', q') in the lexicographic order used for neighbours
__device__ __forceinline__ bool key_less(double d0, int q0, double d1, int q1) {
  return d0 < d1 || (d0 == d1 && q0 < q1);
}

// ------------------------------------------------------------------------------------------
// exact kNN: QB query rows per block, keys streamed 256 at a time (one key per thread)
// ------------------------------------------------------------------------------------------
// Queries per block: 4 while the keys fit in one XCD's L2 (4 MiB), so that key reads are L2 hits
// and twice the blocks (less LDS each, more per CU) hide their latency, or while the wide grid
// would have fewer than two blocks per CU; otherwise 8, halving the key reads that go past L2.
constexpr int kQBWide = 8, kQBNarrow = 4;
constexpr int kQDc = 256;   // query coordinates staged per chunk
constexpr int kSortP = 512; // bitonic width of a merge (k + 256 <= 320 entries)

// Block-wide bitonic sort of P (power of two) (d, q) pairs in LDS.
__device__ void block_bitonic(double* kd, int* kq, int P) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const double d0 = kd[lo], d1 = kd[hi];
        const int q0 = kq[lo], q1 = kq[hi];
        const bool swap = up ? key_less(d1, q1, d0, q0) : key_less(d0, q0, d1, q1);
        if (swap) {
          kd[lo] = d1;
          kd[hi] = d0;
          kq[lo] = q1;
          kq[hi] = q0;
        }
      }
      __syncthreads();
    }
  }
}

// Queries are rows of x (rows[] or all, the point itself excluded) or, with y, the rows of y
// (nothing excluded).  The result does not depend on kQB.
template <int kQB>
__device__ __forceinline__ void knn_exact_block(const float* __restrict__ x, int64_t n, int d, int k, int bf16,
                                                const int32_t* __restrict__ rows, int64_t n_rows,
                                                int32_t* __restrict__ out_idx, double* __restrict__ out_d2,
                                                const float* __restrict__ y, int64_t bid) {
  const float* __restrict__ qsrc = y ? y : x;
  const bool vec4 = (d & 3) == 0 && ((uintptr_t)x & 15) == 0;
  __shared__ double qs[kQB][kQDc];
  __shared__ double ld[kQB][64];
  __shared__ int lq[kQB][64];
  __shared__ double bd[kQB][kBlock];
  __shared__ int bq[kQB][kBlock];
  __shared__ int bcnt[kQB];
  __shared__ double sd[kSortP];
  __shared__ int sq[kSortP];
  const int tid = threadIdx.x;
  const int64_t r0 = bid * kQB;
  const int nq = (int)min<int64_t>(kQB, n_rows - r0);
  __shared__ int64_t qrow[kQB];
  if (tid < kQB) qrow[tid] = (tid < nq) ? (rows ? rows[r0 + tid] : r0 + tid) : -1;
  for (int e = tid; e < kQB * 64; e += kBlock) {
    ld[e / 64][e % 64] = INFINITY;
    lq[e / 64][e % 64] = INT32_MAX;
  }
  if (tid < kQB) bcnt[tid] = 0;
  __syncthreads();

  // the queries' coordinates c0 .. c0 + kQDc - 1 into qs (zeros past d and past the last query)
  auto stage_queries = [&](int c0, int dc) __attribute__((always_inline)) {
    for (int e = tid; e < kQB * kQDc; e += kBlock) {
      const int i = e / kQDc, j = e % kQDc;
      double v = 0.0;
      if (i < nq && j < dc) {
        float f = qsrc[qrow[i] * d + c0 + j];
        if (bf16) f = bf16_round(f);
        v = (double)f;
      }
      qs[i][j] = v;
    }
  };
  // with one chunk (d <= kQDc: every served job's width) the queries are staged once for all key
  // blocks; re-staging them for each block had cost two barriers and a round of loads per block
  const bool one_chunk = d <= kQDc;
  if (one_chunk) {
    stage_queries(0, d);
    __syncthreads();
  }
  for (int64_t k0 = 0; k0 < n; k0 += kBlock) {
    const int64_t q = k0 + tid;
    double acc[kQB];
#pragma unroll
    for (int i = 0; i < kQB; ++i) acc[i] = 0.0;
    for (int c0 = 0; c0 < d; c0 += kQDc) {
      const int dc = min(kQDc, d - c0);
      if (!one_chunk) {
        __syncthreads();
        stage_queries(c0, dc);
        __syncthreads();
      }
      if (q < n) {
        const float* xq = x + q * d + c0;
        // the key's coordinates in order; 16 bytes per load where rows allow it (each thread
        // walks its own row, so single floats re-fetch every cache line from L2 up to 16 times),
        // four such loads issued together before their coordinates are used (one at a time, each
        // load's latency stood between two groups of FP64 updates)
        auto scan = [&](auto bf_c) __attribute__((always_inline)) {
          constexpr bool BF = decltype(bf_c)::value;
          auto coord = [&](float f, int jj) __attribute__((always_inline)) {
            if (BF) f = bf16_round(f);
            const double xv = (double)f;
#pragma unroll
            for (int i = 0; i < kQB; ++i) acc[i] = sqdist_step(acc[i], qs[i][jj], xv);
          };
          int j = 0;
          if (vec4) {
            for (; j + 16 <= dc; j += 16) {
              float4 f4[4];
#pragma unroll
              for (int w = 0; w < 4; ++w) f4[w] = *reinterpret_cast<const float4*>(xq + j + 4 * w);
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                coord(f4[w].x, j + 4 * w);
                coord(f4[w].y, j + 4 * w + 1);
                coord(f4[w].z, j + 4 * w + 2);
                coord(f4[w].w, j + 4 * w + 3);
              }
            }
            for (; j + 4 <= dc; j += 4) {
              const float4 f4 = *reinterpret_cast<const float4*>(xq + j);
              coord(f4.x, j);
              coord(f4.y, j + 1);
              coord(f4.z, j + 2);
              coord(f4.w, j + 3);
            }
          }
          for (; j < dc; ++j) coord(xq[j], j);
        };
        if (bf16) scan(std::true_type{});
        else scan(std::false_type{});
      }
    }
    // filter against the current k-th best of each query
#pragma unroll
    for (int i = 0; i < kQB; ++i) {
      if (i < nq && q < n && (y || q != qrow[i]) && key_less(acc[i], (int)q, ld[i][k - 1], lq[i][k - 1])) {
        const int pos = atomicAdd(&bcnt[i], 1);
        bd[i][pos] = acc[i];
        bq[i][pos] = (int)q;
      }
    }
    __syncthreads();
    for (int i = 0; i < nq; ++i) {
      const int cnt = bcnt[i];
      if (cnt == 0) continue;
      int P = 1;
      while (P < k + cnt) P <<= 1;
      for (int e = tid; e < P; e += kBlock) {
        if (e < k) {
          sd[e] = ld[i][e];
          sq[e] = lq[i][e];
        } else if (e < k + cnt) {
          sd[e] = bd[i][e - k];
          sq[e] = bq[i][e - k];
        } else {
          sd[e] = INFINITY;
          sq[e] = INT32_MAX;
        }
      }
      __syncthreads();
      block_bitonic(sd, sq, P);
      for (int e = tid; e < k; e += kBlock) {
        ld[i][e] = sd[e];
        lq[i][e] = sq[e];
      }
      if (tid == 0) bcnt[i] = 0;
      __syncthreads();
    }
    // the next block's filter writes bcnt, bd and bq: every thread must be past this block's
    // merges first (with several chunks the staging barrier at the top of the block does this)
    if (one_chunk) __syncthreads();
  }
  for (int e = tid; e < nq * k; e += kBlock) {
    const int i = e / k, j = e % k;
    out_idx[qrow[i] * k + j] = lq[i][j];
    out_d2[qrow[i] * k + j] = ld[i][j];
  }
}

template <int kQB>
__global__ __launch_bounds__(kBlock) void knn_exact_kernel(const float* __restrict__ x, int64_t n, int d, int k,
                                                           int bf16, const int32_t* __restrict__ rows,
                                                           int64_t n_rows, int32_t* __restrict__ out_idx,
                                                           double* __restrict__ out_d2, const float* __restrict__ y) {
  knn_exact_block<kQB>(x, n, d, k, bf16, rows, n_rows, out_idx, out_d2, y, blockIdx.x);
}

// Several problems in one launch: start[j] is the first work-group of job j (njobs + 1 entries);
// every job's work-groups run exactly the single-problem kernel's code on its own points.
template <int kQB>
__global__ __launch_bounds__(kBlock) void knn_exact_packed(const KnnExactJob* __restrict__ jobs,
                                                           const int32_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const KnnExactJob& J = jobs[j];
  knn_exact_block<kQB>(J.x, J.n, J.d, J.k, J.bf16, nullptr, J.n, J.out_idx, J.out_d2, nullptr,
                       (int64_t)blockIdx.x - start[j]);
}

// ------------------------------------------------------------------------------------------
// scans and reductions
// ------------------------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int t = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  const int incl = sh[tid];
  *total = sh[kBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kBlock) void scan_tile_sums(const int32_t* __restrict__ in, int64_t count,
                                                         int32_t* __restrict__ sums) {
  __shared__ int sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int v = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < count) v += in[idx];
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

// exclusive scan of the tile sums by one block, chunk after chunk with a carry
__global__ __launch_bounds__(kBlock) void scan_sums_kernel(int32_t* __restrict__ sums, int64_t nt,
                                                           int32_t* __restrict__ total_out) {
  __shared__ int sh[kBlock];
  int carry = 0;
  for (int64_t c = 0; c < nt; c += kBlock) {
    const int64_t i = c + threadIdx.x;
    const int v = i < nt ? sums[i] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, sh, &tot);
    if (i < nt) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kBlock) void scan_apply(const int32_t* __restrict__ in, int64_t count,
                                                     const int32_t* __restrict__ sums, int32_t* __restrict__ out) {
  __shared__ int sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int vals[kScanItems];
  int v = 0;
  for (int i = 0; i < kScanItems; ++i) {
    vals[i] = (base + i < count) ? in[base + i] : 0;
    v += vals[i];
  }
  int tot;
  int run = block_exclusive_scan(v, sh, &tot) + sums[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < count) out[base + i] = run;
    run += vals[i];
  }
}

__global__ __launch_bounds__(kBlock) void sum_f64_kernel(const double* __restrict__ v, int64_t count,
                                                         double* __restrict__ part, double* __restrict__ out,
                                                         uint32_t* arrive) {
  __shared__ double sh[kBlock];
  __shared__ int is_last;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sh[0];
    __threadfence();
    is_last = atomicAdd(arrive, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double t = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kBlock)
    t += __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out = sh[0];
    *arrive = 0u;
  }
}

// ------------------------------------------------------------------------------------------
// CSR from kNN lists (OR rule)
// ------------------------------------------------------------------------------------------
__global__ void count_edges_kernel(const int32_t* __restrict__ knn, int64_t n, int k, int32_t* __restrict__ cap) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int own = 0;
  for (int j = 0; j < k; ++j) {
    const int q = knn[p * k + j];
    if (q != p) {
      ++own;
      atomicAdd(&cap[q], 1);
    }
  }
  atomicAdd(&cap[p], own);
}

__global__ void fill_edges_kernel(const int32_t* __restrict__ knn, int64_t n, int k, const int32_t* __restrict__ off,
                                  int32_t* __restrict__ fill, int32_t* __restrict__ cols) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  for (int j = 0; j < k; ++j) {
    const int q = knn[p * k + j];
    if (q != p) {
      cols[off[p] + atomicAdd(&fill[p], 1)] = q;
      cols[off[q] + atomicAdd(&fill[q], 1)] = (int)p;
    }
  }
}

// one wave per row, rows of up to 64 entries: bitonic sort across lanes
__global__ __launch_bounds__(kBlock) void sort_small_kernel(const int32_t* __restrict__ row_ptr, int64_t n,
                                                            int32_t* __restrict__ cols, int32_t* __restrict__ long_rows,
                                                            int32_t* __restrict__ n_long) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int beg = row_ptr[row], len = row_ptr[row + 1] - beg;
  if (len > 64) {
    if (lane == 0) long_rows[atomicAdd(n_long, 1)] = (int)row;
    return;
  }
  if (len <= 1) return;
  int v = lane < len ? cols[beg + lane] : INT32_MAX;
  for (int size = 2; size <= 64; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int o = __shfl_xor(v, stride);
      const bool up = ((lane & size) == 0);
      const bool lower = ((lane & stride) == 0);
      const int mn = min(v, o), mx = max(v, o);
      v = (up == lower) ? mn : mx;
    }
  }
  if (lane < len) cols[beg + lane] = v;
}

// one block per long row: bitonic sort in LDS (rows up to kBigSort entries) or in a global
// scratch area (longer rows; one row per launch)
constexpr int kBigSort = 8192;

__device__ void bitonic_int(int* a, int P) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const int x0 = a[lo], x1 = a[hi];
        if ((x0 > x1) == up) {
          a[lo] = x1;
          a[hi] = x0;
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kBlock) void sort_long_kernel(const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ rows, int32_t* __restrict__ cols,
                                                           int32_t* __restrict__ scratch) {
  __shared__ int sh[kBigSort];
  const int row = rows[blockIdx.x];
  const int beg = row_ptr[row], len = row_ptr[row + 1] - beg;
  int P = 1;
  while (P < len) P <<= 1;
  int* a = (P <= kBigSort) ? sh : scratch;
  for (int e = threadIdx.x; e < P; e += blockDim.x) a[e] = e < len ? cols[beg + e] : INT32_MAX;
  __syncthreads();
  bitonic_int(a, P);
  for (int e = threadIdx.x; e < len; e += blockDim.x) cols[beg + e] = a[e];
}

// distinct entries per sorted row
__global__ __launch_bounds__(kBlock) void unique_count_kernel(const int32_t* __restrict__ row_ptr, int64_t n,
                                                              const int32_t* __restrict__ cols,
                                                              int32_t* __restrict__ uniq) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int beg = row_ptr[row], end = row_ptr[row + 1];
  int c = 0;
  for (int j = beg + lane; j < end; j += 64) c += (j == beg || cols[j] != cols[j - 1]);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane == 0) uniq[row] = c;
}

__global__ __launch_bounds__(kBlock) void unique_copy_kernel(const int32_t* __restrict__ row_ptr, int64_t n,
                                                             const int32_t* __restrict__ cols,
                                                             const int32_t* __restrict__ out_ptr,
                                                             int32_t* __restrict__ out_cols) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int beg = row_ptr[row], end = row_ptr[row + 1];
  int base = out_ptr[row];
  for (int j0 = beg; j0 < end; j0 += 64) {
    const int j = j0 + lane;
    const bool keep = j < end && (j == beg || cols[j] != cols[j - 1]);
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (keep) out_cols[base + before] = cols[j];
    base += __popcll(m);
  }
}

__global__ void row_lengths_kernel(const int32_t* __restrict__ row_ptr, int64_t n, const int32_t* __restrict__ perm,
                                   int32_t* __restrict__ len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = perm ? perm[i] : i;
  len[i] = row_ptr[r + 1] - row_ptr[r];
}

__global__ __launch_bounds__(kBlock) void relabel_copy_kernel(const int32_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ cols, int64_t n,
                                                              const int32_t* __restrict__ perm,
                                                              const int32_t* __restrict__ iperm,
                                                              const int32_t* __restrict__ new_ptr,
                                                              int32_t* __restrict__ new_cols) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t r = perm[i];
  const int beg = row_ptr[r], end = row_ptr[r + 1];
  const int nb = new_ptr[i];
  for (int j = beg + lane; j < end; j += 64) new_cols[nb + (j - beg)] = iperm[cols[j]];
}

__global__ void degree_minmax_kernel(const int32_t* __restrict__ row_ptr, int64_t n, int32_t* out) {
  int mn = INT32_MAX, mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int l = row_ptr[i + 1] - row_ptr[i];
    mn = min(mn, l);
    mx = max(mx, l);
  }
  atomicMin(&out[0], mn);
  atomicMax(&out[1], mx);
}

__global__ void init_minmax_kernel(int32_t* out) {
  out[0] = INT32_MAX;
  out[1] = 0;
}

__global__ void set_last_kernel(int32_t* arr, int64_t pos, const int32_t* total) { arr[pos] = *total; }

// zero padding after the last column entry, and the entry count
__global__ void csr_tail_kernel(const int32_t* __restrict__ rp, int64_t n, int32_t* __restrict__ ci,
                                int32_t* __restrict__ nnz_out) {
  const int32_t nnz = rp[n];
  if (threadIdx.x < kColPad) ci[(int64_t)nnz + threadIdx.x] = 0;
  if (threadIdx.x == 0 && nnz_out) *nnz_out = nnz;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------------
slk_status knn_exact(const float* x, int64_t n, int32_t d, int32_t k, int32_t bf16, const int32_t* rows,
                     int64_t n_rows, int32_t* out_idx, double* out_d2, hipStream_t s, const float* y) {
  if (n_rows <= 0) return SLK_OK;
  if (k > 64) return fail(SLK_ERR_INVALID_ARG, "k > 64");
  if (tune_knn_width(n, d, n_rows) == kQBNarrow) {
    const int64_t grid = (n_rows + kQBNarrow - 1) / kQBNarrow;
    hipLaunchKernelGGL(knn_exact_kernel<kQBNarrow>, dim3((unsigned)grid), dim3(kBlock), 0, s, x, n, d, k, bf16, rows,
                       n_rows, out_idx, out_d2, y);
  } else {
    const int64_t grid = (n_rows + kQBWide - 1) / kQBWide;
    hipLaunchKernelGGL(knn_exact_kernel<kQBWide>, dim3((unsigned)grid), dim3(kBlock), 0, s, x, n, d, k, bf16, rows,
                       n_rows, out_idx, out_d2, y);
  }
  SLK_LAUNCHED("knn_exact_kernel");
  return SLK_OK;
}

slk_status knn_exact_group(const KnnExactJob* jobs_host, int njobs, hipStream_t s) {
  if (njobs <= 0) return SLK_OK;
  std::vector<int32_t> start(njobs + 1);
  int64_t b = 0;
  for (int j = 0; j < njobs; ++j) {
    if (jobs_host[j].k > 64) return fail(SLK_ERR_INVALID_ARG, "k > 64");
    start[j] = (int32_t)b;
    b += (jobs_host[j].n + kQBNarrow - 1) / kQBNarrow;
    if (b >= (int64_t)INT32_MAX) return fail(SLK_ERR_INVALID_ARG, "too many rows in one grouped search");
  }
  start[njobs] = (int32_t)b;
  Scratch sc(s);
  KnnExactJob* jd;
  int32_t* sd;
  SLK_TRY(sc.get(&jd, njobs));
  SLK_TRY(sc.get(&sd, njobs + 1));
  SLK_HIP(hipMemcpyAsync(jd, jobs_host, sizeof(KnnExactJob) * njobs, hipMemcpyHostToDevice, s));
  SLK_HIP(hipMemcpyAsync(sd, start.data(), sizeof(int32_t) * (njobs + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(knn_exact_packed<kQBNarrow>, dim3((unsigned)b), dim3(kBlock), 0, s, jd, sd, njobs);
  SLK_LAUNCHED("knn_exact_packed");
  // the host arrays above are released when this returns: wait for the copies
  SLK_HIP(hipStreamSynchronize(s));
  return SLK_OK;
}

slk_status exclusive_scan_i32(const int32_t* in, int64_t count, int32_t* out, hipStream_t s) {
  // out has count + 1 entries; out[count] = total
  Scratch sc(s);
  const int64_t nt = std::max<int64_t>(1, (count + kScanTile - 1) / kScanTile);
  int32_t* sums;
  SLK_TRY(sc.get(&sums, nt));
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)nt), dim3(kBlock), 0, s, in, count, sums);
  SLK_LAUNCHED("scan_tile_sums");
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kBlock), 0, s, sums, nt, out + count);
  SLK_LAUNCHED("scan_sums_kernel");
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nt), dim3(kBlock), 0, s, in, count, sums, out);
  SLK_LAUNCHED("scan_apply");
  return SLK_OK;
}

slk_status sum_f64(const double* v, int64_t count, double* out_dev, hipStream_t s) {
  Scratch sc(s);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((count + kBlock - 1) / kBlock, 1024));
  double* part;
  uint32_t* arrive;
  SLK_TRY(sc.get(&part, grid));
  SLK_TRY(sc.get(&arrive, 1));
  SLK_HIP(hipMemsetAsync(arrive, 0, sizeof(uint32_t), s));
  hipLaunchKernelGGL(sum_f64_kernel, dim3(grid), dim3(kBlock), 0, s, v, count, part, out_dev, arrive);
  SLK_LAUNCHED("sum_f64_kernel");
  return SLK_OK;
}

// Sorts every row of a CSR in place.  The longest row and the number of rows above 64 entries
// come back to the host in one copy (one synchronisation).
slk_status sort_rows(const int32_t* row_ptr, int64_t n, int32_t* cols, hipStream_t s) {
  Scratch sc(s);
  int32_t *long_rows, *info;   // info: [0] rows above 64 entries, [1] INT32_MAX, [2] longest row
  SLK_TRY(sc.get(&long_rows, n));
  SLK_TRY(sc.get(&info, 3));
  SLK_HIP(hipMemsetAsync(info, 0, sizeof(int32_t), s));
  hipLaunchKernelGGL(init_minmax_kernel, dim3(1), dim3(1), 0, s, info + 1);
  const int mgrid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(degree_minmax_kernel, dim3(mgrid), dim3(256), 0, s, row_ptr, n, info + 1);
  SLK_LAUNCHED("degree_minmax_kernel");
  hipLaunchKernelGGL(sort_small_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kBlock), 0, s, row_ptr, n, cols, long_rows,
                     info);
  SLK_LAUNCHED("sort_small_kernel");
  int32_t h[3] = {0, 0, 0};
  SLK_HIP(hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  const int32_t h_long = h[0], max_len = h[2];
  if (h_long == 0) return SLK_OK;
  if (max_len <= kBigSort) {
    hipLaunchKernelGGL(sort_long_kernel, dim3(h_long), dim3(kBlock), 0, s, row_ptr, long_rows, cols,
                       (int32_t*)nullptr);
    SLK_LAUNCHED("sort_long_kernel");
    return SLK_OK;
  }
  // rows longer than the LDS tile: one launch per row with a global scratch area
  int P = 1;
  while (P < max_len) P <<= 1;
  int32_t* scr;
  SLK_TRY(sc.get(&scr, P));
  for (int i = 0; i < h_long; ++i) {
    hipLaunchKernelGGL(sort_long_kernel, dim3(1), dim3(kBlock), 0, s, row_ptr, long_rows + i, cols, scr);
    SLK_LAUNCHED("sort_long_kernel");
  }
  return SLK_OK;
}

slk_status launch_degree_minmax(const int32_t* row_ptr, int64_t n, int32_t* mm_dev, hipStream_t s) {
  hipLaunchKernelGGL(init_minmax_kernel, dim3(1), dim3(1), 0, s, mm_dev);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(degree_minmax_kernel, dim3(grid), dim3(256), 0, s, row_ptr, n, mm_dev);
  SLK_LAUNCHED("degree_minmax_kernel");
  return SLK_OK;
}

slk_status degree_stats(const int32_t* row_ptr, int64_t n, int32_t* mn, int32_t* mx, hipStream_t s) {
  Scratch sc(s);
  int32_t* mm;
  SLK_TRY(sc.get(&mm, 2));
  hipLaunchKernelGGL(init_minmax_kernel, dim3(1), dim3(1), 0, s, mm);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(degree_minmax_kernel, dim3(grid), dim3(256), 0, s, row_ptr, n, mm);
  SLK_LAUNCHED("degree_minmax_kernel");
  int32_t h[2];
  SLK_HIP(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, s));
  SLK_HIP(hipStreamSynchronize(s));
  *mn = h[0];
  *mx = h[1];
  return SLK_OK;
}

// OR-symmetrised, sorted, duplicate-free CSR of the kNN lists.  The column array is allocated at
// its upper bound 2 n k (+ pad), so nothing but the row sort reads back to the host; the number
// of entries is left in *nnz_dev.
slk_status build_csr(int64_t n, int32_t k, const int32_t* knn_idx, int32_t** row_ptr_out, int32_t** col_idx_out,
                     int32_t* nnz_dev, hipStream_t s) {
  Scratch sc(s);
  int32_t *cap, *off, *fill, *cols, *uniq;
  const int64_t bound = 2 * n * (int64_t)k;   // every kNN entry adds at most two
  SLK_TRY(sc.get(&cap, n));
  SLK_TRY(sc.get(&off, n + 1));
  SLK_TRY(sc.get(&fill, n));
  SLK_TRY(sc.get(&uniq, n));
  SLK_TRY(sc.get(&cols, bound));
  SLK_HIP(hipMemsetAsync(cap, 0, sizeof(int32_t) * n, s));
  SLK_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * n, s));
  const unsigned g1 = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(count_edges_kernel, dim3(g1), dim3(256), 0, s, knn_idx, n, k, cap);
  SLK_LAUNCHED("count_edges_kernel");
  SLK_TRY(exclusive_scan_i32(cap, n, off, s));
  hipLaunchKernelGGL(fill_edges_kernel, dim3(g1), dim3(256), 0, s, knn_idx, n, k, off, fill, cols);
  SLK_LAUNCHED("fill_edges_kernel");
  SLK_TRY(sort_rows(off, n, cols, s));
  const unsigned g4 = (unsigned)((n + 3) / 4);
  hipLaunchKernelGGL(unique_count_kernel, dim3(g4), dim3(kBlock), 0, s, off, n, cols, uniq);
  SLK_LAUNCHED("unique_count_kernel");
  int32_t* rp = nullptr;
  SLK_HIP(graph_alloc((void**)&rp, sizeof(int32_t) * (n + 1), s));
  slk_status st = exclusive_scan_i32(uniq, n, rp, s);
  if (st != SLK_OK) {
    graph_free(rp, graph_pool(), s);
    return st;
  }
  int32_t* ci = nullptr;
  if (graph_alloc((void**)&ci, sizeof(int32_t) * (bound + kColPad), s) != hipSuccess) {
    (void)hipGetLastError();
    graph_free(rp, graph_pool(), s);
    return fail(SLK_ERR_OUT_OF_MEMORY, "CSR columns");
  }
  hipLaunchKernelGGL(unique_copy_kernel, dim3(g4), dim3(kBlock), 0, s, off, n, cols, rp, ci);
  SLK_LAUNCHED("unique_copy_kernel");
  hipLaunchKernelGGL(csr_tail_kernel, dim3(1), dim3(64), 0, s, rp, n, ci, nnz_dev);
  SLK_LAUNCHED("csr_tail_kernel");
  *row_ptr_out = rp;
  *col_idx_out = ci;
  return SLK_OK;
}

slk_status relabel_csr(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* perm,
                       const int32_t* iperm, int32_t* new_row_ptr, int32_t* new_col_idx, hipStream_t s) {
  Scratch sc(s);
  int32_t* len;
  SLK_TRY(sc.get(&len, n));
  hipLaunchKernelGGL(row_lengths_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, row_ptr, n, perm, len);
  SLK_LAUNCHED("row_lengths_kernel");
  SLK_TRY(exclusive_scan_i32(len, n, new_row_ptr, s));
  hipLaunchKernelGGL(relabel_copy_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kBlock), 0, s, row_ptr, col_idx, n, perm,
                     iperm, new_row_ptr, new_col_idx);
  SLK_LAUNCHED("relabel_copy_kernel");
  SLK_TRY(sort_rows(new_row_ptr, n, new_col_idx, s));
  return SLK_OK;
}

}  // namespace slk
