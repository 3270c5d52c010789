// DBSCAN clustering of detections in (time, DM, SNR) (Sec. 2.3), for gfx950.
//
// The detections arrive in (DM index, sample) order, as the detection stage
// writes them, so the neighbours of a point lie in the 2*dm_eps + 1 DM rows
// around it, each a contiguous run of samples found by binary search.  A
// point q is a neighbour of p when it lies within t_eps samples, dm_eps DM
// indices and snr_eps of SNR (the SNR difference in FP32), p included.
//   1. row starts: one lower bound per DM index;
//   2. neighbour counts (one thread per point and DM row, summed with
//      atomics): core points have at least min_pts;
//   3. each core point hooked under its lowest core neighbour, then the
//      union of core points with their lower-indexed core neighbours, in a
//      lock-free union-find that always hooks the larger root under the
//      smaller one, so every component's root is its lowest core index
//      whatever the order of the unions (path halving keeps finds short);
//   4. each core point takes its root; a border point takes the root of its
//      lowest-indexed core neighbour (an atomic minimum over its rows); noise
//      takes -1;
//   5. the roots are numbered in index order (per-chunk counts, one
//      workgroup's scan of them, per-root ranks) and the labels written.
// Every result is a function of the input alone, bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"

namespace mbtp {
namespace {

struct ClusterArgs {
  const CandDev* c;
  int32_t n, ndms, dm_eps;
  int64_t t_eps;
  float snr_eps;
  int32_t min_pts;
  const int32_t* row_start;   // [ndms + 1]
};

__global__ __launch_bounds__(256) void cluster_rows_kernel(const CandDev* __restrict__ c, int32_t n, int32_t ndms,
                                                           int32_t* __restrict__ row_start) {
  const int64_t d = blockIdx.x * 256ll + threadIdx.x;
  if (d > ndms) return;
  int32_t lo = 0, hi = n;                 // first index with dm_index >= d
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (c[mid].dm_index < d) lo = mid + 1; else hi = mid;
  }
  row_start[d] = lo;
}

// Calls visit(j) for every neighbour j of point p (index i) in DM row dd.
template <class F>
__device__ inline void for_row(const ClusterArgs& A, const CandDev& p, int32_t dd, F&& visit) {
  int32_t lo = A.row_start[dd];
  const int32_t end = A.row_start[dd + 1];
  const int64_t smin = p.sample - A.t_eps, smax = p.sample + A.t_eps;
  int32_t hi = end;
  while (lo < hi) {                       // first sample >= smin
    const int32_t mid = lo + (hi - lo) / 2;
    if (A.c[mid].sample < smin) lo = mid + 1; else hi = mid;
  }
  for (int32_t j = lo; j < end && A.c[j].sample <= smax; ++j)
    if (fabsf(A.c[j].snr - p.snr) <= A.snr_eps) visit(j);
}

__device__ inline int32_t uf_load(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t uf_find(int32_t* parent, int32_t x) {
  while (true) {
    const int32_t p = uf_load(parent + x);
    if (p == x) return x;
    const int32_t g = uf_load(parent + p);
    if (g != p) atomicCAS(parent + x, p, g);   // path halving: p -> g only shortens the path
    x = g;
  }
}

__device__ inline void uf_unite(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) { const int32_t t = a; a = b; b = t; }
    if (atomicCAS(parent + a, a, b) == a) return;   // a was still a root: hooked under b
  }
}

// The neighbourhood passes run one thread per (point, DM row of its
// neighbourhood), grid-stride: a point inside a pulse's bow-tie has hundreds
// of neighbours, and a thread per point would leave the pass as long as its
// longest scan (for the unions, a chain of dependent L2 round trips per
// neighbour).  Per-point results are combined with integer atomics, which
// are order-independent.
template <class F>
__device__ inline void for_point_rows(const ClusterArgs& A, F&& body) {
  const int64_t R = 2 * (int64_t)A.dm_eps + 1, total = (int64_t)A.n * R;
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int32_t i = (int32_t)(t / R);
    const CandDev p = A.c[i];
    const int64_t dd = (int64_t)p.dm_index - A.dm_eps + t % R;
    if (dd < 0 || dd >= A.ndms) continue;
    body(i, p, (int32_t)dd);
  }
}

__global__ __launch_bounds__(256) void cluster_init_kernel(int32_t n, int32_t* __restrict__ cnt,
                                                           int32_t* __restrict__ parent, int32_t* __restrict__ bmin) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  cnt[i] = 0;
  parent[i] = i;
  bmin[i] = n;
}

// Neighbour counts: cnt[i] >= min_pts makes i a core point.
__global__ __launch_bounds__(256) void cluster_count_kernel(ClusterArgs A, int32_t* cnt) {
  for_point_rows(A, [&](int32_t i, const CandDev& p, int32_t dd) {
    int32_t k = 0;
    for_row(A, p, dd, [&](int32_t) { ++k; });
    if (k) atomicAdd(cnt + i, k);
  });
}

// Points every core point at its lowest-indexed core neighbour (itself if
// none is lower): a forest of real core-core edges, shallow for dense
// clusters, so that the unions below mostly find their sets already joined.
__global__ __launch_bounds__(256) void cluster_hook_kernel(ClusterArgs A, const int32_t* __restrict__ cnt,
                                                           int32_t* parent) {
  for_point_rows(A, [&](int32_t i, const CandDev& p, int32_t dd) {
    if (cnt[i] < A.min_pts) return;
    int32_t best = i;
    for_row(A, p, dd, [&](int32_t j) {
      if (j < best && cnt[j] >= A.min_pts) best = j;
    });
    if (best < i) atomicMin(parent + i, best);
  });
}

// Union of every core point with its lower-indexed core neighbours.
__global__ __launch_bounds__(256) void cluster_union_kernel(ClusterArgs A, const int32_t* __restrict__ cnt,
                                                            int32_t* parent) {
  for_point_rows(A, [&](int32_t i, const CandDev& p, int32_t dd) {
    if (cnt[i] < A.min_pts) return;
    for_row(A, p, dd, [&](int32_t j) {
      if (j < i && cnt[j] >= A.min_pts) uf_unite(parent, i, j);
    });
  });
}

// Lowest-indexed core neighbour of every non-core point (n if none).
__global__ __launch_bounds__(256) void cluster_border_kernel(ClusterArgs A, const int32_t* __restrict__ cnt,
                                                             int32_t* bmin) {
  for_point_rows(A, [&](int32_t i, const CandDev& p, int32_t dd) {
    if (cnt[i] >= A.min_pts) return;
    int32_t best = A.n;
    for_row(A, p, dd, [&](int32_t j) {
      if (j < best && cnt[j] >= A.min_pts) best = j;
    });
    if (best < A.n) atomicMin(bmin + i, best);
  });
}

__global__ __launch_bounds__(256) void cluster_root_kernel(ClusterArgs A, const int32_t* __restrict__ cnt,
                                                           const int32_t* __restrict__ bmin, int32_t* parent,
                                                           int32_t* __restrict__ root) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= A.n) return;
  if (cnt[i] >= A.min_pts) root[i] = uf_find(parent, i);
  else root[i] = bmin[i] < A.n ? uf_find(parent, bmin[i]) : -1;
}

// Numbering: roots per 256-point chunk, an exclusive scan of the chunk
// counts in one workgroup, each root's rank, then the labels.
__device__ inline int32_t block_exclusive(int32_t f, int32_t* wsum, int32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = f;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int32_t before = 0;
  total = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    if (k < w) before += wsum[k];
    total += wsum[k];
  }
  return before + x - f;
}

__global__ __launch_bounds__(256) void cluster_chunk_count_kernel(int32_t n, const int32_t* __restrict__ root,
                                                                  int32_t* __restrict__ chunk) {
  __shared__ int32_t wsum[4];
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  int32_t total;
  block_exclusive((i < n && root[i] == i) ? 1 : 0, wsum, total);
  if (threadIdx.x == 0) chunk[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void cluster_chunk_scan_kernel(int32_t nchunks, int32_t* __restrict__ chunk,
                                                                  int32_t* __restrict__ nclusters) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int32_t base = 0; base < nchunks; base += 1024) {
    const int32_t b = base + threadIdx.x;
    const int32_t f = b < nchunks ? chunk[b] : 0;
    int32_t total;
    const int32_t ex = block_exclusive(f, wsum, total);
    const int32_t carry = carry_s;
    if (b < nchunks) chunk[b] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *nclusters = carry_s;
}

__global__ __launch_bounds__(256) void cluster_rank_kernel(int32_t n, const int32_t* __restrict__ root,
                                                           const int32_t* __restrict__ chunk,
                                                           int32_t* __restrict__ rank) {
  __shared__ int32_t wsum[4];
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  const int32_t f = (i < n && root[i] == i) ? 1 : 0;
  int32_t total;
  const int32_t ex = block_exclusive(f, wsum, total);
  if (f) rank[i] = chunk[blockIdx.x] + ex;
}

__global__ __launch_bounds__(256) void cluster_label_kernel(int32_t n, const int32_t* __restrict__ root,
                                                            const int32_t* __restrict__ rank,
                                                            int32_t* __restrict__ labels) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t r = root[i];
  labels[i] = r < 0 ? -1 : rank[r];
}

}  // namespace

size_t cluster_work_bytes(int64_t n, int32_t ndms) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up(4 * (size_t)(ndms + 1)) + 4 * up(4 * (size_t)n) + up(4 * (size_t)((n + 255) / 256 + 1));
}

hipError_t launch_cluster(const CandDev* c, int32_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps, float snr_eps,
                          int32_t min_pts, int32_t* labels, int32_t* nclusters, void* work, hipStream_t s) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  char* w = static_cast<char*>(work);
  int32_t* row_start = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)(ndms + 1));
  int32_t* core = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* parent = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* root = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* rank = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* chunk = reinterpret_cast<int32_t*>(w);
  ClusterArgs A{c, n, ndms, dm_eps, t_eps, snr_eps, min_pts, row_start};
  const int32_t nchunks = (int32_t)((n + 255) / 256);
  const unsigned gn = (unsigned)nchunks;
  const int64_t rows_threads = (int64_t)n * (2 * (int64_t)dm_eps + 1);
  const unsigned gr = (unsigned)std::min<int64_t>((rows_threads + 255) / 256, int64_t(1) << 20);
  int32_t* bmin = rank;                   // free until the numbering
  hipLaunchKernelGGL(cluster_rows_kernel, dim3((unsigned)((ndms + 1 + 255) / 256)), dim3(256), 0, s, c, n, ndms,
                     row_start);
  if (n > 0) {
    hipLaunchKernelGGL(cluster_init_kernel, dim3(gn), dim3(256), 0, s, n, core, parent, bmin);
    hipLaunchKernelGGL(cluster_count_kernel, dim3(gr), dim3(256), 0, s, A, core);
    hipLaunchKernelGGL(cluster_hook_kernel, dim3(gr), dim3(256), 0, s, A, core, parent);
    hipLaunchKernelGGL(cluster_union_kernel, dim3(gr), dim3(256), 0, s, A, core, parent);
    hipLaunchKernelGGL(cluster_border_kernel, dim3(gr), dim3(256), 0, s, A, core, bmin);
    hipLaunchKernelGGL(cluster_root_kernel, dim3(gn), dim3(256), 0, s, A, core, bmin, parent, root);
    hipLaunchKernelGGL(cluster_chunk_count_kernel, dim3(gn), dim3(256), 0, s, n, root, chunk);
  }
  hipLaunchKernelGGL(cluster_chunk_scan_kernel, dim3(1), dim3(1024), 0, s, nchunks, chunk, nclusters);
  if (n > 0) {
    hipLaunchKernelGGL(cluster_rank_kernel, dim3(gn), dim3(256), 0, s, n, root, chunk, rank);
    hipLaunchKernelGGL(cluster_label_kernel, dim3(gn), dim3(256), 0, s, n, root, rank, labels);
  }
  return hipGetLastError();
}

}  // namespace mbtp
