// Clustering of detections in (time, DM, SNR) (Sec. 2.3), for gfx950: the
// exact DBSCAN below, the paper's FDBSCAN (expansion from representative
// points in index order, further down), and the DM-SNR classification of
// the clusters (Eqs. 3-4).
//
// DBSCAN:
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

// Joins the sets of a and b; returns the root the joined set had when the
// join (or the finding that they were joined) took effect.
__device__ inline int32_t uf_unite(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return a;
    if (a < b) { const int32_t t = a; a = b; b = t; }
    if (atomicCAS(parent + a, a, b) == a) return b;   // a was still a root: hooked under b
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
    // i's root, kept from one union to the next: sets only ever merge, so a
    // neighbour whose root was ever seen equal to it is already joined
    int32_t ri = uf_find(parent, i);
    for_row(A, p, dd, [&](int32_t j) {
      if (j < i && cnt[j] >= A.min_pts && uf_find(parent, j) != ri) ri = uf_unite(parent, ri, j);
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

// ---- FDBSCAN (Sec. 2.3) ------------------------------------------------------
// The paper's FDBSCAN: points are visited in index order; an unclassified
// core point starts a cluster, every unlabelled member of its neighbourhood
// joins it, and the expansion continues only from the representatives of a
// neighbourhood: with the expanding point at the origin, the member lying
// farthest in each direction of each dimension (sample, DM index, SNR; SNR
// offsets in FP32), the lowest index among equally far ones.  A point is
// region-queried at most once.
//
// A point's representatives depend on the data alone, so they are formed
// for every core point in parallel beforehand (fdb_reps_kernel).  What
// follows the visiting order runs on one workgroup (fdb_expand_kernel): it
// finds the next unclassified core point in index order and expands its
// cluster level by level.  Within a cluster every join writes the same
// number, and the points expanded are the closure of the start point under
// "representative of an expanded core point not queried before", which does
// not depend on the order the queue is served in; so labels, cluster count
// and query count equal those of the sequential algorithm.
constexpr int32_t kFdbUnclassified = -2;

// Key of a representative: its positive offset in the high word, the
// complement of its index in the low word, so an atomic maximum keeps the
// farthest member and, among equally far ones, the lowest index.  0: none.
__device__ inline uint64_t fdb_key(uint32_t off_bits, int32_t j) {
  return ((uint64_t)off_bits << 32) | (uint64_t)(0xffffffffu - (uint32_t)j);
}

__global__ __launch_bounds__(256) void fdb_init_kernel(int32_t n, int32_t* __restrict__ cnt,
                                                       uint64_t* __restrict__ keys, int32_t* __restrict__ queried,
                                                       int32_t* __restrict__ labels) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  cnt[i] = 0;
  queried[i] = 0;
  labels[i] = kFdbUnclassified;
#pragma unroll
  for (int k = 0; k < 6; ++k) keys[6 * (int64_t)i + k] = 0;
}

// Representatives of every core point: per (point, DM row) the row's
// farthest members in the six directions, combined over the rows with 64-bit
// atomic maxima (order-independent).  keys[6i + k]: k = 0/1 sample +/-,
// 2/3 DM index +/-, 4/5 SNR +/-.
__global__ __launch_bounds__(256) void fdb_reps_kernel(ClusterArgs A, const int32_t* __restrict__ cnt,
                                                       uint64_t* __restrict__ keys) {
  for_point_rows(A, [&](int32_t i, const CandDev& p, int32_t dd) {
    if (cnt[i] < A.min_pts) return;
    uint64_t k[6] = {0, 0, 0, 0, 0, 0};
    for_row(A, p, dd, [&](int32_t j) {
      const CandDev& q = A.c[j];
      const int64_t ds = q.sample - p.sample;
      const int32_t dm = q.dm_index - p.dm_index;
      const float dq = q.snr - p.snr;                 // FP32, as stored
      if (ds > 0) k[0] = max(k[0], fdb_key((uint32_t)ds, j));
      if (ds < 0) k[1] = max(k[1], fdb_key((uint32_t)(-ds), j));
      if (dm > 0) k[2] = max(k[2], fdb_key((uint32_t)dm, j));
      if (dm < 0) k[3] = max(k[3], fdb_key((uint32_t)(-dm), j));
      if (dq > 0.0f) k[4] = max(k[4], fdb_key(__float_as_uint(dq), j));
      if (-dq > 0.0f) k[5] = max(k[5], fdb_key(__float_as_uint(-dq), j));
    });
#pragma unroll
    for (int m = 0; m < 6; ++m)
      if (k[m]) atomicMax(reinterpret_cast<unsigned long long*>(keys + 6 * (int64_t)i + m), (unsigned long long)k[m]);
  });
}

// The visiting order, on one 1024-thread workgroup.  Unclassified non-core
// points that the sequential scan passes are region-queried there (counted,
// marked) and stay unclassified until a cluster takes them or the end makes
// them noise.
__global__ __launch_bounds__(1024) void fdb_expand_kernel(ClusterArgs A, const int32_t* __restrict__ cnt,
                                                          const uint64_t* __restrict__ keys,
                                                          int32_t* __restrict__ queried, int32_t* __restrict__ fa,
                                                          int32_t* __restrict__ fb, int32_t* __restrict__ labels,
                                                          int32_t* __restrict__ nclusters,
                                                          int64_t* __restrict__ nqueries) {
  __shared__ int32_t s_first, s_next, s_seeds;
  __shared__ int32_t s_cnt[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int32_t n = A.n;
  const int64_t R = 2 * (int64_t)A.dm_eps + 1;
  int32_t cursor = 0, ncl = 0;
  int64_t nq = 0;                                  // kept by thread 0
  for (;;) {
    // the next unclassified core point at or after the cursor
    int32_t first = n;
    for (int32_t base = cursor; base < n && first == n; base += 1024) {
      const int32_t i = base + tid;
      const bool unl = i < n && labels[i] == kFdbUnclassified;
      const bool core = unl && cnt[i] >= A.min_pts;
      if (tid == 0) s_first = n;
      __syncthreads();
      if (core) atomicMin(&s_first, i);
      __syncthreads();
      const int32_t f = s_first;
      const bool visited = unl && !core && i < f;
      if (visited) queried[i] = 1;
      const int c = __popcll(__ballot(visited));
      if (lane == 0) s_cnt[w] = c;
      __syncthreads();
      if (tid == 0)
        for (int k = 0; k < 16; ++k) nq += s_cnt[k];
      first = f;
      __syncthreads();
    }
    if (first == n) break;
    cursor = first + 1;
    const int32_t cid = ncl++;
    if (tid == 0) {
      queried[first] = 1;
      nq += 1;
      fa[0] = first;
    }
    int32_t* cur = fa;
    int32_t* nxt = fb;
    int32_t nfront = 1;
    __syncthreads();
    while (nfront > 0) {
      if (tid == 0) { s_next = 0; s_seeds = 0; }
      // every member of the frontier points' neighbourhoods that carries no
      // label joins the cluster (all writers write cid)
      const int64_t items = (int64_t)nfront * R;
      for (int64_t t = tid; t < items; t += 1024) {
        const int32_t f = cur[t / R];
        const CandDev p = A.c[f];
        const int64_t dd = (int64_t)p.dm_index - A.dm_eps + t % R;
        if (dd < 0 || dd >= A.ndms) continue;
        for_row(A, p, (int32_t)dd, [&](int32_t j) {
          if (labels[j] < 0) labels[j] = cid;
        });
      }
      __syncthreads();
      // their representatives are queried once each; core ones expand next
      for (int64_t t = tid; t < (int64_t)nfront * 6; t += 1024) {
        const uint64_t k = keys[6 * (int64_t)cur[t / 6] + t % 6];
        if (k == 0) continue;
        const int32_t r = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
        if (atomicExch(queried + r, 1) != 0) continue;
        atomicAdd(&s_seeds, 1);
        if (cnt[r] >= A.min_pts) nxt[atomicAdd(&s_next, 1)] = r;
      }
      __syncthreads();
      nfront = s_next;
      if (tid == 0) nq += s_seeds;
      int32_t* tmp = cur;
      cur = nxt;
      nxt = tmp;
      __syncthreads();
    }
  }
  for (int32_t i = tid; i < n; i += 1024)
    if (labels[i] == kFdbUnclassified) labels[i] = -1;
  if (tid == 0) {
    *nclusters = ncl;
    if (nqueries) *nqueries = nq;
  }
}

// ---- DM-SNR classification of clusters (Eqs. 3-4) ---------------------------
// One 1024-thread workgroup per cluster.  LDS holds, per DM row, the count
// and the largest SNR of the cluster's detections (an order-preserving int
// key for atomicMax), then the compacted sequence of rows that hold any.
struct ClusterInfoDev {
  int32_t peak_dm_index, npoints, ndm_rows, cls;
  int64_t t_first, t_last;
  float peak_snr;
  int32_t reserved;
  double rmse;
};

struct ClassifyArgs {
  const CandDev* c;
  const int32_t* labels;
  int32_t n, ndms, k;
  double dm_start, dm_step, tsamp_s, bw_mhz, f_ghz, rmse_max, dm_min;
  ClusterInfoDev* info;
};

__device__ inline int32_t snr_key(float x) {
  const int32_t b = __float_as_int(x);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ inline float snr_of_key(int32_t k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

// (count, snr key, -dm) lexicographic maximum
__device__ inline bool peak_better(int32_t c1, int32_t k1, int32_t d1, int32_t c2, int32_t k2, int32_t d2) {
  if (c1 != c2) return c1 > c2;
  if (k1 != k2) return k1 > k2;
  return d1 < d2;
}

__device__ inline int64_t shfl_xor64(int64_t v, int m) {
  const int32_t lo = __shfl_xor((int32_t)(v & 0xffffffff), m, 64), hi = __shfl_xor((int32_t)(v >> 32), m, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ __launch_bounds__(1024) void classify_kernel(ClassifyArgs A) {
  extern __shared__ int32_t lds[];
  int32_t* cnt = lds;                       // [ndms]
  int32_t* skey = lds + A.ndms;             // [ndms]
  int32_t* seqd = lds + 2 * A.ndms;         // [ndms]
  float* seqv = reinterpret_cast<float*>(lds + 3 * A.ndms);   // [ndms]
  __shared__ int32_t wsum[16];
  __shared__ int32_t wc[16], wk[16], wd[16], npts_s[16];
  __shared__ int64_t wlo[16], whi[16];
  __shared__ double wsq[16];
  __shared__ int32_t peak_s, ppos_s, nrows_s;
  const int32_t cl = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int32_t d = tid; d < A.ndms; d += 1024) { cnt[d] = 0; skey[d] = INT32_MIN; }
  __syncthreads();
  int32_t np = 0;
  for (int32_t i = tid; i < A.n; i += 1024) {
    if (A.labels[i] != cl) continue;
    const int32_t d = A.c[i].dm_index;
    if (d < 0 || d >= A.ndms) continue;
    atomicAdd(cnt + d, 1);
    atomicMax(skey + d, snr_key(A.c[i].snr));
    ++np;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) np += __shfl_xor(np, off, 64);
  if (lane == 0) npts_s[w] = np;
  __syncthreads();
  // peak row
  int32_t bc = -1, bk = INT32_MIN, bd = A.ndms;
  for (int32_t d = tid; d < A.ndms; d += 1024)
    if (cnt[d] > 0 && peak_better(cnt[d], skey[d], d, bc, bk, bd)) { bc = cnt[d]; bk = skey[d]; bd = d; }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t c2 = __shfl_xor(bc, off, 64), k2 = __shfl_xor(bk, off, 64), d2 = __shfl_xor(bd, off, 64);
    if (peak_better(c2, k2, d2, bc, bk, bd)) { bc = c2; bk = k2; bd = d2; }
  }
  if (lane == 0) { wc[w] = bc; wk[w] = bk; wd[w] = bd; }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < 16; ++k)
      if (peak_better(wc[k], wk[k], wd[k], wc[0], wk[0], wd[0])) { wc[0] = wc[k]; wk[0] = wk[k]; wd[0] = wd[k]; }
    peak_s = wd[0];
  }
  __syncthreads();
  const int32_t peak = peak_s;
  ClusterInfoDev* rec = A.info + cl;
  if (peak >= A.ndms) {                     // no detection carries this label
    if (tid == 0) {
      rec->peak_dm_index = -1; rec->npoints = 0; rec->ndm_rows = 0; rec->cls = 3;
      rec->t_first = 0; rec->t_last = 0; rec->peak_snr = 0.0f; rec->reserved = 0; rec->rmse = __builtin_nan("");
    }
    return;
  }
  // first and last sample at the peak row
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  for (int32_t i = tid; i < A.n; i += 1024)
    if (A.labels[i] == cl && A.c[i].dm_index == peak) {
      const int64_t t = A.c[i].sample;
      lo = t < lo ? t : lo;
      hi = t > hi ? t : hi;
    }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t l2 = shfl_xor64(lo, off), h2 = shfl_xor64(hi, off);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  if (lane == 0) { wlo[w] = lo; whi[w] = hi; }
  // compacted sequence of rows holding detections
  int32_t carry = 0;
  for (int32_t base = 0; base < A.ndms; base += 1024) {
    const int32_t d = base + tid;
    const int32_t f = (d < A.ndms && cnt[d] > 0) ? 1 : 0;
    int32_t total;
    const int32_t ex = block_exclusive(f, wsum, total);
    if (f) {
      seqd[carry + ex] = d;
      seqv[carry + ex] = snr_of_key(skey[d]);
      if (d == peak) ppos_s = carry + ex;
    }
    carry += total;
    __syncthreads();
  }
  if (tid == 0) nrows_s = carry;
  __syncthreads();
  const int32_t L = nrows_s, pp = ppos_s;
  if (tid == 0) {
    int64_t l = wlo[0], h = whi[0];
    for (int k = 1; k < 16; ++k) { l = wlo[k] < l ? wlo[k] : l; h = whi[k] > h ? whi[k] : h; }
    rec->peak_dm_index = peak;
    int32_t np_all = 0;
    for (int k = 0; k < 16; ++k) np_all += npts_s[k];
    rec->npoints = np_all;
    rec->ndm_rows = L;
    rec->t_first = l;
    rec->t_last = h;
    rec->peak_snr = snr_of_key(skey[peak]);
    rec->reserved = 0;
    wlo[0] = l;
    whi[0] = h;
  }
  __syncthreads();
  if (A.dm_start + peak * A.dm_step < A.dm_min) {
    if (tid == 0) { rec->cls = 1; rec->rmse = __builtin_nan(""); }
    return;
  }
  const int32_t hw = (A.k - 1) / 2;
  auto smooth = [&](int32_t p) {
    const int32_t a = p - hw < 0 ? 0 : p - hw, b = p + hw + 1 > L ? L : p + hw + 1;
    double sum = 0.0;
    for (int32_t j = a; j < b; ++j) sum += (double)seqv[j];
    return sum / (double)(b - a);
  };
  const double sp = smooth(pp);
  const double width_ms = (double)(whi[0] - wlo[0] + 1) * A.tsamp_s * 1e3;
  const double f3 = A.f_ghz * A.f_ghz * A.f_ghz;
  double sq = 0.0;
  for (int32_t p = tid; p < L; p += 1024) {
    const double norm = smooth(p) / sp;
    const double ddm = (double)(seqd[p] - peak) * A.dm_step;
    const double z = fabs(6.91e-3 * ddm * A.bw_mhz / (width_ms * f3));
    const double model = z > 0.0 ? 0.88622692545275801 * erf(z) / z : 1.0;   // sqrt(pi) / 2
    sq += (norm - model) * (norm - model);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
  if (lane == 0) wsq[w] = sq;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int k = 0; k < 16; ++k) sum += wsq[k];
    const double rmse = sqrt(sum / (double)L);
    rec->rmse = rmse;
    rec->cls = rmse <= A.rmse_max ? 0 : 2;
  }
}

}  // namespace

hipError_t launch_classify(const CandDev* c, const int32_t* labels, int32_t n, int32_t nclusters, int32_t ndms,
                           double dm_start, double dm_step, double tsamp_s, double bw_mhz, double f_ghz, int32_t k,
                           double rmse_max, double dm_min, void* info, hipStream_t s) {
  if (nclusters == 0) return hipSuccess;
  ClassifyArgs A{c, labels, n, ndms, k, dm_start, dm_step, tsamp_s, bw_mhz, f_ghz, rmse_max, dm_min,
                 static_cast<ClusterInfoDev*>(info)};
  hipLaunchKernelGGL(classify_kernel, dim3((unsigned)nclusters), dim3(1024), 16 * (size_t)ndms, s, A);
  return hipGetLastError();
}

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

size_t fdbscan_work_bytes(int64_t n, int32_t ndms) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up(4 * (size_t)(ndms + 1)) + 4 * up(4 * (size_t)n) + up(48 * (size_t)n);
}

hipError_t launch_fdbscan(const CandDev* c, int32_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps, float snr_eps,
                          int32_t min_pts, int32_t* labels, int32_t* nclusters, int64_t* nqueries, void* work,
                          hipStream_t s) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  char* w = static_cast<char*>(work);
  int32_t* row_start = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)(ndms + 1));
  int32_t* cnt = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* queried = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* fa = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  int32_t* fb = reinterpret_cast<int32_t*>(w);
  w += up(4 * (size_t)n);
  uint64_t* keys = reinterpret_cast<uint64_t*>(w);
  ClusterArgs A{c, n, ndms, dm_eps, t_eps, snr_eps, min_pts, row_start};
  const unsigned gn = (unsigned)((n + 255) / 256);
  const int64_t rows_threads = (int64_t)n * (2 * (int64_t)dm_eps + 1);
  const unsigned gr = (unsigned)std::min<int64_t>((rows_threads + 255) / 256, int64_t(1) << 20);
  hipLaunchKernelGGL(cluster_rows_kernel, dim3((unsigned)((ndms + 1 + 255) / 256)), dim3(256), 0, s, c, n, ndms,
                     row_start);
  if (n > 0) {
    hipLaunchKernelGGL(fdb_init_kernel, dim3(gn), dim3(256), 0, s, n, cnt, keys, queried, labels);
    hipLaunchKernelGGL(cluster_count_kernel, dim3(gr), dim3(256), 0, s, A, cnt);
    hipLaunchKernelGGL(fdb_reps_kernel, dim3(gr), dim3(256), 0, s, A, cnt, keys);
  }
  hipLaunchKernelGGL(fdb_expand_kernel, dim3(1), dim3(1024), 0, s, A, cnt, keys, queried, fa, fb, labels, nclusters,
                     nqueries);
  return hipGetLastError();
}

}  // namespace mbtp
