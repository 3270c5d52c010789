// Per-DM detrending and normalisation (Sec. 2.2.3) and the n-sigma event
// threshold (Sec. 2.3) over a dedispersed plane D[ndms][ld_out] (FP32).
//
// The row passes run one workgroup per DM row, and every row is split into
// kDetectSegs segments of whole 256-sample groups; a lane reads 4
// consecutive samples per group with one 16-byte load.
//
// norm:   one pass forms sum D, sum (t - tbar) D and sum D^2 in FP64; the
//         least-squares line and the residual sum of squares follow in
//         closed form, unless that sum is small against sum D^2, when the
//         row is read again and the residuals are summed directly.
// detect: pass A counts z > nsigma per (row, segment) and finds the row's
//         peak; a single-workgroup exclusive scan turns counts into output
//         offsets; pass B rescans only the segments with hits and writes the
//         triplets in (DM, sample) order with a wave prefix sum per group.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "internal.h"

namespace mbtp {

// The allocation-free detection's counts and offsets per (row, segment): a
// fixed array, one copy on each GPU the library runs on, held until the
// process ends.  Host code never passes this name to a kernel (on the host
// it is only a handle of the symbol); it uses the device address that
// detect_scratch_setup looked up for the current device.
static __device__ __align__(256) int64_t scratch[2 * kDetectSegs * kDetectNoAllocMaxDms];

namespace {

constexpr double kDegenerateRtol = 1e-9;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup of the per-row passes that read a whole row (normalisation and
// the detection count): 512 threads, so that four fit a CU and the 640 rows
// of the benchmark plane are all resident at once (1024-thread workgroups
// left a quarter of the rows to a second, mostly empty round).
constexpr int kRowThreads = 512;
constexpr int kRowWaves = kRowThreads / 64;

// Block sums of three values over kRowThreads threads in a fixed order.
__device__ inline void block_sum3(double& a, double& b, double& c, double* sh /* 3 * kRowWaves */) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[kRowWaves + w] = b;
    sh[2 * kRowWaves + w] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
#pragma unroll
  for (int k = 0; k < kRowWaves; ++k) {
    a += sh[k];
    b += sh[kRowWaves + k];
    c += sh[2 * kRowWaves + k];
  }
}

// Segment w of a row of nout samples: whole 256-sample groups.
__device__ inline void segment(int64_t nout, int w, int64_t& lo, int64_t& hi) {
  const int64_t seg = ((nout + 256 * kDetectSegs - 1) / (256 * kDetectSegs)) * 256;
  lo = min(nout, (int64_t)w * seg);
  hi = min(nout, lo + seg);
}

__global__ __launch_bounds__(kRowThreads) void norm_kernel(const float* __restrict__ out, int64_t ld_out,
                                                           int64_t nout, NormDev* __restrict__ norm) {
  __shared__ double sh[3 * kRowWaves];
  const int d = blockIdx.x;
  const float* row = out + (int64_t)d * ld_out;
  const float4* row4 = reinterpret_cast<const float4*>(row);
  const double N = (double)nout;
  const double tbar = 0.5 * (N - 1.0);
  double s1 = 0.0, st = 0.0, s2 = 0.0;
  auto acc4 = [&](const float4 v, int64_t i) {
    const double t = (double)(4 * i) - tbar;
    const double a0 = v.x, a1 = v.y, a2 = v.z, a3 = v.w;
    s1 += (a0 + a1) + (a2 + a3);
    st += (t * a0 + (t + 1.0) * a1) + ((t + 2.0) * a2 + (t + 3.0) * a3);
    s2 += (a0 * a0 + a1 * a1) + (a2 * a2 + a3 * a3);
  };
  // 4 samples per thread per step (rows are 16-byte aligned, ld_out % 4 ==
  // 0), four 16-byte loads in flight; each thread adds its quads in order
  const int64_t n4 = nout / 4;
  int64_t i = threadIdx.x;
  for (; i + 3 * kRowThreads < n4; i += 4 * kRowThreads) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = row4[i + u * kRowThreads];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc4(v[u], i + u * kRowThreads);
  }
  for (; i < n4; i += kRowThreads) acc4(row4[i], i);
  for (int64_t k = 4 * n4 + threadIdx.x; k < nout; k += kRowThreads) {
    const double v = row[k];
    s1 += v; st += ((double)k - tbar) * v; s2 += v * v;
  }
  block_sum3(s1, st, s2, sh);
  const double stt = N * (N * N - 1.0) / 12.0;
  const double b = stt > 0.0 ? st / stt : 0.0;
  const double a = (nout > 0 ? s1 / N : 0.0) - b * tbar;
  // Residual sum of squares from the same pass: (S2 - S1^2/N) - St^2/Stt.
  // Kept when it is not small against S2, where its cancellation error stays
  // far below the row's own rounding; otherwise (a large mean against the
  // scatter, an exactly linear or constant row) the row is read again and
  // the residuals summed directly.  The branch is uniform per workgroup.
  double r2 = nout > 0 ? (s2 - s1 * s1 / N) - (stt > 0.0 ? st * st / stt : 0.0) : 0.0;
  if (r2 > 1e-4 * s2) {
    if (threadIdx.x == 0) {
      NormDev nd;
      nd.a = a;
      nd.b = b;
      nd.sigma = sqrt(r2 / N);
      nd.degenerate = nd.sigma <= kDegenerateRtol * sqrt(s2 / N) ? 1 : 0;
      nd.reserved = 0;
      norm[d] = nd;
    }
    return;
  }
  r2 = 0.0;
  for (int64_t i = threadIdx.x; i < n4; i += kRowThreads) {
    const float4 v = reinterpret_cast<const float4*>(row)[i];
    const double t = (double)(4 * i);
    const double r0 = ((double)v.x - a) - b * t;
    const double r1 = ((double)v.y - a) - b * (t + 1.0);
    const double rr2 = ((double)v.z - a) - b * (t + 2.0);
    const double r3 = ((double)v.w - a) - b * (t + 3.0);
    r2 += (r0 * r0 + r1 * r1) + (rr2 * rr2 + r3 * r3);
  }
  for (int64_t k = 4 * n4 + threadIdx.x; k < nout; k += kRowThreads) {
    const double r = ((double)row[k] - a) - b * (double)k;
    r2 += r * r;
  }
  {
    double z1 = 0.0, z2 = 0.0;
    block_sum3(r2, z1, z2, sh);
  }
  if (threadIdx.x == 0) {
    NormDev nd;
    nd.a = a;
    nd.b = b;
    nd.sigma = nout > 0 ? sqrt(r2 / N) : 0.0;
    const double rms = nout > 0 ? sqrt(s2 / N) : 0.0;
    nd.degenerate = (nout == 0 || nd.sigma <= kDegenerateRtol * rms) ? 1 : 0;
    nd.reserved = 0;
    norm[d] = nd;
  }
}

// Residual of sample t from the row's line, formed in FP64 with separate
// roundings: r = (D - a) - b t.  z = r / sigma.  The threshold test z > nsigma
// is taken as r > nsigma * sigma (the same comparison in both passes; it can
// differ from the quotient only for z within rounding of nsigma).
__device__ inline double resid(float v, int64_t t, const NormDev& n) {
  return __dsub_rn(__dsub_rn((double)v, n.a), __dmul_rn(n.b, (double)t));
}

// The 4 samples of a lane at t (a multiple of 4, t < hi): one 16-byte load;
// rows are ld_out >= nout apart with ld_out % 4 == 0, so it stays in its row.
__device__ inline float4 quad_at(const float* row, int64_t t) {
  return *reinterpret_cast<const float4*>(row + t);
}

// Pass A: hits per (row, segment) and the row's peak.  Wave w takes
// segments w and w + kRowWaves; a lane reads 4 consecutive samples per
// 256-sample group, two groups in flight.
__global__ __launch_bounds__(kRowThreads) void detect_count_kernel(const float* __restrict__ out,
                                                                   int64_t ld_out, int64_t nout,
                                                                   const NormDev* __restrict__ norm,
                                                                   double nsigma, int64_t sample0,
                                                                   const int64_t* __restrict__ d_sample0,
                                                                   int64_t* __restrict__ counts,
                                                                   PeakDev* __restrict__ peaks) {
  static_assert(kDetectSegs == 2 * kRowWaves, "two segments per wave");
  __shared__ double shr[kRowWaves];
  __shared__ int64_t sht[kRowWaves];
  const int d = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* row = out + (int64_t)d * ld_out;
  const NormDev n = norm[d];
  const double thr = nsigma * n.sigma;
  double best = -INFINITY;
  int64_t bt = INT64_MAX;
  auto scan_quad = [&](const float4 q, int64_t t, int64_t hi, int64_t& cnt) {
    const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (t + j < hi) {
        const double r = resid(qv[j], t + j, n);
        cnt += (r > thr) ? 1 : 0;
        if (r > best) { best = r; bt = t + j; }   // ascending t per lane keeps the earliest
      }
    }
  };
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int sg = wave + half * kRowWaves;
    int64_t lo, hi;
    segment(nout, sg, lo, hi);
    int64_t cnt = 0;
    if (!n.degenerate) {
      int64_t t0 = lo;
      for (; t0 + 256 < hi; t0 += 512) {
        const int64_t ta = t0 + 4 * lane, tb = ta + 256;
        const float4 qa = quad_at(row, ta);                 // ta < hi
        const float4 qb = tb < hi ? quad_at(row, tb) : make_float4(0.f, 0.f, 0.f, 0.f);
        scan_quad(qa, ta, hi, cnt);
        if (tb < hi) scan_quad(qb, tb, hi, cnt);
      }
      for (; t0 < hi; t0 += 256) {
        const int64_t t = t0 + 4 * lane;
        if (t < hi) scan_quad(quad_at(row, t), t, hi, cnt);
      }
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0) counts[(int64_t)d * kDetectSegs + sg] = cnt;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int64_t ot = __shfl_xor(bt, off, 64);
    if (ob > best || (ob == best && ot < bt)) { best = ob; bt = ot; }
  }
  if (lane == 0) {
    shr[wave] = best;
    sht[wave] = bt;
  }
  __syncthreads();
  if (threadIdx.x == 0 && peaks) {
    if (d_sample0) sample0 += *d_sample0;
    PeakDev p;
    p.reserved = 0;
    if (n.degenerate || nout == 0) {
      p.sample = sample0;
      p.snr = 0.0f;
    } else {
      double br = shr[0];
      int64_t btt = sht[0];
      for (int k = 1; k < kRowWaves; ++k)
        if (shr[k] > br || (shr[k] == br && sht[k] < btt)) { br = shr[k]; btt = sht[k]; }
      p.sample = sample0 + btt;
      p.snr = (float)(br / n.sigma);
    }
    peaks[d] = p;
  }
}

// Exclusive scan of the per-(row, segment) counts on one 1024-thread
// workgroup, 4096 counts at a time: each thread loads 4 consecutive counts,
// the thread totals are scanned across the wave (shuffles) and across the
// 16 waves (LDS), and a running carry joins the chunks.
__global__ __launch_bounds__(1024) void detect_scan_kernel(const int64_t* __restrict__ counts,
                                                           int64_t n, int64_t* __restrict__ offsets,
                                                           int64_t* __restrict__ total) {
  __shared__ int64_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += 4096) {
    const int64_t i0 = base + 4 * (int64_t)tid;
    int64_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = i0 + k < n ? counts[i0 + k] : 0;
    const int64_t s = (v[0] + v[1]) + (v[2] + v[3]);
    int64_t inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t run = carry + inc - s, chunk = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < w) run += wsum[k];
      chunk += wsum[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < n) offsets[i0 + k] = run;
      run += v[k];
    }
    carry += chunk;
    __syncthreads();
  }
  if (tid == 0) *total = carry;
}

// Exclusive prefix sum over the 64 lanes of a wave.
__device__ inline int wave_prefix_excl(int c, int lane, int& total) {
  int inc = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  total = __shfl(inc, 63, 64);
  return inc - c;
}

// Pass B: each wave rescans its segment (only if it holds hits) and writes
// them in sample order: within a 256-sample group, lane-ordered prefix sums
// of the lanes' hit counts; a running offset across groups.  No barriers.
__global__ __launch_bounds__(1024) void detect_write_kernel(const float* __restrict__ out,
                                                            int64_t ld_out, int64_t nout,
                                                            const NormDev* __restrict__ norm,
                                                            double nsigma, int64_t sample0,
                                                            const int64_t* __restrict__ d_sample0,
                                                            double dm_start, double dm_step,
                                                            const int64_t* __restrict__ counts,
                                                            const int64_t* __restrict__ offsets,
                                                            CandDev* __restrict__ cands,
                                                            int64_t capacity) {
  const int d = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t slot = (int64_t)d * kDetectSegs + wave;
  if (counts[slot] == 0) return;
  int64_t pos = offsets[slot];
  if (pos >= capacity) return;
  if (d_sample0) sample0 += *d_sample0;
  const float* row = out + (int64_t)d * ld_out;
  const NormDev n = norm[d];
  const double thr = nsigma * n.sigma;
  const float dmv = (float)(dm_start + (double)d * dm_step);
  int64_t lo, hi;
  segment(nout, wave, lo, hi);
  for (int64_t t0 = lo; t0 < hi && pos < capacity; t0 += 256) {
    const int64_t t = t0 + 4 * lane;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    bool hit[4] = {false, false, false, false};
    if (t < hi) {
      const float4 q = quad_at(row, t);
      const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (t + j < hi) {
          r[j] = resid(qv[j], t + j, n);
          hit[j] = r[j] > thr;
        }
      }
    }
    const int c = (int)hit[0] + (int)hit[1] + (int)hit[2] + (int)hit[3];
    int total;
    int64_t k = pos + wave_prefix_excl(c, lane, total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (hit[j]) {
        if (k < capacity) {
          CandDev cd;
          cd.dm_index = d;
          cd.reserved = 0;
          cd.sample = sample0 + t + j;
          cd.snr = (float)(r[j] / n.sigma);
          cd.dm = dmv;
          cands[k] = cd;
        }
        ++k;
      }
    }
    pos += total;
  }
}

}  // namespace

hipError_t launch_norm(const float* out, int64_t ld_out, int64_t nout, int32_t ndms, NormDev* norm,
                       hipStream_t s) {
  hipLaunchKernelGGL(norm_kernel, dim3((unsigned)ndms), dim3(kRowThreads), 0, s, out, ld_out, nout, norm);
  return hipGetLastError();
}

hipError_t launch_detect(const float* out, int64_t ld_out, int64_t nout, int32_t ndms,
                         const NormDev* norm, int64_t sample0, const int64_t* d_sample0, double nsigma,
                         double dm_start, double dm_step, CandDev* cands, int64_t capacity, int64_t* d_count,
                         PeakDev* peaks, void* work, hipStream_t s) {
  int64_t* counts = static_cast<int64_t*>(work);
  int64_t* offsets = counts + kDetectSegs * (int64_t)ndms;
  hipLaunchKernelGGL(detect_count_kernel, dim3((unsigned)ndms), dim3(kRowThreads), 0, s, out, ld_out, nout,
                     norm, nsigma, sample0, d_sample0, counts, peaks);
  hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(1024), 0, s, counts,
                     kDetectSegs * (int64_t)ndms, offsets, d_count);
  hipLaunchKernelGGL(detect_write_kernel, dim3((unsigned)ndms), dim3(1024), 0, s, out, ld_out, nout,
                     norm, nsigma, sample0, d_sample0, dm_start, dm_step, counts, offsets, cands, capacity);
  return hipGetLastError();
}

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices];   // device address of `scratch` per device
}  // namespace

hipError_t detect_scratch_setup(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *ptr = g_scratch_dev[dev];
  return hipSuccess;
}

hipError_t launch_detect_noalloc(const float* out, int64_t ld_out, int64_t nout, int32_t ndms,
                                 const NormDev* norm, int64_t sample0, const int64_t* d_sample0, double nsigma,
                                 double dm_start, double dm_step, CandDev* cands, int64_t capacity,
                                 int64_t* d_count, PeakDev* peaks, hipStream_t s) {
  if (ndms < 1 || ndms > kDetectNoAllocMaxDms) return hipErrorInvalidValue;
  void* work = nullptr;
  hipError_t e = detect_scratch_setup(&work);
  if (e != hipSuccess) return e;
  // every (row, segment) count is written by the count pass and every offset
  // by the scan before anything reads them, so nothing needs clearing
  return launch_detect(out, ld_out, nout, ndms, norm, sample0, d_sample0, nsigma, dm_start, dm_step, cands,
                       capacity, d_count, peaks, work, s);
}

}  // namespace mbtp
