// Per-DM detrending and normalisation (Sec. 2.2.3) and the n-sigma event
// threshold (Sec. 2.3) over a dedispersed plane D[ndms][ld_out] (FP32).
//
// norm:   one workgroup per DM row.  Pass 1 forms sum D, sum (t - tbar) D and
//         sum D^2 in FP64; the least-squares line follows in closed form.
//         Pass 2 forms the residual sum of squares.  Rows are read twice;
//         the second read mostly hits the L2 / MALL.
// detect: pass A counts z > nsigma per row and finds the row's peak; a
//         single-workgroup exclusive scan turns counts into output offsets;
//         pass B writes the triplets in (DM, sample) order with ballots.
// z = (D - a - b t) / sigma is formed in FP64 the same way in both passes.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace mbtp {
namespace {

constexpr double kDegenerateRtol = 1e-9;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// 256-thread block sum with a fixed tree; sh must hold 4 doubles.
__device__ inline double block_sum_256(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ __launch_bounds__(256) void norm_kernel(const float* __restrict__ out, int64_t ld_out,
                                                   int64_t nout, NormDev* __restrict__ norm) {
  __shared__ double sh[4];
  const int d = blockIdx.x;
  const float* row = out + (int64_t)d * ld_out;
  const double N = (double)nout;
  const double tbar = 0.5 * (N - 1.0);
  double s1 = 0.0, st = 0.0, s2 = 0.0;
  // 4 samples per thread per step (rows are 16-byte aligned, ld_out % 4 == 0)
  const int64_t n4 = nout / 4;
  for (int64_t i = threadIdx.x; i < n4; i += 256) {
    const float4 v = reinterpret_cast<const float4*>(row)[i];
    const double t = (double)(4 * i) - tbar;
    const double a0 = v.x, a1 = v.y, a2 = v.z, a3 = v.w;
    s1 += (a0 + a1) + (a2 + a3);
    st += (t * a0 + (t + 1.0) * a1) + ((t + 2.0) * a2 + (t + 3.0) * a3);
    s2 += (a0 * a0 + a1 * a1) + (a2 * a2 + a3 * a3);
  }
  for (int64_t i = 4 * n4 + threadIdx.x; i < nout; i += 256) {
    const double v = row[i];
    s1 += v; st += ((double)i - tbar) * v; s2 += v * v;
  }
  s1 = block_sum_256(s1, sh);
  st = block_sum_256(st, sh);
  s2 = block_sum_256(s2, sh);
  const double stt = N * (N * N - 1.0) / 12.0;
  const double b = stt > 0.0 ? st / stt : 0.0;
  const double a = (nout > 0 ? s1 / N : 0.0) - b * tbar;
  double r2 = 0.0;
  for (int64_t i = threadIdx.x; i < n4; i += 256) {
    const float4 v = reinterpret_cast<const float4*>(row)[i];
    const double t = (double)(4 * i);
    const double r0 = ((double)v.x - a) - b * t;
    const double r1 = ((double)v.y - a) - b * (t + 1.0);
    const double rr2 = ((double)v.z - a) - b * (t + 2.0);
    const double r3 = ((double)v.w - a) - b * (t + 3.0);
    r2 += (r0 * r0 + r1 * r1) + (rr2 * rr2 + r3 * r3);
  }
  for (int64_t i = 4 * n4 + threadIdx.x; i < nout; i += 256) {
    const double r = ((double)row[i] - a) - b * (double)i;
    r2 += r * r;
  }
  r2 = block_sum_256(r2, sh);
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

__device__ inline double zval(const float* row, int64_t t, const NormDev& n) {
  if (n.degenerate) return 0.0;
  return (((double)row[t] - n.a) - n.b * (double)t) / n.sigma;
}

// Pass A: count and peak per row.
__global__ __launch_bounds__(256) void detect_count_kernel(const float* __restrict__ out,
                                                           int64_t ld_out, int64_t nout,
                                                           const NormDev* __restrict__ norm,
                                                           double nsigma, int64_t sample0,
                                                           int64_t* __restrict__ counts,
                                                           PeakDev* __restrict__ peaks) {
  __shared__ double shz[4];
  __shared__ int64_t sht[4];
  __shared__ int64_t shc[4];
  const int d = blockIdx.x;
  const float* row = out + (int64_t)d * ld_out;
  const NormDev n = norm[d];
  int64_t cnt = 0;
  double best = -INFINITY;
  int64_t bt = INT64_MAX;
  for (int64_t t = threadIdx.x; t < nout; t += 256) {
    const double z = zval(row, t, n);
    cnt += (z > nsigma) ? 1 : 0;
    if (z > best) { best = z; bt = t; }   // ascending t per thread: keeps the earliest
  }
  // wave reduction: (max z, min t)
  for (int off = 32; off >= 1; off >>= 1) {
    const double oz = __shfl_xor(best, off, 64);
    const int64_t ot = __shfl_xor(bt, off, 64);
    const int64_t oc = __shfl_xor(cnt, off, 64);
    cnt += oc;
    if (oz > best || (oz == best && ot < bt)) { best = oz; bt = ot; }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { shz[w] = best; sht[w] = bt; shc[w] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bz = shz[0];
    int64_t btt = sht[0];
    int64_t c = shc[0];
    for (int k = 1; k < 4; ++k) {
      c += shc[k];
      if (shz[k] > bz || (shz[k] == bz && sht[k] < btt)) { bz = shz[k]; btt = sht[k]; }
    }
    counts[d] = c;
    if (peaks) {
      PeakDev p;
      p.sample = sample0 + (nout > 0 ? btt : 0);
      p.snr = nout > 0 ? (float)bz : 0.0f;
      p.reserved = 0;
      peaks[d] = p;
    }
  }
}

// Exclusive scan of the per-row counts (one 1024-thread workgroup).
__global__ __launch_bounds__(1024) void detect_scan_kernel(const int64_t* __restrict__ counts,
                                                           int32_t ndms, int64_t* __restrict__ offsets,
                                                           int64_t* __restrict__ total) {
  __shared__ int64_t sh[1024];
  int64_t carry = 0;
  for (int32_t base = 0; base < ndms; base += 1024) {
    const int32_t i = base + threadIdx.x;
    const int64_t v = (i < ndms) ? counts[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < ndms) offsets[i] = carry + sh[threadIdx.x] - v;
    carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// Pass B: write the triplets of each row in sample order.
__global__ __launch_bounds__(256) void detect_write_kernel(const float* __restrict__ out,
                                                           int64_t ld_out, int64_t nout,
                                                           const NormDev* __restrict__ norm,
                                                           double nsigma, int64_t sample0,
                                                           double dm_start, double dm_step,
                                                           const int64_t* __restrict__ offsets,
                                                           CandDev* __restrict__ cands,
                                                           int64_t capacity) {
  __shared__ int wcount[4];
  const int d = blockIdx.x;
  const float* row = out + (int64_t)d * ld_out;
  const NormDev n = norm[d];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float dmv = (float)(dm_start + (double)d * dm_step);
  int64_t pos = offsets[d];
  for (int64_t t0 = 0; t0 < nout; t0 += 256) {
    const int64_t t = t0 + threadIdx.x;
    double z = 0.0;
    bool hit = false;
    if (t < nout) {
      z = zval(row, t, n);
      hit = z > nsigma;
    }
    const unsigned long long bal = __ballot(hit);
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int k = 0; k < wave; ++k) before += wcount[k];
    const int total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    if (hit) {
      const unsigned long long lower = (lane == 0) ? 0ull : (bal & ((1ull << lane) - 1ull));
      const int64_t k = pos + before + __popcll(lower);
      if (k < capacity) {
        CandDev cd;
        cd.dm_index = d;
        cd.reserved = 0;
        cd.sample = sample0 + t;
        cd.snr = (float)z;
        cd.dm = dmv;
        cands[k] = cd;
      }
    }
    pos += total;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_norm(const float* out, int64_t ld_out, int64_t nout, int32_t ndms, NormDev* norm,
                       hipStream_t s) {
  hipLaunchKernelGGL(norm_kernel, dim3((unsigned)ndms), dim3(256), 0, s, out, ld_out, nout, norm);
  return hipGetLastError();
}

hipError_t launch_detect(const float* out, int64_t ld_out, int64_t nout, int32_t ndms,
                         const NormDev* norm, int64_t sample0, double nsigma, double dm_start,
                         double dm_step, CandDev* cands, int64_t capacity, int64_t* d_count,
                         PeakDev* peaks, void* work, hipStream_t s) {
  int64_t* counts = static_cast<int64_t*>(work);
  int64_t* offsets = counts + ndms + 1;
  hipLaunchKernelGGL(detect_count_kernel, dim3((unsigned)ndms), dim3(256), 0, s, out, ld_out, nout,
                     norm, nsigma, sample0, counts, peaks);
  hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(1024), 0, s, counts, ndms, offsets, d_count);
  hipLaunchKernelGGL(detect_write_kernel, dim3((unsigned)ndms), dim3(256), 0, s, out, ld_out, nout,
                     norm, nsigma, sample0, dm_start, dm_step, offsets, cands, capacity);
  return hipGetLastError();
}

}  // namespace mbtp
