// Windowed median filter of a dedispersed plane (Sec. 2.2.3, Eq. 2), for
// gfx950.  Every sample becomes the median of the 2h+1 samples centred on
// it; beyond a row's ends the end sample repeats.
//
// One 256-thread workgroup per 1024 outputs of a row: the tile and its
// h-sample halo are staged in LDS (clamped indices, coalesced loads), then
// each thread takes 4 outputs 256 apart (coalesced stores, conflict-free LDS
// reads), gathers its 2h+1 window samples into registers and selects the
// median with a compile-time compare-exchange network.  fminf / fmaxf return
// one of their operands, so the output is exactly one of the inputs.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mbtp {
namespace {

constexpr int kMedTile = 1024;
constexpr int kMedThreads = 256;

template <int H>
__global__ __launch_bounds__(kMedThreads) void median_kernel(const float* __restrict__ in, int64_t ld_in,
                                                             float* __restrict__ out, int64_t ld_out,
                                                             int64_t ncols, int64_t ntiles) {
  __shared__ float sh[kMedTile + 2 * kMedianMaxHalf];
  const int64_t row = blockIdx.x / ntiles;
  const int64_t t0 = (blockIdx.x % ntiles) * kMedTile;
  const float* r = in + row * ld_in;
  for (int i = threadIdx.x; i < kMedTile + 2 * H; i += kMedThreads) {
    int64_t t = t0 - H + i;
    t = t < 0 ? 0 : (t >= ncols ? ncols - 1 : t);
    sh[i] = r[t];
  }
  __syncthreads();
  float* o = out + row * ld_out;
#pragma unroll
  for (int j = 0; j < kMedTile / kMedThreads; ++j) {
    const int k = threadIdx.x + kMedThreads * j;
    const int64_t m = t0 + k;
    if (m < ncols) {
      float v[2 * H + 1];
#pragma unroll
      for (int q = 0; q < 2 * H + 1; ++q) v[q] = sh[k + q];
      // after pass i, v[i] is the i-th smallest of the window
#pragma unroll
      for (int i = 0; i <= H; ++i)
#pragma unroll
        for (int q = i + 1; q < 2 * H + 1; ++q) {
          const float a = v[i], b = v[q];
          v[i] = fminf(a, b);
          v[q] = fmaxf(a, b);
        }
      o[m] = v[H];
    }
  }
}

template <int H>
hipError_t launch_h(const float* in, int64_t ld_in, float* out, int64_t ld_out, int32_t nrows,
                    int64_t ncols, hipStream_t s) {
  const int64_t ntiles = (ncols + kMedTile - 1) / kMedTile;
  hipLaunchKernelGGL(median_kernel<H>, dim3((unsigned)(ntiles * nrows)), dim3(kMedThreads), 0, s, in,
                     ld_in, out, ld_out, ncols, ntiles);
  return hipGetLastError();
}

}  // namespace

int64_t median_max_workgroups() { return 2147483647; }

int64_t median_tile() { return kMedTile; }

hipError_t launch_median(const float* in, int64_t ld_in, float* out, int64_t ld_out, int32_t nrows,
                         int64_t ncols, int32_t half_width, hipStream_t s) {
  switch (half_width) {
#define MBTP_H(h) case h: return launch_h<h>(in, ld_in, out, ld_out, nrows, ncols, s);
    MBTP_H(0) MBTP_H(1) MBTP_H(2) MBTP_H(3) MBTP_H(4) MBTP_H(5) MBTP_H(6) MBTP_H(7) MBTP_H(8)
    MBTP_H(9) MBTP_H(10) MBTP_H(11) MBTP_H(12) MBTP_H(13) MBTP_H(14) MBTP_H(15) MBTP_H(16)
#undef MBTP_H
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mbtp
