// Windowed median filter of a dedispersed plane (Sec. 2.2.3, Eq. 2), for
// gfx950.  Every sample becomes the median of the 2h+1 samples centred on
// it; beyond a row's ends the end sample repeats.
//
// One 256-thread workgroup per 1024 outputs of a row.  The tile and its
// halo are staged in LDS, indices clamped to the row, with the left halo
// rounded up to a quad so the tile body stays 16-byte aligned there; the
// body is loaded with 16-byte loads when both planes allow it.  Each thread
// then takes 4 consecutive outputs: their 2h+4 window samples come from a few
// 16-byte LDS reads (consecutive lanes, consecutive addresses), each
// output's median from a compile-time compare-exchange network, and the 4
// results leave in one 16-byte store.  fminf / fmaxf return one of their
// operands, so every output is exactly one of the inputs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mbtp {
namespace {

constexpr int kMedTile = 1024;
constexpr int kMedThreads = 256;

template <int H>
__global__ __launch_bounds__(kMedThreads) void median_kernel(const float* __restrict__ in, int64_t ld_in,
                                                             float* __restrict__ out, int64_t ld_out,
                                                             int64_t ncols, int64_t ntiles, int vec) {
  constexpr int HP = (H + 3) & ~3;                  // left halo, whole quads
  constexpr int NS = kMedTile + 2 * HP;             // staged samples
  constexpr int O = HP - H;                         // first window sample of a thread's quad
  constexpr int NQ = (O + 3 + 2 * H) / 4 + 1;       // quads read per thread
  __shared__ float4 sh4[(kMedTile + 2 * ((kMedianMaxHalf + 3) & ~3)) / 4];
  float* sh = reinterpret_cast<float*>(sh4);
  const int64_t row = blockIdx.x / ntiles;
  const int64_t t0 = (blockIdx.x % ntiles) * kMedTile;
  const float* r = in + row * ld_in;
  const bool full = vec && t0 + kMedTile <= ncols;  // uniform
  if (full) {
    // body: 16-byte loads; halos: clamped scalar loads
    reinterpret_cast<float4*>(sh + HP)[threadIdx.x] = reinterpret_cast<const float4*>(r + t0)[threadIdx.x];
    if (threadIdx.x < 2 * HP) {
      const int i = threadIdx.x < HP ? threadIdx.x : kMedTile + threadIdx.x;
      int64_t t = t0 - HP + i;
      t = t < 0 ? 0 : (t >= ncols ? ncols - 1 : t);
      sh[i] = r[t];
    }
  } else {
    for (int i = threadIdx.x; i < NS; i += kMedThreads) {
      int64_t t = t0 - HP + i;
      t = t < 0 ? 0 : (t >= ncols ? ncols - 1 : t);
      sh[i] = r[t];
    }
  }
  __syncthreads();
  float w[4 * NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const float4 v4 = sh4[threadIdx.x + q];
    w[4 * q] = v4.x; w[4 * q + 1] = v4.y; w[4 * q + 2] = v4.z; w[4 * q + 3] = v4.w;
  }
  float res[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v[2 * H + 1];
#pragma unroll
    for (int q = 0; q < 2 * H + 1; ++q) v[q] = w[O + j + q];
    // after pass i, v[i] is the i-th smallest of the window
#pragma unroll
    for (int i = 0; i <= H; ++i)
#pragma unroll
      for (int q = i + 1; q < 2 * H + 1; ++q) {
        const float a = v[i], b = v[q];
        v[i] = fminf(a, b);
        v[q] = fmaxf(a, b);
      }
    res[j] = v[H];
  }
  const int64_t m = t0 + 4 * threadIdx.x;
  float* o = out + row * ld_out;
  if (full) {
    // nontemporal: the filtered plane is written once and read by the next stage
    __builtin_nontemporal_store(f32x4{res[0], res[1], res[2], res[3]}, reinterpret_cast<f32x4*>(o + m));
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (m + j < ncols) o[m + j] = res[j];
  }
}

template <int H>
hipError_t launch_h(const float* in, int64_t ld_in, float* out, int64_t ld_out, int32_t nrows,
                    int64_t ncols, hipStream_t s) {
  const int64_t ntiles = (ncols + kMedTile - 1) / kMedTile;
  // 16-byte accesses when every row of both planes starts 16-byte aligned
  const int vec = (reinterpret_cast<uintptr_t>(in) % 16 == 0 && ld_in % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0 && ld_out % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(median_kernel<H>, dim3((unsigned)(ntiles * nrows)), dim3(kMedThreads), 0, s, in,
                     ld_in, out, ld_out, ncols, ntiles, vec);
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
