// Channelised power of beamformed voltages (Sec. 2.2), for gfx950: 16-bit
// complex samples (re, im) in the beam's channel/time order (Sec. 2.1) ->
// FP32 power in the same channel rows, the filterbank the rest of the path
// reads.
//
// A stream of 4 bytes in and 4 bytes out per sample.  One 256-thread
// workgroup covers 4096 samples of one channel row: each thread takes four
// 16-byte loads of 4 complex samples, forms re^2 + im^2 exactly in 32-bit
// unsigned integers (at most 2^31) and rounds it once to FP32, and writes 4
// powers with one 16-byte nontemporal store (the plane is written once and
// read by the next stage, so its lines are not kept in the caches).  The
// row's tail, and planes whose rows are not 16-byte aligned, take the
// per-sample path.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mbtp {
namespace {

constexpr int kPowerTile = 4096;    // samples of a row per workgroup

__device__ inline float power_of(uint32_t w) {
  const int32_t re = (int16_t)(w & 0xffffu), im = (int16_t)(w >> 16);
  const uint32_t p = (uint32_t)(re * re) + (uint32_t)(im * im);
  return (float)p;                  // one rounding to nearest
}

__global__ __launch_bounds__(256) void power_kernel(const uint32_t* __restrict__ in, int64_t ld_in, int64_t T,
                                                    float* __restrict__ out, int64_t ld_out, int64_t ntiles,
                                                    int vec) {
  const int64_t row = blockIdx.x / ntiles;
  const int64_t base = (blockIdx.x % ntiles) * kPowerTile;
  const uint32_t* r = in + row * ld_in;
  float* o = out + row * ld_out;
#pragma unroll
  for (int k = 0; k < kPowerTile / 1024; ++k) {
    const int64_t m = base + 1024 * k + 4 * threadIdx.x;
    if (vec && m + 3 < T) {
      const uint4 w = *reinterpret_cast<const uint4*>(r + m);
      __builtin_nontemporal_store(f32x4{power_of(w.x), power_of(w.y), power_of(w.z), power_of(w.w)},
                                  reinterpret_cast<f32x4*>(o + m));
    } else {
      for (int q = 0; q < 4; ++q)
        if (m + q < T) o[m + q] = power_of(r[m + q]);
    }
  }
}

}  // namespace

hipError_t launch_power(const int16_t* in, int64_t ld_in, int32_t C, int64_t T, float* out, int64_t ld_out,
                        hipStream_t s) {
  const int64_t ntiles = (T + kPowerTile - 1) / kPowerTile;
  const int vec = (reinterpret_cast<uintptr_t>(in) % 16 == 0 && ld_in % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0 && ld_out % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(power_kernel, dim3((unsigned)(C * ntiles)), dim3(256), 0, s,
                     reinterpret_cast<const uint32_t*>(in), ld_in, T, out, ld_out, ntiles, vec);
  return hipGetLastError();
}

}  // namespace mbtp
