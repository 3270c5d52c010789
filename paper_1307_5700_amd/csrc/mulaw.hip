// mu-law codec of the data writer (Sec. 2.4, Eq. 5), for gfx950.
//
// Encode: one 1024-thread workgroup per row of an FP32 power plane.  The
// row's largest |x| (X) comes from one pass of 16-byte loads and a block
// max; a second pass (mostly from L2) maps every sample to its 8-bit code
//   q = floor(255 * log1p(mu * x / X) / log1p(mu) + 1/2),  x < 0 taken as 0,
// in FP64 with each operation rounded on its own (no contraction), so the
// code, a decision taken in floating point, follows the same steps
// wherever it is computed.  X is stored per row for the decoder.
// Decode: x = X / mu * expm1(q / 255 * log1p(mu)), FP64, rounded to FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mbtp {
namespace {

constexpr double kLevels = 255.0;

__device__ inline uint8_t code_of(float x, double mu, double Xd, double l1mu) {
  if (!(Xd > 0.0)) return 0;
  const double xd = x > 0.0f ? (double)x : 0.0;
  const double t = __ddiv_rn(__dmul_rn(mu, xd), Xd);
  const double v = __ddiv_rn(__dmul_rn(kLevels, log1p(t)), l1mu);
  return (uint8_t)floor(__dadd_rn(v, 0.5));
}

__global__ __launch_bounds__(1024) void mulaw_encode_kernel(const float* __restrict__ in, int64_t ld_in,
                                                            int64_t ncols, double mu, double l1mu,
                                                            uint8_t* __restrict__ codes, int64_t ld_codes,
                                                            float* __restrict__ xmax, int vin, int vout) {
  __shared__ float sh[16];
  const int64_t row = blockIdx.x;
  const float* r = in + row * ld_in;
  uint8_t* c = codes + row * ld_codes;
  const int tid = threadIdx.x;
  const int64_t n4 = vin ? ncols / 4 : 0;
  float m = 0.0f;
  for (int64_t i = tid; i < n4; i += 1024) {
    const float4 v = reinterpret_cast<const float4*>(r)[i];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
  }
  for (int64_t i = 4 * n4 + tid; i < ncols; i += 1024) m = fmaxf(m, fabsf(r[i]));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((tid & 63) == 0) sh[tid >> 6] = m;
  __syncthreads();
  float X = 0.0f;
#pragma unroll
  for (int k = 0; k < 16; ++k) X = fmaxf(X, sh[k]);
  if (tid == 0) xmax[row] = X;
  const double Xd = X;
  const int64_t q4 = (vin && vout) ? ncols / 4 : 0;
  for (int64_t i = tid; i < q4; i += 1024) {
    const float4 v = reinterpret_cast<const float4*>(r)[i];
    const uint32_t w = (uint32_t)code_of(v.x, mu, Xd, l1mu) | ((uint32_t)code_of(v.y, mu, Xd, l1mu) << 8) |
                       ((uint32_t)code_of(v.z, mu, Xd, l1mu) << 16) | ((uint32_t)code_of(v.w, mu, Xd, l1mu) << 24);
    reinterpret_cast<uint32_t*>(c)[i] = w;
  }
  for (int64_t i = 4 * q4 + tid; i < ncols; i += 1024) c[i] = code_of(r[i], mu, Xd, l1mu);
}

__device__ inline float value_of(uint8_t q, double scale, double step) {
  return (float)__dmul_rn(scale, expm1(__dmul_rn((double)q / kLevels, step)));
}

__global__ __launch_bounds__(256) void mulaw_decode_kernel(const uint8_t* __restrict__ codes, int64_t ld_codes,
                                                           const float* __restrict__ xmax, int64_t ncols,
                                                           int64_t ntiles, double mu, double l1mu,
                                                           float* __restrict__ out, int64_t ld_out, int vec) {
  const int64_t row = blockIdx.x / ntiles;
  const int64_t m = (blockIdx.x % ntiles) * 1024 + 4 * threadIdx.x;
  const uint8_t* c = codes + row * ld_codes;
  float* o = out + row * ld_out;
  const double scale = __ddiv_rn((double)xmax[row], mu);
  if (vec && m + 3 < ncols) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(c + m);
    *reinterpret_cast<float4*>(o + m) = make_float4(value_of(w & 0xffu, scale, l1mu), value_of((w >> 8) & 0xffu, scale, l1mu),
                                                    value_of((w >> 16) & 0xffu, scale, l1mu), value_of(w >> 24, scale, l1mu));
  } else {
    for (int j = 0; j < 4; ++j)
      if (m + j < ncols) o[m + j] = value_of(c[m + j], scale, l1mu);
  }
}

}  // namespace

hipError_t launch_mulaw_encode(const float* in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                               uint8_t* codes, int64_t ld_codes, float* xmax, hipStream_t s) {
  const int vin = (reinterpret_cast<uintptr_t>(in) % 16 == 0 && ld_in % 4 == 0) ? 1 : 0;
  const int vout = (reinterpret_cast<uintptr_t>(codes) % 4 == 0 && ld_codes % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(mulaw_encode_kernel, dim3((unsigned)nrows), dim3(1024), 0, s, in, ld_in, ncols,
                     (double)mu, log1p((double)mu), codes, ld_codes, xmax, vin, vout);
  return hipGetLastError();
}

hipError_t launch_mulaw_decode(const uint8_t* codes, int64_t ld_codes, const float* xmax, int32_t nrows,
                               int64_t ncols, float mu, float* out, int64_t ld_out, hipStream_t s) {
  const int64_t ntiles = (ncols + 1023) / 1024;
  const int vec = (reinterpret_cast<uintptr_t>(codes) % 4 == 0 && ld_codes % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0 && ld_out % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(mulaw_decode_kernel, dim3((unsigned)(ntiles * nrows)), dim3(256), 0, s, codes, ld_codes,
                     xmax, ncols, ntiles, (double)mu, log1p((double)mu), out, ld_out, vec);
  return hipGetLastError();
}

}  // namespace mbtp
