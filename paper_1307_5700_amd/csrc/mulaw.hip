// mu-law codec of the data writer (Sec. 2.4, Eq. 5), for gfx950.
//
// Encode: one 1024-thread workgroup per row of an FP32 power plane.  The
// row's largest |x| (X) comes from one pass of 16-byte loads and a block
// max.  The code of a sample is the nearest level of Eq. (5),
//   q = floor(255 * log1p(mu * x / X) / log1p(mu) + 1/2),  x < 0 taken as 0,
// i.e. the number of level boundaries b_k = X/mu * expm1((k - 1/2)/255 *
// log1p(mu)), k = 1..255, that x reaches.  The 255 boundaries are formed in
// FP64 once per row and rounded up to FP32: x is an FP32 value, so x >= b_k
// exactly when x reaches the rounded-up boundary.  A sample's code is then
// an FP32 log estimate corrected by one comparison on each side against the
// boundaries in LDS, which makes it exact whatever the estimate's error (at
// most one level).  X is stored per row for the decoder.
// Decode: x = X / mu * expm1(q / 255 * log1p(mu)), FP64, rounded to FP32;
// the 256 values of a row are formed once per workgroup in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mbtp {
namespace {

constexpr double kLevels = 255.0;
constexpr int kDecodeTile = 8192;     // samples per decode workgroup (one 256-entry table each)

// Rows of at most kHeld * 4096 samples (16-byte aligned) are held in
// registers between the max pass and the code pass, so the plane is read
// from HBM once; longer or unaligned rows are read twice.
constexpr int kHeld = 16;          // float4 per thread

template <bool HELD>
__global__ __launch_bounds__(1024) void mulaw_encode_kernel(const float* __restrict__ in, int64_t ld_in,
                                                            int64_t ncols, double mu, double l1mu,
                                                            uint8_t* __restrict__ codes, int64_t ld_codes,
                                                            float* __restrict__ xmax, int vin, int vout) {
  __shared__ float sh[16];
  __shared__ float bound[257];           // bound[k]: least FP32 x with code >= k (k = 1..255)
  const int64_t row = blockIdx.x;
  const float* r = in + row * ld_in;
  uint8_t* c = codes + row * ld_codes;
  const int tid = threadIdx.x;
  const int64_t n4 = vin ? ncols / 4 : 0;
  float m = 0.0f;
  float4 held[HELD ? kHeld : 1];
  if (HELD) {
#pragma unroll
    for (int k = 0; k < kHeld; ++k) {
      const int64_t i = tid + 1024 * k;
      held[k] = i < n4 ? reinterpret_cast<const float4*>(r)[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  // expm1 of level boundary tid - 1/2, independent of the row: formed while
  // the row's loads are in flight
  double e = 0.0;
  if (tid >= 1 && tid <= 255) e = expm1(__dmul_rn(((double)tid - 0.5) / kLevels, l1mu));
  if (HELD) {
#pragma unroll
    for (int k = 0; k < kHeld; ++k)
      m = fmaxf(m, fmaxf(fmaxf(fabsf(held[k].x), fabsf(held[k].y)), fmaxf(fabsf(held[k].z), fabsf(held[k].w))));
  } else {
    for (int64_t i = tid; i < n4; i += 1024) {
      const float4 v = reinterpret_cast<const float4*>(r)[i];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
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
  if (tid >= 1 && tid <= 255) {
    const double b = __dmul_rn(__ddiv_rn((double)X, mu), e);
    float f = (float)b;
    if ((double)f < b) f = nextafterf(f, INFINITY);
    bound[tid] = f;
  } else if (tid == 0) {
    bound[0] = -INFINITY;
  } else if (tid == 256) {
    bound[256] = INFINITY;
  }
  __syncthreads();
  if (!(X > 0.0f)) {
    // a row of zeros: every code is 0
    for (int64_t i = tid; i < ncols; i += 1024) c[i] = 0;
    return;
  }
  const float s = (float)(mu / (double)X), inv = (float)(kLevels / l1mu);
  auto code = [&](float x) -> uint32_t {
    const float xc = fmaxf(x, 0.0f);
    int q = (int)(inv * __logf(1.0f + s * xc) + 0.5f);
    q = q < 0 ? 0 : (q > 255 ? 255 : q);
    q += (xc >= bound[q + 1]) ? 1 : 0;
    q -= (xc < bound[q]) ? 1 : 0;
    return (uint32_t)q;
  };
  if (HELD) {
#pragma unroll
    for (int k = 0; k < kHeld; ++k) {
      const int64_t i = tid + 1024 * k;
      if (i >= n4) break;
      const float4 v = held[k];
      const uint32_t w = code(v.x) | (code(v.y) << 8) | (code(v.z) << 16) | (code(v.w) << 24);
      if (vout) {
        __builtin_nontemporal_store(w, reinterpret_cast<uint32_t*>(c) + i);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) c[4 * i + j] = (uint8_t)(w >> (8 * j));
      }
    }
    for (int64_t i = 4 * n4 + tid; i < ncols; i += 1024) c[i] = (uint8_t)code(r[i]);
    return;
  }
  const int64_t q4 = (vin && vout) ? ncols / 4 : 0;
  for (int64_t i = tid; i < q4; i += 1024) {
    const float4 v = reinterpret_cast<const float4*>(r)[i];
    __builtin_nontemporal_store(code(v.x) | (code(v.y) << 8) | (code(v.z) << 16) | (code(v.w) << 24),
                                reinterpret_cast<uint32_t*>(c) + i);
  }
  for (int64_t i = 4 * q4 + tid; i < ncols; i += 1024) c[i] = (uint8_t)code(r[i]);
}

__global__ __launch_bounds__(256) void mulaw_decode_kernel(const uint8_t* __restrict__ codes, int64_t ld_codes,
                                                           const float* __restrict__ xmax, int64_t ncols,
                                                           int64_t ntiles, double mu, double l1mu,
                                                           float* __restrict__ out, int64_t ld_out, int vec) {
  __shared__ float lut[256];
  const int64_t row = blockIdx.x / ntiles;
  const int64_t base = (blockIdx.x % ntiles) * kDecodeTile;
  const uint8_t* c = codes + row * ld_codes;
  float* o = out + row * ld_out;
  const double scale = __ddiv_rn((double)xmax[row], mu);
  lut[threadIdx.x] = (float)__dmul_rn(scale, expm1(__dmul_rn((double)threadIdx.x / kLevels, l1mu)));
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < kDecodeTile / 1024; ++j) {
    const int64_t m = base + 1024 * j + 4 * threadIdx.x;
    if (vec && m + 3 < ncols) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(c + m);
      __builtin_nontemporal_store(f32x4{lut[w & 0xffu], lut[(w >> 8) & 0xffu], lut[(w >> 16) & 0xffu], lut[w >> 24]},
                                  reinterpret_cast<f32x4*>(o + m));
    } else {
      for (int q = 0; q < 4; ++q)
        if (m + q < ncols) o[m + q] = lut[c[m + q]];
    }
  }
}

// ---- 4+4-bit codec of 16-bit complex voltages -------------------------------
// Encode: one 1024-thread workgroup per channel row of (re, im) int16 pairs.
// X is the row's largest |component| (an integer up to 32768).  A
// component's magnitude level is the number of boundaries
// b_k = X/mu * expm1((k - 1/2)/7 * log1p(mu)), k = 1..7, that |x| reaches;
// |x| is an integer, so that is the number of integer thresholds ceil(b_k)
// (formed in FP64) it reaches.  The nibble is the level with the sign of x
// in bit 3; the real part's nibble is the byte's low half.
constexpr int kCplxLevels = 7;

__device__ inline uint32_t cplx_nibble(int32_t x, const int32_t (&thr)[kCplxLevels]) {
  const int32_t a = x < 0 ? -x : x;
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < kCplxLevels; ++k) m += a >= thr[k] ? 1u : 0u;
  return m | (x < 0 ? 8u : 0u);
}

__device__ inline uint32_t cplx_byte(uint32_t w, const int32_t (&thr)[kCplxLevels]) {
  return cplx_nibble((int16_t)(w & 0xffffu), thr) | (cplx_nibble((int16_t)(w >> 16), thr) << 4);
}

__device__ inline int32_t cplx_absmax(uint32_t w) {
  const int32_t re = (int16_t)(w & 0xffffu), im = (int16_t)(w >> 16);
  return max(re < 0 ? -re : re, im < 0 ? -im : im);
}

__global__ __launch_bounds__(1024) void mulaw_encode_complex_kernel(const uint32_t* __restrict__ in, int64_t ld_in,
                                                                    int64_t ncols, double mu, double l1mu,
                                                                    uint8_t* __restrict__ codes, int64_t ld_codes,
                                                                    int32_t* __restrict__ xmax, int vin, int vout) {
  __shared__ int32_t sh[16];
  __shared__ int32_t thr_s[kCplxLevels];
  const int64_t row = blockIdx.x;
  const uint32_t* r = in + row * ld_in;
  uint8_t* c = codes + row * ld_codes;
  const int tid = threadIdx.x;
  // boundary k + 1/2 without X, formed while the row is read
  double e = 0.0;
  if (tid < kCplxLevels) e = expm1(__dmul_rn(((double)tid + 0.5) / kCplxLevels, l1mu));
  const int64_t n4 = vin ? ncols / 4 : 0;
  int32_t m = 0;
  for (int64_t i = tid; i < n4; i += 1024) {
    const uint4 w = reinterpret_cast<const uint4*>(r)[i];
    m = max(m, max(max(cplx_absmax(w.x), cplx_absmax(w.y)), max(cplx_absmax(w.z), cplx_absmax(w.w))));
  }
  for (int64_t i = 4 * n4 + tid; i < ncols; i += 1024) m = max(m, cplx_absmax(r[i]));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if ((tid & 63) == 0) sh[tid >> 6] = m;
  __syncthreads();
  int32_t X = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) X = max(X, sh[k]);
  if (tid == 0) xmax[row] = X;
  if (tid < kCplxLevels) thr_s[tid] = (int32_t)ceil(__dmul_rn(__ddiv_rn((double)X, mu), e));
  __syncthreads();
  if (X == 0) {
    // a row of zeros: every code is 0
    for (int64_t i = tid; i < ncols; i += 1024) c[i] = 0;
    return;
  }
  int32_t thr[kCplxLevels];
#pragma unroll
  for (int k = 0; k < kCplxLevels; ++k) thr[k] = thr_s[k];
  const int64_t q4 = (vin && vout) ? ncols / 4 : 0;
  for (int64_t i = tid; i < q4; i += 1024) {
    const uint4 w = reinterpret_cast<const uint4*>(r)[i];
    __builtin_nontemporal_store(cplx_byte(w.x, thr) | (cplx_byte(w.y, thr) << 8) | (cplx_byte(w.z, thr) << 16) |
                                    (cplx_byte(w.w, thr) << 24),
                                reinterpret_cast<uint32_t*>(c) + i);
  }
  for (int64_t i = 4 * q4 + tid; i < ncols; i += 1024) c[i] = (uint8_t)cplx_byte(r[i], thr);
}

// Decode: one 256-thread workgroup per kDecodeTile complex samples of a row;
// the 16 values of a row's nibbles are formed once in LDS, and each thread
// turns two codes at a time into 4 FP32 values.
__global__ __launch_bounds__(256) void mulaw_decode_complex_kernel(const uint8_t* __restrict__ codes,
                                                                   int64_t ld_codes, const int32_t* __restrict__ xmax,
                                                                   int64_t ncols, int64_t ntiles, double mu,
                                                                   double l1mu, float* __restrict__ out,
                                                                   int64_t ld_out, int vec) {
  __shared__ float lut[16];
  const int64_t row = blockIdx.x / ntiles;
  const int64_t base = (blockIdx.x % ntiles) * kDecodeTile;
  const uint8_t* c = codes + row * ld_codes;
  float* o = out + row * 2 * ld_out;
  if (threadIdx.x < 16) {
    const int mag = threadIdx.x & 7;
    const float v =
        (float)__dmul_rn(__ddiv_rn((double)xmax[row], mu), expm1(__dmul_rn((double)mag / kCplxLevels, l1mu)));
    lut[threadIdx.x] = threadIdx.x >= 8 ? -v : v;
  }
  __syncthreads();
  // a 1024-code slab is 512 float4 of output: lane-consecutive 16-byte
  // stores, each of two codes (re, im, re, im)
#pragma unroll 4
  for (int j = 0; j < 2 * kDecodeTile / 1024; ++j) {
    const int64_t m = base + 512 * j + 2 * threadIdx.x;
    if (vec && m + 1 < ncols) {
      const uint32_t w = *reinterpret_cast<const uint16_t*>(c + m);
      __builtin_nontemporal_store(f32x4{lut[w & 15u], lut[(w >> 4) & 15u], lut[(w >> 8) & 15u], lut[w >> 12]},
                                  reinterpret_cast<f32x4*>(o + 2 * m));
    } else {
      for (int q = 0; q < 2; ++q)
        if (m + q < ncols) {
          const uint32_t b = c[m + q];
          o[2 * (m + q)] = lut[b & 15u];
          o[2 * (m + q) + 1] = lut[b >> 4];
        }
    }
  }
}

}  // namespace

hipError_t launch_mulaw_encode_complex(const int16_t* in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                                       uint8_t* codes, int64_t ld_codes, int32_t* xmax, hipStream_t s) {
  const int vin = (reinterpret_cast<uintptr_t>(in) % 16 == 0 && ld_in % 4 == 0) ? 1 : 0;
  const int vout = (reinterpret_cast<uintptr_t>(codes) % 4 == 0 && ld_codes % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(mulaw_encode_complex_kernel, dim3((unsigned)nrows), dim3(1024), 0, s,
                     reinterpret_cast<const uint32_t*>(in), ld_in, ncols, (double)mu, log1p((double)mu), codes,
                     ld_codes, xmax, vin, vout);
  return hipGetLastError();
}

hipError_t launch_mulaw_decode_complex(const uint8_t* codes, int64_t ld_codes, const int32_t* xmax, int32_t nrows,
                                       int64_t ncols, float mu, float* out, int64_t ld_out, hipStream_t s) {
  const int64_t ntiles = (ncols + kDecodeTile - 1) / kDecodeTile;
  const int vec = (reinterpret_cast<uintptr_t>(codes) % 2 == 0 && ld_codes % 2 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0 && ld_out % 2 == 0) ? 1 : 0;
  hipLaunchKernelGGL(mulaw_decode_complex_kernel, dim3((unsigned)(ntiles * nrows)), dim3(256), 0, s, codes,
                     ld_codes, xmax, ncols, ntiles, (double)mu, log1p((double)mu), out, ld_out, vec);
  return hipGetLastError();
}

hipError_t launch_mulaw_encode(const float* in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                               uint8_t* codes, int64_t ld_codes, float* xmax, hipStream_t s) {
  const int vin = (reinterpret_cast<uintptr_t>(in) % 16 == 0 && ld_in % 4 == 0) ? 1 : 0;
  const int vout = (reinterpret_cast<uintptr_t>(codes) % 4 == 0 && ld_codes % 4 == 0) ? 1 : 0;
  if (vin && ncols <= (int64_t)kHeld * 4096)
    hipLaunchKernelGGL(mulaw_encode_kernel<true>, dim3((unsigned)nrows), dim3(1024), 0, s, in, ld_in, ncols,
                       (double)mu, log1p((double)mu), codes, ld_codes, xmax, vin, vout);
  else
    hipLaunchKernelGGL(mulaw_encode_kernel<false>, dim3((unsigned)nrows), dim3(1024), 0, s, in, ld_in, ncols,
                       (double)mu, log1p((double)mu), codes, ld_codes, xmax, vin, vout);
  return hipGetLastError();
}

hipError_t launch_mulaw_decode(const uint8_t* codes, int64_t ld_codes, const float* xmax, int32_t nrows,
                               int64_t ncols, float mu, float* out, int64_t ld_out, hipStream_t s) {
  const int64_t ntiles = (ncols + kDecodeTile - 1) / kDecodeTile;
  const int vec = (reinterpret_cast<uintptr_t>(codes) % 4 == 0 && ld_codes % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0 && ld_out % 4 == 0) ? 1 : 0;
  hipLaunchKernelGGL(mulaw_decode_kernel, dim3((unsigned)(ntiles * nrows)), dim3(256), 0, s, codes, ld_codes,
                     xmax, ncols, ntiles, (double)mu, log1p((double)mu), out, ld_out, vec);
  return hipGetLastError();
}

}  // namespace mbtp
