// Brute-force incoherent dedispersion (Sec. 2.2.2) fused with the cleaning
// of the RFI pass (Sec. 2.2.1), for gfx950.
//
//   D[d][t] = sum_c y[c][t + s[d][c]],   y = cleaned sample (FP32)
//
// Workgroup = 256 threads = 4 wave64s covering a block of 4*G adjacent DMs
// and 256*Q consecutive outputs.  For each block of BC channels the
// workgroup stages, per channel, the input span its DMs need into LDS as four
// copies shifted by 0..3 samples, so that any DM's window starts 16-byte
// aligned in one of them; each lane then reads 4 consecutive outputs' terms
// with one ds_read_b128 (lanes contiguous: no bank conflicts).  On gfx950
// b128 LDS reads deliver about 2.6x the bytes per clock of b32 reads, and LDS
// reads are what bound this kernel.
//
// Staging: the span of channel c starts at the aligned virtual sample
// a_c = t0 + (s[d0][c] & ~3).  Each lane takes aligned quads of 4 samples
// with one vector load (plus the quad after it, for the shifted copies),
// applies the cleaning (bandpass subtraction, flagged chunk or spectrum -> 0)
// and writes the four copies with ds_write_b128.  The loads of channel block
// k+1 are issued into registers before block k is accumulated, so their HBM
// latency overlaps the LDS-bound accumulation.
//
// Accumulation: per (DM, channel) one scalar offset from the host-built relb
// table, one VALU address add, Q b128 reads and 4Q FP32 adds.  Sums form in
// partials of kAccGroup channels added to the running total in ascending
// order, so the order of every addition depends only on the channel index,
// never on the tiling, the stream position or the batch.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <type_traits>

#include "internal.h"

namespace mbtp {
namespace {

template <typename T> struct Quad;
template <> struct Quad<float> {
  using Raw = float4;
  static __device__ inline Raw load(const float* p) { return *reinterpret_cast<const float4*>(p); }
  static __device__ inline float4 widen(Raw r) { return r; }
  static __device__ inline float one(const float* p) { return *p; }
};
template <> struct Quad<__half> {
  using Raw = uint2;
  static __device__ inline Raw load(const __half* p) { return *reinterpret_cast<const uint2*>(p); }
  static __device__ inline float4 widen(Raw r) {
    const float2 a = __half22float2(*reinterpret_cast<const __half2*>(&r.x));
    const float2 b = __half22float2(*reinterpret_cast<const __half2*>(&r.y));
    return make_float4(a.x, a.y, b.x, b.y);
  }
  static __device__ inline float one(const __half* p) { return __half2float(*p); }
};
template <> struct Quad<uint8_t> {
  using Raw = uint32_t;
  static __device__ inline Raw load(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }
  static __device__ inline float4 widen(Raw r) {
    return make_float4((float)(r & 0xffu), (float)((r >> 8) & 0xffu), (float)((r >> 16) & 0xffu),
                       (float)(r >> 24));
  }
  static __device__ inline float one(const uint8_t* p) { return (float)*p; }
};

// One aligned quad of virtual samples in flight.
enum : uint32_t { kReady = 0, kChunk = 1 };

template <typename TIN> struct Staged {
  float4 v;                          // ring / tail values (and f32 chunk values)
  typename Quad<TIN>::Raw raw;       // u8 / f16 chunk values
  uint32_t g;                        // spectrum-flag bytes of the quad
  uint32_t meta;                     // kind | chunk-flag << 1
};

// Chunk index of chunk sample t (W a power of two: a shift).
__device__ inline uint32_t chunk_of(const CleanView& cv, int64_t t) {
  return cv.wshift >= 0 ? (uint32_t)t >> cv.wshift : (uint32_t)t / cv.W;
}

struct RowCtx {
  const void* xrow;
  const float* ringrow;
  const uint8_t* cfrow;
  float fit;
  int64_t a;     // virtual index of the row's first staged sample (aligned)
};

template <typename TIN, bool CLEAN>
__device__ inline float clean_one(const DedispArgs& A, const TIN* xrow, const uint8_t* cfrow, float fit,
                                  int64_t t) {
  const float v = Quad<TIN>::one(xrow + t);
  if (!CLEAN) return v;
  const bool f = (cfrow[chunk_of(A.clean, t)] & 2) || A.clean.gflags[t];
  return f ? 0.0f : v - fit;
}

// Issues the loads of the quad at virtual index tau (a multiple of 4).
template <typename TIN, bool CLEAN, bool RING>
__device__ inline void issue(Staged<TIN>& s, const DedispArgs& A, const RowCtx& r, int64_t tau,
                             int64_t V) {
  const TIN* xrow = static_cast<const TIN*>(r.xrow);
  const int64_t v = RING ? A.ring_valid : 0;
  if (tau >= v && tau + 3 < V) {
    const int64_t t = tau - v;
    if constexpr (std::is_same<TIN, float>::value) s.v = Quad<TIN>::load(xrow + t);
    else s.raw = Quad<TIN>::load(xrow + t);
    uint32_t meta = kChunk;
    if (CLEAN) {
      s.g = *reinterpret_cast<const uint32_t*>(A.clean.gflags + t);
      meta |= (uint32_t)(r.cfrow[chunk_of(A.clean, t)] & 2);
    }
    s.meta = meta;
  } else if (RING && tau < v) {
    int64_t p = A.ring_p0 + tau;
    if (p >= A.R) p -= A.R;
    s.v = *reinterpret_cast<const float4*>(r.ringrow + p);
    s.meta = kReady;
  } else {
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t ti = tau + i;
      e[i] = (ti < V) ? clean_one<TIN, CLEAN>(A, xrow, r.cfrow, r.fit, ti - v) : 0.0f;
    }
    s.v = make_float4(e[0], e[1], e[2], e[3]);
    s.meta = kReady;
  }
}

template <typename TIN, bool CLEAN>
__device__ inline float4 finish(const Staged<TIN>& s, float fit) {
  if ((s.meta & 1) == kReady) return s.v;
  float4 f;
  if constexpr (std::is_same<TIN, float>::value) f = s.v;
  else f = Quad<TIN>::widen(s.raw);
  if (CLEAN) {
    const bool cf = (s.meta & 2) != 0;
    f.x = (cf || (s.g & 0xffu)) ? 0.0f : f.x - fit;
    f.y = (cf || (s.g & 0xff00u)) ? 0.0f : f.y - fit;
    f.z = (cf || (s.g & 0xff0000u)) ? 0.0f : f.z - fit;
    f.w = (cf || (s.g & 0xff000000u)) ? 0.0f : f.w - fit;
  }
  return f;
}

template <typename TIN, bool CLEAN, bool RING, int G, int Q, int BC>
__global__ __launch_bounds__(256) void dedisp_kernel(DedispArgs A, const int32_t* __restrict__ relb,
                                                     const float* __restrict__ fit32) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  constexpr int BD = 4 * G, BT = 256 * Q;
  constexpr int RPW = BC / 4;                      // staged rows per wave
  constexpr int KM = kStageQuads / RPW;            // quad pairs per lane per row
  static_assert(BC % 4 == 0 && G % 4 == 0 && RPW * KM == kStageQuads, "tiling");
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;

  // Workgroup id -> tile.  Consecutive workgroups go to different XCDs; give
  // each XCD a contiguous range of tiles, DM block fastest, so the blocks
  // that share a time tile run on the same L2 at about the same time.
  const int ntile = A.n_dblocks * A.n_ttiles;
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int q8 = ntile >> 3, rem = ntile & 7;
  const int tile = xcd * q8 + min(xcd, rem) + slot;
  const int dblock = tile % A.n_dblocks;
  const int ttile = tile / A.n_dblocks;

  const int C = A.C;
  const int d0 = dblock * BD;
  const int dlast = min(d0 + BD, A.ndms) - 1;
  const int64_t t0 = (int64_t)ttile * BT;            // virtual index of this tile's first output
  const int RS = A.rs;
  const int RS4 = RS >> 2;
  const int64_t V = (RING ? A.ring_valid : 0) + A.L;
  const int32_t* __restrict__ dl = A.delays;

  Staged<TIN> st[RPW][KM];
  float rowfit[RPW];
  int offreg = 0;                                    // one relb entry per thread per block
  int* lds_off = reinterpret_cast<int*>(lds + BC * 4 * RS);   // [BC][BD]

  auto row_ctx = [&](int c) {
    RowCtx r;
    r.xrow = static_cast<const TIN*>(A.x) + (int64_t)c * A.ld;
    r.ringrow = RING ? A.ring + (int64_t)c * A.R : nullptr;
    r.cfrow = CLEAN ? A.clean.cflags + (int64_t)c * A.clean.J : nullptr;
    r.fit = CLEAN ? fit32[c] : 0.0f;
    r.a = t0 + (dl[(int64_t)d0 * C + c] & ~3);
    return r;
  };

  // Loads of channel block cb0 into registers: per lane one aligned quad per
  // (row, k) at staged position 4m, m = lane + 64k, and one relb entry.
  auto issue_block = [&](int cb0) {
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int c = cb0 + wave + 4 * rr;
      if (c < C) {
        const RowCtx r = row_ctx(c);
        rowfit[rr] = r.fit;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const int m = lane + 64 * k;
          if (m < RS4) issue<TIN, CLEAN, RING>(st[rr][k], A, r, r.a + 4 * m, V);
          else { st[rr][k].v = make_float4(0.f, 0.f, 0.f, 0.f); st[rr][k].meta = kReady; }
        }
      }
    }
    if (tid < BD * BC) {
      const int dd = tid % BD, cb = tid / BD;
      const int d = min(d0 + dd, dlast);
      offreg = (cb0 + cb < C) ? relb[(int64_t)d * A.relb_ld + cb0 + cb] : 0;
    }
  };

  // Cleans the block's quads and writes the four shifted copies.  The quad
  // after a lane's quad is the next lane's (a DPP wave shift); lane 63 takes
  // lane 0's quad of the next k.  The last quad of a row has no successor in
  // registers, but no DM window ever reads the copies it would feed.
  auto write_block = [&](int cb0) {
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int cb = wave + 4 * rr;
      if (cb0 + cb < C) {
        float* row = lds + cb * 4 * RS;
        float4 lo[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) lo[k] = finish<TIN, CLEAN>(st[rr][k], rowfit[rr]);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          float4 hi;
          hi.x = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(lo[k].x), 0x130, 0xf, 0xf, false));
          hi.y = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(lo[k].y), 0x130, 0xf, 0xf, false));
          hi.z = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(lo[k].z), 0x130, 0xf, 0xf, false));
          if (k + 1 < KM) {
            const float4 nx = lo[(k + 1) % KM];
            const float ax = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(nx.x), 0));
            const float ay = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(nx.y), 0));
            const float az = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(nx.z), 0));
            if (lane == 63) { hi.x = ax; hi.y = ay; hi.z = az; }
          }
          const int m = lane + 64 * k;
          if (m < RS4) {
            const float4 l = lo[k];
            *reinterpret_cast<float4*>(row + 4 * m) = l;
            *reinterpret_cast<float4*>(row + RS + 4 * m) = make_float4(l.y, l.z, l.w, hi.x);
            *reinterpret_cast<float4*>(row + 2 * RS + 4 * m) = make_float4(l.z, l.w, hi.x, hi.y);
            *reinterpret_cast<float4*>(row + 3 * RS + 4 * m) = make_float4(l.w, hi.x, hi.y, hi.z);
          }
        }
      }
    }
    if (tid < BD * BC) lds_off[tid] = offreg;       // [cb][dd] with dd fastest
  };

  float4 acc[G][Q], tot[G][Q];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      acc[g][q] = make_float4(0.f, 0.f, 0.f, 0.f);
      tot[g][q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

  issue_block(0);
  write_block(0);
  __syncthreads();
  for (int cb0 = 0; cb0 < C; cb0 += BC) {
    const int next = cb0 + BC;
    if (next < C) issue_block(next);
    // ---- accumulate channel block cb0 ----
#pragma unroll
    for (int cb = 0; cb < BC; ++cb) {
      const int c = cb0 + cb;
      if (c < C) {
        const char* rowb = reinterpret_cast<const char*>(lds + cb * 4 * RS) + 16 * lane;
        int off[G];
#pragma unroll
        for (int g = 0; g < G; g += 4) {
          const int4 o4 = *reinterpret_cast<const int4*>(lds_off + cb * BD + wave * G + g);
          off[g] = o4.x; off[g + 1] = o4.y; off[g + 2] = o4.z; off[g + 3] = o4.w;
        }
        float4 v[G][Q];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int q = 0; q < Q; ++q) v[g][q] = reinterpret_cast<const float4*>(rowb + off[g])[64 * q];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            acc[g][q].x += v[g][q].x; acc[g][q].y += v[g][q].y;
            acc[g][q].z += v[g][q].z; acc[g][q].w += v[g][q].w;
          }
        if (((c + 1) & (kAccGroup - 1)) == 0) {
#pragma unroll
          for (int g = 0; g < G; ++g)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
              tot[g][q].x += acc[g][q].x; tot[g][q].y += acc[g][q].y;
              tot[g][q].z += acc[g][q].z; tot[g][q].w += acc[g][q].w;
              acc[g][q] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
      }
    }
    __syncthreads();
    if (next < C) {
      write_block(next);
      __syncthreads();
    }
  }
  if ((C & (kAccGroup - 1)) != 0) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        tot[g][q].x += acc[g][q].x; tot[g][q].y += acc[g][q].y;
        tot[g][q].z += acc[g][q].z; tot[g][q].w += acc[g][q].w;
      }
  }
  // ---- store: output j sits at virtual index phase + j ----
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int d = d0 + wave * G + g;
    if (d > dlast) continue;
    float* orow = A.out + (int64_t)d * A.ld_out;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t j = t0 + 4 * lane + 256 * q - A.phase;
      if (A.phase == 0 && j + 3 < A.nout) {
        *reinterpret_cast<float4*>(orow + j) = tot[g][q];
      } else {
        const float vv[4] = {tot[g][q].x, tot[g][q].y, tot[g][q].z, tot[g][q].w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (j + i >= 0 && j + i < A.nout) orow[j + i] = vv[i];
      }
    }
  }
}

// Per-(DM, channel) LDS byte offset of the DM's window inside the channel's
// 4-copy region: with p = s[d][c] - (s[d0][c] & ~3), the window starts at
// position p & ~3 of copy p & 3.
__global__ void relb_kernel(const int32_t* __restrict__ delays, int32_t C, int32_t ndms, int32_t BD,
                            int32_t RS, int32_t ldr, int32_t* __restrict__ relb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ldr * ndms) return;
  const int32_t d = (int32_t)(i / ldr), c = (int32_t)(i % ldr);
  if (c >= C) { relb[i] = 0; return; }
  const int32_t d0 = (d / BD) * BD;
  const int32_t p = delays[(int64_t)d * C + c] - (delays[(int64_t)d0 * C + c] & ~3);
  relb[i] = ((p & 3) * RS + (p & ~3)) * 4;
}

// Ring update: write the chunk's last min(L, R) cleaned samples at ring
// position (seen + t) mod R.
template <typename TIN, bool CLEAN>
__global__ __launch_bounds__(256) void ring_update_kernel(const TIN* __restrict__ x, int64_t ld,
                                                          int64_t L, int32_t C, CleanView cv,
                                                          const float* __restrict__ fit32,
                                                          float* __restrict__ ring, int64_t R,
                                                          int64_t seen) {
  const int c = blockIdx.y;
  const int64_t n = min(L, R);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || c >= C) return;
  const int64_t t = L - n + i;
  float v = Quad<TIN>::one(x + (int64_t)c * ld + t);
  if (CLEAN) {
    const bool flagged = (cv.cflags[(int64_t)c * cv.J + chunk_of(cv, t)] & 2) || cv.gflags[t];
    v = flagged ? 0.0f : v - fit32[c];
  }
  ring[(int64_t)c * R + (seen + t) % R] = v;
}

template <typename TIN, bool CLEAN, bool RING, int G, int Q, int BC>
hipError_t launch_one(const DedispArgs& a, const int32_t* relb, const float* fit32, size_t lds,
                      hipStream_t s) {
  const unsigned grid = (unsigned)a.n_dblocks * (unsigned)a.n_ttiles;
  hipLaunchKernelGGL((dedisp_kernel<TIN, CLEAN, RING, G, Q, BC>), dim3(grid), dim3(256), lds, s,
                     a, relb, fit32);
  return hipGetLastError();
}

#define MBTP_TILINGS(X) X(8, 2, 4) X(4, 2, 4) X(8, 1, 4) X(16, 1, 4) X(4, 1, 8) X(4, 1, 4)

template <typename TIN, bool CLEAN, bool RING>
hipError_t launch_tiled(const Tiling& t, const DedispArgs& a, const int32_t* relb,
                        const float* fit32, size_t lds, hipStream_t s) {
#define MBTP_TILE(G_, Q_, BC_) \
  if (t.G == G_ && t.Q == Q_ && t.BC == BC_) return launch_one<TIN, CLEAN, RING, G_, Q_, BC_>(a, relb, fit32, lds, s);
  MBTP_TILINGS(MBTP_TILE)
#undef MBTP_TILE
  return hipErrorInvalidValue;
}

}  // namespace

#define MBTP_LIST(G_, Q_, BC_) {G_, Q_, BC_},
static const Tiling kTilings[] = {MBTP_TILINGS(MBTP_LIST)};
#undef MBTP_LIST

int n_tilings() { return (int)(sizeof(kTilings) / sizeof(kTilings[0])); }
Tiling tiling_at(int i) { return kTilings[i]; }

hipError_t launch_relb(const int32_t* delays, int32_t C, int32_t ndms, int32_t BD, int32_t RS,
                       int32_t ldr, int32_t* relb, hipStream_t s) {
  const int64_t n = (int64_t)ldr * ndms;
  hipLaunchKernelGGL(relb_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, delays, C,
                     ndms, BD, RS, ldr, relb);
  return hipGetLastError();
}

hipError_t launch_dedisp(int dtype, bool clean, bool ring, const Tiling& t, const DedispArgs& a,
                         const int32_t* relb, const float* fit32, size_t lds, hipStream_t s) {
#define MBTP_D(TIN_)                                                                         \
  if (clean) {                                                                                \
    if (ring) return launch_tiled<TIN_, true, true>(t, a, relb, fit32, lds, s);                \
    return launch_tiled<TIN_, true, false>(t, a, relb, fit32, lds, s);                         \
  } else {                                                                                    \
    if (ring) return launch_tiled<TIN_, false, true>(t, a, relb, fit32, lds, s);               \
    return launch_tiled<TIN_, false, false>(t, a, relb, fit32, lds, s);                        \
  }
  switch (dtype) {
    case 0: { MBTP_D(uint8_t) }
    case 1: { MBTP_D(__half) }
    default: { MBTP_D(float) }
  }
#undef MBTP_D
}

hipError_t launch_ring_update(int dtype, bool clean, const void* x, int64_t ld, int64_t L, int32_t C,
                              const CleanView& cv, const float* fit32, float* ring, int64_t R,
                              int64_t seen, hipStream_t s) {
  const int64_t n = L < R ? L : R;
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)C);
#define MBTP_R(TIN_)                                                                              \
  if (clean) hipLaunchKernelGGL((ring_update_kernel<TIN_, true>), grid, dim3(256), 0, s,          \
                                static_cast<const TIN_*>(x), ld, L, C, cv, fit32, ring, R, seen); \
  else hipLaunchKernelGGL((ring_update_kernel<TIN_, false>), grid, dim3(256), 0, s,               \
                          static_cast<const TIN_*>(x), ld, L, C, cv, fit32, ring, R, seen);
  switch (dtype) {
    case 0: { MBTP_R(uint8_t) break; }
    case 1: { MBTP_R(__half) break; }
    default: { MBTP_R(float) break; }
  }
#undef MBTP_R
  return hipGetLastError();
}

}  // namespace mbtp
