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
  uint32_t meta;                     // kind; chunk sample index t << 1 for chunk quads
};

// Chunk index of chunk sample t (W is a power of two).
__device__ inline uint32_t chunk_of(const CleanView& cv, int64_t t) {
  return (uint32_t)t >> cv.wshift;
}

template <typename TIN, bool CLEAN>
__device__ inline float clean_one(const DedispArgs& A, const TIN* xrow, int64_t c, float fit,
                                  int64_t t) {
  const float v = Quad<TIN>::one(xrow + t);
  if (!CLEAN) return v;
  const bool f = (A.clean.cflags[c * A.clean.J + chunk_of(A.clean, t)] & 2) || A.clean.gflags[t];
  return f ? 0.0f : v - fit;
}

// Row of one staged channel: where its window starts and, for cleaning, the
// 64 chunk flags around the window and whether any spectrum in it is flagged.
struct RowMeta {
  int64_t a;        // virtual index of the window's first sample (aligned)
  uint32_t m_lo, m_hi;  // chunk flags j0..j0+63 (bit per chunk)
  int32_t j0;
  int32_t g_lo, g_hi;   // prefix counts of flagged spectra bracketing the window
};

// Issues the loads of the quad at virtual index tau (a multiple of 4).
template <typename TIN, bool CLEAN, bool RING>
__device__ inline void issue(Staged<TIN>& s, const DedispArgs& A, const TIN* xrow,
                             const float* ringrow, int64_t c, float fit, int64_t tau, int64_t V,
                             int64_t p0) {
  const int64_t v = RING ? A.ring_valid : 0;
  if (tau >= v && tau + 3 < V) {
    const int64_t t = tau - v;
    if constexpr (std::is_same<TIN, float>::value) s.v = Quad<TIN>::load(xrow + t);
    else s.raw = Quad<TIN>::load(xrow + t);
    s.meta = kChunk | ((uint32_t)t << 1);
  } else if (RING && tau < v) {
    int64_t p = p0 + tau;
    if (p >= A.R) p -= A.R;
    s.v = *reinterpret_cast<const float4*>(ringrow + p);
    s.meta = kReady;
  } else {
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t ti = tau + i;
      e[i] = (ti < V) ? clean_one<TIN, CLEAN>(A, xrow, c, fit, ti - v) : 0.0f;
    }
    s.v = make_float4(e[0], e[1], e[2], e[3]);
    s.meta = kReady;
  }
}

// Widens and cleans a landed quad.  Chunk flags come from the row's 64-bit
// mask; spectrum flags are read per quad only when the window holds any.
template <typename TIN, bool CLEAN>
__device__ inline float4 finish(const Staged<TIN>& s, const DedispArgs& A, const RowMeta& rm,
                                bool any_g, float fit) {
  if ((s.meta & 1) == kReady) return s.v;
  float4 f;
  if constexpr (std::is_same<TIN, float>::value) f = s.v;
  else f = Quad<TIN>::widen(s.raw);
  if (CLEAN) {
    const uint32_t t = s.meta >> 1;
    const int jr = (int)chunk_of(A.clean, t) - rm.j0;          // 0..63
    const uint32_t word = jr < 32 ? rm.m_lo : rm.m_hi;
    const bool cf = (word >> (jr & 31)) & 1u;
    uint32_t g = 0;
    if (any_g) g = *reinterpret_cast<const uint32_t*>(A.clean.gflags + t);
    f.x = (cf || (g & 0xffu)) ? 0.0f : f.x - fit;
    f.y = (cf || (g & 0xff00u)) ? 0.0f : f.y - fit;
    f.z = (cf || (g & 0xff0000u)) ? 0.0f : f.z - fit;
    f.w = (cf || (g & 0xff000000u)) ? 0.0f : f.w - fit;
  }
  return f;
}

// One (DM block, time tile) of one launch item; all threads of the
// workgroup call it.  lds: the dynamic LDS of the workgroup.
template <typename TIN, bool CLEAN, bool RING, int NW, int G, int Q, int BC>
__device__ __forceinline__ void dedisp_tile(const DedispArgs& A, const int32_t* __restrict__ relb,
                                            const float* __restrict__ fit32, float* lds,
                                            int dblock, int ttile) {
  constexpr int NT = 64 * NW, BD = NW * G, BT = 256 * Q;
  // staging: NW >= BC: WPR waves share a row, each loads all of it and writes
  // CPW of its 4 copies; NW < BC: each wave stages RPW whole rows
  constexpr int WPR = NW >= BC ? NW / BC : 1;
  constexpr int RPW = NW >= BC ? 1 : BC / NW;
  constexpr int CPW = 4 / WPR;
  constexpr int KM = kStageQuads / RPW;
  static_assert(G % 4 == 0 && WPR * CPW == 4 && (NW >= BC ? NW % BC == 0 : BC % NW == 0) &&
                RPW * KM == kStageQuads && BD * BC <= NT, "tiling");
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;

  const int C = A.C;
  const int d0 = dblock * BD;
  const int dlast = min(d0 + BD, A.ndms) - 1;
  const int64_t t0 = (int64_t)ttile * BT;            // virtual index of this tile's first output
  const int RS = A.rs;
  const int RS4 = RS >> 2;
  const int64_t vring = RING ? A.ring_valid : 0;
  const int64_t V = vring + A.L;
  // ring position of virtual sample 0: from the beam's device-side sample
  // count when given (so a captured launch stays right on replay)
  int64_t p0 = A.ring_p0;
  if (RING && A.seen_dev != nullptr && A.R > 0) {
    const int64_t sn = *A.seen_dev;
    p0 = (sn - vring) % A.R;
  }
  const int32_t* __restrict__ dl = A.delays + (int64_t)d0 * C;   // DM d0's delays
  int* lds_off = reinterpret_cast<int*>(lds + BC * 4 * RS);      // [BC][BD]

  auto row_of = [&](int rr) { return NW >= BC ? wave / WPR : wave + NW * rr; };

  Staged<TIN> st[RPW][KM];
  RowMeta rm[RPW];
  int basen[RPW];        // s[d0][c] of the row in the block after next (vector load, lands early)
  int offreg = 0;

  // Cleaning metadata of row c (vector loads: they count on vmcnt only, so
  // nothing scalar is pending while LDS reads are in flight).
  auto load_meta = [&](RowMeta& m, int c, int64_t a) {
    m.a = a;
    if (CLEAN) {
      int64_t tlo = a - vring, thi = a - vring + RS + 4;
      tlo = tlo < 0 ? 0 : (tlo > A.L ? A.L : tlo);
      thi = thi < 0 ? 0 : (thi > A.L ? A.L : thi);
      if (thi <= tlo) { m.j0 = 0; m.m_lo = m.m_hi = 0; m.g_lo = m.g_hi = 0; return; }
      const int jlo = (int)chunk_of(A.clean, tlo);
      const int w0 = jlo >> 5;
      m.j0 = w0 * 32;
      const int vz = lane * A.zero;     // 0, but lane-dependent: vector loads
      const uint32_t* cb = A.clean.cbits + (int64_t)c * A.clean.JW + vz;
      m.m_lo = cb[w0];
      m.m_hi = (w0 + 1 < A.clean.JW) ? cb[w0 + 1] : 0u;
      m.g_lo = A.clean.gspan[(tlo >> 8) + vz];
      m.g_hi = A.clean.gspan[((thi - 1) >> 8) + 1 + vz];
    }
  };

  auto issue_block = [&](int cb0) {
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int c = cb0 + row_of(rr);
      if (c < C) {
        const int base = __builtin_amdgcn_readfirstlane(basen[rr]);
        const int64_t a = t0 + (base & ~3);
        const TIN* xrow = static_cast<const TIN*>(A.x) + (int64_t)c * A.ld;
        const float* ringrow = RING ? A.ring + (int64_t)c * A.R : nullptr;
        const float fit = CLEAN ? fit32[c + lane * A.zero] : 0.0f;
        load_meta(rm[rr], c, a);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const int m = lane + 64 * k;
          if (m < RS4) issue<TIN, CLEAN, RING>(st[rr][k], A, xrow, ringrow, c, fit, a + 4 * m, V, p0);
          else { st[rr][k].v = make_float4(0.f, 0.f, 0.f, 0.f); st[rr][k].meta = kReady; }
        }
      }
      const int cn = cb0 + BC + row_of(rr);
      if (cn < C) basen[rr] = dl[cn + lane * A.zero];
    }
    if (tid < BD * BC) {
      const int dd = tid % BD, cb = tid / BD;
      const int d = min(d0 + dd, dlast);
      offreg = (cb0 + cb < C) ? relb[(int64_t)d * A.relb_ld + cb0 + cb] : 0;
    }
  };

  // Cleans the block's quads and writes the shifted copies.  The quad after a
  // lane's quad is the next lane's (a DPP wave shift); lane 63 takes lane 0's
  // quad of the next k.  The last quad of a row has no successor in
  // registers, but no DM window reads the copy positions it would feed.
  auto write_block = [&](int cb0) {
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int cb = row_of(rr);
      const int c = cb0 + cb;
      if (c < C) {
        const float fit = CLEAN ? fit32[c] : 0.0f;
        const bool any_g = CLEAN && (__builtin_amdgcn_readfirstlane(rm[rr].g_hi - rm[rr].g_lo) != 0);
        float* row = lds + cb * 4 * RS;
        float4 lo[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) lo[k] = finish<TIN, CLEAN>(st[rr][k], A, rm[rr], any_g, fit);
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
            // copy r holds the window shifted by r samples; with WPR waves per
            // row, wave (wave % WPR) writes copies [CPW*(wave % WPR), +CPW)
            const int wr = NW >= BC ? wave % WPR : 0;
            float* p = row + 4 * m;
            if (CPW == 4 || wr == 0) *reinterpret_cast<float4*>(p) = l;
            if (CPW == 4 || (CPW == 2 && wr == 0) || (CPW == 1 && wr == 1))
              *reinterpret_cast<float4*>(p + RS) = make_float4(l.y, l.z, l.w, hi.x);
            if (CPW == 4 || (CPW == 2 && wr == 1) || (CPW == 1 && wr == 2))
              *reinterpret_cast<float4*>(p + 2 * RS) = make_float4(l.z, l.w, hi.x, hi.y);
            if (CPW == 4 || (CPW == 2 && wr == 1) || (CPW == 1 && wr == 3))
              *reinterpret_cast<float4*>(p + 3 * RS) = make_float4(l.w, hi.x, hi.y, hi.z);
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

#pragma unroll
  for (int rr = 0; rr < RPW; ++rr) {
    const int c = row_of(rr);
    basen[rr] = c < C ? dl[c] : 0;
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

template <typename TIN, bool CLEAN, bool RING, int NW, int G, int Q, int BC>
__global__ __launch_bounds__(64 * NW) void dedisp_kernel(DedispArgs A, const int32_t* __restrict__ relb,
                                                         const float* __restrict__ fit32) {
  extern __shared__ float4 lds4[];
  // Workgroup id -> tile.  Consecutive workgroups go to different XCDs; give
  // each XCD a contiguous range of tiles, DM block fastest, so the blocks
  // that share a time tile run on the same L2 at about the same time.
  const int ntile = A.n_dblocks * A.n_ttiles;
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int q8 = ntile >> 3, rem = ntile & 7;
  const int tile = xcd * q8 + min(xcd, rem) + slot;
  dedisp_tile<TIN, CLEAN, RING, NW, G, Q, BC>(A, relb, fit32, reinterpret_cast<float*>(lds4),
                                              tile % A.n_dblocks, tile / A.n_dblocks);
}

// Persistent launch over the tiles of several items (beams, chunks, plans of
// one tiling).  Workgroups take tiles from an atomic counter in item order,
// heaviest items first, until the counter passes the total; every
// workgroup reaches that exit.
template <typename TIN, bool CLEAN, int NW, int G, int Q, int BC>
__global__ __launch_bounds__(64 * NW) void dedisp_batch_kernel(BatchArgs B) {
  extern __shared__ float4 lds4[];
  __shared__ int tile_sh;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) tile_sh = atomicAdd(B.counter, 1);
    __syncthreads();
    const int t = tile_sh;
    if (t >= B.total) break;
    int i = 0;
    while (i + 1 < B.nitems && t >= B.item[i + 1].tile0) ++i;
    const BatchItem& it = B.item[i];
    const int local = t - it.tile0;
    dedisp_tile<TIN, CLEAN, true, NW, G, Q, BC>(it.a, it.relb, it.fit32, reinterpret_cast<float*>(lds4),
                                                local % it.a.n_dblocks, local / it.a.n_dblocks);
  }
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

// Advances a beam's device-side sample count after a chunk.
__global__ void beam_advance_kernel(int64_t* seen, int64_t L) { *seen += L; }

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
                                                          const int64_t* __restrict__ seen_dev) {
  const int c = blockIdx.y;
  const int64_t seen = *seen_dev;
  const int64_t n = min(L, R);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || c >= C) return;
  const int64_t t = L - n + i;
  float v = Quad<TIN>::one(x + (int64_t)c * ld + t);
  if (CLEAN) {
    const bool flagged = (cv.cflags[(int64_t)c * cv.J + ((uint32_t)t >> cv.wshift)] & 2) || cv.gflags[t];
    v = flagged ? 0.0f : v - fit32[c];
  }
  ring[(int64_t)c * R + (seen + t) % R] = v;
}

template <typename TIN, bool CLEAN, bool RING, int NW, int G, int Q, int BC>
hipError_t launch_one(const DedispArgs& a, const int32_t* relb, const float* fit32, size_t lds,
                      hipStream_t s) {
  const unsigned grid = (unsigned)a.n_dblocks * (unsigned)a.n_ttiles;
  auto kern = dedisp_kernel<TIN, CLEAN, RING, NW, G, Q, BC>;
  // raise the kernel's LDS limit once, on its first (normally eager) launch,
  // so that no attribute call happens while a stream is being captured
  static int lds_set = 0;
  if (lds > 64 * 1024 && lds_set < (int)lds) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_set = 160 * 1024;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), lds, s, a, relb, fit32);
  return hipGetLastError();
}

// Compiled tilings: (waves per workgroup, DMs per wave, float4 groups per
// lane, channels per LDS stage).
#define MBTP_TILINGS(X) X(4, 4, 2, 4) X(8, 4, 2, 8) X(8, 4, 1, 4) X(4, 8, 1, 4) X(8, 4, 2, 4) X(8, 8, 1, 4)

template <typename TIN, bool CLEAN, bool RING>
hipError_t launch_tiled(const Tiling& t, const DedispArgs& a, const int32_t* relb,
                        const float* fit32, size_t lds, hipStream_t s) {
#define MBTP_TILE(NW_, G_, Q_, BC_) \
  if (t.NW == NW_ && t.G == G_ && t.Q == Q_ && t.BC == BC_) \
    return launch_one<TIN, CLEAN, RING, NW_, G_, Q_, BC_>(a, relb, fit32, lds, s);
  MBTP_TILINGS(MBTP_TILE)
#undef MBTP_TILE
  return hipErrorInvalidValue;
}

}  // namespace

#define MBTP_LIST(NW_, G_, Q_, BC_) {NW_, G_, Q_, BC_},
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
                              int64_t* seen_dev, hipStream_t s) {
  const int64_t n = L < R ? L : R;
  if (n > 0) {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)C);
#define MBTP_R(TIN_)                                                                                 \
    if (clean) hipLaunchKernelGGL((ring_update_kernel<TIN_, true>), grid, dim3(256), 0, s,           \
                                  static_cast<const TIN_*>(x), ld, L, C, cv, fit32, ring, R, seen_dev); \
    else hipLaunchKernelGGL((ring_update_kernel<TIN_, false>), grid, dim3(256), 0, s,                \
                            static_cast<const TIN_*>(x), ld, L, C, cv, fit32, ring, R, seen_dev);
    switch (dtype) {
      case 0: { MBTP_R(uint8_t) break; }
      case 1: { MBTP_R(__half) break; }
      default: { MBTP_R(float) break; }
    }
#undef MBTP_R
  }
  hipLaunchKernelGGL(beam_advance_kernel, dim3(1), dim3(1), 0, s, seen_dev, L);
  return hipGetLastError();
}

namespace {
template <typename TIN, bool CLEAN, int NW, int G, int Q, int BC>
hipError_t launch_batch_one(BatchArgs& b, size_t lds, hipStream_t s) {
  auto kern = dedisp_batch_kernel<TIN, CLEAN, NW, G, Q, BC>;
  hipError_t e;
  // attribute and occupancy queries once per instantiation and LDS size (on
  // the first, normally eager, launch), none while a stream is captured
  static int lds_set = 0;
  static size_t occ_lds = 0;
  static int occ = 0, cus = 0;
  if (lds > 64 * 1024 && lds_set == 0) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_set = 1;
  }
  if (occ_lds != lds || cus == 0) {
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern),
                                                          64 * NW, lds)) != hipSuccess) return e;
    occ_lds = lds;
  }
  const int per_cu = occ < 1 ? 1 : occ;
  const int grid = b.total < cus * per_cu ? b.total : cus * per_cu;
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, b.counter);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), lds, s, b);
  return hipGetLastError();
}

template <typename TIN, bool CLEAN>
hipError_t launch_batch_tiled(const Tiling& t, BatchArgs& b, size_t lds, hipStream_t s) {
#define MBTP_TILE(NW_, G_, Q_, BC_) \
  if (t.NW == NW_ && t.G == G_ && t.Q == Q_ && t.BC == BC_) \
    return launch_batch_one<TIN, CLEAN, NW_, G_, Q_, BC_>(b, lds, s);
  MBTP_TILINGS(MBTP_TILE)
#undef MBTP_TILE
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_dedisp_batch(int dtype, bool clean, const Tiling& t, BatchArgs& b, size_t lds,
                               hipStream_t s) {
  switch (dtype) {
    case 0: return clean ? launch_batch_tiled<uint8_t, true>(t, b, lds, s) : launch_batch_tiled<uint8_t, false>(t, b, lds, s);
    case 1: return clean ? launch_batch_tiled<__half, true>(t, b, lds, s) : launch_batch_tiled<__half, false>(t, b, lds, s);
    default: return clean ? launch_batch_tiled<float, true>(t, b, lds, s) : launch_batch_tiled<float, false>(t, b, lds, s);
  }
}

}  // namespace mbtp
