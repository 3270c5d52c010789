// Brute-force incoherent dedispersion (Sec. 2.2.2) of 8-bit filterbanks
// without cleaning, summed exactly in integers, for gfx950.
//
//   D[d][t] = sum_c x[c][t + s[d][c]],   x[c][t] in 0..255
//
// The tile is that of the warp-specialised float kernel: a workgroup of 16
// wave64s covers 48 adjacent DMs x 512 consecutive outputs.  Four producer
// waves stage a block of 4 channels into LDS while twelve consumer waves
// (4 DMs each) accumulate the block before it, over two LDS stages with one
// barrier per block.  Producers keep four blocks of loads in flight and
// stage each row only as far as its block's windows read; consumers add a
// block's last channel after the barrier that ends it.
//
// What changes is the width of a term.  Samples are staged as 16-bit
// integers, in eight copies shifted by 0..7 samples, so every (DM, channel)
// window starts 16-byte aligned in one copy.  A lane reads the terms of its
// 8 consecutive outputs with one ds_read_b128 and adds them with four
// v_pk_add_u16 (two 16-bit additions per lane and instruction, at the rate
// of one FP32 add).  Per output that halves both the LDS bytes read and the
// VALU instructions of the float kernel.  16-bit partials hold up to 257
// channels of 8-bit samples; they are widened into 32-bit totals every 256
// channels.
//
// The sum is exact, and so is its conversion to FP32 (C * 255 < 2^24 for
// C <= 65535).  The float kernels' partials and totals of 8-bit data are
// exact integers as well, so both give the same result bit for bit.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>
#include <utility>

#include "internal.h"
#include "tile_map.h"

namespace mbtp {
namespace {

constexpr int kProd = 4;                         // producer waves: one staged row each
constexpr int kCons = kU8BD / kU8G;              // consumer waves
constexpr int kWaves = kProd + kCons;
constexpr int kFold = 256;                       // channels per 16-bit partial
constexpr int kPF = 4;                           // blocks of producer loads in flight
static_assert(kProd == kU8BC && kCons == 12 && kU8BT == 64 * 8, "integer tile");
static_assert(kFold % kU8BC == 0 && kU8BC == 4, "partials close on block boundaries; four channels a block");

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Two u16 lanes of a += b (v_pk_add_u16; a partial never exceeds 16 bits).
__device__ inline uint32_t add_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}

// Samples i and i+1 (0 <= i <= 13) of the 16 bytes w[0..3] as a pair of
// u16 (sample i in the low half).  v_perm_b32 picks bytes of {hi, lo}:
// selector values 0-3 are lo's bytes, 4-7 hi's, 12 gives a zero byte.
// Two encodings of the same pair (ALT: the operands swapped); a pair that
// two copies share is formed once in each, so that every copy's four words
// are computed into their own registers instead of being moved there.
template <int I, bool ALT>
__device__ inline uint32_t pair16(const uint32_t (&w)[4]) {
  constexpr int k = I / 4, b = I % 4;
  constexpr int hk = k + 1 < 4 ? k + 1 : 3;
  if constexpr (!ALT) {
    constexpr uint32_t sel = (uint32_t)b | 0x0c00u | ((uint32_t)(b + 1) << 16) | 0x0c000000u;
    return __builtin_amdgcn_perm(w[hk], w[k], sel);
  } else {
    // w[k] as the high operand: its bytes are selectors 4-7, w[hk]'s 0-3
    constexpr uint32_t b0 = (uint32_t)b + 4, b1 = b + 1 < 4 ? (uint32_t)b + 5 : (uint32_t)(b + 1 - 4);
    constexpr uint32_t sel = b0 | 0x0c00u | (b1 << 16) | 0x0c000000u;
    return __builtin_amdgcn_perm(w[k], w[hk], sel);
  }
}

// f(integral_constant<int, j>) for j = 0 .. N-1, unrolled.
template <typename F, int... J>
__device__ inline void static_for_seq(F& f, std::integer_sequence<int, J...>) {
  (f(std::integral_constant<int, J>{}), ...);
}
template <int N, typename F>
__device__ inline void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// x of the next lane; lane 63 (no next lane) returns old.
__device__ inline uint32_t next_lane(uint32_t x, uint32_t old) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, 0x130, 0xf, 0xf, false);
}

// x of the next lane, lane 63 taking lane 0's (wave rotate).
__device__ inline uint32_t rotate_lane(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x134, 0xf, 0xf, false);
}

typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Copies r = P, P+2, P+4, P+6 (P = 0 or 1) of one staged octet: copy r holds
// samples r .. r+7 of the octet and its successor as four u16 pairs.  Copies
// P and P+4 are the even-aligned windows at 0 and 2 of the pairs P, P+2, ..,
// P+12; copies P+2 and P+6 those of a second run of pairs from P+2, each an
// 8-register tuple, so all four are written from their tuple's registers.
template <int P>
__device__ inline void copies16(const uint32_t (&w)[4], u32x8& a, u32x8& b) {
  a = u32x8{pair16<P, false>(w), pair16<P + 2, false>(w), pair16<P + 4, false>(w), pair16<P + 6, false>(w),
            pair16<P + 8, false>(w), pair16<P + 10, false>(w), pair16<P + 12, false>(w), 0u};
  b = u32x8{pair16<P + 2, true>(w), pair16<P + 4, true>(w), pair16<P + 6, true>(w), pair16<P + 8, true>(w),
            pair16<P + 10, true>(w), pair16<P + 12, true>(w), 0u, 0u};
}

__global__ __launch_bounds__(64 * kWaves) void dedisp_u8_kernel(DedispArgs A, const int32_t* relb) {
  extern __shared__ uint4 lds_u4[];
  char* const lds = reinterpret_cast<char*>(lds_u4);
  const TileIdx ti = xcd_tile(blockIdx.x, A.n_dblocks, A.n_ttiles, A.ndms % kU8BD != 0);
  if (ti.dblock >= A.n_dblocks || ti.ttile >= A.n_ttiles) return;   // uniform: never taken
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int C = A.C;
  const int d0 = ti.dblock * kU8BD;
  const int dlast = min(d0 + kU8BD, A.ndms) - 1;
  const int32_t t0 = ti.ttile * kU8BT;             // chunk index of the tile's first output
  const int32_t L = (int32_t)A.L;                  // <= 2^30
  // LDS stage: kU8BC rows of 8 copies x kU8RS samples (u16), then the
  // block's [kU8BC][kU8BD] window offsets (bytes from the stage start).  The
  // plan's rows use the first A.rs samples of each copy; the fixed stride
  // makes every copy's offset an immediate.
  const int nocts = A.rs >> 3;
  constexpr int row_bytes = 16 * kU8RS;
  constexpr int stage_bytes = kU8BC * row_bytes + kU8BC * kU8BD * 4;

  if (wave < kProd) {
    // ---- producer: stages row `wave` of every block ----
    const int32_t* __restrict__ dl = A.delays + (int64_t)d0 * C;      // DM d0's delays
    const int32_t* __restrict__ dz = A.delays + (int64_t)dlast * C;   // the block's last DM's
    const int vz = lane * A.zero;                  // 0, but lane-dependent: vector loads
    uint2 raw[kPF][kU8KM];                         // kPF blocks of loads in flight
    int offreg[kPF];
    int nwr[kPF];                                  // octets written of each set's row
    // s[d0][c] and s[dlast][c] of each set's next row, loaded kPF blocks
    // before they are used, so that waiting for them waits only for loads
    // already consumed
    int basen[kPF], lastn[kPF];
#pragma unroll
    for (int j = 0; j < kPF; ++j) {
      basen[j] = dl[min(j * kU8BC + wave, C - 1) + vz];
      lastn[j] = dz[min(j * kU8BC + wave, C - 1) + vz];
    }

    // Issues the loads of the block starting at channel cb0 into set S.
    // Every call issues the same loads whatever the block (rows past the
    // last channel and blocks past the end load a valid row that is never
    // written), so the compiler's static wait counts only ever wait for the
    // set about to be written.
    auto issue = [&](int cb0, auto set_c) {
      constexpr int S = decltype(set_c)::value;
      const int base = __builtin_amdgcn_readfirstlane(basen[S]);
      const int last = __builtin_amdgcn_readfirstlane(lastn[S]);
      basen[S] = dl[min(cb0 + kPF * kU8BC + wave, C - 1) + vz];
      lastn[S] = dz[min(cb0 + kPF * kU8BC + wave, C - 1) + vz];
      const int c = min(cb0 + wave, C - 1);
      const int32_t a = t0 + (base & ~7);          // chunk index of the row's first staged sample
      // The block's windows in this row start at most (s[dlast][c] - a) & ~7
      // positions in (delays grow with DM), so its consumers read the first
      // that / 8 + 64 octets of each copy; the copies of the last of them
      // take samples from the octet after it.  A row near the top of the
      // band, where the delay spread is small, stages only that much.
      const int nw = min(((last - (base & ~7)) >> 3) + 64, nocts);
      nwr[S] = nw;
      const uint8_t* xrow = static_cast<const uint8_t*>(A.x) + (int64_t)c * A.ld;
#pragma unroll
      for (int k = 0; k < kU8KM; ++k) {
        const int m = lane + 64 * k;
        const int32_t off = a + 8 * m;
        // the octet holding a chunk sample lies inside its row (ld and the
        // row bases are multiples of 8); octets past the chunk or past the
        // row's span read the row's first one: they feed no output that is
        // stored
        raw[S][k] = *reinterpret_cast<const uint2*>(xrow + (uint32_t)((m <= nw && off < L) ? off : 0));
      }
      const int dd = tid % kU8BD, cb = min(tid / kU8BD, kU8BC - 1);
      const int d = min(d0 + dd, dlast);
      const int cc = min(cb0 + cb, A.relb_ld - 1);
      offreg[S] = relb[(int64_t)d * A.relb_ld + cc];
    };

    // Writes the block starting at cb0 from set S into LDS stage `stage`.
    auto write = [&](int cb0, int stage, auto set_c) {
      constexpr int S = decltype(set_c)::value;
      char* const st = lds + stage * stage_bytes;
      char* const row = st + wave * row_bytes;
      if (cb0 + wave >= C) {
        // rows past the last channel: the offset table points them at the
        // first 512 samples of copy 0, which read as zeros
        *reinterpret_cast<uint4*>(row + 16 * lane) = make_uint4(0u, 0u, 0u, 0u);
      } else {
#pragma unroll
        for (int k = 0; k < kU8KM; ++k) {
          // w[0..1]: this octet; w[2..3]: the next one, the next lane's
          // (lane 63 takes lane 0's of k+1).  The last k's lane 63 and the
          // row's last octet feed no window.
          uint32_t w[4];
          w[0] = raw[S][k].x;
          w[1] = raw[S][k].y;
          const bool more = k + 1 < kU8KM;
          const uint2 nx = raw[S][(k + 1) % kU8KM];
          w[2] = next_lane(w[0], more ? rotate_lane(nx.x) : 0u);
          w[3] = next_lane(w[1], more ? rotate_lane(nx.y) : 0u);
          const int m = lane + 64 * k;
          if (m < nwr[S]) {
            char* p = row + 16 * m;                // position 8m of copy 0 (2 bytes a sample)
            u32x8 e, e2, o, o2;
            copies16<0>(w, e, e2);
            copies16<1>(w, o, o2);
            constexpr int cs = 2 * kU8RS;          // bytes between copies
            *reinterpret_cast<u32x4*>(p) = e.s0123;
            *reinterpret_cast<u32x4*>(p + 1 * cs) = o.s0123;
            *reinterpret_cast<u32x4*>(p + 2 * cs) = e2.s0123;
            *reinterpret_cast<u32x4*>(p + 3 * cs) = o2.s0123;
            *reinterpret_cast<u32x4*>(p + 4 * cs) = e.s2345;
            *reinterpret_cast<u32x4*>(p + 5 * cs) = o.s2345;
            *reinterpret_cast<u32x4*>(p + 6 * cs) = e2.s2345;
            *reinterpret_cast<u32x4*>(p + 7 * cs) = o2.s2345;
          }
        }
      }
      if (tid < kU8BC * kU8BD) reinterpret_cast<int*>(st + kU8BC * row_bytes)[tid] = offreg[S];
    };

    // Block b is staged in LDS stage b & 1 from load set b mod kPF.  Its
    // loads are issued kPF blocks before it is written.
    using S0 = std::integral_constant<int, 0>;
    static_for<kPF>([&](auto j) { issue(decltype(j)::value * kU8BC, j); });
    write(0, 0, S0{});
    issue(kPF * kU8BC, S0{});
    asm volatile("" ::: "memory");   // no load sinks past the first barrier
    __syncthreads();
    // kPF blocks per iteration keep the set indices compile-time.  Each step
    // (the consumers accumulate block b) writes block b+1 and reissues its
    // set for block b+1+kPF.  Every step issues its loads and ends in a
    // barrier, past the last block too, so that every path through the loop
    // has the same loads in flight and the compiler's wait counts stay
    // exact; the consumers add the barriers of the steps past the last block.
    for (int cb0 = 0; cb0 < C; cb0 += kPF * kU8BC) {
      static_for<kPF>([&](auto j) {
        using SN = std::integral_constant<int, (decltype(j)::value + 1) % kPF>;
        const int b = cb0 + decltype(j)::value * kU8BC;
        if (b + kU8BC < C) write(b + kU8BC, (b / kU8BC + 1) & 1, SN{});
        issue(b + (kPF + 1) * kU8BC, SN{});
        __syncthreads();
      });
    }
    return;                                        // producers hold no outputs
  }

  // ---- consumer: DMs d0 + aw*G .. +G-1, outputs t0 + 8*lane .. +7 ----
  const int aw = wave - kProd;
  __syncthreads();
  uint32_t acc[kU8G][4], tot[kU8G][8];
#pragma unroll
  for (int g = 0; g < kU8G; ++g) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) tot[g][j] = 0u;
  }
  auto fold = [&] {
#pragma unroll
    for (int g = 0; g < kU8G; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        tot[g][2 * j] += acc[g][j] & 0xffffu;
        tot[g][2 * j + 1] += acc[g][j] >> 16;
        acc[g][j] = 0u;
      }
  };
  // a consumer whose DMs all lie past the grid's last reads nothing, but
  // keeps the barriers
  const bool idle = d0 + aw * kU8G > dlast;
  // The adds of a block's last channel wait until after the barrier that
  // ends the block (its reads have landed by then: the barrier waits for
  // them), where they overlap the next block's offset reads.
  uint4 vp[kU8G];                                  // last channel of the previous block
  bool pend = false;
  int pcb0 = 0;
  auto add4 = [&](const uint4 (&t)[kU8G]) {
#pragma unroll
    for (int g = 0; g < kU8G; ++g) {
      acc[g][0] = add_u16x2(acc[g][0], t[g].x);
      acc[g][1] = add_u16x2(acc[g][1], t[g].y);
      acc[g][2] = add_u16x2(acc[g][2], t[g].z);
      acc[g][3] = add_u16x2(acc[g][3], t[g].w);
    }
  };
  auto settle = [&] {                              // the deferred adds, then the block's fold
    if (pend) {
      add4(vp);
      if (((pcb0 + kU8BC) & (kFold - 1)) == 0) fold();
      pend = false;
    }
  };
  int cur = 0;
  for (int cb0 = 0; cb0 < C; cb0 += kU8BC) {
    if (!idle) {
      const char* const st = lds + cur * stage_bytes;
      const int* const offs = reinterpret_cast<const int*>(st + kU8BC * row_bytes) + aw * kU8G;
      const char* const lb = st + 16 * lane;
      // the block's offsets, the previous block's deferred adds while they
      // are read, then the reads of channels 0 and 1, and per channel the
      // adds followed at once by the read of the channel two on into the
      // registers they freed; the last channel's adds are deferred
      int o[kU8BC][4];
#pragma unroll
      for (int cb = 0; cb < kU8BC; ++cb) {
        const int4 o4 = *reinterpret_cast<const int4*>(offs + cb * kU8BD);
        o[cb][0] = o4.x; o[cb][1] = o4.y; o[cb][2] = o4.z; o[cb][3] = o4.w;
      }
      settle();
      uint4 v[2][kU8G];
#pragma unroll
      for (int g = 0; g < kU8G; ++g) v[0][g] = *reinterpret_cast<const uint4*>(lb + o[0][g]);
#pragma unroll
      for (int g = 0; g < kU8G; ++g) v[1][g] = *reinterpret_cast<const uint4*>(lb + o[1][g]);
      add4(v[0]);
#pragma unroll
      for (int g = 0; g < kU8G; ++g) v[0][g] = *reinterpret_cast<const uint4*>(lb + o[2][g]);
      add4(v[1]);
#pragma unroll
      for (int g = 0; g < kU8G; ++g) vp[g] = *reinterpret_cast<const uint4*>(lb + o[3][g]);
      add4(v[0]);
      pend = true;
      pcb0 = cb0;
    }
    __syncthreads();
    cur ^= 1;
  }
  settle();
  // the producers' steps past the last block (their loop runs in groups of kPF)
  const int nblk = (C + kU8BC - 1) / kU8BC;
  for (int k = nblk; k % kPF != 0; ++k) __syncthreads();
  fold();
  // ---- store: 8 outputs per lane and DM ----
  // (A.out may start anywhere in a row, after outputs another launch writes:
  // rows are a multiple of 4 floats apart, so whether a lane's 8 outputs
  // are 16-byte aligned is the same for every lane and row)
  const int64_t j = (int64_t)t0 + 8 * lane;
  const bool aligned = (reinterpret_cast<uintptr_t>(A.out) & 15) == 0;
#pragma unroll
  for (int g = 0; g < kU8G; ++g) {
    const int d = d0 + aw * kU8G + g;
    if (d > dlast) continue;
    float* orow = A.out + (int64_t)d * A.ld_out;
    float f[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = (float)tot[g][i];
    if (aligned && j + 7 < A.nout) {
      *reinterpret_cast<float4*>(orow + j) = make_float4(f[0], f[1], f[2], f[3]);
      *reinterpret_cast<float4*>(orow + j + 4) = make_float4(f[4], f[5], f[6], f[7]);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (j + i < A.nout) orow[j + i] = f[i];
    }
  }
}

// Per-(DM, channel) LDS byte offset of the window from the stage start:
// row c mod 4, copy p & 7, position p & ~7 (copies kU8RS samples apart),
// with p = s[d][c] - (s[d0][c] & ~7)
// and d0 the first DM of d's block.  Channels past the last point at the
// start of copy 0 of their row, which the producers fill with zeros.
__global__ void relb_u8_kernel(const int32_t* __restrict__ delays, int32_t C, int32_t ndms,
                               int32_t ldr, int32_t* __restrict__ relb) {
  constexpr int32_t RS = kU8RS;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ldr * ndms) return;
  const int32_t d = (int32_t)(i / ldr), c = (int32_t)(i % ldr);
  const int32_t row = (c % kU8BC) * 8 * RS;
  if (c >= C) { relb[i] = 2 * row; return; }
  const int32_t d0 = (d / kU8BD) * kU8BD;
  const int32_t p = delays[(int64_t)d * C + c] - (delays[(int64_t)d0 * C + c] & ~7);
  relb[i] = 2 * (row + (p & 7) * RS + (p & ~7));
}

}  // namespace

hipError_t launch_relb_u8(const int32_t* delays, int32_t C, int32_t ndms, int32_t ldr, int32_t* relb,
                          hipStream_t s) {
  const int64_t n = (int64_t)ldr * ndms;
  hipLaunchKernelGGL(relb_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, delays, C, ndms, ldr,
                     relb);
  return hipGetLastError();
}

hipError_t dedisp_u8_prepare() {
  const void* k = reinterpret_cast<const void*>(dedisp_u8_kernel);
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, k);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024 - (int)fa.sharedSizeBytes);
}

hipError_t launch_dedisp_u8(const DedispArgs& a, const int32_t* relb, size_t lds, hipStream_t s) {
  const unsigned grid = (unsigned)a.n_dblocks * (unsigned)a.n_ttiles;
  hipLaunchKernelGGL(dedisp_u8_kernel, dim3(grid), dim3(64 * kWaves), lds, s, a, relb);
  return hipGetLastError();
}

}  // namespace mbtp
