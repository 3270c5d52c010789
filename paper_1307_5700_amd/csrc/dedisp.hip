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
#include "tile_map.h"

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

// One aligned quad of virtual samples in flight.  Every quad is one vector
// load from an address that is always in bounds, with no branch around it:
// divergent load paths that write the same registers make the compiler wait
// for every outstanding load at their join, which would serialise the
// prefetch of the next channel block with the accumulation of this one.
// Which samples of the quad are valid, whether it comes from the ring, and
// the cleaning are all applied with selects when the quad is written to LDS.
// The quad's chunk index is not kept: it follows from the row's (uniform)
// window start and the lane's quad number when the quad is written.
template <typename TIN, bool RING> struct Staged {
  typename Quad<TIN>::Raw raw;       // chunk values (f32: chunk or ring values)
  float4 rv;                         // ring values (u8 / f16 with a ring only)
  uint32_t g;                        // spectrum flags of the 4 samples (cleaning)
};
constexpr int32_t kNoQuad = 0x3fffffff;

// Chunk index of chunk sample t (W is a power of two).
__device__ inline uint32_t chunk_of(const CleanView& cv, int64_t t) {
  return (uint32_t)t >> cv.wshift;
}

// Row of one staged channel: where its window starts and, for cleaning, the
// 64 chunk flags around the window.
struct RowMeta {
  int64_t a;        // virtual index of the window's first sample (aligned)
  uint32_t m_lo, m_hi;  // chunk flags j0..j0+63 (bit per chunk)
  int32_t j0;
};

// Issues the load of the quad whose first sample has chunk index t (a
// multiple of 4; t < 0: the quad lies in the ring, which precedes the chunk
// in virtual time); `live` is false for lanes past the end of their range.
// Rows are ld >= L apart with ld a multiple of 4, so the aligned quad
// holding any chunk sample lies inside its row.  Indices are 32-bit and
// relative to the row bases, which are uniform.  pv = ring position of
// chunk sample 0.
template <typename TIN, bool CLEAN, bool RING>
__device__ inline void issue(Staged<TIN, RING>& s, const DedispArgs& A, const TIN* xrow,
                             const float* ringrow, int32_t t, bool live, int32_t pv) {
  const int32_t L = (int32_t)A.L;
  const bool in_chunk = live && (uint32_t)t < (uint32_t)L;
  const uint32_t off = in_chunk ? (uint32_t)t : 0u;
  // the 4 spectrum flags of the quad (the flag array is padded to 256 bytes)
  if (CLEAN) s.g = *reinterpret_cast<const uint32_t*>(A.clean.gflags + off);
  if constexpr (RING) {
    const bool in_ring = live && t < 0;
    int32_t p = pv + t;
    if (p < 0) p += (int32_t)A.R;
    const uint32_t poff = in_ring ? (uint32_t)p : 0u;
    if constexpr (std::is_same<TIN, float>::value) {
      const float* pr = in_ring ? ringrow + poff : xrow + off;
      s.raw = *reinterpret_cast<const float4*>(pr);
    } else {
      s.raw = Quad<TIN>::load(xrow + off);
      if (A.ring_valid > 0)        // uniform: the ring exists
        s.rv = *reinterpret_cast<const float4*>(ringrow + poff);
      else
        s.rv = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  } else {
    s.raw = Quad<TIN>::load(xrow + off);
  }
}

// Widens and cleans a landed quad: samples past the chunk end are 0; ring
// samples were cleaned when they entered the ring.  Chunk flags come from
// the row's 64-bit mask, spectrum flags from the word loaded with the quad.
// tq: chunk index of the quad's first sample (as issued); live: the lane's
// quad is in its range.
template <typename TIN, bool CLEAN, bool RING>
__device__ inline float4 finish(const Staged<TIN, RING>& s, const DedispArgs& A, const RowMeta& rm,
                                float fit, int32_t tq, bool live) {
  float4 f;
  if constexpr (std::is_same<TIN, float>::value) f = s.raw;
  else f = Quad<TIN>::widen(s.raw);
  const int32_t L = (int32_t)A.L;                            // <= 2^30: 32-bit compares
  // < 0: ring quad; >= L (kNoQuad): nothing to stage
  const int32_t t = !live ? kNoQuad : (RING && tq < 0 ? -1 : (tq < L ? tq : kNoQuad));
  const bool ring = RING && t < 0;
  const int32_t tc = (uint32_t)t < (uint32_t)L ? t : 0;      // in-range stand-in for the chunk index
  const int32_t left = L - t;                                // valid samples from t on
  bool z0 = left <= 0, z1 = left <= 1, z2 = left <= 2, z3 = left <= 3;
  float sub = 0.0f;
  if (CLEAN) {
    const int jr = (int)chunk_of(A.clean, tc) - rm.j0;       // 0..63 inside the window
    const uint32_t word = jr < 32 ? rm.m_lo : rm.m_hi;
    const bool cf = ((word >> (jr & 31)) & 1u) != 0;
    const uint32_t g = s.g;
    z0 = z0 || cf || (g & 0xffu); z1 = z1 || cf || (g & 0xff00u);
    z2 = z2 || cf || (g & 0xff0000u); z3 = z3 || cf || (g & 0xff000000u);
    sub = fit;
  }
  float4 r;
  r.x = z0 ? 0.0f : f.x - sub;
  r.y = z1 ? 0.0f : f.y - sub;
  r.z = z2 ? 0.0f : f.z - sub;
  r.w = z3 ? 0.0f : f.w - sub;
  if constexpr (RING) {
    if constexpr (std::is_same<TIN, float>::value) {
      if (ring) r = f;
    } else {
      if (ring) r = s.rv;
    }
  }
  return r;
}

// The G per-DM LDS offsets of one wave for one staged channel (int2 or
// int4 broadcast reads).
template <int G>
__device__ inline void load_offsets(const int* src, int (&o)[G]) {
  if constexpr (G == 2) {
    const int2 o2 = *reinterpret_cast<const int2*>(src);
    o[0] = o2.x; o[1] = o2.y;
  } else {
#pragma unroll
    for (int g = 0; g < G; g += 4) {
      const int4 o4 = *reinterpret_cast<const int4*>(src + g);
      o[g] = o4.x; o[g + 1] = o4.y; o[g + 2] = o4.z; o[g + 3] = o4.w;
    }
  }
}

// x of the next lane; lane 63 (no next lane) returns old.
__device__ inline float next_quad(float x, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), 0x130, 0xf, 0xf, false));
}

// x of the next lane, lane 63 taking lane 0's (wave rotate).
__device__ inline float wave_rotate(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x134, 0xf, 0xf, false));
}

// acc[q] += the 4 window samples that start r (uniform, 0..3) samples into
// the lane's aligned quad v[q]; the samples past the quad are the next
// lane's, taken by a DPP wave shift fused into the add (lane 63 adds 0).
// One block of code per residue, chosen by scalar branches: the adds of the
// cases must not be merged behind the branch (the compiler would then keep
// every routed value live in registers), and the accumulators stay in the
// same registers whatever the residue.  The s_nop covers the wait a DPP
// source needs after a VALU write.
template <int Q>
__device__ inline void add_shifted(float4 (&acc)[Q], const float4 (&v)[Q], int r);

template <>
__device__ inline void add_shifted<1>(float4 (&acc)[1], const float4 (&v)[1], int r) {
  asm(
      "s_cmp_eq_u32 %8, 0\n\t"
      "s_cbranch_scc1 .Lr0_%=\n\t"
      "s_cmp_eq_u32 %8, 1\n\t"
      "s_cbranch_scc1 .Lr1_%=\n\t"
      "s_cmp_eq_u32 %8, 2\n\t"
      "s_cbranch_scc1 .Lr2_%=\n\t"
      "v_add_f32 %0, %7, %0\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %1, %4, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %2, %5, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %3, %6, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "s_branch .Lend_%=\n\t"
      ".Lr0_%=:\n\t"
      "v_add_f32 %0, %4, %0\n\t"
      "v_add_f32 %1, %5, %1\n\t"
      "v_add_f32 %2, %6, %2\n\t"
      "v_add_f32 %3, %7, %3\n\t"
      "s_branch .Lend_%=\n\t"
      ".Lr1_%=:\n\t"
      "v_add_f32 %0, %5, %0\n\t"
      "v_add_f32 %1, %6, %1\n\t"
      "v_add_f32 %2, %7, %2\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %3, %4, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "s_branch .Lend_%=\n\t"
      ".Lr2_%=:\n\t"
      "v_add_f32 %0, %6, %0\n\t"
      "v_add_f32 %1, %7, %1\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %2, %4, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %3, %5, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      ".Lend_%=:"
      : "+v"(acc[0].x), "+v"(acc[0].y), "+v"(acc[0].z), "+v"(acc[0].w)
      : "v"(v[0].x), "v"(v[0].y), "v"(v[0].z), "v"(v[0].w), "s"(r)
      : "scc");
}

template <>
__device__ inline void add_shifted<2>(float4 (&acc)[2], const float4 (&v)[2], int r) {
  asm(
      "s_cmp_eq_u32 %16, 0\n\t"
      "s_cbranch_scc1 .Lr0_%=\n\t"
      "s_cmp_eq_u32 %16, 1\n\t"
      "s_cbranch_scc1 .Lr1_%=\n\t"
      "s_cmp_eq_u32 %16, 2\n\t"
      "s_cbranch_scc1 .Lr2_%=\n\t"
      "v_add_f32 %0, %11, %0\n\t"
      "v_add_f32 %4, %15, %4\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %1, %8, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %2, %9, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %3, %10, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %5, %12, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %6, %13, %6 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %7, %14, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "s_branch .Lend_%=\n\t"
      ".Lr0_%=:\n\t"
      "v_add_f32 %0, %8, %0\n\t"
      "v_add_f32 %1, %9, %1\n\t"
      "v_add_f32 %2, %10, %2\n\t"
      "v_add_f32 %3, %11, %3\n\t"
      "v_add_f32 %4, %12, %4\n\t"
      "v_add_f32 %5, %13, %5\n\t"
      "v_add_f32 %6, %14, %6\n\t"
      "v_add_f32 %7, %15, %7\n\t"
      "s_branch .Lend_%=\n\t"
      ".Lr1_%=:\n\t"
      "v_add_f32 %0, %9, %0\n\t"
      "v_add_f32 %1, %10, %1\n\t"
      "v_add_f32 %2, %11, %2\n\t"
      "v_add_f32 %4, %13, %4\n\t"
      "v_add_f32 %5, %14, %5\n\t"
      "v_add_f32 %6, %15, %6\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %3, %8, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %7, %12, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "s_branch .Lend_%=\n\t"
      ".Lr2_%=:\n\t"
      "v_add_f32 %0, %10, %0\n\t"
      "v_add_f32 %1, %11, %1\n\t"
      "v_add_f32 %4, %14, %4\n\t"
      "v_add_f32 %5, %15, %5\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %2, %8, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %3, %9, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %6, %12, %6 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %7, %13, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      ".Lend_%=:"
      : "+v"(acc[0].x), "+v"(acc[0].y), "+v"(acc[0].z), "+v"(acc[0].w), "+v"(acc[1].x), "+v"(acc[1].y), "+v"(acc[1].z), "+v"(acc[1].w)
      : "v"(v[0].x), "v"(v[0].y), "v"(v[0].z), "v"(v[0].w), "v"(v[1].x), "v"(v[1].y), "v"(v[1].z), "v"(v[1].w), "s"(r)
      : "scc");
}

// One (DM block, time tile) of one launch item; all threads of the
// workgroup call it.  lds: the dynamic LDS of the workgroup.
template <typename TIN, bool CLEAN, bool RING, int NW, int G, int Q, int BC, int P, bool SKIP_IDLE>
__device__ __forceinline__ void dedisp_tile(const DedispArgs& A, const int32_t* relb,
                                            const float* fit32, float* lds,
                                            int dblock, int ttile) {
  // P bit 3: warp specialisation.  The first kProducers waves only stage
  // (producers), the others only accumulate (consumers), each role in its
  // own loop with one barrier per channel block, so staging of block k+1
  // overlaps the accumulation of block k and neither role holds the other's
  // registers.  Otherwise every wave stages and accumulates.
  constexpr bool WS = (P & 8) != 0;
  constexpr int kProducers = (P & 64) ? 8 : 4;      // P bit 6: eight producers
  constexpr int NSW = WS ? kProducers : NW;        // staging waves
  constexpr int NAW = WS ? NW - kProducers : NW;   // accumulating waves
  // P bit 5: one staged copy per channel.  A window then starts anywhere in
  // an aligned quad; each lane reads the aligned quads and takes the samples
  // past its quad from the next lane (DPP), so lane 63 of a 256-sample stripe
  // yields no outputs and stripes advance by 252 samples.
  constexpr bool SC = (P & 32) != 0;
  constexpr int NCP = SC ? 1 : 4;                  // staged copies per channel
  constexpr int STRIPE = SC ? 252 : 256;           // outputs per stripe
  constexpr int BD = NAW * G, BT = STRIPE * Q;
  // staging: NSW >= BC: WPR waves share a row and split its quads (each a
  // contiguous range, one quad of overlap); NSW < BC: each wave stages RPW
  // whole rows.  KM quads per lane and row cover rows of up to
  // 64*kStageQuads quads.
  constexpr int WPR = NSW >= BC ? NSW / BC : 1;
  constexpr int RPW = NSW >= BC ? 1 : BC / NSW;
  constexpr int QWMAX = (64 * kStageQuads - 1 + WPR - 1) / WPR + 1;
  constexpr int KM = RPW > 1 ? kStageQuads / RPW : (QWMAX + 63) / 64;
  static_assert((G == 2 || G % 4 == 0) && (NSW >= BC ? NSW % BC == 0 : BC % NSW == 0) &&
                (RPW == 1 || RPW * KM == kStageQuads) && BD * BC <= 64 * NSW &&
                kAccGroup % BC == 0 && (!WS || ((P & 2) != 0 && NAW > 0)) && (!SC || (P & 5) == 0),
                "tiling");
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int aw = WS ? wave - kProducers : wave;     // accumulating wave index

  const int C = A.C;
  const int d0 = dblock * BD;
  const int dlast = min(d0 + BD, A.ndms) - 1;
  const int64_t t0 = (int64_t)ttile * BT;            // virtual index of this tile's first output
  const int RS = A.rs;
  const int RS4 = RS >> 2;
  const int64_t vring = RING ? A.ring_valid : 0;
  // ring position of virtual sample 0: from the beam's device-side sample
  // count when given (so a captured launch stays right on replay)
  int64_t p0 = A.ring_p0;
  if (RING && A.seen_dev != nullptr && A.R > 0) {
    const int64_t sn = *A.seen_dev;
    p0 = (sn - vring) % A.R;
  }
  // ring position of chunk sample 0
  const int32_t pv = (RING && A.R > 0) ? (int32_t)((p0 + vring) % A.R) : 0;
  const int32_t* __restrict__ dl = A.delays + (int64_t)d0 * C;   // DM d0's delays
  const int32_t* __restrict__ dz = A.delays + (int64_t)dlast * C; // the block's last DM's
  // LDS: one stage (or two, double-buffered) of BC rows x NCP copies x RS
  // samples followed by the stage's [BC][BD] window offsets
  constexpr bool DB = (P & 2) != 0;
  const int stage_floats = BC * NCP * RS + BC * BD;
  auto stage_rows = [&](int b) { return lds + b * stage_floats; };
  auto stage_off = [&](int b) { return reinterpret_cast<int*>(lds + b * stage_floats + BC * NCP * RS); };

  auto row_of = [&](int rr) { return NSW >= BC ? wave / WPR : wave + NSW * rr; };
  // this wave's quads of its row(s): [m0, mend); the last quad of a range
  // that is not the row's last is written by the next wave as well, which
  // alone has its successor quad and so writes its shifted copies
  const int wr = NSW >= BC ? wave % WPR : 0;
  const int qw = WPR > 1 ? (RS4 - 1 + WPR - 1) / WPR + 1 : RS4;
  const int m0 = wr * (qw - 1);
  const int mend = min(m0 + qw, RS4);

  // Staging state of a block in flight.  Producers with a prefetch depth of
  // two (P bit 4) keep two sets, used alternately; otherwise set 0.
  constexpr bool PF2 = WS && (P & 16) != 0;
  constexpr int NSET = PF2 ? 2 : 1;
  Staged<TIN, RING> st[NSET][RPW][KM];
  RowMeta rm[NSET][RPW];
  int basen[RPW];        // s[d0][c] of the row in the block after next (vector load, lands early)
  int lastn[RPW];        // s[dlast][c] of the same row
  // With four copies and one wave per row, a row stages only the span its
  // block's windows read: they start at most (s[dlast][c] - s[d0][c] + 3)
  // & ~3 positions in (delays grow with DM), so the consumers read the first
  // that / 4 + BT / 4 quads of each copy, and the copies of the last of them
  // take samples from the quad after it.  A row near the top of the band,
  // where the delay spread is small, stages that much less.  The persistent
  // kernel, whose tile loop leaves few registers, trims only cleaned 8-bit
  // rows (its other variants would spill).
  constexpr bool TRIM = NCP == 4 && WPR == 1 && (SKIP_IDLE || (sizeof(TIN) == 1 && CLEAN));
  int rowq[NSET][RPW];   // quads staged of the row (live: m < rowq)
  float fitn[NSET][RPW]; // bandpass value of the row being staged (loaded with its quads)
  int32_t rowt[NSET][RPW]; // chunk index of the staged row's window start (uniform)
  int offreg[NSET] = {};

  // Cleaning metadata of row c (vector loads: they count on vmcnt only, so
  // nothing scalar is pending while LDS reads are in flight).  Both words
  // are loaded from clamped indices on every path, with nothing computed
  // from them until the block is written: a block's loads never depend on
  // the data and nothing waits for them early, so they stay in flight
  // behind the next block's.  A window with no chunk sample never reads the
  // words; one whose chunks all fit the first word never reads the second.
  auto load_meta = [&](RowMeta& m, int c, int64_t a) {
    m.a = a;
    if (CLEAN) {
      int64_t tlo = a - vring;
      tlo = tlo < 0 ? 0 : (tlo > A.L ? A.L : tlo);
      const int w0 = (int)chunk_of(A.clean, tlo) >> 5;
      const int jw = (int)A.clean.JW;
      m.j0 = w0 * 32;
      const int vz = lane * A.zero;     // 0, but lane-dependent: vector loads
      const uint32_t* cb = A.clean.cbits + (int64_t)c * A.clean.JW + vz;
      m.m_lo = cb[max(min(w0, jw - 1), 0)];
      m.m_hi = cb[max(min(w0 + 1, jw - 1), 0)];
    }
  };

  // Issues the loads of channel block cb0.  Rows past the last channel (and
  // blocks past the end) load a valid row instead, whose values are never
  // written: every call issues the same loads, see load_meta.
  auto issue_block = [&](int cb0, auto set_c) {
    constexpr int S = decltype(set_c)::value;
    // the window bases of the rows of the block after this one go first:
    // the next call waits for them, and so for nothing issued after them
    int base_now[RPW], last_now[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      base_now[rr] = __builtin_amdgcn_readfirstlane(basen[rr]);
      if (TRIM) last_now[rr] = __builtin_amdgcn_readfirstlane(lastn[rr]);
      basen[rr] = dl[min(cb0 + BC + row_of(rr), C - 1) + lane * A.zero];
      if (TRIM) lastn[rr] = dz[min(cb0 + BC + row_of(rr), C - 1) + lane * A.zero];
    }
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int c = min(cb0 + row_of(rr), C - 1);
      {
        const int base = base_now[rr];
        const int64_t a = t0 + (base & ~3);
        const int32_t aw = (int32_t)(a - vring);     // chunk index of the window start
        rowt[S][rr] = aw;
        const int rq = TRIM ? min(mend, ((last_now[rr] - (base & ~3)) >> 2) + BT / 4 + 1) : mend;
        rowq[S][rr] = rq;
        const TIN* xrow = static_cast<const TIN*>(A.x) + (int64_t)c * A.ld;
        const float* ringrow = RING ? A.ring + (int64_t)c * A.R : nullptr;
        load_meta(rm[S][rr], c, a);
        if (CLEAN) fitn[S][rr] = fit32[c + lane * A.zero];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const int m = m0 + lane + 64 * k;
          issue<TIN, CLEAN, RING>(st[S][rr][k], A, xrow, ringrow, aw + 4 * m, m < rq, pv);
        }
      }
    }
    {
      // unconditional load from a clamped index (no load inside a divergent
      // branch, see Staged); rows past C get offset 0 when it is written
      const int dd = tid % BD, cb = min(tid / BD, BC - 1);
      const int d = min(d0 + dd, dlast);
      const int cc = min(cb0 + cb, C - 1);
      offreg[S] = relb[(int64_t)d * A.relb_ld + cc];
    }
  };

  // Cleans the block's quads and writes the shifted copies.  The quad after a
  // lane's quad is the next lane's (a DPP wave shift); lane 63 takes lane 0's
  // quad of the next k.  The last quad of a row has no successor in
  // registers, but no DM window reads the copy positions it would feed.
  auto write_block = [&](int cb0, int buf, auto set_c) {
    constexpr int S = decltype(set_c)::value;
    float* const rows = stage_rows(buf);
    int* const lds_off = stage_off(buf);
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int cb = row_of(rr);
      const int c = cb0 + cb;
      float* row = rows + cb * NCP * RS;
      if (c >= C) {
        // rows past the last channel read as zeros (offset 0 of copy 0), so
        // the accumulation of a block needs no per-channel bound test
        for (int m = m0 + lane; m < mend; m += 64)
          *reinterpret_cast<float4*>(row + 4 * m) = make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        const float fit = CLEAN ? fitn[S][rr] : 0.0f;
        // Fast path (uniform per row): the wave's quads all lie inside the
        // chunk and none of their chunks or spectra is flagged, so a quad
        // needs only widening and the bandpass subtraction.
        const int rq = rowq[S][rr];
        const int32_t t_lo = rowt[S][rr] + 4 * m0, t_hi = rowt[S][rr] + 4 * rq;
        bool fast = t_lo >= 0 && t_hi <= (int32_t)A.L;
        if (CLEAN) {
          uint32_t gor = 0;
#pragma unroll
          for (int k = 0; k < KM; ++k) gor |= st[S][rr][k].g;
          const uint32_t mbits = __builtin_amdgcn_readfirstlane(rm[S][rr].m_lo | rm[S][rr].m_hi);
          fast = fast && mbits == 0 && __builtin_amdgcn_ballot_w64(gor != 0) == 0;
        }
        // Writes the cleaned quads lo[] (each branch below has its own copy,
        // so the two cleaning paths need no register moves to merge).
        auto write_quads = [&](const float4 (&lo)[KM]) {
          if constexpr (SC) {
#pragma unroll
            for (int k = 0; k < KM; ++k) {
              const int m = m0 + lane + 64 * k;
              if (m < rq) *reinterpret_cast<float4*>(row + 4 * m) = lo[k];
            }
          } else {
#pragma unroll
            for (int k = 0; k < KM; ++k) {
              // hi = the first three samples of the next quad: the next
              // lane's (wave shift); lane 63 keeps the `old` operand, lane
              // 0's quad of k+1 brought over by a wave rotate.  The last
              // k's lane 63 feeds no window.
              float4 hi;
              const float4 nx = lo[(k + 1) % KM];
              const bool more = k + 1 < KM;
              hi.x = next_quad(lo[k].x, more ? wave_rotate(nx.x) : 0.0f);
              hi.y = next_quad(lo[k].y, more ? wave_rotate(nx.y) : 0.0f);
              hi.z = next_quad(lo[k].z, more ? wave_rotate(nx.z) : 0.0f);
              const int m = m0 + lane + 64 * k;
              if (m < rq) {
                const float4 l = lo[k];
                // copy r holds the window shifted by r samples
                float* p = row + 4 * m;
                *reinterpret_cast<float4*>(p) = l;
                if (WPR == 1 || m + 1 < mend || wr == WPR - 1) {
                  *reinterpret_cast<float4*>(p + RS) = make_float4(l.y, l.z, l.w, hi.x);
                  *reinterpret_cast<float4*>(p + 2 * RS) = make_float4(l.z, l.w, hi.x, hi.y);
                  *reinterpret_cast<float4*>(p + 3 * RS) = make_float4(l.w, hi.x, hi.y, hi.z);
                }
              }
            }
          }
        };
        if (fast) {
          float4 lo[KM];
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            float4 f;
            if constexpr (std::is_same<TIN, float>::value) f = st[S][rr][k].raw;
            else f = Quad<TIN>::widen(st[S][rr][k].raw);
            if (CLEAN) { f.x -= fit; f.y -= fit; f.z -= fit; f.w -= fit; }
            lo[k] = f;
          }
          write_quads(lo);
        } else {
          float4 lo[KM];
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            const int m = m0 + lane + 64 * k;
            lo[k] = finish<TIN, CLEAN, RING>(st[S][rr][k], A, rm[S][rr], fit, rowt[S][rr] + 4 * m, m < rq);
          }
          write_quads(lo);
        }
      }
    }
    if (tid < BD * BC) lds_off[tid] = (cb0 + tid / BD < C) ? offreg[S] : 0;   // [cb][dd], dd fastest
  };

  // Running sums; zeroed where the accumulating loop starts, so that they
  // are not live while producers stage.
  float4 acc[G][Q], tot[G][Q];
  auto zero_sums = [&] {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        acc[g][q] = make_float4(0.f, 0.f, 0.f, 0.f);
        tot[g][q] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
  };

#pragma unroll
  for (int rr = 0; rr < RPW; ++rr) {
    const int c = row_of(rr);
    basen[rr] = dl[min(c, C - 1)];
    if (TRIM) lastn[rr] = dz[min(c, C - 1)];
  }
  // Single buffer: per block, issue the loads of block k+1, accumulate block
  // k, barrier, write block k+1, barrier.  Double buffer: block k+1 is
  // written into the other stage while block k is accumulated (its loads
  // were issued one block earlier), then the loads of block k+2 are issued;
  // one barrier per block.
  // Accumulates channel block cb0 from LDS stage cur into acc (and tot at
  // every kAccGroup-th channel).
  auto accumulate = [&](int cb0, int cur) {
    // ---- accumulate channel block cb0 ----
    // Straight-line over the BC channels (rows past C are zeros).
    const char* base = reinterpret_cast<const char*>(stage_rows(cur)) + 16 * lane;
    const int* lds_off = stage_off(cur);
    if constexpr (SC) {
      // The block's window offsets first (uniform: SGPRs), then per DM the
      // adds of channel cb, routed by the window's residue r (element e of a
      // lane's outputs is element e + r of its aligned quad, or e + r - 4 of
      // the next lane's), each followed at once by the reads of channel
      // cb+1 into the same registers.  The values and the order of the adds
      // are those of the four-copy layout.
      int offs[BC][G];
#pragma unroll
      for (int cb = 0; cb < BC; ++cb) {
        int o[G];
        load_offsets(lds_off + cb * BD + aw * G, o);
#pragma unroll
        for (int g = 0; g < G; ++g) offs[cb][g] = __builtin_amdgcn_readfirstlane(o[g]);
      }
      float4 v[G][Q];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int q = 0; q < Q; ++q) v[g][q] = reinterpret_cast<const float4*>(base + (offs[0][g] & ~3))[63 * q];
#pragma unroll
      for (int cb = 0; cb < BC; ++cb) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          add_shifted<Q>(acc[g], v[g], offs[cb][g] & 3);
          if (cb + 1 < BC) {
            const char* rowb = base + (cb + 1) * 4 * RS + (offs[cb + 1][g] & ~3);
#pragma unroll
            for (int q = 0; q < Q; ++q) v[g][q] = reinterpret_cast<const float4*>(rowb)[63 * q];
          }
        }
      }
    } else if constexpr ((P & 4) != 0) {
      // pipelined: two register sets; the reads of channel cb+1 and the
      // offsets of channel cb+2 are issued before the adds of channel cb
      // (for tilings whose occupancy does not drop with the extra registers)
      int off[2][G];
      float4 v[2][G][Q];
      load_offsets(lds_off + 0 * BD + aw * G, off[0]);
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int q = 0; q < Q; ++q) v[0][g][q] = reinterpret_cast<const float4*>(base + off[0][g])[64 * q];
      if (BC > 1) load_offsets(lds_off + 1 * BD + aw * G, off[1]);
#pragma unroll
      for (int cb = 0; cb < BC; ++cb) {
        if (cb + 1 < BC) {
          const char* rowb = base + (cb + 1) * 16 * RS;
#pragma unroll
          for (int g = 0; g < G; ++g)
#pragma unroll
            for (int q = 0; q < Q; ++q)
              v[(cb + 1) & 1][g][q] = reinterpret_cast<const float4*>(rowb + off[(cb + 1) & 1][g])[64 * q];
        }
        if (cb + 2 < BC) load_offsets(lds_off + (cb + 2) * BD + aw * G, off[cb & 1]);
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const float4 w = v[cb & 1][g][q];
            acc[g][q].x += w.x; acc[g][q].y += w.y;
            acc[g][q].z += w.z; acc[g][q].w += w.w;
          }
      }
    } else if constexpr ((P & 1) == 0) {
      // serial: per channel the offsets, then its G*Q reads, then the adds;
      // latency is hidden by the other resident waves
#pragma unroll
      for (int cb = 0; cb < BC; ++cb) {
        const char* rowb = base + cb * 16 * RS;
        int off[G];
        load_offsets(lds_off + cb * BD + aw * G, off);
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
      }
    } else {
      // rolling: the block's offsets first (uniform: SGPRs), then per DM
      // group g the adds of channel cb are followed at once by the reads of
      // channel cb+1 into the same registers, so up to G*Q reads stay in
      // flight with no second set of registers
      int off[BC][G];
#pragma unroll
      for (int cb = 0; cb < BC; ++cb) {
        load_offsets(lds_off + cb * BD + aw * G, off[cb]);
#pragma unroll
        for (int g = 0; g < G; ++g) off[cb][g] = __builtin_amdgcn_readfirstlane(off[cb][g]);
      }
      float4 v[G][Q];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int q = 0; q < Q; ++q) v[g][q] = reinterpret_cast<const float4*>(base + off[0][g])[64 * q];
#pragma unroll
      for (int cb = 0; cb < BC; ++cb) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            acc[g][q].x += v[g][q].x; acc[g][q].y += v[g][q].y;
            acc[g][q].z += v[g][q].z; acc[g][q].w += v[g][q].w;
          }
          if (cb + 1 < BC) {
            const char* rowb = base + (cb + 1) * 16 * RS;
#pragma unroll
            for (int q = 0; q < Q; ++q) v[g][q] = reinterpret_cast<const float4*>(rowb + off[cb + 1][g])[64 * q];
          }
        }
      }
    }
    // partial sums close at every kAccGroup-th channel (BC divides kAccGroup)
    if (((cb0 + BC) & (kAccGroup - 1)) == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          tot[g][q].x += acc[g][q].x; tot[g][q].y += acc[g][q].y;
          tot[g][q].z += acc[g][q].z; tot[g][q].w += acc[g][q].w;
          acc[g][q] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
  };

  // Single buffer: per block, issue the loads of block k+1, accumulate block
  // k, barrier, write block k+1, barrier.  Double buffer: block k+1 is
  // written into the other stage while block k is accumulated (its loads
  // were issued one block earlier), then the loads of block k+2 are issued;
  // one barrier per block.  Warp-specialised: the same double-buffered
  // schedule, producers and consumers in separate loops that execute the same
  // number of barriers (one before the loop, one per block).
  const bool stager = !WS || wave < kProducers;
  using Set0 = std::integral_constant<int, 0>;
  using SetL = std::integral_constant<int, NSET - 1>;   // second set (or set 0)
  auto prologue = [&] {
    issue_block(0, Set0{});
    write_block(0, 0, Set0{});
    if (DB) issue_block(BC, Set0{});
    if (PF2) issue_block(2 * BC, SetL{});
    // keeps the compiler from sinking any of these loads below the first
    // barrier into the loop's preheader: the wait counts at the loop head
    // hold for every path into it, so one late load there would make the
    // first step of every iteration wait for all loads
    asm volatile("" ::: "memory");
  };
  if constexpr (WS) {
    // Each role's whole life sits in its own branch (the first barrier
    // included), so no staging register is live in the accumulating loop
    // and the kernel needs the larger role's registers, not their sum.
    if (stager) {
      prologue();
      __syncthreads();
      if constexpr (PF2) {
        // block k+1 sits in set k & 1: two steps per iteration keep the set
        // indices compile-time; each step writes block k+1 and issues block
        // k+3 into the set it freed.  The issues are unconditional (past the
        // end they load rows that are never written) so that the wait for a
        // set only ever covers that set; the second step's barrier exists
        // only when its block does, so producers and consumers execute the
        // same number of barriers.
        int cur = 0;
        for (int cb0 = 0; cb0 < C; cb0 += 2 * BC) {
          if (cb0 + BC < C) write_block(cb0 + BC, cur ^ 1, Set0{});
          issue_block(cb0 + 3 * BC, Set0{});
          __syncthreads();
          cur ^= 1;
          if (cb0 + 2 * BC < C) write_block(cb0 + 2 * BC, cur ^ 1, SetL{});
          issue_block(cb0 + 4 * BC, SetL{});
          if (cb0 + BC < C) {
            __syncthreads();
            cur ^= 1;
          }
        }
      } else {
        int cur = 0;
        for (int cb0 = 0; cb0 < C; cb0 += BC) {
          const int next = cb0 + BC;
          if (next < C) write_block(next, cur ^ 1, Set0{});
          issue_block(next + BC, Set0{});          // past the end: unused
          __syncthreads();
          cur ^= 1;
        }
      }
      return;                   // producers hold no outputs
    }
    __syncthreads();
    zero_sums();
    // a consumer whose DMs all lie past the grid's last (the last DM block
    // of a grid that BD does not divide) reads nothing, but keeps the
    // barriers (not in the persistent kernel, whose registers are full)
    const bool idle = SKIP_IDLE && d0 + aw * G > dlast;
    int cur = 0;
    for (int cb0 = 0; cb0 < C; cb0 += BC) {
      if (!idle) accumulate(cb0, cur);
      __syncthreads();
      cur ^= 1;
    }
  } else {
    prologue();
    __syncthreads();
    zero_sums();
    int cur = 0;
    for (int cb0 = 0; cb0 < C; cb0 += BC) {
      const int next = cb0 + BC;
      if constexpr (DB) {
        if (next < C) write_block(next, cur ^ 1, Set0{});
        issue_block(next + BC, Set0{});            // past the end: unused
      } else {
        if (next < C) issue_block(next, Set0{});
      }
      accumulate(cb0, cur);
      __syncthreads();
      if constexpr (DB) {
        cur ^= 1;
      } else if (next < C) {
        write_block(next, 0, Set0{});
        __syncthreads();
      }
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
    const int d = d0 + aw * G + g;
    if (d > dlast) continue;
    float* orow = A.out + (int64_t)d * A.ld_out;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (SC && lane == 63) continue;          // feeds lane 62 only
      const int64_t j = t0 + 4 * lane + STRIPE * q - A.phase;
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

template <typename TIN, bool CLEAN, bool RING, int NW, int G, int Q, int BC, int P>
__global__ __launch_bounds__(64 * NW) void dedisp_kernel(DedispArgs A, const int32_t* relb,
                                                         const float* fit32) {
  extern __shared__ float4 lds4[];
  constexpr int BD = ((P & 8) ? NW - ((P & 64) ? 8 : 4) : NW) * G;
  const TileIdx ti = xcd_tile(blockIdx.x, A.n_dblocks, A.n_ttiles, A.ndms % BD != 0);
  const int dblock = ti.dblock, ttile = ti.ttile;
  if (dblock >= A.n_dblocks || ttile >= A.n_ttiles) return;   // uniform: never taken
  dedisp_tile<TIN, CLEAN, RING, NW, G, Q, BC, P, true>(A, relb, fit32, reinterpret_cast<float*>(lds4),
                                                       dblock, ttile);
}

// Persistent launch over the tiles of several items (beams, chunks, plans of
// one tiling).  Workgroups take tiles from an atomic counter in item order,
// heaviest items first, until the counter passes the total; every
// workgroup reaches that exit.
template <typename TIN, bool CLEAN, int NW, int G, int Q, int BC, int P>
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
    dedisp_tile<TIN, CLEAN, true, NW, G, Q, BC, P, false>(it.a, it.relb, it.fit32, reinterpret_cast<float*>(lds4),
                                                local % it.a.n_dblocks, local / it.a.n_dblocks);
  }
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

// Device-side stream position of a beam: st[0] samples seen since the stream
// (re)started, st[1] absolute index of the last chunk's first output, st[2]
// absolute index of the stream's first sample.  After a chunk of L samples
// the first output is max(0, seen - s_max) samples into the stream.
__global__ void beam_advance_kernel(int64_t* st, int64_t L, int64_t smax) {
  const int64_t seen = st[0];
  st[1] = st[2] + (seen > smax ? seen - smax : 0);
  st[0] = seen + L;
}

// Restarts a beam's stream at absolute sample `base` (the ring is forgotten).
__global__ void beam_seek_kernel(int64_t* st, int64_t base) {
  st[0] = 0;
  st[1] = base;
  st[2] = base;
}

// Per-(DM, channel) window offset inside the channel's staged region, with
// p = s[d][c] - (s[d0][c] & ~3).  Four copies: the window starts at position
// p & ~3 of copy p & 3 (LDS byte offset).  One copy: byte offset of the
// aligned quad holding the window start, p & ~3, with the residue p & 3 in
// the two low bits (the offset itself is a multiple of 16).
__global__ void relb_kernel(const int32_t* __restrict__ delays, int32_t C, int32_t ndms, int32_t BD,
                            int32_t RS, int32_t copies, int32_t ldr, int32_t* __restrict__ relb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ldr * ndms) return;
  const int32_t d = (int32_t)(i / ldr), c = (int32_t)(i % ldr);
  if (c >= C) { relb[i] = 0; return; }
  const int32_t d0 = (d / BD) * BD;
  const int32_t p = delays[(int64_t)d * C + c] - (delays[(int64_t)d0 * C + c] & ~3);
  relb[i] = copies == 1 ? (p & ~3) * 4 + (p & 3) : ((p & 3) * RS + (p & ~3)) * 4;
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

// The P a kernel variant is compiled with: the second prefetch set (P bit 4)
// does not fit the registers of the persistent kernel (its tile loop holds
// more state), which keeps one block in flight.  The LDS layout and every
// addition are the same.
template <typename TIN>
constexpr int kernel_p(int P, bool ring, bool batch) {
  (void)ring;
  return ((P & 16) != 0 && batch) ? (P & ~16) : P;
}

template <typename TIN, bool CLEAN, bool RING, int NW, int G, int Q, int BC, int P>
hipError_t launch_one(const DedispArgs& a, const int32_t* relb, const float* fit32, size_t lds,
                      hipStream_t s) {
  // the LDS limit was raised when the plan was created (dedisp_prepare), so
  // a launch makes no attribute call and is safe inside stream capture
  const unsigned grid = (unsigned)a.n_dblocks * (unsigned)a.n_ttiles;
  constexpr int KP = kernel_p<TIN>(P, RING, false);
  hipLaunchKernelGGL((dedisp_kernel<TIN, CLEAN, RING, NW, G, Q, BC, KP>), dim3(grid), dim3(64 * NW), lds, s,
                     a, relb, fit32);
  return hipGetLastError();
}

// Compiled tilings: (waves per workgroup, DMs per wave, float4 groups per
// lane, channels per LDS stage, P: bit 0 rolling accumulation, bit 1 double-
// buffered LDS stages, bit 2 pipelined accumulation with two register sets,
// bit 3 warp specialisation: four producer waves, the rest consumers, bit 4
// with bit 3: producers keep two blocks of loads in flight, bit 5: one
// staged copy per channel).
// The plan takes the first that fits its LDS and staging limits: 48 DMs per
// block first (twelve consumer waves share every staged block), then 32.
// The four with 16 and 8 DMs per block serve DM grids whose delay spread per
// DM step is large (coarse steps, slow sampling).  The last stages one copy
// per channel (a quarter of the LDS writes, residues routed in the adds):
// the autotuner may pick it where staging dominates.
#define MBTP_TILINGS(X) X(16, 4, 2, 4, 26) X(12, 4, 2, 4, 26) X(8, 4, 2, 8, 0) X(16, 2, 2, 4, 3) \
  X(8, 4, 2, 4, 2) X(12, 2, 2, 4, 26) X(4, 4, 2, 4, 0) X(4, 2, 2, 4, 0) X(4, 2, 1, 4, 0)         \
  X(12, 4, 2, 4, 42)

template <typename TIN, bool CLEAN, bool RING>
hipError_t launch_tiled(const Tiling& t, const DedispArgs& a, const int32_t* relb,
                        const float* fit32, size_t lds, hipStream_t s) {
#define MBTP_TILE(NW_, G_, Q_, BC_, P_) \
  if (t.NW == NW_ && t.G == G_ && t.Q == Q_ && t.BC == BC_ && t.P == P_) \
    return launch_one<TIN, CLEAN, RING, NW_, G_, Q_, BC_, P_>(a, relb, fit32, lds, s);
  MBTP_TILINGS(MBTP_TILE)
#undef MBTP_TILE
  return hipErrorInvalidValue;
}

}  // namespace

#define MBTP_LIST(NW_, G_, Q_, BC_, P_) {NW_, G_, Q_, BC_, P_},
static const Tiling kTilings[] = {MBTP_TILINGS(MBTP_LIST)};
#undef MBTP_LIST

int n_tilings() { return (int)(sizeof(kTilings) / sizeof(kTilings[0])); }
Tiling tiling_at(int i) { return kTilings[i]; }

hipError_t launch_relb(const int32_t* delays, int32_t C, int32_t ndms, int32_t BD, int32_t RS,
                       int32_t copies, int32_t ldr, int32_t* relb, hipStream_t s) {
  const int64_t n = (int64_t)ldr * ndms;
  hipLaunchKernelGGL(relb_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, delays, C,
                     ndms, BD, RS, copies, ldr, relb);
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
                              int64_t* seen_dev, int64_t smax, hipStream_t s) {
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
  hipLaunchKernelGGL(beam_advance_kernel, dim3(1), dim3(1), 0, s, seen_dev, L, smax);
  return hipGetLastError();
}

hipError_t launch_beam_seek(int64_t* seen_dev, int64_t base, hipStream_t s) {
  hipLaunchKernelGGL(beam_seek_kernel, dim3(1), dim3(1), 0, s, seen_dev, base);
  return hipGetLastError();
}

namespace {
template <typename TIN, bool CLEAN, int NW, int G, int Q, int BC, int P>
hipError_t launch_batch_one(BatchArgs& b, size_t lds, int grid_cap, hipStream_t s) {
  const int grid = b.total < grid_cap ? b.total : grid_cap;
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, b.counter);
  hipLaunchKernelGGL((dedisp_batch_kernel<TIN, CLEAN, NW, G, Q, BC, kernel_p<TIN>(P, true, true)>), dim3(grid),
                     dim3(64 * NW), lds, s, b);
  return hipGetLastError();
}

// Raises the LDS limit of every kernel variant of one (storage type, tiling)
// and returns the persistent kernel's resident workgroups per CU at `lds`
// bytes, without and with cleaning.
template <typename TIN, int NW, int G, int Q, int BC, int P>
hipError_t prepare_one(size_t lds, int occ[2]) {
  constexpr int P0 = kernel_p<TIN>(P, false, false), PR = kernel_p<TIN>(P, true, false),
                PB = kernel_p<TIN>(P, true, true);
  const void* ks[6] = {
      reinterpret_cast<const void*>(dedisp_kernel<TIN, false, false, NW, G, Q, BC, P0>),
      reinterpret_cast<const void*>(dedisp_kernel<TIN, false, true, NW, G, Q, BC, PR>),
      reinterpret_cast<const void*>(dedisp_kernel<TIN, true, false, NW, G, Q, BC, P0>),
      reinterpret_cast<const void*>(dedisp_kernel<TIN, true, true, NW, G, Q, BC, PR>),
      reinterpret_cast<const void*>(dedisp_batch_kernel<TIN, false, NW, G, Q, BC, PB>),
      reinterpret_cast<const void*>(dedisp_batch_kernel<TIN, true, NW, G, Q, BC, PB>)};
  hipError_t e;
  for (const void* k : ks) {
    // dynamic + static LDS of a workgroup must fit the CU's 160 KiB
    hipFuncAttributes fa;
    if ((e = hipFuncGetAttributes(&fa, k)) != hipSuccess) return e;
    const int dyn_max = 160 * 1024 - (int)fa.sharedSizeBytes;
    if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_max)) != hipSuccess)
      return e;
  }
  for (int c = 0; c < 2; ++c)
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[c], ks[4 + c], 64 * NW, lds)) != hipSuccess)
      return e;
  return hipSuccess;
}

template <typename TIN>
hipError_t prepare_tiled(const Tiling& t, size_t lds, int occ[2]) {
#define MBTP_TILE(NW_, G_, Q_, BC_, P_) \
  if (t.NW == NW_ && t.G == G_ && t.Q == Q_ && t.BC == BC_ && t.P == P_) \
    return prepare_one<TIN, NW_, G_, Q_, BC_, P_>(lds, occ);
  MBTP_TILINGS(MBTP_TILE)
#undef MBTP_TILE
  return hipErrorInvalidValue;
}

template <typename TIN, bool CLEAN>
hipError_t launch_batch_tiled(const Tiling& t, BatchArgs& b, size_t lds, int grid_cap, hipStream_t s) {
#define MBTP_TILE(NW_, G_, Q_, BC_, P_) \
  if (t.NW == NW_ && t.G == G_ && t.Q == Q_ && t.BC == BC_ && t.P == P_) \
    return launch_batch_one<TIN, CLEAN, NW_, G_, Q_, BC_, P_>(b, lds, grid_cap, s);
  MBTP_TILINGS(MBTP_TILE)
#undef MBTP_TILE
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_dedisp_batch(int dtype, bool clean, const Tiling& t, BatchArgs& b, size_t lds,
                               int grid_cap, hipStream_t s) {
  switch (dtype) {
    case 0: return clean ? launch_batch_tiled<uint8_t, true>(t, b, lds, grid_cap, s) : launch_batch_tiled<uint8_t, false>(t, b, lds, grid_cap, s);
    case 1: return clean ? launch_batch_tiled<__half, true>(t, b, lds, grid_cap, s) : launch_batch_tiled<__half, false>(t, b, lds, grid_cap, s);
    default: return clean ? launch_batch_tiled<float, true>(t, b, lds, grid_cap, s) : launch_batch_tiled<float, false>(t, b, lds, grid_cap, s);
  }
}

hipError_t dedisp_prepare(int dtype, const Tiling& t, size_t lds, int occ[2]) {
  switch (dtype) {
    case 0: return prepare_tiled<uint8_t>(t, lds, occ);
    case 1: return prepare_tiled<__half>(t, lds, occ);
    default: return prepare_tiled<float>(t, lds, occ);
  }
}

}  // namespace mbtp
