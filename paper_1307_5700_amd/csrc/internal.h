// Internal interface between the host runtime (mbtp.cpp) and the HIP kernel
// files.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mbtp {

// Four FP32 lanes as a clang vector: the operand type of 16-byte
// __builtin_nontemporal_store, which streaming writers use for planes that
// are written once and read by the next stage.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Samples of one wave-span of the statistics pass: a wave covers 256
// consecutive samples of one channel, 4 per lane.
constexpr int kSpan = 256;
// Channels summed into one FP32 partial before it is added to the running
// total of a dedispersed sample; a fixed constant so every tiling, batch and
// replay adds in the same order.
constexpr int kAccGroup = 32;

// Header at offset 0 of an RFI state buffer (256 bytes reserved).
struct RfiHeader {
  double sigma;       // per-sample noise std implied by the fit RMSE
  double rmse0;       // RMSE of the first fit
  double rmse;        // RMSE of the final fit
  double sum_fit;     // sum_c f_c
  double thr_spec;    // k_spec * sigma / sqrt(C)
  double k_chan;      // chunk threshold factor (chunk thr = k_chan*sigma/sqrt(L_j))
  unsigned long long n_masked, n_chunk, n_chunk_ext, n_spec;
  int64_t nsamps, nchunks;
  int32_t error;      // 1: every channel masked
  int32_t pad;
};
static_assert(sizeof(RfiHeader) <= 256, "header too large");

// Geometry and byte offsets of an RFI state buffer for C channels, T
// samples and chunk width W (a multiple of kSpan).
struct RfiGeom {
  int64_t C, T, W, J, nspans, CG, ngroups;
  size_t off_hdr, off_fit, off_fit32, off_bsum, off_binterp, off_span, off_chunk, off_spart;
  size_t off_flags, off_lcount, off_list, off_gflags, off_masked, off_cbits, total;
  int64_t JW;                // 32-bit words per channel of the chunk-flag bitmask
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline RfiGeom rfi_geometry(int64_t C, int64_t T, int64_t W) {
  RfiGeom g;
  g.C = C; g.T = T; g.W = W;
  g.J = (T + W - 1) / W;
  g.nspans = (T + kSpan - 1) / kSpan;
  // channels per statistics workgroup: at most 8 groups of partial spectrum
  // sums, chosen from C alone, so the state size never decreases with T (a
  // buffer sized for the longest chunk holds any shorter one)
  int64_t cg = 64;
  while (cg < 512 && (C + cg - 1) / cg > 8) cg *= 2;
  g.CG = cg;
  g.ngroups = (C + cg - 1) / cg;
  size_t o = 0;
  g.off_hdr = o;      o = align256(o + 256);
  g.off_fit = o;      o = align256(o + sizeof(double) * C);
  g.off_fit32 = o;    o = align256(o + sizeof(float) * C);
  g.off_bsum = o;     o = align256(o + sizeof(double) * C);
  g.off_binterp = o;  o = align256(o + sizeof(double) * C);
  g.off_span = o;     o = align256(o + sizeof(double) * C * g.nspans);
  g.off_chunk = o;    o = align256(o + sizeof(double) * C * g.J);
  g.off_spart = o;    o = align256(o + sizeof(double) * g.ngroups * T);
  g.off_flags = o;    o = align256(o + size_t(C) * g.J);
  g.off_lcount = o;   o = align256(o + sizeof(int32_t) * g.J);
  g.off_list = o;     o = align256(o + sizeof(int32_t) * C * g.J);
  g.off_gflags = o;   o = align256(o + size_t(T));
  g.off_masked = o;   o = align256(o + size_t(C));
  g.JW = (g.J + 31) / 32;
  g.off_cbits = o;    o = align256(o + sizeof(uint32_t) * C * g.JW);
  g.total = o;
  return g;
}

struct RfiParamsDev {
  int32_t p, W, mask_passes;
  double k_mask, k_chan, k_spec;
};

hipError_t launch_rfi(int dtype, const void* x, int64_t ld, const RfiGeom& g,
                      const RfiParamsDev& prm, char* state, hipStream_t s);

// Cleaning applied while staging samples for dedispersion.
struct CleanView {
  const double* fit;         // f[C]
  const uint8_t* cflags;     // [C][J], bit1 = flagged after extension
  const uint8_t* gflags;     // [T]
  const uint32_t* cbits;     // [C][JW]: bit j%32 of word j/32 = chunk j flagged (extended)
  int64_t JW;
  int64_t J;
  uint32_t W;
  int32_t wshift;            // log2(W)
};

// Everything one dedispersion launch needs.
//
// Virtual input of a launch: the v ring samples that precede the chunk, then
// the chunk's L samples (v, the ring length R and the ring position of virtual
// sample 0 are multiples of 4, so every aligned quad of virtual samples lies
// wholly in the ring or wholly in the chunk).  Output j of this launch is the
// dedispersed sample at virtual index phase + j.
struct DedispArgs {
  const void* x;             // chunk [C][ld], L samples
  int64_t ld, L;
  const float* ring;         // [C][R] circular (stream mode) or null
  int64_t R;                 // ring length, multiple of 4
  int64_t ring_valid;        // v: ring samples preceding the chunk
  int64_t ring_p0;           // ring position of virtual sample 0
  int64_t phase;             // virtual index of output 0
  const int32_t* delays;     // [ndms][C]
  int32_t C, ndms;
  int64_t nout;
  float* out;                // [ndms][ld_out]
  int64_t ld_out;
  CleanView clean;
  int32_t n_dblocks, n_ttiles;
  int32_t rs;                // LDS copy length in floats (multiple of 4)
  int32_t relb_ld;           // row stride of the relb table (channels rounded up to 4)
  int32_t zero;              // always 0: gives per-row loads a lane-dependent address so
                             // they are vector loads, never scalar ones
  const int64_t* seen_dev;   // beam's device-side sample count (ring position), or null
};

// One item of a batched persistent launch, and the launch's arguments
// (passed by value: at most kMaxBatch items, within the 4 KiB argument limit).
constexpr int kMaxBatch = 16;
struct BatchItem {
  DedispArgs a;
  const int32_t* relb;
  const float* fit32;
  int32_t tile0;             // first global tile of this item
  int32_t pad;
};
struct BatchArgs {
  BatchItem item[kMaxBatch];
  int32_t nitems, total;
  int* counter;              // zeroed by the launcher before the launch
};
static_assert(sizeof(BatchArgs) <= 4096, "batch arguments exceed the kernel argument limit");

struct Tiling {
  int NW, G, Q, BC;   // waves per workgroup, DMs per wave, float4 groups per lane,
                      // channels per LDS stage
  int P;              // bit 0: rolling accumulation loop; bit 1: two LDS stages
  // P bit 3: warp specialisation with 4 producer waves (8 with P bit 6)
  int staging_waves() const { return (P & 8) ? ((P & 64) ? 8 : 4) : NW; }
  int BD() const { return ((P & 8) ? NW - staging_waves() : NW) * G; }   // consumers x G
  // P bit 5: one staged copy per channel (lane 63 of every 256-sample stripe
  // only feeds its neighbour, so a stripe yields 252 outputs); else four
  // shifted copies
  int copies() const { return (P & 32) ? 1 : 4; }
  int BT() const { return ((P & 32) ? 252 : 256) * Q; }
  int threads() const { return 64 * NW; }
};

// Quads of staged samples each thread prefetches per channel block.
constexpr int kStageQuads = 4;

// Variants compiled into the library.
int n_tilings();
Tiling tiling_at(int i);

// Per-(DM, channel) LDS byte offsets of a tiling (see dedisp.hip).
hipError_t launch_relb(const int32_t* delays, int32_t C, int32_t ndms, int32_t BD, int32_t RS,
                       int32_t copies, int32_t ldr, int32_t* relb, hipStream_t s);

hipError_t launch_dedisp(int dtype, bool clean, bool ring, const Tiling& t, const DedispArgs& a,
                         const int32_t* relb, const float* fit32, size_t lds_bytes,
                         hipStream_t s);

// One persistent launch over the tiles of all items (same dtype, cleaning
// and tiling); lds = the largest item's LDS; at most grid_cap workgroups.
hipError_t launch_dedisp_batch(int dtype, bool clean, const Tiling& t, BatchArgs& b, size_t lds,
                               int grid_cap, hipStream_t s);

// At plan creation: raises the LDS limit of every dedispersion kernel of the
// storage type and tiling, and returns the persistent kernel's resident
// workgroups per CU at `lds` bytes (occ[0] without, occ[1] with cleaning).
hipError_t dedisp_prepare(int dtype, const Tiling& t, size_t lds, int occ[2]);

// Integer kernel for 8-bit data without cleaning (dedisp_u8.hip): 12
// consumer waves of kU8G DMs, kU8BT outputs per tile, kU8BC channels per
// LDS stage staged as eight shifted 16-bit copies kU8RS samples apart, of
// which a plan's rows use the first `rs` (a multiple of 8, at most kU8RS);
// two stages of 160,256 bytes.
constexpr int kU8G = 4, kU8BD = 48, kU8BT = 512, kU8BC = 4, kU8KM = 3, kU8RS = 1240;
static_assert(kU8RS % 8 == 0 && kU8RS / 8 <= 64 * kU8KM, "integer staging rows");
// Per-(DM, channel) LDS byte offsets of the integer kernel (ldr: table row
// stride, channels rounded up to 4).
hipError_t launch_relb_u8(const int32_t* delays, int32_t C, int32_t ndms, int32_t ldr, int32_t* relb,
                          hipStream_t s);
// Raises the integer kernel's LDS limit (at plan creation).
hipError_t dedisp_u8_prepare();
// One single-shot launch: a.rs, a.n_dblocks and a.n_ttiles in the integer
// kernel's geometry; a.x 8-byte aligned with a.ld a multiple of 8.
hipError_t launch_dedisp_u8(const DedispArgs& a, const int32_t* relb, size_t lds, hipStream_t s);

// Writes the chunk's last min(L, R) cleaned samples into the ring at the
// positions given by the beam's device-side sample count, then advances the
// beam's device-side position (seen_dev: [seen, first output of the chunk,
// stream base], see beam_advance_kernel).
hipError_t launch_ring_update(int dtype, bool clean, const void* x, int64_t ld, int64_t L,
                              int32_t C, const CleanView& cv, const float* fit32, float* ring,
                              int64_t R, int64_t* seen_dev, int64_t smax, hipStream_t s);
// Restarts a beam's device-side position at absolute sample `base`.
hipError_t launch_beam_seek(int64_t* seen_dev, int64_t base, hipStream_t s);

struct NormDev { double a, b, sigma; int32_t degenerate, reserved; };
struct CandDev { int32_t dm_index, reserved; int64_t sample; float snr, dm; };
struct PeakDev { int64_t sample; float snr; int32_t reserved; };

hipError_t launch_norm(const float* out, int64_t ld_out, int64_t nout, int32_t ndms,
                       NormDev* norm, hipStream_t s);

// Windowed median filter (median.hip): half widths 0..kMedianMaxHalf; one
// workgroup per median_tile() outputs of a row.
constexpr int kMedianMaxHalf = 16;
int64_t median_tile();
int64_t median_max_workgroups();
hipError_t launch_median(const float* in, int64_t ld_in, float* out, int64_t ld_out, int32_t nrows,
                         int64_t ncols, int32_t half_width, hipStream_t s);

// Power of beamformed voltages (power.hip): [C][ld_in] complex int16 ->
// [C][ld_out] FP32.
hipError_t launch_power(const int16_t* in, int64_t ld_in, int32_t C, int64_t T, float* out, int64_t ld_out,
                        hipStream_t s);

// mu-law codec of the data writer (mulaw.hip).
hipError_t launch_mulaw_encode(const float* in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                               uint8_t* codes, int64_t ld_codes, float* xmax, hipStream_t s);
hipError_t launch_mulaw_decode(const uint8_t* codes, int64_t ld_codes, const float* xmax, int32_t nrows,
                               int64_t ncols, float mu, float* out, int64_t ld_out, hipStream_t s);
// DBSCAN clustering of detections (cluster.hip); the candidates are in
// (dm_index, sample) order, n < 2^31.
size_t cluster_work_bytes(int64_t n, int32_t ndms);
hipError_t launch_cluster(const CandDev* c, int32_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps, float snr_eps,
                          int32_t min_pts, int32_t* labels, int32_t* nclusters, void* work, hipStream_t s);

// 4+4-bit codec of 16-bit complex voltages (mulaw.hip); ld_in, ncols and
// ld_out count complex samples.
hipError_t launch_mulaw_encode_complex(const int16_t* in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                                       uint8_t* codes, int64_t ld_codes, int32_t* xmax, hipStream_t s);
hipError_t launch_mulaw_decode_complex(const uint8_t* codes, int64_t ld_codes, const int32_t* xmax, int32_t nrows,
                                       int64_t ncols, float mu, float* out, int64_t ld_out, hipStream_t s);

hipError_t launch_detect(const float* out, int64_t ld_out, int64_t nout, int32_t ndms,
                         const NormDev* norm, int64_t sample0, const int64_t* d_sample0, double nsigma,
                         double dm_start, double dm_step, CandDev* cands, int64_t capacity,
                         int64_t* d_count, PeakDev* peaks, void* work, hipStream_t s);

// Segments (one wave each) per DM row in the detection kernels.
constexpr int kDetectSegs = 16;

inline size_t detect_work_bytes(int32_t ndms) {
  // counts and offsets per (row, segment)
  return align256(sizeof(int64_t) * 2 * kDetectSegs * size_t(ndms));
}

// FDBSCAN of detections (cluster.hip): workspace bytes and the launches.
size_t fdbscan_work_bytes(int64_t n, int32_t ndms);
hipError_t launch_fdbscan(const CandDev* c, int32_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps, float snr_eps,
                          int32_t min_pts, int32_t* labels, int32_t* nclusters, int64_t* nqueries, void* work,
                          hipStream_t s);

// Most DM rows the allocation-free detection can take: its counts and
// offsets live in a fixed device array of detect_work_bytes(this) = 2 MiB.
constexpr int32_t kDetectNoAllocMaxDms = 8192;

// Looks up, once per device, the device address of the allocation-free
// detection's scratch array on the current device (no allocation).
hipError_t detect_scratch_setup(void** ptr);

// launch_detect with the counts and offsets in that scratch array (found
// with detect_scratch_setup on the current device); ndms must not exceed
// kDetectNoAllocMaxDms.
hipError_t launch_detect_noalloc(const float* out, int64_t ld_out, int64_t nout, int32_t ndms,
                                 const NormDev* norm, int64_t sample0, const int64_t* d_sample0, double nsigma,
                                 double dm_start, double dm_step, CandDev* cands, int64_t capacity,
                                 int64_t* d_count, PeakDev* peaks, hipStream_t s);

}  // namespace mbtp
