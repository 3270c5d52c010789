// Host runtime behind the C ABI of include/mbtp.h: argument validation, the
// FP64 delay table of Eq. (1), the choice of dedispersion tiling, device
// memory owned by plans and beams, and the launch sequence of each call.
//
// Compiled with -ffp-contract=off: the delay table is formed with plain
// IEEE FP64 multiplies, divides and adds, in the order written.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/mbtp.h"
#include "internal.h"

using namespace mbtp;

namespace {

thread_local std::string g_err;

mb_status fail(mb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

mb_status ok() {
  g_err.clear();
  return MB_OK;
}

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(MB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

// Eq. (1) with k = 4.15e6 ms MHz^2 = 4150 s MHz^2, f_ref the highest channel
// centre, rounded to the nearest sample (halves up).
constexpr double kDispersionS = 4150.0;

void build_delays(const mb_plan_desc& d, std::vector<int32_t>& out, int32_t& smax) {
  const int C = d.nchans, N = d.ndms;
  std::vector<double> f(C);
  double fref = -1.0;
  for (int c = 0; c < C; ++c) {
    f[c] = d.f_ch0_mhz + (double)c * d.df_mhz;
    if (f[c] > fref) fref = f[c];
  }
  std::vector<double> inv(C);
  const double iref = 1.0 / (fref * fref);
  for (int c = 0; c < C; ++c) inv[c] = 1.0 / (f[c] * f[c]) - iref;
  out.assign((size_t)N * C, 0);
  smax = 0;
  for (int k = 0; k < N; ++k) {
    const double dm = d.dm_start + (double)k * d.dm_step;
    const double kd = kDispersionS * dm;
    for (int c = 0; c < C; ++c) {
      const double v = kd * inv[c] / d.tsamp_s;
      const int32_t s = (int32_t)floor(v + 0.5);
      out[(size_t)k * C + c] = s;
      if (s > smax) smax = s;
    }
  }
}

bool check_aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int dtype_bytes(int dt) { return dt == MB_U8 ? 1 : (dt == MB_F16 ? 2 : 4); }

}  // namespace

struct mb_plan {
  mb_plan_desc desc;
  int device = 0;
  int32_t smax = 0;
  std::vector<int32_t> h_delays;
  int32_t* d_delays = nullptr;
  int32_t* d_relb = nullptr;
  Tiling tiling{4, 4, 2, 4, 0};
  int tile_index = 1;          // 1-based index in the compiled list
  int rs = 0;
  size_t lds = 0;
  int n_dblocks = 0;
  int relb_ld = 0;
  int cus = 0;                 // compute units of the plan's device
  int batch_occ[2] = {1, 1};   // persistent workgroups per CU (no cleaning, cleaning)
  // 8-bit plans: the exact integer kernel for chunks without cleaning, when
  // its staging fits (copy length rs8 samples, lds8 bytes, offsets d_relb8)
  bool u8_int = false;
  int rs8 = 0;
  size_t lds8 = 0;
  int32_t* d_relb8 = nullptr;
};

struct mb_beam {
  const mb_plan* plan = nullptr;
  float* d_ring = nullptr;
  // device-side position: [0] samples seen since the stream (re)started (the
  // ring position kernels read), [1] absolute index of the last chunk's first
  // output, [2] absolute index of the stream's first sample
  int64_t* d_seen = nullptr;
  int64_t R = 0;
  int64_t seen = 0;            // host copy of [0]
  int64_t base = 0;            // host copy of [2]
};

namespace {

// Largest spread s[dlast][c] - s[d0][c] over DM blocks of size BD.
int32_t span_max(const mb_plan& p, int BD) {
  const int C = p.desc.nchans, N = p.desc.ndms;
  int32_t m = 0;
  for (int d0 = 0; d0 < N; d0 += BD) {
    const int dl = (d0 + BD < N ? d0 + BD : N) - 1;
    for (int c = 0; c < C; ++c) {
      const int32_t s = p.h_delays[(size_t)dl * C + c] - p.h_delays[(size_t)d0 * C + c];
      if (s > m) m = s;
    }
  }
  return m;
}

// chunk lengths up to 2^30 keep every window-relative sample index of the
// kernels (chunk, ring and staging margin) inside 32 bits
constexpr int64_t kMaxSamps = int64_t(1) << 30;
constexpr int32_t kMaxDms = 65535;                 // DM trials of one plan
constexpr int32_t kMaxClassifyDms = 4000;          // per-row tables of one cluster in 64 KB of LDS
constexpr size_t kMaxLds = 160 * 1024 - 256;   // gfx950 LDS per workgroup, less the persistent kernel's static LDS

// LDS copy length: the largest window start (span + 3, rounded down to 4)
// plus the tile, plus the quad read after the last one.
void tiling_geometry(const mb_plan& p, const Tiling& t, int& rs, size_t& lds) {
  const int sp = span_max(p, t.BD());
  rs = (t.BT() + sp + 7 + 3) & ~3;
  // the staged copies of each channel, then the block's [BC][BD] offsets
  lds = ((size_t)t.BC * t.copies() * rs * sizeof(float) + (size_t)t.BC * t.BD() * sizeof(int32_t)) *
        ((t.P & 2) ? 2 : 1);   // P bit 1: two stages (double buffer)
}

// A tiling fits when its LDS fits and each lane's prefetch registers cover
// its share of a channel block.
// Staging registers: with NSW >= BC staging waves, WPR waves split a row of
// rs/4 quads into ranges of qw quads (one quad of overlap) and each lane
// holds KM of them; with NSW < BC a wave stages BC/NSW whole rows.  Same
// rule as the kernel.
bool tiling_fits(const Tiling& t, int rs, size_t lds) {
  const int rs4 = rs / 4;
  if (lds > kMaxLds) return false;
  const int nsw = t.staging_waves();
  if (nsw >= t.BC) {
    const int wpr = nsw / t.BC;
    const int qwmax = (64 * kStageQuads - 1 + wpr - 1) / wpr + 1;
    const int km = (qwmax + 63) / 64;
    const int qw = wpr > 1 ? (rs4 - 1 + wpr - 1) / wpr + 1 : rs4;
    return qw <= 64 * km;
  }
  const int rows_per_wave = t.BC / nsw;
  return rows_per_wave * ((rs4 + 63) / 64) <= kStageQuads;
}

mb_status choose_tiling(mb_plan& p) {
  const int n = n_tilings();
  int pick = -1;
  if (p.desc.tile_hint > 0) {
    if (p.desc.tile_hint > n) return fail(MB_EINVAL, "tile_hint %d out of range 1..%d", p.desc.tile_hint, n);
    pick = p.desc.tile_hint - 1;
    int rs; size_t lds;
    tiling_geometry(p, tiling_at(pick), rs, lds);
    if (!tiling_fits(tiling_at(pick), rs, lds))
      return fail(MB_EINVAL, "tiling %d does not fit this plan (LDS %zu bytes, row %d)", p.desc.tile_hint, lds, rs);
  } else {
    // preference order of the compiled list; the first that fits in LDS
    for (int i = 0; i < n && pick < 0; ++i) {
      int rs; size_t lds;
      tiling_geometry(p, tiling_at(i), rs, lds);
      if (tiling_fits(tiling_at(i), rs, lds)) pick = i;
    }
    if (pick < 0) return fail(MB_EINVAL, "the DM step is too coarse for the compiled tilings (LDS)");
  }
  p.tiling = tiling_at(pick);
  p.tile_index = pick + 1;
  tiling_geometry(p, p.tiling, p.rs, p.lds);
  p.n_dblocks = (p.desc.ndms + p.tiling.BD() - 1) / p.tiling.BD();
  return MB_OK;
}

// Geometry of the integer kernel for 8-bit data: each staged copy holds the
// largest window start (span + 7, rounded down to 8) plus the tile, plus the
// octet after the last one read, whose successor the producers need.
void u8_geometry(mb_plan& p) {
  const int sp = span_max(p, kU8BD);
  const int rs = ((sp + 7) & ~7) + kU8BT + 8;
  const size_t lds = 2 * ((size_t)kU8BC * 16 * kU8RS + (size_t)kU8BC * kU8BD * sizeof(int32_t));
  p.u8_int = p.desc.in_dtype == MB_U8 && rs <= kU8RS && lds <= kMaxLds;
  p.rs8 = rs;
  p.lds8 = lds;
}

mb_status validate_rfi(const mb_rfi_params& r, int C) {
  if (r.poly_order < 0 || r.poly_order > 8) return fail(MB_EINVAL, "rfi.poly_order %d not in 0..8", r.poly_order);
  if (r.window < kSpan || (r.window & (r.window - 1)) != 0)
    return fail(MB_EINVAL, "rfi.window %d must be a power of two >= %d", r.window, kSpan);
  if (!(r.k_mask > 0) || !(r.k_chan > 0) || !(r.k_spec > 0))
    return fail(MB_EINVAL, "rfi threshold factors must be positive");
  if (r.mask_passes < 1 || r.mask_passes > 16) return fail(MB_EINVAL, "rfi.mask_passes %d not in 1..16", r.mask_passes);
  if (r.reserved != 0) return fail(MB_EINVAL, "rfi.reserved must be 0");
  (void)C;
  return MB_OK;
}

// Arguments shared by both detection entry points.
mb_status validate_detect(const mb_plan* plan, const float* d_out, int64_t nout, int64_t ld_out,
                          const mb_norm* d_norm, int64_t sample0, double nsigma, const mb_candidate* d_cands,
                          int64_t capacity, const int64_t* d_count) {
  if (!plan) return fail(MB_EINVAL, "plan is NULL");
  if (nout < 0 || sample0 < 0) return fail(MB_EINVAL, "nout and sample0 must be >= 0");
  if (nout > 0 && (!d_out || !check_aligned(d_out, 16) || ld_out < nout || ld_out % 4 != 0))
    return fail(MB_EINVAL, "output plane must be 16-byte aligned with ld_out >= nout, ld_out %% 4 == 0");
  if (!d_norm || !d_count) return fail(MB_EINVAL, "norm and count must not be NULL");
  if (capacity < 0 || (capacity > 0 && !d_cands)) return fail(MB_EINVAL, "capacity > 0 needs a candidate buffer");
  if (!isfinite(nsigma)) return fail(MB_EINVAL, "nsigma must be finite");
  return MB_OK;
}

mb_status validate_input(const mb_plan* plan, const void* d_in, int64_t nsamps, int64_t ld) {
  if (!plan) return fail(MB_EINVAL, "plan is NULL");
  if (!d_in) return fail(MB_EINVAL, "input pointer is NULL");
  if (!check_aligned(d_in, 16)) return fail(MB_EINVAL, "input pointer must be 16-byte aligned");
  if (nsamps < 1) return fail(MB_EINVAL, "nsamps must be >= 1");
  if (nsamps > kMaxSamps) return fail(MB_EINVAL, "nsamps must be <= 2^30");
  if (ld < nsamps || ld % 4 != 0) return fail(MB_EINVAL, "ld (%lld) must be >= nsamps and a multiple of 4", (long long)ld);
  return MB_OK;
}

}  // namespace

extern "C" {

const char* mb_status_str(mb_status s) {
  switch (s) {
    case MB_OK: return "ok";
    case MB_EINVAL: return "invalid argument";
    case MB_ENOMEM: return "out of device memory";
    case MB_EDEVICE: return "HIP runtime error";
    case MB_ECAPACITY: return "capacity exceeded";
    case MB_EBUSY: return "busy";
    default: return "unknown status";
  }
}

const char* mb_last_error(void) { return g_err.c_str(); }

void mb_rfi_defaults(mb_rfi_params* p) {
  if (!p) return;
  p->poly_order = 3;
  p->window = 256;
  p->k_mask = 5.0;
  p->k_chan = 5.0;
  p->k_spec = 5.0;
  p->mask_passes = 8;
  p->reserved = 0;
}

mb_status dedisp_plan_create(const mb_plan_desc* desc, mb_plan** out) {
  if (!desc || !out) return fail(MB_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  const mb_plan_desc& d = *desc;
  if (d.nchans < 1 || d.nchans > 65535) return fail(MB_EINVAL, "nchans %d not in 1..65535", d.nchans);
  if (d.ndms < 1 || d.ndms > 65535) return fail(MB_EINVAL, "ndms %d not in 1..65535", d.ndms);
  if (!(d.tsamp_s > 0) || !isfinite(d.tsamp_s)) return fail(MB_EINVAL, "tsamp_s must be > 0");
  if (!(d.df_mhz != 0) || !isfinite(d.df_mhz)) return fail(MB_EINVAL, "df_mhz must be non-zero");
  if (!(d.dm_start >= 0) || !(d.dm_step >= 0) || !isfinite(d.dm_start) || !isfinite(d.dm_step))
    return fail(MB_EINVAL, "dm_start and dm_step must be >= 0");
  const double flo = d.df_mhz > 0 ? d.f_ch0_mhz : d.f_ch0_mhz + (d.nchans - 1) * d.df_mhz;
  if (!(flo > 0) || !isfinite(d.f_ch0_mhz)) return fail(MB_EINVAL, "channel centres must be > 0 MHz");
  if (d.in_dtype != MB_U8 && d.in_dtype != MB_F16 && d.in_dtype != MB_F32)
    return fail(MB_EINVAL, "in_dtype %d unknown", d.in_dtype);
  if (d.tile_hint < 0) return fail(MB_EINVAL, "tile_hint must be >= 0");
  mb_status st = validate_rfi(d.rfi, d.nchans);
  if (st) return st;

  mb_plan* p = new (std::nothrow) mb_plan;
  if (!p) return fail(MB_ENOMEM, "host allocation failed");
  p->desc = d;
  build_delays(d, p->h_delays, p->smax);
  // the largest delay must leave room in 32-bit sample arithmetic
  if ((double)p->smax > 1.0e9) {
    delete p;
    return fail(MB_EINVAL, "largest delay %d samples is too large", p->smax);
  }
  st = choose_tiling(*p);
  if (st) { delete p; return st; }
  u8_geometry(*p);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return fail(MB_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)); }
  const size_t tb = sizeof(int32_t) * p->h_delays.size();
  p->relb_ld = (d.nchans + 3) & ~3;
  const size_t rb = sizeof(int32_t) * (size_t)p->relb_ld * d.ndms;
  if (hipMalloc(&p->d_delays, tb) != hipSuccess || hipMalloc(&p->d_relb, rb) != hipSuccess ||
      (p->u8_int && hipMalloc(&p->d_relb8, rb) != hipSuccess)) {
    (void)hipFree(p->d_delays);
    (void)hipFree(p->d_relb);
    delete p;
    return fail(MB_ENOMEM, "hipMalloc of %zu bytes failed", tb + rb);
  }
  e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e == hipSuccess) e = dedisp_prepare(d.in_dtype, p->tiling, p->lds, p->batch_occ);
  if (e == hipSuccess) e = hipMemcpy(p->d_delays, p->h_delays.data(), tb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_relb(p->d_delays, d.nchans, d.ndms, p->tiling.BD(), p->rs, p->tiling.copies(),
                                        p->relb_ld, p->d_relb, nullptr);
  if (e == hipSuccess && p->u8_int) e = dedisp_u8_prepare();
  if (e == hipSuccess && p->u8_int)
    e = launch_relb_u8(p->d_delays, d.nchans, d.ndms, p->relb_ld, p->d_relb8, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  // the allocation-free detection's scratch address on this device, looked
  // up here so that later calls (possibly under graph capture) only read it
  void* scratch_dev = nullptr;
  if (e == hipSuccess) e = detect_scratch_setup(&scratch_dev);
  if (e != hipSuccess) {
    (void)hipFree(p->d_delays);
    (void)hipFree(p->d_relb);
    (void)hipFree(p->d_relb8);
    delete p;
    return fail(MB_EDEVICE, "plan upload failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return ok();
}

mb_status dedisp_plan_destroy(mb_plan* plan) {
  if (!plan) return ok();
  (void)hipFree(plan->d_delays);
  (void)hipFree(plan->d_relb);
  (void)hipFree(plan->d_relb8);
  delete plan;
  return ok();
}

mb_status dedisp_plan_info(const mb_plan* plan, mb_plan_info* info) {
  if (!plan || !info) return fail(MB_EINVAL, "plan and info must not be NULL");
  info->nchans = plan->desc.nchans;
  info->ndms = plan->desc.ndms;
  info->max_delay = plan->smax;
  info->dm_block = plan->tiling.BD();
  info->time_tile = plan->tiling.BT();
  info->chan_block = plan->tiling.BC;
  info->tile_index = plan->tile_index;
  info->waves = plan->tiling.NW;
  info->lds_bytes = (int64_t)plan->lds;
  info->u8_integer = plan->u8_int ? 1 : 0;
  info->reserved = 0;
  return ok();
}

mb_status dedisp_tilings(int32_t* count) {
  if (!count) return fail(MB_EINVAL, "count is NULL");
  *count = n_tilings();
  return ok();
}

mb_status dedisp_plan_delays(const mb_plan* plan, int32_t* h_delays) {
  if (!plan || !h_delays) return fail(MB_EINVAL, "plan and h_delays must not be NULL");
  memcpy(h_delays, plan->h_delays.data(), sizeof(int32_t) * plan->h_delays.size());
  return ok();
}

mb_status rfi_state_layout(const mb_plan* plan, int64_t nsamps, mb_rfi_layout* layout) {
  if (!plan || !layout) return fail(MB_EINVAL, "plan and layout must not be NULL");
  if (nsamps < 1 || nsamps > kMaxSamps) return fail(MB_EINVAL, "nsamps must be in 1..2^30");
  const RfiGeom g = rfi_geometry(plan->desc.nchans, nsamps, plan->desc.rfi.window);
  layout->total_bytes = g.total;
  layout->fit_f64 = g.off_fit;
  layout->bandpass_f64 = g.off_binterp;
  layout->chunk_sum_f64 = g.off_chunk;
  layout->chunk_flags_u8 = g.off_flags;
  layout->spectrum_flags_u8 = g.off_gflags;
  layout->masked_u8 = g.off_masked;
  layout->nchunks = g.J;
  return ok();
}

mb_status rfi_threshold(const mb_plan* plan, const void* d_in, int64_t nsamps, int64_t ld,
                        void* d_state, size_t state_bytes, void* stream) {
  mb_status st = validate_input(plan, d_in, nsamps, ld);
  if (st) return st;
  const int C = plan->desc.nchans;
  const mb_rfi_params& r = plan->desc.rfi;
  if (C < r.poly_order + 2) return fail(MB_EINVAL, "RFI fit needs nchans >= poly_order + 2");
  if (!d_state || !check_aligned(d_state, 256)) return fail(MB_EINVAL, "state must be non-NULL and 256-byte aligned");
  const RfiGeom g = rfi_geometry(C, nsamps, r.window);
  if (state_bytes < g.total) return fail(MB_EINVAL, "state buffer has %zu bytes, needs %zu", state_bytes, g.total);
  RfiParamsDev prm;
  prm.p = r.poly_order;
  prm.W = r.window;
  prm.mask_passes = r.mask_passes;
  prm.k_mask = r.k_mask;
  prm.k_chan = r.k_chan;
  prm.k_spec = r.k_spec;
  HIP_TRY(launch_rfi(plan->desc.in_dtype, d_in, ld, g, prm, static_cast<char*>(d_state),
                     static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status rfi_report(const mb_plan* plan, const void* d_state, mb_rfi_report* h_report, void* stream) {
  if (!plan || !d_state || !h_report) return fail(MB_EINVAL, "plan, state and report must not be NULL");
  RfiHeader h;
  HIP_TRY(hipMemcpyAsync(&h, d_state, sizeof(h), hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream)));
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  h_report->sigma = h.sigma;
  h_report->rmse0 = h.rmse0;
  h_report->rmse = h.rmse;
  h_report->sum_fit = h.sum_fit;
  h_report->n_masked = (int64_t)h.n_masked;
  h_report->n_chunk_flags = (int64_t)h.n_chunk;
  h_report->n_chunk_flags_ext = (int64_t)h.n_chunk_ext;
  h_report->n_spectrum_flags = (int64_t)h.n_spec;
  h_report->nsamps = h.nsamps;
  h_report->nchunks = h.nchunks;
  h_report->error = h.error;
  h_report->reserved = 0;
  return ok();
}

mb_status dedisp_beam_create(const mb_plan* plan, mb_beam** out) {
  if (!plan || !out) return fail(MB_EINVAL, "plan and out must not be NULL");
  *out = nullptr;
  mb_beam* b = new (std::nothrow) mb_beam;
  if (!b) return fail(MB_ENOMEM, "host allocation failed");
  b->plan = plan;
  b->R = ((int64_t)plan->smax + 3) & ~(int64_t)3;
  if (b->R > 0) {
    const size_t bytes = sizeof(float) * (size_t)plan->desc.nchans * (size_t)b->R;
    if (hipMalloc(&b->d_ring, bytes) != hipSuccess) {
      delete b;
      return fail(MB_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
  }
  const int64_t zero[3] = {0, 0, 0};
  if (hipMalloc(&b->d_seen, sizeof(zero)) != hipSuccess ||
      hipMemcpy(b->d_seen, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(b->d_ring);
    (void)hipFree(b->d_seen);
    delete b;
    return fail(MB_ENOMEM, "beam state allocation failed");
  }
  *out = b;
  return ok();
}

mb_status dedisp_beam_destroy(mb_beam* beam) {
  if (!beam) return ok();
  (void)hipFree(beam->d_ring);
  (void)hipFree(beam->d_seen);
  delete beam;
  return ok();
}

mb_status dedisp_beam_reset(mb_beam* beam) {
  if (!beam) return fail(MB_EINVAL, "beam is NULL");
  const int64_t zero[3] = {0, 0, 0};
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(beam->d_seen, zero, sizeof(zero), hipMemcpyHostToDevice));
  beam->seen = 0;
  beam->base = 0;
  return ok();
}

mb_status dedisp_beam_seek(mb_beam* beam, int64_t position, void* stream) {
  if (!beam) return fail(MB_EINVAL, "beam is NULL");
  if (position < 0 || position > (int64_t(1) << 62)) return fail(MB_EINVAL, "position must be in [0, 2^62]");
  HIP_TRY(launch_beam_seek(beam->d_seen, position, static_cast<hipStream_t>(stream)));
  beam->seen = 0;
  beam->base = position;
  return ok();
}

mb_status dedisp_beam_sample0_ptr(const mb_beam* beam, const int64_t** d_sample0) {
  if (!beam || !d_sample0) return fail(MB_EINVAL, "beam and d_sample0 must not be NULL");
  *d_sample0 = beam->d_seen + 1;
  return ok();
}

mb_status dedisp_beam_advance(mb_beam* beam, int64_t nsamps) {
  if (!beam || nsamps < 0 || nsamps % 4 != 0) return fail(MB_EINVAL, "beam non-NULL, nsamps >= 0 and a multiple of 4");
  beam->seen += nsamps;
  return ok();
}

mb_status dedisp_beam_position(const mb_beam* beam, int64_t* seen) {
  if (!beam || !seen) return fail(MB_EINVAL, "beam and seen must not be NULL");
  *seen = beam->seen;
  return ok();
}

}  // extern "C"

namespace {

// One item of an execute call, validated and turned into launch arguments.
struct Prepared {
  const mb_plan* plan;
  mb_beam* beam;
  const void* d_in;
  int64_t nsamps, ld;
  bool clean;
  CleanView cv;
  const float* fit32;
  DedispArgs a;
  float* d_out;
  int64_t ld_out;
  mb_norm* d_norm;
  int64_t nout, sample0;
};

mb_status prepare(const mb_plan* plan, mb_beam* beam, const void* d_in, int64_t nsamps, int64_t ld,
                  const void* d_rfi_state, float* d_out, int64_t ld_out, mb_norm* d_norm, Prepared& P) {
  mb_status st = validate_input(plan, d_in, nsamps, ld);
  if (st) return st;
  if (beam && beam->plan != plan) return fail(MB_EINVAL, "beam was created from another plan");
  if (d_rfi_state && !check_aligned(d_rfi_state, 256)) return fail(MB_EINVAL, "RFI state must be 256-byte aligned");
  // Streaming keeps ring length, ring position and chunk starts on
  // multiples of 4 so that staged quads never straddle the ring/chunk edge.
  if (beam && nsamps % 4 != 0) return fail(MB_EINVAL, "streaming chunks must hold a multiple of 4 samples");
  const int64_t smax = plan->smax;
  const int64_t R = beam ? beam->R : 0;
  const int64_t seen = beam ? beam->seen : 0;
  const int64_t v = beam ? (seen < R ? seen : R) : 0;          // ring samples staged
  const int64_t veff = beam ? (seen < smax ? seen : smax) : 0;  // of which needed
  const int64_t phase = v - veff;
  const int64_t nout = veff + nsamps - smax;
  if (!beam && nout <= 0)
    return fail(MB_EINVAL, "nsamps (%lld) must exceed the largest delay (%lld)", (long long)nsamps, (long long)smax);
  const int64_t nout_c = nout > 0 ? nout : 0;
  if (nout_c > 0) {
    if (!d_out || !check_aligned(d_out, 16)) return fail(MB_EINVAL, "output must be non-NULL and 16-byte aligned");
    if (ld_out < nout_c || ld_out % 4 != 0)
      return fail(MB_EINVAL, "ld_out (%lld) must be >= nout (%lld) and a multiple of 4", (long long)ld_out, (long long)nout_c);
  }
  if (d_norm && !check_aligned(d_norm, 8)) return fail(MB_EINVAL, "norm must be 8-byte aligned");
  if (beam && beam->base + seen > (int64_t(1) << 62) - nsamps)
    return fail(MB_EINVAL, "absolute sample index of the stream would exceed 2^62");
  P = Prepared{};
  P.plan = plan;
  P.beam = beam;
  P.d_in = d_in;
  P.nsamps = nsamps;
  P.ld = ld;
  P.clean = d_rfi_state != nullptr;
  P.d_out = d_out;
  P.ld_out = ld_out;
  P.d_norm = d_norm;
  P.nout = nout_c;
  P.sample0 = (beam ? beam->base : 0) + seen - veff;
  if (P.clean) {
    const RfiGeom g = rfi_geometry(plan->desc.nchans, nsamps, plan->desc.rfi.window);
    const char* stp = static_cast<const char*>(d_rfi_state);
    CleanView& cv = P.cv;
    cv.fit = reinterpret_cast<const double*>(stp + g.off_fit);
    cv.cflags = reinterpret_cast<const uint8_t*>(stp + g.off_flags);
    cv.gflags = reinterpret_cast<const uint8_t*>(stp + g.off_gflags);
    cv.J = g.J;
    cv.cbits = reinterpret_cast<const uint32_t*>(stp + g.off_cbits);
    cv.JW = g.JW;
    cv.W = (uint32_t)plan->desc.rfi.window;
    cv.wshift = 0;
    while ((1u << cv.wshift) < cv.W) ++cv.wshift;
    P.fit32 = reinterpret_cast<const float*>(stp + g.off_fit32);
  }
  DedispArgs& A = P.a;
  A.x = d_in;
  A.ld = ld;
  A.L = nsamps;
  A.ring = beam ? beam->d_ring : nullptr;
  A.R = R;
  A.ring_valid = v;
  A.ring_p0 = (R > 0) ? (seen - v) % R : 0;
  A.phase = phase;
  A.delays = plan->d_delays;
  A.C = plan->desc.nchans;
  A.ndms = plan->desc.ndms;
  A.nout = nout_c;
  A.out = d_out;
  A.ld_out = ld_out;
  A.clean = P.cv;
  A.n_dblocks = plan->n_dblocks;
  A.n_ttiles = (int32_t)((phase + nout_c + plan->tiling.BT() - 1) / plan->tiling.BT());
  A.rs = plan->rs;
  A.relb_ld = plan->relb_ld;
  A.zero = 0;
  A.seen_dev = beam ? beam->d_seen : nullptr;
  return MB_OK;
}

// Whether a prepared item's outputs that read only its own chunk run on the
// exact integer kernel: 8-bit samples, no cleaning, and rows the kernel can
// read as aligned octets.  Its results equal the float kernels' bit for bit.
bool uses_u8_int(const Prepared& P) {
  return P.plan->u8_int && !P.clean && P.nsamps > P.plan->smax &&
         (reinterpret_cast<uintptr_t>(P.d_in) & 7) == 0 && P.ld % 8 == 0;
}

// Normalisation and ring update of a prepared item, after its dedispersion.
mb_status finish_item(Prepared& P, hipStream_t s) {
  const mb_plan* plan = P.plan;
  if (P.d_norm)
    HIP_TRY(launch_norm(P.d_out, P.ld_out, P.nout, plan->desc.ndms, reinterpret_cast<NormDev*>(P.d_norm), s));
  if (P.beam) {
    HIP_TRY(launch_ring_update(plan->desc.in_dtype, P.clean, P.d_in, P.ld, P.nsamps, plan->desc.nchans,
                               P.cv, P.fit32, P.beam->d_ring, P.beam->R, P.beam->d_seen, plan->smax, s));
    P.beam->seen += P.nsamps;
  }
  return MB_OK;
}

}  // namespace

extern "C" {

mb_status dedisp_execute(const mb_plan* plan, mb_beam* beam, const void* d_in, int64_t nsamps,
                         int64_t ld, const void* d_rfi_state, float* d_out, int64_t ld_out,
                         mb_norm* d_norm, mb_exec_info* info, void* stream) {
  Prepared P;
  mb_status st = prepare(plan, beam, d_in, nsamps, ld, d_rfi_state, d_out, ld_out, d_norm, P);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool ring = beam != nullptr && P.a.ring_valid > 0;
  const bool integer = P.nout > 0 && uses_u8_int(P);
  if (integer) {
    // The last nsamps - s_max outputs read only this chunk's samples: the
    // integer kernel sums them as a single shot over the chunk.  With ring
    // samples staged, the float ring kernel forms the outputs before them
    // (the first min(seen, s_max), which read ring samples too).
    const int64_t n2 = P.nsamps - plan->smax, n1 = P.nout - n2;
    if (ring && n1 > 0) {
      DedispArgs a = P.a;
      a.nout = n1;
      a.n_ttiles = (int32_t)((a.phase + n1 + plan->tiling.BT() - 1) / plan->tiling.BT());
      HIP_TRY(launch_dedisp(plan->desc.in_dtype, false, true, plan->tiling, a, plan->d_relb, P.fit32, plan->lds, s));
    }
    DedispArgs a = P.a;
    a.ring = nullptr;
    a.R = 0;
    a.ring_valid = 0;
    a.ring_p0 = 0;
    a.phase = 0;
    a.seen_dev = nullptr;
    a.nout = n2;
    a.out = P.d_out + n1;
    a.rs = plan->rs8;
    a.n_dblocks = (plan->desc.ndms + kU8BD - 1) / kU8BD;
    a.n_ttiles = (int32_t)((n2 + kU8BT - 1) / kU8BT);
    HIP_TRY(launch_dedisp_u8(a, plan->d_relb8, plan->lds8, s));
  } else if (P.nout > 0) {
    HIP_TRY(launch_dedisp(plan->desc.in_dtype, P.clean, ring, plan->tiling, P.a, plan->d_relb, P.fit32,
                          plan->lds, s));
  }
  st = finish_item(P, s);
  if (st) return st;
  if (info) {
    info->nout = P.nout;
    info->sample0 = P.sample0;
    info->integer_kernel = integer ? 1 : 0;
    info->reserved = 0;
  }
  return ok();
}

mb_status dedisp_batch_workspace_size(int32_t nitems, size_t* bytes) {
  if (!bytes || nitems < 1) return fail(MB_EINVAL, "nitems must be >= 1 and bytes non-NULL");
  *bytes = 256 * (size_t)((nitems + kMaxBatch - 1) / kMaxBatch);
  return ok();
}

mb_status dedisp_execute_batch(const mb_batch_item* items, int32_t nitems, void* d_work,
                               size_t work_bytes, mb_exec_info* infos, void* stream) {
  if (!items || nitems < 1) return fail(MB_EINVAL, "items must be non-NULL and nitems >= 1");
  const int32_t nlaunch = (nitems + kMaxBatch - 1) / kMaxBatch;
  if (!d_work || !check_aligned(d_work, 256) || work_bytes < 256 * (size_t)nlaunch)
    return fail(MB_EINVAL, "workspace must be 256-byte aligned with %zu bytes", 256 * (size_t)nlaunch);
  std::vector<Prepared> P(nitems);
  const mb_plan* p0 = items[0].plan;
  if (!p0) return fail(MB_EINVAL, "item 0 has no plan");
  const bool clean0 = items[0].d_rfi_state != nullptr;
  for (int32_t i = 0; i < nitems; ++i) {
    const mb_batch_item& it = items[i];
    if (!it.plan) return fail(MB_EINVAL, "item %d has no plan", i);
    if (it.plan->desc.in_dtype != p0->desc.in_dtype)
      return fail(MB_EINVAL, "item %d: all items of a batch share the storage type", i);
    const Tiling& t = it.plan->tiling;
    if (t.NW != p0->tiling.NW || t.G != p0->tiling.G || t.Q != p0->tiling.Q || t.BC != p0->tiling.BC ||
        t.P != p0->tiling.P)
      return fail(MB_EINVAL, "item %d: all plans of a batch must use the same tiling (tile_hint)", i);
    if ((it.d_rfi_state != nullptr) != clean0)
      return fail(MB_EINVAL, "item %d: either every item or none has an RFI state", i);
    for (int32_t j = 0; j < i; ++j)
      if (it.beam && it.beam == items[j].beam) return fail(MB_EINVAL, "item %d: a beam appears twice", i);
    mb_status st = prepare(it.plan, it.beam, it.d_in, it.nsamps, it.ld, it.d_rfi_state, it.d_out,
                           it.ld_out, it.d_norm, P[i]);
    if (st) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // heaviest tiles first: cost of a tile grows with its channel count
  std::vector<int32_t> order(nitems);
  for (int32_t i = 0; i < nitems; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return P[x].plan->desc.nchans > P[y].plan->desc.nchans;
  });
  for (int32_t l = 0; l < nlaunch; ++l) {
    BatchArgs b;
    memset(&b, 0, sizeof(b));
    b.counter = reinterpret_cast<int*>(static_cast<char*>(d_work) + 256 * (size_t)l);
    size_t lds = 0;
    int32_t total = 0;
    int grid_cap = 1 << 30;
    for (int32_t k = l * kMaxBatch; k < nitems && k < (l + 1) * kMaxBatch; ++k) {
      const Prepared& q = P[order[k]];
      if (q.nout <= 0) continue;
      BatchItem& bi = b.item[b.nitems++];
      bi.a = q.a;
      bi.relb = q.plan->d_relb;
      bi.fit32 = q.fit32;
      bi.tile0 = total;
      total += q.a.n_dblocks * q.a.n_ttiles;
      if (q.plan->lds > lds) lds = q.plan->lds;
      const int occ = q.plan->batch_occ[clean0 ? 1 : 0];
      const int cap = q.plan->cus * (occ < 1 ? 1 : occ);
      if (cap < grid_cap) grid_cap = cap;
    }
    b.total = total;
    if (total > 0) HIP_TRY(launch_dedisp_batch(p0->desc.in_dtype, clean0, p0->tiling, b, lds, grid_cap, s));
  }
  for (int32_t i = 0; i < nitems; ++i) {
    mb_status st = finish_item(P[i], s);
    if (st) return st;
    if (infos) {
      infos[i].nout = P[i].nout;
      infos[i].sample0 = P[i].sample0;
      infos[i].integer_kernel = 0;
      infos[i].reserved = 0;
    }
  }
  return ok();
}

mb_status dedisp_normalise(const mb_plan* plan, const float* d_out, int64_t nout, int64_t ld_out,
                           mb_norm* d_norm, void* stream) {
  if (!plan || !d_norm) return fail(MB_EINVAL, "plan and norm must not be NULL");
  if (nout < 0) return fail(MB_EINVAL, "nout must be >= 0");
  if (nout > 0 && (!d_out || !check_aligned(d_out, 16) || ld_out < nout || ld_out % 4 != 0))
    return fail(MB_EINVAL, "output plane must be 16-byte aligned with ld_out >= nout, ld_out %% 4 == 0");
  if (!check_aligned(d_norm, 8)) return fail(MB_EINVAL, "norm must be 8-byte aligned");
  HIP_TRY(launch_norm(d_out, ld_out, nout, plan->desc.ndms, reinterpret_cast<NormDev*>(d_norm),
                      static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status median_filter(const float* d_in, int64_t ld_in, float* d_out, int64_t ld_out, int32_t nrows,
                        int64_t ncols, int32_t half_width, void* stream) {
  if (nrows < 0 || ncols < 0) return fail(MB_EINVAL, "nrows and ncols must be >= 0");
  if (half_width < 0 || half_width > kMedianMaxHalf)
    return fail(MB_EINVAL, "half_width %d not in 0..%d", half_width, kMedianMaxHalf);
  if (nrows == 0 || ncols == 0) return ok();
  if (!d_in || !d_out) return fail(MB_EINVAL, "planes must not be NULL");
  if (ld_in < ncols || ld_out < ncols) return fail(MB_EINVAL, "ld_in and ld_out must be >= ncols");
  if (ncols > kMaxSamps) return fail(MB_EINVAL, "ncols %lld exceeds %lld", (long long)ncols, (long long)kMaxSamps);
  const int64_t ntiles = (ncols + median_tile() - 1) / median_tile();
  if (ntiles > median_max_workgroups() / nrows) return fail(MB_EINVAL, "plane too large for one launch");
  // the two planes' spans must not intersect
  const uintptr_t i0 = reinterpret_cast<uintptr_t>(d_in);
  const uintptr_t i1 = i0 + sizeof(float) * (size_t)((nrows - 1) * ld_in + ncols);
  const uintptr_t o0 = reinterpret_cast<uintptr_t>(d_out);
  const uintptr_t o1 = o0 + sizeof(float) * (size_t)((nrows - 1) * ld_out + ncols);
  if (i0 < o1 && o0 < i1) return fail(MB_EINVAL, "d_out must not overlap d_in");
  HIP_TRY(launch_median(d_in, ld_in, d_out, ld_out, nrows, ncols, half_width, static_cast<hipStream_t>(stream)));
  return ok();
}

// A plane [nrows][ld] of elem-byte samples, ncols used per row: its byte span.
static mb_status plane_span(const void* p, int64_t ld, int32_t nrows, int64_t ncols, size_t elem, const char* what,
                     uintptr_t& lo, uintptr_t& hi) {
  if (!p) return fail(MB_EINVAL, "%s must not be NULL", what);
  if (ld < ncols) return fail(MB_EINVAL, "%s: leading dimension %lld below ncols %lld", what, (long long)ld,
                              (long long)ncols);
  lo = reinterpret_cast<uintptr_t>(p);
  hi = lo + elem * (size_t)((nrows - 1) * ld + ncols);
  return MB_OK;
}

static mb_status mulaw_check(int32_t nrows, int64_t ncols, float mu) {
  if (nrows < 0 || ncols < 0) return fail(MB_EINVAL, "nrows and ncols must be >= 0");
  if (!(mu > 0.0f) || !isfinite(mu)) return fail(MB_EINVAL, "mu must be finite and > 0");
  if (ncols > kMaxSamps) return fail(MB_EINVAL, "ncols %lld exceeds %lld", (long long)ncols, (long long)kMaxSamps);
  if ((ncols + 1023) / 1024 > 2147483647 / (nrows > 0 ? nrows : 1))
    return fail(MB_EINVAL, "plane too large for one launch");
  return MB_OK;
}

mb_status power_from_voltages(const int16_t* d_in, int64_t ld_in, int32_t nchans, int64_t nsamps, float* d_out,
                              int64_t ld_out, void* stream) {
  if (nchans < 0 || nsamps < 0) return fail(MB_EINVAL, "nchans and nsamps must be >= 0");
  if (nchans == 0 || nsamps == 0) return ok();
  if (nsamps > kMaxSamps) return fail(MB_EINVAL, "nsamps %lld exceeds %lld", (long long)nsamps, (long long)kMaxSamps);
  if ((nsamps + 4095) / 4096 > 2147483647 / nchans) return fail(MB_EINVAL, "plane too large for one launch");
  uintptr_t i0, i1, o0, o1;
  mb_status st;
  // input rows of ld_in complex samples, 4 bytes each
  if ((st = plane_span(d_in, ld_in, nchans, nsamps, 4, "input", i0, i1)) != MB_OK) return st;
  if ((st = plane_span(d_out, ld_out, nchans, nsamps, 4, "output", o0, o1)) != MB_OK) return st;
  if (i0 < o1 && o0 < i1) return fail(MB_EINVAL, "output must not overlap the input");
  HIP_TRY(launch_power(d_in, ld_in, nchans, nsamps, d_out, ld_out, static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status mulaw_encode(const float* d_in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                       uint8_t* d_codes, int64_t ld_codes, float* d_xmax, void* stream) {
  mb_status st = mulaw_check(nrows, ncols, mu);
  if (st != MB_OK) return st;
  if (nrows == 0) return ok();
  if (!d_xmax) return fail(MB_EINVAL, "xmax must not be NULL");
  uintptr_t i0 = 0, i1 = 0, c0 = 0, c1 = 0;
  if (ncols > 0) {
    if ((st = plane_span(d_in, ld_in, nrows, ncols, 4, "input", i0, i1)) != MB_OK) return st;
    if ((st = plane_span(d_codes, ld_codes, nrows, ncols, 1, "codes", c0, c1)) != MB_OK) return st;
    if (i0 < c1 && c0 < i1) return fail(MB_EINVAL, "codes must not overlap the input");
  }
  HIP_TRY(launch_mulaw_encode(d_in, ld_in, nrows, ncols, mu, d_codes, ld_codes, d_xmax,
                              static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status mulaw_decode(const uint8_t* d_codes, int64_t ld_codes, const float* d_xmax, int32_t nrows,
                       int64_t ncols, float mu, float* d_out, int64_t ld_out, void* stream) {
  mb_status st = mulaw_check(nrows, ncols, mu);
  if (st != MB_OK) return st;
  if (nrows == 0 || ncols == 0) return ok();
  if (!d_xmax) return fail(MB_EINVAL, "xmax must not be NULL");
  uintptr_t c0, c1, o0, o1;
  if ((st = plane_span(d_codes, ld_codes, nrows, ncols, 1, "codes", c0, c1)) != MB_OK) return st;
  if ((st = plane_span(d_out, ld_out, nrows, ncols, 4, "output", o0, o1)) != MB_OK) return st;
  if (c0 < o1 && o0 < c1) return fail(MB_EINVAL, "output must not overlap the codes");
  HIP_TRY(launch_mulaw_decode(d_codes, ld_codes, d_xmax, nrows, ncols, mu, d_out, ld_out,
                              static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status mulaw_encode_complex(const int16_t* d_in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                               uint8_t* d_codes, int64_t ld_codes, int32_t* d_xmax, void* stream) {
  mb_status st = mulaw_check(nrows, ncols, mu);
  if (st != MB_OK) return st;
  if (nrows == 0) return ok();
  if (!d_xmax) return fail(MB_EINVAL, "xmax must not be NULL");
  uintptr_t i0 = 0, i1 = 0, c0 = 0, c1 = 0;
  if (ncols > 0) {
    if ((st = plane_span(d_in, ld_in, nrows, ncols, 4, "input", i0, i1)) != MB_OK) return st;
    if ((st = plane_span(d_codes, ld_codes, nrows, ncols, 1, "codes", c0, c1)) != MB_OK) return st;
    if (i0 < c1 && c0 < i1) return fail(MB_EINVAL, "codes must not overlap the input");
  }
  HIP_TRY(launch_mulaw_encode_complex(d_in, ld_in, nrows, ncols, mu, d_codes, ld_codes, d_xmax,
                                      static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status mulaw_decode_complex(const uint8_t* d_codes, int64_t ld_codes, const int32_t* d_xmax, int32_t nrows,
                               int64_t ncols, float mu, float* d_out, int64_t ld_out, void* stream) {
  mb_status st = mulaw_check(nrows, ncols, mu);
  if (st != MB_OK) return st;
  if (nrows == 0 || ncols == 0) return ok();
  if (!d_xmax) return fail(MB_EINVAL, "xmax must not be NULL");
  uintptr_t c0, c1, o0, o1;
  if ((st = plane_span(d_codes, ld_codes, nrows, ncols, 1, "codes", c0, c1)) != MB_OK) return st;
  if ((st = plane_span(d_out, ld_out, nrows, ncols, 8, "output", o0, o1)) != MB_OK) return st;
  if (c0 < o1 && o0 < c1) return fail(MB_EINVAL, "output must not overlap the codes");
  HIP_TRY(launch_mulaw_decode_complex(d_codes, ld_codes, d_xmax, nrows, ncols, mu, d_out, ld_out,
                                      static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status cluster_workspace_size(int64_t n, int32_t ndms, size_t* bytes) {
  if (!bytes) return fail(MB_EINVAL, "bytes must not be NULL");
  if (n < 0 || n > 2147483647 - 1024) return fail(MB_EINVAL, "n must be in [0, 2^31 - 1024)");
  if (ndms < 1 || ndms > kMaxDms) return fail(MB_EINVAL, "ndms must be in [1, %d]", kMaxDms);
  *bytes = cluster_work_bytes(n, ndms);
  return ok();
}

mb_status cluster_candidates(const mb_candidate* d_cands, int64_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps,
                             float snr_eps, int32_t min_pts, int32_t* d_labels, int32_t* d_nclusters, void* d_work,
                             size_t work_bytes, void* stream) {
  size_t need = 0;
  mb_status st = cluster_workspace_size(n, ndms, &need);
  if (st != MB_OK) return st;
  if (t_eps < 0 || t_eps > (int64_t(1) << 40)) return fail(MB_EINVAL, "t_eps must be in [0, 2^40]");
  if (dm_eps < 0 || dm_eps > kMaxDms) return fail(MB_EINVAL, "dm_eps must be in [0, %d]", kMaxDms);
  if (!(snr_eps >= 0.0f) || !isfinite(snr_eps)) return fail(MB_EINVAL, "snr_eps must be finite and >= 0");
  if (min_pts < 1) return fail(MB_EINVAL, "min_pts must be >= 1");
  if (!d_nclusters || !d_work) return fail(MB_EINVAL, "nclusters and work must not be NULL");
  if (n > 0 && (!d_cands || !d_labels)) return fail(MB_EINVAL, "candidates and labels must not be NULL");
  if (work_bytes < need) return fail(MB_EINVAL, "work is %zu bytes, %zu needed", work_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0) return fail(MB_EINVAL, "work must be 256-byte aligned");
  const uintptr_t w0 = reinterpret_cast<uintptr_t>(d_work), w1 = w0 + need;
  const uintptr_t l0 = reinterpret_cast<uintptr_t>(d_labels), l1 = l0 + 4 * (size_t)n;
  const uintptr_t c0 = reinterpret_cast<uintptr_t>(d_cands), c1 = c0 + sizeof(mb_candidate) * (size_t)n;
  if (n > 0 && ((l0 < w1 && w0 < l1) || (l0 < c1 && c0 < l1) || (c0 < w1 && w0 < c1)))
    return fail(MB_EINVAL, "candidates, labels and work must not overlap");
  HIP_TRY(launch_cluster(reinterpret_cast<const CandDev*>(d_cands), (int32_t)n, ndms, t_eps, dm_eps, snr_eps, min_pts,
                         d_labels, d_nclusters, d_work, static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status fdbscan_workspace_size(int64_t n, int32_t ndms, size_t* bytes) {
  if (!bytes) return fail(MB_EINVAL, "bytes must not be NULL");
  if (n < 0 || n > 2147483647 - 1024) return fail(MB_EINVAL, "n must be in [0, 2^31 - 1024)");
  if (ndms < 1 || ndms > kMaxDms) return fail(MB_EINVAL, "ndms must be in [1, %d]", kMaxDms);
  *bytes = fdbscan_work_bytes(n, ndms);
  return ok();
}

mb_status fdbscan_candidates(const mb_candidate* d_cands, int64_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps,
                             float snr_eps, int32_t min_pts, int32_t* d_labels, int32_t* d_nclusters,
                             int64_t* d_nqueries, void* d_work, size_t work_bytes, void* stream) {
  size_t need = 0;
  mb_status st = fdbscan_workspace_size(n, ndms, &need);
  if (st != MB_OK) return st;
  if (t_eps < 0 || t_eps > 2147483647) return fail(MB_EINVAL, "t_eps must be in [0, 2^31)");
  if (dm_eps < 0 || dm_eps > kMaxDms) return fail(MB_EINVAL, "dm_eps must be in [0, %d]", kMaxDms);
  if (!(snr_eps >= 0.0f) || !isfinite(snr_eps)) return fail(MB_EINVAL, "snr_eps must be finite and >= 0");
  if (min_pts < 1) return fail(MB_EINVAL, "min_pts must be >= 1");
  if (!d_nclusters || !d_work) return fail(MB_EINVAL, "nclusters and work must not be NULL");
  if (n > 0 && (!d_cands || !d_labels)) return fail(MB_EINVAL, "candidates and labels must not be NULL");
  if (work_bytes < need) return fail(MB_EINVAL, "work is %zu bytes, %zu needed", work_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0) return fail(MB_EINVAL, "work must be 256-byte aligned");
  if (d_nqueries && reinterpret_cast<uintptr_t>(d_nqueries) % 8 != 0)
    return fail(MB_EINVAL, "nqueries must be 8-byte aligned");
  const uintptr_t w0 = reinterpret_cast<uintptr_t>(d_work), w1 = w0 + need;
  const uintptr_t l0 = reinterpret_cast<uintptr_t>(d_labels), l1 = l0 + 4 * (size_t)n;
  const uintptr_t c0 = reinterpret_cast<uintptr_t>(d_cands), c1 = c0 + sizeof(mb_candidate) * (size_t)n;
  if (n > 0 && ((l0 < w1 && w0 < l1) || (l0 < c1 && c0 < l1) || (c0 < w1 && w0 < c1)))
    return fail(MB_EINVAL, "candidates, labels and work must not overlap");
  HIP_TRY(launch_fdbscan(reinterpret_cast<const CandDev*>(d_cands), (int32_t)n, ndms, t_eps, dm_eps, snr_eps,
                         min_pts, d_labels, d_nclusters, d_nqueries, d_work, static_cast<hipStream_t>(stream)));
  return ok();
}

// Defined with the clustering kernels (cluster.hip).
extern "C++" {
namespace mbtp {
hipError_t launch_classify(const CandDev* c, const int32_t* labels, int32_t n, int32_t nclusters, int32_t ndms,
                           double dm_start, double dm_step, double tsamp_s, double bw_mhz, double f_ghz, int32_t k,
                           double rmse_max, double dm_min, void* info, hipStream_t s);
}
}

mb_status classify_clusters(const mb_candidate* d_cands, const int32_t* d_labels, int64_t n, int32_t nclusters,
                            int32_t ndms, double dm_start, double dm_step, double tsamp_s, double bw_mhz,
                            double f_ghz, int32_t k, double rmse_max, double dm_min, mb_cluster_info* d_info,
                            void* stream) {
  static_assert(sizeof(mb_cluster_info) == 48, "cluster record layout");
  if (n < 0 || n > 2147483647 - 1024) return fail(MB_EINVAL, "n must be in [0, 2^31 - 1024)");
  if (nclusters < 0) return fail(MB_EINVAL, "nclusters must be >= 0");
  if (ndms < 1 || ndms > kMaxClassifyDms) return fail(MB_EINVAL, "ndms must be in [1, %d]", kMaxClassifyDms);
  if (k < 1 || k % 2 == 0) return fail(MB_EINVAL, "k must be odd and >= 1");
  if (!(tsamp_s > 0.0) || !(bw_mhz > 0.0) || !(f_ghz > 0.0) || !isfinite(tsamp_s) || !isfinite(bw_mhz) ||
      !isfinite(f_ghz) || !isfinite(dm_start) || !isfinite(dm_step) || !isfinite(dm_min) || std::isnan(rmse_max))
    return fail(MB_EINVAL, "tsamp, bandwidth and frequency must be finite and > 0; DM values finite");
  if (nclusters == 0) return ok();
  if (!d_info || (n > 0 && (!d_cands || !d_labels))) return fail(MB_EINVAL, "buffers must not be NULL");
  HIP_TRY(mbtp::launch_classify(reinterpret_cast<const CandDev*>(d_cands), d_labels, (int32_t)n, nclusters, ndms, dm_start,
                          dm_step, tsamp_s, bw_mhz, f_ghz, k, rmse_max, dm_min, d_info,
                          static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status detect_workspace_size(const mb_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MB_EINVAL, "plan and bytes must not be NULL");
  *bytes = detect_work_bytes(plan->desc.ndms);
  return ok();
}

mb_status detect_candidates(const mb_plan* plan, const float* d_out, int64_t nout, int64_t ld_out,
                            const mb_norm* d_norm, int64_t sample0, const int64_t* d_sample0,
                            double nsigma, mb_candidate* d_cands, int64_t capacity, int64_t* d_count,
                            mb_peak* d_peaks, void* d_work, size_t work_bytes, void* stream) {
  mb_status st = validate_detect(plan, d_out, nout, ld_out, d_norm, sample0, nsigma, d_cands, capacity, d_count);
  if (st) return st;
  const size_t need = detect_work_bytes(plan->desc.ndms);
  if (!d_work || work_bytes < need || !check_aligned(d_work, 256))
    return fail(MB_EINVAL, "workspace must be 256-byte aligned with at least %zu bytes", need);
  HIP_TRY(launch_detect(d_out, ld_out, nout, plan->desc.ndms, reinterpret_cast<const NormDev*>(d_norm),
                        sample0, d_sample0, nsigma, plan->desc.dm_start, plan->desc.dm_step,
                        reinterpret_cast<CandDev*>(d_cands), capacity, d_count,
                        reinterpret_cast<PeakDev*>(d_peaks), d_work, static_cast<hipStream_t>(stream)));
  return ok();
}

mb_status detect_candidates_noalloc(const mb_plan* plan, const float* d_out, int64_t nout, int64_t ld_out,
                                    const mb_norm* d_norm, int64_t sample0, const int64_t* d_sample0,
                                    double nsigma, mb_candidate* d_cands, int64_t capacity, int64_t* d_count,
                                    mb_peak* d_peaks, void* stream) {
  mb_status st = validate_detect(plan, d_out, nout, ld_out, d_norm, sample0, nsigma, d_cands, capacity, d_count);
  if (st) return st;
  if (plan->desc.ndms > MB_DETECT_NOALLOC_MAX_DMS)
    return fail(MB_EINVAL, "detect_candidates_noalloc takes at most %d DMs (plan has %d)",
                MB_DETECT_NOALLOC_MAX_DMS, plan->desc.ndms);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device)
    return fail(MB_EINVAL, "current device %d is not the plan's device %d", dev, plan->device);
  HIP_TRY(launch_detect_noalloc(d_out, ld_out, nout, plan->desc.ndms, reinterpret_cast<const NormDev*>(d_norm),
                                sample0, d_sample0, nsigma, plan->desc.dm_start, plan->desc.dm_step,
                                reinterpret_cast<CandDev*>(d_cands), capacity, d_count,
                                reinterpret_cast<PeakDev*>(d_peaks), static_cast<hipStream_t>(stream)));
  return ok();
}

struct mb_step_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct Item { mb_beam* beam; int64_t nsamps, nout, sample0; int32_t integer_kernel; };
  std::vector<Item> items;
};

mb_status dedisp_step_graph_create(const mb_step_item* items, int32_t nitems, void* d_batch_work,
                                   size_t batch_work_bytes, void* stream, mb_step_graph** out) {
  if (!out) return fail(MB_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (!items || nitems < 1 || nitems > 64) return fail(MB_EINVAL, "nitems must be in 1..64");
  if (!stream) return fail(MB_EINVAL, "the null stream cannot be captured; pass a stream");
  const bool batch = nitems > 1 || d_batch_work != nullptr;
  for (int32_t i = 0; i < nitems; ++i) {
    const mb_step_item& it = items[i];
    if (!it.plan) return fail(MB_EINVAL, "item %d: plan is NULL", i);
    if (!it.d_norm) return fail(MB_EINVAL, "item %d: the step needs d_norm", i);
    if (it.beam) {
      if (it.beam->plan != it.plan) return fail(MB_EINVAL, "item %d: beam was created from another plan", i);
      if (it.beam->seen < it.beam->R)
        return fail(MB_EINVAL, "item %d: the beam is not in steady state (%lld of %lld ring samples seen)", i,
                    (long long)it.beam->seen, (long long)it.beam->R);
      for (int32_t k = 0; k < i; ++k)
        if (items[k].beam == it.beam) return fail(MB_EINVAL, "items %d and %d share a beam", k, i);
    }
  }
  mb_step_graph* g = new (std::nothrow) mb_step_graph;
  if (!g) return fail(MB_ENOMEM, "host allocation failed");
  g->items.resize(nitems);
  std::vector<int64_t> seen(nitems);
  for (int32_t i = 0; i < nitems; ++i) seen[i] = items[i].beam ? items[i].beam->seen : 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    return fail(MB_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  mb_status st = MB_OK;
  std::string why;
  std::vector<mb_exec_info> infos(nitems);
  for (int32_t i = 0; i < nitems && st == MB_OK; ++i) {
    const mb_step_item& it = items[i];
    if (it.d_rfi_state)
      st = rfi_threshold(it.plan, it.d_in, it.nsamps, it.ld, it.d_rfi_state, it.rfi_state_bytes, stream);
  }
  if (st == MB_OK) {
    if (!batch) {
      const mb_step_item& it = items[0];
      st = dedisp_execute(it.plan, it.beam, it.d_in, it.nsamps, it.ld, it.d_rfi_state, it.d_out, it.ld_out,
                          it.d_norm, &infos[0], stream);
    } else {
      std::vector<mb_batch_item> bi(nitems);
      for (int32_t i = 0; i < nitems; ++i) {
        const mb_step_item& it = items[i];
        bi[i] = mb_batch_item{it.plan, it.beam, it.d_in, it.nsamps, it.ld, it.d_rfi_state, it.d_out, it.ld_out,
                              it.d_norm};
      }
      st = dedisp_execute_batch(bi.data(), nitems, d_batch_work, batch_work_bytes, infos.data(), stream);
    }
  }
  for (int32_t i = 0; i < nitems && st == MB_OK; ++i) {
    const mb_step_item& it = items[i];
    const int64_t* d_s0 = it.beam ? it.beam->d_seen + 1 : nullptr;
    st = detect_candidates(it.plan, it.d_out, infos[i].nout, it.ld_out, it.d_norm, it.beam ? 0 : infos[i].sample0,
                           d_s0, it.nsigma, it.d_cands, it.capacity, it.d_count, it.d_peaks, it.d_detect_work,
                           it.detect_work_bytes, stream);
  }
  if (st != MB_OK) why = g_err;
  // the captured calls advanced the host counts of the beams; nothing ran
  for (int32_t i = 0; i < nitems; ++i)
    if (items[i].beam) items[i].beam->seen = seen[i];
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (st != MB_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    delete g;
    if (st != MB_OK) return fail(st, "capturing the step: %s", why.c_str());
    return fail(MB_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(MB_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  g->graph = graph;
  for (int32_t i = 0; i < nitems; ++i)
    g->items[i] = mb_step_graph::Item{items[i].beam, items[i].nsamps, infos[i].nout, infos[i].sample0,
                                      infos[i].integer_kernel};
  *out = g;
  return ok();
}

mb_status dedisp_step_graph_launch(mb_step_graph* graph, void* stream, mb_exec_info* infos) {
  if (!graph) return fail(MB_EINVAL, "graph is NULL");
  HIP_TRY(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
  for (size_t i = 0; i < graph->items.size(); ++i) {
    mb_step_graph::Item& it = graph->items[i];
    int64_t s0 = it.sample0;
    if (it.beam) {
      // steady state: the first output lies s_max samples before the chunk
      s0 = it.beam->base + it.beam->seen - it.beam->plan->smax;
      it.beam->seen += it.nsamps;
    }
    if (infos) infos[i] = mb_exec_info{it.nout, s0, it.integer_kernel, 0};
  }
  return ok();
}

mb_status dedisp_step_graph_destroy(mb_step_graph* graph) {
  if (!graph) return ok();
  // a launch may still be running on some stream: let it finish first
  hipError_t e = hipDeviceSynchronize();
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  if (e != hipSuccess) return fail(MB_EDEVICE, "hipDeviceSynchronize: %s", hipGetErrorString(e));
  return ok();
}

}  // extern "C"
