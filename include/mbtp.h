/*
 * mbtp.h - C ABI of the MI355X multibeam transient hot path.
 *
 * One beam's channelised power (beam/channel/time order, Sec. 2.1) passes
 * through the thresholding RFI pass (Sec. 2.2.1), brute-force incoherent
 * dedispersion over a grid of trial DMs with the integer cold-plasma delays
 * of Eq. (1) (Sec. 2.2.2), per-DM detrending and normalisation
 * (Sec. 2.2.3) and the n-sigma event threshold that yields
 * (time, DM, intensity) triplets (Sec. 2.3).
 *
 * Conventions shared by every call:
 *  - Device pointers ("d_" prefix) are HIP device memory owned by the
 *    caller.  Host pointers ("h_" prefix or plain structs) are host memory.
 *    The library allocates device memory only inside *_create calls and
 *    frees it in the matching *_destroy.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call that takes a stream only enqueues work on it and returns;
 *    results are valid once the stream has reached that point.  Calls on
 *    one plan from several streams are safe: a plan is immutable after
 *    creation.  A beam (streaming state) or an RFI state buffer must be used
 *    by one stream at a time.
 *  - Filterbanks are x[c][t]: channel c's samples are contiguous in time,
 *    row c starts at element c*ld.  The device pointer must be 16-byte
 *    aligned and ld a multiple of 4 elements, and the buffer must hold
 *    nchans*ld elements: kernels read whole aligned groups of 4 samples, so
 *    when nsamps is not a multiple of 4 the last group of a row reaches into
 *    the row's padding (those values are never used).
 *  - Every call validates its arguments before enqueuing anything; on an
 *    error nothing is enqueued, the call returns a non-zero mb_status and
 *    mb_last_error() (per thread) describes it.  No C++ exception crosses
 *    this interface.
 *  - The plan, its delay table and all launches use the HIP device that is
 *    current when dedisp_plan_create is called; later calls must be made
 *    with that device current.
 */
#ifndef MBTP_H
#define MBTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mb_status;
enum {
  MB_OK = 0,
  MB_EINVAL = 1,     /* invalid argument or shape; nothing was enqueued   */
  MB_ENOMEM = 2,     /* a create call could not allocate device memory    */
  MB_EDEVICE = 3,    /* a HIP runtime call failed                          */
  MB_ECAPACITY = 4,  /* more results than the caller's buffer holds        */
  MB_EBUSY = 5       /* resource in use                                    */
};

/* Storage type of filterbank samples.  All are widened exactly to FP32 and
 * accumulated in FP32 (u8: 0..255; f16: IEEE binary16; f32: binary32). */
typedef int32_t mb_dtype;
enum { MB_U8 = 0, MB_F16 = 1, MB_F32 = 2 };

/* Factors of the thresholding RFI pass (Sec. 2.2.1).  Defaults in
 * brackets; mb_rfi_defaults() fills them. */
typedef struct {
  int32_t poly_order;   /* p of the bandpass polynomial, 0..8 [3]           */
  int32_t window;       /* W_c, chunk width in samples, power of 2 >= 256 [256] */
  double k_mask;        /* channel masking factor x RMSE of the fit [5]      */
  double k_chan;        /* chunk-mean threshold in noise stds [5]            */
  double k_spec;        /* spectrum-mean threshold in noise stds [5]         */
  int32_t mask_passes;  /* most fit-and-mask rounds, 1..16 [8]; rounds stop
                           early once one masks no new channel              */
  int32_t reserved;     /* must be 0                                         */
} mb_rfi_params;

/* Observing and survey parameters of one beam (Sec. 1.1, Sec. 2.2.2) and
 * the factors of its RFI pass (Sec. 2.2.1), like the paper's one
 * configuration file for all operating parameters.
 * Channel c has centre frequency f_ch0_mhz + c*df_mhz (df may be negative).
 * Trial DM d is dm_start + d*dm_step (pc cm^-3), d = 0..ndms-1. */
typedef struct {
  int32_t nchans;      /* C, 1..65535                                      */
  int32_t ndms;        /* 1..65535                                         */
  double f_ch0_mhz;    /* > 0                                              */
  double df_mhz;       /* != 0, all channel centres > 0                    */
  double tsamp_s;      /* sampling time > 0                                */
  double dm_start;     /* >= 0                                             */
  double dm_step;      /* >= 0                                             */
  mb_dtype in_dtype;   /* storage type of the filterbanks executed        */
  int32_t tile_hint;   /* 0: library's choice; k > 0: k-th compiled
                          dedispersion tiling (results do not depend on it) */
  mb_rfi_params rfi;   /* used by rfi_threshold                           */
} mb_plan_desc;

typedef struct {
  int32_t nchans, ndms;
  int32_t max_delay;    /* s_max: largest entry of the delay table        */
  int32_t dm_block;     /* DMs per dedispersion workgroup (tiling info)   */
  int32_t time_tile;    /* output samples per dedispersion workgroup      */
  int32_t chan_block;   /* channels per LDS stage                         */
  int32_t tile_index;   /* 1-based index of the compiled tiling in use    */
  int32_t waves;        /* wave64s per dedispersion workgroup             */
  int64_t lds_bytes;    /* LDS per dedispersion workgroup                 */
  int32_t u8_integer;   /* 1: 8-bit chunks without cleaning can run on the
                           exact integer kernel (see dedisp_execute)       */
  int32_t reserved;
} mb_plan_info;

/* Summary of one RFI pass, read back with rfi_report(). */
typedef struct {
  double sigma;           /* per-sample noise std implied by the fit RMSE    */
  double rmse0;           /* RMSE of the first fit (masking criterion)       */
  double rmse;            /* RMSE of the final fit                           */
  double sum_fit;         /* sum over channels of the fitted bandpass        */
  int64_t n_masked;       /* channels replaced by their neighbours' mean     */
  int64_t n_chunk_flags;  /* chunks over threshold                           */
  int64_t n_chunk_flags_ext; /* after extension to time-adjacent chunks      */
  int64_t n_spectrum_flags;  /* spectra over threshold                       */
  int64_t nsamps, nchunks;
  int32_t error;          /* 0, or 1 when every channel got masked (then no
                             sample is flagged and the fit is not usable)    */
  int32_t reserved;
} mb_rfi_report;

/* Byte offsets of the arrays inside an RFI state buffer (for inspection). */
typedef struct {
  size_t total_bytes;
  size_t fit_f64;          /* f[C], fitted bandpass (FP64)                  */
  size_t bandpass_f64;     /* B[C], time-averaged bandpass (FP64)           */
  size_t chunk_sum_f64;    /* M[C][J], sum of raw samples per chunk (FP64)  */
  size_t chunk_flags_u8;   /* [C][J]: bit0 chunk over threshold, bit1 after
                              extension to time-adjacent chunks             */
  size_t spectrum_flags_u8;/* [T]: 1 where the spectrum was flagged         */
  size_t masked_u8;        /* [C]: 1 where the channel was interpolated     */
  int64_t nchunks;         /* J = ceil(T / W_c)                             */
} mb_rfi_layout;

/* Per-DM detrend line and scale (Sec. 2.2.3): for output sample t' of this
 * block (0-based), z = (D[t'] - a - b*t') / sigma.  degenerate != 0 when
 * sigma <= 1e-9 * rms(D) (e.g. an exactly linear series); then z = 0. */
typedef struct {
  double a, b, sigma;
  int32_t degenerate;
  int32_t reserved;
} mb_norm;

/* One (time, DM, intensity) triplet (Sec. 2.3). */
typedef struct {
  int32_t dm_index;
  int32_t reserved;
  int64_t sample;   /* absolute sample index of the dedispersed series   */
  float snr;        /* z, the normalised intensity                       */
  float dm;         /* trial DM value, pc cm^-3                          */
} mb_candidate;

/* Largest z of one DM row (earliest sample on ties). */
typedef struct {
  int64_t sample;
  float snr;
  int32_t reserved;
} mb_peak;

/* Streaming position of a beam after an execute (host-known). */
typedef struct {
  int64_t nout;      /* dedispersed samples produced per DM by this call   */
  int64_t sample0;   /* absolute index of the first of them                */
  int32_t integer_kernel; /* 1 when the exact integer kernel dedispersed it */
  int32_t reserved;
} mb_exec_info;

typedef struct mb_plan mb_plan;
typedef struct mb_beam mb_beam;

/* ---- plan ------------------------------------------------------------- */

/* Builds the integer delay table of Eq. (1) on the host in FP64,
 *   s[d][c] = floor(4150 * DM_d * (f_c^-2 - f_ref^-2) / tsamp + 1/2),
 * 4150 s MHz^2 being the paper's 4.15e6 ms and f_ref the highest channel
 * centre, copies it to the current device and picks the dedispersion
 * tiling.  *out receives a plan to release with dedisp_plan_destroy.
 * Errors: MB_EINVAL (bad descriptor), MB_ENOMEM, MB_EDEVICE. */
mb_status dedisp_plan_create(const mb_plan_desc* desc, mb_plan** out);
mb_status dedisp_plan_destroy(mb_plan* plan);
mb_status dedisp_plan_info(const mb_plan* plan, mb_plan_info* info);
/* Copies the delay table, int32 [ndms][nchans] row-major, to host memory. */
mb_status dedisp_plan_delays(const mb_plan* plan, int32_t* h_delays);
/* Number of compiled dedispersion tilings; valid tile_hint values are
 * 1..count.  Host only, no device call.  EINVAL if count is NULL. */
mb_status dedisp_tilings(int32_t* count);

/* ---- RFI thresholding (Sec. 2.2.1) ------------------------------------ */

void mb_rfi_defaults(mb_rfi_params* p);

/* Size and layout of the caller-owned device buffer that holds one RFI
 * pass's statistics, fitted bandpass and flags for nsamps samples.  The
 * size never decreases with nsamps, so a buffer sized for the longest chunk
 * serves every shorter chunk of the same plan. */
mb_status rfi_state_layout(const mb_plan* plan, int64_t nsamps, mb_rfi_layout* layout);

/* Runs the three stages of Sec. 2.2.1, with the plan's RFI factors, on d_in
 * (plan's in_dtype, [C][nsamps] with leading dimension ld): per-channel and per-chunk sums and per-sample
 * spectrum sums in one HBM pass (FP64 accumulation), the bandpass fit with
 * channel masking on one workgroup, chunk flags with extension to the
 * adjacent chunks, and spectrum flags.  Masking: the time-averaged bandpass
 * is fitted, channels whose residual exceeds k_mask times the fit's RMSE are
 * masked (replaced by the mean of their nearest unmasked neighbours) and the
 * round repeats on the interpolated bandpass until a round masks no new
 * channel or mask_passes rounds have run (a bright channel can hide a fainter
 * one in the first RMSE); the last fit is the bandpass the pass subtracts.  The input is not modified; the
 * cleaning is applied on the fly by dedisp_execute.  d_state must be at
 * least layout.total_bytes and 256-byte aligned; its previous contents are
 * overwritten.  Errors: MB_EINVAL (shape, params, small state buffer). */
mb_status rfi_threshold(const mb_plan* plan, const void* d_in, int64_t nsamps,
                        int64_t ld, void* d_state, size_t state_bytes, void* stream);

/* Waits for the stream and copies the pass summary to *h_report. */
mb_status rfi_report(const mb_plan* plan, const void* d_state, mb_rfi_report* h_report,
                     void* stream);

/* ---- dedispersion (Sec. 2.2.2) + normalisation (Sec. 2.2.3) ------------ */

/* Dedisperses d_in into d_out (FP32, [ndms][ld_out]):
 *   D[d][t] = sum_c y[c][t + s[d][c]],
 * y being the stored sample widened to FP32, or, when d_rfi_state is not
 * NULL (the state rfi_threshold wrote for this same d_in and nsamps), the
 * sample minus the fitted bandpass f_c rounded to FP32, or 0 where its chunk
 * or spectrum was flagged.
 * Sums are FP32, channels accumulated in ascending order in blocks of 32
 * (a fixed order, so results do not depend on the tiling).  8-bit samples
 * without cleaning sum to integers below 2^24, which FP32 holds exactly:
 * such a chunk's outputs are the exact sums, whatever the tiling.  For an
 * 8-bit chunk without cleaning, longer than s_max, whose rows start 8-byte
 * aligned with ld a multiple of 8, the outputs that read only the chunk's
 * own samples run on an integer kernel (16-bit partial sums) that gives
 * these same bits faster; info->integer_kernel reports it.
 *
 * beam == NULL: single shot over nsamps samples; nout = nsamps - s_max
 * outputs per DM (MB_EINVAL if nsamps <= s_max).
 * beam != NULL: the chunk continues the beam's stream; nsamps must be a
 * multiple of 4 (MB_EINVAL otherwise).  The beam keeps the last s_max
 * cleaned samples of every channel on the device, so the chunk
 * yields nout = min(seen, s_max) + nsamps - s_max outputs (0 until s_max
 * samples have been seen), starting at absolute sample
 * max(0, seen - s_max), "seen" counting the samples before this chunk.
 *
 * d_in holds C rows ld samples apart (ld >= nsamps, a multiple of 4, the
 * pointer 16-byte aligned).  The kernels load aligned groups of 4 samples
 * (8 on the integer kernel) whole, so every row must be readable up to
 * sample min(ld, nsamps rounded up to a multiple of 8); samples past nsamps
 * enter no sum.
 *
 * d_norm (nullable, [ndms]) receives each DM's detrend line and scale over
 * the outputs of this call (Sec. 2.2.3).  info (nullable, host) receives
 * nout and sample0.  d_out must be 16-byte aligned with ld_out >= nout a
 * multiple of 4, and hold ndms*ld_out floats (the normalisation and
 * detection read rows in aligned groups of 4).  Errors: MB_EINVAL. */
mb_status dedisp_execute(const mb_plan* plan, mb_beam* beam, const void* d_in,
                         int64_t nsamps, int64_t ld, const void* d_rfi_state,
                         float* d_out, int64_t ld_out, mb_norm* d_norm,
                         mb_exec_info* info, void* stream);

/* Detrend line and scale of every row of a dedispersed plane (Sec. 2.2.3),
 * exactly as dedisp_execute forms them: d_out [ndms][ld_out] FP32 with nout
 * samples per row (16-byte aligned, ld_out % 4 == 0), d_norm [ndms]. */
mb_status dedisp_normalise(const mb_plan* plan, const float* d_out, int64_t nout,
                           int64_t ld_out, mb_norm* d_norm, void* stream);

/* Windowed median filter of a dedispersed plane (Sec. 2.2.3, Eq. 2): every
 * sample of every row becomes the median of the 2*half_width + 1 samples
 * centred on it; beyond a row's ends the end sample repeats, so every window
 * has an odd count and the result is one of its samples (bit-exact against
 * any correct median).  The filter sees only the samples of this call.
 * d_in [nrows][ld_in] and d_out [nrows][ld_out] are FP32 device planes with
 * ncols samples per row (ld_in, ld_out >= ncols); the caller owns both, and
 * d_out must not overlap d_in.  half_width 0..16 (0 copies the plane).
 * Asynchronous on stream.  Errors: MB_EINVAL for negative sizes, a
 * half_width out of range, NULL planes, a leading dimension below ncols,
 * overlapping planes or a plane beyond one launch (nothing is enqueued). */
mb_status median_filter(const float* d_in, int64_t ld_in, float* d_out, int64_t ld_out,
                        int32_t nrows, int64_t ncols, int32_t half_width, void* stream);

/* Channelised power of beamformed voltages (Sec. 2.2): d_in holds a
 * beam's 16-bit complex samples in channel/time order (Sec. 2.1), channel
 * row c at d_in + 2*c*ld_in, each sample a (re, im) pair of int16 (ld_in >=
 * nsamps, in complex samples); d_out [nchans][ld_out] FP32 (ld_out >=
 * nsamps) receives re^2 + im^2, exact in integers and rounded once to FP32:
 * the filterbank layout rfi_threshold and dedisp_execute read.  Device
 * planes owned by the caller; the output must not overlap the input.
 * Asynchronous on stream.  Errors: MB_EINVAL for negative sizes, NULL or
 * overlapping planes, a leading dimension below the row length, or a plane
 * beyond one launch. */
mb_status power_from_voltages(const int16_t* d_in, int64_t ld_in, int32_t nchans, int64_t nsamps,
                              float* d_out, int64_t ld_out, void* stream);

/* mu-law codec of the data writer (Sec. 2.4, Eq. 5) for FP32 power planes.
 * mulaw_encode: for every row of d_in [nrows][ld_in] (ncols samples, ld_in
 * >= ncols) X = the row's largest |x| goes to d_xmax[row], and every sample
 * to the 8-bit code q = floor(255 * log1p(mu * x / X) / log1p(mu) + 1/2)
 * in d_codes [nrows][ld_codes] (x < 0 counts as 0; a row of zeros gives
 * X = 0 and codes 0).  The code is the number of level boundaries
 * X/mu * expm1((k - 1/2)/255 * log1p(mu)), k = 1..255, formed in FP64, that
 * x reaches.  mulaw_decode: x = X / mu * expm1(q / 255 * log1p(mu)), FP64,
 * rounded to FP32, into d_out [nrows][ld_out].  mu finite and > 0 (255 as
 * in G.711).  Device planes owned by the caller; outputs must not overlap
 * inputs.  Asynchronous on stream.  Errors: MB_EINVAL for negative sizes,
 * a bad mu, NULL or overlapping planes, a leading dimension below ncols or a
 * plane beyond one launch (nothing is enqueued). */
mb_status mulaw_encode(const float* d_in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                       uint8_t* d_codes, int64_t ld_codes, float* d_xmax, void* stream);
mb_status mulaw_decode(const uint8_t* d_codes, int64_t ld_codes, const float* d_xmax, int32_t nrows,
                       int64_t ncols, float mu, float* d_out, int64_t ld_out, void* stream);

/* DBSCAN clustering of detections in (time, DM, SNR) (Sec. 2.3).  d_cands:
 * n candidates in (dm_index, sample) order, as detect_candidates writes
 * them, with 0 <= dm_index < ndms (other orders give unspecified labels).
 * Candidate q is in the neighbourhood of p when |sample_q - sample_p| <=
 * t_eps, |dm_index_q - dm_index_p| <= dm_eps and |snr_q - snr_p| <= snr_eps
 * (the difference in FP32); p is in its own.  p is a core point when its
 * neighbourhood holds at least min_pts candidates.  A cluster is a maximal
 * set of core points linked through each other's neighbourhoods, plus the
 * border points they reach; a border point reached from two clusters joins
 * the one of its lowest-indexed core neighbour.  This is the exact result
 * that the paper's FDBSCAN approximates.  d_labels [n] (device) receives
 * -1 for noise and otherwise the cluster number, clusters numbered 0, 1, ...
 * in order of their lowest-indexed core point; d_nclusters (device, one
 * int32) the number of clusters.  d_work: cluster_workspace_size bytes,
 * 256-byte aligned, caller-owned.  Asynchronous on stream; the result is a
 * function of the input alone.  Errors: MB_EINVAL for n outside
 * [0, 2^31 - 1024), ndms outside 1..65535, negative or non-finite extents,
 * min_pts < 1, NULL or overlapping buffers, or a short workspace. */
mb_status cluster_workspace_size(int64_t n, int32_t ndms, size_t* bytes);
mb_status cluster_candidates(const mb_candidate* d_cands, int64_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps,
                             float snr_eps, int32_t min_pts, int32_t* d_labels, int32_t* d_nclusters,
                             void* d_work, size_t work_bytes, void* stream);

/* FDBSCAN clustering of detections as the paper runs it (Sec. 2.3), with
 * the inputs, neighbourhoods and core points of cluster_candidates.  Points
 * are visited in index order; an unclassified point that is not a core point
 * is region-queried and left unclassified; an unclassified core point starts
 * a new cluster, which every unlabelled member of its neighbourhood joins;
 * the cluster then grows only from representatives: for each dimension
 * (sample, DM index, SNR, the SNR offset in FP32) and each direction, the
 * member of the expanding point's neighbourhood lying farthest from it (the
 * lowest index among equally far ones; none where no member lies off the
 * point in that direction).  Every representative is region-queried at most
 * once; a core one adds its unlabelled neighbours to the cluster and its own
 * representatives to the seeds.  Points left unclassified are noise.  Unlike
 * cluster_candidates this can lose a border point or split a cluster that
 * is reachable only through a core point that is never a representative.
 * d_labels [n] receives -1 for noise, else the cluster number in order of
 * creation; d_nclusters (device int32) the cluster count; d_nqueries
 * (device int64, nullable, 8-byte aligned) the number of region queries.
 * d_work: fdbscan_workspace_size bytes, 256-byte aligned, caller-owned.  The
 * visiting order runs on one workgroup.  Asynchronous on stream; the result
 * is a function of the input alone.  Errors: as cluster_candidates, and
 * MB_EINVAL for t_eps >= 2^31. */
mb_status fdbscan_workspace_size(int64_t n, int32_t ndms, size_t* bytes);
mb_status fdbscan_candidates(const mb_candidate* d_cands, int64_t n, int32_t ndms, int64_t t_eps, int32_t dm_eps,
                             float snr_eps, int32_t min_pts, int32_t* d_labels, int32_t* d_nclusters,
                             int64_t* d_nqueries, void* d_work, size_t work_bytes, void* stream);

/* Per-cluster result of the DM-SNR classification. */
typedef struct {
  int32_t peak_dm_index;  /* row with the most detections (ties: larger SNR, then lower index) */
  int32_t npoints;        /* detections carrying the label                                     */
  int32_t ndm_rows;       /* DM rows holding any of them                                       */
  int32_t cls;            /* 0 candidate, 1 peak DM below dm_min (broadband RFI),
                             2 RMSE above rmse_max (RFI), 3 no detection carries the label     */
  int64_t t_first, t_last;/* first and last sample at the peak row                            */
  float peak_snr;         /* largest SNR at the peak row                                      */
  int32_t reserved;
  double rmse;            /* NaN for classes 1 and 3                                          */
} mb_cluster_info;

/* DM-SNR classification of clusters (Sec. 2.3, Eqs. 3-4), one workgroup per
 * cluster.  d_cands [n] and d_labels [n] as cluster_candidates leaves them
 * (0 <= dm_index < ndms); d_info [nclusters] receives one record per label
 * 0..nclusters-1.  Per cluster: the signature is the largest SNR of every DM
 * row holding its detections, in DM order; it is smoothed by a centred
 * k-point moving average (truncated at the ends) and divided by its value at
 * the peak row.  A peak DM (dm_start + index * dm_step) below dm_min gives
 * class 1.  Otherwise the width W = (t_last - t_first + 1) * tsamp_s and the
 * curve sqrt(pi)/2 * erf(z)/z, z = 6.91e-3 * dDM * bw_mhz / (W_ms * f_ghz^3)
 * (bw_mhz the band's width, f_ghz its centre) give the model at each row's
 * DM error from the peak; the RMSE between the two decides class 0 (at most
 * rmse_max) or 2.  Arithmetic in FP64.  Device buffers owned by the caller.
 * Asynchronous on stream.  Errors: MB_EINVAL for sizes out of range, ndms
 * above 4000, an even k, non-positive or non-finite tsamp/bandwidth/
 * frequency, or NULL buffers. */
mb_status classify_clusters(const mb_candidate* d_cands, const int32_t* d_labels, int64_t n, int32_t nclusters,
                            int32_t ndms, double dm_start, double dm_step, double tsamp_s, double bw_mhz,
                            double f_ghz, int32_t k, double rmse_max, double dm_min, mb_cluster_info* d_info,
                            void* stream);

/* 4+4-bit mu-law codec of 16-bit complex voltages (Sec. 2.4, Eq. 5), the
 * data writer's format for complex channelised series.  mulaw_encode_complex:
 * d_in holds nrows channel rows of (re, im) int16 pairs, row r at
 * d_in + 2*r*ld_in (ld_in >= ncols, both in complex samples).  Each row's
 * largest |component| X (over both parts) goes to d_xmax[r] (int32, up to
 * 32768) and each complex sample to one byte of d_codes [nrows][ld_codes]:
 * the real part's nibble in bits 0-3, the imaginary part's in bits 4-7.  A
 * nibble is the sign of x in bit 3 and, in bits 0-2, the number of level
 * boundaries X/mu * expm1((k - 1/2)/7 * log1p(mu)), k = 1..7, formed in
 * FP64, that |x| reaches (a row of zeros gives X = 0 and codes 0).
 * mulaw_decode_complex: each nibble becomes sign * X/mu * expm1(m/7 *
 * log1p(mu)), FP64 rounded to FP32, into d_out, nrows rows of ld_out
 * (re, im) FP32 pairs (ld_out >= ncols, in complex samples).  mu finite
 * and > 0.  Device planes owned by the caller; outputs must not overlap
 * inputs.  Asynchronous on stream.  Errors: MB_EINVAL for negative sizes,
 * a bad mu, NULL or overlapping planes, a leading dimension below ncols or
 * a plane beyond one launch (nothing is enqueued). */
mb_status mulaw_encode_complex(const int16_t* d_in, int64_t ld_in, int32_t nrows, int64_t ncols, float mu,
                               uint8_t* d_codes, int64_t ld_codes, int32_t* d_xmax, void* stream);
mb_status mulaw_decode_complex(const uint8_t* d_codes, int64_t ld_codes, const int32_t* d_xmax, int32_t nrows,
                               int64_t ncols, float mu, float* d_out, int64_t ld_out, void* stream);

/* ---- batched launch ------------------------------------------------------ */

/* One beam chunk of a batch: the arguments of one dedisp_execute call. */
typedef struct {
  const mb_plan* plan;
  mb_beam* beam;               /* NULL: single shot; a beam appears at most once */
  const void* d_in;
  int64_t nsamps, ld;
  const void* d_rfi_state;     /* either every item of a batch has one, or none */
  float* d_out;
  int64_t ld_out;
  mb_norm* d_norm;             /* nullable */
} mb_batch_item;

/* Bytes of caller-owned device workspace for a batch of nitems (a tile
 * counter per launch of up to 16 items). */
mb_status dedisp_batch_workspace_size(int32_t nitems, size_t* bytes);

/* Dedisperses many beams' chunks (Sec. 2, multibeam: beams are independent)
 * in one persistent launch per 16 items: workgroups take (item, DM block,
 * time tile) work from an atomic counter, heaviest channel counts first, so
 * beams with uneven channel counts, DM plans and chunk lengths share the GPU.
 * Every item gives exactly the result dedisp_execute gives it alone (same
 * summation order), including streaming beams.  All plans must share the
 * storage type and the tiling (plan_info dm_block/time_tile/chan_block, set
 * through tile_hint).  infos (nullable, host, [nitems]) receives each item's
 * nout and sample0.  d_work: dedisp_batch_workspace_size bytes, 256-byte
 * aligned.  Arguments of every item are validated before anything is
 * enqueued.  Errors: MB_EINVAL. */
mb_status dedisp_execute_batch(const mb_batch_item* items, int32_t nitems, void* d_work,
                               size_t work_bytes, mb_exec_info* infos, void* stream);

/* ---- captured chunk steps (HIP graphs) ---------------------------------- */

/* One beam's chunk step for dedisp_step_graph_create: the RFI pass (when
 * d_rfi_state is given), dedispersion with normalisation, and detection,
 * with the arguments of rfi_threshold, dedisp_execute and
 * detect_candidates.  All buffers are the caller's and must stay valid while
 * the graph exists; each launch reads the current contents of d_in. */
typedef struct {
  const mb_plan* plan;
  mb_beam* beam;              /* NULL: single shot; else in steady state     */
  const void* d_in;
  int64_t nsamps, ld;
  void* d_rfi_state;          /* NULL: no RFI pass                           */
  size_t rfi_state_bytes;
  float* d_out;
  int64_t ld_out;
  mb_norm* d_norm;            /* required                                    */
  double nsigma;
  mb_candidate* d_cands;
  int64_t capacity;
  int64_t* d_count;
  mb_peak* d_peaks;           /* nullable                                    */
  void* d_detect_work;
  size_t detect_work_bytes;
} mb_step_item;

typedef struct mb_step_graph mb_step_graph;

/* Captures the chunk step of nitems beams (1..64) into one HIP graph on
 * `stream` (not the null stream): every item's RFI pass, then one
 * dedispersion of all items (dedisp_execute for a single item without
 * d_batch_work, else dedisp_execute_batch with that workspace, Sec. 2's
 * multibeam step), then every item's detection.  Nothing runs during the
 * capture.  A streaming beam must be in steady state (it has seen at least
 * its ring length R of samples, see dedisp_beam_create) and keeps the chunk
 * length: the ring position and the detections' absolute samples are read
 * on the device at run time, so every launch processes the next chunk of
 * each beam.  The beams' host-side counts are left as they were.  Errors:
 * MB_EINVAL (arguments, a beam not in steady state; nothing captured),
 * MB_EDEVICE (capture or instantiation failed). */
mb_status dedisp_step_graph_create(const mb_step_item* items, int32_t nitems, void* d_batch_work,
                                   size_t batch_work_bytes, void* stream, mb_step_graph** out);
/* Enqueues one replay on `stream` and advances every streaming beam's
 * host-side count by its chunk length.  infos (nullable, host, [nitems])
 * receives each item's nout and the absolute index of its first output.
 * A beam must not be used by other calls between create and the last
 * launch, except through launches of this graph. */
mb_status dedisp_step_graph_launch(mb_step_graph* graph, void* stream, mb_exec_info* infos);
/* Waits for the device to be idle (a launch may still be running), then
 * frees the graph. */
mb_status dedisp_step_graph_destroy(mb_step_graph* graph);

/* ---- streaming state --------------------------------------------------- */

/* A beam's device-resident overlap ring: the last R cleaned FP32 samples of
 * every channel, R = s_max rounded up to a multiple of 4, plus the absolute
 * sample count, kept both on the host and on the device (the kernels read the
 * ring position from the device copy, so a captured steady-state chunk step,
 * fixed chunk length and seen >= R, stays correct on replay; the host copy is
 * then advanced with dedisp_beam_advance).  Allocates nchans * R * 4 + 8
 * bytes on the plan's device. */
mb_status dedisp_beam_create(const mb_plan* plan, mb_beam** out);
mb_status dedisp_beam_destroy(mb_beam* beam);
/* Forgets the stream history (the next chunk is the first, starting at
 * absolute sample 0).  Waits for the device to be idle. */
mb_status dedisp_beam_reset(mb_beam* beam);
/* Forgets the stream history without waiting: the next chunk is the first
 * of a stream whose first sample has absolute index `position` (0..2^62), so
 * after a gap in the input (dropped chunks, Sec. 3's soft-real-time policy)
 * outputs and detections keep absolute sample indices.  The device-side
 * position is written by a kernel enqueued on `stream`; the host-side count
 * changes at once, so the next chunk must be enqueued after this call, on
 * the same stream or one ordered after it.  Errors: MB_EINVAL. */
mb_status dedisp_beam_seek(mb_beam* beam, int64_t position, void* stream);
/* Device address of an int64 that every execute of a chunk on this beam
 * sets, in stream order, to the absolute index of the chunk's first output
 * (mb_exec_info.sample0).  Passed to detect_candidates as d_sample0, it keeps
 * the triplets of a captured chunk step on the right samples at every replay.
 * The address is valid until the beam is destroyed. */
mb_status dedisp_beam_sample0_ptr(const mb_beam* beam, const int64_t** d_sample0);
/* Advances the host-side sample count by nsamps without launching anything:
 * for chunks enqueued by replaying a captured graph. */
mb_status dedisp_beam_advance(mb_beam* beam, int64_t nsamps);
mb_status dedisp_beam_position(const mb_beam* beam, int64_t* seen);

/* ---- event detection (Sec. 2.3) ---------------------------------------- */

/* Bytes of caller-owned device workspace detect_candidates needs. */
mb_status detect_workspace_size(const mb_plan* plan, size_t* bytes);

/* Thresholds z = (D[d][t] - a_d - b_d*t) / sigma_d > nsigma (strict, FP64)
 * over d_out [ndms][ld_out], t < nout, with d_norm from dedisp_execute.
 * Writes candidates in (dm_index, sample) order, sample = s0 + t, where s0 is
 * sample0 plus, when d_sample0 (device int64, nullable) is given, the value it
 * holds when the kernels run (dedisp_beam_sample0_ptr):
 * the first min(count, capacity) to d_cands, the true count to *d_count
 * (device int64).  More than capacity is not an error at enqueue time: the
 * caller compares *d_count with capacity once the stream has run.
 * d_peaks (nullable, [ndms]) receives each row's largest z and its earliest
 * sample.  d_work: at least detect_workspace_size bytes, 256-byte aligned. */
mb_status detect_candidates(const mb_plan* plan, const float* d_out, int64_t nout,
                            int64_t ld_out, const mb_norm* d_norm, int64_t sample0,
                            const int64_t* d_sample0, double nsigma, mb_candidate* d_cands, int64_t capacity,
                            int64_t* d_count, mb_peak* d_peaks, void* d_work,
                            size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * detection as detect_candidates, with the same arguments, outputs and
 * errors, but no d_work.  Its counts and offsets live in a fixed device array
 * inside the library (2 MiB, one copy per GPU, kept until the process ends),
 * so the plan may have at most MB_DETECT_NOALLOC_MAX_DMS DMs (else
 * MB_EINVAL).  The call allocates nothing: the array's device address is
 * looked up once per device when a plan is created there (or on the first
 * call on that device).  The current device must be the plan's (else
 * MB_EINVAL).  Every call on one GPU shares that array, so calls whose work
 * overlaps on one GPU (on different streams, or from different threads
 * without ordering) race and must not be made; calls ordered on one stream
 * are safe, since each call writes every count and offset it reads. */
#define MB_DETECT_NOALLOC_MAX_DMS 8192
mb_status detect_candidates_noalloc(const mb_plan* plan, const float* d_out, int64_t nout,
                                    int64_t ld_out, const mb_norm* d_norm, int64_t sample0,
                                    const int64_t* d_sample0, double nsigma, mb_candidate* d_cands,
                                    int64_t capacity, int64_t* d_count, mb_peak* d_peaks, void* stream);

/* ---- errors ------------------------------------------------------------ */

const char* mb_status_str(mb_status s);
/* Description of the last error on the calling thread ("" if none). */
const char* mb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MBTP_H */
