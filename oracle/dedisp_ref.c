/*
 * Oracle (test infrastructure only): plain FP64 brute-force incoherent
 * dedispersion, Sec. 2.2.2 of the paper.
 *
 *   D[d][t] = sum over channels c (ascending) of y[c][t + s[d][c]]
 *
 * y is the (cleaned) filterbank in channel-major, time-contiguous order
 * (Sec. 2.1: beam/channel/time), s the integer delay table of Eq. (1).
 * No blocking, no reordering: one FP64 accumulator per output, channels
 * summed in ascending order.  OpenMP splits the work over DM trials only,
 * which does not change any result.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the GPU path.
 */
#include <stdint.h>
#include <omp.h>

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Full plane, FP64 input (cleaned samples). */
void oracle_dedisperse_f64(const double* y, int64_t nchans, int64_t ld_y,
                           const int32_t* delays, int64_t ndms, int64_t nout,
                           double* out, int64_t ld_out, int nthreads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t d = 0; d < ndms; ++d) {
    double* row = out + d * ld_out;
    for (int64_t t = 0; t < nout; ++t) row[t] = 0.0;
    for (int64_t c = 0; c < nchans; ++c) {
      const double* src = y + c * ld_y + delays[d * nchans + c];
      for (int64_t t = 0; t < nout; ++t) row[t] += src[t];
    }
  }
}

/* Full plane, FP32 input (raw stored values widened exactly: u8, f16 and
 * f32 all embed exactly in f32), accumulated in FP64. */
void oracle_dedisperse_f32(const float* x, int64_t nchans, int64_t ld_x,
                           const int32_t* delays, int64_t ndms, int64_t nout,
                           double* out, int64_t ld_out, int nthreads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t d = 0; d < ndms; ++d) {
    double* row = out + d * ld_out;
    for (int64_t t = 0; t < nout; ++t) row[t] = 0.0;
    for (int64_t c = 0; c < nchans; ++c) {
      const float* src = x + c * ld_x + delays[d * nchans + c];
      for (int64_t t = 0; t < nout; ++t) row[t] += (double)src[t];
    }
  }
}

/* Selected DM rows only (rows[i] is a DM index); out is [nrows][ld_out]. */
void oracle_dedisperse_rows_f64(const double* y, int64_t nchans, int64_t ld_y,
                                const int32_t* delays, int64_t nrows,
                                const int32_t* rows, int64_t nout, double* out,
                                int64_t ld_out, int nthreads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t d = rows[i];
    double* row = out + i * ld_out;
    for (int64_t t = 0; t < nout; ++t) row[t] = 0.0;
    for (int64_t c = 0; c < nchans; ++c) {
      const double* src = y + c * ld_y + delays[d * nchans + c];
      for (int64_t t = 0; t < nout; ++t) row[t] += src[t];
    }
  }
}

void oracle_dedisperse_rows_f32(const float* x, int64_t nchans, int64_t ld_x,
                                const int32_t* delays, int64_t nrows,
                                const int32_t* rows, int64_t nout, double* out,
                                int64_t ld_out, int nthreads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t d = rows[i];
    double* row = out + i * ld_out;
    for (int64_t t = 0; t < nout; ++t) row[t] = 0.0;
    for (int64_t c = 0; c < nchans; ++c) {
      const float* src = x + c * ld_x + delays[d * nchans + c];
      for (int64_t t = 0; t < nout; ++t) row[t] += (double)src[t];
    }
  }
}
