// Thresholding RFI pass of Sec. 2.2.1 on gfx950: bandpass correction,
// channel (chunk) thresholding and spectrum thresholding.
//
// HBM work is one read of the filterbank (rfi_stats_kernel); everything
// after it touches per-channel, per-chunk or per-sample statistics only,
// except the spectrum pass, which re-reads the few samples of flagged chunks.
// All statistics are accumulated in FP64 in a fixed order, so a flag differs
// from an FP64 reference only for a statistic within rounding of its
// threshold.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <math.h>

#include "internal.h"

namespace mbtp {
namespace {

template <typename T> struct Vec4Load;

template <> struct Vec4Load<float> {
  static __device__ inline void load(const float* p, double v[4]) {
    float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  static __device__ inline double one(const float* p) { return (double)*p; }
};
template <> struct Vec4Load<__half> {
  static __device__ inline void load(const __half* p, double v[4]) {
    uint2 q = *reinterpret_cast<const uint2*>(p);
    __half2 a = *reinterpret_cast<__half2*>(&q.x), b = *reinterpret_cast<__half2*>(&q.y);
    float2 fa = __half22float2(a), fb = __half22float2(b);
    v[0] = fa.x; v[1] = fa.y; v[2] = fb.x; v[3] = fb.y;
  }
  static __device__ inline double one(const __half* p) { return (double)__half2float(*p); }
};
template <> struct Vec4Load<uint8_t> {
  static __device__ inline void load(const uint8_t* p, double v[4]) {
    uint32_t q = *reinterpret_cast<const uint32_t*>(p);
    v[0] = (double)(q & 0xffu); v[1] = (double)((q >> 8) & 0xffu);
    v[2] = (double)((q >> 16) & 0xffu); v[3] = (double)(q >> 24);
  }
  static __device__ inline double one(const uint8_t* p) { return (double)*p; }
};

// v of another lane by a DPP move of both halves: the source lane of
// control CTRL in the rows of ROW_MASK, 0 where there is none.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_take(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed order, valid in lane 63: row
// shifts by 1, 2, 4 and 8 leave each 16-lane row's sum in its last lane,
// then the row broadcasts of lanes 15 and 31 carry rows 0-2 into row 3.
__device__ inline double wave_total(double v) {
  v += dpp_take<0x111, 0xf>(v);   // row_shr:1
  v += dpp_take<0x112, 0xf>(v);   // row_shr:2
  v += dpp_take<0x114, 0xf>(v);   // row_shr:4
  v += dpp_take<0x118, 0xf>(v);   // row_shr:8
  v += dpp_take<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_take<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Block-wide FP64 sum over a 1024-thread block; fixed reduction tree.
__device__ inline double block_sum_1024(double v, double* sh) {
  v = wave_total(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 63) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < 64) {
    r = (lane < 16) ? sh[lane] : 0.0;
    r = wave_total(r);
    if (lane == 63) sh[16] = r;
  }
  __syncthreads();
  return sh[16];
}

// ---------------------------------------------------------------------------
// Statistics pass: one read of x.  Workgroup = (256-sample span, group of CG
// channels); wave w takes channels g*CG + w, +4, ...; lane l holds samples
// t0+4l..t0+4l+3.  Writes per-(channel, span) sums and per-(group, sample)
// partial spectrum sums.
// ---------------------------------------------------------------------------
template <typename TIN>
__global__ __launch_bounds__(256) void rfi_stats_kernel(const TIN* __restrict__ x, int64_t ld,
                                                        int64_t C, int64_t T, int64_t nspans,
                                                        int64_t CG, double* __restrict__ span_sum,
                                                        double* __restrict__ spart) {
  __shared__ double col_sh[4][kSpan];
  const int span = blockIdx.x, g = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t0 = (int64_t)span * kSpan;
  const int64_t tl = t0 + 4 * lane;
  const int64_t cb = (int64_t)g * CG, ce = min(C, cb + CG);
  const bool full = (tl + 3 < T);
  double col[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t c = cb + wave;
  if (t0 + kSpan <= T) {
    // (uniform: the whole span lies in the chunk, so every lane takes this
    // path and the wave sums see the full wave) four of the wave's channels
    // at a time, their loads in flight together; the sums take them in the
    // same order as one at a time
    for (; c + 12 < ce; c += 16) {
      double v[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) Vec4Load<TIN>::load(x + (c + 4 * u) * ld + tl, v[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) col[i] += v[u][i];
        const double rs = wave_total((v[u][0] + v[u][1]) + (v[u][2] + v[u][3]));
        if (lane == 63) span_sum[(c + 4 * u) * nspans + span] = rs;
      }
    }
  }
  for (; c < ce; c += 4) {
    double v[4];
    const TIN* row = x + c * ld + tl;
    if (full) {
      Vec4Load<TIN>::load(row, v);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (tl + i < T) ? Vec4Load<TIN>::one(row + i) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) col[i] += v[i];
    double rs = wave_total((v[0] + v[1]) + (v[2] + v[3]));
    if (lane == 63) span_sum[c * nspans + span] = rs;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) col_sh[wave][4 * lane + i] = col[i];
  __syncthreads();
  const int64_t t = t0 + threadIdx.x;
  if (t < T) {
    const int k = threadIdx.x;
    spart[(int64_t)g * T + t] = ((col_sh[0][k] + col_sh[1][k]) + col_sh[2][k]) + col_sh[3][k];
  }
}

// Per-(channel, chunk) sums from the span sums, and per-channel totals.
// One wave per channel, lanes over chunks.
__global__ __launch_bounds__(256) void rfi_chunks_kernel(const double* __restrict__ span_sum,
                                                         int64_t C, int64_t nspans, int64_t spc,
                                                         int64_t J, double* __restrict__ chunk_sum,
                                                         double* __restrict__ bsum) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= C) return;
  double part = 0.0;
  for (int64_t j = lane; j < J; j += 64) {
    double m = 0.0;
    const int64_t s1 = min(nspans, (j + 1) * spc);
    for (int64_t s = j * spc; s < s1; ++s) m += span_sum[c * nspans + s];
    chunk_sum[c * J + j] = m;
    part += m;
  }
  part = wave_total(part);
  if (lane == 63) bsum[c] = part;
}

// ---------------------------------------------------------------------------
// Bandpass fit on one 1024-thread workgroup.  The least-squares polynomial of
// degree p over u_c in [-1, 1] is solved through the normal equations in the
// Legendre basis (well conditioned on equispaced points; same polynomial
// space, hence the same fit as any other basis up to rounding), by Cholesky.
// ---------------------------------------------------------------------------
constexpr int kMaxP = 8;

// Legendre polynomials P_0..P_D at u (three-term recurrence), unrolled.
template <int D>
__device__ inline void legendre(double u, double (&P)[D + 1]) {
  P[0] = 1.0;
  if constexpr (D >= 1) P[1] = u;
#pragma unroll
  for (int k = 1; k < D; ++k) P[k + 1] = ((2 * k + 1) * u * P[k] - k * P[k - 1]) / (k + 1);
}

__device__ inline double u_of(int64_t c, int64_t C) {
  return (2.0 * (double)c - (double)(C - 1)) / (double)(C - 1);
}

// Block-wide sums of NV values per thread at once (1024 threads): each wave
// reduces its values, then thread k < NV adds the 16 wave results of value k.
// Fixed order; two barriers for the whole batch.
template <int NV>
__device__ inline void block_sums_1024(const double (&v)[NV], double* sh /* 16*NV + NV */,
                                       double (&out)[NV]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double r = wave_total(v[k]);
    if (lane == 63) sh[w * NV + k] = r;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
    for (int ww = 0; ww < 16; ++ww) t += sh[ww * NV + threadIdx.x];
    sh[16 * NV + threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = sh[16 * NV + k];
}

// Packed lower-triangular index of (i, j), j <= i.
constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Cholesky factor (packed lower, in L) of the Legendre Gram matrix of degree
// D over the C channel positions.  All threads call it; every array has a
// compile-time size, so nothing leaves registers.
template <int D>
__device__ void gram_cholesky(int64_t C, double* sh, double* L) {
  constexpr int N = D + 1, NG = N * (N + 1) / 2;
  double Gl[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) Gl[i] = 0.0;
  for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
    double P[N];
    legendre<D>(u_of(c, C), P);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) Gl[tri(i, j)] += P[i] * P[j];
  }
  double G[NG];
  block_sums_1024<NG>(Gl, sh, G);
  if (threadIdx.x == 0) {
    double Lr[NG];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        double v = G[tri(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= Lr[tri(i, k)] * Lr[tri(j, k)];
        if (i == j) Lr[tri(i, i)] = sqrt(v > 0.0 ? v : 0.0);
        else Lr[tri(i, j)] = v / Lr[tri(j, j)];
      }
#pragma unroll
    for (int i = 0; i < NG; ++i) L[i] = Lr[i];
  }
  __syncthreads();
}

// Least-squares fit of v[c] with the factored Gram matrix: writes the fitted
// curve to fit[c] and returns the RMSE of v - fit.  All threads call it.
template <int D>
__device__ double fit_poly(const double* v, int64_t C, const double* L, double* fit, double* sh,
                           double* coef_sh) {
  constexpr int N = D + 1;
  double hl[N];
#pragma unroll
  for (int i = 0; i < N; ++i) hl[i] = 0.0;
  for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
    double P[N];
    legendre<D>(u_of(c, C), P);
    const double vc = v[c];
#pragma unroll
    for (int i = 0; i < N; ++i) hl[i] += P[i] * vc;
  }
  double h[N];
  block_sums_1024<N>(hl, sh, h);
  if (threadIdx.x == 0) {
    double Lr[N * (N + 1) / 2];
#pragma unroll
    for (int i = 0; i < N * (N + 1) / 2; ++i) Lr[i] = L[i];
    double y[N], x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {            // L y = h
      double t = h[i];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= Lr[tri(i, k)] * y[k];
      y[i] = t / Lr[tri(i, i)];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {       // L^T x = y
      double t = y[i];
#pragma unroll
      for (int k = i + 1; k < N; ++k) t -= Lr[tri(k, i)] * x[k];
      x[i] = t / Lr[tri(i, i)];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) coef_sh[i] = x[i];
  }
  __syncthreads();
  double coef[N];
#pragma unroll
  for (int i = 0; i < N; ++i) coef[i] = coef_sh[i];
  double ssq[1] = {0.0};
  for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
    double P[N];
    legendre<D>(u_of(c, C), P);
    double f = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) f += coef[i] * P[i];
    fit[c] = f;
    const double r = v[c] - f;
    ssq[0] += r * r;
  }
  double tot[1];
  block_sums_1024<1>(ssq, sh, tot);
  return sqrt(tot[0] / (double)C);
}

template <int D>
__global__ __launch_bounds__(1024) void rfi_fit_kernel(int64_t C, int64_t T, RfiParamsDev prm,
                                                       const double* __restrict__ bsum,
                                                       double* __restrict__ binterp,
                                                       double* __restrict__ fit,
                                                       float* __restrict__ fit32,
                                                       uint8_t* __restrict__ masked,
                                                       RfiHeader* __restrict__ hdr) {
  constexpr int NG = (D + 1) * (D + 2) / 2;
  __shared__ double sh[17 * NG + 17];
  __shared__ double coef_sh[D + 1];
  __shared__ double L[NG];
  const double invT = 1.0 / (double)T;
  for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
    binterp[c] = bsum[c] * invT;
    masked[c] = 0;
  }
  gram_cholesky<D>(C, sh, L);   // (its barriers also publish binterp/masked)
  double rmse0 = 0.0;
  int any_left = 1;
  // Fit-and-mask rounds: each fits the interpolated bandpass and masks the
  // channels whose raw residual exceeds k_mask times that fit's RMSE (the
  // mask only grows).  They stop after a round that masks no new channel,
  // whose fit is then already the final one, or after mask_passes rounds.
  const int passes = prm.mask_passes < 1 ? 1 : prm.mask_passes;
  bool settled = false;
  double rmse = 0.0;
  for (int pass = 0; pass < passes; ++pass) {
    const double rmse_i = fit_poly<D>(binterp, C, L, fit, sh, coef_sh);
    if (pass == 0) rmse0 = rmse_i;
    rmse = rmse_i;
    const double thr = prm.k_mask * rmse_i;
    int bits = 0;                            // bit 0: an unmasked channel is left; bit 1: the mask grew
    for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
      const double r = bsum[c] * invT - fit[c];
      if (fabs(r) > thr && !masked[c]) { masked[c] = 1; bits |= 2; }
      bits |= masked[c] ? 0 : 1;
    }
    // the block-wide ORs also publish masked[]
    const int all = __syncthreads_or(bits & 1) | (__syncthreads_or(bits & 2) ? 2 : 0);
    any_left = all & 1;
    if (!any_left) break;
    if (!(all & 2)) { settled = true; break; }
    // nearest unmasked neighbour on each side (one side at a band edge)
    for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
      if (!masked[c]) { binterp[c] = bsum[c] * invT; continue; }
      int64_t l = c - 1, r = c + 1;
      while (l >= 0 && masked[l]) --l;
      while (r < C && masked[r]) ++r;
      double v;
      if (l >= 0 && r < C) v = (bsum[l] * invT + bsum[r] * invT) * 0.5;
      else if (l >= 0) v = bsum[l] * invT;
      else v = bsum[r] * invT;
      binterp[c] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    hdr->nsamps = T;
    hdr->nchunks = (T + prm.W - 1) / prm.W;
  }
  if (!any_left) {
    for (int64_t c = threadIdx.x; c < C; c += blockDim.x) fit32[c] = 0.0f;
    if (threadIdx.x == 0) {
      hdr->error = 1; hdr->sigma = 0.0; hdr->rmse0 = rmse0; hdr->rmse = 0.0;
      hdr->sum_fit = 0.0; hdr->thr_spec = 0.0; hdr->k_chan = prm.k_chan;
      hdr->n_masked = (unsigned long long)C; hdr->n_chunk = hdr->n_chunk_ext = hdr->n_spec = 0;
    }
    return;
  }
  if (!settled) rmse = fit_poly<D>(binterp, C, L, fit, sh, coef_sh);
  double sums[2] = {0.0, 0.0};
  for (int64_t c = threadIdx.x; c < C; c += blockDim.x) {
    fit32[c] = (float)fit[c];
    sums[0] += fit[c];
    sums[1] += masked[c] ? 1.0 : 0.0;
  }
  double tot[2];
  block_sums_1024<2>(sums, sh, tot);
  if (threadIdx.x == 0) {
    const double sigma = rmse * sqrt((double)T * (double)C / (double)(C - prm.p - 1));
    hdr->sigma = sigma;
    hdr->rmse0 = rmse0;
    hdr->rmse = rmse;
    hdr->sum_fit = tot[0];
    hdr->thr_spec = prm.k_spec * sigma / sqrt((double)C);
    hdr->k_chan = prm.k_chan;
    hdr->n_masked = (unsigned long long)tot[1];
    hdr->n_chunk = hdr->n_chunk_ext = hdr->n_spec = 0;
    hdr->error = 0;
  }
}

// The same fit-and-mask rounds for up to kFitRegMaxC channels with the
// interpolated bandpass in registers: thread k owns channels k, k + 1024,
// ... (KC of them), the mask is mirrored in LDS for the neighbour search,
// and every thread solves the tiny normal equations itself, so a round is
// two block sums and two block-wide ORs.  The sums run over the same
// per-thread partials and the same reduction tree as rfi_fit_kernel, so
// both give the same fit.
constexpr int64_t kFitRegMaxC = 2048;

template <int D>
__device__ inline void cholesky_packed(const double* G, double* L) {
  constexpr int N = D + 1;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double v = G[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
      if (i == j) L[tri(i, i)] = sqrt(v > 0.0 ? v : 0.0);
      else L[tri(i, j)] = v / L[tri(j, j)];
    }
}

template <int D>
__device__ inline void chol_solve(const double* L, const double* h, double* x) {
  constexpr int N = D + 1;
  double y[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = h[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[tri(i, k)] * y[k];
    y[i] = t / L[tri(i, i)];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double t = y[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) t -= L[tri(k, i)] * x[k];
    x[i] = t / L[tri(i, i)];
  }
}

template <int D, int KC>
__global__ __launch_bounds__(1024) void rfi_fit_reg_kernel(int64_t C, int64_t T, RfiParamsDev prm,
                                                           const double* __restrict__ bsum,
                                                           double* __restrict__ binterp,
                                                           double* __restrict__ fit,
                                                           float* __restrict__ fit32,
                                                           uint8_t* __restrict__ masked,
                                                           RfiHeader* __restrict__ hdr) {
  constexpr int N = D + 1, NG = N * (N + 1) / 2;
  __shared__ double sh[17 * NG + 17];
  __shared__ uint8_t msk[kFitRegMaxC];
  const int tid = threadIdx.x;
  const double invT = 1.0 / (double)T;
  double bi[KC];
  uint32_t mine = 0;                         // bit k: channel tid + 1024k is masked
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int64_t c = tid + 1024 * k;
    bi[k] = c < C ? bsum[c] * invT : 0.0;
    if (c < C) msk[c] = 0;
  }
  // Gram matrix of the Legendre basis over the channel positions, factored
  // by every thread
  double L[NG];
  {
    double Gl[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) Gl[i] = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int64_t c = tid + 1024 * k;
      if (c < C) {
        double P[N];
        legendre<D>(u_of(c, C), P);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j) Gl[tri(i, j)] += P[i] * P[j];
      }
    }
    double G[NG];
    block_sums_1024<NG>(Gl, sh, G);
    cholesky_packed<D>(G, L);
  }
  // least-squares coefficients of bi and the RMSE of bi - fit
  double coef[N];
  auto fit_round = [&]() -> double {
    double hl[N];
#pragma unroll
    for (int i = 0; i < N; ++i) hl[i] = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int64_t c = tid + 1024 * k;
      if (c < C) {
        double P[N];
        legendre<D>(u_of(c, C), P);
#pragma unroll
        for (int i = 0; i < N; ++i) hl[i] += P[i] * bi[k];
      }
    }
    double h[N];
    block_sums_1024<N>(hl, sh, h);
    chol_solve<D>(L, h, coef);
    double ssq[1] = {0.0};
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int64_t c = tid + 1024 * k;
      if (c < C) {
        double P[N];
        legendre<D>(u_of(c, C), P);
        double f = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) f += coef[i] * P[i];
        const double r = bi[k] - f;
        ssq[0] += r * r;
      }
    }
    double tot[1];
    block_sums_1024<1>(ssq, sh, tot);
    return sqrt(tot[0] / (double)C);
  };
  auto fit_at = [&](int64_t c) {
    double P[N];
    legendre<D>(u_of(c, C), P);
    double f = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) f += coef[i] * P[i];
    return f;
  };
  double rmse0 = 0.0, rmse = 0.0;
  int any_left = 1;
  bool settled = false;
  const int passes = prm.mask_passes < 1 ? 1 : prm.mask_passes;
  for (int pass = 0; pass < passes; ++pass) {
    const double rmse_i = fit_round();
    if (pass == 0) rmse0 = rmse_i;
    rmse = rmse_i;
    const double thr = prm.k_mask * rmse_i;
    int bits = 0;                            // bit 0: an unmasked channel is left; bit 1: the mask grew
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int64_t c = tid + 1024 * k;
      if (c < C) {
        if (!((mine >> k) & 1u) && fabs(bsum[c] * invT - fit_at(c)) > thr) {
          mine |= 1u << k;
          msk[c] = 1;
          bits |= 2;
        }
        bits |= ((mine >> k) & 1u) ? 0 : 1;
      }
    }
    // the block-wide ORs also publish msk[]
    const int all = __syncthreads_or(bits & 1) | (__syncthreads_or(bits & 2) ? 2 : 0);
    any_left = all & 1;
    if (!any_left) break;
    if (!(all & 2)) { settled = true; break; }
    // masked channels take the mean of their nearest unmasked neighbours
    // (one side at a band edge); the others keep their own mean
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int64_t c = tid + 1024 * k;
      if (c < C && ((mine >> k) & 1u)) {
        int64_t l = c - 1, r = c + 1;
        while (l >= 0 && msk[l]) --l;
        while (r < C && msk[r]) ++r;
        double v;
        if (l >= 0 && r < C) v = (bsum[l] * invT + bsum[r] * invT) * 0.5;
        else if (l >= 0) v = bsum[l] * invT;
        else v = bsum[r] * invT;
        bi[k] = v;
      }
    }
  }
  if (tid == 0) {
    hdr->nsamps = T;
    hdr->nchunks = (T + prm.W - 1) / prm.W;
  }
  if (!any_left) {
    for (int64_t c = tid; c < C; c += 1024) {
      fit32[c] = 0.0f;
      masked[c] = 1;
      binterp[c] = bsum[c] * invT;
    }
    if (tid == 0) {
      hdr->error = 1; hdr->sigma = 0.0; hdr->rmse0 = rmse0; hdr->rmse = 0.0;
      hdr->sum_fit = 0.0; hdr->thr_spec = 0.0; hdr->k_chan = prm.k_chan;
      hdr->n_masked = (unsigned long long)C; hdr->n_chunk = hdr->n_chunk_ext = hdr->n_spec = 0;
    }
    return;
  }
  if (!settled) rmse = fit_round();
  double sums[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int64_t c = tid + 1024 * k;
    if (c < C) {
      const double f = fit_at(c);
      fit[c] = f;
      fit32[c] = (float)f;
      binterp[c] = bi[k];
      masked[c] = (uint8_t)((mine >> k) & 1u);
      sums[0] += f;
      sums[1] += ((mine >> k) & 1u) ? 1.0 : 0.0;
    }
  }
  double tot[2];
  block_sums_1024<2>(sums, sh, tot);
  if (tid == 0) {
    const double sigma = rmse * sqrt((double)T * (double)C / (double)(C - prm.p - 1));
    hdr->sigma = sigma;
    hdr->rmse0 = rmse0;
    hdr->rmse = rmse;
    hdr->sum_fit = tot[0];
    hdr->thr_spec = prm.k_spec * sigma / sqrt((double)C);
    hdr->k_chan = prm.k_chan;
    hdr->n_masked = (unsigned long long)tot[1];
    hdr->n_chunk = hdr->n_chunk_ext = hdr->n_spec = 0;
    hdr->error = 0;
  }
}

// ---------------------------------------------------------------------------
// Chunk flags: one workgroup per chunk j, threads over channels.  F[c][j] is
// |M[c][j]/L_j - f_c| > k_chan*sigma/sqrt(L_j); the extended flag also takes
// the time-adjacent chunks j-1 and j+1 of the same channel.  The flagged
// channels of chunk j are listed in ascending order for the spectrum pass.
// ---------------------------------------------------------------------------
__device__ inline bool chunk_over(const double* M, const double* fit, int64_t c, int64_t j,
                                  int64_t J, int64_t T, int64_t W, double sigma, double k) {
  const int64_t L = min(W, T - j * W);
  const double m = M[c * J + j] / (double)L - fit[c];
  return fabs(m) > k * sigma / sqrt((double)L);
}

__global__ __launch_bounds__(256) void rfi_chunk_flags_kernel(const double* __restrict__ M,
                                                              const double* __restrict__ fit,
                                                              int64_t C, int64_t T, int64_t W,
                                                              int64_t J, RfiHeader* __restrict__ hdr,
                                                              uint8_t* __restrict__ flags,
                                                              int32_t* __restrict__ lcount,
                                                              int32_t* __restrict__ list) {
  __shared__ int wcount[4];
  const int64_t j = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool err = hdr->error != 0;
  const double sigma = hdr->sigma, k = hdr->k_chan;
  int64_t base = 0;
  int n0 = 0, n1 = 0;
  for (int64_t c0 = 0; c0 < C; c0 += 256) {
    const int64_t c = c0 + threadIdx.x;
    bool f0 = false, fx = false;
    if (c < C && !err) {
      f0 = chunk_over(M, fit, c, j, J, T, W, sigma, k);
      const bool fm = (j > 0) && chunk_over(M, fit, c, j - 1, J, T, W, sigma, k);
      const bool fp = (j + 1 < J) && chunk_over(M, fit, c, j + 1, J, T, W, sigma, k);
      fx = f0 || fm || fp;
    }
    if (c < C) flags[c * J + j] = (uint8_t)((f0 ? 1 : 0) | (fx ? 2 : 0));
    n0 += f0; n1 += fx;
    const unsigned long long bal = __ballot(fx);
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wcount[w];
    const int total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    if (fx) {
      const unsigned long long lower = (lane == 0) ? 0ull : (bal & ((1ull << lane) - 1ull));
      list[j * C + base + before + __popcll(lower)] = (int32_t)c;
    }
    base += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) lcount[j] = (int32_t)base;
  // counts (integer atomics: order-free)
  int a0 = n0, a1 = n1;
  for (int off = 32; off >= 1; off >>= 1) {
    a0 += __shfl_xor(a0, off, 64);
    a1 += __shfl_xor(a1, off, 64);
  }
  if (lane == 0 && (a0 | a1)) {
    atomicAdd(&hdr->n_chunk, (unsigned long long)a0);
    atomicAdd(&hdr->n_chunk_ext, (unsigned long long)a1);
  }
}

// ---------------------------------------------------------------------------
// Spectrum flags: s[t] = (sum_c (x - f_c) - sum over flagged chunks' (x - f_c)) / C,
// G[t] = |s[t]| > k_spec*sigma/sqrt(C).  One thread per sample.
// ---------------------------------------------------------------------------
template <typename TIN>
__global__ __launch_bounds__(256) void rfi_spectrum_flags_kernel(
    const TIN* __restrict__ x, int64_t ld, int64_t C, int64_t T, int64_t W, int64_t J,
    const double* __restrict__ spart, int64_t ngroups, const double* __restrict__ fit,
    const int32_t* __restrict__ lcount, const int32_t* __restrict__ list,
    RfiHeader* __restrict__ hdr, uint8_t* __restrict__ gflags) {
  __shared__ int wc[4];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  bool g = false;
  if (t < T && hdr->error == 0) {
    double S = 0.0;
    for (int64_t k = 0; k < ngroups; ++k) S += spart[k * T + t];
    const int64_t j = t / W;
    double corr = 0.0;
    const int n = lcount[j];
    const int32_t* lj = list + j * C;
    // the flagged channels of the chunk in ascending order, eight loads in
    // flight at a time; the additions keep that order
    int k = 0;
    for (; k + 8 <= n; k += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t c = lj[k + u];
        v[u] = Vec4Load<TIN>::one(x + c * ld + t) - fit[c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) corr += v[u];
    }
    for (; k < n; ++k) {
      const int64_t c = lj[k];
      corr += Vec4Load<TIN>::one(x + c * ld + t) - fit[c];
    }
    const double s = ((S - hdr->sum_fit) - corr) / (double)C;
    g = fabs(s) > hdr->thr_spec;
  }
  if (t < T) gflags[t] = g ? 1 : 0;
  const int cnt = __popcll(__ballot(g));
  if (lane == 0) wc[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = wc[0] + wc[1] + wc[2] + wc[3];
    if (tot) atomicAdd(&hdr->n_spec, (unsigned long long)tot);
  }
}

// Tables that let dedispersion staging skip per-sample flag reads: the
// extended chunk flags as one bit per chunk, and the exclusive prefix count of
// flagged spectra per 256-sample span (one 1024-thread workgroup scans it).
__global__ __launch_bounds__(256) void rfi_chunk_bits_kernel(const uint8_t* __restrict__ flags,
                                                             int64_t C, int64_t J, int64_t JW,
                                                             uint32_t* __restrict__ cbits) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= C * JW) return;
  const int64_t c = i / JW, w = i % JW;
  uint32_t word = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t j = w * 32 + b;
    if (j < J && (flags[c * J + j] & 2)) word |= 1u << b;
  }
  cbits[i] = word;
}

// The register-resident fit where its registers hold without spilling
// (degree <= 4, up to 2048 channels), else the fit through global memory.
template <int D>
void launch_fit(const RfiGeom& g, const RfiParamsDev& prm, const double* bsum, double* binterp, double* fit,
                float* fit32, uint8_t* masked, RfiHeader* hdr, hipStream_t s) {
  if constexpr (D <= 4) {
    if (g.C <= 1024) {
      hipLaunchKernelGGL((rfi_fit_reg_kernel<D, 1>), dim3(1), dim3(1024), 0, s, g.C, g.T, prm, bsum, binterp, fit,
                         fit32, masked, hdr);
      return;
    }
    if (g.C <= 2048) {
      hipLaunchKernelGGL((rfi_fit_reg_kernel<D, 2>), dim3(1), dim3(1024), 0, s, g.C, g.T, prm, bsum, binterp, fit,
                         fit32, masked, hdr);
      return;
    }
  }
  hipLaunchKernelGGL(rfi_fit_kernel<D>, dim3(1), dim3(1024), 0, s, g.C, g.T, prm, bsum, binterp, fit, fit32,
                     masked, hdr);
}

template <typename TIN>
hipError_t launch_rfi_t(const TIN* x, int64_t ld, const RfiGeom& g, const RfiParamsDev& prm,
                        char* st, hipStream_t s) {
  double* span_sum = reinterpret_cast<double*>(st + g.off_span);
  double* spart = reinterpret_cast<double*>(st + g.off_spart);
  double* chunk = reinterpret_cast<double*>(st + g.off_chunk);
  double* bsum = reinterpret_cast<double*>(st + g.off_bsum);
  double* binterp = reinterpret_cast<double*>(st + g.off_binterp);
  double* fit = reinterpret_cast<double*>(st + g.off_fit);
  float* fit32 = reinterpret_cast<float*>(st + g.off_fit32);
  uint8_t* masked = reinterpret_cast<uint8_t*>(st + g.off_masked);
  uint8_t* flags = reinterpret_cast<uint8_t*>(st + g.off_flags);
  uint8_t* gflags = reinterpret_cast<uint8_t*>(st + g.off_gflags);
  int32_t* lcount = reinterpret_cast<int32_t*>(st + g.off_lcount);
  int32_t* list = reinterpret_cast<int32_t*>(st + g.off_list);
  RfiHeader* hdr = reinterpret_cast<RfiHeader*>(st + g.off_hdr);
  uint32_t* cbits = reinterpret_cast<uint32_t*>(st + g.off_cbits);

  hipLaunchKernelGGL(rfi_stats_kernel<TIN>, dim3((unsigned)g.nspans, (unsigned)g.ngroups),
                     dim3(256), 0, s, x, ld, g.C, g.T, g.nspans, g.CG, span_sum, spart);
  hipLaunchKernelGGL(rfi_chunks_kernel, dim3((unsigned)((g.C + 3) / 4)), dim3(256), 0, s,
                     span_sum, g.C, g.nspans, g.W / kSpan, g.J, chunk, bsum);
  switch (prm.p) {
#define MBTP_FIT(D_) \
    case D_: launch_fit<D_>(g, prm, bsum, binterp, fit, fit32, masked, hdr, s); break;
    MBTP_FIT(0) MBTP_FIT(1) MBTP_FIT(2) MBTP_FIT(3) MBTP_FIT(4) MBTP_FIT(5) MBTP_FIT(6)
    MBTP_FIT(7) MBTP_FIT(8)
#undef MBTP_FIT
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(rfi_chunk_flags_kernel, dim3((unsigned)g.J), dim3(256), 0, s, chunk, fit,
                     g.C, g.T, g.W, g.J, hdr, flags, lcount, list);
  hipLaunchKernelGGL(rfi_spectrum_flags_kernel<TIN>, dim3((unsigned)((g.T + 255) / 256)),
                     dim3(256), 0, s, x, ld, g.C, g.T, g.W, g.J, spart, g.ngroups, fit, lcount,
                     list, hdr, gflags);
  hipLaunchKernelGGL(rfi_chunk_bits_kernel, dim3((unsigned)((g.C * g.JW + 255) / 256)), dim3(256), 0,
                     s, flags, g.C, g.J, g.JW, cbits);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rfi(int dtype, const void* x, int64_t ld, const RfiGeom& g,
                      const RfiParamsDev& prm, char* state, hipStream_t s) {
  switch (dtype) {
    case 0: return launch_rfi_t(static_cast<const uint8_t*>(x), ld, g, prm, state, s);
    case 1: return launch_rfi_t(static_cast<const __half*>(x), ld, g, prm, state, s);
    default: return launch_rfi_t(static_cast<const float*>(x), ld, g, prm, state, s);
  }
}

}  // namespace mbtp
