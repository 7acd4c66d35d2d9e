// Device helpers shared by the characteristic-function kernels (grouped
// counts and joint distributions): per-sample occupation sums over a mode
// range, exp(x) cis(phase) in FP64 or FP32, the magnitude bound of a
// sample's factor e^{n (e^{i theta} - 1)} over the grid and the band of grid
// points where it can exceed e^kLogEps.
#pragma once

#include "common.h"

namespace mp {

// Terms of a sample's characteristic function with log-magnitude below kLogEps
// (e^-46 ~ 1e-20) are not evaluated.  The magnitude test is exact, so each
// sub-ensemble mean of chi changes by less than 1e-20 per grid point and P(m)
// (an average of those means) by less than 1e-20 absolute.
constexpr double kLogEps = -46.0;

// Samples per wave of the per-sample occupation kernels (one wave per sample
// at a time, lanes over modes).
constexpr int kOccPerWave = 16;

// Log-weights of a sample's two parity terms (matrix-P estimator),
// c1 = log(e^n / (2 cosh n)) and c2 = log(e^-n / (2 cosh n)), in forms that
// cannot overflow.  `finite` is false when n or one of the sample's bin sums
// is not finite (an amplitude beyond a reduced precision's range): both
// weights are then NaN, so the sample reaches the FP64 accumulators, and
// mp_check_finite, as NaN instead of reading as a sample of very large |n|.
__device__ inline void parity_log_weights(double n, bool finite, double& c1, double& c2) {
  const double L = log1p(exp(-2.0 * fabs(n)));
  c1 = (n >= 0.0 ? 0.0 : 2.0 * n) - L;
  c2 = (n >= 0.0 ? -2.0 * n : 0.0) - L;
  if (!finite) c1 = c2 = __builtin_nan("");
}

// One sample's partial n'_j sums over a mode range, wave-reduced.
template <typename CT>
__device__ inline void run_sum(const CT* __restrict__ ca, const CT* __restrict__ cb, int64_t ldm,
                               int lo, int hi, int lane, double& re, double& im) {
  double sr = 0.0, si = 0.0;
  int j = lo + lane;
  for (; j + 192 < hi; j += 256) {
    double a[4], b[4], c[4], e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = (double)ca[j + 64 * u];
      b[u] = (double)ca[ldm + j + 64 * u];
      c[u] = (double)cb[j + 64 * u];
      e[u] = (double)cb[ldm + j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // alpha' = a + i b, beta' = c - i e  ->  n' = (a c + b e) + i (b c - a e)
      sr += a[u] * c[u] + b[u] * e[u];
      si += b[u] * c[u] - a[u] * e[u];
    }
  }
  for (; j < hi; j += 64) {
    const double a = (double)ca[j], b = (double)ca[ldm + j];
    const double c = (double)cb[j], e = (double)cb[ldm + j];
    sr += a * c + b * e;
    si += b * c - a * e;
  }
  re = wave_sum(sr);
  im = wave_sum(si);
}

// One sample's occupation sum over one bin run from the occupation-fused
// GEMM's partials: the run's slots [slot0, slot0 + nblk) (one per 128-mode
// block it touches), four floats per (slot, sample) at part[(slot E + k) 4]:
// (re, im) from the Re-row half and from the Im-row half.  Wave-reduced.
__device__ inline void run_sum_partials(const float* __restrict__ part, int64_t E, int slot0,
                                        int nblk, int64_t k, int lane, double& re, double& im) {
  double sr = 0.0, si = 0.0;
  for (int t = lane; t < nblk; t += 64) {
    const float4 v = *(const float4*)(part + ((int64_t)(slot0 + t) * E + k) * 4);
    sr += (double)v.x + (double)v.z;
    si += (double)v.y + (double)v.w;
  }
  re = wave_sum(sr);
  im = wave_sum(si);
}

// Slots of a run [lo, hi) in the fused partials: the 128-mode blocks it touches.
__host__ __device__ inline int run_blocks(int lo, int hi) { return ((hi - 1) >> 7) - (lo >> 7) + 1; }

__device__ inline double reduce_2pi(double ph) {
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  constexpr double kInvTwoPi = 0.15915494309189533576888376337251;
  return ph - kTwoPi * rint(ph * kInvTwoPi);
}

template <bool F64>
__device__ inline void cis_exp(double ex, double ph, double& re, double& im) {
  if constexpr (F64) {
    const double mag = exp(ex);
    double s, c;
    sincos(ph, &s, &c);
    re = mag * c;
    im = mag * s;
  } else {
    const float mag = expf((float)ex);
    float s, c;
    sincosf((float)reduce_2pi(ph), &s, &c);
    re = (double)(mag * c);
    im = (double)(mag * s);
  }
}

__device__ inline double fmax_exponent(double R, double I) {
  // max over theta of -(1 - cos t) R + |sin t| |I|
  if (R <= 0.0) return 2.0 * fabs(R) + fabs(I);
  const double t = atan2(fabs(I), R);
  return -(1.0 - cos(t)) * R + sin(t) * fabs(I);
}

// Smallest h such that f(theta_k) + offset < kLogEps for every grid point at
// circular distance > h from theta = 0 (the last grid point at or below pi
// where it reaches the threshold); -1 when no point reaches it.
__device__ inline int band_halfwidth(double R, double I, double offset, int K) {
  const double fmax = fmax_exponent(R, I);
  const int half = K / 2;
  // a sample that is not finite takes the whole axis, so its NaN reaches every
  // point of the sums (and no index is formed from it)
  if (!isfinite(fmax + offset)) return half;
  if (fmax + offset < kLogEps) return -1;
  if (R <= 0.0) return half;
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  auto f = [&](int k) {
    const double t = kTwoPi * k / K;
    return -(1.0 - cos(t)) * R + fabs(sin(t)) * fabs(I) + offset;
  };
  // On [0, pi], f(theta) = rho cos(theta - phi) - R + offset with
  // rho = |n|, phi = atan2(|Im n|, Re n): it rises to its maximum at phi and
  // falls after, so the grid points with f >= eps form one run.  Its last
  // point from the closed form phi + acos((R + eps - offset) / rho), then
  // corrected on the grid (the closed form lands at or after the point
  // below phi, and rounding moves it by a point or two); -1 when no grid
  // point reaches eps.
  const double rho = hypot(R, I), phi = atan2(fabs(I), R);
  const double c = (R + kLogEps - offset) / rho;
  int k = c <= -1.0 ? half : (int)floor((phi + acos(fmin(c, 1.0))) / kTwoPi * K);
  k = k < 0 ? 0 : (k > half ? half : k);
  while (k < half && f(k + 1) >= kLogEps) ++k;
  while (k >= 0 && f(k) < kLogEps) --k;
  return k;
}

// Box half-width on axis b of term tau (0: about theta = 0, 1: about pi) for
// one sample record r = (Re n_0, Im n_0, .., Re n_{d-1}, Im n_{d-1}, c1, c2):
// band_halfwidth of the axis with every other axis at its maximum.  About
// theta = pi the exponent is 2 Re n_b + f_b(phi) with Im n_b negated (the same
// bound) and the offset holds c2 + 2 sum_b Re n_b; +1 there because for odd K
// the grid is not symmetric about pi.  c2 = -inf (the +P estimator) removes
// the second term.
__device__ inline int record_band(const double* __restrict__ r, int d, int tau, int b, int K) {
  double fsum = 0.0, rsum = 0.0, fb = 0.0;
  for (int q = 0; q < d; ++q) {
    const double f = fmax_exponent(r[2 * q], r[2 * q + 1]);
    fsum += f;
    rsum += r[2 * q];
    if (q == b) fb = f;
  }
  const double R = r[2 * b], I = r[2 * b + 1];
  if (tau == 0) return band_halfwidth(R, I, r[2 * d] + fsum - fb, K);
  const double c2 = r[2 * d + 1];
  if (c2 == -INFINITY) return -1;
  const int h = band_halfwidth(R, I, c2 + 2.0 * rsum + fsum - fb, K);
  return h < 0 ? h : min(h + 1, K / 2);
}

// circular distance of k from the centre c on a grid of K points
__device__ inline int circ_dist(int k, int c, int K) {
  int d = k - c;
  d = ((d % K) + K) % K;
  return d <= K / 2 ? d : K - d;
}

}  // namespace mp
