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
// circular distance > h from theta = 0; -1 when no point reaches the threshold.
__device__ inline int band_halfwidth(double R, double I, double offset, int K) {
  const double fmax = fmax_exponent(R, I);
  if (fmax + offset < kLogEps) return -1;
  const int half = K / 2;
  if (R <= 0.0) return half;
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  auto f = [&](int k) {
    const double t = kTwoPi * k / K;
    return -(1.0 - cos(t)) * R + fabs(sin(t)) * fabs(I) + offset;
  };
  if (f(half) >= kLogEps) return half;
  // f decreases on [theta*, pi]: search the last k >= k* with f(k) >= eps
  int lo = (int)floor(atan2(fabs(I), R) / kTwoPi * K);  // f(lo) may be >= eps
  int hi = half;                                      // f(hi) < eps
  if (f(lo) < kLogEps) return lo > 0 ? lo : 0;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (f(mid) >= kLogEps) lo = mid; else hi = mid;
  }
  return lo;
}

// circular distance of k from the centre c on a grid of K points
__device__ inline int circ_dist(int k, int c, int K) {
  int d = k - c;
  d = ((d % K) + K) % K;
  return d <= K / 2 ? d : K - d;
}

}  // namespace mp
