// Grouped photon-count observables: occupations, matrix-P parity weight and
// characteristic function (fused), deterministic sub-ensemble reduction, and
// the FP64 inverse DFT to P(m) with the sub-ensemble error sigma_T.
//
// Paper, eq. c-number-variable: per sample the pattern observable is
// G(m) = g0(n_S, m) prod_i n_i^c_i e^{-n_i} / c_i!, with
// g0 = (1 + pi_m e^{2 (n_S - n)}) / (1 + e^{-2n}).  Summed over the patterns of
// each bin (multinomial theorem) and over all counts with weights z_b^m_b,
//     chi(z) = (e^X + e^{-X - 2n}) / (1 + e^{-2n}) = cosh(n + X) / cosh(n),
//     X = sum_b n_b (z_b - 1),
// so the count distribution of the ensemble is the inverse DFT of the mean
// chi on z = e^{2 pi i k / K}.  Each evaluation also carries the window shift
// z^{-m_lo}, and both terms are formed as exp(real exponent) * cis(phase)
// with the exponent shifted by -log(1 + e^{-2|n|}) so that nothing overflows
// for either sign of n.  The positive-P variant (Appendix A) drops g0: chi = e^X.
//
// Sub-ensembles (Appendix A): samples g in [s N_S, (s+1) N_S) form
// sub-ensemble s; P is the mean of the sub-ensemble estimates and sigma_T
// their standard deviation over sqrt(N_R).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "chi.h"
#include "common.h"

namespace mp {

constexpr int kSBlk = 64;       // samples per workgroup of the fused kernel
constexpr int kCountThreads = 256;
constexpr int kEpt = 4;         // accumulator entries per thread per pass
constexpr int kMaxDist = MP_MAX_BINS + 1;
struct CountsParams {
  int M;
  int64_t ldm;
  int64_t E;        // samples in the chunk
  int64_t e0;       // global index of the chunk's first sample
  int64_t ns;       // samples per sub-ensemble
  int d;
  int mode;         // mp_bin_mode
  int est;          // mp_estimator
  int n_runs;
  int run_lo[MP_MAX_RUNS], run_hi[MP_MAX_RUNS], run_bin[MP_MAX_RUNS];
  int n_dist;
  int dist_src[kMaxDist];  // bin index feeding each distribution, -1 = total
  int m_lo[kMaxDist], K[kMaxDist];
  int off[kMaxDist + 1];   // entry offsets (prefix sums of K)
  int entries;
  // block -> (sub-ensemble, tile) arithmetic
  int64_t s_first, s_last;
  int t_first, t_mid, t_last, n_mid;
};

__host__ __device__ inline int64_t sub_lo(const CountsParams& p, int64_t s) {
  int64_t a = s * p.ns;
  return a > p.e0 ? a : p.e0;
}
__host__ __device__ inline int64_t sub_hi(const CountsParams& p, int64_t s) {
  int64_t a = (s + 1) * p.ns, b = p.e0 + p.E;
  return a < b ? a : b;
}

// Block b -> sub-ensemble s and global sample range [lo, hi).
__device__ inline void block_samples(const CountsParams& p, int b, int64_t& s, int64_t& lo,
                                     int64_t& hi) {
  int tile;
  if (b < p.t_first) {
    s = p.s_first;
    tile = b;
  } else {
    b -= p.t_first;
    if (b < p.n_mid * p.t_mid) {
      s = p.s_first + 1 + b / p.t_mid;
      tile = b % p.t_mid;
    } else {
      s = p.s_last;
      tile = b - p.n_mid * p.t_mid;
    }
  }
  const int64_t a = sub_lo(p, s), z = sub_hi(p, s);
  lo = a + (int64_t)tile * kSBlk;
  hi = lo + kSBlk < z ? lo + kSBlk : z;
}

// Occupations of one sample: nb[b] = sum of n'_j over the modes of bin b
// (every lane holds the wave-reduced sums).
template <typename CT>
__device__ inline void sample_bin_sums(const CountsParams& p, const CT* __restrict__ ca,
                                       const CT* __restrict__ cb, int lane,
                                       double (&nb)[MP_MAX_BINS][2]) {
#pragma unroll
  for (int b = 0; b < MP_MAX_BINS; ++b) nb[b][0] = nb[b][1] = 0.0;
  for (int q = 0; q < p.n_runs; ++q) {
    double re, im;
    run_sum<CT>(ca, cb, p.ldm, p.run_lo[q], p.run_hi[q], lane, re, im);
    const int bq = p.run_bin[q];
#pragma unroll
    for (int b = 0; b < MP_MAX_BINS; ++b)
      if (b == bq) {
        nb[b][0] += re;
        nb[b][1] += im;
      }
  }
}

// Occupation feeding distribution q: bin dist_src[q], or the total over the
// d bins when dist_src[q] = -1.
__device__ inline void dist_occupation(const CountsParams& p, const double (&nb)[MP_MAX_BINS][2],
                                       int q, double& vr, double& vi) {
  double tr = 0.0, ti = 0.0;
#pragma unroll
  for (int b = 0; b < MP_MAX_BINS; ++b)
    if (b < p.d) {
      tr += nb[b][0];
      ti += nb[b][1];
    }
  vr = tr;
  vi = ti;
  const int src = p.dist_src[q];
#pragma unroll
  for (int b = 0; b < MP_MAX_BINS; ++b)
    if (b == src) {
      vr = nb[b][0];
      vi = nb[b][1];
    }
}

// Sources of a sample's bin sums for counts_fused: the propagated amplitudes C
// (mp_propagate) or the per-block partials of the occupation-fused GEMM.
template <typename CT>
struct FromC {
  const CT* C;
  __device__ inline void bin_sums(const CountsParams& p, int64_t k, int lane,
                                  double (&nb)[MP_MAX_BINS][2]) const {
    const int64_t ldc = 2 * p.ldm;
    sample_bin_sums<CT>(p, C + k * ldc, C + (p.E + k) * ldc, lane, nb);
  }
};

struct FromPartials {
  const float* part;  // FusedOut layout, E = p.E
  __device__ inline void bin_sums(const CountsParams& p, int64_t k, int lane,
                                  double (&nb)[MP_MAX_BINS][2]) const {
#pragma unroll
    for (int b = 0; b < MP_MAX_BINS; ++b) nb[b][0] = nb[b][1] = 0.0;
    int slot0 = 0;
    for (int q = 0; q < p.n_runs; ++q) {
      const int nblk = run_blocks(p.run_lo[q], p.run_hi[q]);
      double sr, si;
      run_sum_partials(part, p.E, slot0, nblk, k, lane, sr, si);
      const int bq = p.run_bin[q];
#pragma unroll
      for (int b = 0; b < MP_MAX_BINS; ++b)
        if (b == bq) {
          nb[b][0] += sr;
          nb[b][1] += si;
        }
      slot0 += nblk;
    }
  }
};

template <typename Src, bool F64>
__global__ __launch_bounds__(kCountThreads) void counts_fused(CountsParams p, Src src,
                                                              const double* __restrict__ nglob,
                                                              double* __restrict__ partials) {
  __shared__ double s_nb[kSBlk][kMaxDist][2];
  __shared__ double s_c1[kSBlk], s_c2[kSBlk];
  __shared__ int s_skip2[kSBlk];
  int64_t sub, lo, hi;
  block_samples(p, blockIdx.x, sub, lo, hi);
  const int nsmp = (int)(hi - lo);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  // Phase 1: per-sample bin occupations n_b (wave per sample, lanes over modes
  // or over the fused GEMM's block partials).
  for (int i = wave; i < nsmp; i += kCountThreads / 64) {
    const int64_t k = lo + i - p.e0;  // chunk-local sample index
    double nb[MP_MAX_BINS][2];
    src.bin_sums(p, k, lane, nb);
    if (lane == 0) {
      for (int q = 0; q < p.n_dist; ++q) dist_occupation(p, nb, q, s_nb[i][q][0], s_nb[i][q][1]);
      const double n = nglob[k];
      bool finite = p.est == MP_PLUS_P || isfinite(n);
      for (int q = 0; q < p.n_dist; ++q)
        finite = finite && isfinite(s_nb[i][q][0]) && isfinite(s_nb[i][q][1]);
      if (p.est == MP_PLUS_P) {
        s_c1[i] = finite ? 0.0 : __builtin_nan("");
        s_c2[i] = 0.0;
        s_skip2[i] = 1;
      } else {
        parity_log_weights(n, finite, s_c1[i], s_c2[i]);
        // |e^{-X}| <= e^{2 |n_b|}: skip the parity partner when it underflows
        double mx = 0.0;
        for (int q = 0; q < p.n_dist; ++q) {
          const double a = sqrt(s_nb[i][q][0] * s_nb[i][q][0] + s_nb[i][q][1] * s_nb[i][q][1]);
          mx = a > mx ? a : mx;
        }
        s_skip2[i] = (2.0 * mx + s_c2[i] < -800.0) ? 1 : 0;
      }
    }
  }
  __syncthreads();

  // Phase 2: characteristic function on the window grid, summed over samples.
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  for (int base = 0; base < p.entries; base += kCountThreads * kEpt) {
    double ar[kEpt], ai[kEpt], cm1[kEpt], sn[kEpt], thl[kEpt];
    int dq[kEpt];
#pragma unroll
    for (int u = 0; u < kEpt; ++u) {
      ar[u] = ai[u] = 0.0;
      const int e = base + threadIdx.x + u * kCountThreads;
      int q = 0;
      while (q + 1 < p.n_dist && e >= p.off[q + 1]) ++q;
      dq[u] = (e < p.entries) ? q : -1;
      const int K = p.K[q];
      const int kk = (e < p.entries) ? e - p.off[q] : 0;
      const double th = kTwoPi * (double)kk / (double)K;
      double s, c;
      sincos(th, &s, &c);
      sn[u] = s;
      cm1[u] = -2.0 * sin(0.5 * th) * sin(0.5 * th);  // cos(th) - 1 without cancellation
      const int64_t red = ((int64_t)kk * (int64_t)p.m_lo[q]) % K;
      thl[u] = kTwoPi * (double)red / (double)K;     // th * m_lo reduced mod 2 pi
    }
    for (int i = 0; i < nsmp; ++i) {
      const double c1 = s_c1[i], c2 = s_c2[i];
      const bool skip2 = s_skip2[i] != 0;
#pragma unroll
      for (int u = 0; u < kEpt; ++u) {
        if (dq[u] < 0) continue;
        const double nr = s_nb[i][dq[u]][0], ni = s_nb[i][dq[u]][1];
        // log-magnitudes of the two terms are xr + c1 and c2 - xr; a term
        // below e^kLogEps is skipped (a NaN one is kept: it must reach the sums)
        const double xr = cm1[u] * nr - sn[u] * ni;
        const bool t1 = !(xr + c1 <= kLogEps), t2 = !skip2 && !(c2 - xr <= kLogEps);
        if (!(t1 || t2)) continue;
        const double xi = cm1[u] * ni + sn[u] * nr;
        double tr, ti;
        if (t1) {
          cis_exp<F64>(xr + c1, xi - thl[u], tr, ti);
          ar[u] += tr;
          ai[u] += ti;
        }
        if (t2) {
          cis_exp<F64>(c2 - xr, -xi - thl[u], tr, ti);
          ar[u] += tr;
          ai[u] += ti;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kEpt; ++u) {
      const int e = base + threadIdx.x + u * kCountThreads;
      if (e < p.entries) {
        double* dst = partials + ((int64_t)blockIdx.x * p.entries + e) * 2;
        dst[0] = ar[u];
        dst[1] = ai[u];
      }
    }
  }
}

// acc[s] += sum over the tiles of s of the partials, in tile order.
__global__ void counts_reduce(CountsParams p, const double* __restrict__ partials,
                              double* __restrict__ acc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.entries) return;
  const int64_t s = p.s_first + blockIdx.y;
  int b0, nt;
  if (s == p.s_first) {
    b0 = 0;
    nt = p.t_first;
  } else if (s == p.s_last) {
    b0 = p.t_first + p.n_mid * p.t_mid;
    nt = p.t_last;
  } else {
    b0 = p.t_first + (int)(s - p.s_first - 1) * p.t_mid;
    nt = p.t_mid;
  }
  double re = 0.0, im = 0.0;
  for (int t = 0; t < nt; ++t) {
    const double* src = partials + ((int64_t)(b0 + t) * p.entries + e) * 2;
    re += src[0];
    im += src[1];
  }
  double* dst = acc + (s * (int64_t)p.entries + e) * 2;
  dst[0] += re;
  dst[1] += im;
}

// ---------------------------------------------------------------- joint, d = 2

// Joint distribution of two bins.  Per sample the generating function
// factorises,
//     chi(z1, z2) = e^{c1} u1(z1) u2(z2) + e^{c2} v1(z1) v2(z2),
//     u_b = e^{X_b} z_b^{-m_lo_b},  v_b = e^{-X_b} z_b^{-m_lo_b},
// so the sum over a sub-ensemble is a sum of rank-1 outer products.  For
// theta in [0, pi] the exponent of |u_b| is
//     f_b(theta) = -(1 - cos theta) Re n_b + |sin theta| |Im n_b|
// (v_b: the same about theta = pi, plus 2 Re n_b), which rises to its maximum
// at tan theta* = |Im n_b| / Re n_b and then falls monotonically.  Each sample
// gets, per term and bin, the half-width of the band around theta = 0 (u) or
// pi (v) outside which its term is below e^-46 (~1e-20) for every value of the
// other bin; the chunk's band is the maximum over its samples.  Terms outside
// the band are bounded by that threshold, not approximated.


struct Joint2Params {
  int M;
  int64_t ldm, E, e0, ns;
  int est;
  int n_runs;
  int run_lo[MP_MAX_RUNS], run_hi[MP_MAX_RUNS], run_bin[MP_MAX_RUNS];
  int m_lo[2], K[2];
  int64_t s_first, s_last;
};

// Per-sample record (one wave per sample, lane 0 writes): n1, n2 (complex),
// c1, c2 (c2 = -inf for +P; both NaN for a sample that is not finite).
// record_bands then sets the chunk's bands
// band[0..3] = u1, u2, v1, v2 half-widths (atomic max, -1 = empty).
// PART: the bin sums come from the occupation-fused GEMM's partials (slots in
// run order) instead of the propagated amplitudes C.
template <typename CT, bool PART>
__device__ inline void joint2_sample(const Joint2Params& p, const CT* __restrict__ C,
                                     const float* __restrict__ part,
                                     const double* __restrict__ nglob, double* __restrict__ rec,
                                     int64_t k, int lane) {
  const int64_t ldc = 2 * p.ldm;
  const CT* ca = PART ? nullptr : C + k * ldc;
  const CT* cb = PART ? nullptr : C + (p.E + k) * ldc;
  double R1 = 0.0, I1 = 0.0, R2 = 0.0, I2 = 0.0;
  int slot0 = 0;
  for (int q = 0; q < p.n_runs; ++q) {
    double re, im;
    if constexpr (PART) {
      const int nblk = run_blocks(p.run_lo[q], p.run_hi[q]);
      run_sum_partials(part, p.E, slot0, nblk, k, lane, re, im);
      slot0 += nblk;
    } else {
      run_sum<CT>(ca, cb, p.ldm, p.run_lo[q], p.run_hi[q], lane, re, im);
    }
    const bool first = p.run_bin[q] == 0;
    R1 += first ? re : 0.0;
    I1 += first ? im : 0.0;
    R2 += first ? 0.0 : re;
    I2 += first ? 0.0 : im;
  }
  if (lane != 0) return;
  const double n = nglob[k];
  const bool sums_finite = isfinite(R1) && isfinite(I1) && isfinite(R2) && isfinite(I2);
  double c1 = 0.0, c2 = -INFINITY;
  if (p.est != MP_PLUS_P)
    parity_log_weights(n, sums_finite && isfinite(n), c1, c2);
  else if (!sums_finite)
    c1 = c2 = __builtin_nan("");
  double* r = rec + k * 6;
  r[0] = R1;
  r[1] = I1;
  r[2] = R2;
  r[3] = I2;
  r[4] = c1;
  r[5] = c2;
}

template <typename CT, bool PART>
__global__ __launch_bounds__(256) void joint2_occupations(Joint2Params p, const CT* __restrict__ C,
                                                          const float* __restrict__ part,
                                                          const double* __restrict__ nglob,
                                                          double* __restrict__ rec) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * (4 * kOccPerWave) + wave;
  for (int j = 0; j < kOccPerWave; ++j) {
    const int64_t k = base + 4 * j;
    if (k >= p.E) return;
    joint2_sample<CT, PART>(p, C, part, nglob, rec, k, lane);
  }
}

__global__ void joint2_band_init(int* band) {
  if (threadIdx.x < 4) band[threadIdx.x] = -1;
}

// Box half-widths from the per-sample records (layout of record_band): block
// row blockIdx.y = tau d + b, one sample per thread, a wave maximum, then one
// atomic maximum per wave into band[tau * band_stride + b].
__global__ __launch_bounds__(256) void record_bands(const double* __restrict__ rec, int64_t E,
                                                    int d, int K0, int K1, int K2, int K3,
                                                    int band_stride, int* __restrict__ band) {
  const int tau = blockIdx.y / d, b = blockIdx.y % d;
  const int K = b == 0 ? K0 : (b == 1 ? K1 : (b == 2 ? K2 : K3));
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int h = k < E ? record_band(rec + k * (2 * d + 2), d, tau, b, K) : -1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) h = max(h, __shfl_xor(h, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(&band[tau * band_stride + b], h);
}

mp_status record_bands_launch(const double* rec, int64_t E, int d, const int32_t* K,
                              int band_stride, int* band, hipStream_t stream) {
  hipLaunchKernelGGL(record_bands, dim3((unsigned)((E + 255) / 256), (unsigned)(2 * d)), dim3(256),
                     0, stream, rec, E, d, K[0], d > 1 ? K[1] : 1, d > 2 ? K[2] : 1,
                     d > 3 ? K[3] : 1, band_stride, band);
  MP_HIP_LAUNCH_CHECK("mp_binned_counts box bounds launch");
  return MP_OK;
}

template <bool F64>
__device__ inline void factor(double R, double I, double c, int k, int K, int m_lo, double sign,
                              double& fr, double& fi) {
  // e^{sign X(theta_k) + c} z^{-m_lo}, X = n (e^{i theta} - 1)
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  const double th = kTwoPi * (double)k / (double)K;
  const double sh = sin(0.5 * th);
  const double cm1 = -2.0 * sh * sh, sn = sin(th);
  const double xr = cm1 * R - sn * I, xi = cm1 * I + sn * R;
  const int64_t red = ((int64_t)k * (int64_t)m_lo) % K;
  const double thl = kTwoPi * (double)red / (double)K;
  cis_exp<F64>(sign * xr + c, sign * xi - thl, fr, fi);
}

constexpr int kJT = 16;    // output tile kJT x kJT per workgroup
constexpr int kJS = 64;    // samples staged per round

// acc[s][k1][k2] += sum over the chunk's samples of sub-ensemble s of the
// band-limited outer products.  Grid: (tiles over K1 x K2, sub-ensembles).
template <bool F64>
__global__ __launch_bounds__(256) void joint2_accumulate(Joint2Params p, const double* __restrict__ rec,
                                                         const int* __restrict__ band,
                                                         double* __restrict__ acc) {
  __shared__ double f1[kJS][kJT][2], f2[kJS][kJT][2];
  const int K1 = p.K[0], K2 = p.K[1];
  const int tiles2 = (K2 + kJT - 1) / kJT;
  const int t1 = blockIdx.x / tiles2, t2 = blockIdx.x % tiles2;
  const int64_t s = p.s_first + blockIdx.y;
  const int tid = threadIdx.x, r1 = tid / kJT, r2 = tid % kJT;
  const int k1 = t1 * kJT + r1, k2 = t2 * kJT + r2;
  int64_t lo = s * p.ns, hi = (s + 1) * p.ns;
  lo = lo > p.e0 ? lo : p.e0;
  hi = hi < p.e0 + p.E ? hi : p.e0 + p.E;
  double ar = 0.0, ai = 0.0;
  for (int term = 0; term < 2; ++term) {
    const int h1 = band[term == 0 ? 0 : 2], h2 = band[term == 0 ? 1 : 3];
    if (h1 < 0 || h2 < 0) continue;
    const int c1 = term == 0 ? 0 : K1 / 2, c2 = term == 0 ? 0 : K2 / 2;
    // does the tile meet the band box?  (tile-uniform decision)
    bool any1 = false, any2 = false;
    for (int q = 0; q < kJT; ++q) {
      any1 |= (t1 * kJT + q < K1) && circ_dist(t1 * kJT + q, c1, K1) <= h1;
      any2 |= (t2 * kJT + q < K2) && circ_dist(t2 * kJT + q, c2, K2) <= h2;
    }
    if (!any1 || !any2) continue;
    const double sign = term == 0 ? 1.0 : -1.0;
    const bool mine = k1 < K1 && k2 < K2 && circ_dist(k1, c1, K1) <= h1 && circ_dist(k2, c2, K2) <= h2;
    for (int64_t base = lo; base < hi; base += kJS) {
      const int nsmp = (int)(hi - base < kJS ? hi - base : kJS);
      // stage the factors of nsmp samples for the tile's kJT k1 and kJT k2 values
      for (int w = tid; w < 2 * kJS * kJT; w += 256) {
        const int which = w / (kJS * kJT), rem = w % (kJS * kJT);
        const int i = rem / kJT, q = rem % kJT;
        double fr = 0.0, fi = 0.0;
        if (i < nsmp) {
          const double* r = rec + (base + i - p.e0) * 6;
          const double cterm = term == 0 ? r[4] : r[5];
          // the product's log-magnitude at the band centre (c, or c + 2 Re n_1
          // + 2 Re n_2 for the second term) is shared evenly between the two
          // factors, so neither overflows while the other underflows in FP32
          const double share = 0.5 * (cterm + (term == 0 ? 0.0 : 2.0 * (r[0] + r[2])));
          if (which == 0) {
            const int kk = t1 * kJT + q;
            if (kk < K1 && cterm != -INFINITY)
              factor<F64>(r[0], r[1], share - (term == 0 ? 0.0 : 2.0 * r[0]), kk, K1, p.m_lo[0],
                          sign, fr, fi);
          } else {
            const int kk = t2 * kJT + q;
            if (kk < K2 && cterm != -INFINITY)
              factor<F64>(r[2], r[3], share - (term == 0 ? 0.0 : 2.0 * r[2]), kk, K2, p.m_lo[1],
                          sign, fr, fi);
          }
        }
        double(*dst)[kJT][2] = which == 0 ? f1 : f2;
        dst[i][q][0] = fr;
        dst[i][q][1] = fi;
      }
      __syncthreads();
      if (mine) {
        for (int i = 0; i < nsmp; ++i) {
          const double xr = f1[i][r1][0], xi = f1[i][r1][1];
          const double yr = f2[i][r2][0], yi = f2[i][r2][1];
          ar += xr * yr - xi * yi;
          ai += xr * yi + xi * yr;
        }
      }
      __syncthreads();
    }
  }
  if (k1 < K1 && k2 < K2 && (ar != 0.0 || ai != 0.0)) {
    double* dst = acc + ((int64_t)s * K1 * K2 + (int64_t)k1 * K2 + k2) * 2;
    dst[0] += ar;
    dst[1] += ai;
  }
}

// part != nullptr: the bin sums come from the occupation-fused GEMM's partials
// (runs in the order built here, as fused_runs builds them) and C is unused.
mp_status joint2_launch(int32_t M, int64_t E, const void* C, const double* n, mp_precision prec,
                        mp_estimator est, const int32_t* bin_of_mode, const int32_t* m_lo,
                        const int32_t* K, int32_t n_sub, int64_t ns, int64_t e0, double* acc,
                        void* ws, size_t ws_bytes, hipStream_t stream, const float* part) {
  Joint2Params p{};
  p.M = M;
  p.ldm = ld_modes(M);
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  p.est = est;
  p.n_runs = 0;
  for (int j = 0; j < M;) {
    const int b = bin_of_mode[j];
    int j2 = j + 1;
    while (j2 < M && bin_of_mode[j2] == b) ++j2;
    if (b >= 0) {
      MP_CHECK_ARG(p.n_runs < MP_MAX_RUNS, MP_ERR_UNSUPPORTED,
                   "mp_binned_counts: bins form more than %d contiguous mode runs", MP_MAX_RUNS);
      p.run_lo[p.n_runs] = j;
      p.run_hi[p.n_runs] = j2;
      p.run_bin[p.n_runs] = b;
      ++p.n_runs;
    }
    j = j2;
  }
  for (int b = 0; b < 2; ++b) {
    p.m_lo[b] = m_lo[b];
    p.K[b] = K[b];
  }
  p.s_first = e0 / ns;
  p.s_last = (e0 + E - 1) / ns;
  MP_CHECK_ARG(p.s_last < n_sub, MP_ERR_SHAPE,
               "mp_binned_counts: samples [%lld, %lld) exceed n_sub * samples_per_sub = %lld",
               (long long)e0, (long long)(e0 + E), (long long)n_sub * ns);
  const size_t need = 256 + (size_t)E * 48;
  MP_CHECK_ARG(ws && ws_bytes >= need, MP_ERR_WORKSPACE,
               "mp_binned_counts: workspace of %zu bytes needed, %zu given", need, ws_bytes);
  int* band = (int*)ws;
  double* rec = (double*)((char*)ws + 256);
  hipLaunchKernelGGL(joint2_band_init, dim3(1), dim3(64), 0, stream, band);
  const unsigned blocks = (unsigned)((E + 4 * kOccPerWave - 1) / (4 * kOccPerWave));
  if (part)
    hipLaunchKernelGGL((joint2_occupations<float, true>), dim3(blocks), dim3(256), 0, stream, p,
                       (const float*)nullptr, part, n, rec);
  else if (prec == MP_FP64)
    hipLaunchKernelGGL((joint2_occupations<double, false>), dim3(blocks), dim3(256), 0, stream, p,
                       (const double*)C, (const float*)nullptr, n, rec);
  else
    hipLaunchKernelGGL((joint2_occupations<float, false>), dim3(blocks), dim3(256), 0, stream, p,
                       (const float*)C, (const float*)nullptr, n, rec);
  MP_HIP_LAUNCH_CHECK("mp_binned_counts joint occupations launch");
  const mp_status sb = record_bands_launch(rec, E, 2, K, 2, band, stream);
  if (sb != MP_OK) return sb;
  const unsigned tiles = (unsigned)(((K[0] + kJT - 1) / kJT) * ((K[1] + kJT - 1) / kJT));
  const unsigned nst = (unsigned)(p.s_last - p.s_first + 1);
  if (prec == MP_FP64)
    hipLaunchKernelGGL(joint2_accumulate<true>, dim3(tiles, nst), dim3(256), 0, stream, p, rec,
                       band, acc);
  else
    hipLaunchKernelGGL(joint2_accumulate<false>, dim3(tiles, nst), dim3(256), 0, stream, p, rec,
                       band, acc);
  MP_HIP_LAUNCH_CHECK("mp_binned_counts joint accumulate launch");
  return MP_OK;
}

// ---------------------------------------------------------------- finalize

struct FinalParams {
  int n_dist;
  int K[kMaxDist];
  int off[kMaxDist + 1];
  int entries;
  int n_sub;
  double inv_ns;
};

// One workgroup per output point; threads split the frequency sum, and the
// sub-ensemble estimates are folded with Welford's update.
__global__ __launch_bounds__(256) void counts_finalize(FinalParams p, const double* __restrict__ acc,
                                                       double* __restrict__ P_re,
                                                       double* __restrict__ P_im,
                                                       double* __restrict__ sigma) {
  __shared__ double red_r[256], red_i[256];
  const int e = blockIdx.x;
  int q = 0;
  while (q + 1 < p.n_dist && e >= p.off[q + 1]) ++q;
  const int K1 = p.K[q], l1 = e - p.off[q], nterms = K1;
  double mean_r = 0.0, mean_i = 0.0, m2 = 0.0;
  for (int s = 0; s < p.n_sub; ++s) {
    const double* a = acc + ((int64_t)s * p.entries + p.off[q]) * 2;
    double sr = 0.0, si = 0.0;
    for (int t = threadIdx.x; t < nterms; t += 256) {
      const double frac = (double)(((int64_t)t * l1) % K1) / K1;
      double sw, cw;
      sincospi(-2.0 * frac, &sw, &cw);
      const double xr = a[2 * t], xi = a[2 * t + 1];
      sr += xr * cw - xi * sw;
      si += xr * sw + xi * cw;
    }
    red_r[threadIdx.x] = sr;
    red_i[threadIdx.x] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        red_r[threadIdx.x] += red_r[threadIdx.x + w];
        red_i[threadIdx.x] += red_i[threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double ps_r = red_r[0] * p.inv_ns / nterms, ps_i = red_i[0] * p.inv_ns / nterms;
      const double dr = ps_r - mean_r;
      mean_r += dr / (s + 1);
      mean_i += (ps_i - mean_i) / (s + 1);
      m2 += dr * (ps_r - mean_r);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    P_re[e] = mean_r;
    if (P_im) P_im[e] = mean_i;
    sigma[e] = p.n_sub > 1 ? sqrt(m2 / (p.n_sub - 1) / p.n_sub) : __builtin_nan("");
  }
}

size_t jointd_workspace(int32_t d, const int32_t* K, int64_t E);
size_t jointd_finalize_workspace(int32_t d, const int32_t* K);
mp_status jointd_launch(int32_t M, int64_t E, const void* C, const double* n, mp_precision prec,
                        mp_estimator est, int32_t d, const int32_t* bin_of_mode,
                        const int32_t* m_lo, const int32_t* K, int32_t n_sub, int64_t ns,
                        int64_t e0, double* acc, void* ws, size_t ws_bytes, hipStream_t stream,
                        const float* part);
mp_status jointd_finalize(int32_t d, const int32_t* K, int32_t n_sub, int64_t ns,
                          const double* acc, double* P_re, double* P_im, double* sigma, void* ws,
                          size_t ws_bytes, hipStream_t stream);

size_t finalize_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub) {
  if (mode == MP_JOINT && d >= 2) return jointd_finalize_workspace(d, K);
  return 0;
}

// ---------------------------------------------------------------- host side

static int64_t entries_of(int d, mp_bin_mode mode, const int32_t* K) {
  if (mode == MP_JOINT) {
    int64_t e = 1;
    for (int b = 0; b < d; ++b) e *= K[b];
    return e;
  }
  int nd = d + (mode == MP_MARGINALS_AND_TOTAL ? 1 : 0);
  int64_t e = 0;
  for (int q = 0; q < nd; ++q) e += K[q];
  return e;
}

int64_t acc_entries(int32_t d, mp_bin_mode mode, const int32_t* K) {
  if (!K || d < 1 || d > MP_MAX_BINS) return -1;
  return entries_of(d, mode, K);
}

// Fills the tiling part of the parameters; returns the number of blocks.
static int64_t plan_tiles(CountsParams& p) {
  p.s_first = p.e0 / p.ns;
  p.s_last = (p.e0 + p.E - 1) / p.ns;
  auto tiles = [&](int64_t s) { return (int)((sub_hi(p, s) - sub_lo(p, s) + kSBlk - 1) / kSBlk); };
  p.t_first = tiles(p.s_first);
  p.t_mid = (int)((p.ns + kSBlk - 1) / kSBlk);
  p.n_mid = p.s_last > p.s_first + 1 ? (int)(p.s_last - p.s_first - 1) : 0;
  p.t_last = p.s_last != p.s_first ? tiles(p.s_last) : 0;
  return (int64_t)p.t_first + (int64_t)p.n_mid * p.t_mid + p.t_last;
}

// Contiguous mode runs of the bins (modes with bin -1 are skipped); false if
// there are more than MP_MAX_RUNS.
static bool fill_runs(CountsParams& p, int32_t M, const int32_t* bin_of_mode) {
  p.n_runs = 0;
  for (int j = 0; j < M;) {
    const int b = bin_of_mode[j];
    int j2 = j + 1;
    while (j2 < M && bin_of_mode[j2] == b) ++j2;
    if (b >= 0) {
      if (p.n_runs >= MP_MAX_RUNS) return false;
      p.run_lo[p.n_runs] = j;
      p.run_hi[p.n_runs] = j2;
      p.run_bin[p.n_runs] = b;
      ++p.n_runs;
    }
    j = j2;
  }
  return true;
}

size_t binned_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int64_t E, int32_t n_sub,
                        int64_t ns, int64_t e0) {
  if (!K || d < 1 || d > MP_MAX_BINS || E < 1 || ns < 1 || e0 < 0) return 0;
  if (mode == MP_JOINT && d == 2) return 256 + (size_t)E * 48;
  if (mode == MP_JOINT && d >= 3) return jointd_workspace(d, K, E);
  CountsParams p{};
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  const int64_t blocks = plan_tiles(p);
  return (size_t)blocks * (size_t)entries_of(d, mode, K) * 16;
}

// Parameters of a d = 1, marginal or marginal + total accumulation.
static mp_status setup_counts(CountsParams& p, const char* who, int32_t M, int64_t E, int32_t d,
                              const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                              const int32_t* K, int32_t n_sub, int64_t ns, int64_t e0,
                              mp_estimator est, int64_t& blocks) {
  p.M = M;
  p.ldm = ld_modes(M);
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  p.d = d;
  p.mode = mode;
  p.est = est;
  if (!fill_runs(p, M, bin_of_mode)) {
    set_error("%s: bins form more than %d contiguous mode runs", who, MP_MAX_RUNS);
    return MP_ERR_UNSUPPORTED;
  }
  p.n_dist = mode == MP_JOINT ? 1 : d + (mode == MP_MARGINALS_AND_TOTAL ? 1 : 0);
  p.off[0] = 0;
  for (int q = 0; q < p.n_dist; ++q) {
    p.dist_src[q] = q < d ? q : -1;
    p.m_lo[q] = m_lo[q];
    p.K[q] = K[q];
    p.off[q + 1] = p.off[q] + K[q];
  }
  p.entries = p.off[p.n_dist];
  blocks = plan_tiles(p);
  if (p.s_last >= n_sub) {
    set_error("%s: samples [%lld, %lld) exceed n_sub * samples_per_sub = %lld", who,
              (long long)e0, (long long)(e0 + E), (long long)n_sub * ns);
    return MP_ERR_SHAPE;
  }
  if (blocks >= 0x7FFFFFFF) {
    set_error("%s: chunk too large", who);
    return MP_ERR_UNSUPPORTED;
  }
  return MP_OK;
}

mp_status binned_counts_launch(int32_t M, int64_t E, const void* C, const double* n,
                               mp_precision prec, mp_estimator est, int32_t d,
                               const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                               const int32_t* K, int32_t n_sub, int64_t ns, int64_t e0,
                               double* acc, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (mode == MP_JOINT && d == 2)
    return joint2_launch(M, E, C, n, prec, est, bin_of_mode, m_lo, K, n_sub, ns, e0, acc, ws,
                         ws_bytes, stream, nullptr);
  if (mode == MP_JOINT && d >= 3)
    return jointd_launch(M, E, C, n, prec, est, d, bin_of_mode, m_lo, K, n_sub, ns, e0, acc, ws,
                         ws_bytes, stream, nullptr);
  MP_CHECK_ARG(mode != MP_JOINT || d == 1, MP_ERR_UNSUPPORTED,
               "mp_binned_counts: joint distributions need d <= 4 (d = %d)", d);
  CountsParams p{};
  int64_t blocks = 0;
  const mp_status st = setup_counts(p, "mp_binned_counts", M, E, d, bin_of_mode, mode, m_lo, K,
                                    n_sub, ns, e0, est, blocks);
  if (st != MP_OK) return st;
  const size_t need = (size_t)blocks * (size_t)p.entries * 16;
  MP_CHECK_ARG(ws && ws_bytes >= need, MP_ERR_WORKSPACE,
               "mp_binned_counts: workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (prec == MP_FP64) {
    hipLaunchKernelGGL((counts_fused<FromC<double>, true>), dim3((unsigned)blocks),
                       dim3(kCountThreads), 0, stream, p, FromC<double>{(const double*)C}, n,
                       (double*)ws);
  } else {
    hipLaunchKernelGGL((counts_fused<FromC<float>, false>), dim3((unsigned)blocks),
                       dim3(kCountThreads), 0, stream, p, FromC<float>{(const float*)C}, n,
                       (double*)ws);
  }
  MP_HIP_LAUNCH_CHECK("mp_binned_counts fused launch");
  const int ns_touched = (int)(p.s_last - p.s_first + 1);
  hipLaunchKernelGGL(counts_reduce, dim3((p.entries + 255) / 256, ns_touched), dim3(256), 0, stream,
                     p, (const double*)ws, acc);
  MP_HIP_LAUNCH_CHECK("mp_binned_counts reduce launch");
  return MP_OK;
}

mp_status gemm_fused_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                            const void* ab, const FusedOut& fo, hipStream_t stream);

// Workspace of mp_propagate_counts: the GEMM's partials (slots x E x 16 B),
// then the counts kernel's per-block partials.
static void propagate_counts_sizes(const CountsParams& p, int64_t blocks, size_t& part_bytes,
                                   size_t& total) {
  int slot_off[MP_MAX_RUNS];
  const int64_t slots = fused_slots(p.n_runs, p.run_lo, p.run_hi, slot_off);
  part_bytes = ((size_t)slots * (size_t)p.E * 16 + 255) / 256 * 256;
  total = part_bytes + (size_t)blocks * (size_t)p.entries * 16;
}

// Runs of a bin partition for the fused partials of a joint distribution of
// d >= 2 bins: maximal ranges of modes with one bin >= 0, in mode order (the
// order in which the joint paths walk them).
static mp_status fused_runs(int32_t M, const int32_t* bin_of_mode, FusedOut& fo) {
  fo.n_runs = 0;
  for (int j = 0; j < M;) {
    const int b = bin_of_mode[j];
    int j2 = j + 1;
    while (j2 < M && bin_of_mode[j2] == b) ++j2;
    if (b >= 0) {
      MP_CHECK_ARG(fo.n_runs < MP_MAX_RUNS, MP_ERR_UNSUPPORTED,
                   "mp_propagate_counts: bins form more than %d contiguous mode runs", MP_MAX_RUNS);
      fo.run_lo[fo.n_runs] = j;
      fo.run_hi[fo.n_runs] = j2;
      ++fo.n_runs;
    }
    j = j2;
  }
  fused_slots(fo.n_runs, fo.run_lo, fo.run_hi, fo.slot_off);
  return MP_OK;
}

static size_t joint_part_bytes(const FusedOut& fo, int64_t E) {
  const int64_t slots = fo.n_runs ? fo.slot_off[fo.n_runs - 1] +
                                        run_blocks(fo.run_lo[fo.n_runs - 1], fo.run_hi[fo.n_runs - 1])
                                  : 0;
  return ((size_t)slots * (size_t)E * 16 + 255) / 256 * 256;
}

size_t propagate_counts_workspace(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                                  mp_bin_mode mode, const int32_t* K, int32_t n_sub, int64_t ns,
                                  int64_t e0) {
  if (mode == MP_JOINT && d >= 2) {  // the partials, then the joint path's workspace
    FusedOut fo{};
    if (fused_runs(M, bin_of_mode, fo) != MP_OK) return 0;
    return joint_part_bytes(fo, E) + binned_workspace(d, mode, K, E, n_sub, ns, e0);
  }
  CountsParams p{};
  std::vector<int32_t> m_lo(MP_MAX_BINS + 1, 0);
  int64_t blocks = 0;
  if (setup_counts(p, "mp_propagate_counts_workspace", M, E, d, bin_of_mode, mode, m_lo.data(), K,
                   n_sub, ns, e0, MP_MATRIX_P, blocks) != MP_OK)
    return 0;
  size_t part_bytes, total;
  propagate_counts_sizes(p, blocks, part_bytes, total);
  return total;
}

// The occupation-fused GEMM's output description for a chunk of E samples:
// the runs of the bin partition, their slots, and the partials at the start of
// ws (the counts kernel's per-block partials follow them).
mp_status fused_out_setup(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                          mp_bin_mode mode, const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                          int64_t ns, int64_t e0, mp_estimator est, void* ws, size_t ws_bytes,
                          FusedOut& fo) {
  if (mode == MP_JOINT && d >= 2) {
    fo = FusedOut{};
    const mp_status sr = fused_runs(M, bin_of_mode, fo);
    if (sr != MP_OK) return sr;
    const size_t total =
        joint_part_bytes(fo, E) + binned_workspace(d, mode, K, E, n_sub, ns, e0);
    MP_CHECK_ARG(ws && ws_bytes >= total, MP_ERR_WORKSPACE,
                 "mp_propagate_counts: workspace of %zu bytes needed, %zu given", total, ws_bytes);
    fo.part = (float*)ws;
    fo.E = E;
    return MP_OK;
  }
  CountsParams p{};
  int64_t blocks = 0;
  const mp_status st = setup_counts(p, "mp_propagate_counts", M, E, d, bin_of_mode, mode, m_lo, K,
                                    n_sub, ns, e0, est, blocks);
  if (st != MP_OK) return st;
  size_t part_bytes, total;
  propagate_counts_sizes(p, blocks, part_bytes, total);
  MP_CHECK_ARG(ws && ws_bytes >= total, MP_ERR_WORKSPACE,
               "mp_propagate_counts: workspace of %zu bytes needed, %zu given", total, ws_bytes);
  fo = FusedOut{};
  fo.part = (float*)ws;
  fo.E = E;
  fo.n_runs = p.n_runs;
  for (int q = 0; q < p.n_runs; ++q) {
    fo.run_lo[q] = p.run_lo[q];
    fo.run_hi[q] = p.run_hi[q];
  }
  fused_slots(p.n_runs, fo.run_lo, fo.run_hi, fo.slot_off);
  return MP_OK;
}

// Counts from the partials an occupation-fused GEMM left at the start of ws
// (laid out by fused_out_setup with the same arguments).  The fused GEMM runs
// in FP32 or a split precision, so the joint paths take their FP32 factor
// tables.
mp_status counts_from_partials_launch(int32_t M, int64_t E, const double* n, mp_estimator est,
                                      int32_t d, const int32_t* bin_of_mode, mp_bin_mode mode,
                                      const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                      int64_t ns, int64_t e0, double* acc, void* ws,
                                      size_t ws_bytes, hipStream_t stream) {
  if (mode == MP_JOINT && d >= 2) {
    // the joint paths read the bin sums from the partials; their own
    // workspace follows them
    FusedOut fo{};
    const mp_status sr = fused_runs(M, bin_of_mode, fo);
    if (sr != MP_OK) return sr;
    const size_t pb = joint_part_bytes(fo, E);
    MP_CHECK_ARG(ws && ws_bytes >= pb, MP_ERR_WORKSPACE,
                 "mp_propagate_counts: workspace of %zu bytes needed, %zu given", pb, ws_bytes);
    void* jws = (char*)ws + pb;
    const size_t jbytes = ws_bytes - pb;
    return d == 2 ? joint2_launch(M, E, nullptr, n, MP_FP32, est, bin_of_mode, m_lo, K, n_sub, ns,
                                  e0, acc, jws, jbytes, stream, (const float*)ws)
                  : jointd_launch(M, E, nullptr, n, MP_FP32, est, d, bin_of_mode, m_lo, K, n_sub,
                                  ns, e0, acc, jws, jbytes, stream, (const float*)ws);
  }
  CountsParams p{};
  int64_t blocks = 0;
  const mp_status st = setup_counts(p, "mp_propagate_counts", M, E, d, bin_of_mode, mode, m_lo, K,
                                    n_sub, ns, e0, est, blocks);
  if (st != MP_OK) return st;
  size_t part_bytes, total;
  propagate_counts_sizes(p, blocks, part_bytes, total);
  MP_CHECK_ARG(ws && ws_bytes >= total, MP_ERR_WORKSPACE,
               "mp_propagate_counts: workspace of %zu bytes needed, %zu given", total, ws_bytes);
  double* blk = (double*)((char*)ws + part_bytes);
  hipLaunchKernelGGL((counts_fused<FromPartials, false>), dim3((unsigned)blocks),
                     dim3(kCountThreads), 0, stream, p, FromPartials{(const float*)ws}, n, blk);
  MP_HIP_LAUNCH_CHECK("mp_propagate_counts counts launch");
  const int ns_touched = (int)(p.s_last - p.s_first + 1);
  hipLaunchKernelGGL(counts_reduce, dim3((p.entries + 255) / 256, ns_touched), dim3(256), 0, stream,
                     p, (const double*)blk, acc);
  MP_HIP_LAUNCH_CHECK("mp_propagate_counts reduce launch");
  return MP_OK;
}

mp_status propagate_counts_launch(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                                  const void* ab, const double* n, const void* packed, int32_t d,
                                  const int32_t* bin_of_mode, mp_bin_mode mode,
                                  const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                  int64_t ns, int64_t e0, double* acc, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  FusedOut fo;
  mp_status st = fused_out_setup(M, E, d, bin_of_mode, mode, m_lo, K, n_sub, ns, e0, est, ws,
                                 ws_bytes, fo);
  if (st != MP_OK) return st;
  if (fo.n_runs > 0 && (st = gemm_fused_launch(M, E, packed, prec, ab, fo, stream)) != MP_OK)
    return st;
  return counts_from_partials_launch(M, E, n, est, d, bin_of_mode, mode, m_lo, K, n_sub, ns, e0,
                                     acc, ws, ws_bytes, stream);
}

// One distribution through the bilinear form alpha^T W beta (W packed by
// bilinear_pack_launch; the mode set S is inside W): the GEMM's partials cover
// one run of all M input modes, which the d = 1 counting kernels then read.
mp_status gemm_bilinear_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                               const void* ab, const FusedOut& fo, hipStream_t stream);

mp_status propagate_counts_bilinear_launch(int32_t M, int64_t E, mp_precision prec,
                                           mp_estimator est, const void* ab, const double* n,
                                           const void* packed, const int32_t* m_lo,
                                           const int32_t* K, int32_t n_sub, int64_t ns,
                                           int64_t e0, double* acc, void* ws, size_t ws_bytes,
                                           hipStream_t stream) {
  const std::vector<int32_t> all(M, 0);
  FusedOut fo;
  mp_status st = fused_out_setup(M, E, 1, all.data(), MP_JOINT, m_lo, K, n_sub, ns, e0, est, ws,
                                 ws_bytes, fo);
  if (st != MP_OK) return st;
  if ((st = gemm_bilinear_launch(M, E, packed, prec, ab, fo, stream)) != MP_OK) return st;
  return counts_from_partials_launch(M, E, n, est, 1, all.data(), MP_JOINT, m_lo, K, n_sub, ns,
                                     e0, acc, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------- no-allocation variant

// Scratch of mp_propagate_counts_noalloc: the occupation-fused GEMM's
// per-block partials followed by the counting kernel's per-tile partials, in
// a device array that every GPU the library runs on holds from module load to
// process exit.  In host code the array's name is only a stand-in for the
// symbol, never a device address: the address is looked up once per device
// (with that device current) and kept, and only that address reaches kernels.
// Each call writes every scratch byte it later reads (the GEMM epilogue every
// (slot, sample) partial of the chunk, the counting kernel every entry of its
// tile), so nothing has to start at zero and the previous call's contents are
// never read.  Calls that overlap on one GPU share the array and race.
static __device__ __align__(256) unsigned char scratch[MP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxScratchDevices];

static mp_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error("mp_propagate_counts_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    return MP_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxScratchDevices) {
    set_error("mp_propagate_counts_noalloc: device %d beyond the %d supported", dev,
              kMaxScratchDevices);
    return MP_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("mp_propagate_counts_noalloc: hipGetSymbolAddress of the scratch array: %s",
                hipGetErrorString(e));
      return MP_ERR_HIP;
    }
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return MP_OK;
}

// mp_propagate_counts with the library's scratch as its workspace; arguments
// validated by the caller as for mp_propagate_counts.  Sizes are checked before
// any HIP call.
mp_status propagate_counts_noalloc_launch(int32_t M, int64_t E, mp_precision prec,
                                          mp_estimator est, const void* ab, const double* n,
                                          const void* packed, int32_t d,
                                          const int32_t* bin_of_mode, mp_bin_mode mode,
                                          const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                          int64_t ns, int64_t e0, double* acc,
                                          hipStream_t stream) {
  MP_CHECK_ARG(mode != MP_JOINT || d == 1, MP_ERR_UNSUPPORTED,
               "mp_propagate_counts_noalloc: joint distributions of %d bins are not supported "
               "(use mp_propagate_counts)", d);
  const size_t need = propagate_counts_workspace(M, E, d, bin_of_mode, mode, K, n_sub, ns, e0);
  MP_CHECK_ARG(need > 0, MP_ERR_UNSUPPORTED,
               "mp_propagate_counts_noalloc: bins form more than %d contiguous mode runs",
               MP_MAX_RUNS);
  MP_CHECK_ARG(need <= (size_t)MP_NOALLOC_SCRATCH_BYTES, MP_ERR_WORKSPACE,
               "mp_propagate_counts_noalloc: this chunk needs %zu bytes of scratch, more than "
               "the library's %zu (split the chunk, or pass a workspace to "
               "mp_propagate_counts)", need, (size_t)MP_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  const mp_status st = scratch_of_current_device(&ws);
  if (st != MP_OK) return st;
  return propagate_counts_launch(M, E, prec, est, ab, n, packed, d, bin_of_mode, mode, m_lo, K,
                                 n_sub, ns, e0, acc, ws, (size_t)MP_NOALLOC_SCRATCH_BYTES, stream);
}

mp_status counts_finalize_launch(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                                 int64_t ns, const double* acc, double* P_re, double* P_im,
                                 double* sigma, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (mode == MP_JOINT && d >= 2)
    return jointd_finalize(d, K, n_sub, ns, acc, P_re, P_im, sigma, ws, ws_bytes, stream);
  FinalParams p{};
  p.n_dist = mode == MP_JOINT ? 1 : d + (mode == MP_MARGINALS_AND_TOTAL ? 1 : 0);
  p.off[0] = 0;
  for (int q = 0; q < p.n_dist; ++q) {
    p.K[q] = K[q];
    p.off[q + 1] = p.off[q] + K[q];
  }
  p.entries = (int)entries_of(d, mode, K);
  p.n_sub = n_sub;
  p.inv_ns = 1.0 / (double)ns;
  hipLaunchKernelGGL(counts_finalize, dim3(p.entries), dim3(256), 0, stream, p, acc, P_re, P_im,
                     sigma);
  MP_HIP_LAUNCH_CHECK("mp_counts_finalize launch");
  return MP_OK;
}


// ---------------------------------------------------------------- finiteness

__global__ void zero_i64(int64_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

// Grid-stride count of non-finite entries, one atomic add per wave.
__global__ __launch_bounds__(256) void count_nonfinite(const double* __restrict__ x, int64_t n,
                                                       int64_t* __restrict__ count) {
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    c += isfinite(x[i]) ? 0 : 1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c != 0) atomicAdd((unsigned long long*)count, (unsigned long long)c);
}

mp_status check_finite_launch(const double* x, int64_t n, int64_t* scratch, int64_t* n_bad,
                              hipStream_t stream) {
  hipLaunchKernelGGL(zero_i64, dim3(1), dim3(64), 0, stream, scratch);
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(count_nonfinite, dim3((unsigned)blocks), dim3(256), 0, stream, x, n, scratch);
  MP_HIP_LAUNCH_CHECK("mp_check_finite launch");
  int64_t c = 0;
  hipError_t e = hipMemcpyAsync(&c, scratch, sizeof(c), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    set_error("mp_check_finite: %s", hipGetErrorString(e));
    return MP_ERR_HIP;
  }
  if (n_bad) *n_bad = c;
  if (c != 0) {
    set_error("mp_check_finite: %lld of %lld values are NaN or infinite", (long long)c,
              (long long)n);
    return MP_ERR_NONFINITE;
  }
  return MP_OK;
}

// ---------------------------------------------------------------- per-sample observables

// Occupation of every distribution for every sample of the chunk (wave per
// sample): nq[(k n_dist + q) 2 + {0, 1}] = (Re, Im) n_q of chunk sample k.
template <typename CT>
__device__ inline void occupation_sample(const CountsParams& p, const CT* __restrict__ C,
                                         double* __restrict__ nq, int64_t k, int lane) {
  const int64_t ldc = 2 * p.ldm;
  double nb[MP_MAX_BINS][2];
  sample_bin_sums<CT>(p, C + k * ldc, C + (p.E + k) * ldc, lane, nb);
  if (lane == 0)
    for (int q = 0; q < p.n_dist; ++q) {
      double vr, vi;
      dist_occupation(p, nb, q, vr, vi);
      nq[(k * p.n_dist + q) * 2] = vr;
      nq[(k * p.n_dist + q) * 2 + 1] = vi;
    }

}

template <typename CT>
__global__ __launch_bounds__(256) void occupations_kernel(CountsParams p, const CT* __restrict__ C,
                                                          double* __restrict__ nq) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * (4 * kOccPerWave) + wave;
  for (int j = 0; j < kOccPerWave; ++j) {
    const int64_t k = base + 4 * j;
    if (k >= p.E) return;
    occupation_sample<CT>(p, C, nq, k, lane);
  }
}

struct SampleStatParams {
  int64_t E, e0, ns;   // chunk size, first global sample, samples per sub-ensemble
  int64_t s_first;     // first sub-ensemble the chunk touches
  int n_dist;
  int est;             // mp_estimator
  int kmax;            // moments
  int q, m, n_bins;    // histogram: distribution, count, bins
  double o_min, inv_width;
};

// Normally ordered moments (eq. moment with the parity-projected weights):
// per sample n_q^k, times tanh(n) for odd k on the matrix-P path (+P: 1).
// Block (s, q): the chunk's samples of sub-ensemble s_first + blockIdx.x,
// summed in a fixed order (strided per thread, then a tree in LDS) and added
// to acc[s][q][k - 1] (re, im).
__global__ __launch_bounds__(256) void moments_kernel(SampleStatParams p, const double* __restrict__ n,
                                                      const double* __restrict__ nq,
                                                      double* __restrict__ acc) {
  __shared__ double red[256][2];
  const int64_t s = p.s_first + blockIdx.x;
  const int q = blockIdx.y;
  int64_t lo = s * p.ns, hi = (s + 1) * p.ns;
  lo = lo > p.e0 ? lo : p.e0;
  hi = hi < p.e0 + p.E ? hi : p.e0 + p.E;
  double sr[MP_MAX_MOMENTS], si[MP_MAX_MOMENTS];
#pragma unroll
  for (int o = 0; o < MP_MAX_MOMENTS; ++o) sr[o] = si[o] = 0.0;
  for (int64_t g = lo + threadIdx.x; g < hi; g += 256) {
    const int64_t k = g - p.e0;
    const double zr = nq[(k * p.n_dist + q) * 2], zi = nq[(k * p.n_dist + q) * 2 + 1];
    double w = 1.0;  // +P
    if (p.est != MP_PLUS_P) {
      const double nk = n[k];
      w = isfinite(nk) ? tanh(nk) : __builtin_nan("");
    }
    double pr = 1.0, pi = 0.0;
#pragma unroll
    for (int o = 0; o < MP_MAX_MOMENTS; ++o) {
      if (o < p.kmax) {
        const double tr = pr * zr - pi * zi;
        pi = pr * zi + pi * zr;
        pr = tr;
        const double f = (o & 1) ? 1.0 : w;  // order o + 1 odd -> weight w
        sr[o] += f * pr;
        si[o] += f * pi;
      }
    }
  }
  for (int o = 0; o < p.kmax; ++o) {
    red[threadIdx.x][0] = sr[o];
    red[threadIdx.x][1] = si[o];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        red[threadIdx.x][0] += red[threadIdx.x + w][0];
        red[threadIdx.x][1] += red[threadIdx.x + w][1];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double* dst = acc + ((s * p.n_dist + q) * p.kmax + o) * 2;
      dst[0] += red[0][0];
      dst[1] += red[0][1];
    }
    __syncthreads();
  }
}

// Per-sample count observable of distribution q at count m (eq.
// c-number-variable for one bin: g0 n_q^m e^{-n_q} / m!, with g0 formed as in
// counts_fused; +P: n_q^m e^{-n_q} / m!), real part, binned into n_bins equal
// bins from o_min (bin 0: below, bin n_bins + 1: at or above the top or not
// finite).  Counts are added as FP64 ones, exact and order-independent.
__global__ __launch_bounds__(256) void histogram_kernel(SampleStatParams p, const double* __restrict__ n,
                                                        const double* __restrict__ nq,
                                                        double* __restrict__ hist) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= p.E) return;
  const double zr = nq[(k * p.n_dist + p.q) * 2], zi = nq[(k * p.n_dist + p.q) * 2 + 1];
  const double mag = sqrt(zr * zr + zi * zi);
  // log(n_q^m / m!) as (real, phase); 0^0 = 1
  double lr, lp;
  if (p.m == 0) {
    lr = 0.0;
    lp = 0.0;
  } else if (mag == 0.0) {
    lr = -INFINITY;
    lp = 0.0;
  } else {
    lr = p.m * log(mag);
    lp = p.m * atan2(zi, zr);
  }
  lr -= lgamma((double)p.m + 1.0);
  double G;
  if (p.est == MP_PLUS_P) {
    G = exp(lr - zr) * cos(lp - zi);
  } else {
    const double nn = n[k];
    const double L = log1p(exp(-2.0 * fabs(nn)));
    const double c1 = (nn >= 0.0 ? 0.0 : 2.0 * nn) - L;
    const double c2 = (nn >= 0.0 ? -2.0 * nn : 0.0) - L;
    const double par = (p.m & 1) ? -1.0 : 1.0;
    G = exp(lr - zr + c1) * cos(lp - zi) + par * exp(lr + zr + c2) * cos(lp + zi);
  }
  if (!isfinite(zr) || !isfinite(zi) || (p.est != MP_PLUS_P && !isfinite(n[k])))
    G = __builtin_nan("");
  int64_t b;
  if (!(G == G) || G - G != 0.0) {
    b = p.n_bins + 1;  // not finite
  } else {
    const double x = (G - p.o_min) * p.inv_width;
    b = x < 0.0 ? 0 : (x >= (double)p.n_bins ? p.n_bins + 1 : (int64_t)x + 1);
  }
  const int64_t s = (p.e0 + k) / p.ns;
  atomicAdd(hist + s * (p.n_bins + 2) + b, 1.0);
}

// Mean over sub-ensembles of scale * acc[s][v] / samples_per_sub and sigma_T =
// sd of its real part over the sub-ensembles / sqrt(n_sub) (NaN for one).
__global__ __launch_bounds__(256) void subensemble_stats_kernel(int n_sub, int64_t n_vals, int ncomp,
                                                                double scale,
                                                                const double* __restrict__ acc,
                                                                double* __restrict__ mean,
                                                                double* __restrict__ sigma) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= n_vals) return;
  double m[2] = {0.0, 0.0};
  for (int s = 0; s < n_sub; ++s)
    for (int c = 0; c < ncomp; ++c) m[c] += acc[((int64_t)s * n_vals + v) * ncomp + c] * scale;
  for (int c = 0; c < ncomp; ++c) {
    m[c] /= n_sub;
    mean[v * ncomp + c] = m[c];
  }
  double ss = 0.0;
  for (int s = 0; s < n_sub; ++s) {
    const double dlt = acc[((int64_t)s * n_vals + v) * ncomp] * scale - m[0];
    ss += dlt * dlt;
  }
  sigma[v] = n_sub > 1 ? sqrt(ss / (n_sub - 1) / n_sub) : NAN;
}

mp_status occupations_launch(int32_t M, int64_t E, const void* C, mp_precision prec, int32_t d,
                             const int32_t* bin_of_mode, mp_bin_mode mode, double* nq,
                             hipStream_t stream) {
  CountsParams p{};
  p.M = M;
  p.ldm = ld_modes(M);
  p.E = E;
  p.d = d;
  p.mode = mode;
  if (!fill_runs(p, M, bin_of_mode)) {
    set_error("mp_occupations: bins form more than %d contiguous mode runs", MP_MAX_RUNS);
    return MP_ERR_UNSUPPORTED;
  }
  p.n_dist = d + (mode == MP_MARGINALS_AND_TOTAL ? 1 : 0);
  for (int q = 0; q < p.n_dist; ++q) p.dist_src[q] = q < d ? q : -1;
  const int64_t blocks = (E + 4 * kOccPerWave - 1) / (4 * kOccPerWave);
  if (prec == MP_FP64)
    hipLaunchKernelGGL(occupations_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream, p,
                       (const double*)C, nq);
  else
    hipLaunchKernelGGL(occupations_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream, p,
                       (const float*)C, nq);
  MP_HIP_LAUNCH_CHECK("mp_occupations launch");
  return MP_OK;
}

mp_status moments_launch(int64_t E, const double* n, const double* nq, int32_t n_dist,
                         int32_t kmax, mp_estimator est, int64_t ns, int64_t e0, double* acc,
                         hipStream_t stream) {
  SampleStatParams p{};
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  p.s_first = e0 / ns;
  p.n_dist = n_dist;
  p.est = est;
  p.kmax = kmax;
  const int64_t n_touched = (e0 + E - 1) / ns - p.s_first + 1;
  hipLaunchKernelGGL(moments_kernel, dim3((unsigned)n_touched, (unsigned)n_dist), dim3(256), 0,
                     stream, p, n, nq, acc);
  MP_HIP_LAUNCH_CHECK("mp_moments_accumulate launch");
  return MP_OK;
}

mp_status histogram_launch(int64_t E, const double* n, const double* nq, int32_t n_dist, int32_t q,
                           int32_t m, mp_estimator est, double o_min, double width,
                           int32_t n_bins, int64_t ns, int64_t e0, double* hist,
                           hipStream_t stream) {
  SampleStatParams p{};
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  p.n_dist = n_dist;
  p.est = est;
  p.q = q;
  p.m = m;
  p.n_bins = n_bins;
  p.o_min = o_min;
  p.inv_width = 1.0 / width;
  hipLaunchKernelGGL(histogram_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, stream, p,
                     n, nq, hist);
  MP_HIP_LAUNCH_CHECK("mp_observable_histogram launch");
  return MP_OK;
}

mp_status subensemble_stats_launch(int32_t n_sub, int64_t ns, int64_t n_vals, int32_t ncomp,
                                   double scale, const double* acc, double* mean, double* sigma,
                                   hipStream_t stream) {
  hipLaunchKernelGGL(subensemble_stats_kernel, dim3((unsigned)((n_vals + 255) / 256)), dim3(256), 0,
                     stream, n_sub, n_vals, ncomp, scale / (double)ns, acc, mean, sigma);
  MP_HIP_LAUNCH_CHECK("mp_subensemble_stats launch");
  return MP_OK;
}

}  // namespace mp
