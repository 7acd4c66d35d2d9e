// Phase-space amplitudes of squeezed vacuum inputs.
//
// Paper, main text: a squeezed input is a real coherent-state integral with
// the even weight xi(alpha); with the unnormalised +P kernel the density
// matrix is reproduced by a real Gaussian pair per mode with variances
// sinh r cosh r and covariance sinh^2 r, and the parity-projected
// distribution (Omega_00 = 1) is sampled the same way.  Two independent
// normals give the pair exactly:
//     alpha = c+ w1 + c- w2,  beta = c+ w1 - c- w2,
//     c+ = sqrt(e^{2r} - 1) / 2,  c- = sqrt(1 - e^{-2r}) / 2.
//
// Noise: one Philox4x64-10 block (Salmon et al., SC'11) per (sample, mode
// pair) with counter (g, p, net, 0) and key (seed, 0); Box-Muller on words
// (0,1) for mode 2p and (2,3) for mode 2p+1.
//
// One wavefront per sample: lanes stride over mode pairs, so the column of
// the sample (contiguous over modes) is written with coalesced stores, and
// n = alpha . beta is reduced across the wave with shuffles.
#include <hip/hip_runtime.h>

#include "common.h"

namespace mp {

__device__ inline void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                     uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull, kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t hi0 = __umul64hi(kMul0, c0), lo0 = kMul0 * c0;
    const uint64_t hi1 = __umul64hi(kMul1, c2), lo1 = kMul1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
}

__device__ inline void box_muller(uint64_t xe, uint64_t xo, double& w1, double& w2) {
  const double u = (double)((xe >> 11) + 1ull) * 0x1p-53;
  const double v = (double)(xo >> 11) * 0x1p-53;
  const double rho = sqrt(-2.0 * log(u));
  double s, c;
  sincos(2.0 * M_PI * v, &s, &c);
  w1 = rho * c;
  w2 = rho * s;
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_val(uint16_t h) { return (double)__uint_as_float(((uint32_t)h) << 16); }

// Rounds x to the storage precision, stores it, and returns the stored value.
template <int PREC>
__device__ inline double store_pair(void* ab, int64_t plane, int64_t off, double x0, double x1,
                                    double& y1) {
  if constexpr (PREC == MP_FP64) {
    typedef __attribute__((ext_vector_type(2))) double d2;
    *(d2*)((double*)ab + off) = d2{x0, x1};
    y1 = x1;
    return x0;
  } else if constexpr (PREC == MP_FP32) {
    typedef __attribute__((ext_vector_type(2))) float f2;
    const float f0 = (float)x0, f1 = (float)x1;
    *(f2*)((float*)ab + off) = f2{f0, f1};
    y1 = f1;
    return f0;
  } else if constexpr (PREC == MP_SPLIT_BF16) {
    const uint16_t h0 = bf16_rne((float)x0), h1 = bf16_rne((float)x1);
    const uint16_t l0 = bf16_rne((float)(x0 - bf16_val(h0)));
    const uint16_t l1 = bf16_rne((float)(x1 - bf16_val(h1)));
    uint16_t* p = (uint16_t*)ab;
    *(uint32_t*)(p + off) = (uint32_t)h0 | ((uint32_t)h1 << 16);
    *(uint32_t*)(p + plane + off) = (uint32_t)l0 | ((uint32_t)l1 << 16);
    y1 = bf16_val(h1) + bf16_val(l1);
    return bf16_val(h0) + bf16_val(l0);
  } else {
    const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
    const _Float16 l0 = (_Float16)(x0 - (double)h0);
    const _Float16 l1 = (_Float16)(x1 - (double)h1);
    _Float16* p = (_Float16*)ab;
    typedef __attribute__((ext_vector_type(2))) _Float16 h2;
    *(h2*)(p + off) = h2{h0, h1};
    *(h2*)(p + plane + off) = h2{l0, l1};
    y1 = (double)h1 + (double)l1;
    return (double)h0 + (double)l0;
  }
}

template <int PREC>
__global__ __launch_bounds__(256) void sample_kernel(int M, int64_t ldm, int64_t g0, int64_t E,
                                                     const double* __restrict__ r, uint64_t seed,
                                                     uint32_t net, void* __restrict__ ab,
                                                     double* __restrict__ n_out) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= E) return;
  const uint64_t g = (uint64_t)(g0 + k);
  const int64_t plane = ldm * 2 * E;
  const int64_t col_a = k * ldm, col_b = (E + k) * ldm;
  double nsum = 0.0;
  for (int64_t p = lane; p < ldm / 2; p += 64) {
    const int64_t j0 = 2 * p;
    double a0 = 0, b0 = 0, a1 = 0, b1 = 0;
    if (j0 < M) {
      uint64_t c0 = g, c1 = (uint64_t)p, c2 = net, c3 = 0;
      philox4x64_10(c0, c1, c2, c3, seed, 0);
      double w1, w2;
      box_muller(c0, c1, w1, w2);
      double rj = r[j0];
      double cp = 0.5 * sqrt(expm1(2.0 * rj)), cm = 0.5 * sqrt(-expm1(-2.0 * rj));
      a0 = cp * w1 + cm * w2;
      b0 = cp * w1 - cm * w2;
      if (j0 + 1 < M) {
        box_muller(c2, c3, w1, w2);
        rj = r[j0 + 1];
        cp = 0.5 * sqrt(expm1(2.0 * rj));
        cm = 0.5 * sqrt(-expm1(-2.0 * rj));
        a1 = cp * w1 + cm * w2;
        b1 = cp * w1 - cm * w2;
      }
    }
    double ya1, yb1;
    const double ya0 = store_pair<PREC>(ab, plane, col_a + j0, a0, a1, ya1);
    const double yb0 = store_pair<PREC>(ab, plane, col_b + j0, b0, b1, yb1);
    nsum += ya0 * yb0 + ya1 * yb1;
  }
  nsum = wave_sum(nsum);
  if (lane == 0) n_out[k] = nsum;
}

mp_status sample_launch(int32_t M, int64_t g0, int64_t E, const double* r, uint64_t seed,
                        uint32_t net, mp_precision prec, void* ab, double* n_out,
                        hipStream_t stream) {
  const int64_t ldm = ld_modes(M);
  const int64_t blocks = (E + 3) / 4;
  if (blocks > 0x7FFFFFFF) {
    set_error("mp_sample: E too large for one launch");
    return MP_ERR_UNSUPPORTED;
  }
  switch (prec) {
    case MP_FP64:
      hipLaunchKernelGGL(sample_kernel<MP_FP64>, dim3((unsigned)blocks), dim3(256), 0, stream, M,
                         ldm, g0, E, r, seed, net, ab, n_out);
      break;
    case MP_FP32:
      hipLaunchKernelGGL(sample_kernel<MP_FP32>, dim3((unsigned)blocks), dim3(256), 0, stream, M,
                         ldm, g0, E, r, seed, net, ab, n_out);
      break;
    case MP_SPLIT_BF16:
      hipLaunchKernelGGL(sample_kernel<MP_SPLIT_BF16>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         M, ldm, g0, E, r, seed, net, ab, n_out);
      break;
    case MP_SPLIT_FP16:
      hipLaunchKernelGGL(sample_kernel<MP_SPLIT_FP16>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         M, ldm, g0, E, r, seed, net, ab, n_out);
      break;
  }
  MP_HIP_LAUNCH_CHECK("mp_sample launch");
  return MP_OK;
}

}  // namespace mp
