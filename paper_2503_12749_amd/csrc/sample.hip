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
// One wavefront per group of samples: lanes stride over mode pairs, so each
// sample's column (contiguous over modes) is written with coalesced stores,
// and n = alpha . beta is reduced across the wave with shuffles.  The FP64
// path evaluates Box-Muller with the library's FP64 log and sincos; the FP32
// and split paths evaluate it by short FP64 series and round the radius and
// the angle's sine and cosine to FP32 once (no systematic error beyond that
// rounding).
#include <hip/hip_runtime.h>

#include "common.h"

namespace mp {

// Full 128-bit product of two 64-bit words from four 32 x 32 -> 64
// multiply-adds (each partial sum fits in 64 bits): a b = p00 +
// (a0 b1 + a1 b0) 2^32 + a1 b1 2^64 with the carries taken through t1, t2.
__device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t1 = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t t2 = (uint64_t)a1 * b0 + (uint32_t)t1;
  hi = (uint64_t)a1 * b1 + (t1 >> 32) + (t2 >> 32);
  lo = (t2 << 32) | (uint32_t)p00;
}

__device__ inline void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                     uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull, kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(kMul0, c0, hi0, lo0);
    mulhilo64(kMul1, c2, hi1, lo1);
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

// The same transform for the paths that store FP32 or split 16-bit
// amplitudes.  Both parts are evaluated in FP64 by short series and rounded to
// FP32 once, so the amplitudes carry only that rounding: a library FP32
// logarithm was measured to bias -ln u by about +4e-8 on average, which biases
// every photon number the same way (the radius) and does not average out.
//   radius: u = m 2^k with m in [sqrt(1/2), sqrt(2)), s = (m - 1) / (m + 1)
//     (|s| <= 0.172), ln m = 2 atanh s = 2 s (1 + s^2/3 + ... + s^12/13),
//     the first omitted term below 1.3e-12 relative;
//   angle: 2 pi v = pi x 2^-52 (x = xo >> 11); the top two bits of x give the
//     quarter turn q, the other 51 the fraction f in [0, 1/2) with
//     angle = q pi/2 + pi f, and f >= 1/4 is reflected to g = 1/2 - f (sine
//     and cosine swap), exactly on the integer; sin and cos of pi g in
//     [0, pi/4] from their Taylor series to t^13 and t^12 (first omitted terms
//     below 3e-14 and 4e-13).
__device__ inline double neg_log_unit(double u) {
  int k;
  double m = frexp(u, &k);  // u = m 2^k, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    k -= 1;
  }
  // s = (m - 1) / (m + 1): hardware reciprocal refined by two Newton steps
  const double d = m + 1.0;
  double rd = __builtin_amdgcn_rcp(d);
  rd = fma(rd, fma(-d, rd, 1.0), rd);
  rd = fma(rd, fma(-d, rd, 1.0), rd);
  const double s = (m - 1.0) * rd;
  const double s2 = s * s;
  double p = 1.0 / 13.0;
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  p = fma(p, s2, 1.0);
  constexpr double kLn2 = 0.69314718055994530942;
  return -fma((double)k, kLn2, 2.0 * s * p);
}

__device__ inline void sincos_eighth(double t, double& s, double& c) {
  const double t2 = t * t;
  double ps = 1.0 / 6227020800.0;  // 1/13!
  ps = fma(ps, t2, -1.0 / 39916800.0);
  ps = fma(ps, t2, 1.0 / 362880.0);
  ps = fma(ps, t2, -1.0 / 5040.0);
  ps = fma(ps, t2, 1.0 / 120.0);
  ps = fma(ps, t2, -1.0 / 6.0);
  ps = fma(ps, t2, 1.0);
  double pc = 1.0 / 479001600.0;  // 1/12!
  pc = fma(pc, t2, -1.0 / 3628800.0);
  pc = fma(pc, t2, 1.0 / 40320.0);
  pc = fma(pc, t2, -1.0 / 720.0);
  pc = fma(pc, t2, 1.0 / 24.0);
  pc = fma(pc, t2, -0.5);
  pc = fma(pc, t2, 1.0);
  s = t * ps;
  c = pc;
}

__device__ inline void box_muller_f32(uint64_t xe, uint64_t xo, float& w1, float& w2) {
  const double u = (double)((xe >> 11) + 1ull) * 0x1p-53;
  const float rho = sqrtf((float)(2.0 * neg_log_unit(u)));  // two unbiased roundings
  const uint64_t x = xo >> 11;
  const uint32_t q = (uint32_t)(x >> 51);
  const uint64_t fx = x & ((1ull << 51) - 1ull);  // f = fx 2^-52
  const bool upper = (fx >> 50) != 0;              // f >= 1/4
  const uint64_t gx = upper ? (1ull << 51) - fx : fx;  // g 2^52, at most 2^50: exact in FP64
  constexpr double kPi = 3.14159265358979323846;
  double s, c;
  sincos_eighth((double)gx * (0x1p-52 * kPi), s, c);
  const float sf = (float)(upper ? c : s);  // sin(pi f), cos(pi f)
  const float cf = (float)(upper ? s : c);
  const float cq = (q & 1u) ? -sf : cf;  // cos(q pi/2 + pi f) for q = 0, 1
  const float sq = (q & 1u) ? cf : sf;
  const float sign = (q & 2u) ? -1.0f : 1.0f;  // q = 2, 3: half a turn more
  w1 = rho * (sign * cq);
  w2 = rho * (sign * sq);
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Stores the amplitudes of modes (2p, 2p+1) of one column in the storage
// precision and returns the stored values (hi + lo for the split forms).
__device__ inline void store_pair_f64(void* ab, int64_t off, double x0, double x1) {
  typedef __attribute__((ext_vector_type(2))) double d2;
  *(d2*)((double*)ab + off) = d2{x0, x1};
}

// Split storage: element j of a column sits at 64 (j / 32) + j % 32 (hi) and
// 32 further (lo); off is the hi position of the even mode 2p, whose partner
// 2p + 1 shares its block.
template <int PREC>
__device__ inline void store_pair_f32(void* ab, int64_t off, float x0, float x1, double& y0,
                                      double& y1) {
  if constexpr (PREC == MP_FP32) {
    typedef __attribute__((ext_vector_type(2))) float f2;
    *(f2*)((float*)ab + off) = f2{x0, x1};
    y0 = x0;
    y1 = x1;
  } else if constexpr (PREC == MP_SPLIT_BF16) {
    // x - hi is exact in FP32 (at most 16 significant bits remain)
    const uint16_t h0 = bf16_rne(x0), h1 = bf16_rne(x1);
    const uint16_t l0 = bf16_rne(x0 - bf16_val(h0)), l1 = bf16_rne(x1 - bf16_val(h1));
    uint16_t* q = (uint16_t*)ab;
    *(uint32_t*)(q + off) = (uint32_t)h0 | ((uint32_t)h1 << 16);
    *(uint32_t*)(q + off + 32) = (uint32_t)l0 | ((uint32_t)l1 << 16);
    y0 = (double)bf16_val(h0) + (double)bf16_val(l0);
    y1 = (double)bf16_val(h1) + (double)bf16_val(l1);
  } else if constexpr (PREC == MP_SPLIT1T_FP16) {
    // one FP16 value per entry (off from split1t_offset)
    const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
    typedef __attribute__((ext_vector_type(2))) _Float16 h2;
    *(h2*)((_Float16*)ab + off) = h2{h0, h1};
    y0 = (double)(float)h0;
    y1 = (double)(float)h1;
  } else {
    const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
    const _Float16 l0 = (_Float16)(x0 - (float)h0), l1 = (_Float16)(x1 - (float)h1);
    _Float16* q = (_Float16*)ab;
    typedef __attribute__((ext_vector_type(2))) _Float16 h2;
    *(h2*)(q + off) = h2{h0, h1};
    *(h2*)(q + off + 32) = h2{l0, l1};
    y0 = (double)(float)h0 + (double)(float)l0;
    y1 = (double)(float)h1 + (double)(float)l1;
  }
}

// Two values as e4m3 codes (first in the low byte) by the hardware pack
// conversion, which rounds to nearest even and gives e4m3_rne's codes for
// every input below 448 in magnitude (checked over 4e6 inputs, every rounding
// tie and the subnormal range included); inputs are clamped to +-448 first,
// e4m3_rne's saturation.  One instruction instead of e4m3_rne's integer
// sequence, in a kernel bound by its ALU work.
__device__ inline uint16_t e4m3_pair(float x0, float x1) {
  x0 = fminf(fmaxf(x0, -448.0f), 448.0f);
  x1 = fminf(fmaxf(x1, -448.0f), 448.0f);
  return (uint16_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x0, x1, 0, false) & 0xFFFF);
}

// MP_SPLIT1T_FP16 storage: mode j of storage column c (column pairs, each
// 32-mode block holding the pair's two runs of 32 values side by side).
__device__ inline int64_t split1t_offset(int64_t c, int64_t j, int64_t ldm) {
  return (c >> 1) * 2 * ldm + 64 * (j >> 5) + (j & 31) + (c & 1) * 32;
}

// Each wavefront owns wave_samples<PREC>() consecutive samples; its lanes
// stride over mode pairs, so the coefficients c+, c- of a lane's modes are
// computed once and reused for all of the wave's samples, and every store of
// one sample's column is coalesced across the wave.  8 samples for FP64, 4
// otherwise: the samples of a wave are unrolled, and with 8 the
// reduced-precision instances needed 225-278 VGPRs (one or two waves per
// SIMD; the e4m3 form one), with 4 they need 153-183 (two or three) for a
// kernel bound by its ALU work.
constexpr int kWaveSamples = 8;
template <int PREC>
constexpr int wave_samples() { return PREC == MP_FP64 ? kWaveSamples : 4; }

template <int PREC>
__global__ __launch_bounds__(256) void sample_kernel(int M, int64_t ldm, int64_t g0, int64_t E,
                                                     const double* __restrict__ r, uint64_t seed,
                                                     uint32_t net, void* __restrict__ ab,
                                                     double* __restrict__ n_out) {
  constexpr int WS = wave_samples<PREC>();
  const int lane = threadIdx.x & 63;
  const int64_t k0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * WS;
  if (k0 >= E) return;
  const int nk = (int)(E - k0 < WS ? E - k0 : WS);
  double nsum[WS];
#pragma unroll
  for (int s = 0; s < WS; ++s) nsum[s] = 0.0;
  for (int64_t p = lane; p < ldm / 2; p += 64) {
    const int64_t j0 = 2 * p;
    // c+ = sqrt(e^{2r} - 1) / 2, c- = sqrt(1 - e^{-2r}) / 2; zero on padding
    double cp0 = 0.0, cm0 = 0.0, cp1 = 0.0, cm1 = 0.0;
    if (j0 < M) {
      const double r0 = r[j0];
      cp0 = 0.5 * sqrt(expm1(2.0 * r0));
      cm0 = 0.5 * sqrt(-expm1(-2.0 * r0));
    }
    if (j0 + 1 < M) {
      const double r1 = r[j0 + 1];
      cp1 = 0.5 * sqrt(expm1(2.0 * r1));
      cm1 = 0.5 * sqrt(-expm1(-2.0 * r1));
    }
#pragma unroll
    for (int s = 0; s < WS; ++s) {
      if (s >= nk) break;
      const int64_t k = k0 + s;
      // column stride ldm (FP64, FP32) or 2 ldm (split, hi and lo
      // interleaved); the T-split form stores column pairs, beta from E2 on
      int64_t col_a, col_b;
      if constexpr (PREC == MP_FP64 || PREC == MP_FP32) {
        col_a = k * ldm + j0;
        col_b = (E + k) * ldm + j0;
      } else if constexpr (PREC == MP_SPLIT1T_FP16 || PREC == MP_SPLIT1T_F8) {
        col_a = split1t_offset(k, j0, ldm);
        col_b = split1t_offset(split1t_half(E) + k, j0, ldm);
      } else {
        col_a = k * 2 * ldm + 64 * (j0 >> 5) + (j0 & 31);
        col_b = (E + k) * 2 * ldm + 64 * (j0 >> 5) + (j0 & 31);
      }
      uint64_t c0 = (uint64_t)(g0 + k), c1 = (uint64_t)p, c2 = net, c3 = 0;
      if (j0 < M) philox4x64_10(c0, c1, c2, c3, seed, 0);
      if constexpr (PREC == MP_FP64) {
        double w1 = 0.0, w2 = 0.0, w3 = 0.0, w4 = 0.0;
        if (j0 < M) {
          box_muller(c0, c1, w1, w2);
          if (j0 + 1 < M) box_muller(c2, c3, w3, w4);
        }
        const double a0 = cp0 * w1 + cm0 * w2, b0 = cp0 * w1 - cm0 * w2;
        const double a1 = cp1 * w3 + cm1 * w4, b1 = cp1 * w3 - cm1 * w4;
        store_pair_f64(ab, col_a, a0, a1);
        store_pair_f64(ab, col_b, b0, b1);
        nsum[s] += a0 * b0 + a1 * b1;
      } else {
        float w1 = 0.0f, w2 = 0.0f, w3 = 0.0f, w4 = 0.0f;
        if (j0 < M) {
          box_muller_f32(c0, c1, w1, w2);
          if (j0 + 1 < M) box_muller_f32(c2, c3, w3, w4);
        }
        const float fp0 = (float)cp0, fm0 = (float)cm0, fp1 = (float)cp1, fm1 = (float)cm1;
        const float a0 = fp0 * w1 + fm0 * w2, b0 = fp0 * w1 - fm0 * w2;
        const float a1 = fp1 * w3 + fm1 * w4, b1 = fp1 * w3 - fm1 * w4;
        // the pair forms store the FP16 operand (and then its e4m3 copy)
        constexpr int SP = PREC == MP_SPLIT1T_F8 ? MP_SPLIT1T_FP16 : PREC;
        double ya0, ya1, yb0, yb1;
        store_pair_f32<SP>(ab, col_a, a0, a1, ya0, ya1);
        store_pair_f32<SP>(ab, col_b, b0, b1, yb0, yb1);
        nsum[s] += ya0 * yb0 + ya1 * yb1;
        if constexpr (PREC == MP_SPLIT1T_F8) {
          // e4m3 copies of the stored FP16 values, after the FP16 part
          uint8_t* b8 = (uint8_t*)ab + 4 * split1t_half(E) * ldm;
          const int64_t e2 = split1t_half(E);
          // lanes 2q and 2q + 1 hold modes 4q' .. 4q' + 3 of a 64-mode block:
          // the even lane stores the four codes as one word
          const uint32_t ca = e4m3_pair((float)ya0, (float)ya1);
          const uint32_t cb = e4m3_pair((float)yb0, (float)yb1);
          const uint32_t na = (uint32_t)__shfl_xor((int)ca, 1, 64);
          const uint32_t nb = (uint32_t)__shfl_xor((int)cb, 1, 64);
          if ((lane & 1) == 0) {
            *(uint32_t*)(b8 + pair8_offset(k, j0, ldm)) = ca | (na << 16);
            *(uint32_t*)(b8 + pair8_offset(e2 + k, j0, ldm)) = cb | (nb << 16);
          }
          if ((E & 1) && k == E - 1) {
            *(uint16_t*)(b8 + pair8_offset(k, j0, ldm) + 64) = 0;
            *(uint16_t*)(b8 + pair8_offset(e2 + k, j0, ldm) + 64) = 0;
          }
        }
        if constexpr (PREC == MP_SPLIT1T_FP16 || PREC == MP_SPLIT1T_F8) {
          // odd E: the last sample (even k) shares its pairs with the padding
          // columns E and E2 + E, which the GEMM reads; they hold zeros
          if ((E & 1) && k == E - 1) {
            double z0, z1;
            store_pair_f32<SP>(ab, col_a + 32, 0.0f, 0.0f, z0, z1);
            store_pair_f32<SP>(ab, col_b + 32, 0.0f, 0.0f, z0, z1);
          }
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < WS; ++s) {
    const double v = wave_sum(nsum[s]);
    if (lane == 0 && s < nk) n_out[k0 + s] = v;
  }
}

mp_status sample_launch(int32_t M, int64_t g0, int64_t E, const double* r, uint64_t seed,
                        uint32_t net, mp_precision prec, void* ab, double* n_out,
                        hipStream_t stream) {
  const int64_t ldm = ld_modes(M);
  const int64_t ws = prec == MP_FP64 ? wave_samples<MP_FP64>() : wave_samples<MP_FP32>();
  const int64_t blocks = (E + 4 * ws - 1) / (4 * ws);
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
    case MP_SPLIT1_FP16:  // the same split sample layout
      hipLaunchKernelGGL(sample_kernel<MP_SPLIT_FP16>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         M, ldm, g0, E, r, seed, net, ab, n_out);
      break;
    case MP_SPLIT1T_FP16:
      hipLaunchKernelGGL(sample_kernel<MP_SPLIT1T_FP16>, dim3((unsigned)blocks), dim3(256), 0,
                         stream, M, ldm, g0, E, r, seed, net, ab, n_out);
      break;
    case MP_SPLIT1T_F8:
      hipLaunchKernelGGL(sample_kernel<MP_SPLIT1T_F8>, dim3((unsigned)blocks), dim3(256), 0,
                         stream, M, ldm, g0, E, r, seed, net, ab, n_out);
      break;
    default:
      set_error("mp_sample: unknown precision %d", (int)prec);
      return MP_ERR_ARG;
  }
  MP_HIP_LAUNCH_CHECK("mp_sample launch");
  return MP_OK;
}

}  // namespace mp
