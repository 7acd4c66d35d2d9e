// Internal helpers of libmpgbs: status reporting, layout arithmetic, and the
// small device utilities shared by the kernels of this library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "../../include/mpgbs.h"

namespace mp {

// Thread-local message of the last failed call (see mp_last_error).
void set_error(const char* fmt, ...);
void clear_error();

#define MP_CHECK_ARG(cond, code, ...)      \
  do {                                     \
    if (!(cond)) {                         \
      ::mp::set_error(__VA_ARGS__);        \
      return code;                         \
    }                                      \
  } while (0)

#define MP_HIP_LAUNCH_CHECK(what)                                                  \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) {                                                        \
      ::mp::set_error("%s: %s", what, hipGetErrorString(e_));                      \
      return MP_ERR_HIP;                                                           \
    }                                                                              \
  } while (0)

constexpr int kLdAlign = 128;  // mode padding (GEMM tile multiple)

// Output of the occupation-fused GEMM: per (slot, sample) the partial sums of
// alpha'_j beta'_j over the modes of one bin run inside one 128-mode block.
// Run q owns the slots slot_off[q] + (block - run_lo[q] / 128) for the blocks
// it touches.  Each slot holds, per sample, (re, im) from the wave with the
// Re rows of alpha' and (re, im) from the wave with the Im rows: four floats
// at part[(slot * E + sample) * 4].
struct FusedOut {
  float* part;
  int64_t E;
  int n_runs;
  int run_lo[MP_MAX_RUNS], run_hi[MP_MAX_RUNS], slot_off[MP_MAX_RUNS];
};

// One network of a grouped split-precision GEMM launch.
struct GroupNet {
  const uint16_t* A;  // packed [Re T; Im T], hi and lo interleaved in 32-blocks
  const uint16_t* B;  // sampled amplitudes, hi and lo interleaved in 32-blocks
  float* C;
  int64_t ldm, ncols;
  float out_scale;
  int f8_scale_a;  // MP_SPLIT1T_F8: block scale of the FP8 product's A operand
  FusedOut fo;  // the occupation-fused epilogue's output (C unused then)
};

// Slots of the fused partials for a set of runs; fills slot_off and returns
// the total.
inline int64_t fused_slots(int n_runs, const int* run_lo, const int* run_hi, int* slot_off) {
  int64_t s = 0;
  for (int q = 0; q < n_runs; ++q) {
    slot_off[q] = (int)s;
    s += (run_hi[q] - 1) / 128 - run_lo[q] / 128 + 1;
  }
  return s;
}

inline int64_t ld_modes(int32_t M) { return ((int64_t)M + kLdAlign - 1) / kLdAlign * kLdAlign; }

inline size_t elem_bytes_ab(mp_precision p) {
  switch (p) {
    case MP_FP64: return 8;
    case MP_FP32: return 4;
    case MP_SPLIT1T_FP16: return 2;  // one FP16 value (storage columns: split1t_half)
    case MP_SPLIT1T_F8: return 3;    // one FP16 value and its e4m3 copy
    default: return 4;  // hi + lo values of 2 bytes each
  }
}

inline size_t elem_bytes_c(mp_precision p) { return p == MP_FP64 ? 8 : 4; }

inline bool valid_prec(int p) { return p >= MP_FP64 && p <= MP_SPLIT1T_F8; }

// Storage columns per half of the MP_SPLIT1T_FP16 and MP_SPLIT1T_F8 sample
// operands: E rounded up to even, so that the beta columns start a column pair.
__host__ __device__ inline int64_t split1t_half(int64_t E) { return E + (E & 1); }

// Precisions whose sample operand is stored in column pairs (split1t_half).
inline bool pair_columns(mp_precision p) { return p == MP_SPLIT1T_FP16 || p == MP_SPLIT1T_F8; }

// Columns of the sample operand: 2 E, or the storage columns of the pair forms.
inline int64_t ab_columns(int64_t E, mp_precision p) {
  return pair_columns(p) ? 2 * split1t_half(E) : 2 * E;
}

// x in OCP e4m3 (4 exponent bits, bias 7, 3 mantissa bits; no infinities,
// 0x7F and 0xFF are NaN), rounded to nearest even; magnitudes of 448, the
// largest finite value, and above give 448.
__host__ __device__ inline uint8_t e4m3_rne(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  const uint32_t sign = (u >> 24) & 0x80u, a = u & 0x7FFFFFFFu;
  if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);  // |x| >= 448
  if (a >= 0x3C800000u) {                                // |x| >= 2^-6: normal
    const uint32_t r = a + 0x7FFFFu + ((a >> 20) & 1u);  // keep 3 mantissa bits
    const uint32_t v = (((r >> 23) - 120u) << 3) | ((r >> 20) & 7u);
    return (uint8_t)(sign | v);
  }
  // subnormal: multiples of 2^-9 (code 8 is 2^-6, the smallest normal)
  const float m = __builtin_fabsf(x) * 512.0f;  // exact, below 8
  uint32_t q = (uint32_t)m;
  const float f = m - (float)q;
  if (f > 0.5f || (f == 0.5f && (q & 1u))) ++q;
  return (uint8_t)(sign | q);
}

// Scale exponent of the e4m3 remainder of a prescaled FP16 operand: with the
// prescale 2^e of fp16 T (|T_ij| <= 1, so |x| <= 2^e) the remainder x - hi is
// at most one unit in the last place of hi, 2^(e - 10), and 2^(18 - e) maps
// it to at most 256 (e4m3 reaches 448).
__host__ __device__ inline int e4m3_lo_scale_exp(int e) { return 18 - e; }

// Byte offset of entry j of row (or storage column) r in an e4m3 operand
// stored in pairs: rows 2q and 2q + 1 share, for each 64-deep block, one
// 128-byte line (row 2q's 64 bytes, then row 2q + 1's).
__host__ __device__ inline int64_t pair8_offset(int64_t r, int64_t j, int64_t ldm) {
  return (r >> 1) * 2 * ldm + 128 * (j >> 6) + 64 * (r & 1) + (j & 63);
}

// Wave-wide sums (64 lanes) via cross-lane shuffles.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mp
