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
    default: return 4;  // hi + lo values of 2 bytes each
  }
}

inline size_t elem_bytes_c(mp_precision p) { return p == MP_FP64 ? 8 : 4; }

inline bool valid_prec(int p) { return p >= MP_FP64 && p <= MP_SPLIT1T_FP16; }

// Storage columns per half of the MP_SPLIT1T_FP16 sample operand: E rounded
// up to even, so that the beta columns start a column pair.
__host__ __device__ inline int64_t split1t_half(int64_t E) { return E + (E & 1); }

// Wave-wide sums (64 lanes) via cross-lane shuffles.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mp
