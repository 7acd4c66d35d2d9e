// Diagnostics: the matrix cores' sustained rate on this device.  Every wave
// issues rounds of independent MFMAs on register-resident operands, with
// no memory traffic inside the loop, so the launch runs at whatever clock the
// part holds under a pure matrix load.  That rate, not the nominal peak, is
// the ceiling a GEMM of the same instruction can approach.
#include <hip/hip_runtime.h>

#include "common.h"

namespace mp {

typedef __attribute__((ext_vector_type(16))) float burn_f32x16;
typedef __attribute__((ext_vector_type(4))) double burn_f64x4;
typedef __attribute__((ext_vector_type(8))) _Float16 burn_f16x8;
typedef __attribute__((ext_vector_type(8))) int burn_i32x8;

// Independent accumulators per wave: 16 of 16 registers (FP16, FP32) or 32 of
// 8 (FP64), 256 accumulator registers either way, as in the GEMMs.
template <int KIND>
constexpr int burn_chains() { return KIND == 2 ? 32 : 16; }

// Flops per chain and round of each kind (one MFMA; kind 3: four FP16 MFMAs
// and one FP8 MFMA, the FP8-correction GEMM's mix per 64-deep block).
static double burn_flops(int kind) {
  switch (kind) {
    case 0: return 2.0 * 32 * 32 * 16;  // v_mfma_f32_32x32x16_f16
    case 1: return 2.0 * 32 * 32 * 2;   // v_mfma_f32_32x32x2f32
    case 2: return 2.0 * 16 * 16 * 4;   // v_mfma_f64_16x16x4f64
    default: return 4 * 2.0 * 32 * 32 * 16 + 2.0 * 32 * 32 * 64;
  }
}

template <int KIND>
__global__ __launch_bounds__(256, 1) void mfma_burn(int64_t iters, double* __restrict__ sink) {
  const int t = threadIdx.x;
  // operands that differ across lanes and are not known to the compiler
  const float x = 1.0f + (float)(t & 63) * (1.0f / 64.0f);
  const float y = 0.5f + (float)((t * 7) & 63) * (1.0f / 128.0f);
  double out = 0.0;
  if constexpr (KIND == 0) {
    burn_f16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (_Float16)(x + 0.125f * e);
      b[e] = (_Float16)(y - 0.0625f * e);
    }
    burn_f32x16 acc[burn_chains<KIND>()];
#pragma unroll
    for (int c = 0; c < burn_chains<KIND>(); ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < burn_chains<KIND>(); ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < burn_chains<KIND>(); ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) out += acc[c][r];
  } else if constexpr (KIND == 3) {
    burn_f16x8 a, b;
    burn_i32x8 a8, b8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (_Float16)(x + 0.125f * e);
      b[e] = (_Float16)(y - 0.0625f * e);
      a8[e] = 0x38383838 + (t & 3);         // e4m3 codes near 1
      b8[e] = 0x30303030 + ((t >> 2) & 3);  // near 1/2
    }
    burn_f32x16 acc[burn_chains<KIND>()];
#pragma unroll
    for (int c = 0; c < burn_chains<KIND>(); ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < burn_chains<KIND>(); ++c)
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
#pragma unroll
      for (int c = 0; c < burn_chains<KIND>(); ++c)
        acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[c], 0, 0, 0, 127, 0,
                                                                 127);
    }
#pragma unroll
    for (int c = 0; c < burn_chains<KIND>(); ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) out += acc[c][r];
  } else if constexpr (KIND == 1) {
    burn_f32x16 acc[burn_chains<KIND>()];
#pragma unroll
    for (int c = 0; c < burn_chains<KIND>(); ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < burn_chains<KIND>(); ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < burn_chains<KIND>(); ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) out += acc[c][r];
  } else {
    constexpr int NC = burn_chains<KIND>();
    const double xd = x, yd = y;
    const burn_f64x4 zero = {0.0, 0.0, 0.0, 0.0};
    // the first round from a zero accumulator, so that every value the loop
    // carries comes out of an MFMA (with zero-initialised accumulators the
    // compiler carried them in VGPRs and copied them to AGPRs and back in
    // every round)
    burn_f64x4 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(xd, yd, zero, 0, 0, 0);
    for (int64_t it = 1; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(xd, yd, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) out += acc[c][r];
  }
  sink[(int64_t)blockIdx.x * blockDim.x + t] = out;
}

}  // namespace mp

using namespace mp;

extern "C" {

mp_status mp_mfma_sustained(int32_t kind, int64_t iters, double* sink, size_t sink_bytes,
                            double* flops, void* stream) {
  clear_error();
  MP_CHECK_ARG(kind >= 0 && kind <= 3, MP_ERR_ARG, "mp_mfma_sustained: kind %d not in [0, 3]",
               kind);
  MP_CHECK_ARG(iters >= 1, MP_ERR_ARG, "mp_mfma_sustained: iters must be >= 1");
  MP_CHECK_ARG(sink, MP_ERR_ARG, "mp_mfma_sustained: null sink");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    set_error("mp_mfma_sustained: device query failed");
    return MP_ERR_HIP;
  }
  MP_CHECK_ARG(sink_bytes >= (size_t)cus * 256 * sizeof(double), MP_ERR_WORKSPACE,
               "mp_mfma_sustained: sink of %zu bytes needed (256 doubles per compute unit)",
               (size_t)cus * 256 * sizeof(double));
  hipStream_t s = (hipStream_t)stream;
  switch (kind) {
    case 0: hipLaunchKernelGGL(mfma_burn<0>, dim3(cus), dim3(256), 0, s, iters, sink); break;
    case 1: hipLaunchKernelGGL(mfma_burn<1>, dim3(cus), dim3(256), 0, s, iters, sink); break;
    case 2: hipLaunchKernelGGL(mfma_burn<2>, dim3(cus), dim3(256), 0, s, iters, sink); break;
    default: hipLaunchKernelGGL(mfma_burn<3>, dim3(cus), dim3(256), 0, s, iters, sink); break;
  }
  MP_HIP_LAUNCH_CHECK("mp_mfma_sustained launch");
  const int chains = kind == 2 ? burn_chains<2>() : burn_chains<0>();
  if (flops) *flops = (double)cus * 4 * chains * (double)iters * burn_flops(kind);
  return MP_OK;
}

}  // extern "C"
