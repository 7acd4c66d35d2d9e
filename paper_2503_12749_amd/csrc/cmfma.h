// Complex tile products on the FP32 matrix cores, shared by the pair-moment
// sums and the joint-distribution box contractions.
//
// A 128 x 128 complex tile C += A B^T over a slab of kSlab samples, with the
// four real planes of the operands in LDS as [sample][row] (A re, A im) and
// [sample][col] (B re, B im), each row kTile floats.  v_mfma_f32_32x32x2f32
// takes lane l's A[l % 32][l / 32] and B[l / 32][l % 32], so every fragment
// is one LDS float per lane; output register r of lane l is element
// (8 (r / 4) + 4 (l / 32) + r % 4, l % 32) of a 32 x 32 block.  Wave
// (wi, wj) owns rows [64 wi, 64 wi + 64) and columns [64 wj, 64 wj + 64):
//   Re += Ar Br^T - Ai Bi^T,   Im += Ar Bi^T + Ai Br^T.
#pragma once

#include <hip/hip_runtime.h>

namespace mp {

namespace cmfma {

typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kTile = 128;  // rows and columns of the complex tile
constexpr int kSlab = 32;   // samples per slab

__device__ __attribute__((always_inline)) inline void zero(f32x16 (&accR)[2][2],
                                                            f32x16 (&accI)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        accR[a][b][q] = 0.f;
        accI[a][b][q] = 0.f;
      }
}

// One slab: are, aim, bre, bim point at [kSlab][kTile] planes in LDS.
__device__ __attribute__((always_inline)) inline void slab(const float* are, const float* aim,
                                                            const float* bre, const float* bim,
                                                            int wi, int wj, int lane,
                                                            f32x16 (&accR)[2][2],
                                                            f32x16 (&accI)[2][2]) {
  const int lr = lane & 31, lh = lane >> 5;
#pragma unroll 4
  for (int t = 0; t < kSlab / 2; ++t) {
    const int kk = 2 * t + lh;
    float ar[2], ai[2], br[2], bi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      ar[a] = are[kk * kTile + 64 * wi + 32 * a + lr];
      ai[a] = aim[kk * kTile + 64 * wi + 32 * a + lr];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      br[b] = bre[kk * kTile + 64 * wj + 32 * b + lr];
      bi[b] = bim[kk * kTile + 64 * wj + 32 * b + lr];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accR[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a], br[b], accR[a][b], 0, 0, 0);
        accR[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[a], bi[b], accR[a][b], 0, 0, 0);
        accI[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a], bi[b], accI[a][b], 0, 0, 0);
        accI[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[a], br[b], accI[a][b], 0, 0, 0);
      }
  }
}

// Three-product form of one slab: P1 += Ar Br^T, P2 += Ai Bi^T,
// P3 += (Ar + Ai)(Br + Bi)^T, so that Re = P1 - P2 and Im = P3 - P1 - P2.
__device__ __attribute__((always_inline)) inline void slab3(const float* are, const float* aim,
                                                             const float* bre, const float* bim,
                                                             int wi, int wj, int lane,
                                                             f32x16 (&p1)[2][2], f32x16 (&p2)[2][2],
                                                             f32x16 (&p3)[2][2]) {
  const int lr = lane & 31, lh = lane >> 5;
#pragma unroll 4
  for (int t = 0; t < kSlab / 2; ++t) {
    const int kk = 2 * t + lh;
    float ar[2], ai[2], br[2], bi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      ar[a] = are[kk * kTile + 64 * wi + 32 * a + lr];
      ai[a] = aim[kk * kTile + 64 * wi + 32 * a + lr];
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      br[b] = bre[kk * kTile + 64 * wj + 32 * b + lr];
      bi[b] = bim[kk * kTile + 64 * wj + 32 * b + lr];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        p1[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a], br[b], p1[a][b], 0, 0, 0);
        p2[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[a], bi[b], p2[a][b], 0, 0, 0);
        p3[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[a] + ai[a], br[b] + bi[b], p3[a][b], 0,
                                                        0, 0);
      }
  }
}

// Tile row and column of output register q of 32 x 32 block (a, b).
__device__ __attribute__((always_inline)) inline int out_row(int wi, int a, int q, int lane) {
  return 64 * wi + 32 * a + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
}
__device__ __attribute__((always_inline)) inline int out_col(int wj, int b, int lane) {
  return 64 * wj + 32 * b + (lane & 31);
}

}  // namespace cmfma

}  // namespace mp
