// Linear-network propagation of the phase-space amplitudes on CDNA4 MFMA.
//
// The paper's network step maps alpha' = T alpha and beta' = T* beta (main
// text, characteristics of the linear-network equation; loss enters as a
// sub-unitary T).  alpha and beta are real, so the complex products reduce to
// one real GEMM
//     C (2 ldm x 2E) = A (2 ldm x ldm) * B (ldm x 2E),  A = [Re T; Im T],
// with B = [alpha | beta] column-major (each sample column contiguous over the
// modes) and C column-major.  Both operands are K-contiguous, so every lane of
// a wavefront feeds its MFMA fragment from one 16-byte LDS read.
//
// Kernels: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_32x32x2) and split
// BF16 (three v_mfma_f32_32x32x16_bf16 products hi*hi + hi*lo + lo*hi with
// FP32 accumulation).  Tile 128 x 128 per 256-thread workgroup, four waves of
// 64 x 64, LDS double buffering, and a tile order grouped per XCD so that the
// workgroups sharing one L2 reuse the same rows of A and columns of B.
#include <hip/hip_runtime.h>

#include "common.h"

namespace mp {

typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

constexpr int BM = 128;  // tile rows (output rows of C)
constexpr int BN = 128;  // tile columns (samples, alpha and beta columns)
constexpr int kThreads = 256;
constexpr int kXcds = 8;     // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kGroupM = 8;   // row tiles per group in the grouped tile order

// ---------------------------------------------------------------- packing

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// A[i][j] (row-major, 2 ldm x ldm) from T (row-major complex M x M).
template <int PREC>
__global__ void pack_transmission(const double* __restrict__ T, int M, int64_t ldm,
                                  void* __restrict__ A) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = 2 * ldm * ldm;
  if (idx >= total) return;
  int64_t row = idx / ldm, j = idx % ldm;
  int64_t i = row < ldm ? row : row - ldm;
  double v = 0.0;
  if (i < M && j < M) v = T[2 * (i * M + j) + (row < ldm ? 0 : 1)];
  if constexpr (PREC == MP_FP64) {
    ((double*)A)[idx] = v;
  } else if constexpr (PREC == MP_FP32) {
    ((float*)A)[idx] = (float)v;
  } else if constexpr (PREC == MP_SPLIT_BF16) {
    uint16_t hi = f32_to_bf16_rne((float)v);
    uint16_t lo = f32_to_bf16_rne((float)(v - (double)bf16_to_f32(hi)));
    ((uint16_t*)A)[idx] = hi;
    ((uint16_t*)A)[idx + total] = lo;
  } else {
    _Float16 hi = (_Float16)v;
    _Float16 lo = (_Float16)((v - (double)hi) * 2048.0);
    ((_Float16*)A)[idx] = hi;
    ((_Float16*)A)[idx + total] = lo;
  }
}

// ---------------------------------------------------------------- tile order

// Maps the linear block id to (tile_m, tile_n).  Blocks are dispatched to the
// XCDs round-robin, so block b runs on XCD b % 8; each XCD gets one
// contiguous range of the grouped tile sequence.
__device__ inline bool tile_of_block(int tiles_m, int tiles_n, int& tm, int& tn) {
  int total = tiles_m * tiles_n;
  int per_xcd = (total + kXcds - 1) / kXcds;
  int b = blockIdx.x;
  int t = (b % kXcds) * per_xcd + b / kXcds;
  if (t >= total) return false;
  int group = kGroupM * tiles_n;
  int gid = t / group;
  int first_m = gid * kGroupM;
  int gsize = min(kGroupM, tiles_m - first_m);
  int r = t % group;
  tm = first_m + r % gsize;
  tn = r / gsize;
  return true;
}

// ---------------------------------------------------------------- loaders

// Global -> register staging of one K-slab of a 128-row (or 128-column)
// operand tile: 128 rows of BK contiguous elements, as 16-byte vectors.
template <typename E, int BK>
struct Slab {
  static constexpr int kVec = 16 / sizeof(E);
  static constexpr int kVecsPerRow = BK / kVec;
  static constexpr int kPerThread = 128 * kVecsPerRow / kThreads;
  u32x4 v[kPerThread];

  // rows are valid when row < nrows (columns of B beyond 2E read as zero)
  __device__ inline void load(const E* __restrict__ base, int64_t ld, int64_t row0, int64_t k0,
                              int64_t nrows) {
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      int vi = threadIdx.x + i * kThreads;
      int row = vi / kVecsPerRow, kv = vi % kVecsPerRow;
      int64_t grow = row0 + row;
      if (grow < nrows) {
        v[i] = *(const u32x4*)(base + grow * ld + k0 + kv * kVec);
      } else {
        v[i] = u32x4{0, 0, 0, 0};
      }
    }
  }
  template <int LDK>
  __device__ inline void store(E* lds) const {
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      int vi = threadIdx.x + i * kThreads;
      int row = vi / kVecsPerRow, kv = vi % kVecsPerRow;
      *(u32x4*)(lds + row * LDK + kv * kVec) = v[i];
    }
  }
};

// ---------------------------------------------------------------- FP64

// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16]; output
// register r is row (l/16) + 4 r, column l%16.  Within one BK = 16 slab lane
// group h = l/16 supplies k = 4h + s at MFMA step s (the same permutation of
// k on both operands), so each lane reads 4 consecutive doubles per row.
__global__ __launch_bounds__(kThreads) void gemm_f64(const double* __restrict__ A,
                                                     const double* __restrict__ B,
                                                     double* __restrict__ C, int64_t ldm,
                                                     int64_t ncols) {
  constexpr int BK = 16, LDK = BK + 2;
  __shared__ __attribute__((aligned(16))) double sA[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) double sB[2][BN * LDK];
  const int tiles_m = (int)(2 * ldm / BM), tiles_n = (int)((ncols + BN - 1) / BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lh = lane >> 4;

  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0, 0, 0, 0};

  Slab<double, BK> la, lb;
  const int KT = (int)(ldm / BK);
  la.load(A, ldm, m0, 0, 2 * ldm);
  lb.load(B, ldm, n0, 0, ncols);
  la.store<LDK>(sA[0]);
  lb.store<LDK>(sB[0]);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) {
      la.load(A, ldm, m0, (int64_t)(kt + 1) * BK, 2 * ldm);
      lb.load(B, ldm, n0, (int64_t)(kt + 1) * BK, ncols);
    }
    double a[4][4], b[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double* pa = sA[cur] + (wm * 64 + i * 16 + lr) * LDK + 4 * lh;
      const double* pb = sB[cur] + (wn * 64 + i * 16 + lr) * LDK + 4 * lh;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a[i][s] = pa[s];
        b[i][s] = pb[s];
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    if (kt + 1 < KT) {
      la.store<LDK>(sA[cur ^ 1]);
      lb.store<LDK>(sB[cur ^ 1]);
    }
    __syncthreads();
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int64_t col = n0 + wn * 64 + j * 16 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // the f64 16x16 output interleaves rows: register r holds row lh + 4 r
      double* p = C + col * ldc + m0 + wm * 64 + i * 16 + lh;
      p[0] = acc[i][j][0];
      p[4] = acc[i][j][1];
      p[8] = acc[i][j][2];
      p[12] = acc[i][j][3];
    }
  }
}

// ---------------------------------------------------------------- FP32

// v_mfma_f32_32x32x2f32: lane l holds A[l%32][l/32], B[l/32][l%32]; output
// register r is row 8 (r/4) + 4 (l/32) + r%4, column l%32.  Within one
// BK = 32 slab lane half h supplies k = 16h + s at step s.
__global__ __launch_bounds__(kThreads) void gemm_f32(const float* __restrict__ A,
                                                     const float* __restrict__ B,
                                                     float* __restrict__ C, int64_t ldm,
                                                     int64_t ncols) {
  constexpr int BK = 32, LDK = BK + 4;
  __shared__ __attribute__((aligned(16))) float sA[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) float sB[2][BN * LDK];
  const int tiles_m = (int)(2 * ldm / BM), tiles_n = (int)((ncols + BN - 1) / BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  Slab<float, BK> la, lb;
  const int KT = (int)(ldm / BK);
  la.load(A, ldm, m0, 0, 2 * ldm);
  lb.load(B, ldm, n0, 0, ncols);
  la.store<LDK>(sA[0]);
  lb.store<LDK>(sB[0]);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) {
      la.load(A, ldm, m0, (int64_t)(kt + 1) * BK, 2 * ldm);
      lb.load(B, ldm, n0, (int64_t)(kt + 1) * BK, ncols);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // 4 groups of 4 consecutive k per lane
      f32x4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *(const f32x4*)(sA[cur] + (wm * 64 + i * 32 + lr) * LDK + 16 * lh + 4 * q);
        b[i] = *(const f32x4*)(sB[cur] + (wn * 64 + i * 32 + lr) * LDK + 16 * lh + 4 * q);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < KT) {
      la.store<LDK>(sA[cur ^ 1]);
      lb.store<LDK>(sB[cur ^ 1]);
    }
    __syncthreads();
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    int64_t col = n0 + wn * 64 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        int64_t row = m0 + wm * 64 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]};
      }
  }
}

// ---------------------------------------------------------------- split BF16

// v_mfma_f32_32x32x16_bf16: lane l holds A[l%32][8 (l/32) + e], e = 0..7, and
// the same for B; outputs as in the 32x32 FP32 form.  Within one BK = 32 slab
// lane half h supplies k = 16h + 8s + e at step s (s = 0, 1).  Each operand is
// x = hi + lo (both BF16); the product keeps hi*hi + hi*lo + lo*hi.
__global__ __launch_bounds__(kThreads) void gemm_split_bf16(const uint16_t* __restrict__ A,
                                                            const uint16_t* __restrict__ B,
                                                            float* __restrict__ C, int64_t ldm,
                                                            int64_t ncols) {
  constexpr int BK = 32, LDK = BK + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sAh[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[2][BN * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[2][BN * LDK];
  const int tiles_m = (int)(2 * ldm / BM), tiles_n = (int)((ncols + BN - 1) / BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;
  const int64_t planeA = 2 * ldm * ldm, planeB = ldm * ncols;
  const uint16_t* Al = A + planeA;
  const uint16_t* Bl = B + planeB;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  Slab<uint16_t, BK> lah, lal, lbh, lbl;
  const int KT = (int)(ldm / BK);
  lah.load(A, ldm, m0, 0, 2 * ldm);
  lal.load(Al, ldm, m0, 0, 2 * ldm);
  lbh.load(B, ldm, n0, 0, ncols);
  lbl.load(Bl, ldm, n0, 0, ncols);
  lah.store<LDK>(sAh[0]);
  lal.store<LDK>(sAl[0]);
  lbh.store<LDK>(sBh[0]);
  lbl.store<LDK>(sBl[0]);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) {
      const int64_t k0 = (int64_t)(kt + 1) * BK;
      lah.load(A, ldm, m0, k0, 2 * ldm);
      lal.load(Al, ldm, m0, k0, 2 * ldm);
      lbh.load(B, ldm, n0, k0, ncols);
      lbl.load(Bl, ldm, n0, k0, ncols);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int offA = (wm * 64 + i * 32 + lr) * LDK + 16 * lh + 8 * s;
        const int offB = (wn * 64 + i * 32 + lr) * LDK + 16 * lh + 8 * s;
        ah[i] = *(const bf16x8*)(sAh[cur] + offA);
        al[i] = *(const bf16x8*)(sAl[cur] + offA);
        bh[i] = *(const bf16x8*)(sBh[cur] + offB);
        bl[i] = *(const bf16x8*)(sBl[cur] + offB);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < KT) {
      lah.store<LDK>(sAh[cur ^ 1]);
      lal.store<LDK>(sAl[cur ^ 1]);
      lbh.store<LDK>(sBh[cur ^ 1]);
      lbl.store<LDK>(sBl[cur ^ 1]);
    }
    __syncthreads();
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    int64_t col = n0 + wn * 64 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        int64_t row = m0 + wm * 64 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]};
      }
  }
}

// ---------------------------------------------------------------- host side

size_t propagate_workspace(int32_t M, mp_precision prec) {
  int64_t ldm = ld_modes(M);
  size_t elems = (size_t)(2 * ldm * ldm);
  switch (prec) {
    case MP_FP64: return elems * 8;
    case MP_FP32: return elems * 4;
    default: return elems * 4;  // two 16-bit planes
  }
}

static int grid_tiles(int64_t ldm, int64_t ncols) {
  int64_t tiles = (2 * ldm / BM) * ((ncols + BN - 1) / BN);
  int64_t per = (tiles + kXcds - 1) / kXcds;
  return (int)(per * kXcds);
}

mp_status propagate_launch(int32_t M, int64_t E, const double* T, mp_precision prec,
                           const void* ab, void* C, void* ws, hipStream_t stream) {
  const int64_t ldm = ld_modes(M);
  const int64_t ncols = 2 * E;
  const int64_t pack_total = 2 * ldm * ldm;
  const int pack_blocks = (int)((pack_total + 255) / 256);
  const int grid = grid_tiles(ldm, ncols);
  switch (prec) {
    case MP_FP64:
      hipLaunchKernelGGL(pack_transmission<MP_FP64>, dim3(pack_blocks), dim3(256), 0, stream, T, M,
                         ldm, ws);
      hipLaunchKernelGGL(gemm_f64, dim3(grid), dim3(kThreads), 0, stream, (const double*)ws,
                         (const double*)ab, (double*)C, ldm, ncols);
      break;
    case MP_FP32:
      hipLaunchKernelGGL(pack_transmission<MP_FP32>, dim3(pack_blocks), dim3(256), 0, stream, T, M,
                         ldm, ws);
      hipLaunchKernelGGL(gemm_f32, dim3(grid), dim3(kThreads), 0, stream, (const float*)ws,
                         (const float*)ab, (float*)C, ldm, ncols);
      break;
    case MP_SPLIT_BF16:
      hipLaunchKernelGGL(pack_transmission<MP_SPLIT_BF16>, dim3(pack_blocks), dim3(256), 0, stream,
                         T, M, ldm, ws);
      hipLaunchKernelGGL(gemm_split_bf16, dim3(grid), dim3(kThreads), 0, stream,
                         (const uint16_t*)ws, (const uint16_t*)ab, (float*)C, ldm, ncols);
      break;
    default:
      set_error("mp_propagate: precision %d not supported by this build", (int)prec);
      return MP_ERR_UNSUPPORTED;
  }
  MP_HIP_LAUNCH_CHECK("mp_propagate launch");
  return MP_OK;
}

}  // namespace mp
