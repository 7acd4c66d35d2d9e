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

#include <cstdlib>

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
                                  void* __restrict__ A, int scale_exp) {
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
    // FP16: A is packed as T * 2^scale_exp so that both halves stay normal
    const double x = ldexp(v, scale_exp);
    _Float16 hi = (_Float16)x;
    _Float16 lo = (_Float16)(x - (double)hi);
    ((_Float16*)A)[idx] = hi;
    ((_Float16*)A)[idx + total] = lo;
  }
}

// ---------------------------------------------------------------- tile order

// Tile order.  Blocks are dispatched to the XCDs round-robin, so block b
// runs on XCD b % 8 and, with one workgroup per CU, the 32 blocks
// b / 8 = 32 s .. 32 s + 31 of every XCD run together in "step" s.
//
// Order 1 (default): in each step all eight XCDs work on the same group of 8
// row tiles, each XCD on its own 4 column tiles, and consecutive steps move
// along the columns.  The A rows of a group are then shared by every XCD
// through the infinity cache (MALL) and fetched from HBM about once per
// group, instead of once per XCD and column block.
// Order 0: each XCD takes one contiguous range of a sequence grouped by 8
// row tiles (XCD-local L2 reuse only).
constexpr int kStepRows = 8, kStepColsPerXcd = 4;

static int tile_order() {
  static int v = [] {
    const char* e = getenv("MPGBS_TILE_ORDER");
    return e ? atoi(e) : 1;
  }();
  return v;
}

__device__ inline bool tile_of_block_mall(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int b = blockIdx.x, x = b % kXcds, q = b / kXcds;
  const int per_xcd = kStepRows * kStepColsPerXcd;   // 32 blocks of one XCD per step
  const int s = q / per_xcd, j = q % per_xcd;
  const int cols_per_step = kXcds * kStepColsPerXcd;  // 32 column tiles per step
  const int n_cg = (tiles_n + cols_per_step - 1) / cols_per_step;
  const int rg = s / n_cg, cg = s % n_cg;
  tm = rg * kStepRows + j % kStepRows;
  tn = cg * cols_per_step + x * kStepColsPerXcd + j / kStepRows;
  return tm < tiles_m && tn < tiles_n;
}

__host__ __device__ inline int mall_grid_blocks(int tiles_m, int tiles_n) {
  const int n_cg = (tiles_n + kXcds * kStepColsPerXcd - 1) / (kXcds * kStepColsPerXcd);
  const int n_rg = (tiles_m + kStepRows - 1) / kStepRows;
  return n_rg * n_cg * kXcds * kStepRows * kStepColsPerXcd;
}

__device__ inline bool tile_of_block_grouped(int tiles_m, int tiles_n, int& tm, int& tn) {
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

__device__ inline bool tile_of_block(int tiles_m, int tiles_n, int order, int& tm, int& tn) {
  return order == 1 ? tile_of_block_mall(tiles_m, tiles_n, tm, tn)
                    : tile_of_block_grouped(tiles_m, tiles_n, tm, tn);
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
                                                     int64_t ncols, int order) {
  constexpr int BK = 16, LDK = BK + 2;
  __shared__ __attribute__((aligned(16))) double sA[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) double sB[2][BN * LDK];
  const int tiles_m = (int)(2 * ldm / BM), tiles_n = (int)((ncols + BN - 1) / BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
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
                                                     int64_t ncols, int order) {
  constexpr int BK = 32, LDK = BK + 4;
  __shared__ __attribute__((aligned(16))) float sA[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) float sB[2][BN * LDK];
  const int tiles_m = (int)(2 * ldm / BM), tiles_n = (int)((ncols + BN - 1) / BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
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
                                                            int64_t ncols, int order) {
  constexpr int BK = 32, LDK = BK + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sAh[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sAl[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sBh[2][BN * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sBl[2][BN * LDK];
  const int tiles_m = (int)(2 * ldm / BM), tiles_n = (int)((ncols + BN - 1) / BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
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

// ---------------------------------------------------------------- split, 256 x 256

// Split-precision GEMM with a 256 x 256 workgroup tile: four waves of
// 128 x 128 (4 x 4 MFMA 32x32x16 tiles, 256 accumulator registers per lane),
// BK = 32, two LDS stages of four 256 x 32 planes (A hi/lo, B hi/lo).  Rows
// of a plane are 64 bytes without padding; 16-byte chunk c of row r is
// stored at chunk c ^ f(r), f(r) = ((r >> 1) & 3) ^ ((r >> 3) & 1), which keeps
// both the 16-byte fragment reads (32 consecutive rows, one chunk) and the
// staging writes free of bank conflicts for 32- and 64-bank LDS.  Within a
// k16 step the three products run as three sweeps over the 16 tiles, so
// consecutive MFMAs never depend on each other.  `out_scale` undoes the
// power-of-two prescale of the packed A operand.
template <typename H>
struct SplitMfma;
template <>
struct SplitMfma<__bf16> {
  typedef bf16x8 frag;
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SplitMfma<_Float16> {
  typedef f16x8 frag;
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

__device__ inline int swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }

constexpr int S_BM = 256, S_BN = 256, S_BK = 32;
constexpr int S_PLANE = S_BM * S_BK;  // elements of one LDS plane

template <typename H>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_256(const uint16_t* __restrict__ A,
                                                              const uint16_t* __restrict__ B,
                                                              float* __restrict__ C, int64_t ldm,
                                                              int64_t ncols, float out_scale, int order) {
  typedef typename SplitMfma<H>::frag frag;
  __shared__ __attribute__((aligned(16))) uint16_t lds[2][4][S_PLANE];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * S_BM, n0 = (int64_t)tn * S_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;
  const int64_t planeA = 2 * ldm * ldm, planeB = ldm * ncols;

  // staging: thread tid moves 16-byte vector vi = tid + 256 i (i < 4) of each
  // plane: row vi >> 2, chunk vi & 3
  const uint16_t* src[4];
  int64_t nvalid[4];
  src[0] = A + m0 * ldm;
  src[1] = A + planeA + m0 * ldm;
  src[2] = B + n0 * ldm;
  src[3] = B + planeB + n0 * ldm;
  nvalid[0] = nvalid[1] = S_BM;
  nvalid[2] = nvalid[3] = ncols - n0;
  u32x4 stage[4][4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int vi = tid + i * kThreads;
        const int row = vi >> 2, c = vi & 3;
        if (row < nvalid[p])
          stage[p][i] = *(const u32x4*)(src[p] + (int64_t)row * ldm + k0 + c * 8);
        else
          stage[p][i] = u32x4{0, 0, 0, 0};
      }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int vi = tid + i * kThreads;
        const int row = vi >> 2, c = vi & 3;
        *(u32x4*)(&lds[st][p][row * S_BK + ((c ^ swz(row)) << 3)]) = stage[p][i];
      }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / S_BK);
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) gload((int64_t)(kt + 1) * S_BK);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      frag ah[4], al[4], bh[4], bl[4];
      const int chunk = 2 * lh + s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra = wm * 128 + i * 32 + lr;
        const int rb = wn * 128 + i * 32 + lr;
        const int oa = ra * S_BK + ((chunk ^ swz(ra)) << 3);
        const int ob = rb * S_BK + ((chunk ^ swz(rb)) << 3);
        ah[i] = *(const frag*)(&lds[cur][0][oa]);
        al[i] = *(const frag*)(&lds[cur][1][oa]);
        bh[i] = *(const frag*)(&lds[cur][2][ob]);
        bl[i] = *(const frag*)(&lds[cur][3][ob]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(al[i], bh[j], acc[i][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah[i], bl[j], acc[i][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah[i], bh[j], acc[i][j]);
    }
    // stage cur ^ 1 was last read before the previous barrier
    if (kt + 1 < KT) lstore(cur ^ 1);
    __syncthreads();
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = n0 + wn * 128 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t row = m0 + wm * 128 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g] * out_scale, acc[i][j][4 * g + 1] * out_scale,
                  acc[i][j][4 * g + 2] * out_scale, acc[i][j][4 * g + 3] * out_scale};
      }
  }
}

// Same tile and LDS layout as gemm_split_256, fed by gfx950's direct
// global-to-LDS loads (global_load_lds_dwordx4): lane l of a wave writes the
// 16 bytes at LDS slot base + 16 l, so each lane fetches the global chunk that
// the swizzled layout puts in its slot.  Wave w fills plane w (A hi, A lo,
// B hi, B lo) of the next stage while all waves compute on the current one;
// no staging registers and no LDS stores in the shader.  Columns of B past
// the end are clamped to the last valid column (their outputs are dropped).
// Both k16 fragment sets of a slab are read up front so that the LDS reads
// of the second step overlap the MFMAs of the first.
typedef __attribute__((address_space(3))) void lds_void;

template <typename H>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_256_dma(const uint16_t* __restrict__ A,
                                                                  const uint16_t* __restrict__ B,
                                                                  float* __restrict__ C,
                                                                  int64_t ldm, int64_t ncols,
                                                                  float out_scale, int order) {
  typedef typename SplitMfma<H>::frag frag;
  __shared__ __attribute__((aligned(1024))) uint16_t lds[2][4][S_PLANE];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * S_BM, n0 = (int64_t)tn * S_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  // this wave's plane: source rows and their lane offsets within one 16-row load
  const uint16_t* plane_src;
  int64_t row_limit;
  if (wave < 2) {
    plane_src = A + (wave == 1 ? 2 * ldm * ldm : 0) + m0 * ldm;
    row_limit = S_BM;
  } else {
    plane_src = B + (wave == 3 ? ldm * ncols : 0) + n0 * ldm;
    row_limit = ncols - n0;
  }
  // load q (0..15) covers rows 16 q .. 16 q + 15; lane l -> row 16 q + l / 4,
  // physical chunk l % 4, logical chunk (l % 4) ^ swz(row); swz(row) depends
  // only on row % 16, so the per-lane chunk offset is the same for every q
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ swz(lrow);
  auto issue = [&](int st, int64_t k0) {
    lds_void* dst = (lds_void*)&lds[st][wave][0];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      int64_t row = 16 * q + lrow;
      row = row < row_limit ? row : row_limit - 1;
      const uint16_t* g = plane_src + row * ldm + k0 + lchunk * 8;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)((char*)dst + q * 1024), 16, 0, 0);
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / S_BK);
  issue(0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    // stage cur ^ 1 was last read before the previous barrier
    if (kt + 1 < KT) issue(cur ^ 1, (int64_t)(kt + 1) * S_BK);
    frag ah[2][4], al[2][4], bh[2][4], bl[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int chunk = 2 * lh + s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra = wm * 128 + i * 32 + lr;
        const int rb = wn * 128 + i * 32 + lr;
        const int oa = ra * S_BK + ((chunk ^ swz(ra)) << 3);
        const int ob = rb * S_BK + ((chunk ^ swz(rb)) << 3);
        al[s][i] = *(const frag*)(&lds[cur][1][oa]);
        bh[s][i] = *(const frag*)(&lds[cur][2][ob]);
        ah[s][i] = *(const frag*)(&lds[cur][0][oa]);
        bl[s][i] = *(const frag*)(&lds[cur][3][ob]);
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(al[s][i], bh[s][j], acc[i][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah[s][i], bl[s][j], acc[i][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah[s][i], bh[s][j], acc[i][j]);
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next stage have landed
    __syncthreads();
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = n0 + wn * 128 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t row = m0 + wm * 128 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g] * out_scale, acc[i][j][4 * g + 1] * out_scale,
                  acc[i][j][4 * g + 2] * out_scale, acc[i][j][4 * g + 3] * out_scale};
      }
  }
}

// Deeper-prefetch variant: BK = 16 and a ring of four LDS stages (4 planes of
// 256 rows x 32 bytes = 32 KB per stage), so the direct-to-LDS loads of slab
// kt + 3 are in flight while slab kt is multiplied; the wait before each
// barrier only drains the loads of slab kt + 1 (vmcnt counts the loads issued
// after it).  Rows hold two 16-byte chunks; chunk c of row r sits at
// c ^ g(r), g(r) = ((r >> 2) ^ (r >> 3)) & 1, conflict-free for 32- and
// 64-bank LDS.
__device__ inline int swz2(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

constexpr int R_BK = 16, R_STAGES = 4;
constexpr int R_PLANE = S_BM * R_BK;  // elements of one plane of one stage

// Workgroup barrier without the memory fence of __syncthreads: the fence
// would drain every in-flight direct-to-LDS load.  LDS visibility is ensured
// by the explicit vmcnt waits before it; the empty asm statements stop the
// compiler from moving LDS accesses across the barrier.
__device__ inline void barrier_no_fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int N>
__device__ inline void wait_vm() {
  // s_waitcnt vmcnt(N), expcnt and lgkmcnt unconstrained (gfx9 encoding)
  __builtin_amdgcn_s_waitcnt(((N & 15) | ((N >> 4) << 14)) | (7 << 4) | (15 << 8));
}

template <typename H>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_256_ring(const uint16_t* __restrict__ A,
                                                                   const uint16_t* __restrict__ B,
                                                                   float* __restrict__ C,
                                                                   int64_t ldm, int64_t ncols,
                                                                   float out_scale, int order) {
  typedef typename SplitMfma<H>::frag frag;
  __shared__ __attribute__((aligned(1024))) uint16_t lds[R_STAGES][4][R_PLANE];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * S_BM, n0 = (int64_t)tn * S_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  const uint16_t* plane_src;
  int64_t row_limit;
  if (wave < 2) {
    plane_src = A + (wave == 1 ? 2 * ldm * ldm : 0) + m0 * ldm;
    row_limit = S_BM;
  } else {
    plane_src = B + (wave == 3 ? ldm * ncols : 0) + n0 * ldm;
    row_limit = ncols - n0;
  }
  // load q (0..7) covers rows 32 q .. 32 q + 31: lane l -> row 32 q + l / 2,
  // physical chunk l % 2, logical chunk (l % 2) ^ swz2(row); swz2 depends on
  // row % 16 only
  const int lrow = lane >> 1;
  const int lchunk = (lane & 1) ^ swz2(lrow);
  const uint16_t* lsrc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int64_t row = 32 * q + lrow;
    row = row < row_limit ? row : row_limit - 1;
    lsrc[q] = plane_src + row * ldm + lchunk * 8;
  }
  auto issue = [&](int st, int64_t k0) {
    char* dst = (char*)&lds[st][wave][0];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(lsrc[q] + k0), (lds_void*)(dst + q * 1024), 16,
                                       0, 0);
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / R_BK);  // >= 8
  issue(0, 0);
  issue(1, R_BK);
  issue(2, 2 * R_BK);
  wait_vm<16>();
  barrier_no_fence();
  const int oa_row[4] = {wm * 128 + lr, wm * 128 + 32 + lr, wm * 128 + 64 + lr, wm * 128 + 96 + lr};
  const int ob_row[4] = {wn * 128 + lr, wn * 128 + 32 + lr, wn * 128 + 64 + lr, wn * 128 + 96 + lr};
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 3;
    // stage (kt + 3) & 3 was last read in iteration kt - 1, before its barrier
    if (kt + 3 < KT) issue((kt + 3) & 3, (int64_t)(kt + 3) * R_BK);
    frag ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oa = oa_row[i] * R_BK + ((lh ^ swz2(oa_row[i])) << 3);
      const int ob = ob_row[i] * R_BK + ((lh ^ swz2(ob_row[i])) << 3);
      al[i] = *(const frag*)(&lds[cur][1][oa]);
      bh[i] = *(const frag*)(&lds[cur][2][ob]);
      ah[i] = *(const frag*)(&lds[cur][0][oa]);
      bl[i] = *(const frag*)(&lds[cur][3][ob]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(al[i], bh[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah[i], bl[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah[i], bh[j], acc[i][j]);
    // stage of slab kt + 1 must have landed: loads of later slabs may stay in flight
    const int later = (kt + 3 < KT ? kt + 3 : KT - 1) - (kt + 1);
    if (later >= 2)
      wait_vm<16>();
    else if (later == 1)
      wait_vm<8>();
    else
      wait_vm<0>();
    barrier_no_fence();
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = n0 + wn * 128 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t row = m0 + wm * 128 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g] * out_scale, acc[i][j][4 * g + 1] * out_scale,
                  acc[i][j][4 * g + 2] * out_scale, acc[i][j][4 * g + 3] * out_scale};
      }
  }
}

// Ping-pong schedule of the two-stage direct-to-LDS kernel.  Fragments of a
// slab's two k16 steps live in two register sets F0, F1.  Per slab kt:
//   read F1 (kt, step 1) | MFMAs on F0 | drain own loads of slab kt + 1 |
//   barrier | load slab kt + 2 into the stage just freed |
//   read F0 (kt + 1, step 0) | MFMAs on F1.
// The barrier sits between two MFMA groups, and the LDS reads after it
// overlap the second group, so neither the barrier nor the LDS latency
// leaves the matrix pipe idle for a whole fragment round trip.
template <typename H>
__device__ __attribute__((always_inline)) inline void split_pp_tile(uint16_t (*lds)[4][S_PLANE], const uint16_t* __restrict__ A,
                                     const uint16_t* __restrict__ B, float* __restrict__ C,
                                     int64_t ldm, int64_t ncols, int64_t m0, int64_t n0,
                                     float out_scale) {
  typedef typename SplitMfma<H>::frag frag;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  const uint16_t* plane_src;
  int64_t row_limit;
  if (wave < 2) {
    plane_src = A + (wave == 1 ? 2 * ldm * ldm : 0) + m0 * ldm;
    row_limit = S_BM;
  } else {
    plane_src = B + (wave == 3 ? ldm * ncols : 0) + n0 * ldm;
    row_limit = ncols - n0;
  }
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ swz(lrow);
  auto issue = [&](int st, int64_t k0) {
    char* dst = (char*)&lds[st][wave][0];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      int64_t row = 16 * q + lrow;
      row = row < row_limit ? row : row_limit - 1;
      const uint16_t* g = plane_src + row * ldm + k0 + lchunk * 8;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + q * 1024), 16, 0, 0);
    }
  };
  int oa[2][4], ob[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra = wm * 128 + i * 32 + lr, rb = wn * 128 + i * 32 + lr;
      oa[s][i] = ra * S_BK + (((2 * lh + s) ^ swz(ra)) << 3);
      ob[s][i] = rb * S_BK + (((2 * lh + s) ^ swz(rb)) << 3);
    }
  frag ah0[4], al0[4], bh0[4], bl0[4], ah1[4], al1[4], bh1[4], bl1[4];
  auto read0 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al0[i] = *(const frag*)(&lds[st][1][oa[0][i]]);
      bh0[i] = *(const frag*)(&lds[st][2][ob[0][i]]);
      ah0[i] = *(const frag*)(&lds[st][0][oa[0][i]]);
      bl0[i] = *(const frag*)(&lds[st][3][ob[0][i]]);
    }
  };
  auto read1 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al1[i] = *(const frag*)(&lds[st][1][oa[1][i]]);
      bh1[i] = *(const frag*)(&lds[st][2][ob[1][i]]);
      ah1[i] = *(const frag*)(&lds[st][0][oa[1][i]]);
      bl1[i] = *(const frag*)(&lds[st][3][ob[1][i]]);
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / S_BK);  // >= 4
  issue(0, 0);
  wait_vm<0>();
  barrier_no_fence();
  issue(1, S_BK);
  read0(0);
  // scheduling-group masks: MFMA, LDS read, global (direct-to-LDS) load
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    // phase A: MFMAs on F0 with the reads of F1 threaded between them
    read1(cur);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(al0[i], bh0[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah0[i], bl0[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah0[i], bh0[j], acc[i][j]);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 16, 0);
    __builtin_amdgcn_sched_barrier(0);
    // own loads of slab kt + 1 landed, own reads of stage cur complete
    __builtin_amdgcn_s_waitcnt(0);
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: MFMAs on F1 with the next loads and the reads of F0 threaded in.
    // In the last two slabs the loads repeat the final slab into the stage
    // just freed and the reads fetch unused fragments: both stay in bounds
    // and keep the loop free of branches around the MFMA stream.
    issue(cur, (int64_t)min(kt + 2, KT - 1) * S_BK);
    read0(cur ^ 1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(al1[i], bh1[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah1[i], bl1[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = SplitMfma<H>::mma(ah1[i], bh1[j], acc[i][j]);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 16, 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_s_waitcnt(0);  // the repeated tail loads land before the wave ends
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = n0 + wn * 128 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t row = m0 + wm * 128 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g] * out_scale, acc[i][j][4 * g + 1] * out_scale,
                  acc[i][j][4 * g + 2] * out_scale, acc[i][j][4 * g + 3] * out_scale};
      }
  }
}

template <typename H>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_256_pp(const uint16_t* __restrict__ A,
                                                                 const uint16_t* __restrict__ B,
                                                                 float* __restrict__ C,
                                                                 int64_t ldm, int64_t ncols,
                                                                 float out_scale, int order) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[2][4][S_PLANE];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
  split_pp_tile<H>(lds, A, B, C, ldm, ncols, (int64_t)tm * S_BM, (int64_t)tn * S_BN, out_scale);
}

// ---------------------------------------------------------------- FP32, 256 x 256

// FP32 twin of the split ping-pong kernel: the same 256 x 256 tile, four
// waves of 128 x 128, two direct-to-LDS stages and the same swizzled LDS
// rows (BK = 16 floats = 64 bytes per row), with v_mfma_f32_32x32x2f32.
// Lane half h supplies k = 8 h + s at step s (s = 0..7) of a slab, the same
// permutation on both operands; F0 holds steps 0-3 (chunk 2 h) and F1 steps
// 4-7 (chunk 2 h + 1).  Wave w loads half (w & 1) of operand w >> 1.
constexpr int F_BK = 16;
constexpr int F_PLANE = S_BM * F_BK;  // floats of one LDS operand plane

__global__ __launch_bounds__(kThreads, 1) void gemm_f32_pp(const float* __restrict__ A,
                                                           const float* __restrict__ B,
                                                           float* __restrict__ C, int64_t ldm,
                                                           int64_t ncols, int order) {
  __shared__ __attribute__((aligned(1024))) float lds[2][2][F_PLANE];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, order, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * S_BM, n0 = (int64_t)tn * S_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  const int op = wave >> 1, half = wave & 1;
  const float* src = op == 0 ? A + m0 * ldm : B + n0 * ldm;
  const int64_t row_limit = op == 0 ? S_BM : ncols - n0;
  const int lrow = lane >> 2;
  // lane l writes LDS slot 16 l of each 1 KB block: row 16 q + l / 4 of the
  // wave's half, slot l % 4, which holds global chunk (l % 4) ^ swz(row)
  auto issue = [&](int st, int64_t k0) {
    char* dst = (char*)&lds[st][op][0] + half * (128 * F_BK * 4);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = half * 128 + 16 * q + lrow;
      const int64_t row = r < row_limit ? r : row_limit - 1;
      const float* g = src + row * ldm + k0 + (((lane & 3) ^ swz(r)) << 2);
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + q * 1024), 16, 0, 0);
    }
  };
  int oa[2][4], ob[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra = wm * 128 + i * 32 + lr, rb = wn * 128 + i * 32 + lr;
      oa[s][i] = ra * F_BK + (((2 * lh + s) ^ swz(ra)) << 2);
      ob[s][i] = rb * F_BK + (((2 * lh + s) ^ swz(rb)) << 2);
    }
  f32x4 a0[4], b0[4], a1[4], b1[4];
  auto read0 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a0[i] = *(const f32x4*)(&lds[st][0][oa[0][i]]);
      b0[i] = *(const f32x4*)(&lds[st][1][ob[0][i]]);
    }
  };
  auto read1 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a1[i] = *(const f32x4*)(&lds[st][0][oa[1][i]]);
      b1[i] = *(const f32x4*)(&lds[st][1][ob[1][i]]);
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / F_BK);  // >= 8
  issue(0, 0);
  wait_vm<0>();
  barrier_no_fence();
  issue(1, F_BK);
  read0(0);
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    // phase A: steps 0-3 on F0 with the reads of F1 threaded between them
    read1(cur);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[i][s], b0[j][s], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 4, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 32, 0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);  // own loads of slab kt + 1 landed, reads of stage cur done
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: steps 4-7 on F1 with the loads of slab kt + 2 and the reads of
    // F0 of slab kt + 1 threaded in (the last two slabs repeat the final slab
    // into the freed stage, in bounds, so the loop has no branches)
    issue(cur, (int64_t)min(kt + 2, KT - 1) * F_BK);
    read0(cur ^ 1);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[i][s], b1[j][s], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 4, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 16, 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_s_waitcnt(0);  // the repeated tail loads land before the wave ends
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = n0 + wn * 128 + j * 32 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t row = m0 + wm * 128 + i * 32 + 8 * g + 4 * lh;
        *(f32x4*)(C + col * ldc + row) =
            f32x4{acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]};
      }
  }
}

// ---------------------------------------------------------------- grouped

// Persistent grouped launch over many networks: one workgroup per CU walks a
// work list of (network, tile) items with stride gridDim.x; the list is
// ordered so that the items an XCD processes at the same time are
// neighbouring tiles of one network.

template <typename H>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_grouped(const GroupNet* __restrict__ nets,
                                                                  const int4* __restrict__ items,
                                                                  int n_items) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[2][4][S_PLANE];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];  // (net, tile_m, tile_n, unused); net < 0: idle slot
    if (w.x < 0) continue;
    const GroupNet g = nets[w.x];
    split_pp_tile<H>(lds, g.A, g.B, g.C, g.ldm, g.ncols, (int64_t)w.y * S_BM, (int64_t)w.z * S_BN,
                     g.out_scale);
    __syncthreads();  // the next item reuses the LDS stages
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

// Split-GEMM variant: 3 = two-stage direct-to-LDS ping-pong (default),
// 2 = four-stage direct-to-LDS ring, 1 = two-stage direct-to-LDS,
// 0 = register staging.
static int split_variant() {
  static int v = [] {
    const char* e = getenv("MPGBS_SPLIT_VARIANT");
    return e ? atoi(e) : 3;
  }();
  return v;
}

// FP32 GEMM variant: 1 = 256 x 256 direct-to-LDS ping-pong (default),
// 0 = 128 x 128 register staging.
static int f32_variant() {
  static int v = [] {
    const char* e = getenv("MPGBS_F32_VARIANT");
    return e ? atoi(e) : 1;
  }();
  return v;
}

static int grid_tiles(int64_t ldm, int64_t ncols, int bm, int bn) {
  const int tiles_m = (int)(2 * ldm / bm), tiles_n = (int)((ncols + bn - 1) / bn);
  if (tile_order() == 1) return mall_grid_blocks(tiles_m, tiles_n);
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  const int64_t per = (tiles + kXcds - 1) / kXcds;
  return (int)(per * kXcds);
}

// Power-of-two prescale of T for the FP16 split operand: |T_ij| ~ M^-1/2 for
// a spread-out network, so 2^floor(log2(M)/2) brings typical entries near 1.
static int fp16_scale_exp(int32_t M) {
  int e = 0;
  while ((1LL << (2 * (e + 1))) <= (long long)M) ++e;
  return e;
}

// ---- used by plans (plan.hip)

int split_scale_exp(int32_t M, mp_precision prec) {
  return prec == MP_SPLIT_FP16 ? fp16_scale_exp(M) : 0;
}

mp_status pack_launch(int32_t M, const double* T, mp_precision prec, void* packed,
                      hipStream_t stream) {
  const int64_t ldm = ld_modes(M);
  const int blocks = (int)((2 * ldm * ldm + 255) / 256);
  switch (prec) {
    case MP_FP64:
      hipLaunchKernelGGL(pack_transmission<MP_FP64>, dim3(blocks), dim3(256), 0, stream, T, M, ldm,
                         packed, 0);
      break;
    case MP_FP32:
      hipLaunchKernelGGL(pack_transmission<MP_FP32>, dim3(blocks), dim3(256), 0, stream, T, M, ldm,
                         packed, 0);
      break;
    case MP_SPLIT_BF16:
      hipLaunchKernelGGL(pack_transmission<MP_SPLIT_BF16>, dim3(blocks), dim3(256), 0, stream, T,
                         M, ldm, packed, 0);
      break;
    case MP_SPLIT_FP16:
      hipLaunchKernelGGL(pack_transmission<MP_SPLIT_FP16>, dim3(blocks), dim3(256), 0, stream, T,
                         M, ldm, packed, fp16_scale_exp(M));
      break;
  }
  MP_HIP_LAUNCH_CHECK("transmission pack launch");
  return MP_OK;
}

// GEMM on an already packed operand (one network).
template <typename H>
static void split_gemm(int variant, int grid, hipStream_t stream, const void* packed,
                       const void* ab, void* C, int64_t ldm, int64_t ncols, float scale) {
  const uint16_t* A = (const uint16_t*)packed;
  const uint16_t* B = (const uint16_t*)ab;
  float* Cf = (float*)C;
  if (variant == 3)
    hipLaunchKernelGGL(gemm_split_256_pp<H>, dim3(grid), dim3(kThreads), 0, stream, A, B, Cf, ldm,
                       ncols, scale, tile_order());
  else if (variant == 2)
    hipLaunchKernelGGL(gemm_split_256_ring<H>, dim3(grid), dim3(kThreads), 0, stream, A, B, Cf,
                       ldm, ncols, scale, tile_order());
  else if (variant == 1)
    hipLaunchKernelGGL(gemm_split_256_dma<H>, dim3(grid), dim3(kThreads), 0, stream, A, B, Cf,
                       ldm, ncols, scale, tile_order());
  else
    hipLaunchKernelGGL(gemm_split_256<H>, dim3(grid), dim3(kThreads), 0, stream, A, B, Cf, ldm,
                       ncols, scale, tile_order());
}

mp_status gemm_packed_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                             const void* ab, void* C, hipStream_t stream) {
  const int64_t ldm = ld_modes(M), ncols = 2 * E;
  switch (prec) {
    case MP_FP64:
      hipLaunchKernelGGL(gemm_f64, dim3(grid_tiles(ldm, ncols, BM, BN)), dim3(kThreads), 0, stream,
                         (const double*)packed, (const double*)ab, (double*)C, ldm, ncols, tile_order());
      break;
    case MP_FP32:
      if (f32_variant() == 1)
        hipLaunchKernelGGL(gemm_f32_pp, dim3(grid_tiles(ldm, ncols, S_BM, S_BN)), dim3(kThreads), 0,
                           stream, (const float*)packed, (const float*)ab, (float*)C, ldm, ncols,
                           tile_order());
      else
        hipLaunchKernelGGL(gemm_f32, dim3(grid_tiles(ldm, ncols, BM, BN)), dim3(kThreads), 0,
                           stream, (const float*)packed, (const float*)ab, (float*)C, ldm, ncols,
                           tile_order());
      break;
    case MP_SPLIT_BF16:
      split_gemm<__bf16>(split_variant(), grid_tiles(ldm, ncols, S_BM, S_BN), stream, packed, ab,
                         C, ldm, ncols, 1.0f);
      break;
    case MP_SPLIT_FP16:
      split_gemm<_Float16>(split_variant(), grid_tiles(ldm, ncols, S_BM, S_BN), stream, packed, ab,
                           C, ldm, ncols, ldexpf(1.0f, -fp16_scale_exp(M)));
      break;
  }
  MP_HIP_LAUNCH_CHECK("mp_propagate gemm launch");
  return MP_OK;
}

mp_status grouped_launch(const GroupNet* d_nets, const int4* d_items, int n_items, int grid,
                         mp_precision prec, hipStream_t stream) {
  if (prec == MP_SPLIT_BF16)
    hipLaunchKernelGGL(gemm_split_grouped<__bf16>, dim3(grid), dim3(kThreads), 0, stream, d_nets,
                       d_items, n_items);
  else if (prec == MP_SPLIT_FP16)
    hipLaunchKernelGGL(gemm_split_grouped<_Float16>, dim3(grid), dim3(kThreads), 0, stream, d_nets,
                       d_items, n_items);
  else {
    set_error("grouped GEMM: split precisions only");
    return MP_ERR_UNSUPPORTED;
  }
  MP_HIP_LAUNCH_CHECK("plan grouped gemm launch");
  return MP_OK;
}

mp_status propagate_launch(int32_t M, int64_t E, const double* T, mp_precision prec,
                           const void* ab, void* C, void* ws, hipStream_t stream) {
  const mp_status st = pack_launch(M, T, prec, ws, stream);
  if (st != MP_OK) return st;
  return gemm_packed_launch(M, E, ws, prec, ab, C, stream);
}

}  // namespace mp
