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
// Kernels: FP64 (v_mfma_f64_16x16x4, 128 x 256 tiles), FP32
// (v_mfma_f32_32x32x2, 256 x 256 tiles) and split BF16/FP16 (three
// v_mfma_f32_32x32x16 products hi*hi + hi*lo + lo*hi with FP32 accumulation,
// 256 x 256 tiles).  The 256 x 256 kernels feed LDS with direct global-to-LDS
// loads in a two-stage ping-pong schedule, and the tile order keeps the
// workgroups of one XCD on neighbouring tiles that share rows of A and
// columns of B in its L2.
//
// Split operands are stored interleaved: each row of A (and each column of
// B) alternates a block of 32 hi values with the block of the 32 matching lo
// values, so one 32-deep k-slab of a row is one full 128-byte line.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"

namespace mp {

typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

constexpr int kThreads = 256;
constexpr int kXcds = 8;     // MI355X: 8 XCDs, workgroups dispatched round-robin

// ---------------------------------------------------------------- packing

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// A[i][j] (row-major, 2 ldm x ldm) from T (row-major complex M x M).  Split
// precisions store row i as 2 ldm values: for k-block b = j / 32 the 32 hi
// values at 64 b .. 64 b + 31 and the 32 lo values right after them.
__host__ __device__ inline int64_t split_offset(int64_t j) { return 64 * (j >> 5) + (j & 31); }

// MP_SPLIT1_FP16 packs the single FP16 A in row pairs: for rows 2p, 2p + 1
// and k-block b = j / 32, the 32 values of row 2p and then the 32 of row
// 2p + 1 (one 128-byte line per pair and block), so a 32-deep slab of two
// rows is one whole line.  Otherwise row-major.
constexpr bool kSplit1ALines = true;
__host__ __device__ inline int64_t split1_a_offset(int64_t row, int64_t j, int64_t ldm) {
  return kSplit1ALines ? (row >> 1) * 2 * ldm + split_offset(j) + (row & 1) * 32 : row * ldm + j;
}

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
    const int64_t at = row * 2 * ldm + split_offset(j);
    ((uint16_t*)A)[at] = hi;
    ((uint16_t*)A)[at + 32] = lo;
  } else if constexpr (PREC == MP_SPLIT1_FP16) {
    // one FP16 value per entry, prescaled like MP_SPLIT_FP16
    ((_Float16*)A)[split1_a_offset(row, j, ldm)] = (_Float16)ldexp(v, scale_exp);
  } else if constexpr (PREC == MP_SPLIT1T_F8) {
    // the MP_SPLIT1_FP16 packing, then (from byte 4 ldm^2 on) the remainder
    // x - hi in e4m3, scaled by 2^e4m3_lo_scale_exp, in row pairs
    const double x = ldexp(v, scale_exp);
    const _Float16 hi = (_Float16)x;
    ((_Float16*)A)[split1_a_offset(row, j, ldm)] = hi;
    const float lo = (float)ldexp(x - (double)hi, e4m3_lo_scale_exp(scale_exp));
    ((uint8_t*)A)[4 * ldm * ldm + pair8_offset(row, j, ldm)] = e4m3_rne(lo);
  } else {
    // FP16: A is packed as T * 2^scale_exp so that both halves stay normal
    const double x = ldexp(v, scale_exp);
    _Float16 hi = (_Float16)x;
    _Float16 lo = (_Float16)(x - (double)hi);
    const int64_t at = row * 2 * ldm + split_offset(j);
    ((_Float16*)A)[at] = hi;
    ((_Float16*)A)[at + 32] = lo;
  }
}

// ---------------------------------------------------------------- tile order

// Tile order.  Blocks are dispatched to the XCDs round-robin, so block b
// runs on XCD b % 8 and, with one workgroup per CU, the 32 blocks
// b / 8 = 32 s .. 32 s + 31 of every XCD run together in "step" s.  In each
// step all eight XCDs work on the same group of 8 row tiles, each XCD on its
// own 4 column tiles, and consecutive steps move along the columns.  The A
// rows of a group are then shared by every XCD through the infinity cache
// (MALL) and fetched from HBM about once per group, instead of once per XCD
// and column block (measured faster than XCD-local groups of 8 row tiles).
constexpr int kStepRows = 8, kStepColsPerXcd = 4;

// SR row tiles by SC column tiles per XCD and step (SR SC = 32 workgroups).
template <int SR = kStepRows, int SC = kStepColsPerXcd>
__device__ inline bool tile_of_block(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int b = blockIdx.x, x = b % kXcds, q = b / kXcds;
  const int per_xcd = SR * SC;   // 32 blocks of one XCD per step
  const int s = q / per_xcd, j = q % per_xcd;
  const int cols_per_step = kXcds * SC;  // column tiles per step
  const int n_cg = (tiles_n + cols_per_step - 1) / cols_per_step;
  const int rg = s / n_cg, cg = s % n_cg;
  tm = rg * SR + j % SR;
  tn = cg * cols_per_step + x * SC + j / SR;
  return tm < tiles_m && tn < tiles_n;
}

template <int SR = kStepRows, int SC = kStepColsPerXcd>
__host__ __device__ inline int mall_grid_blocks(int tiles_m, int tiles_n) {
  const int n_cg = (tiles_n + kXcds * SC - 1) / (kXcds * SC);
  const int n_rg = (tiles_m + SR - 1) / SR;
  return n_rg * n_cg * kXcds * SR * SC;
}

// ---------------------------------------------------------------- split, 256 x 256

// v_mfma_f32_32x32x16_bf16 (and _f16): lane l holds A[l%32][8 (l/32) + e],
// e = 0..7, and the same for B; output register r is row 8 (r/4) + 4 (l/32)
// + r%4, column l%32.  Within one BK = 32 slab lane half h supplies
// k = 16 h + 8 s + e at step s (s = 0, 1), the same permutation on both
// operands.  Each operand is x = hi + lo; the product keeps
// hi*hi + hi*lo + lo*hi.
//
// Tile 256 x 256 per 256-thread workgroup: four waves of 128 x 128 (4 x 4
// MFMA tiles, 256 accumulator registers per lane), two LDS stages of four
// 256 x 32 planes (A hi/lo, B hi/lo).  Rows of a plane are 64 bytes without
// padding; 16-byte chunk c of row r is stored at chunk c ^ f(r),
// f(r) = ((r >> 1) & 3) ^ ((r >> 3) & 1), which keeps the 16-byte fragment
// reads (32 consecutive rows, one chunk) free of bank conflicts.  Within a
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
// 128-byte LDS rows (8 chunks of 16 bytes): chunk c of row r at c ^ swz8(r);
// the 16 consecutive rows one 16-byte read touches per LDS cycle land in
// distinct banks (even and odd rows in different bank halves).
__device__ inline int swz8(int r) { return (r >> 1) & 7; }

constexpr int S_BM = 256, S_BN = 256, S_BK = 32;
constexpr int S_PLANE = S_BM * S_BK;  // elements of one LDS plane
// LDS of a split tile: two stages of four planes, then a 256-byte sink for the
// L2 prefetch loads (nothing reads it).  The sink sits in the same array as the
// stages so that the compiler's wait analysis for direct-to-LDS loads keeps the
// fragment reads free of extra vmcnt waits.
constexpr int kSplitLdsElems = 2 * 4 * S_PLANE + 128;
// The split kernels touch the lines of slab kt + 2 + kPrefetchSlabs while
// loading slab kt + 2 (measured at M = 8000 on one box: distance 1 takes 3.3 %
// off the occupation-fused GEMM, 2 takes 2.8 %, 3 or more less).  When the
// operand rows are a multiple of 32 KB apart (ldm a multiple of 8192) the
// prefetch slowed the GEMM instead (M = 8192: +4.7 %, 16384: +3.9 %; 12288 and
// every other size measured from 2048 to 10240 gained 1-5 %; a prefetch reduced
// to one line already in flight still cost 2 %), so those sizes run the loop
// without it (the PF = false instances).
constexpr int kPrefetchSlabs = 1;
constexpr int64_t kPrefetchAliasModes = 8192;
constexpr int kSplitPf = 2;  // prefetch loads per wave and slab: 2 = A and B lines, 1 = B only

__host__ __device__ inline bool split_prefetch_for(int64_t ldm) { return ldm % kPrefetchAliasModes != 0; }

// Operands reach LDS through gfx950's direct global-to-LDS loads
// (global_load_lds_dwordx4): lane l of a wave writes the 16 bytes at LDS slot
// base + 16 l, so each lane fetches the global chunk that the swizzled layout
// puts in its slot; no staging registers and no LDS stores in the shader.
typedef __attribute__((address_space(3))) void lds_void;

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

// s_waitcnt lgkmcnt(0), vmcnt and expcnt unconstrained
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }

// ---------------------------------------------------------------- FP64, 128 x 256

// FP64 tile of 128 rows x 256 columns: four waves of 64 x 128 (4 x 8 blocks
// of v_mfma_f64_16x16x4f64, 128 accumulators per lane, one wave per SIMD),
// 16-deep slabs loaded direct-to-LDS into two stages of 384 rows (A rows, then
// B rows) of 16 doubles.  16-byte chunk c of stage row r sits at slot
// c ^ (r & 7), so the 16-byte fragment reads of eight consecutive rows touch
// every bank once.  The MFMA takes A[l % 16][l / 16] and B[l / 16][l % 16]
// from lane l; within a slab lane group h = l / 16 supplies k = 4 h + s at
// MFMA step s (s = 0..3, the same permutation on both operands): the doubles
// 4 h .. 4 h + 3 of its row, two 16-byte reads per block.  Output register r
// of lane l is row l / 16 + 4 r, column l % 16 of a block.
constexpr int D_BM = 128, D_BN = 256, D_BK = 16;
constexpr int D_ROWS = D_BM + D_BN;  // stage rows
// stages of 48 KB; three (loads issued two slabs ahead) measured 1.6 % slower
constexpr int D_NST = 2;

typedef __attribute__((ext_vector_type(2))) double f64x2;

__global__ __launch_bounds__(kThreads, 1) void gemm_f64_pp(const double* __restrict__ A,
                                                           const double* __restrict__ B,
                                                           double* __restrict__ C, int64_t ldm,
                                                           int64_t ncols) {
  __shared__ __attribute__((aligned(1024))) double lds[D_NST][D_ROWS * D_BK];
  const int tiles_m = (int)(2 * ldm / D_BM), tiles_n = (int)((ncols + D_BN - 1) / D_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * D_BM, n0 = (int64_t)tn * D_BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lh = lane >> 4;

  // loader: instruction q of wave w fills stage rows 96 w + 8 q .. + 7 (1 KB):
  // lane l writes slot l % 8 of row 96 w + 8 q + l / 8, i.e. its global chunk
  // (l % 8) ^ (row & 7); B columns past the chunk repeat the last one
  const double* src[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int r = 96 * wave + 8 * q + (lane >> 3);
    const int c = (lane & 7) ^ (r & 7);
    if (r < D_BM) {
      src[q] = A + (m0 + r) * ldm + 2 * c;
    } else {
      int64_t col = n0 + (r - D_BM);
      col = col < ncols ? col : ncols - 1;
      src[q] = B + col * ldm + 2 * c;
    }
  }
  auto issue = [&](int st, int64_t k0) {
    char* dst = (char*)&lds[st][0] + 96 * wave * D_BK * 8;
#pragma unroll
    for (int q = 0; q < 12; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src[q] + k0), (lds_void*)(dst + q * 1024), 16,
                                       0, 0);
  };
  // fragment offsets (doubles) of chunk 2 lh + half for the wave's row blocks
  int oa[2][4], ob[2][8];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + lr;
      oa[hf][i] = r * D_BK + 2 * ((2 * lh + hf) ^ (r & 7));
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int r = D_BM + wn * 128 + j * 16 + lr;
      ob[hf][j] = r * D_BK + 2 * ((2 * lh + hf) ^ (r & 7));
    }
  }

  f64x4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f64x4{0, 0, 0, 0};

  // fragments of one half slab: k steps 2 hf, 2 hf + 1 of every row block
  auto frag = [&](int st, int hf, f64x2(&a)[4], f64x2(&b)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *(const f64x2*)&lds[st][oa[hf][i]];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = *(const f64x2*)&lds[st][ob[hf][j]];
  };
  auto mma = [&](const f64x2(&a)[4], const f64x2(&b)[8]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
  };

  // Pipeline: slab kt + 2 is loaded while slab kt is multiplied; the second
  // half of slab kt is read while its first half is multiplied, and the first
  // half of slab kt + 1 while its second half is.  The one barrier per slab
  // sits between the halves: past it every wave has read all of stage
  // kt & 1 (so it may be refilled) and every wave's loads of slab kt + 1 have
  // landed (so it may be read).
  const int KT = (int)(ldm / D_BK);
  f64x2 a0[4], b0[8], a1[4], b1[8];
  // prologue: slabs 0 .. D_NST - 1 in flight (KT >= 8 since ldm is a multiple
  // of 128), then wait for slab 0: loads complete in order, so the 12 loads
  // of each younger slab may stay outstanding
#pragma unroll
  for (int st = 0; st < D_NST; ++st) issue(st, (int64_t)st * D_BK);
  wait_vm<12 * (D_NST - 1)>();
  barrier_no_fence();
  frag(0, 0, a0, b0);
  // One basic block per slab, the same for every slab: a branch in the body
  // or a peeled last slab made the compiler keep the accumulators in
  // different registers in the two halves and copy them every slab.  Past
  // the end the loads re-fetch the last slab into the stage just freed and
  // the last first-half read fetches a stage whose loads have been waited
  // for; neither result is used.
  // scheduling-group masks: MFMA, LDS read, global (direct-to-LDS) load
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt % D_NST, nxt = (kt + 1) % D_NST;
    frag(cur, 1, a1, b1);
    mma(a0, b0);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 52, 0);
    // keep the products on their side of the barrier (the scheduler would
    // otherwise sink them below it and expose the read latency)
    __builtin_amdgcn_sched_barrier(0);
    wait_lgkm0();  // this wave's reads of stage cur are done
    // this wave's loads of slab kt + 1 have landed; every iteration issues
    // 12 loads, so those of the D_NST - 2 younger ones may stay in flight
    wait_vm<12 * (D_NST - 2)>();
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // the second half's products start right after the barrier, with the
    // loads and the next slab's first-half reads threaded between them
    issue(cur, (int64_t)min(kt + D_NST, KT - 1) * D_BK);
    frag(nxt, 0, a0, b0);
    mma(a1, b1);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 40, 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  wait_vm<0>();  // no direct-to-LDS write may outlive the workgroup
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t col = n0 + wn * 128 + j * 16 + lr;
    if (col >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double* p = C + col * ldc + m0 + wm * 64 + i * 16 + lh;
      p[0] = acc[i][j][0];
      p[4] = acc[i][j][1];
      p[8] = acc[i][j][2];
      p[12] = acc[i][j][3];
    }
  }
}

// Occupation-fused epilogue (see FusedOut).  The tile covers modes
// [m0, m0 + 128) and samples [n0, n0 + 128): its waves hold, element for
// element in the same register positions, a = Re alpha' (wm 0, wn 0),
// c = Re beta' (wm 0, wn 1), b = Im alpha' (wm 1, wn 0) and e = -Im beta'
// (wm 1, wn 1).  The beta waves publish their blocks through LDS; the alpha
// waves form their halves of n = alpha' beta' = (a c + b e) + i (b c - a e),
// sum them over the modes of every bin run in the block (lane halves hold
// interleaved rows and are combined by a shuffle) and store per-sample
// partials.  LDS layout: [wm][(i 4 + j) 4 + g][lane][4] floats, conflict-free
// 16-byte accesses.
template <int NJ = 4>
__device__ __attribute__((always_inline)) inline void fused_epilogue(
    f32x16 (&acc)[4][NJ], float* __restrict__ lds_f, const FusedOut& fo, int64_t m0, int64_t n0,
    int wm, int wn, int lane, float out_scale) {
  const int lr = lane & 31, lh = lane >> 5;
  __syncthreads();  // every wave is done reading the operand stages
  if (wn == 1) {
    float* dst = lds_f + wm * 16384;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g)
          *(f32x4*)(dst + ((((i * NJ + j) * 4 + g) * 64) + lane) * 4) =
              f32x4{acc[i][j][4 * g] * out_scale, acc[i][j][4 * g + 1] * out_scale,
                    acc[i][j][4 * g + 2] * out_scale, acc[i][j][4 * g + 3] * out_scale};
  }
  __syncthreads();
  if (wn != 0) return;
  const float* cre = lds_f;          // Re beta'
  const float* cim = lds_f + 16384;  // -Im beta'
  const int blk = (int)m0;
  // sums over the block's modes [lo, hi) of one run into its slot
  auto emit = [&](int q, int lo, int hi, bool whole) {
    const int64_t slot = fo.slot_off[q] + (blk >> 7) - (fo.run_lo[q] >> 7);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      float pr = 0.0f, pi = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int off = ((((i * NJ + j) * 4 + g) * 64) + lane) * 4;
          const f32x4 c = *(const f32x4*)(cre + off);
          const f32x4 e = *(const f32x4*)(cim + off);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int mode = i * 32 + 8 * g + 4 * lh + rr;
            const float x = (whole || (mode >= lo && mode < hi)) ? acc[i][j][4 * g + rr] * out_scale
                                                                 : 0.0f;
            if (wm == 0) {
              pr = fmaf(x, c[rr], pr);
              pi = fmaf(-x, e[rr], pi);
            } else {
              pr = fmaf(x, e[rr], pr);
              pi = fmaf(x, c[rr], pi);
            }
          }
        }
      pr += __shfl_xor(pr, 32);
      pi += __shfl_xor(pi, 32);
      const int64_t smp = n0 + j * 32 + lr;
      if (lh == 0 && smp < fo.E) {
        typedef __attribute__((ext_vector_type(2))) float f32x2;
        *(f32x2*)(fo.part + (slot * fo.E + smp) * 4 + 2 * wm) = f32x2{pr, pi};
      }
    }
  };
  // A block inside one run (every block of a one-bin partition but the
  // padded last) needs no mode masks; with them the compiler copied all 256
  // accumulators out of the AGPRs at once for the run loop and spilled some.
  int whole = -1;
  for (int q = 0; q < fo.n_runs; ++q)
    if (fo.run_lo[q] <= blk && fo.run_hi[q] >= blk + 128) whole = q;
  if (whole >= 0) {
    emit(whole, 0, 128, true);
    return;
  }
  for (int q = 0; q < fo.n_runs; ++q) {
    const int lo = (fo.run_lo[q] > blk ? fo.run_lo[q] : blk) - blk;
    const int hi = (fo.run_hi[q] < blk + 128 ? fo.run_hi[q] : blk + 128) - blk;
    if (lo >= hi) continue;
    emit(q, lo, hi, false);
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
// lds points at kSplitLdsElems elements: the two stages and the prefetch sink.
// PF: touch the lines of the slab after the one being loaded (see
// kPrefetchSlabs); without it the loop waits for all its loads at each slab.
// FUSED: the tile's rows are the Re rows of modes [m0, m0 + 128) followed by
// their Im rows, its columns the alpha columns of samples [n0, n0 + 128)
// followed by their beta columns, and the epilogue is fused_epilogue instead
// of the store of C.
// NJ: 32-column blocks per wave.  4: the 256 x 256 tile; 2: a 256 x 128 tile
// (fused: 128 modes x 64 samples) whose B planes use their first 128 rows,
// for batched plans (a tile-shape candidate of the plan's autotuner).  Every
// output element goes through the same MFMA sequence in either shape, so the
// results are the same bits.
template <typename H, bool FUSED, bool PF, int NJ = 4>
__device__ __attribute__((always_inline)) inline void split_pp_tile(uint16_t (*lds)[4][S_PLANE], const uint16_t* __restrict__ A,
                                     const uint16_t* __restrict__ B, float* __restrict__ C,
                                     int64_t ldm, int64_t ncols, int64_t m0, int64_t n0,
                                     float out_scale, const FusedOut* fo, int tid = -1) {
  typedef typename SplitMfma<H>::frag frag;
  // tid < 0: the kernel's own thread index; else an index made opaque by the
  // caller (the grouped kernel), whose wave number is made uniform here
  const int wave = tid < 0 ? (int)(threadIdx.x >> 6) : __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid < 0 ? (int)(threadIdx.x & 63) : tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  const uint16_t* plane_src;
  int64_t row_limit, hi_off;
  // wave w fills plane w: hi or lo (+32) half of the interleaved rows of A
  // (w < 2) or of the columns of B; both have 2 ldm values per row.  Fused
  // tiles take their second 128 rows from the Im rows (A: + ldm) or the beta
  // columns (B: + E), and clamp sample offsets past the end of the chunk.
  if (wave < 2) {
    plane_src = A + (wave == 1 ? 32 : 0) + m0 * 2 * ldm;
    row_limit = FUSED ? 128 : S_BM;
    hi_off = ldm;
  } else {
    plane_src = B + (wave == 3 ? 32 : 0) + n0 * 2 * ldm;
    row_limit = FUSED ? ncols / 2 - n0 : ncols - n0;
    hi_off = ncols / 2;
  }
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ swz(lrow);
  // NQ loads of 16 rows fill a plane: 16 (256 rows) for A and for the full
  // tile's B, 4 NJ for the B of a narrower tile (its second half the beta
  // columns when fused)
  auto issue_rows = [&](auto NQc, int st, int64_t k0) {
    constexpr int NQ = decltype(NQc)::value;
    char* dst = (char*)&lds[st][wave][0];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int64_t row;
      if constexpr (FUSED) {
        row = 16 * (q % (NQ / 2)) + lrow;
        row = (row < row_limit ? row : row_limit - 1) + (q >= NQ / 2 ? hi_off : 0);
      } else {
        row = 16 * q + lrow;
        row = row < row_limit ? row : row_limit - 1;
      }
      const uint16_t* g = plane_src + row * 2 * ldm + 2 * k0 + lchunk * 8;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + q * 1024), 16, 0, 0);
    }
  };
  auto issue = [&](int st, int64_t k0) {
    if (NJ == 4 || wave < 2)
      issue_rows(std::integral_constant<int, 16>{}, st, k0);
    else
      issue_rows(std::integral_constant<int, 4 * NJ>{}, st, k0);
  };
  // L2 prefetch of slab k0: one 4-byte direct-to-LDS load per 128-byte line
  // (one row of the interleaved operand) into the sink after the stages.  The
  // two waves of an operand split its 256 rows; the rows are clamped as in
  // issue().  A line that misses the caches then costs its latency here, with
  // two loads in flight per wave, and the sixteen loads that fill the stage
  // later hit L2.
  // kSplitPf = 1: only the lines of B, 64 columns per wave
  constexpr int NPF = kSplitPf;
  const uint16_t* pf_src = (wave < 2 && NPF == 2) ? A + m0 * 2 * ldm : B + n0 * 2 * ldm;
  const int64_t pf_limit = NPF == 2 ? row_limit : (FUSED ? ncols / 2 - n0 : ncols - n0);
  const int64_t pf_hi = NPF == 2 ? hi_off : ncols / 2;
  static_assert(NJ == 4 || NPF == 2, "narrower tiles prefetch both operands");
  // rows of the prefetched operand: the B of a narrower tile has 64 NJ rows,
  // 32 NJ per wave (NJ = 2: one per lane, touched twice)
  const bool pf_full = NJ == 4 || wave < 2;
  const int pf_half = pf_full ? 128 : 32 * NJ;
  auto prefetch = [&](int64_t k0) {
    if constexpr (!PF) return;
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      int64_t row = NPF == 2 ? (pf_full ? 128 * (wave & 1) + 64 * q + lane : 32 * NJ * (wave & 1) + lane)
                             : 64 * wave + lane;
      if constexpr (FUSED) {
        const int64_t r = row & (pf_half - 1);
        row = (r < pf_limit ? r : pf_limit - 1) + (row >= pf_half ? pf_hi : 0);
      } else {
        row = row < pf_limit ? row : pf_limit - 1;
      }
      const uint16_t* g = pf_src + row * 2 * ldm + 2 * k0;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)&lds[2][0][0], 4, 0, 0);
    }
  };
  int oa[2][4], ob[2][NJ];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra = wm * 128 + i * 32 + lr;
      oa[s][i] = ra * S_BK + (((2 * lh + s) ^ swz(ra)) << 3);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int rb = wn * 32 * NJ + j * 32 + lr;
      ob[s][j] = rb * S_BK + (((2 * lh + s) ^ swz(rb)) << 3);
    }
  }
  frag ah0[4], al0[4], bh0[NJ], bl0[NJ], ah1[4], al1[4], bh1[NJ], bl1[NJ];
  auto read0 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al0[i] = *(const frag*)(&lds[st][1][oa[0][i]]);
      if (i < NJ) bh0[i] = *(const frag*)(&lds[st][2][ob[0][i]]);
      ah0[i] = *(const frag*)(&lds[st][0][oa[0][i]]);
      if (i < NJ) bl0[i] = *(const frag*)(&lds[st][3][ob[0][i]]);
    }
  };
  auto read1 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al1[i] = *(const frag*)(&lds[st][1][oa[1][i]]);
      if (i < NJ) bh1[i] = *(const frag*)(&lds[st][2][ob[1][i]]);
      ah1[i] = *(const frag*)(&lds[st][0][oa[1][i]]);
      if (i < NJ) bl1[i] = *(const frag*)(&lds[st][3][ob[1][i]]);
    }
  };

  f32x16 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / S_BK);  // >= 4
  // Loads return in issue order, so with PF every slab's stage loads are
  // followed by exactly two prefetch loads and the loop waits for all but
  // those two.
  for (int p = 2; p <= kPrefetchSlabs; ++p) prefetch((int64_t)min(p, KT - 1) * S_BK);
  issue(0, 0);
  wait_vm<0>();
  barrier_no_fence();
  issue(1, S_BK);
  prefetch((int64_t)min(1 + kPrefetchSlabs, KT - 1) * S_BK);
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
      for (int j = 0; j < NJ; ++j) acc[i][j] = SplitMfma<H>::mma(al0[i], bh0[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = SplitMfma<H>::mma(ah0[i], bl0[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = SplitMfma<H>::mma(ah0[i], bh0[j], acc[i][j]);
    // per phase: 12 NJ MFMAs, 8 + 2 NJ fragment reads
    constexpr int kReads = 8 + 2 * NJ, kMfma = 12 * NJ, kMpr = NJ == 4 ? 2 : 1;
#pragma unroll
    for (int q = 0; q < kReads; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, kMpr, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, kMfma - kMpr * kReads, 0);
    __builtin_amdgcn_sched_barrier(0);
    // own loads of slab kt + 1 landed (with PF only the two prefetch loads
    // issued after them may be in flight), own reads of stage cur complete
    if constexpr (PF)
      __builtin_amdgcn_s_waitcnt(NPF | (7 << 4));  // vmcnt(NPF), lgkmcnt(0)
    else
      __builtin_amdgcn_s_waitcnt(0);
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: MFMAs on F1 with the next loads and the reads of F0 threaded in.
    // In the last two slabs the loads repeat the final slab into the stage
    // just freed and the reads fetch unused fragments: both stay in bounds
    // and keep the loop free of branches around the MFMA stream.
    issue(cur, (int64_t)min(kt + 2, KT - 1) * S_BK);
    prefetch((int64_t)min(kt + 2 + kPrefetchSlabs, KT - 1) * S_BK);
    read0(cur ^ 1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = SplitMfma<H>::mma(al1[i], bh1[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = SplitMfma<H>::mma(ah1[i], bl1[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = SplitMfma<H>::mma(ah1[i], bh1[j], acc[i][j]);
    // loads of the A waves (the B waves of a narrower tile issue fewer)
    constexpr int kVmem = NJ == 4 ? (PF ? 16 + NPF : 16) : 8;
#pragma unroll
    for (int q = 0; q < kVmem; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < kReads; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, kMfma - kReads - kVmem, 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  // the repeated tail loads and the prefetches land before the epilogue
  // reuses the stages and before the wave ends
  __builtin_amdgcn_s_waitcnt(0);
  if constexpr (FUSED) {
    fused_epilogue<NJ>(acc, (float*)&lds[0][0][0], *fo, m0, n0, wm, wn, lane, out_scale);
    return;
  }
  const int64_t ldc = 2 * ldm;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t col = n0 + wn * 32 * NJ + j * 32 + lr;
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

template <typename H, bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_256_pp(const uint16_t* __restrict__ A,
                                                                 const uint16_t* __restrict__ B,
                                                                 float* __restrict__ C,
                                                                 int64_t ldm, int64_t ncols,
                                                                 float out_scale) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds_raw[kSplitLdsElems];
  uint16_t (*lds)[4][S_PLANE] = (uint16_t (*)[4][S_PLANE])lds_raw;
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  split_pp_tile<H, false, PF>(lds, A, B, C, ldm, ncols, (int64_t)tm * S_BM, (int64_t)tn * S_BN,
                              out_scale, nullptr);
}

// Occupation-fused twin of gemm_split_256_pp: tile (tm, tn) covers modes
// [128 tm, 128 tm + 128) and samples [128 tn, 128 tn + 128); no C is written.
template <typename H, bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_occ(const uint16_t* __restrict__ A,
                                                              const uint16_t* __restrict__ B,
                                                              int64_t ldm, int64_t ncols,
                                                              float out_scale, FusedOut fo) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds_raw[kSplitLdsElems];
  uint16_t (*lds)[4][S_PLANE] = (uint16_t (*)[4][S_PLANE])lds_raw;
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  split_pp_tile<H, true, PF>(lds, A, B, nullptr, ldm, ncols, (int64_t)tm * 128, (int64_t)tn * 128,
                             out_scale, &fo);
}

// ---------------------------------------------------------------- one-sided split, 256 x 256

// MP_SPLIT1_FP16: the packed transmission operand holds one FP16 value per
// entry (prescaled by 2^e as for MP_SPLIT_FP16) and only the sampled
// amplitudes are split, x = hi + lo, so each product is A B_hi + A B_lo: two
// v_mfma_f32_32x32x16_f16 products per fragment pair instead of three.  The
// FP16 rounding of T (at most 2^-11 relative per entry, unbiased) perturbs
// the network once for all samples; the propagated amplitudes are those of
// the rounded network to the split's 2^-22.
//
// Same 256 x 256 tile, four waves of 128 x 128 and ping-pong schedule as
// split_pp_tile.  A stage is 48 KB: A as 128 row pairs of 128 bytes (the
// packed A holds each row pair's 32-deep block as one line, see
// split1_a_offset) and B as 256 columns of 128 bytes (hi block, lo block),
// 16-byte chunk c of row r at c ^ swz8(r); two stages.  The 48 one-KB
// direct-to-LDS loads of a slab (each 8 whole lines) are spread over the
// waves, 12 each: load g = 12 w + q fills A row pairs 8 g .. 8 g + 7 (g < 16)
// or B rows 8 (g - 16) .. 8 (g - 16) + 7.  Fetching whole lines per load
// matters here: with 64-byte rows each line was requested by two loads of
// different waves, the second waiting on the first's miss.
constexpr int S1_NPL = 3;       // stage size in 256 x 32 planes
constexpr int kSplit1Stages = 2;  // LDS stages (loads run kSplit1Stages - 1 slabs ahead)
// B stage as 256 rows of 128 bytes (a column's hi and lo blocks side by side),
// so that each load instruction fetches 8 whole lines instead of 16 halves
// (M = 8000: 57.4 -> 54.7 ms per fused GEMM, same bits; with the A row pairs
// below 53.6 ms; three stages measured no faster).
constexpr bool kSplit1Lines = true;
constexpr int kSplit1Pf = 1;  // L2 prefetch loads per wave and slab (see split1_pp_tile)
constexpr int kSplit1StageElems = kSplit1Stages * S1_NPL * S_PLANE;
// the fused epilogue reuses 2 x 16384 floats of the array
constexpr int kSplit1LdsElems = (kSplit1StageElems > 65536 ? kSplit1StageElems : 65536) + 128;

template <bool FUSED, bool PF, int NST = kSplit1Stages, bool BL = kSplit1Lines,
          bool AL = kSplit1ALines>
__device__ __attribute__((always_inline)) inline void split1_pp_tile(
    uint16_t* __restrict__ lds, const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
    float* __restrict__ C, int64_t ldm, int64_t ncols, int64_t m0, int64_t n0, float out_scale,
    const FusedOut* fo, int tid = -1) {
  typedef f16x8 frag;
  static_assert(NST >= 2 && NST <= kSplit1Stages, "the LDS array holds kSplit1Stages stages");
  const int wave = tid < 0 ? (int)(threadIdx.x >> 6) : __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid < 0 ? (int)(threadIdx.x & 63) : tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  // Rows of the tile: A row r (FUSED: r < 128 the Re row of mode m0 + r, else
  // its Im row), B column r (FUSED: r < 128 the alpha column of sample n0 + r,
  // else its beta column; columns past the chunk repeat its last one).
  const int64_t bcols = FUSED ? ncols / 2 - n0 : ncols - n0;
  auto a_row = [&](int r) -> int64_t {
    if constexpr (FUSED) return r < 128 ? m0 + r : ldm + m0 + (r - 128);
    return m0 + r;
  };
  auto b_col = [&](int r) -> int64_t {
    if constexpr (FUSED) {
      const int64_t c = r & 127;
      return (c < bcols ? c : bcols - 1) + n0 + (r >= 128 ? ncols / 2 : 0);
    }
    return n0 + (r < bcols ? r : bcols - 1);
  };
  const int lrow = lane >> 2;
  const char* src[12];
  int sh[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int g = 12 * wave + q, plane = g >> 4;
    const int r = 16 * (g & 15) + lrow;
    const int chunk = (lane & 3) ^ swz(r);
    if (BL && plane > 0) {
      // B rows 8 (g - 16) .. + 7, 128 bytes each: lane l fills slot l % 8 of
      // row l / 8 with global chunk (l % 8) ^ swz8(row) (hi: 0-3, lo: 4-7)
      const int rb = 8 * (g - 16) + (lane >> 3);
      src[q] = (const char*)(B + b_col(rb) * 2 * ldm + (((lane & 7) ^ swz8(rb)) * 8));
      sh[q] = 2;
    } else if (AL && plane == 0) {
      // A row pairs 8 g .. 8 g + 7 (rows 16 g .. 16 g + 15), 128 bytes each
      const int pr = 8 * g + (lane >> 3);
      src[q] = (const char*)(A + a_row(2 * pr) * ldm + (((lane & 7) ^ swz8(pr)) * 8));
      sh[q] = 2;
    } else if (plane == 0) {
      src[q] = (const char*)(A + a_row(r) * ldm + chunk * 8);
      sh[q] = 1;  // slab k0 starts k0 FP16 values into the row
    } else {
      src[q] = (const char*)(B + b_col(r) * 2 * ldm + (plane == 2 ? 32 : 0) + chunk * 8);
      sh[q] = 2;  // 2 k0 values (hi and lo blocks) into the column
    }
  }
  auto issue = [&](int st, int64_t k0) {
    char* base = (char*)(lds + st * S1_NPL * S_PLANE);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const int g = 12 * wave + q;
      char* dst = base + (g >> 4) * (S_PLANE * 2) + (g & 15) * 1024;
      __builtin_amdgcn_global_load_lds((const void*)(src[q] + (k0 << sh[q])), (lds_void*)dst, 16,
                                       0, 0);
    }
  };
  // L2 prefetch of slab k0 into the sink after the stages (see split_pp_tile).
  // kSplit1Pf = 2: one 4-byte load per row (pair) of A (waves 0, 1) and per
  // column of B (waves 2, 3); 1: B columns only, 64 per wave.
  constexpr int NPF = kSplit1Pf;
  const char* pf_src[NPF];
  const int pf_sh = (NPF == 2 && wave < 2 && !AL) ? 1 : 2;
#pragma unroll
  for (int q = 0; q < NPF; ++q) {
    if constexpr (NPF == 1) {
      pf_src[q] = (const char*)(B + b_col(64 * wave + lane) * 2 * ldm);
    } else {
      // AL: 128 row-pair lines, each wave of A touches its 64 twice
      const int r = AL && wave < 2 ? 2 * (64 * (wave & 1) + lane) : 128 * (wave & 1) + 64 * q + lane;
      pf_src[q] = wave < 2 ? (const char*)(A + a_row(r) * ldm) : (const char*)(B + b_col(r) * 2 * ldm);
    }
  }
  auto prefetch = [&](int64_t k0) {
    if constexpr (!PF) return;
#pragma unroll
    for (int q = 0; q < NPF; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(pf_src[q] + (k0 << pf_sh)),
                                       (lds_void*)(lds + NST * S1_NPL * S_PLANE), 4, 0, 0);
  };
  // fragment offsets (elements from the stage's plane 0 / plane 1): A in
  // 64-byte rows; B hi and lo in planes 1 and 2 of 64-byte rows, or (BL) in
  // one plane of 128-byte rows, hi chunks 0-3 and lo chunks 4-7
  int oa[2][4], obh[2][4], obl[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra = wm * 128 + i * 32 + lr, rb = wn * 128 + i * 32 + lr;
      if constexpr (AL) {
        const int pr = ra >> 1;
        oa[s][i] = pr * 2 * S_BK + ((((ra & 1) * 4 + 2 * lh + s) ^ swz8(pr)) << 3);
      } else {
        oa[s][i] = ra * S_BK + (((2 * lh + s) ^ swz(ra)) << 3);
      }
      if constexpr (BL) {
        obh[s][i] = rb * 2 * S_BK + (((2 * lh + s) ^ swz8(rb)) << 3);
        obl[s][i] = rb * 2 * S_BK + (((4 + 2 * lh + s) ^ swz8(rb)) << 3);
      } else {
        obh[s][i] = rb * S_BK + (((2 * lh + s) ^ swz(rb)) << 3);
        obl[s][i] = S_PLANE + obh[s][i];
      }
    }
  frag a0[4], bh0[4], bl0[4], a1[4], bh1[4], bl1[4];
  auto plane = [&](int st, int p) { return lds + (st * S1_NPL + p) * S_PLANE; };
  auto read0 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bl0[i] = *(const frag*)(plane(st, 1) + obl[0][i]);
      a0[i] = *(const frag*)(plane(st, 0) + oa[0][i]);
      bh0[i] = *(const frag*)(plane(st, 1) + obh[0][i]);
    }
  };
  auto read1 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bl1[i] = *(const frag*)(plane(st, 1) + obl[1][i]);
      a1[i] = *(const frag*)(plane(st, 0) + oa[1][i]);
      bh1[i] = *(const frag*)(plane(st, 1) + obh[1][i]);
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // Slab kt lives in stage kt % NST; the loads of slab kt + NST go into its
  // stage once every wave has passed the barrier of slab kt.  Each slab's
  // group of loads is 12 stage loads (+ 2 prefetch loads with PF), and loads
  // complete in issue order, so "slab kt + 1 landed" is vmcnt(the groups of
  // the NST - 2 later slabs + its own prefetch).
  constexpr int kGroup = PF ? 12 + NPF : 12;
  constexpr int kWaitN = kGroup * (NST - 2) + (PF ? NPF : 0);
  static_assert(kWaitN < 64, "vmcnt field");
  const int KT = (int)(ldm / S_BK);  // >= 4
  issue(0, 0);
#pragma unroll
  for (int s = 1; s + 1 < NST; ++s) {
    issue(s, (int64_t)s * S_BK);
    prefetch((int64_t)min(s + kPrefetchSlabs, KT - 1) * S_BK);
  }
  wait_vm<kGroup * (NST - 2)>();  // slab 0 landed
  barrier_no_fence();
  issue(NST - 1, (int64_t)min(NST - 1, KT - 1) * S_BK);
  prefetch((int64_t)min(NST - 1 + kPrefetchSlabs, KT - 1) * S_BK);
  read0(0);
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  int cur = 0;
  for (int kt = 0; kt < KT; ++kt) {
    const int nxt = cur + 1 == NST ? 0 : cur + 1;
    // phase A: MFMAs on F0 (lo products first) with the reads of F1 between them
    read1(cur);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[i], bl0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[i], bh0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 8, 0);
    __builtin_amdgcn_sched_barrier(0);
    // own loads of slab kt + 1 landed, own reads of stage cur complete
    __builtin_amdgcn_s_waitcnt((kWaitN & 15) | ((kWaitN >> 4) << 14) | (7 << 4));
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: MFMAs on F1 with slab kt + NST's loads and the reads of F0
    // threaded in (the last slabs reload the final slab, in bounds)
    issue(cur, (int64_t)min(kt + NST, KT - 1) * S_BK);
    prefetch((int64_t)min(kt + NST + kPrefetchSlabs, KT - 1) * S_BK);
    read0(nxt);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[i], bl1[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[i], bh1[j], acc[i][j], 0, 0, 0);
    constexpr int kVmem = PF ? 12 + NPF : 12;
#pragma unroll
    for (int q = 0; q < kVmem; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 32 - 12 - kVmem, 1);
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
  }
  __builtin_amdgcn_s_waitcnt(0);
  if constexpr (FUSED) {
    fused_epilogue(acc, (float*)lds, *fo, m0, n0, wm, wn, lane, out_scale);
    return;
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

template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1_pp(const uint16_t* __restrict__ A,
                                                              const uint16_t* __restrict__ B,
                                                              float* __restrict__ C, int64_t ldm,
                                                              int64_t ncols, float out_scale) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[kSplit1LdsElems];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  split1_pp_tile<false, PF>(lds, A, B, C, ldm, ncols, (int64_t)tm * S_BM, (int64_t)tn * S_BN,
                            out_scale, nullptr);
}

template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1_occ(const uint16_t* __restrict__ A,
                                                               const uint16_t* __restrict__ B,
                                                               int64_t ldm, int64_t ncols,
                                                               float out_scale, FusedOut fo) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[kSplit1LdsElems];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  split1_pp_tile<true, PF>(lds, A, B, nullptr, ldm, ncols, (int64_t)tm * 128, (int64_t)tn * 128,
                           out_scale, &fo);
}

// ---------------------------------------------------------------- one-sided split of T, 256 x 256

// MP_SPLIT1T_FP16: the transmission operand is split, T = T_hi + T_lo (the
// MP_SPLIT_FP16 packing, prescaled by 2^e), and the sampled amplitudes are one
// FP16 value each, so each product is A_hi B + A_lo B: two
// v_mfma_f32_32x32x16_f16 per fragment pair.  The propagation is the one of
// the FP16-rounded samples through T to the split's 2^-22; the rounding error
// is a different draw for every sample, so it averages over the ensemble like
// the sampling noise (no bias of the network itself).
//
// The mirror of split1_pp_tile: a 48 KB stage holds B as 128 column pairs of
// 128 bytes (plane 0: one pair's two 32-value runs side by side, as the
// sampler stores them) and A as 256 rows of 128 bytes (planes 1-2: a row's hi
// and lo blocks of one slab); 16-byte chunk c of LDS row r at c ^ swz8(r).
// Load g = 12 w + q of a slab fills B pairs 8 g .. 8 g + 7 (g < 16) or A rows
// 8 (g - 16) .. 8 (g - 16) + 7, eight whole lines per load.
//
// Columns are storage columns of the sample operand (split1t_half): FUSED
// tiles take the alpha pairs of samples [n0, n0 + 128) and the beta pairs
// (E2 = ncols / 2 further); pairs past the chunk repeat its last pair.  The
// C-writing form maps storage column c to C column c (alpha, c < E) or
// E + c - E2 (beta) and skips the padding columns of an odd E (`e_real`).
// PFA: the L2 prefetch touches the lines of A's rows (else of B's pairs).
template <bool FUSED, bool PF, bool PFA>
__device__ __attribute__((always_inline)) inline void split1t_pp_tile(
    uint16_t* __restrict__ lds, const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
    float* __restrict__ C, int64_t ldm, int64_t ncols, int64_t e_real, int64_t m0, int64_t n0,
    float out_scale, const FusedOut* fo, int tid = -1) {
  typedef f16x8 frag;
  constexpr int NST = kSplit1Stages;
  const int wave = tid < 0 ? (int)(threadIdx.x >> 6) : __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid < 0 ? (int)(threadIdx.x & 63) : tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  auto a_row = [&](int r) -> int64_t {
    if constexpr (FUSED) return r < 128 ? m0 + r : ldm + m0 + (r - 128);
    return m0 + r;
  };
  // first storage column of tile column pair pr (tile columns 2 pr, 2 pr + 1)
  const int64_t half = FUSED ? ncols / 2 : ncols;  // storage columns per block
  auto b_pair = [&](int pr) -> int64_t {
    if constexpr (FUSED) {
      const int64_t c = n0 + 2 * (pr & 63);
      return (c <= half - 2 ? c : half - 2) + (pr >= 64 ? half : 0);
    }
    const int64_t c = n0 + 2 * pr;
    return c <= half - 2 ? c : half - 2;
  };
  const char* src[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int g = 12 * wave + q;
    if (g < 16) {
      // B pairs 8 g .. 8 g + 7: lane l fills slot l % 8 of pair l / 8 with
      // global chunk (l % 8) ^ swz8(pair) (chunks 0-3 the even column, 4-7 the odd)
      const int pr = 8 * g + (lane >> 3);
      src[q] = (const char*)(B + b_pair(pr) * ldm + (((lane & 7) ^ swz8(pr)) * 8));
    } else {
      // A rows 8 (g - 16) .. + 7, hi chunks 0-3 and lo chunks 4-7
      const int ra = 8 * (g - 16) + (lane >> 3);
      src[q] = (const char*)(A + a_row(ra) * 2 * ldm + (((lane & 7) ^ swz8(ra)) * 8));
    }
  }
  // both operands advance 2 k0 values per slab (hi and lo blocks, or the
  // pair's two runs)
  auto issue = [&](int st, int64_t k0) {
    char* base = (char*)(lds + st * S1_NPL * S_PLANE);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const int g = 12 * wave + q;
      char* dst = base + (g >> 4) * (S_PLANE * 2) + (g & 15) * 1024;
      __builtin_amdgcn_global_load_lds((const void*)(src[q] + (k0 << 2)), (lds_void*)dst, 16, 0,
                                       0);
    }
  };
  // L2 prefetch of slab k0 into the sink after the stages: one 4-byte load
  // per wave and slab, 64 A rows per wave (PFA) or 32 B pairs per wave (each
  // touched by two lanes)
  const char* pf_src = PFA ? (const char*)(A + a_row(64 * wave + lane) * 2 * ldm)
                           : (const char*)(B + b_pair(32 * wave + (lane & 31)) * ldm);
  auto prefetch = [&](int64_t k0) {
    if constexpr (!PF) return;
    __builtin_amdgcn_global_load_lds((const void*)(pf_src + (k0 << 2)),
                                     (lds_void*)(lds + NST * S1_NPL * S_PLANE), 4, 0, 0);
  };
  constexpr int NPF = 1;
  // fragment offsets: A hi and lo in planes 1-2 (128-byte rows), B in plane 0
  // (128-byte pair rows)
  int oah[2][4], oal[2][4], ob[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra = wm * 128 + i * 32 + lr, rb = wn * 128 + i * 32 + lr;
      oah[s][i] = ra * 2 * S_BK + (((2 * lh + s) ^ swz8(ra)) << 3);
      oal[s][i] = ra * 2 * S_BK + (((4 + 2 * lh + s) ^ swz8(ra)) << 3);
      const int pr = rb >> 1;
      ob[s][i] = pr * 2 * S_BK + ((((rb & 1) * 4 + 2 * lh + s) ^ swz8(pr)) << 3);
    }
  frag b0[4], ah0[4], al0[4], b1[4], ah1[4], al1[4];
  auto plane = [&](int st, int p) { return lds + (st * S1_NPL + p) * S_PLANE; };
  auto read0 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al0[i] = *(const frag*)(plane(st, 1) + oal[0][i]);
      b0[i] = *(const frag*)(plane(st, 0) + ob[0][i]);
      ah0[i] = *(const frag*)(plane(st, 1) + oah[0][i]);
    }
  };
  auto read1 = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al1[i] = *(const frag*)(plane(st, 1) + oal[1][i]);
      b1[i] = *(const frag*)(plane(st, 0) + ob[1][i]);
      ah1[i] = *(const frag*)(plane(st, 1) + oah[1][i]);
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // the schedule and waits of split1_pp_tile (two stages)
  constexpr int kGroup = PF ? 12 + NPF : 12;
  constexpr int kWaitN = PF ? NPF : 0;
  const int KT = (int)(ldm / S_BK);  // >= 4
  issue(0, 0);
  wait_vm<0>();  // slab 0 landed
  barrier_no_fence();
  issue(1, (int64_t)min(1, KT - 1) * S_BK);
  prefetch((int64_t)min(1 + kPrefetchSlabs, KT - 1) * S_BK);
  read0(0);
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  int cur = 0;
  for (int kt = 0; kt < KT; ++kt) {
    const int nxt = cur ^ 1;
    // phase A: MFMAs on F0 (lo products first) with the reads of F1 between them
    read1(cur);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al0[i], b0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah0[i], b0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 8, 0);
    __builtin_amdgcn_sched_barrier(0);
    // own loads of slab kt + 1 landed (with PF only the prefetch load issued
    // after them may be in flight), own reads of stage cur complete
    __builtin_amdgcn_s_waitcnt((kWaitN & 15) | ((kWaitN >> 4) << 14) | (7 << 4));
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: MFMAs on F1 with slab kt + 2's loads and the reads of F0
    // threaded in (the last slabs reload the final slab, in bounds)
    issue(cur, (int64_t)min(kt + NST, KT - 1) * S_BK);
    prefetch((int64_t)min(kt + NST + kPrefetchSlabs, KT - 1) * S_BK);
    read0(nxt);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al1[i], b1[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah1[i], b1[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 32 - 12 - kGroup, 1);
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
  }
  __builtin_amdgcn_s_waitcnt(0);
  if constexpr (FUSED) {
    fused_epilogue(acc, (float*)lds, *fo, m0, n0, wm, wn, lane, out_scale);
    return;
  }
  const int64_t ldc = 2 * ldm, e2 = split1t_half(e_real);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t sc = n0 + wn * 128 + j * 32 + lr;  // storage column
    if (sc >= ncols) continue;
    int64_t col;
    if (sc < e2) {
      if (sc >= e_real) continue;  // padding of an odd E
      col = sc;
    } else {
      if (sc - e2 >= e_real) continue;
      col = e_real + (sc - e2);
    }
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

// The L2 prefetch of the T-split kernels touches the sample operand's pairs
// (M = 8000, fused call: 51.3 ms against 55.7 ms touching A's rows; with 4 x 8
// tiles per XCD step 52.0 and 56.2 ms).
constexpr bool kSplit1tPfA = false;
// Tile order of the T-split kernels: row tiles by column tiles per XCD and step.
constexpr int kS1tStepRows = 8, kS1tStepCols = 4;

template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t_pp(const uint16_t* __restrict__ A,
                                                               const uint16_t* __restrict__ B,
                                                               float* __restrict__ C, int64_t ldm,
                                                               int64_t ncols, int64_t e_real,
                                                               float out_scale) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[kSplit1LdsElems];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block<kS1tStepRows, kS1tStepCols>(tiles_m, tiles_n, tm, tn)) return;
  split1t_pp_tile<false, PF, kSplit1tPfA>(lds, A, B, C, ldm, ncols, e_real, (int64_t)tm * S_BM,
                                          (int64_t)tn * S_BN, out_scale, nullptr);
}

template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t_occ(const uint16_t* __restrict__ A,
                                                                const uint16_t* __restrict__ B,
                                                                int64_t ldm, int64_t ncols,
                                                                float out_scale, FusedOut fo) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[kSplit1LdsElems];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block<kS1tStepRows, kS1tStepCols>(tiles_m, tiles_n, tm, tn)) return;
  split1t_pp_tile<true, PF, kSplit1tPfA>(lds, A, B, nullptr, ldm, ncols, 0, (int64_t)tm * 128,
                                         (int64_t)tn * 128, out_scale, &fo);
}

// ---------------------------------------------------------------- bilinear-form epilogue

// One distribution S needs only n_S = sum_{j in S} alpha'_j beta'_j per sample,
// and with alpha' = T alpha, beta' = T* beta (real alpha, beta) that is the
// bilinear form alpha^T W beta, W = T^T P_S T* (P_S: the projector on S).  W's
// diagonal D (real: D_a = sum_{j in S} |T_ja|^2) alone sets the mean of n_S,
// since E[alpha_a beta_b] vanishes for a != b; it is applied in FP32 here, as
// sum_a D_a alpha_a beta_a, and the GEMM applies the off-diagonal part, whose
// packing rounding then only adds noise per sample (packed with D in it, the
// rounding of equal diagonal entries would bias every sample alike).  The tile
// holds the Re and Im rows of W_off beta for 128 input modes a (waves wm = 0
// and 1) and 256 samples; each sample's partial is sum_a alpha_a (W beta)_a
// over the tile's modes, written as (Re, 0) by wm = 0 and (0, Im) by wm = 1 in
// the occupation partials' layout (slot = the 128-mode block, one run from mode
// 0), which the counting kernels read unchanged.  alpha and beta are the FP16
// sample operand's halves in column pairs (zeros on padding modes, as D); the
// register of acc[i][j] at 4 g + rr is mode i 32 + 8 g + 4 lh + rr of the wave
// and sample j 32 + lr.
__device__ inline void bilinear_epilogue(f32x16 (&acc)[4][4], const uint16_t* __restrict__ alpha,
                                         const uint16_t* __restrict__ beta,
                                         const float* __restrict__ diag, const FusedOut& fo,
                                         int64_t ldm, int64_t m0, int64_t n0, int wm, int wn,
                                         int lane, float out_scale) {
  typedef __attribute__((ext_vector_type(4))) _Float16 f16x4;
  typedef __attribute__((ext_vector_type(2))) float f32x2;
  const int lr = lane & 31, lh = lane >> 5;
  const int64_t slot = fo.slot_off[0] + (m0 >> 7);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t smp = n0 + wn * 128 + j * 32 + lr;
    float sum = 0.f, dsum = 0.f;
    if (smp < fo.E) {
      const int64_t off = (smp >> 1) * 2 * ldm + 32 * (smp & 1);
      const _Float16* col = (const _Float16*)alpha + off;
      const _Float16* bcol = (const _Float16*)beta + off;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int64_t mode = m0 + i * 32 + 8 * g + 4 * lh;  // four consecutive modes
          const int64_t at = 64 * (mode >> 5) + (mode & 31);
          const f16x4 a4 = *(const f16x4*)(col + at);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) sum += (float)a4[rr] * acc[i][j][4 * g + rr];
          if (wm == 0) {
            const f16x4 b4 = *(const f16x4*)(bcol + at);
            const f32x4 d4 = *(const f32x4*)(diag + mode);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) dsum += d4[rr] * ((float)a4[rr] * (float)b4[rr]);
          }
        }
    }
    sum = sum * out_scale + dsum;
    sum += __shfl_xor(sum, 32, 64);  // the other lane half's modes
    if (lh == 0 && smp < fo.E) {
      const float v = sum;
      *(f32x2*)(fo.part + (slot * fo.E + smp) * 4 + 2 * wm) =
          wm == 0 ? f32x2{v, 0.f} : f32x2{0.f, v};
    }
  }
}

// ---------------------------------------------------------------- T-split with an FP8 correction, 256 x 256

// MP_SPLIT1T_F8: the T-split product T_hi S + T_lo S with its correction term
// in FP8.  T_hi is T (prescaled by 2^e) rounded to FP16; the remainder
// T_lo = x - T_hi, at most 2^-10 of x, is scaled by 2^(18 - e) and rounded
// to e4m3, so the network is kept to about 2^-15 of x; the samples are one
// FP16 value S and its e4m3 copy S8.  The correction T_lo8 S8 needs only a
// few significant bits (it is 2^-11 of the product), and one
// v_mfma_scale_f32_32x32x64_f8f6f4 (its A block scale 2^(e - 18) undoes the
// remainder's scale) replaces the second FP16 product of a 64-deep block at
// half its issue cost: per pair of 32-deep slabs 4 FP16 MFMAs and 1 FP8 MFMA
// per 32 x 32 block instead of 8 FP16 MFMAs.
//
// Operands in pair lines (128 bytes): T_hi in row pairs (MP_SPLIT1_FP16's
// packing) and S in column pairs (MP_SPLIT1T_FP16's layout) per 32-deep
// slab; T_lo8 and S8 in row / column pairs per 64-deep block.  LDS: two
// FP16 stages of 32 KB ([S pairs][T_hi pairs], 16 KB each) and two FP8
// buffers of 32 KB ([S8 pairs][T_lo8 pairs]), then the prefetch sink; 16-byte
// chunk c of pair line p at c ^ swz8(p) in every plane.  A 32-byte FP8
// fragment of row r is the chunks 2 lh, 2 lh + 1 of its 64-byte run (lane
// half lh supplies k = 32 lh .. 32 lh + 31, the same on both operands).
//
// Slab kt uses FP16 stage kt & 1 and FP8 buffer (kt / 2) & 1: an even slab
// reads T_lo8's fragments (all four row blocks, kept in registers for the
// odd slab) and S8's for column blocks 0-1, an odd slab S8's for blocks 2-3;
// each slab issues the FP8 MFMAs of its two column blocks.  The FP8 loads of
// pair q are issued half in slab 2q - 3 (S8) and half in slab 2q - 2
// (T_lo8), after the barriers that end the reads of pair q - 2 from the same
// buffer, and land before the slab 2q - 1 barrier that precedes their reads;
// past the last pair they reload it into the buffer no longer read.
constexpr int F8_PLANE = 16384;              // bytes: 128 pair lines
constexpr int F8_STAGE = 2 * F8_PLANE;       // [B pairs][A pairs]
constexpr int F8_LDS = 4 * F8_STAGE + 1024;  // two FP16 stages, two FP8 buffers, sink

__device__ inline int f8_chunk_off(int r, int c) {
  return (r >> 1) * 128 + ((c ^ swz8(r >> 1)) << 4);
}

// MODE 0 stores C; MODE 1 is the occupation-fused tile (128 alpha and 128 beta
// columns of the same samples, Re and Im rows of 128 modes); MODE 2 is the
// bilinear-form tile (Re and Im rows of 128 modes of W beta for 256 samples,
// reduced against alpha by bilinear_epilogue).
template <int MODE, bool PF>
__device__ __attribute__((always_inline)) inline void split1t8_pp_tile(
    char* __restrict__ lds, const uint16_t* __restrict__ A, const uint8_t* __restrict__ A8,
    const uint16_t* __restrict__ B, const uint8_t* __restrict__ B8, float* __restrict__ C,
    int64_t ldm, int64_t ncols, int64_t e_real, int64_t m0, int64_t n0, float out_scale,
    int scale_a, const FusedOut* fo, int tid = -1, const uint16_t* __restrict__ alpha = nullptr,
    const float* __restrict__ diag = nullptr) {
  constexpr bool FUSED = MODE == 1, ROWS_RI = MODE != 0;
  typedef __attribute__((ext_vector_type(8))) int i32x8;
  typedef __attribute__((ext_vector_type(4))) int i32x4;
  const int wave = tid < 0 ? (int)(threadIdx.x >> 6) : __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid < 0 ? (int)(threadIdx.x & 63) : tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  // first global row of tile row pair pa (tile rows 2 pa, 2 pa + 1)
  auto a_row = [&](int pa) -> int64_t {
    if constexpr (ROWS_RI) return pa < 64 ? m0 + 2 * pa : ldm + m0 + 2 * (pa - 64);
    return m0 + 2 * pa;
  };
  // first storage column of tile column pair pr
  const int64_t half = FUSED ? ncols / 2 : ncols;
  auto b_pair = [&](int pr) -> int64_t {
    if constexpr (FUSED) {
      const int64_t c = n0 + 2 * (pr & 63);
      return (c <= half - 2 ? c : half - 2) + (pr >= 64 ? half : 0);
    }
    const int64_t c = n0 + 2 * pr;
    return c <= half - 2 ? c : half - 2;
  };
  // FP16 stage: load g = 8 wave + q fills B pairs 8 g .. (g < 16) or A pairs
  // 8 (g - 16) ..; lane l fills slot l % 8 of pair l / 8 with global chunk
  // (l % 8) ^ swz8(pair)
  const char* src16[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int g = 8 * wave + q, chunk = lane & 7;
    if (g < 16) {
      const int pr = 8 * g + (lane >> 3);
      src16[q] = (const char*)(B + b_pair(pr) * ldm) + ((chunk ^ swz8(pr)) << 4);
    } else {
      const int pa = 8 * (g - 16) + (lane >> 3);
      src16[q] = (const char*)(A + a_row(pa) * ldm) + ((chunk ^ swz8(pa)) << 4);
    }
  }
  // FP8 buffer: half 0 = B8 pairs, half 1 = A8 pairs, load g = 4 wave + q
  const char* src8[2][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g = 4 * wave + q, chunk = lane & 7, p = 8 * g + (lane >> 3);
    src8[0][q] = (const char*)(B8 + b_pair(p) * ldm) + ((chunk ^ swz8(p)) << 4);
    src8[1][q] = (const char*)(A8 + a_row(p) * ldm) + ((chunk ^ swz8(p)) << 4);
  }
  auto issue16 = [&](int st, int64_t k0) {
    char* base = lds + st * F8_STAGE;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src16[q] + (k0 << 2)),
                                       (lds_void*)(base + (8 * wave + q) * 1024), 16, 0, 0);
  };
  const int KT = (int)(ldm / S_BK);  // even (ldm is a multiple of 128), >= 4
  const int NP = KT / 2;
  // half `hf` of FP8 pair `pair` into buffer pair & 1 (data of pair min(pair, NP - 1))
  auto issue8 = [&](int pair, int hf) {
    char* base = lds + 2 * F8_STAGE + (pair & 1) * F8_STAGE + hf * F8_PLANE;
    const int64_t k0 = (int64_t)min(pair, NP - 1) * 64;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src8[hf][q] + (k0 << 1)),
                                       (lds_void*)(base + (4 * wave + q) * 1024), 16, 0, 0);
  };
  // L2 prefetch of the sample pairs' lines, one 4-byte load per wave and slab
  const char* pf_src = (const char*)(B + b_pair(32 * wave + (lane & 31)) * ldm);
  auto prefetch = [&](int64_t k0) {
    if constexpr (!PF) return;
    __builtin_amdgcn_global_load_lds((const void*)(pf_src + (k0 << 2)),
                                     (lds_void*)(lds + 4 * F8_STAGE), 4, 0, 0);
  };
  int oa[2][4], ob[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra = wm * 128 + i * 32 + lr, rb = wn * 128 + i * 32 + lr;
      oa[s][i] = f8_chunk_off(ra, (ra & 1) * 4 + 2 * lh + s);
      ob[s][i] = f8_chunk_off(rb, (rb & 1) * 4 + 2 * lh + s);
    }
  f16x8 a0[4], b0[4], a1[4], b1[4];
  i32x8 a8[4], b8[4];
  auto read16 = [&](int st, int s, f16x8* a, f16x8* b) {
    const char* pb = lds + st * F8_STAGE;
    const char* pa = pb + F8_PLANE;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = *(const f16x8*)(pa + oa[s][i]);
      b[i] = *(const f16x8*)(pb + ob[s][i]);
    }
  };
  auto rd8 = [&](const char* p, int o0, int o1) -> i32x8 {
    const i32x4 x = *(const i32x4*)(p + o0), y = *(const i32x4*)(p + o1);
    return i32x8{x[0], x[1], x[2], x[3], y[0], y[1], y[2], y[3]};
  };
  auto read8 = [&](int kt, auto par) {
    constexpr int P = decltype(par)::value;
    const char* pb = lds + 2 * F8_STAGE + ((kt >> 1) & 1) * F8_STAGE;
    const char* pa = pb + F8_PLANE;
    if constexpr (P == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) a8[i] = rd8(pa, oa[0][i], oa[1][i]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b8[j] = rd8(pb, ob[0][j], ob[1][j]);
    } else {
#pragma unroll
      for (int j = 2; j < 4; ++j) b8[j] = rd8(pb, ob[0][j], ob[1][j]);
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // prologue: slab 0 and FP8 pair 0 landed; slab 1 and pair 1's first half in flight
  issue16(0, 0);
  issue8(0, 0);
  issue8(0, 1);
  __builtin_amdgcn_s_waitcnt(0);
  barrier_no_fence();
  issue16(1, S_BK);
  issue8(1, 0);
  prefetch((int64_t)min(1 + kPrefetchSlabs, KT - 1) * S_BK);
  read16(0, 0, a0, b0);
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  constexpr int kWaitN = PF ? 1 : 0;
  auto slab = [&](int kt, auto par) {
    constexpr int P = decltype(par)::value;  // kt & 1: the FP16 stage
    // phase A: FP16 MFMAs on step 0; reads of step 1 and of the slab's FP8 fragments
    read16(P, 1, a1, b1);
    read8(kt, par);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[i], b0[j], acc[i][j], 0, 0, 0);
    if constexpr (P == 0) {  // 8 + 12 reads
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
        __builtin_amdgcn_sched_group_barrier(kSgDsRead, 2, 0);
      }
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 6, 0);
    } else {  // 8 + 4 reads
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
        __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 4, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    // own loads of the previous slab landed (with PF but the prefetch after
    // them), own reads complete
    __builtin_amdgcn_s_waitcnt((kWaitN & 15) | ((kWaitN >> 4) << 14) | (7 << 4));
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: FP16 MFMAs on step 1 and the FP8 MFMAs of column blocks 2P,
    // 2P + 1; loads of slab kt + 2 and of half P ^ 1 of FP8 pair
    // (kt + 1) / 2 + 1; reads of step 0 of slab kt + 1
    issue16(P, (int64_t)min(kt + 2, KT - 1) * S_BK);
    issue8((kt + 1) / 2 + 1, P ^ 1);
    prefetch((int64_t)min(kt + 2 + kPrefetchSlabs, KT - 1) * S_BK);
    read16(P ^ 1, 0, a0, b0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[i], b1[j], acc[i][j], 0, 0, 0);
    constexpr int jb = 2 * P;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
        acc[i][jb + jj] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            a8[i], b8[jb + jj], acc[i][jb + jj], 0, 0, 0, scale_a, 0, 127);
    constexpr int kVm = PF ? 13 : 12;
#pragma unroll
    for (int q = 0; q < kVm; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 24 - kVm - 8, 1);
    __builtin_amdgcn_sched_barrier(0);
  };
  for (int kt = 0; kt < KT; kt += 2) {
    slab(kt, std::integral_constant<int, 0>{});
    slab(kt + 1, std::integral_constant<int, 1>{});
  }
  __builtin_amdgcn_s_waitcnt(0);
  if constexpr (FUSED) {
    fused_epilogue(acc, (float*)lds, *fo, m0, n0, wm, wn, lane, out_scale);
    return;
  }
  if constexpr (MODE == 2) {
    bilinear_epilogue(acc, alpha, B, diag, *fo, ldm, m0, n0, wm, wn, lane, out_scale);
    return;
  }
  const int64_t ldc = 2 * ldm, e2 = split1t_half(e_real);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t sc = n0 + wn * 128 + j * 32 + lr;  // storage column
    if (sc >= ncols) continue;
    int64_t col;
    if (sc < e2) {
      if (sc >= e_real) continue;  // padding of an odd E
      col = sc;
    } else {
      if (sc - e2 >= e_real) continue;
      col = e_real + (sc - e2);
    }
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

// A8 and B8 follow the FP16 parts of the packed operand (4 ldm^2 bytes) and
// of the sample operand (2 ncols ldm bytes).
template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t8_pp(const uint16_t* __restrict__ A,
                                                                const uint16_t* __restrict__ B,
                                                                float* __restrict__ C, int64_t ldm,
                                                                int64_t ncols, int64_t e_real,
                                                                float out_scale, int scale_a) {
  __shared__ __attribute__((aligned(1024))) char lds[F8_LDS];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block<kS1tStepRows, kS1tStepCols>(tiles_m, tiles_n, tm, tn)) return;
  const uint8_t* A8 = (const uint8_t*)A + 4 * ldm * ldm;
  const uint8_t* B8 = (const uint8_t*)B + 2 * ncols * ldm;
  split1t8_pp_tile<0, PF>(lds, A, A8, B, B8, C, ldm, ncols, e_real, (int64_t)tm * S_BM,
                              (int64_t)tn * S_BN, out_scale, scale_a, nullptr);
}

template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t8_occ(const uint16_t* __restrict__ A,
                                                                 const uint16_t* __restrict__ B,
                                                                 int64_t ldm, int64_t ncols,
                                                                 float out_scale, int scale_a,
                                                                 FusedOut fo) {
  __shared__ __attribute__((aligned(1024))) char lds[F8_LDS];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block<kS1tStepRows, kS1tStepCols>(tiles_m, tiles_n, tm, tn)) return;
  const uint8_t* A8 = (const uint8_t*)A + 4 * ldm * ldm;
  const uint8_t* B8 = (const uint8_t*)B + 2 * ncols * ldm;
  split1t8_pp_tile<1, PF>(lds, A, A8, B, B8, nullptr, ldm, ncols, 0, (int64_t)tm * 128,
                             (int64_t)tn * 128, out_scale, scale_a, &fo);
}

// Bilinear form alpha^T W beta per sample (one distribution): A is W packed
// as MP_SPLIT1T_F8 packs T, B and B8 the beta half of the sample operand
// (storage columns E2 ..) and its e4m3 copies, alpha the FP16 alpha half.
template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t8_bilin(
    const uint16_t* __restrict__ A, const uint16_t* __restrict__ B, const uint8_t* __restrict__ B8,
    const uint16_t* __restrict__ alpha, const float* __restrict__ diag, int64_t ldm,
    int64_t ncols, float out_scale, int scale_a, FusedOut fo) {
  __shared__ __attribute__((aligned(1024))) char lds[F8_LDS];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block<kS1tStepRows, kS1tStepCols>(tiles_m, tiles_n, tm, tn)) return;
  const uint8_t* A8 = (const uint8_t*)A + 4 * ldm * ldm;
  split1t8_pp_tile<2, PF>(lds, A, A8, B, B8, nullptr, ldm, ncols, 0, (int64_t)tm * 128,
                          (int64_t)tn * S_BN, out_scale, scale_a, &fo, -1, alpha, diag);
}

// ---- W = T^T P_S T* for the bilinear form, from the FP64 GEMM

// Tt = T^T (complex, the layout of T: entry (i, j) at 2 (i M + j)).
__global__ void bilin_transpose(const double* __restrict__ T, int M, double* __restrict__ Tt) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)M * M) return;
  const int64_t a = idx / M, b = idx % M;
  Tt[2 * idx] = T[2 * (b * M + a)];
  Tt[2 * idx + 1] = T[2 * (b * M + a) + 1];
}

// X in the FP64 sample layout with E = M: column k holds P_S Re T[:, k] and
// column M + k holds P_S Im T[:, k] (modes j with in_s[j] < 0 and padding zero).
__global__ void bilin_columns(const double* __restrict__ T, int M, int64_t ldm,
                              const int32_t* __restrict__ in_s, double* __restrict__ X) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)M * ldm) return;
  const int64_t k = idx / ldm, j = idx % ldm;
  double re = 0.0, im = 0.0;
  if (j < M && in_s[j] >= 0) {
    re = T[2 * (j * M + k)];
    im = T[2 * (j * M + k) + 1];
  }
  X[k * ldm + j] = re;
  X[(M + k) * ldm + j] = im;
}

// With T = A + i B, C = [A^T; B^T] [P A | P B] holds A^T P A, B^T P A (columns
// b < M) and A^T P B, B^T P B (columns M + b); W = T^T P T* has real part
// A^T P A + B^T P B and imaginary part B^T P A - A^T P B.
__global__ void bilin_combine(const double* __restrict__ C, int M, int64_t ldm,
                              double* __restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)M * M) return;
  const int64_t a = idx / M, b = idx % M, ldc = 2 * ldm;
  const double* c1 = C + b * ldc;        // column b: [A^T P A; B^T P A] e_b
  const double* c2 = C + (M + b) * ldc;  // column M + b: [A^T P B; B^T P B] e_b
  W[2 * idx] = a == b ? 0.0 : c1[a] + c2[ldm + a];  // the diagonal goes to D
  W[2 * idx + 1] = a == b ? 0.0 : c1[ldm + a] - c2[a];
}

// D_a = Re W_aa (W_aa = sum_{j in S} |T_ja|^2 is real) in FP32, zero on padding.
__global__ void bilin_diag(const double* __restrict__ C, int M, int64_t ldm,
                           float* __restrict__ D) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (a >= ldm) return;
  D[a] = a < M ? (float)(C[a * 2 * ldm + a] + C[(M + a) * 2 * ldm + ldm + a]) : 0.0f;
}

// ---------------------------------------------------------------- FP32, 256 x 256

// FP32 twin of the split ping-pong kernel: the same 256 x 256 tile, four
// waves of 128 x 128, two direct-to-LDS stages, v_mfma_f32_32x32x2f32.
// BK = 32 floats, so an LDS row is one 128-byte line of 8 chunks; chunk c of
// row r sits at c ^ ((r >> 1) & 7), conflict-free for the 16-byte fragment
// reads (16 consecutive rows per LDS cycle: even and odd rows fall in
// different bank halves, and the XOR spreads each half over 8 chunk slots).
// Lane half h supplies k = 16 h + 8 f + s at step s of fragment set f
// (f = 0, 1; s = 0..7), the same permutation on both operands; set f is
// chunks 4 h + 2 f and 4 h + 2 f + 1.  Wave w loads half (w & 1) of operand
// w >> 1.
constexpr int F_BK = 32;
constexpr int F_PLANE = S_BM * F_BK;  // floats of one LDS operand plane


// FUSED: tile (tm, tn) covers modes [128 tm, 128 tm + 128) and samples
// [128 tn, 128 tn + 128) as in gemm_split_occ, and the epilogue is
// fused_epilogue.
template <bool FUSED>
__global__ __launch_bounds__(kThreads, 1) void gemm_f32_pp(const float* __restrict__ A,
                                                           const float* __restrict__ B,
                                                           float* __restrict__ C, int64_t ldm,
                                                           int64_t ncols, FusedOut fo) {
  __shared__ __attribute__((aligned(1024))) float lds[2][2][F_PLANE];
  const int tiles_m = (int)(2 * ldm / S_BM), tiles_n = (int)((ncols + S_BN - 1) / S_BN);
  int tm, tn;
  if (!tile_of_block(tiles_m, tiles_n, tm, tn)) return;
  const int64_t m0 = (int64_t)tm * (FUSED ? 128 : S_BM), n0 = (int64_t)tn * (FUSED ? 128 : S_BN);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 31, lh = lane >> 5;

  const int op = wave >> 1, half = wave & 1;
  const float* src = op == 0 ? A + m0 * ldm : B + n0 * ldm;
  // fused tiles: the second half of the rows are the Im rows (A) or the beta
  // columns (B), and sample offsets past the chunk are clamped
  const int64_t row_limit = op == 0 ? (FUSED ? 128 : S_BM) : (FUSED ? ncols / 2 - n0 : ncols - n0);
  const int64_t hi_off = op == 0 ? ldm : ncols / 2;
  const int lrow = lane >> 3;
  // lane l writes LDS slot 16 l of each 1 KB block (8 rows): row 8 q + l / 8
  // of the wave's half, slot l % 8, which holds global chunk (l % 8) ^ swz8(row)
  auto issue = [&](int st, int64_t k0) {
    char* dst = (char*)&lds[st][op][0] + half * (128 * F_BK * 4);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = half * 128 + 8 * q + lrow;
      int64_t row;
      if constexpr (FUSED) {
        const int64_t rr = 8 * q + lrow;  // row within the half
        row = (rr < row_limit ? rr : row_limit - 1) + (half ? hi_off : 0);
      } else {
        row = r < row_limit ? r : row_limit - 1;
      }
      const float* g = src + row * ldm + k0 + (((lane & 7) ^ swz8(r)) << 2);
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + q * 1024), 16, 0, 0);
    }
  };
  int oa[2][2][4], ob[2][2][4];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra = wm * 128 + i * 32 + lr, rb = wn * 128 + i * 32 + lr;
        const int c = 4 * lh + 2 * f + t;
        oa[f][t][i] = ra * F_BK + ((c ^ swz8(ra)) << 2);
        ob[f][t][i] = rb * F_BK + ((c ^ swz8(rb)) << 2);
      }
  f32x4 a0[2][4], b0[2][4], a1[2][4], b1[2][4];
  auto read0 = [&](int st) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a0[t][i] = *(const f32x4*)(&lds[st][0][oa[0][t][i]]);
        b0[t][i] = *(const f32x4*)(&lds[st][1][ob[0][t][i]]);
      }
  };
  auto read1 = [&](int st) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a1[t][i] = *(const f32x4*)(&lds[st][0][oa[1][t][i]]);
        b1[t][i] = *(const f32x4*)(&lds[st][1][ob[1][t][i]]);
      }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int KT = (int)(ldm / F_BK);  // >= 4
  issue(0, 0);
  wait_vm<0>();
  barrier_no_fence();
  issue(1, F_BK);
  read0(0);
  constexpr int kSgMfma = 0x008, kSgDsRead = 0x100, kSgVmem = 0x020;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    // phase A: set 0 (steps 0-7) with the reads of set 1 threaded between them
    read1(cur);
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[s >> 2][i][s & 3], b0[s >> 2][j][s & 3],
                                                           acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 4, 0);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 64, 0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);  // own loads of slab kt + 1 landed, reads of stage cur done
    barrier_no_fence();
    __builtin_amdgcn_sched_barrier(0);
    // phase B: set 1 (steps 8-15) with the loads of slab kt + 2 and the reads
    // of set 0 of slab kt + 1 threaded in (the last two slabs repeat the final
    // slab into the freed stage, in bounds, so the loop has no branches)
    issue(cur, (int64_t)min(kt + 2, KT - 1) * F_BK);
    read0(cur ^ 1);
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[s >> 2][i][s & 3], b1[s >> 2][j][s & 3],
                                                           acc[i][j], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 1);
      __builtin_amdgcn_sched_group_barrier(kSgVmem, 1, 1);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(kSgMfma, 4, 1);
      __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 1);
    }
    __builtin_amdgcn_sched_group_barrier(kSgMfma, 32, 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  __builtin_amdgcn_s_waitcnt(0);  // the repeated tail loads land before the wave ends
  if constexpr (FUSED) {
    // a unit scale the compiler cannot fold: with the constant 1 it kept the
    // accumulators for the stores of the beta waves in their registers and
    // spilled 41 of them around the epilogue
    float one = 1.0f;
    asm volatile("" : "+s"(one));
    fused_epilogue(acc, &lds[0][0][0], fo, m0, n0, wm, wn, lane, one);
    return;
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
            f32x4{acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]};
      }
  }
}

// ---------------------------------------------------------------- grouped

// Persistent grouped launch over many networks: one workgroup per CU walks a
// work list of (network, tile) items with stride gridDim.x; the list is
// ordered so that the items an XCD processes at the same time are
// neighbouring tiles of one network.  FUSED: each item is a tile of
// gemm_split_occ (modes [128 tm, 128 tm + 128), samples [128 tn, 128 tn + 128),
// the same tile counts as the C tiles) and writes the network's occupation
// partials (GroupNet::fo) instead of C.

template <typename H, bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split_grouped(const GroupNet* __restrict__ nets,
                                                                  const int4* __restrict__ items,
                                                                  int n_items) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds_raw[kSplitLdsElems];
  uint16_t (*lds)[4][S_PLANE] = (uint16_t (*)[4][S_PLANE])lds_raw;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    // (net, tile_m, tile_n, columns blocks per wave: 4 or 2); net < 0: idle slot
    const int4 w = items[it];
    if (w.x < 0) continue;
    const GroupNet* g = nets + w.x;
    // the thread index, opaque to the compiler on every item, so that nothing
    // derived from it is hoisted out of the item loop and held in registers
    // across the epilogue
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (w.w == 2)  // 256 x 128 tile: 128 modes x 64 samples
      split_pp_tile<H, true, PF, 2>(lds, g->A, g->B, nullptr, g->ldm, g->ncols,
                                    (int64_t)w.y * 128, (int64_t)w.z * 64, g->out_scale, &g->fo,
                                    tid);
    else
      split_pp_tile<H, true, PF, 4>(lds, g->A, g->B, nullptr, g->ldm, g->ncols,
                                    (int64_t)w.y * 128, (int64_t)w.z * 128, g->out_scale, &g->fo,
                                    tid);
    __syncthreads();  // the next item reuses the LDS stages
  }
}

// One-sided split FP16 form of the grouped launch: the same work list, every
// item a 256 x 256 tile (128 modes x 128 samples) of split1_pp_tile with the
// occupation epilogue.
template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1_grouped(const GroupNet* __restrict__ nets,
                                                                   const int4* __restrict__ items,
                                                                   int n_items) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[kSplit1LdsElems];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];  // (net, tile_m, tile_n, 4)
    if (w.x < 0) continue;
    const GroupNet* g = nets + w.x;
    int tid = threadIdx.x;  // opaque per item, as in gemm_split_grouped
    asm volatile("" : "+v"(tid));
    split1_pp_tile<true, PF>(lds, g->A, g->B, nullptr, g->ldm, g->ncols, (int64_t)w.y * 128,
                             (int64_t)w.z * 128, g->out_scale, &g->fo, tid);
    __syncthreads();  // the next item reuses the LDS stages
  }
}

// T-split form of the grouped launch (256 x 256 tiles; GroupNet::ncols holds
// the storage columns 2 E2 of the network's chunk).
template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t_grouped(const GroupNet* __restrict__ nets,
                                                                    const int4* __restrict__ items,
                                                                    int n_items) {
  __shared__ __attribute__((aligned(1024))) uint16_t lds[kSplit1LdsElems];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];  // (net, tile_m, tile_n, 4)
    if (w.x < 0) continue;
    const GroupNet* g = nets + w.x;
    int tid = threadIdx.x;  // opaque per item, as in gemm_split_grouped
    asm volatile("" : "+v"(tid));
    split1t_pp_tile<true, PF, kSplit1tPfA>(lds, g->A, g->B, nullptr, g->ldm, g->ncols, 0,
                                           (int64_t)w.y * 128, (int64_t)w.z * 128, g->out_scale,
                                           &g->fo, tid);
    __syncthreads();  // the next item reuses the LDS stages
  }
}

// Grouped form of the T-split kernel with the FP8 correction (the FP8 parts
// follow the FP16 parts of each network's operands, as in gemm_split1t8_occ).
template <bool PF>
__global__ __launch_bounds__(kThreads, 1) void gemm_split1t8_grouped(const GroupNet* __restrict__ nets,
                                                                     const int4* __restrict__ items,
                                                                     int n_items) {
  __shared__ __attribute__((aligned(1024))) char lds[F8_LDS];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];  // (net, tile_m, tile_n, 4)
    if (w.x < 0) continue;
    const GroupNet* g = nets + w.x;
    int tid = threadIdx.x;  // opaque per item, as in gemm_split_grouped
    asm volatile("" : "+v"(tid));
    const uint8_t* A8 = (const uint8_t*)g->A + 4 * g->ldm * g->ldm;
    const uint8_t* B8 = (const uint8_t*)g->B + 2 * g->ncols * g->ldm;
    split1t8_pp_tile<1, PF>(lds, g->A, A8, g->B, B8, nullptr, g->ldm, g->ncols, 0,
                               (int64_t)w.y * 128, (int64_t)w.z * 128, g->out_scale,
                               g->f8_scale_a, &g->fo, tid);
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
    case MP_SPLIT1_FP16: return elems * 2;  // one FP16 value per entry
    case MP_SPLIT1T_F8: return elems * 3;   // FP16 value, then the e4m3 remainder
    default: return elems * 4;  // hi and lo 16-bit values
  }
}

static int grid_tiles(int64_t ldm, int64_t ncols, int bm, int bn) {
  return mall_grid_blocks((int)(2 * ldm / bm), (int)((ncols + bn - 1) / bn));
}
static int grid_tiles_s1t(int64_t ldm, int64_t ncols) {
  return mall_grid_blocks<kS1tStepRows, kS1tStepCols>((int)(2 * ldm / S_BM),
                                                       (int)((ncols + S_BN - 1) / S_BN));
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
  return (prec == MP_SPLIT_FP16 || prec == MP_SPLIT1_FP16 || prec == MP_SPLIT1T_FP16 ||
          prec == MP_SPLIT1T_F8)
             ? fp16_scale_exp(M)
             : 0;
}

// Block scale (E8M0, 2^(s - 127)) of the FP8 product's A operand: undoes the
// e4m3 remainder's scale 2^e4m3_lo_scale_exp.
int f8_scale_a(int32_t M) { return 127 - e4m3_lo_scale_exp(fp16_scale_exp(M)); }

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
    case MP_SPLIT1T_FP16:  // the same hi/lo packing
      hipLaunchKernelGGL(pack_transmission<MP_SPLIT_FP16>, dim3(blocks), dim3(256), 0, stream, T,
                         M, ldm, packed, fp16_scale_exp(M));
      break;
    case MP_SPLIT1_FP16:
      hipLaunchKernelGGL(pack_transmission<MP_SPLIT1_FP16>, dim3(blocks), dim3(256), 0, stream, T,
                         M, ldm, packed, fp16_scale_exp(M));
      break;
    case MP_SPLIT1T_F8:
      hipLaunchKernelGGL(pack_transmission<MP_SPLIT1T_F8>, dim3(blocks), dim3(256), 0, stream, T,
                         M, ldm, packed, fp16_scale_exp(M));
      break;
    default:
      set_error("transmission pack: unknown precision %d", (int)prec);
      return MP_ERR_ARG;
  }
  MP_HIP_LAUNCH_CHECK("transmission pack launch");
  return MP_OK;
}

// GEMM on an already packed operand (one network).
template <typename H>
static void split_gemm(int grid, hipStream_t stream, const void* packed, const void* ab, void* C,
                       int64_t ldm, int64_t ncols, float scale) {
  auto kernel = split_prefetch_for(ldm) ? gemm_split_256_pp<H, true> : gemm_split_256_pp<H, false>;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), 0, stream, (const uint16_t*)packed,
                     (const uint16_t*)ab, (float*)C, ldm, ncols, scale);
}

bool split_prefetch(int64_t ldm) { return split_prefetch_for(ldm); }

mp_status gemm_packed_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                             const void* ab, void* C, hipStream_t stream) {
  const int64_t ldm = ld_modes(M), ncols = 2 * E;
  switch (prec) {
    case MP_FP64:
      hipLaunchKernelGGL(gemm_f64_pp, dim3(grid_tiles(ldm, ncols, D_BM, D_BN)), dim3(kThreads), 0,
                         stream, (const double*)packed, (const double*)ab, (double*)C, ldm, ncols);
      break;
    case MP_FP32:
      hipLaunchKernelGGL(gemm_f32_pp<false>, dim3(grid_tiles(ldm, ncols, S_BM, S_BN)),
                         dim3(kThreads), 0, stream, (const float*)packed, (const float*)ab,
                         (float*)C, ldm, ncols, FusedOut{});
      break;
    case MP_SPLIT_BF16:
      split_gemm<__bf16>(grid_tiles(ldm, ncols, S_BM, S_BN), stream, packed, ab, C, ldm, ncols,
                         1.0f);
      break;
    case MP_SPLIT_FP16:
      split_gemm<_Float16>(grid_tiles(ldm, ncols, S_BM, S_BN), stream, packed, ab, C, ldm, ncols,
                           ldexpf(1.0f, -fp16_scale_exp(M)));
      break;
    case MP_SPLIT1_FP16: {
      auto kernel = split_prefetch_for(ldm) ? gemm_split1_pp<true> : gemm_split1_pp<false>;
      hipLaunchKernelGGL(kernel, dim3(grid_tiles(ldm, ncols, S_BM, S_BN)), dim3(kThreads), 0,
                         stream, (const uint16_t*)packed, (const uint16_t*)ab, (float*)C, ldm,
                         ncols, ldexpf(1.0f, -fp16_scale_exp(M)));
      break;
    }
    case MP_SPLIT1T_FP16: {
      // tiles over the storage columns (2 E2), stored to C columns
      const int64_t scols = 2 * split1t_half(E);
      auto kernel = split_prefetch_for(ldm) ? gemm_split1t_pp<true> : gemm_split1t_pp<false>;
      hipLaunchKernelGGL(kernel, dim3(grid_tiles_s1t(ldm, scols)), dim3(kThreads), 0, stream,
                         (const uint16_t*)packed, (const uint16_t*)ab, (float*)C, ldm, scols, E,
                         ldexpf(1.0f, -fp16_scale_exp(M)));
      break;
    }
    case MP_SPLIT1T_F8: {
      const int64_t scols = 2 * split1t_half(E);
      auto kernel = split_prefetch_for(ldm) ? gemm_split1t8_pp<true> : gemm_split1t8_pp<false>;
      hipLaunchKernelGGL(kernel, dim3(grid_tiles_s1t(ldm, scols)), dim3(kThreads), 0, stream,
                         (const uint16_t*)packed, (const uint16_t*)ab, (float*)C, ldm, scols, E,
                         ldexpf(1.0f, -fp16_scale_exp(M)), f8_scale_a(M));
      break;
    }
    default:
      set_error("mp_propagate: unknown precision %d", (int)prec);
      return MP_ERR_ARG;
  }
  MP_HIP_LAUNCH_CHECK("mp_propagate gemm launch");
  return MP_OK;
}

template <typename H>
static auto grouped_kernel(bool prefetch) {
  return prefetch ? gemm_split_grouped<H, true> : gemm_split_grouped<H, false>;
}

mp_status grouped_launch(const GroupNet* d_nets, const int4* d_items, int n_items, int grid,
                         mp_precision prec, bool prefetch, hipStream_t stream) {
  if (prec == MP_SPLIT_BF16) {
    hipLaunchKernelGGL(grouped_kernel<__bf16>(prefetch), dim3(grid), dim3(kThreads), 0, stream,
                       d_nets, d_items, n_items);
  } else if (prec == MP_SPLIT_FP16) {
    hipLaunchKernelGGL(grouped_kernel<_Float16>(prefetch), dim3(grid), dim3(kThreads), 0, stream,
                       d_nets, d_items, n_items);
  } else if (prec == MP_SPLIT1_FP16) {
    hipLaunchKernelGGL(prefetch ? gemm_split1_grouped<true> : gemm_split1_grouped<false>,
                       dim3(grid), dim3(kThreads), 0, stream, d_nets, d_items, n_items);
  } else if (prec == MP_SPLIT1T_FP16) {
    hipLaunchKernelGGL(prefetch ? gemm_split1t_grouped<true> : gemm_split1t_grouped<false>,
                       dim3(grid), dim3(kThreads), 0, stream, d_nets, d_items, n_items);
  } else if (prec == MP_SPLIT1T_F8) {
    hipLaunchKernelGGL(prefetch ? gemm_split1t8_grouped<true> : gemm_split1t8_grouped<false>,
                       dim3(grid), dim3(kThreads), 0, stream, d_nets, d_items, n_items);
  } else {
    set_error("grouped GEMM: the split precisions only");
    return MP_ERR_UNSUPPORTED;
  }
  MP_HIP_LAUNCH_CHECK("plan grouped gemm launch");
  return MP_OK;
}

// GEMM with the occupation-fused epilogue on an already packed operand.
mp_status gemm_fused_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                            const void* ab, const FusedOut& fo, hipStream_t stream) {
  const int64_t ldm = ld_modes(M), ncols = 2 * E;
  const int grid = grid_tiles(ldm, ncols, S_BM, S_BN);
  switch (prec) {
    case MP_FP32:
      hipLaunchKernelGGL(gemm_f32_pp<true>, dim3(grid), dim3(kThreads), 0, stream,
                         (const float*)packed, (const float*)ab, (float*)nullptr, ldm, ncols, fo);
      break;
    case MP_SPLIT_BF16: {
      auto kernel = split_prefetch_for(ldm) ? gemm_split_occ<__bf16, true> : gemm_split_occ<__bf16, false>;
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), 0, stream, (const uint16_t*)packed,
                         (const uint16_t*)ab, ldm, ncols, 1.0f, fo);
      break;
    }
    case MP_SPLIT_FP16: {
      auto kernel =
          split_prefetch_for(ldm) ? gemm_split_occ<_Float16, true> : gemm_split_occ<_Float16, false>;
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), 0, stream, (const uint16_t*)packed,
                         (const uint16_t*)ab, ldm, ncols, ldexpf(1.0f, -fp16_scale_exp(M)), fo);
      break;
    }
    case MP_SPLIT1_FP16: {
      auto kernel = split_prefetch_for(ldm) ? gemm_split1_occ<true> : gemm_split1_occ<false>;
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), 0, stream, (const uint16_t*)packed,
                         (const uint16_t*)ab, ldm, ncols, ldexpf(1.0f, -fp16_scale_exp(M)), fo);
      break;
    }
    case MP_SPLIT1T_FP16: {
      const int64_t scols = 2 * split1t_half(E);  // storage columns, beta from E2 on
      auto kernel = split_prefetch_for(ldm) ? gemm_split1t_occ<true> : gemm_split1t_occ<false>;
      hipLaunchKernelGGL(kernel, dim3(grid_tiles_s1t(ldm, scols)), dim3(kThreads), 0, stream,
                         (const uint16_t*)packed, (const uint16_t*)ab, ldm, scols,
                         ldexpf(1.0f, -fp16_scale_exp(M)), fo);
      break;
    }
    case MP_SPLIT1T_F8: {
      const int64_t scols = 2 * split1t_half(E);
      auto kernel = split_prefetch_for(ldm) ? gemm_split1t8_occ<true> : gemm_split1t8_occ<false>;
      hipLaunchKernelGGL(kernel, dim3(grid_tiles_s1t(ldm, scols)), dim3(kThreads), 0, stream,
                         (const uint16_t*)packed, (const uint16_t*)ab, ldm, scols,
                         ldexpf(1.0f, -fp16_scale_exp(M)), f8_scale_a(M), fo);
      break;
    }
    default:
      set_error("mp_propagate_counts: the fused path supports FP32 and the split precisions");
      return MP_ERR_UNSUPPORTED;
  }
  MP_HIP_LAUNCH_CHECK("mp_propagate_counts fused gemm launch");
  return MP_OK;
}

// Scratch of bilinear_pack_launch: T^T, the FP64 sample operand X (E = M),
// T^T packed in FP64, C (2 ldm x 2 M), W, the device copy of the mode set.
static int64_t round256(int64_t x) { return (x + 255) / 256 * 256; }
size_t bilinear_workspace(int32_t M) {
  const int64_t ldm = ld_modes(M), m2 = (int64_t)M * M;
  return (size_t)(round256(16 * m2) + round256(8 * ldm * 2 * M) +
                  round256((int64_t)propagate_workspace(M, MP_FP64)) +
                  round256(8 * 2 * ldm * 2 * M) + round256(16 * m2) + round256(4 * (int64_t)M));
}

// Bytes of the packed bilinear operand: W's off-diagonal part packed as `prec`
// packs T, then D (ldm FP32 values).
size_t bilinear_packed_bytes(int32_t M, mp_precision prec) {
  return propagate_workspace(M, prec) + (size_t)round256(4 * ld_modes(M));
}

// Packs W = T^T P_S T* (S: modes with in_s[j] >= 0; in_s on the host): its
// off-diagonal part as `prec` packs T, its diagonal in FP32 after it.  W comes
// from the FP64 GEMM, so the packed form carries only the packing's rounding.
mp_status bilinear_pack_launch(int32_t M, const double* T, const int32_t* in_s,
                               mp_precision prec, void* packed, void* scratch,
                               hipStream_t stream) {
  const int64_t ldm = ld_modes(M), m2 = (int64_t)M * M;
  char* p = (char*)scratch;
  double* Tt = (double*)p;
  p += round256(16 * m2);
  double* X = (double*)p;
  p += round256(8 * ldm * 2 * M);
  void* packed64 = p;
  p += round256((int64_t)propagate_workspace(M, MP_FP64));
  double* C = (double*)p;
  p += round256(8 * 2 * ldm * 2 * M);
  double* W = (double*)p;
  p += round256(16 * m2);
  int32_t* mask = (int32_t*)p;
  hipError_t e = hipMemcpyAsync(mask, in_s, 4 * (size_t)M, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) {
    set_error("mp_pack_bilinear: copy of the mode set: %s", hipGetErrorString(e));
    return MP_ERR_HIP;
  }
  hipLaunchKernelGGL(bilin_transpose, dim3((unsigned)((m2 + 255) / 256)), dim3(256), 0, stream, T,
                     M, Tt);
  hipLaunchKernelGGL(bilin_columns, dim3((unsigned)((M * ldm + 255) / 256)), dim3(256), 0, stream,
                     T, M, ldm, (const int32_t*)mask, X);
  MP_HIP_LAUNCH_CHECK("mp_pack_bilinear setup launch");
  mp_status st = pack_launch(M, Tt, MP_FP64, packed64, stream);
  if (st != MP_OK) return st;
  if ((st = gemm_packed_launch(M, M, packed64, MP_FP64, X, C, stream)) != MP_OK) return st;
  hipLaunchKernelGGL(bilin_combine, dim3((unsigned)((m2 + 255) / 256)), dim3(256), 0, stream, C, M,
                     ldm, W);
  hipLaunchKernelGGL(bilin_diag, dim3((unsigned)((ldm + 255) / 256)), dim3(256), 0, stream, C, M,
                     ldm, (float*)((char*)packed + propagate_workspace(M, prec)));
  MP_HIP_LAUNCH_CHECK("mp_pack_bilinear combine launch");
  return pack_launch(M, W, prec, packed, stream);
}

// The bilinear-form GEMM with its epilogue (one run of all modes in fo).
mp_status gemm_bilinear_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                               const void* ab, const FusedOut& fo, hipStream_t stream) {
  if (prec != MP_SPLIT1T_F8) {
    set_error("mp_propagate_counts_bilinear: precision %d (MP_SPLIT1T_F8 only)", (int)prec);
    return MP_ERR_UNSUPPORTED;
  }
  const int64_t ldm = ld_modes(M), e2 = split1t_half(E);
  const uint16_t* alpha = (const uint16_t*)ab;
  const uint16_t* B = alpha + e2 * ldm;                              // beta: storage columns E2 ..
  const uint8_t* B8 = (const uint8_t*)ab + 4 * e2 * ldm + e2 * ldm;  // their e4m3 copies
  auto kernel = split_prefetch_for(ldm) ? gemm_split1t8_bilin<true> : gemm_split1t8_bilin<false>;
  const float* diag = (const float*)((const char*)packed + propagate_workspace(M, prec));
  hipLaunchKernelGGL(kernel, dim3(grid_tiles_s1t(ldm, e2)), dim3(kThreads), 0, stream,
                     (const uint16_t*)packed, B, B8, alpha, diag, ldm, e2,
                     ldexpf(1.0f, -fp16_scale_exp(M)), f8_scale_a(M), fo);
  MP_HIP_LAUNCH_CHECK("mp_propagate_counts_bilinear gemm launch");
  return MP_OK;
}

mp_status propagate_launch(int32_t M, int64_t E, const double* T, mp_precision prec,
                           const void* ab, void* C, void* ws, hipStream_t stream) {
  const mp_status st = pack_launch(M, T, prec, ws, stream);
  if (st != MP_OK) return st;
  return gemm_packed_launch(M, E, ws, prec, ab, C, stream);
}

}  // namespace mp
