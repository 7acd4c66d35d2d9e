// Normally ordered pair moments <:n_i n_j:> of single output modes (main
// text, eq. moment, with every output mode its own group): the mixed second
// derivative of the per-sample generating function at z = 1 is n'_i n'_j,
// with weight 1 (even order) for the parity-projected and the +P estimator.
// Per sub-ensemble s the sum over its samples k of n'_ik n'_jk is the complex
// symmetric product X_s X_s^T of the occupation matrix X (modes x samples).
//
//   mode_occupations_kernel  X from the propagated amplitudes C (planar: the
//                            real parts of sample k in column k, the
//                            imaginary parts in column E + k, ldm modes each)
//   pair_corr_f32            FP32 MFMA (three real products per complex
//                            one), 128 x 128 complex tiles of the upper
//                            block triangle, FP32 sums over the chunk's
//                            samples of one sub-ensemble (or of one piece of
//                            them), added into FP64
//   pair_reduce              when a launch has few (tile, sub-ensemble) items,
//                            each is split into pieces of samples that write
//                            FP32 partial tiles; this adds the pieces in
//                            order into the FP64 accumulator
//   pair_corr_f64            FP64 FMA twin (64 x 64 tiles) for the FP64 path
//
// The accumulator is the full matrix, [s][i][j] (re, im): a tile off the
// diagonal adds its block and the transposed block.  Every (sub-ensemble,
// tile) pair has one writer per launch (its workgroup, or pair_reduce over
// its pieces in a fixed order), so the result does not depend on scheduling.
#include "cmfma.h"
#include "common.h"

namespace mp {

namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
using cmfma::f32x16;
typedef __attribute__((ext_vector_type(4))) double f64x4;

template <typename CT> struct Vec4;
template <> struct Vec4<float> { typedef f32x4 t; };
template <> struct Vec4<double> { typedef f64x4 t; };

// n'_ik = alpha'_ik beta'_ik = (a c + b e) + i (b c - a e) with a, b = Re, Im
// alpha' (column k of C) and c, e = Re beta', -Im beta' (column E + k).  One
// thread per four modes of one sample.
template <typename CT>
__global__ __launch_bounds__(256) void mode_occupations_kernel(int64_t ldm, int64_t E,
                                                               const CT* __restrict__ C,
                                                               CT* __restrict__ X) {
  typedef typename Vec4<CT>::t V;
  const int64_t quads = ldm / 4;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= quads * E) return;
  const int64_t k = idx / quads, i = (idx - k * quads) * 4;
  const int64_t ldc = 2 * ldm;
  const V a = *(const V*)(C + k * ldc + i);
  const V b = *(const V*)(C + k * ldc + ldm + i);
  const V c = *(const V*)(C + (E + k) * ldc + i);
  const V e = *(const V*)(C + (E + k) * ldc + ldm + i);
  *(V*)(X + k * ldm + i) = a * c + b * e;
  *(V*)(X + (E + k) * ldm + i) = b * c - a * e;
}

struct PairParams {
  int64_t M, ldm, E, e0, ns, s_first;
  int nb;           // mode blocks per side (ldm / tile)
  int n_pairs;      // nb (nb + 1) / 2
  int pieces;       // sample pieces per (tile, sub-ensemble) item
  int64_t piece;    // samples per piece (a multiple of the slab)
  float* part;      // pieces > 1: partial tiles [item][piece][128 x 128][re, im]
};

// Row-major enumeration of the upper block triangle: (0,0), (0,1), ...
__device__ inline void pair_of_index(int q, int nb, int& I, int& J) {
  int i = 0;
  while (q >= nb - i) {
    q -= nb - i;
    ++i;
  }
  I = i;
  J = i + q;
}

// Workgroup -> (sub-ensemble, piece, tile pair) and the chunk-local sample
// range [k0, k1) of that piece of the sub-ensemble (empty for pieces past a
// short sub-ensemble's end).
__device__ inline void pair_item(const PairParams& p, int& I, int& J, int64_t& s, int& pc,
                                 int64_t& k0, int64_t& k1) {
  const int q = (int)(blockIdx.x % (unsigned)p.n_pairs);
  const int64_t rest = blockIdx.x / (unsigned)p.n_pairs;
  pc = (int)(rest % p.pieces);
  s = p.s_first + rest / p.pieces;
  pair_of_index(q, p.nb, I, J);
  const int64_t lo = s * p.ns - p.e0, hi = (s + 1) * p.ns - p.e0;
  const int64_t a = (lo > 0 ? lo : 0) + pc * p.piece;
  const int64_t b = hi < p.E ? hi : p.E;
  k0 = a;
  k1 = a + p.piece < b ? a + p.piece : b;
}

// Partial tile of (sub-ensemble s, tile pair q, piece pc).
__device__ inline float* part_tile(const PairParams& p, int64_t s, int q, int pc) {
  return p.part + (((s - p.s_first) * p.n_pairs + q) * p.pieces + pc) * (int64_t)(2 * 128 * 128);
}

// Adds one complex value into element (i, j) of sub-ensemble s, and into
// (j, i) when the tile is off the diagonal.
__device__ inline void pair_add(const PairParams& p, double* __restrict__ acc, int64_t s,
                                int64_t i, int64_t j, bool mirror, double re, double im) {
  if (i >= p.M || j >= p.M) return;
  double* o = acc + 2 * ((s * p.M + i) * p.M + j);
  o[0] += re;
  o[1] += im;
  if (mirror) {
    double* t = acc + 2 * ((s * p.M + j) * p.M + i);
    t[0] += re;
    t[1] += im;
  }
}

// ---------------------------------------------------------------- FP32 MFMA

constexpr int PT = 128;  // modes per tile side
constexpr int PK = 32;   // samples per slab
static_assert(PT == cmfma::kTile && PK == cmfma::kSlab, "tile shape of the shared MFMA core");

// v_mfma_f32_32x32x2f32 with A[i][k] = X[I block row i][sample k] and
// B[k][j] = X[J block row j][sample k]: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32], so both fragments are one LDS float per lane from a
// slab stored as [sample][mode].  Output register r of lane l is element
// (8 (r / 4) + 4 (l / 32) + r % 4, l % 32).  Wave (wi, wj) owns rows
// [64 wi, 64 wi + 64) and columns [64 wj, 64 wj + 64) of the complex tile,
// with three real products per fragment pair instead of four:
//   P1 = Xr_I Xr_J^T,  P2 = Xi_I Xi_J^T,  P3 = (Xr + Xi)_I (Xr + Xi)_J^T,
//   Re = P1 - P2,      Im = P3 - P1 - P2.
// 25 % fewer MFMAs; the third accumulator set leaves one workgroup per CU
// (measured at M = 1000: 3.53 ms per chunk against 3.88 ms for the four-
// product form at two workgroups per CU).  The FP32 sums then carry rounding
// of up to 4 K u sum |n'_i||n'_j| in Im (P3 sums (|Re| + |Im|) products)
// instead of 2 K u.  The next slab is loaded into registers while the
// current one is multiplied; samples past the sub-ensemble's range are
// loaded as zeros.
__global__ __launch_bounds__(256, 1) void pair_corr_f32(PairParams p, const float* __restrict__ X,
                                                       double* __restrict__ acc) {
  __shared__ __attribute__((aligned(16))) float lds[4][PK][PT];  // Re I, Im I, Re J, Im J
  int I, J, pc;
  int64_t s, k0, k1;
  pair_item(p, I, J, s, pc, k0, k1);
  const bool diag = I == J;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1;

  // loader: four consecutive modes of rows lrow + 8 u (u < 4) of each plane
  const int lc = (tid & 31) * 4, lrow = tid >> 5;
  const int64_t im_off = p.E * p.ldm;
  const float* src[4] = {X + I * PT + lc, X + im_off + I * PT + lc, X + J * PT + lc,
                         X + im_off + J * PT + lc};
  const int nplanes = diag ? 2 : 4;
  f32x4 st[4][4];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      if (pl < nplanes)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t k = kb + lrow + 8 * u;
          st[pl][u] = k < k1 ? *(const f32x4*)(src[pl] + k * p.ldm) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
  };
  const float* bre = diag ? &lds[0][0][0] : &lds[2][0][0];
  const float* bim = diag ? &lds[1][0][0] : &lds[3][0][0];

  // P1 = Xr Xr^T, P2 = Xi Xi^T, P3 = (Xr + Xi)(Xr + Xi)^T (in accR, accI, acc3)
  f32x16 accR[2][2], accI[2][2], acc3[2][2];
  cmfma::zero(accR, accI);
  cmfma::zero(acc3, acc3);

  load(k0);
  for (int64_t kb = k0; kb < k1; kb += PK) {
    __syncthreads();  // every wave is done with the previous slab
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      if (pl < nplanes)
#pragma unroll
        for (int u = 0; u < 4; ++u) *(f32x4*)&lds[pl][lrow + 8 * u][lc] = st[pl][u];
    __syncthreads();
    if (kb + PK < k1) load(kb + PK);
    cmfma::slab3(&lds[0][0][0], &lds[1][0][0], bre, bim, wi, wj, lane, accR, accI, acc3);
  }
  // Re = P1 - P2, Im = P3 - P1 - P2
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float p1 = accR[a][b][r], p2 = accI[a][b][r];
        accR[a][b][r] = p1 - p2;
        accI[a][b][r] = acc3[a][b][r] - p1 - p2;
      }

  if (p.pieces > 1) {
    // partial tile, element (row, col) at 2 (128 row + col)
    float* t = part_tile(p, s, (int)(blockIdx.x % (unsigned)p.n_pairs), pc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = cmfma::out_row(wi, a, r, lane);
          const int col = cmfma::out_col(wj, b, lane);
          typedef __attribute__((ext_vector_type(2))) float f32x2;
          *(f32x2*)(t + 2 * (row * PT + col)) = f32x2{accR[a][b][r], accI[a][b][r]};
        }
    return;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gi = (int64_t)I * PT + cmfma::out_row(wi, a, r, lane);
        const int64_t gj = (int64_t)J * PT + cmfma::out_col(wj, b, lane);
        pair_add(p, acc, s, gi, gj, !diag, accR[a][b][r], accI[a][b][r]);
      }
}

// Sum of the pieces of each (sub-ensemble, tile pair) item in piece order
// (FP64), added into the accumulator like pair_corr_f32's direct epilogue.
// One thread per tile element; grid (items, 128 x 128 / 256).
__global__ __launch_bounds__(256) void pair_reduce(PairParams p, double* __restrict__ acc) {
  const int q = (int)(blockIdx.x % (unsigned)p.n_pairs);
  const int64_t s = p.s_first + blockIdx.x / (unsigned)p.n_pairs;
  const int e = blockIdx.y * 256 + threadIdx.x;  // row * 128 + col
  int I, J;
  pair_of_index(q, p.nb, I, J);
  double re = 0.0, im = 0.0;
  for (int pc = 0; pc < p.pieces; ++pc) {
    const float* t = part_tile(p, s, q, pc);
    re += (double)t[2 * e];
    im += (double)t[2 * e + 1];
  }
  pair_add(p, acc, s, (int64_t)I * PT + e / PT, (int64_t)J * PT + e % PT, I != J, re, im);
}

// ---------------------------------------------------------------- FP64

constexpr int QT = 64;  // modes per tile side
constexpr int QK = 16;  // samples per slab

// Thread (ty, tx) = (tid / 16, tid % 16) owns rows ty + 16 u and columns
// tx + 16 v (u, v < 4) of a 64 x 64 complex tile; FMAs in the order
// Re += xr_i xr_j, Re -= xi_i xi_j, Im += xr_i xi_j, Im += xi_i xr_j per
// sample.
__global__ __launch_bounds__(256) void pair_corr_f64(PairParams p, const double* __restrict__ X,
                                                    double* __restrict__ acc) {
  __shared__ __attribute__((aligned(32))) double lds[4][QK][QT];
  int I, J, pc;
  int64_t s, k0, k1;
  pair_item(p, I, J, s, pc, k0, k1);
  const bool diag = I == J;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const int lc = (tid & 15) * 4, lrow = tid >> 4;
  const int64_t im_off = p.E * p.ldm;
  const double* src[4] = {X + I * QT + lc, X + im_off + I * QT + lc, X + J * QT + lc,
                          X + im_off + J * QT + lc};
  const int nplanes = diag ? 2 : 4;
  const double* bre = diag ? &lds[0][0][0] : &lds[2][0][0];
  const double* bim = diag ? &lds[1][0][0] : &lds[3][0][0];
  double re[4][4], im[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) re[u][v] = im[u][v] = 0.0;

  for (int64_t kb = k0; kb < k1; kb += QK) {
    __syncthreads();
    const int64_t k = kb + lrow;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      if (pl < nplanes)
        *(f64x4*)&lds[pl][lrow][lc] =
            k < k1 ? *(const f64x4*)(src[pl] + k * p.ldm) : f64x4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    for (int kk = 0; kk < QK; ++kk) {
      double xr[4], xi[4], yr[4], yi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xr[u] = lds[0][kk][ty + 16 * u];
        xi[u] = lds[1][kk][ty + 16 * u];
        yr[u] = bre[kk * QT + tx + 16 * u];
        yi[u] = bim[kk * QT + tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          re[u][v] = fma(xr[u], yr[v], re[u][v]);
          re[u][v] = fma(-xi[u], yi[v], re[u][v]);
          im[u][v] = fma(xr[u], yi[v], im[u][v]);
          im[u][v] = fma(xi[u], yr[v], im[u][v]);
        }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      pair_add(p, acc, s, (int64_t)I * QT + ty + 16 * u, (int64_t)J * QT + tx + 16 * v, !diag,
               re[u][v], im[u][v]);
}

}  // namespace

size_t mode_occupations_bytes(int32_t M, int64_t E, mp_precision prec) {
  return (size_t)(2 * E * ld_modes(M)) * elem_bytes_c(prec);
}

mp_status mode_occupations_launch(int32_t M, int64_t E, const void* C, mp_precision prec, void* X,
                                  hipStream_t stream) {
  const int64_t ldm = ld_modes(M);
  const int64_t blocks = (ldm / 4 * E + 255) / 256;
  if (prec == MP_FP64)
    hipLaunchKernelGGL(mode_occupations_kernel<double>, dim3((unsigned)blocks), dim3(256), 0,
                       stream, ldm, E, (const double*)C, (double*)X);
  else
    hipLaunchKernelGGL(mode_occupations_kernel<float>, dim3((unsigned)blocks), dim3(256), 0,
                       stream, ldm, E, (const float*)C, (float*)X);
  MP_HIP_LAUNCH_CHECK("mp_mode_occupations launch");
  return MP_OK;
}

// Launch shape: (tile, sub-ensemble) items, split into sample pieces when
// there are too few of them to keep every CU busy to the end (FP32 only).
static PairParams pair_plan(int32_t M, int64_t E, mp_precision prec, int64_t ns, int64_t e0) {
  PairParams p{};
  p.M = M;
  p.ldm = ld_modes(M);
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  p.s_first = e0 / ns;
  p.nb = (int)(p.ldm / (prec == MP_FP64 ? QT : PT));
  p.n_pairs = p.nb * (p.nb + 1) / 2;
  const int64_t n_touched = (e0 + E - 1) / ns - p.s_first + 1;
  const int64_t items = n_touched * p.n_pairs;
  const int64_t seg = ns < E ? ns : E;  // longest piece of a sub-ensemble in this chunk
  p.pieces = 1;
  p.piece = seg;
  constexpr int64_t kTargetItems = 2048, kMaxPieces = 8, kMinPiece = 2 * PK;
  if (prec != MP_FP64 && items < kTargetItems) {
    int64_t pcs = (kTargetItems + items - 1) / items;
    pcs = pcs < kMaxPieces ? pcs : kMaxPieces;
    const int64_t by_len = seg / kMinPiece;
    pcs = pcs < by_len ? pcs : by_len;
    if (pcs > 1) {
      p.pieces = (int)pcs;
      p.piece = ((seg + pcs - 1) / pcs + PK - 1) / PK * PK;
    }
  }
  return p;
}

size_t pair_corr_workspace(int32_t M, int64_t E, mp_precision prec, int64_t ns, int64_t e0) {
  const PairParams p = pair_plan(M, E, prec, ns, e0);
  if (p.pieces == 1) return 0;
  const int64_t n_touched = (e0 + E - 1) / ns - p.s_first + 1;
  return (size_t)(n_touched * p.n_pairs * p.pieces) * (2 * PT * PT) * sizeof(float);
}

mp_status pair_corr_launch(int32_t M, int64_t E, const void* X, mp_precision prec, int64_t ns,
                           int64_t e0, double* acc, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
  PairParams p = pair_plan(M, E, prec, ns, e0);
  const size_t need = pair_corr_workspace(M, E, prec, ns, e0);
  if (need > 0 && (!ws || ws_bytes < need)) {
    set_error("mp_pair_correlations_accumulate: workspace of %zu bytes needed, %zu given", need,
              ws_bytes);
    return MP_ERR_WORKSPACE;
  }
  p.part = (float*)ws;
  const int64_t n_touched = (e0 + E - 1) / ns - p.s_first + 1;
  const int64_t blocks = n_touched * p.n_pairs * p.pieces;
  if (blocks > 0x7fffffff) {
    set_error("mp_pair_correlations_accumulate: %lld workgroups exceed the grid limit",
              (long long)blocks);
    return MP_ERR_UNSUPPORTED;
  }
  if (prec == MP_FP64) {
    hipLaunchKernelGGL(pair_corr_f64, dim3((unsigned)blocks), dim3(256), 0, stream, p,
                       (const double*)X, acc);
  } else {
    hipLaunchKernelGGL(pair_corr_f32, dim3((unsigned)blocks), dim3(256), 0, stream, p,
                       (const float*)X, acc);
    if (p.pieces > 1)
      hipLaunchKernelGGL(pair_reduce, dim3((unsigned)(n_touched * p.n_pairs), PT * PT / 256),
                         dim3(256), 0, stream, p, acc);
  }
  MP_HIP_LAUNCH_CHECK("mp_pair_correlations_accumulate launch");
  return MP_OK;
}

}  // namespace mp
