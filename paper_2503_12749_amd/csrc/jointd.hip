// Joint distribution of d = 3 or 4 bin counts (main text, higher-dimensional
// binning; eq. General_GCP with the projector of eq. projection_op), and the
// inverse DFT of every joint grid (d = 2 included).
//
// Per sample the generating function on the grid theta_b = 2 pi k_b / K_b is
//   chi(theta) = cosh(n + sum_b X_b) / cosh(n),   X_b = n_b (e^{i theta_b} - 1)
//              = e^{c1} prod_b e^{X_b} + e^{c2} prod_b e^{-X_b},
// with c1 = -log(1 + e^{-2n}) and c2 = -2n - log(1 + e^{-2n}) (written for
// either sign of n as in the one-distribution path): two rank-1 tensors over
// the d bins.  The first is below e^kLogEps for every sample of a chunk
// outside a box around theta = 0, the second outside a box around theta =
// pi; each box half-width is the chunk's maximum of the samples' exact
// per-axis bounds.  Inside a box the sum of a term over a sub-ensemble's
// samples is a complex contraction over samples,
//   S[(k_1 .. k_{d-1}), k_d] = sum_s A_s[(k_1 .. k_{d-1})] B_s[k_d],
//   A_s = prod_{b<d} f_{s,b}(k_b),   B_s = f_{s,d}(k_d),
// from per-sample factor tables f: e^{+-X_b} times e^{-i theta_b m_lo_b} (the
// window shift), the second term's factors scaled by e^{-2 Re n_b}, and the
// term's constant shared equally by the d factors so that every factor stays
// within the FP32 range.  The contraction runs on the FP32 matrix cores for
// the FP32 and split paths and with FP64 FMAs for the FP64 path.
//
// Kernels per chunk: jointd_occupations (n_b, c1, c2 per sample),
// record_bands (the box half-widths), jointd_factors (the tables of both terms inside their boxes),
// jointd_sum_f32 / jointd_sum_f64 (acc[s][k_1]..[k_d] += S, one launch per
// term, so each accumulator element has one writer per launch).  Finalize:
// the d-dimensional inverse DFT one axis at a time over the nonzero entries
// of each line, per sub-ensemble, folded into the mean and sigma_T with
// Welford's update.
#include <hip/hip_runtime.h>

#include "chi.h"
#include "cmfma.h"
#include "common.h"

namespace mp {

namespace {

constexpr int kJD = 4;  // largest d of this path
constexpr int kAxisMaxK = 4096;  // longest line of the inverse DFT (two-bin windows)

typedef __attribute__((ext_vector_type(4))) float f32x4;
using cmfma::f32x16;

struct JointDParams {
  int M;
  int64_t ldm, E, e0, ns;
  int est, d;
  int n_runs;
  int run_lo[MP_MAX_RUNS], run_hi[MP_MAX_RUNS], run_bin[MP_MAX_RUNS];
  int m_lo[kJD], K[kJD], Kp[kJD];  // window, grid, factor-table row stride
  int64_t s_first;
  int64_t cells;     // prod K_b
  int64_t rows_max;  // prod_{b<d-1} K_b
  int rec;           // doubles per sample record: 2 d + 2
  int64_t tab[2][kJD];  // element offset of each factor table (term, axis)
};

__global__ void band_init(int* band) {
  if (threadIdx.x < 2 * kJD) band[threadIdx.x] = -1;
}

// Per sample (one wave, lane 0 writes): the record (Re n_b, Im n_b for b < d,
// c1, c2; c2 = -inf for +P, both NaN for a sample that is not finite).
// record_bands then sets the box half-widths
// band[term * 4 + b] (atomic max; -1 = term absent).
// PART: the bin sums come from the occupation-fused GEMM's partials (slots in
// run order) instead of the propagated amplitudes C.
template <typename CT, bool PART>
__device__ inline void jointd_sample(const JointDParams& p, const CT* __restrict__ C,
                                     const float* __restrict__ part,
                                     const double* __restrict__ nglob, double* __restrict__ rec,
                                     int64_t k, int lane) {
  const int64_t ldc = 2 * p.ldm;
  const CT* ca = PART ? nullptr : C + k * ldc;
  const CT* cb = PART ? nullptr : C + (p.E + k) * ldc;
  double nr[kJD] = {0.0, 0.0, 0.0, 0.0}, ni[kJD] = {0.0, 0.0, 0.0, 0.0};
  int slot0 = 0;
  for (int q = 0; q < p.n_runs; ++q) {
    double re, im;
    if constexpr (PART) {
      const int nblk = run_blocks(p.run_lo[q], p.run_hi[q]);
      run_sum_partials(part, p.E, slot0, nblk, k, lane, re, im);
      slot0 += nblk;
    } else {
      run_sum<CT>(ca, cb, p.ldm, p.run_lo[q], p.run_hi[q], lane, re, im);
    }
#pragma unroll
    for (int b = 0; b < kJD; ++b)
      if (b == p.run_bin[q]) {
        nr[b] += re;
        ni[b] += im;
      }
  }
  if (lane != 0) return;
  const double n = nglob[k];
  double* r = rec + k * p.rec;
  bool sums_finite = true;
#pragma unroll
  for (int b = 0; b < kJD; ++b)
    if (b < p.d) {
      r[2 * b] = nr[b];
      r[2 * b + 1] = ni[b];
      sums_finite = sums_finite && isfinite(nr[b]) && isfinite(ni[b]);
    }
  double c1 = 0.0, c2 = -INFINITY;
  if (p.est != MP_PLUS_P)
    parity_log_weights(n, sums_finite && isfinite(n), c1, c2);
  else if (!sums_finite)
    c1 = c2 = __builtin_nan("");
  r[2 * p.d] = c1;
  r[2 * p.d + 1] = c2;
}

template <typename CT, bool PART>
__global__ __launch_bounds__(256) void jointd_occupations(JointDParams p, const CT* __restrict__ C,
                                                          const float* __restrict__ part,
                                                          const double* __restrict__ nglob,
                                                          double* __restrict__ rec) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * (4 * kOccPerWave) + wave;
  for (int j = 0; j < kOccPerWave; ++j) {
    const int64_t k = base + 4 * j;
    if (k >= p.E) return;
    jointd_sample<CT, PART>(p, C, part, nglob, rec, k, lane);
  }
}

// Box of a term: half-widths h_b and widths w_b = min(2 h_b + 1, K_b); false
// if the term is absent on some axis (then no sample reaches e^kLogEps).
__device__ inline bool term_box(const JointDParams& p, const int* band, int tau, int (&h)[kJD],
                                int (&w)[kJD]) {
  bool ok = true;
#pragma unroll
  for (int b = 0; b < kJD; ++b) {
    h[b] = 0;
    w[b] = 1;
    if (b < p.d) {
      h[b] = band[tau * kJD + b];
      ok &= h[b] >= 0;
      w[b] = min(2 * h[b] + 1, p.K[b]);
    }
  }
  return ok;
}

// Grid index of box point j on axis b of term tau.
__device__ inline int box_index(const JointDParams& p, int tau, int b, int h, int j) {
  const int K = p.K[b];
  const int c = tau == 0 ? 0 : K / 2;
  return ((c - h + j) % K + K) % K;
}

// Factor f_{s,b}(j) of term tau for chunk sample k and box point j < w_b:
// e^{+-X_b(theta) + share (- 2 Re n_b for the second term)} e^{-i theta m_lo},
// stored in the path's precision (re plane, then im plane).
template <typename CT>
__global__ __launch_bounds__(256) void jointd_factors(JointDParams p, const double* __restrict__ rec,
                                                      const int* __restrict__ band,
                                                      CT* __restrict__ tables) {
  const int tau = blockIdx.y / p.d, b = blockIdx.y % p.d;
  int h[kJD], w[kJD];
  if (!term_box(p, band, tau, h, w)) return;
  const int Kp = p.Kp[b];
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = idx / Kp;
  const int j = (int)(idx - k * Kp);
  if (k >= p.E || j >= w[b]) return;
  const double* r = rec + k * p.rec;
  const double R = r[2 * b], I = r[2 * b + 1];
  double fr = 0.0, fi = 0.0;
  const double cterm = tau == 0 ? r[2 * p.d] : r[2 * p.d + 1];
  if (cterm != -INFINITY) {  // NaN weights are evaluated: they must reach the sums
    double share = cterm;
    if (tau == 1)
      for (int q = 0; q < p.d; ++q) share += 2.0 * r[2 * q];
    share /= p.d;
    const int K = p.K[b];
    const int kg = box_index(p, tau, b, h[b], j);
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double th = kTwoPi * (double)kg / (double)K;
    const double sh = sin(0.5 * th);
    const double cm1 = -2.0 * sh * sh, sn = sin(th);
    const double xr = cm1 * R - sn * I, xi = cm1 * I + sn * R;
    const int64_t red = (((int64_t)kg * (int64_t)p.m_lo[b]) % K + K) % K;
    const double thl = kTwoPi * (double)red / (double)K;
    // FP64 tables take FP64 exp / sincos, FP32 tables FP32 ones (phase
    // reduced in FP64 first)
    constexpr bool kF64 = sizeof(CT) == 8;
    if (tau == 0)
      cis_exp<kF64>(xr + share, xi - thl, fr, fi);
    else
      cis_exp<kF64>(-xr - 2.0 * R + share, -xi - thl, fr, fi);
  }
  CT* t = tables + p.tab[tau][b];
  t[k * Kp + j] = (CT)fr;
  t[p.E * Kp + k * Kp + j] = (CT)fi;
}

// Chunk-local sample range [k0, k1) of sub-ensemble s.
__device__ inline void segment(const JointDParams& p, int64_t s, int64_t& k0, int64_t& k1) {
  const int64_t lo = s * p.ns - p.e0, hi = (s + 1) * p.ns - p.e0;
  k0 = lo > 0 ? lo : 0;
  k1 = hi < p.E ? hi : p.E;
}

// Box point indices (j_0 .. j_{d-2}) of flattened row r (last axis fastest).
__device__ inline void row_point(const JointDParams& p, const int (&w)[kJD], int64_t r,
                                 int (&j)[kJD]) {
#pragma unroll
  for (int b = kJD - 1; b >= 0; --b) {
    j[b] = 0;
    if (b < p.d - 1) {
      j[b] = (int)(r % w[b]);
      r /= w[b];
    }
  }
}

// acc[s] cell of box row r and box column c of term tau.
__device__ inline int64_t cell_of(const JointDParams& p, int tau, const int (&h)[kJD],
                                  const int (&w)[kJD], int64_t r, int c) {
  int j[kJD];
  row_point(p, w, r, j);
  int64_t flat = 0;
#pragma unroll
  for (int b = 0; b < kJD; ++b)
    if (b < p.d - 1) flat = flat * p.K[b] + box_index(p, tau, b, h[b], j[b]);
  return flat * p.K[p.d - 1] + box_index(p, tau, p.d - 1, h[p.d - 1], c);
}

// acc[s] cell of box point indices j (row axes) and box column c of term tau.
__device__ inline int64_t cell_from(const JointDParams& p, int tau, const int (&h)[kJD],
                                    const int (&j)[kJD], int c) {
  int64_t flat = 0;
#pragma unroll
  for (int b = 0; b < kJD; ++b)
    if (b < p.d - 1) flat = flat * p.K[b] + box_index(p, tau, b, h[b], j[b]);
  return flat * p.K[p.d - 1] + box_index(p, tau, p.d - 1, h[p.d - 1], c);
}

// Row widths of the FP32 box contraction: the last row axis (d - 2) padded
// to a multiple of 4, so that the four consecutive rows a thread stages
// share their other axes and take four aligned consecutive table entries.
__device__ inline void padded_widths(const JointDParams& p, const int (&w)[kJD], int (&wp)[kJD]) {
#pragma unroll
  for (int b = 0; b < kJD; ++b) wp[b] = b == p.d - 2 ? (w[b] + 3) & ~3 : w[b];
}

// Product over the row axes of one sample's factors (complex).
template <typename CT>
__device__ inline void row_factor(const JointDParams& p, int tau, const CT* __restrict__ tables,
                                  int64_t k, const int (&j)[kJD], double& ar, double& ai) {
  ar = 1.0;
  ai = 0.0;
#pragma unroll
  for (int b = 0; b < kJD - 1; ++b)
    if (b < p.d - 1) {
      const CT* t = tables + p.tab[tau][b] + k * p.Kp[b] + j[b];
      const double fr = (double)t[0], fi = (double)t[p.E * p.Kp[b]];
      const double nr = ar * fr - ai * fi;
      ai = ar * fi + ai * fr;
      ar = nr;
    }
}

// Workgroup -> (sub-ensemble, row tile, column tile); the grid covers the
// largest possible box and tiles outside the chunk's box return at once.
__device__ inline void sum_item(const JointDParams& p, int tile, int64_t& s, int64_t& rt, int& ct) {
  const int ctn = (p.K[p.d - 1] + tile - 1) / tile;
  const int64_t rtn = (p.rows_max + tile - 1) / tile;
  const int64_t item = blockIdx.x;
  ct = (int)(item % ctn);
  rt = (item / ctn) % rtn;
  s = p.s_first + item / ((int64_t)ctn * rtn);
}

constexpr int PT = 128;  // box rows / columns per FP32 tile
constexpr int PK = 32;   // samples per slab
static_assert(PT == cmfma::kTile && PK == cmfma::kSlab, "tile shape of the shared MFMA core");

// FP32 matrix cores, the 4-product complex scheme of v_mfma_f32_32x32x2f32
// (lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32]; output register
// r of lane l is element (8 (r / 4) + 4 (l / 32) + r % 4, l % 32)); wave
// (wi, wj) owns a 64 x 64 block of the 128 x 128 complex tile.  The row
// operand (the product of the row axes' factors) is formed in FP32 while a
// slab is staged, from 16-byte loads of the last row axis and the column
// axis and scalar loads of the others.
__global__ __launch_bounds__(256, 2) void jointd_sum_f32(JointDParams p, int tau,
                                                        const float* __restrict__ tables,
                                                        const int* __restrict__ band,
                                                        double* __restrict__ acc) {
  __shared__ __attribute__((aligned(16))) float lds[4][PK][PT];  // A re, A im, B re, B im
  int h[kJD], w[kJD], wp[kJD];
  if (!term_box(p, band, tau, h, w)) return;
  padded_widths(p, w, wp);
  int64_t nrows = 1;  // a multiple of 4
#pragma unroll
  for (int b = 0; b < kJD - 1; ++b)
    if (b < p.d - 1) nrows *= wp[b];
  const int ncols = w[p.d - 1];
  int64_t s, rt;
  int ct;
  sum_item(p, PT, s, rt, ct);
  if (rt * PT >= nrows || ct * PT >= ncols) return;
  int64_t k0, k1;
  segment(p, s, k0, k1);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const int lc = (tid & 31) * 4, lrow = tid >> 5;

  // the thread's rows r0 .. r0 + 3 share axes 0 .. d-3 and take entries
  // jl .. jl + 3 (jl a multiple of 4) of the last row axis
  const int64_t r0 = rt * PT + lc;
  const bool rvalid = r0 < nrows;
  int jr[kJD];
  row_point(p, wp, rvalid ? r0 : 0, jr);
  const int al = p.d - 2, bl = p.d - 1;
  const int jl = jr[al], wl = w[al];
  const float* tl = tables + p.tab[tau][al];
  const int64_t tl_im = p.E * p.Kp[al];
  const float* tb = tables + p.tab[tau][bl];
  const int64_t tb_im = p.E * p.Kp[bl];
  const int c0 = ct * PT + lc;
  const bool cvalid = c0 < ncols;  // then c0 + 3 < Kp (both multiples of 4)

  float st[4][4][4];  // [plane][u][e]
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = kb + lrow + 8 * u;
      const bool kv = k < k1;
      float pr = 1.f, pi = 0.f;  // factors of axes 0 .. d-3
#pragma unroll
      for (int b = 0; b < kJD - 2; ++b)
        if (b < al && kv && rvalid) {
          const float* t = tables + p.tab[tau][b] + k * p.Kp[b] + jr[b];
          const float fr = t[0], fi = t[p.E * p.Kp[b]];
          const float nr = pr * fr - pi * fi;
          pi = pr * fi + pi * fr;
          pr = nr;
        }
      const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
      const f32x4 lre = kv && rvalid ? *(const f32x4*)(tl + k * p.Kp[al] + jl) : zero;
      const f32x4 lim = kv && rvalid ? *(const f32x4*)(tl + tl_im + k * p.Kp[al] + jl) : zero;
      const f32x4 bre = kv && cvalid ? *(const f32x4*)(tb + k * p.Kp[bl] + c0) : zero;
      const f32x4 bim = kv && cvalid ? *(const f32x4*)(tb + tb_im + k * p.Kp[bl] + c0) : zero;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // table entries past the box width are never written: select, not multiply
        const bool av = jl + e < wl;
        st[0][u][e] = av ? pr * lre[e] - pi * lim[e] : 0.f;
        st[1][u][e] = av ? pr * lim[e] + pi * lre[e] : 0.f;
        const bool bv = c0 + e < ncols;
        st[2][u][e] = bv ? bre[e] : 0.f;
        st[3][u][e] = bv ? bim[e] : 0.f;
      }
    }
  };

  f32x16 accR[2][2], accI[2][2];
  cmfma::zero(accR, accI);

  load(k0);
  for (int64_t kb = k0; kb < k1; kb += PK) {
    __syncthreads();
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        *(f32x4*)&lds[pl][lrow + 8 * u][lc] =
            f32x4{st[pl][u][0], st[pl][u][1], st[pl][u][2], st[pl][u][3]};
    __syncthreads();
    if (kb + PK < k1) load(kb + PK);
    cmfma::slab(&lds[0][0][0], &lds[1][0][0], &lds[2][0][0], &lds[3][0][0], wi, wj, lane,
                accR, accI);
  }

  double* as = acc + 2 * s * p.cells;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t gr = rt * PT + cmfma::out_row(wi, a, q, lane);
        const int gc = ct * PT + cmfma::out_col(wj, b, lane);
        if (gr < nrows && gc < ncols) {
          int j[kJD];
          row_point(p, wp, gr, j);
          if (j[al] < wl) {
            double* o = as + 2 * cell_from(p, tau, h, j, gc);
            o[0] += accR[a][b][q];
            o[1] += accI[a][b][q];
          }
        }
      }
}

constexpr int QT = 64;  // box rows / columns per FP64 tile
constexpr int QK = 16;  // samples per slab

// FP64 FMAs: thread (ty, tx) owns rows ty + 16 u and columns tx + 16 v of a
// 64 x 64 complex tile; per sample Re += ar br, Re -= ai bi, Im += ar bi,
// Im += ai br.
__global__ __launch_bounds__(256) void jointd_sum_f64(JointDParams p, int tau,
                                                     const double* __restrict__ tables,
                                                     const int* __restrict__ band,
                                                     double* __restrict__ acc) {
  __shared__ double lds[4][QK][QT];
  int h[kJD], w[kJD];
  if (!term_box(p, band, tau, h, w)) return;
  int64_t nrows = 1;
#pragma unroll
  for (int b = 0; b < kJD - 1; ++b)
    if (b < p.d - 1) nrows *= w[b];
  const int ncols = w[p.d - 1];
  int64_t s, rt;
  int ct;
  sum_item(p, QT, s, rt, ct);
  if (rt * QT >= nrows || ct * QT >= ncols) return;
  int64_t k0, k1;
  segment(p, s, k0, k1);
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const int lc = (tid & 15) * 4, lrow = tid >> 4;
  int jr[4][kJD];
  bool rv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t r = rt * QT + lc + e;
    rv[e] = r < nrows;
    row_point(p, w, rv[e] ? r : 0, jr[e]);
  }
  const int bl = p.d - 1;
  const double* tb = tables + p.tab[tau][bl];
  const int64_t tb_im = p.E * p.Kp[bl];
  const int c0 = ct * QT + lc;
  double re[4][4], im[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) re[u][v] = im[u][v] = 0.0;

  for (int64_t kb = k0; kb < k1; kb += QK) {
    __syncthreads();
    const int64_t k = kb + lrow;
    const bool kv = k < k1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double ar = 0.0, ai = 0.0;
      if (kv && rv[e]) row_factor<double>(p, tau, tables, k, jr[e], ar, ai);
      lds[0][lrow][lc + e] = ar;
      lds[1][lrow][lc + e] = ai;
      const bool cv = kv && c0 + e < ncols;
      lds[2][lrow][lc + e] = cv ? tb[k * p.Kp[bl] + c0 + e] : 0.0;
      lds[3][lrow][lc + e] = cv ? tb[tb_im + k * p.Kp[bl] + c0 + e] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < QK; ++kk) {
      double xr[4], xi[4], yr[4], yi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xr[u] = lds[0][kk][ty + 16 * u];
        xi[u] = lds[1][kk][ty + 16 * u];
        yr[u] = lds[2][kk][tx + 16 * u];
        yi[u] = lds[3][kk][tx + 16 * u];
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
  double* as = acc + 2 * s * p.cells;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gr = rt * QT + ty + 16 * u;
      const int gc = ct * QT + tx + 16 * v;
      if (gr < nrows && gc < ncols) {
        double* o = as + 2 * cell_of(p, tau, h, w, gr, gc);
        o[0] += re[u][v];
        o[1] += im[u][v];
      }
    }
}

// ---------------------------------------------------------------- finalize

// Lines along axis a (all other indices fixed), G per workgroup (G = 4 for
// K_a <= 64, 2 for K_a <= 128, else 1; each line owns 256 / G threads, whole
// waves):
//   out[.., l_a, ..] = sum_{k_a with in != 0} in[.., k_a, ..] e^{-2 pi i k_a l_a / K_a},
// with a line's nonzero k_a listed in ascending order (ballot prefix sums
// over its waves) and the twiddles taken from a shared table of
// e^{-2 pi i q / K_a} by (k_a l_a mod K_a).  On the last axis the value times
// `scale` is sub-ensemble s's estimate of P, folded into the running mean
// (P_re, P_im) and sum of squared deviations (m2) with Welford's update.
__global__ __launch_bounds__(256) void jointd_axis(const double* __restrict__ in,
                                                   double* __restrict__ out, int Ka, int G,
                                                   int64_t n_lines, int64_t stride, int last,
                                                   double scale, int s,
                                                   double* __restrict__ P_re,
                                                   double* __restrict__ P_im,
                                                   double* __restrict__ m2) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double* tw = (double*)smem;             // 2 Ka, shared
  double* lines = tw + 2 * Ka;            // G x 2 Ka
  int* lists = (int*)(lines + 2 * G * Ka);  // G x Ka
  __shared__ int wcnt[4];
  __shared__ int total[4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int gsz = 256 / G, g = tid / gsz, gt = tid - g * gsz;
  const int wpg = gsz / 64, wig = gt >> 6;  // waves per line, wave within the line
  const int64_t L = (int64_t)blockIdx.x * G + g;
  const bool active = L < n_lines;
  const int64_t outer = L / stride, inner = L - outer * stride;
  const int64_t base = outer * (int64_t)Ka * stride + inner;
  double* line = lines + 2 * g * Ka;
  int* list = lists + g * Ka;
  for (int k = tid; k < Ka; k += 256) {
    double sw, cw;
    sincospi(-2.0 * (double)k / (double)Ka, &sw, &cw);
    tw[2 * k] = cw;
    tw[2 * k + 1] = sw;
  }
  for (int k = gt; k < Ka; k += gsz) {
    line[2 * k] = active ? in[2 * (base + k * stride)] : 0.0;
    line[2 * k + 1] = active ? in[2 * (base + k * stride) + 1] : 0.0;
  }
  if (gt == 0) total[g] = 0;
  __syncthreads();
  for (int k0 = 0; k0 < Ka; k0 += gsz) {  // same trip count in every line
    const int k = k0 + gt;
    const bool nz = k < Ka && (line[2 * k] != 0.0 || line[2 * k + 1] != 0.0);
    const unsigned long long mask = __ballot(nz);
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wave] = __popcll(mask);
    __syncthreads();
    int off = total[g];
    for (int q = 0; q < wig; ++q) off += wcnt[g * wpg + q];
    if (nz) list[off + pre] = k;
    __syncthreads();
    if (gt == 0)
      for (int q = 0; q < wpg; ++q) total[g] += wcnt[g * wpg + q];
    __syncthreads();
  }
  if (!active) return;
  const int nnz = total[g];
  // k l < 2^24 (Ka <= 4096) is exact in FP32: the quotient estimate is off by
  // at most one, which the correction removes
  const float inv_k = 1.0f / (float)Ka;
  for (int l = gt; l < Ka; l += gsz) {
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < nnz; ++q) {
      const int k = list[q];
      const int kl = k * l;
      int t = kl - (int)((float)kl * inv_k) * Ka;
      t += t < 0 ? Ka : 0;
      t -= t >= Ka ? Ka : 0;
      const double xr = line[2 * k], xi = line[2 * k + 1];
      const double cr = tw[2 * t], ci = tw[2 * t + 1];
      sr += xr * cr - xi * ci;
      si += xr * ci + xi * cr;
    }
    const int64_t cell = base + l * stride;
    if (!last) {
      out[2 * cell] = sr;
      out[2 * cell + 1] = si;
    } else {
      const double vr = sr * scale, vi = si * scale;
      if (s == 0) {
        P_re[cell] = vr;
        if (P_im) P_im[cell] = vi;
        m2[cell] = 0.0;
      } else {
        const double mean = P_re[cell];
        const double dr = vr - mean;
        const double nm = mean + dr / (s + 1);
        P_re[cell] = nm;
        if (P_im) P_im[cell] += (vi - P_im[cell]) / (s + 1);
        m2[cell] += dr * (vr - nm);
      }
    }
  }
}

__global__ void jointd_sigma(int64_t cells, int n_sub, double* __restrict__ sigma) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= cells) return;
  sigma[i] = n_sub > 1 ? sqrt(sigma[i] / (n_sub - 1) / n_sub) : __builtin_nan("");
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Workspace layout of a chunk: band ints, per-sample records, factor tables
// (FP64 elements for the FP64 path, FP32 otherwise).
size_t layout(JointDParams& p, size_t elem) {
  int64_t off = 256;  // band
  off += round_up(p.E * p.rec * 8, 256);
  int64_t tab = 0;
  for (int tau = 0; tau < 2; ++tau)
    for (int b = 0; b < p.d; ++b) {
      p.tab[tau][b] = tab;
      tab += 2 * p.E * p.Kp[b];
    }
  return (size_t)off + (size_t)tab * elem;
}

bool fill_params(JointDParams& p, int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                 const int32_t* m_lo, const int32_t* K, int64_t ns, int64_t e0) {
  p.M = M;
  p.ldm = ld_modes(M);
  p.E = E;
  p.e0 = e0;
  p.ns = ns;
  p.d = d;
  p.rec = 2 * d + 2;
  p.cells = 1;
  p.rows_max = 1;
  for (int b = 0; b < d; ++b) {
    p.m_lo[b] = m_lo ? m_lo[b] : 0;
    p.K[b] = K[b];
    p.Kp[b] = (int)round_up(K[b], 4);
    p.cells *= K[b];
    // the FP32 contraction pads the last row axis to a multiple of 4
    if (b < d - 1) p.rows_max *= b == d - 2 ? round_up(K[b], 4) : K[b];
  }
  p.s_first = e0 / ns;
  p.n_runs = 0;
  if (!bin_of_mode) return true;
  for (int j = 0; j < M;) {
    const int b = bin_of_mode[j];
    int j2 = j + 1;
    while (j2 < M && bin_of_mode[j2] == b) ++j2;
    if (b >= 0) {
      if (p.n_runs >= MP_MAX_RUNS) return false;
      p.run_lo[p.n_runs] = j;
      p.run_hi[p.n_runs] = j2;
      p.run_bin[p.n_runs] = b;
      ++p.n_runs;
    }
    j = j2;
  }
  return true;
}

}  // namespace

mp_status record_bands_launch(const double* rec, int64_t E, int d, const int32_t* K,
                              int band_stride, int* band, hipStream_t stream);

size_t jointd_workspace(int32_t d, const int32_t* K, int64_t E) {
  JointDParams p{};
  fill_params(p, 1, E, d, nullptr, nullptr, K, 1, 0);
  return layout(p, 8);
}

size_t jointd_finalize_workspace(int32_t d, const int32_t* K) {
  int64_t cells = 1;
  for (int b = 0; b < d; ++b) cells *= K[b];
  return (size_t)(256 + 2 * round_up(cells * 16, 256));
}

// part != nullptr: the bin sums come from the occupation-fused GEMM's partials
// (runs in the order fill_params builds them) and C is unused.
mp_status jointd_launch(int32_t M, int64_t E, const void* C, const double* n, mp_precision prec,
                        mp_estimator est, int32_t d, const int32_t* bin_of_mode,
                        const int32_t* m_lo, const int32_t* K, int32_t n_sub, int64_t ns,
                        int64_t e0, double* acc, void* ws, size_t ws_bytes, hipStream_t stream,
                        const float* part) {
  MP_CHECK_ARG(d >= 3 && d <= kJD, MP_ERR_UNSUPPORTED,
               "mp_binned_counts: joint distributions need d <= %d (d = %d)", kJD, d);
  for (int b = 0; b < d; ++b)
    MP_CHECK_ARG(K[b] >= 1 && K[b] <= 1024, MP_ERR_UNSUPPORTED,
                 "mp_binned_counts: joint windows of d >= 3 need 1 <= K <= 1024 (K[%d] = %d)", b, K[b]);
  JointDParams p{};
  int64_t cells = 1;
  for (int b = 0; b < d; ++b) cells *= K[b];
  MP_CHECK_ARG(cells < 0x7fffffff, MP_ERR_UNSUPPORTED,
               "mp_binned_counts: joint grid of %lld cells exceeds 2^31 - 1", (long long)cells);
  MP_CHECK_ARG(fill_params(p, M, E, d, bin_of_mode, m_lo, K, ns, e0), MP_ERR_UNSUPPORTED,
               "mp_binned_counts: bins form more than %d contiguous mode runs", MP_MAX_RUNS);
  p.est = est;
  const int64_t s_last = (e0 + E - 1) / ns;
  MP_CHECK_ARG(s_last < n_sub, MP_ERR_SHAPE,
               "mp_binned_counts: samples [%lld, %lld) exceed n_sub * samples_per_sub = %lld",
               (long long)e0, (long long)(e0 + E), (long long)n_sub * ns);
  const size_t need = layout(p, prec == MP_FP64 ? 8 : 4);
  MP_CHECK_ARG(ws && ws_bytes >= need, MP_ERR_WORKSPACE,
               "mp_binned_counts: workspace of %zu bytes needed, %zu given", need, ws_bytes);
  const int tile = prec == MP_FP64 ? QT : PT;
  const int64_t items = (s_last - p.s_first + 1) * ((p.rows_max + tile - 1) / tile) *
                        ((K[d - 1] + tile - 1) / tile);
  MP_CHECK_ARG(items < 0x7fffffff, MP_ERR_UNSUPPORTED,
               "mp_binned_counts: the joint grid of %lld workgroups is too large", (long long)items);
  int* band = (int*)ws;
  double* rec = (double*)((char*)ws + 256);
  void* tables = (char*)ws + 256 + round_up(E * p.rec * 8, 256);
  hipLaunchKernelGGL(band_init, dim3(1), dim3(64), 0, stream, band);
  const unsigned blocks = (unsigned)((E + 4 * kOccPerWave - 1) / (4 * kOccPerWave));
  int kp_max = 0;
  for (int b = 0; b < d; ++b) kp_max = p.Kp[b] > kp_max ? p.Kp[b] : kp_max;
  const dim3 fgrid((unsigned)((E * kp_max + 255) / 256), (unsigned)(2 * d));
  if (prec == MP_FP64) {
    if (part)
      hipLaunchKernelGGL((jointd_occupations<float, true>), dim3(blocks), dim3(256), 0, stream, p,
                         (const float*)nullptr, part, n, rec);
    else
      hipLaunchKernelGGL((jointd_occupations<double, false>), dim3(blocks), dim3(256), 0, stream,
                         p, (const double*)C, (const float*)nullptr, n, rec);
    const mp_status sb = record_bands_launch(rec, E, d, K, kJD, band, stream);
    if (sb != MP_OK) return sb;
    hipLaunchKernelGGL(jointd_factors<double>, fgrid, dim3(256), 0, stream, p, rec, band,
                       (double*)tables);
    for (int tau = 0; tau < 2; ++tau)
      hipLaunchKernelGGL(jointd_sum_f64, dim3((unsigned)items), dim3(256), 0, stream, p, tau,
                         (const double*)tables, band, acc);
  } else {
    if (part)
      hipLaunchKernelGGL((jointd_occupations<float, true>), dim3(blocks), dim3(256), 0, stream, p,
                         (const float*)nullptr, part, n, rec);
    else
      hipLaunchKernelGGL((jointd_occupations<float, false>), dim3(blocks), dim3(256), 0, stream,
                         p, (const float*)C, (const float*)nullptr, n, rec);
    const mp_status sb = record_bands_launch(rec, E, d, K, kJD, band, stream);
    if (sb != MP_OK) return sb;
    hipLaunchKernelGGL(jointd_factors<float>, fgrid, dim3(256), 0, stream, p, rec, band,
                       (float*)tables);
    for (int tau = 0; tau < 2; ++tau)
      hipLaunchKernelGGL(jointd_sum_f32, dim3((unsigned)items), dim3(256), 0, stream, p, tau,
                         (const float*)tables, band, acc);
  }
  MP_HIP_LAUNCH_CHECK("mp_binned_counts joint (d >= 3) launch");
  return MP_OK;
}

mp_status jointd_finalize(int32_t d, const int32_t* K, int32_t n_sub, int64_t ns,
                          const double* acc, double* P_re, double* P_im, double* sigma, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  const size_t need = jointd_finalize_workspace(d, K);
  MP_CHECK_ARG(ws && ws_bytes >= need, MP_ERR_WORKSPACE,
               "mp_counts_finalize: workspace of %zu bytes needed, %zu given", need, ws_bytes);
  const int kmax = d == 2 ? kAxisMaxK : 1024;
  for (int b = 0; b < d; ++b)
    MP_CHECK_ARG(K[b] >= 1 && K[b] <= kmax, MP_ERR_UNSUPPORTED,
                 "mp_counts_finalize: joint windows of %d bins need 1 <= K <= %d (K[%d] = %d)", d,
                 kmax, b, K[b]);
  static bool lds_set = false;
  if (!lds_set) {
    // a line of the largest grid with its twiddles and index list: 36 B per point
    const hipError_t e = hipFuncSetAttribute((const void*)jointd_axis,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             36 * kAxisMaxK);
    MP_CHECK_ARG(e == hipSuccess, MP_ERR_HIP, "mp_counts_finalize: %s", hipGetErrorString(e));
    lds_set = true;
  }
  int64_t cells = 1;
  for (int b = 0; b < d; ++b) cells *= K[b];
  MP_CHECK_ARG(cells < 0x7fffffff, MP_ERR_UNSUPPORTED,
               "mp_counts_finalize: joint grid of %lld cells exceeds 2^31 - 1", (long long)cells);
  double* buf[2] = {(double*)((char*)ws + 256),
                    (double*)((char*)ws + 256 + round_up(cells * 16, 256))};
  const double scale = 1.0 / ((double)cells * (double)ns);
  for (int s = 0; s < n_sub; ++s) {
    const double* src = acc + 2 * (int64_t)s * cells;
    for (int a = 0; a < d; ++a) {
      int64_t stride = 1;
      for (int b = a + 1; b < d; ++b) stride *= K[b];
      const int last = a == d - 1;
      double* dst = buf[a & 1];
      const int G = K[a] <= 64 ? 4 : (K[a] <= 128 ? 2 : 1);
      const int64_t n_lines = cells / K[a];
      const size_t lds = (size_t)K[a] * (16 + 20 * G);
      hipLaunchKernelGGL(jointd_axis, dim3((unsigned)((n_lines + G - 1) / G)), dim3(256), lds,
                         stream, src, dst, K[a], G, n_lines, stride, last, scale, s, P_re, P_im,
                         sigma);
      src = dst;
    }
  }
  hipLaunchKernelGGL(jointd_sigma, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, stream,
                     cells, n_sub, sigma);
  MP_HIP_LAUNCH_CHECK("mp_counts_finalize joint (d >= 3) launch");
  return MP_OK;
}

}  // namespace mp
