/*
 * mpgbs.h -- C ABI of the MI355X (gfx950) matrix-P Gaussian-boson-sampling
 * hot path: parity-projected phase-space estimates of total and grouped
 * photon-count probabilities (Drummond, Dellios & Reid, "Matrix phase-space
 * representations for Gaussian boson sampling", arXiv:2503.12749).
 *
 * Pipeline, one chunk of E phase-space samples at a time:
 *   mp_sample          real amplitudes (alpha, beta) of squeezed inputs and
 *                      the global photon number n = alpha . beta
 *   mp_propagate       alpha' = T alpha, beta' = T* beta as one real GEMM
 *   mp_binned_counts   occupations, parity weight and characteristic function
 *                      on the count window, accumulated per sub-ensemble
 * and once at the end:
 *   mp_counts_finalize inverse DFT to P(m) and the sub-ensemble error sigma_T
 *
 * Conventions shared by every entry point
 *   - Pointers marked "device" are HIP device (or managed) memory owned by the
 *     caller; "host" pointers are read synchronously during the call.  The
 *     library never allocates, frees or retains caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     asynchronously on it; arguments are validated on the host before any
 *     launch, and a failed validation enqueues nothing.
 *   - Every call returns an mp_status and never throws across the ABI.  The
 *     message of the last non-MP_OK status of the calling thread is returned
 *     by mp_last_error().
 *   - Mode-major buffers use the padded leading dimension ldm = mp_ld_modes(M)
 *     (M rounded up to a multiple of 128); padding rows hold zeros.
 *   - Calls that share buffers must be ordered on one stream; calls on
 *     different streams that write the same accumulator race.
 */
#ifndef MPGBS_H
#define MPGBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MP_OK = 0,
  MP_ERR_ARG = -1,         /* invalid scalar argument or null pointer */
  MP_ERR_SHAPE = -2,       /* sizes inconsistent with each other */
  MP_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  MP_ERR_UNSUPPORTED = -4, /* valid request outside what the library handles */
  MP_ERR_WORKSPACE = -5,   /* workspace missing or smaller than required */
  MP_ERR_NONFINITE = -6    /* a result holds NaN or infinite values (mp_check_finite) */
} mp_status;

typedef enum {
  MP_FP64 = 0,       /* FP64 samples, FP64 MFMA GEMM, FP64 characteristic function */
  MP_FP32 = 1,       /* FP32 samples, FP32 MFMA GEMM, FP32 characteristic function */
  MP_SPLIT_BF16 = 2, /* hi/lo BF16 operands, 3 BF16 MFMA products, FP32 accumulate */
  MP_SPLIT_FP16 = 3, /* hi/lo FP16 operands, 3 FP16 MFMA products, FP32 accumulate */
  MP_SPLIT1_FP16 = 4, /* T as one FP16 value, samples hi/lo FP16 (MP_SPLIT_FP16's sample
                         layout), 2 FP16 MFMA products, FP32 accumulate */
  MP_SPLIT1T_FP16 = 5, /* T hi/lo FP16 (MP_SPLIT_FP16's packing), samples as one FP16
                          value (column pairs, below), 2 FP16 MFMA products, FP32
                          accumulate: the rounding error is per sample and averages
                          like the sampling noise */
  MP_SPLIT1T_F8 = 6,   /* MP_SPLIT1T_FP16 with the correction product in FP8: T as an
                          FP16 value and its FP16 remainder scaled into OCP e4m3, the
                          samples as one FP16 value plus an e4m3 copy (layouts below);
                          C = T_hi S + T_lo8 S8 by one FP16 and one FP8 MFMA product
                          per pair of 32-deep slabs, FP32 accumulate */
  /* Range markers, not values: with them every int is a representable
   * mp_precision, so an out-of-range argument reaches the library's check
   * (MP_ERR_ARG) instead of being undefined on the C++ side.  The same holds
   * for the other enumerations below. */
  MP_PRECISION_RANGE_MIN_ = -0x7fffffff - 1,
  MP_PRECISION_RANGE_MAX_ = 0x7fffffff
} mp_precision;

typedef enum {
  MP_JOINT = 0,              /* joint distribution of the d bin counts (d <= 4) */
  MP_MARGINALS = 1,          /* d one-bin distributions (S = S_b alone) */
  MP_MARGINALS_AND_TOTAL = 2, /* the d marginals plus the total over all bins */
  MP_BIN_MODE_RANGE_MIN_ = -0x7fffffff - 1,
  MP_BIN_MODE_RANGE_MAX_ = 0x7fffffff
} mp_bin_mode;

typedef enum {
  MP_MATRIX_P = 0, /* parity-projected weight g0 (main text, eq. c-number-variable) */
  MP_PLUS_P = 1,   /* positive-P observable, g0 = 1 (Appendix A) */
  MP_ESTIMATOR_RANGE_MIN_ = -0x7fffffff - 1,
  MP_ESTIMATOR_RANGE_MAX_ = 0x7fffffff
} mp_estimator;

#define MP_MAX_BINS 8  /* bins per call */
#define MP_MAX_RUNS 16 /* contiguous mode runs over all bins per call */

/* ---------------------------------------------------------------- sizes */

/* Padded leading dimension of mode-major buffers: M rounded up to 128. */
int64_t mp_ld_modes(int32_t M);

/* Bytes of the amplitude buffer `ab` of mp_sample / mp_propagate. */
size_t mp_ab_bytes(int32_t M, int64_t E, mp_precision prec);

/* Bytes of the propagated buffer `C` of mp_propagate / mp_binned_counts. */
size_t mp_c_bytes(int32_t M, int64_t E, mp_precision prec);

/* ---------------------------------------------------------------- S1 */

/*
 * Phase-space amplitudes of squeezed vacuum inputs (main text, the squeezed
 * state as a real coherent-state integral with weight xi(alpha), sampled with
 * the +P procedure that the parity-projected distribution P_2 reuses).
 *
 * Per mode j the pair (alpha_j, beta_j) is real Gaussian with variances
 * sinh r_j cosh r_j and covariance sinh^2 r_j:
 *   alpha_j = c+ w1 + c- w2,  beta_j = c+ w1 - c- w2,
 *   c+ = sqrt(e^{2 r_j} - 1) / 2,  c- = sqrt(1 - e^{-2 r_j}) / 2.
 * (w1, w2) are Box-Muller normals from one Philox4x64-10 call with counter
 * (g, p, net, 0) and key (seed, 0) for global sample index g and mode pair
 * p = j / 2: words 0,1 feed mode 2p and words 2,3 mode 2p+1, with
 * u = ((x0 >> 11) + 1) 2^-53, v = (x1 >> 11) 2^-53,
 * w1 = sqrt(-2 ln u) cos(2 pi v), w2 = sqrt(-2 ln u) sin(2 pi v).
 * The draw of a sample depends only on (seed, net, g), never on chunking.
 *
 *   M      modes, >= 1                 g0     global index of the first sample
 *   E      samples in this call, >= 1  r      device FP64[M], r_j >= 0 (0 = vacuum)
 *   ab     device, mp_ab_bytes(M, E, prec) bytes, column-major: column k < E
 *          holds alpha of sample g0+k, column E+k its beta (column stride ldm
 *          for FP64 and FP32).
 *          FP64 -> double, FP32 -> float.  SPLIT_* and SPLIT1_FP16 -> 16-bit values with
 *          x = hi + lo (hi = x rounded, lo = the rounded remainder), column
 *          stride 2 ldm: mode j of a column has hi at 64 (j / 32) + j % 32 and
 *          lo 32 values further (blocks of 32 hi values, each followed by
 *          its 32 lo values).
 *          SPLIT1T_FP16 -> one FP16 value per entry, in storage columns: alpha
 *          of sample k in column k, beta in column E2 + k with E2 = E rounded
 *          up to even; columns 2q and 2q + 1 are stored as a pair, mode j of
 *          column c at (c / 2) 2 ldm + 64 (j / 32) + j % 32 + 32 (c % 2) (for
 *          each 32-mode block, the pair's two 32-value runs side by side).
 *          With E odd the storage columns E and E2 + E are padding, written
 *          as zeros.
 *          SPLIT1T_F8 -> the SPLIT1T_FP16 operand (same storage columns and
 *          layout, 2 ldm 2 E2 bytes), followed by the e4m3 copy of each value
 *          (OCP FP8: 4 exponent bits, bias 7, 3 mantissa bits, round to
 *          nearest even): mode j of storage column c at byte (c / 2) 2 ldm +
 *          128 (j / 64) + 64 (c % 2) + j % 64 of that second part (for each
 *          64-mode block, the pair's two 64-byte runs side by side).  The
 *          copies saturate at 448: an amplitude beyond it (possible only
 *          for squeezing r above about 4.6, where the largest amplitude a
 *          Box-Muller pair can give, 8.6 (c+ + c-) ~ 4.3 e^r, reaches 448)
 *          keeps its FP16 value in the main product and enters the
 *          correction term, 2^-11 of that product, as 448.
 *   n_out  device FP64[E]: n = sum_j alpha_j beta_j of the values as stored
 *          (after rounding to `prec`).
 */
mp_status mp_sample(int32_t M, int64_t g0, int64_t E, const double* r, uint64_t seed,
                    uint32_t net, mp_precision prec, void* ab, double* n_out, void* stream);

/* ---------------------------------------------------------------- S2 */

/* Workspace bytes mp_propagate needs (the packed transmission operand). */
size_t mp_propagate_workspace(int32_t M, mp_precision prec);

/*
 * Linear-network propagation alpha' = T alpha, beta' = T* beta (main text,
 * characteristics of the network equation; loss as a sub-unitary T).  Since
 * alpha and beta are real this is one real GEMM
 *     C = [Re T; Im T] (2M x M) * [alpha | beta] (M x 2E).
 *
 *   T   device FP64, complex M x M, row-major, interleaved (re, im):
 *       T[2 (i M + j)] = Re T_ij maps input mode j to output mode i.
 *   ab  device, as written by mp_sample with the same M, E, prec.
 *   C   device, mp_c_bytes(M, E, prec) bytes, column-major with ld = 2 ldm:
 *       column k: rows [0, ldm) = Re alpha'_k, rows [ldm, 2 ldm) = Im alpha'_k;
 *       column E+k: rows [0, ldm) = Re beta'_k, rows [ldm, 2 ldm) = -Im beta'_k.
 *       FP64 -> double, every other precision -> float.
 *   workspace  device, >= mp_propagate_workspace(M, prec) bytes, 256-aligned;
 *       overwritten (T is re-packed on every call).
 */
mp_status mp_propagate(int32_t M, int64_t E, const double* T, mp_precision prec,
                       const void* ab, void* C, void* workspace, size_t ws_bytes,
                       void* stream);

/*
 * The two halves of mp_propagate, for callers that propagate many chunks
 * through one network: mp_pack_transmission writes the packed operand
 * [Re T; Im T] in the GEMM's storage precision into `workspace` (same size
 * and alignment rules as mp_propagate's workspace), and mp_propagate_packed
 * runs the GEMM of mp_propagate on it.  The workspace must hold the packing
 * of the same M and prec, written by a call ordered before this one (same
 * stream, or synchronised); the library cannot check that.  Same layouts of
 * ab and C as mp_propagate.
 */
mp_status mp_pack_transmission(int32_t M, const double* T, mp_precision prec, void* workspace,
                               size_t ws_bytes, void* stream);
mp_status mp_propagate_packed(int32_t M, int64_t E, mp_precision prec, const void* ab, void* C,
                              const void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- S3-S5 */

/* Complex accumulator entries per sub-ensemble for a bin layout:
 * joint -> prod K_b, marginals -> sum K_b (+ K_total). */
int64_t mp_acc_entries(int32_t d, mp_bin_mode mode, const int32_t* K);

/* Workspace bytes mp_binned_counts needs for one call. */
size_t mp_binned_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int64_t E,
                           int32_t n_sub, int64_t samples_per_sub, int64_t e0);

/*
 * Grouped count observables (eq. General_GCP) of one chunk, accumulated per
 * sub-ensemble (Appendix A).  For each sample:
 *   n'_i = alpha'_i beta'_i,  n_b = sum_{i in S_b} n'_i,  n_S = sum_b n_b,
 * and the generating function of eq. c-number-variable summed over patterns,
 *   chi(z) = sum_m G(m) prod_b z_b^m_b = cosh(n + X) / cosh(n),
 *   X = sum_b n_b (z_b - 1)       (MP_PLUS_P: chi = exp(X)),
 * with the global n of the inputs, evaluated on z_b = exp(2 pi i k / K_b) and
 * multiplied by z_b^(-m_lo_b) so that the window [m_lo_b, m_lo_b + K_b) maps
 * to residues 0..K_b-1.  Sums over the samples of each sub-ensemble are added
 * into acc (two-pass, deterministic: no floating-point atomics).
 *
 *   C, n        as written by mp_propagate / mp_sample for this chunk
 *   d           bins, 1..MP_MAX_BINS (MP_JOINT: d <= 4)
 *   bin_of_mode host int32[M], values in [-1, d); -1 = not counted.  Each bin
 *               must be a union of contiguous mode runs, at most MP_MAX_RUNS
 *               runs in total.
 *   m_lo, K     host int32 per distribution (d of them, d+1 with the total
 *               last); m_lo >= 0, 1 <= K <= 65536 (MP_JOINT: K <= 4096 for
 *               d = 2; K <= 1024 and prod K_b < 2^31 for d >= 3)
 *   n_sub, samples_per_sub  sub-ensembles N_R and their size N_S; global
 *               sample g belongs to sub-ensemble g / N_S < n_sub
 *   e0          global index of the chunk's first sample
 *   acc         device FP64, n_sub * mp_acc_entries * 2 doubles (re, im), laid
 *               out [sub-ensemble][distribution][k]; zeroed by the caller
 *               before the first chunk.
 *   workspace   device, >= mp_binned_workspace(...) bytes, 256-aligned.
 *
 * Joint distributions of d = 3 or 4 bins (main text, higher-dimensional
 * binning): per sample chi is the sum of two rank-1 tensors over the bins,
 * e^{c1} prod_b e^{X_b} + e^{c2} prod_b e^{-X_b}.  Each is evaluated only in
 * the box of grid points around theta = 0 (first) or theta = pi (second)
 * outside which every sample of the chunk stays below e^-46 (~1e-20; the
 * bound is exact per sample), as a contraction over samples: products of the
 * first d - 1 bins' per-sample factors against the last bin's, on the FP32
 * matrix cores (FP32 and split paths: factors rounded to FP32, FP32 sums
 * over a chunk's samples of one sub-ensemble, FP64 across chunks) or with
 * FP64 FMAs (FP64 path).  acc is the full grid [s][k_1]..[k_d]; entries
 * outside the boxes stay zero.
 *
 * Non-finite samples: a sample whose n or bin sums are NaN or infinite (an
 * amplitude beyond a reduced precision's range, e.g. FP16 samples at
 * squeezing r above about 9.6) is not dropped by the e^-46 skip or the boxes:
 * it turns the accumulators it reaches NaN (every grid point of its
 * sub-ensemble's distributions), so mp_check_finite on P or acc reports
 * MP_ERR_NONFINITE rather than a finite estimate without it.  The same holds
 * for mp_propagate_counts, mp_moments_accumulate (NaN sums) and
 * mp_observable_histogram (the top, not-finite bin).
 */
mp_status mp_binned_counts(int32_t M, int64_t E, const void* C, const double* n,
                           mp_precision prec, mp_estimator est, int32_t d,
                           const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                           const int32_t* K, int32_t n_sub, int64_t samples_per_sub,
                           int64_t e0, double* acc, void* workspace, size_t ws_bytes,
                           void* stream);

/*
 * mp_propagate_packed followed by mp_binned_counts without materialising C
 * (the occupation-fused GEMM): each 256 x 256 GEMM tile covers the Re and Im
 * rows of 128 modes and the alpha and beta columns of 128 samples, and its
 * epilogue reduces alpha'_j beta'_j over the modes of every bin run in the
 * tile to per-sample partials (16 bytes per run, block and sample, at the
 * start of `workspace`); the counting kernels then read those partials
 * instead of C.  Same estimator, windows, limits and accumulator layout as
 * mp_binned_counts, for every mode: MP_MARGINALS, MP_MARGINALS_AND_TOTAL and
 * MP_JOINT with d = 1 .. 4 (joint distributions of d >= 2 bins take their
 * per-sample bin sums from the partials; the rest of their path is the one
 * mp_binned_counts runs).  The occupations are summed in FP32 within a tile
 * and in FP64 across tiles, so results agree with the unfused path to FP32
 * rounding.
 *
 *   prec       MP_FP32 or any split precision (MP_SPLIT_BF16, MP_SPLIT_FP16,
 *              MP_SPLIT1_FP16, MP_SPLIT1T_FP16, MP_SPLIT1T_F8); MP_FP64:
 *              MP_ERR_UNSUPPORTED
 *   ab, n      as written by mp_sample for this chunk
 *   packed     device, as written by mp_pack_transmission(M, T, prec, ...),
 *              packed_bytes >= mp_propagate_workspace(M, prec), 256-aligned
 *   d ... e0, acc  as for mp_binned_counts
 *   workspace  device, >= mp_propagate_counts_workspace(...) bytes,
 *              256-aligned; overwritten
 */
size_t mp_propagate_counts_workspace(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                                     mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                                     int64_t samples_per_sub, int64_t e0);
mp_status mp_propagate_counts(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                              const void* ab, const double* n, const void* packed,
                              size_t packed_bytes, int32_t d, const int32_t* bin_of_mode,
                              mp_bin_mode mode, const int32_t* m_lo, const int32_t* K,
                              int32_t n_sub, int64_t samples_per_sub, int64_t e0, double* acc,
                              void* workspace, size_t ws_bytes, void* stream);

/*
 * One count distribution through a bilinear form (main text: the generating
 * function of binned counts depends on the samples only through
 * n_S = sum_{j in S} alpha'_j beta'_j, with alpha' = T alpha and beta' = T* beta
 * for the linear network).  For real alpha, beta this is exactly
 *     n_S = alpha^T W beta,   W = T^T P_S T*   (P_S: the projector on S),
 * so one complex M x M operator applied to beta replaces T applied to both
 * alpha and beta: 4 M^2 flops per sample instead of 8 M^2.  W is formed once per
 * network (8 M^3 FP64 flops): its off-diagonal part packed as the precision
 * packs T, its real diagonal D_a = sum_{j in S} |T_ja|^2 in FP32 after it.  D
 * alone sets the mean of n_S (E[alpha_a beta_b] = 0 for a != b), so it is
 * applied exactly, as sum_a D_a alpha_a beta_a in the GEMM's epilogue; the
 * off-diagonal part's packing rounding then only adds noise.  Only one
 * distribution per pass (S, d = 1); marginals and joint distributions need
 * one W per bin and stay with mp_propagate_counts.
 *
 * mp_pack_bilinear forms W on the FP64 matrix cores and packs it, then waits
 * for `stream` (it reads bin_of_mode from host memory on the stream), so it
 * returns once W is packed.
 *   T            device, complex M x M as for mp_propagate
 *   bin_of_mode  host, len M: 0 for the modes of S, -1 for the others
 *   prec         MP_SPLIT1T_F8 (others: MP_ERR_UNSUPPORTED)
 *   packed       device, >= mp_bilinear_packed_bytes(M) bytes, 256-aligned;
 *                overwritten with packed W
 *   scratch      device, >= mp_bilinear_workspace(M) bytes (about 96 M^2
 *                bytes: 6.2 GB at M = 8000), 256-aligned; overwritten
 *
 * mp_propagate_counts_bilinear is mp_propagate_counts for one distribution of
 * the set W was packed for: the FP8-correction GEMM of W against the beta half
 * of the sample operand, its epilogue reducing sum_a alpha_a (W beta)_a over
 * each 128-mode block to the per-sample partials, then the counting kernels.
 *   ab, n        as written by mp_sample(..., MP_SPLIT1T_F8, ...) for this
 *                chunk
 *   packed       as written by mp_pack_bilinear
 *   m_lo, K      host, one window; n_sub ... acc as for mp_binned_counts
 *                with d = 1
 *   workspace    device, >= mp_propagate_counts_workspace(M, E, 1, b, MP_JOINT,
 *                K, n_sub, samples_per_sub, e0) bytes with b all zero,
 *                256-aligned; overwritten
 * Rounding: the T-split form's, with W in place of T (W's packing keeps each
 * entry to about 2^-15; the samples' FP16 rounding averages like the noise).
 */
size_t mp_bilinear_workspace(int32_t M);
size_t mp_bilinear_packed_bytes(int32_t M);
mp_status mp_pack_bilinear(int32_t M, const double* T, const int32_t* bin_of_mode,
                           mp_precision prec, void* packed, size_t packed_bytes, void* scratch,
                           size_t scratch_bytes, void* stream);
mp_status mp_propagate_counts_bilinear(int32_t M, int64_t E, mp_precision prec,
                                       mp_estimator est, const void* ab, const double* n,
                                       const void* packed, size_t packed_bytes,
                                       const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                       int64_t samples_per_sub, int64_t e0, double* acc,
                                       void* workspace, size_t ws_bytes, void* stream);

/*
 * mp_propagate_counts without a workspace, for callers that cannot allocate
 * device memory: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It allocates nothing and calls no allocating
 * routine; the GEMM's partials and the counting kernel's partials live in a
 * scratch array of MP_NOALLOC_SCRATCH_BYTES that each GPU the library runs on
 * holds until the process ends (its address is looked up on the first call on
 * a device, with that device current; `stream` must belong to the current
 * device).  Same arguments, kernels, results and accumulator layout as
 * mp_propagate_counts, for MP_MARGINALS, MP_MARGINALS_AND_TOTAL and MP_JOINT
 * with d = 1 (joint distributions of d >= 2 bins: MP_ERR_UNSUPPORTED).
 *
 *   Returns MP_ERR_WORKSPACE, enqueuing nothing, when the chunk needs more than
 *   MP_NOALLOC_SCRATCH_BYTES (mp_propagate_counts_workspace(...) gives the
 *   need; e.g. total counts at M = 8000 on a 3840-count window take about
 *   2 KB per sample, so chunks up to about 32000 samples fit).
 *   Every call on one GPU uses that GPU's single array, which keeps the last
 *   call's contents (each call writes every scratch byte before it reads it,
 *   so nothing needs clearing): calls that overlap on one GPU (other streams,
 *   other threads) race and must be serialised by the caller.
 */
#define MP_NOALLOC_SCRATCH_BYTES (64u << 20)
mp_status mp_propagate_counts_noalloc(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                                      const void* ab, const double* n, const void* packed,
                                      size_t packed_bytes, int32_t d, const int32_t* bin_of_mode,
                                      mp_bin_mode mode, const int32_t* m_lo, const int32_t* K,
                                      int32_t n_sub, int64_t samples_per_sub, int64_t e0,
                                      double* acc, void* stream);

/*
 * Inverse DFT of each sub-ensemble's mean characteristic function,
 *   P_s(m_lo + l) = (1/K) sum_k chi_s(k) exp(-2 pi i k l / K),
 * then P = mean_s P_s and sigma_T = sd_s(Re P_s) / sqrt(n_sub) (Appendix A;
 * NaN when n_sub = 1).  Counts outside a window alias into it mod K.
 *
 *   acc     device, complete accumulators (all n_sub * samples_per_sub samples)
 *   P_re, P_im, sigma  device FP64[mp_acc_entries]; P_im may be NULL.
 *           Joint layout [k1][k2]; marginal layout concatenated per distribution.
 *   workspace  device, >= mp_finalize_workspace(...) bytes, 256-aligned (may be
 *           NULL when that size is 0).  Joint grids (d = 2, 3, 4) are
 *           transformed one axis at a time per sub-ensemble over the nonzero
 *           entries of each line (acc is zero outside the frequency bands the
 *           chunks touched); layout [k_1]..[k_d]; K <= 4096 for d = 2.
 */
size_t mp_finalize_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub);

mp_status mp_counts_finalize(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                             int64_t samples_per_sub, const double* acc, double* P_re,
                             double* P_im, double* sigma, void* workspace, size_t ws_bytes,
                             void* stream);

/* ---------------------------------------------------------------- per-sample observables */

#define MP_MAX_MOMENTS 8 /* orders per mp_moments_accumulate call */

/*
 * Occupation of each distribution for every sample of a chunk (main text:
 * the grouped occupations n_S = sum over the counted modes of alpha'_j
 * beta'_j that enter the pattern observables): n_q sums over the modes of
 * bin q (q < d) or over all d bins (the total, q = d, with
 * MP_MARGINALS_AND_TOTAL).  The same ensemble then serves every statistic
 * below.
 *
 *   C, M, E, prec  as written by mp_propagate for this chunk
 *   d, bin_of_mode as for mp_binned_counts (host int32[M]); at most
 *                  MP_MAX_RUNS contiguous mode runs
 *   mode           MP_MARGINALS (n_dist = d) or MP_MARGINALS_AND_TOTAL
 *                  (n_dist = d + 1); MP_JOINT is rejected
 *   nq             device FP64, E * n_dist * 2, written: (Re, Im) n_q of chunk
 *                  sample k at nq[2 (k n_dist + q)]
 */
mp_status mp_occupations(int32_t M, int64_t E, const void* C, mp_precision prec, int32_t d,
                         const int32_t* bin_of_mode, mp_bin_mode mode, double* nq, void* stream);

/*
 * Normally ordered moments <:n_q^k:>, k = 1..kmax (main text, eq. moment):
 * per sample n_q^k, with the weight tanh n on odd orders for the
 * parity-projected estimator (the M = 2 projector weights) and no weight for
 * +P, summed per sub-ensemble in a fixed order.
 *
 *   n, nq          per-sample global n (mp_sample) and occupations
 *                  (mp_occupations) of the chunk's E samples, n_dist of them
 *   kmax           1..MP_MAX_MOMENTS
 *   n_sub, samples_per_sub, e0  as for mp_binned_counts
 *   acc            device FP64, n_sub * n_dist * kmax * 2 (re, im), layout
 *                  [s][q][k - 1]; caller-zeroed, added into
 * Means and sigma_T: mp_subensemble_stats(ncomp = 2, scale = 1).
 */
mp_status mp_moments_accumulate(int64_t E, const double* n, const double* nq, int32_t n_dist,
                                int32_t kmax, mp_estimator est, int32_t n_sub,
                                int64_t samples_per_sub, int64_t e0, double* acc, void* stream);

/*
 * Histogram of a per-sample observable (Appendix A, the binned probability
 * density of stochastic trajectories, eq. gen_probability_density): Re G of
 * distribution q at count m, G = g0 n_q^m e^{-n_q} / m! for the
 * parity-projected estimator (eq. c-number-variable for one group) or
 * n_q^m e^{-n_q} / m! for +P (eq. phase_space_projector), into n_bins bins
 * of width `width` starting at o_min.  Bin 0 counts values below o_min, bin
 * n_bins + 1 values at or above o_min + n_bins width and non-finite values.
 *
 *   hist           device FP64, n_sub * (n_bins + 2), layout [s][bin];
 *                  caller-zeroed, added into; the counts are exact integers
 * Densities and sigma_T: mp_subensemble_stats(ncomp = 1, scale = 1 / width).
 */
mp_status mp_observable_histogram(int64_t E, const double* n, const double* nq, int32_t n_dist,
                                  int32_t q, int32_t m, mp_estimator est, double o_min,
                                  double width, int32_t n_bins, int32_t n_sub,
                                  int64_t samples_per_sub, int64_t e0, double* hist,
                                  void* stream);

/*
 * Sub-ensemble statistics (Appendix A): for each of n_vals values,
 *   mean_v  = (1 / n_sub) sum_s scale acc[s][v] / samples_per_sub,
 *   sigma_v = sd over s of the real part of scale acc[s][v] / samples_per_sub,
 *             divided by sqrt(n_sub) (NaN when n_sub = 1).
 *   ncomp  1 (real acc, e.g. histograms) or 2 ((re, im) pairs)
 *   acc    device FP64, n_sub * n_vals * ncomp
 *   mean   device FP64, n_vals * ncomp;  sigma  device FP64, n_vals
 */
mp_status mp_subensemble_stats(int32_t n_sub, int64_t samples_per_sub, int64_t n_vals,
                               int32_t ncomp, double scale, const double* acc, double* mean,
                               double* sigma, void* stream);

/*
 * Normally ordered pair moments of single output modes, <:n_i n_j:> =
 * <a_i^+ a_j^+ a_i a_j> (main text, eq. moment, with every output mode taken
 * as its own group): per sample the mixed second derivative of the
 * generating function at z = 1 is n'_i n'_j, n'_i = alpha'_i beta'_i, with
 * weight 1 (an even order) for both estimators.  Two calls per chunk:
 *
 * mp_mode_occupations: n' of every (mode, sample) of a chunk.
 *   C, M, E, prec  as written by mp_propagate for this chunk (32-byte aligned)
 *   X              device, mp_mode_occupations_bytes(M, E, prec) bytes, FP64
 *                  for MP_FP64 and FP32 otherwise; column-major with
 *                  ld = round_up(M, 128): column k holds Re n'_{., k},
 *                  column E + k holds Im n'_{., k}; padding modes are zero
 *
 * mp_pair_correlations_accumulate: for every sub-ensemble s touched by the
 * chunk, acc[s][i][j] += sum over the chunk's samples k of s of
 * n'_ik n'_jk (complex, symmetric in i, j; both triangles are written).
 *   X              from mp_mode_occupations for this chunk (same M, E, prec)
 *   n_sub, samples_per_sub, e0  as for mp_binned_counts
 *   acc            device FP64, n_sub * M * M * 2 (re, im), layout [s][i][j],
 *                  caller-zeroed, added into (16-byte aligned)
 *   workspace      device, >= mp_pair_correlations_workspace(M, E, prec,
 *                  samples_per_sub, e0) bytes, 256-aligned; may be NULL when
 *                  that size is 0
 * FP64 runs FP64 FMAs; FP32 and the split precisions multiply FP32 values on
 * the FP32 matrix cores, summing in FP32 over the chunk's samples of one
 * sub-ensemble and in FP64 across chunks.  When a chunk has few (128 x 128
 * tile, sub-ensemble) items for the GPU, each is split into up to 8 pieces of
 * samples summed in FP32 into partial tiles in the workspace, and the pieces
 * are then added in order in FP64.  Either way each accumulator element has
 * one writer per call and the sums do not depend on scheduling.
 * Means and sigma_T: mp_subensemble_stats(n_vals = M * M, ncomp = 2, scale = 1).
 */
size_t mp_mode_occupations_bytes(int32_t M, int64_t E, mp_precision prec);
mp_status mp_mode_occupations(int32_t M, int64_t E, const void* C, mp_precision prec, void* X,
                              void* stream);
size_t mp_pair_correlations_workspace(int32_t M, int64_t E, mp_precision prec,
                                      int64_t samples_per_sub, int64_t e0);
mp_status mp_pair_correlations_accumulate(int32_t M, int64_t E, const void* X, mp_precision prec,
                                          int32_t n_sub, int64_t samples_per_sub, int64_t e0,
                                          double* acc, void* workspace, size_t ws_bytes,
                                          void* stream);

/*
 * Synchronous finiteness check of a device FP64 array, for estimates and
 * accumulators that must always be finite (every path evaluates its
 * exponentials in shifted, overflow-free forms; an overflow in a reduced-
 * precision path would show here).  Counts the NaN and infinite entries of
 * x[0, n) on `stream` into `scratch` (device, 8 bytes, caller-owned,
 * overwritten), waits for the stream, stores the count in *n_bad when n_bad
 * is not NULL, and returns MP_ERR_NONFINITE if it is nonzero.
 */
mp_status mp_check_finite(const double* x, int64_t n, int64_t* scratch, int64_t* n_bad,
                          void* stream);

/*
 * Diagnostics: the matrix cores' sustained rate on the current device.  One
 * workgroup of four waves (one per SIMD, the occupancy of the GEMM kernels)
 * per compute unit; every wave issues `iters` rounds of independent MFMAs (16
 * chains for FP16 and FP32, 32 for FP64: 256 accumulator registers, as in the
 * GEMMs) on register-resident operands, with no memory traffic in the loop.
 *   kind   0: v_mfma_f32_32x32x16_f16, 1: v_mfma_f32_32x32x2f32,
 *          2: v_mfma_f64_16x16x4f64, 3: per chain and round four
 *          v_mfma_f32_32x32x16_f16 and one v_mfma_scale_f32_32x32x64_f8f6f4
 *          on e4m3 operands (the MP_SPLIT1T_F8 GEMM's mix per 64-deep
 *          block); other values MP_ERR_ARG
 *   iters  >= 1
 *   sink   device FP64, one value per thread (256 per compute unit), caller-
 *          owned and overwritten (keeps the products live); smaller:
 *          MP_ERR_WORKSPACE
 *   flops  host, may be NULL: the launch's MFMA flop count (kind 3: the
 *          flops of both instructions, 262144 per chain and round)
 * Asynchronous on `stream`; time it with events on that stream.  Not part of
 * the estimator: it measures the ceiling the GEMMs run against (the clock the
 * part holds under a pure matrix load).
 */
mp_status mp_mfma_sustained(int32_t kind, int64_t iters, double* sink, size_t sink_bytes,
                            double* flops, void* stream);

/* ---------------------------------------------------------------- batching */

/* One network of a batched plan: E samples in n_sub sub-ensembles, noise
 * stream `net`, and the distributions to estimate.  d = 0: the total count
 * of all M outputs on the window [m_lo, m_lo + K).  d >= 1: the outputs
 * grouped by bin_of_mode with `mode`, one window per distribution in m_lo_b
 * and K_b (d entries, d + 1 for MP_MARGINALS_AND_TOTAL), exactly as for
 * mp_propagate_counts (joint grids of up to 4 bins); m_lo and K unused.  The
 * host arrays are read during mp_plan_create only. */
typedef struct {
  int32_t M;
  const double* T; /* device, complex M x M row-major interleaved (as mp_propagate) */
  const double* r; /* device FP64[M] */
  uint64_t seed;
  uint32_t net;
  int64_t E;       /* samples; a multiple of n_sub */
  int32_t n_sub;
  int32_t m_lo;
  int32_t K;
  int32_t d;                  /* 0: total counts on (m_lo, K); else bins, as above */
  mp_bin_mode mode;
  const int32_t* bin_of_mode; /* host int32[M], -1 = uncounted (d >= 1) */
  const int32_t* m_lo_b;      /* host int32, one per distribution (d >= 1) */
  const int32_t* K_b;         /* host int32, one per distribution (d >= 1) */
} mp_net_desc;

/*
 * Plan for many independent networks of uneven size (the batched form of the
 * matrix-P pass).  Creation copies r, packs every T (T and r may be freed
 * afterwards), allocates all buffers (the plan owns them), chooses the
 * grouped-GEMM work-list order, L2 prefetch and per-network tile width with a
 * timing autotuner (cached in the JSON file `tune_cache` when it is not NULL),
 * and captures the whole pass in a hipGraph: accumulators cleared by fill
 * kernels, sampling, ONE persistent grouped GEMM launch over all networks'
 * tiles per pass for the split precisions (MP_SPLIT_BF16, MP_SPLIT_FP16,
 * MP_SPLIT1_FP16, MP_SPLIT1T_FP16) with the occupation-fused epilogue of mp_propagate_counts
 * (FP32 plans run mp_propagate_counts per network, FP64 plans one GEMM writing
 * C and the counts from it per network), counts from the per-block occupation
 * partials
 * and inverse DFT per network; only FP64 plans hold a propagated-amplitude
 * buffer C.  Results equal those of mp_propagate_counts (FP32, split) or
 * mp_propagate + mp_binned_counts (FP64) on the same noise, bit for bit.
 * E must be <= chunk or a multiple of it; each pass covers `chunk` samples of
 * every network.  Synchronous; not thread-safe per plan.
 */
mp_status mp_plan_create(void** plan, int32_t n_net, const mp_net_desc* nets,
                         mp_precision prec, mp_estimator est, int64_t chunk,
                         const char* tune_cache);

/* Replays the captured pass after the work already queued on `stream`; the
 * stream waits for the replay.  Results are overwritten by each replay. */
mp_status mp_plan_launch(void* plan, void* stream);

/* Device pointers (owned by the plan) to network i's P_re, P_im and sigma:
 * K entries for d = 0, mp_acc_entries(d, mode, K_b) otherwise (the layout of
 * mp_counts_finalize). */
mp_status mp_plan_result(void* plan, int32_t i, const double** P_re, const double** P_im,
                         const double** sigma);

/* The autotuner's choice: work-list order (0: groups of 8 row x 4 column tiles
 * per XCD, 1: 4 x 8, 2: column-major without grouping) and whether the split
 * GEMM prefetches the next slab's lines into L2 (1) or not (0), the tuned GEMM
 * time of one pass (ms), and the plan's device bytes.  Any output pointer may
 * be NULL. */
mp_status mp_plan_info(void* plan, int32_t* order, int32_t* prefetch, double* tuned_ms,
                       size_t* device_bytes);

/* Tile of network i in the grouped GEMM: 128 modes by 128 or 64 samples (the
 * autotuner's per size class choice for MP_SPLIT_BF16 and MP_SPLIT_FP16; both
 * give the same bits), 128 x 128 for the one-sided splits, 0 x 0 for plans without
 * a grouped launch (FP64, FP32).  i outside [0, n_net): MP_ERR_ARG.  Either
 * output pointer may be NULL. */
mp_status mp_plan_tile(void* plan, int32_t i, int32_t* modes, int32_t* samples);

/* Waits for the plan's stream and frees everything the plan owns. */
mp_status mp_plan_destroy(void* plan);

/* ---------------------------------------------------------------- surrogate */

/*
 * Small MLP trained on method outputs (sweep parameters -> moments of a bin's
 * count distribution) to screen parameter sweeps; the method checks and
 * replaces its predictions.  Layer l maps width[l] -> width[l+1] as
 * y = x W_l + b_l with W_l row-major (width[l] x width[l+1]) followed by b_l,
 * layers concatenated in one FP32 vector `params`; SiLU on hidden layers,
 * linear output.  Forward and backward read weights from `w16`, a BF16 copy
 * of params (same indexing), and accumulate in FP32.  All arrays are device
 * memory; X is batch x width[0], Y batch x width[n_layers], row-major FP32.
 * Widths <= 1024, n_layers <= MP_MLP_MAX_LAYERS.
 */
#define MP_MLP_MAX_LAYERS 8
typedef struct {
  int32_t n_layers;
  int32_t width[MP_MLP_MAX_LAYERS + 1];
} mp_mlp_shape;

int64_t mp_mlp_param_count(const mp_mlp_shape* shape);
size_t mp_mlp_workspace(const mp_mlp_shape* shape, int32_t batch);

/* w16 = BF16(params), round to nearest even. */
mp_status mp_mlp_round(const mp_mlp_shape* shape, const float* params, uint16_t* w16,
                       void* stream);

/* Y = MLP(X). */
mp_status mp_mlp_forward(const mp_mlp_shape* shape, const uint16_t* w16, const float* params,
                         const float* X, int32_t batch, float* Y, void* workspace,
                         size_t ws_bytes, void* stream);

/* loss = mean over all entries of (MLP(X) - Y)^2 (device float[1]) and its
 * gradient with respect to every parameter (grads, FP32, params' layout). */
mp_status mp_mlp_loss_grad(const mp_mlp_shape* shape, const uint16_t* w16, const float* params,
                           const float* X, const float* Y, int32_t batch, float* grads,
                           float* loss, void* workspace, size_t ws_bytes, void* stream);

/* One Adam step (bias-corrected, step >= 1) with decoupled weight decay on
 * params with moments m, v:
 *   p -= lr * (m_hat / (sqrt(v_hat) + eps) + weight_decay * p);
 * refreshes w16. */
mp_status mp_mlp_adam(const mp_mlp_shape* shape, float* params, const float* grads, float* m,
                      float* v, uint16_t* w16, float lr, float beta1, float beta2, float eps,
                      float weight_decay, int32_t step, void* stream);

/* Message of the calling thread's last non-MP_OK status ("" if none). */
const char* mp_last_error(void);

/* Library version string. */
const char* mp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPGBS_H */
