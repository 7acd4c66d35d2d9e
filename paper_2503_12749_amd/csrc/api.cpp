// C ABI of libmpgbs: host-side argument validation and dispatch to the
// kernels of sample.hip, propagate.hip and counts.hip.  Every entry point
// validates synchronously, enqueues nothing on failure, and records a
// thread-local message for mp_last_error().
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"

namespace mp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

mp_status sample_launch(int32_t M, int64_t g0, int64_t E, const double* r, uint64_t seed,
                        uint32_t net, mp_precision prec, void* ab, double* n_out,
                        hipStream_t stream);
size_t propagate_workspace(int32_t M, mp_precision prec);
mp_status pack_launch(int32_t M, const double* T, mp_precision prec, void* packed,
                      hipStream_t stream);
mp_status gemm_packed_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                             const void* ab, void* C, hipStream_t stream);
mp_status propagate_launch(int32_t M, int64_t E, const double* T, mp_precision prec,
                           const void* ab, void* C, void* ws, hipStream_t stream);
int64_t acc_entries(int32_t d, mp_bin_mode mode, const int32_t* K);
size_t binned_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int64_t E, int32_t n_sub,
                        int64_t ns, int64_t e0);
mp_status binned_counts_launch(int32_t M, int64_t E, const void* C, const double* n,
                               mp_precision prec, mp_estimator est, int32_t d,
                               const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                               const int32_t* K, int32_t n_sub, int64_t ns, int64_t e0,
                               double* acc, void* ws, size_t ws_bytes, hipStream_t stream);
mp_status counts_finalize_launch(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                                 int64_t ns, const double* acc, double* P_re, double* P_im,
                                 double* sigma, void* ws, size_t ws_bytes, hipStream_t stream);
size_t finalize_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub);
size_t propagate_counts_workspace(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                                  mp_bin_mode mode, const int32_t* K, int32_t n_sub, int64_t ns,
                                  int64_t e0);
mp_status propagate_counts_launch(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                                  const void* ab, const double* n, const void* packed, int32_t d,
                                  const int32_t* bin_of_mode, mp_bin_mode mode,
                                  const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                  int64_t ns, int64_t e0, double* acc, void* ws, size_t ws_bytes,
                                  hipStream_t stream);
size_t bilinear_workspace(int32_t M);
size_t bilinear_packed_bytes(int32_t M, mp_precision prec);
mp_status bilinear_pack_launch(int32_t M, const double* T, const int32_t* in_s,
                               mp_precision prec, void* packed, void* scratch, hipStream_t stream);
mp_status propagate_counts_bilinear_launch(int32_t M, int64_t E, mp_precision prec,
                                           mp_estimator est, const void* ab, const double* n,
                                           const void* packed, const int32_t* m_lo,
                                           const int32_t* K, int32_t n_sub, int64_t ns,
                                           int64_t e0, double* acc, void* ws, size_t ws_bytes,
                                           hipStream_t stream);
mp_status propagate_counts_noalloc_launch(int32_t M, int64_t E, mp_precision prec,
                                          mp_estimator est, const void* ab, const double* n,
                                          const void* packed, int32_t d,
                                          const int32_t* bin_of_mode, mp_bin_mode mode,
                                          const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                          int64_t ns, int64_t e0, double* acc,
                                          hipStream_t stream);
mp_status occupations_launch(int32_t M, int64_t E, const void* C, mp_precision prec, int32_t d,
                             const int32_t* bin_of_mode, mp_bin_mode mode, double* nq,
                             hipStream_t stream);
mp_status moments_launch(int64_t E, const double* n, const double* nq, int32_t n_dist,
                         int32_t kmax, mp_estimator est, int64_t ns, int64_t e0, double* acc,
                         hipStream_t stream);
mp_status histogram_launch(int64_t E, const double* n, const double* nq, int32_t n_dist, int32_t q,
                           int32_t m, mp_estimator est, double o_min, double width,
                           int32_t n_bins, int64_t ns, int64_t e0, double* hist,
                           hipStream_t stream);
mp_status subensemble_stats_launch(int32_t n_sub, int64_t ns, int64_t n_vals, int32_t ncomp,
                                   double scale, const double* acc, double* mean, double* sigma,
                                   hipStream_t stream);

int64_t mlp_param_count(const mp_mlp_shape* s);
mp_status check_finite_launch(const double* x, int64_t n, int64_t* scratch, int64_t* n_bad,
                              hipStream_t stream);
size_t mode_occupations_bytes(int32_t M, int64_t E, mp_precision prec);
mp_status mode_occupations_launch(int32_t M, int64_t E, const void* C, mp_precision prec, void* X,
                                  hipStream_t stream);
size_t pair_corr_workspace(int32_t M, int64_t E, mp_precision prec, int64_t ns, int64_t e0);
mp_status pair_corr_launch(int32_t M, int64_t E, const void* X, mp_precision prec, int64_t ns,
                           int64_t e0, double* acc, void* ws, size_t ws_bytes,
                           hipStream_t stream);
size_t mlp_workspace(const mp_mlp_shape* s, int32_t batch);
mp_status mlp_forward(const mp_mlp_shape* s, const uint16_t* w16, const float* params,
                      const float* X, int32_t batch, float* Y, void* ws, hipStream_t st);
mp_status mlp_loss_grad(const mp_mlp_shape* s, const uint16_t* w16, const float* params,
                        const float* X, const float* Y, int32_t batch, float* grads, float* loss,
                        void* ws, hipStream_t st);
mp_status mlp_adam_launch(int64_t n, float* params, const float* grads, float* m, float* v,
                          uint16_t* w16, float lr, float b1, float b2, float eps, float wd,
                          int32_t step, hipStream_t st);
mp_status mlp_round_launch(int64_t n, const float* params, uint16_t* w16, hipStream_t st);

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

static bool valid_shape(const mp_mlp_shape* s) {
  if (!s || s->n_layers < 1 || s->n_layers > MP_MLP_MAX_LAYERS) return false;
  for (int l = 0; l <= s->n_layers; ++l)
    if (s->width[l] < 1 || s->width[l] > 1024) return false;
  return true;
}

static int n_dist_of(int32_t d, mp_bin_mode mode) {
  if (mode == MP_JOINT) return d;
  return d + (mode == MP_MARGINALS_AND_TOTAL ? 1 : 0);
}

}  // namespace mp

using namespace mp;

extern "C" {

int64_t mp_ld_modes(int32_t M) { return M < 1 ? -1 : ld_modes(M); }

size_t mp_ab_bytes(int32_t M, int64_t E, mp_precision prec) {
  if (M < 1 || E < 1 || !valid_prec(prec)) return 0;
  return (size_t)ld_modes(M) * (size_t)ab_columns(E, prec) * elem_bytes_ab(prec);
}

size_t mp_c_bytes(int32_t M, int64_t E, mp_precision prec) {
  if (M < 1 || E < 1 || !valid_prec(prec)) return 0;
  return (size_t)(2 * ld_modes(M)) * (size_t)(2 * E) * elem_bytes_c(prec);
}

mp_status mp_sample(int32_t M, int64_t g0, int64_t E, const double* r, uint64_t seed,
                    uint32_t net, mp_precision prec, void* ab, double* n_out, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1, MP_ERR_ARG, "mp_sample: M = %d must be >= 1", M);
  MP_CHECK_ARG(E >= 1, MP_ERR_ARG, "mp_sample: E = %lld must be >= 1", (long long)E);
  MP_CHECK_ARG(g0 >= 0, MP_ERR_ARG, "mp_sample: g0 = %lld must be >= 0", (long long)g0);
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_sample: unknown precision %d", (int)prec);
  MP_CHECK_ARG(r && ab && n_out, MP_ERR_ARG, "mp_sample: null pointer argument");
  MP_CHECK_ARG(aligned(ab, 16), MP_ERR_ARG, "mp_sample: ab must be 16-byte aligned");
  return sample_launch(M, g0, E, r, seed, net, prec, ab, n_out, (hipStream_t)stream);
}

size_t mp_propagate_workspace(int32_t M, mp_precision prec) {
  if (M < 1 || !valid_prec(prec)) return 0;
  return propagate_workspace(M, prec);
}

mp_status mp_propagate(int32_t M, int64_t E, const double* T, mp_precision prec, const void* ab,
                       void* C, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1, MP_ERR_ARG, "mp_propagate: M = %d must be >= 1", M);
  MP_CHECK_ARG(E >= 1, MP_ERR_ARG, "mp_propagate: E = %lld must be >= 1", (long long)E);
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_propagate: unknown precision %d", (int)prec);
  MP_CHECK_ARG(T && ab && C, MP_ERR_ARG, "mp_propagate: null pointer argument");
  MP_CHECK_ARG(aligned(ab, 16) && aligned(C, 16), MP_ERR_ARG,
               "mp_propagate: ab and C must be 16-byte aligned");
  const size_t need = propagate_workspace(M, prec);
  MP_CHECK_ARG(workspace && ws_bytes >= need && aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_propagate: workspace of %zu bytes (256-aligned) needed, %zu given", need,
               ws_bytes);
  return propagate_launch(M, E, T, prec, ab, C, workspace, (hipStream_t)stream);
}

mp_status mp_pack_transmission(int32_t M, const double* T, mp_precision prec, void* workspace,
                               size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1, MP_ERR_ARG, "mp_pack_transmission: M = %d must be >= 1", M);
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_pack_transmission: unknown precision %d",
               (int)prec);
  MP_CHECK_ARG(T, MP_ERR_ARG, "mp_pack_transmission: null pointer argument");
  const size_t need = propagate_workspace(M, prec);
  MP_CHECK_ARG(workspace && ws_bytes >= need && aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_pack_transmission: workspace of %zu bytes (256-aligned) needed, %zu given",
               need, ws_bytes);
  return pack_launch(M, T, prec, workspace, (hipStream_t)stream);
}

mp_status mp_propagate_packed(int32_t M, int64_t E, mp_precision prec, const void* ab, void* C,
                              const void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1, MP_ERR_ARG, "mp_propagate_packed: M = %d must be >= 1", M);
  MP_CHECK_ARG(E >= 1, MP_ERR_ARG, "mp_propagate_packed: E = %lld must be >= 1", (long long)E);
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_propagate_packed: unknown precision %d",
               (int)prec);
  MP_CHECK_ARG(ab && C, MP_ERR_ARG, "mp_propagate_packed: null pointer argument");
  MP_CHECK_ARG(aligned(ab, 16) && aligned(C, 16), MP_ERR_ARG,
               "mp_propagate_packed: ab and C must be 16-byte aligned");
  const size_t need = propagate_workspace(M, prec);
  MP_CHECK_ARG(workspace && ws_bytes >= need && aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_propagate_packed: packed workspace of %zu bytes (256-aligned) needed, %zu given",
               need, ws_bytes);
  return gemm_packed_launch(M, E, workspace, prec, ab, C, (hipStream_t)stream);
}

int64_t mp_acc_entries(int32_t d, mp_bin_mode mode, const int32_t* K) {
  if (!K || d < 1 || d > MP_MAX_BINS || mode < MP_JOINT || mode > MP_MARGINALS_AND_TOTAL) return -1;
  if (mode == MP_JOINT && d > 4) return -1;
  const int nd = n_dist_of(d, mode);
  const int kmax = mode != MP_JOINT || d == 1 ? 65536 : (d == 2 ? 4096 : 1024);
  for (int q = 0; q < nd; ++q)
    if (K[q] < 1 || K[q] > kmax) return -1;
  return acc_entries(d, mode, K);
}

size_t mp_binned_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int64_t E,
                           int32_t n_sub, int64_t samples_per_sub, int64_t e0) {
  if (mp_acc_entries(d, mode, K) < 0) return 0;
  return binned_workspace(d, mode, K, E, n_sub, samples_per_sub, e0);
}

mp_status mp_binned_counts(int32_t M, int64_t E, const void* C, const double* n,
                           mp_precision prec, mp_estimator est, int32_t d,
                           const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                           const int32_t* K, int32_t n_sub, int64_t samples_per_sub, int64_t e0,
                           double* acc, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1 && E >= 1, MP_ERR_ARG, "mp_binned_counts: M and E must be >= 1");
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_binned_counts: unknown precision %d", (int)prec);
  MP_CHECK_ARG(est == MP_MATRIX_P || est == MP_PLUS_P, MP_ERR_ARG,
               "mp_binned_counts: unknown estimator %d", (int)est);
  MP_CHECK_ARG(d >= 1 && d <= MP_MAX_BINS, MP_ERR_ARG, "mp_binned_counts: d = %d outside [1, %d]",
               d, MP_MAX_BINS);
  MP_CHECK_ARG(mode >= MP_JOINT && mode <= MP_MARGINALS_AND_TOTAL, MP_ERR_ARG,
               "mp_binned_counts: unknown bin mode %d", (int)mode);
  MP_CHECK_ARG(C && n && bin_of_mode && m_lo && K && acc, MP_ERR_ARG,
               "mp_binned_counts: null pointer argument");
  MP_CHECK_ARG(n_sub >= 1 && samples_per_sub >= 1 && e0 >= 0, MP_ERR_ARG,
               "mp_binned_counts: n_sub, samples_per_sub must be >= 1 and e0 >= 0");
  for (int j = 0; j < M; ++j)
    MP_CHECK_ARG(bin_of_mode[j] >= -1 && bin_of_mode[j] < d, MP_ERR_ARG,
                 "mp_binned_counts: bin_of_mode[%d] = %d outside [-1, %d)", j, bin_of_mode[j], d);
  const int nd = n_dist_of(d, mode);
  for (int q = 0; q < nd; ++q) {
    MP_CHECK_ARG(K[q] >= 1 && K[q] <= 65536, MP_ERR_ARG,
                 "mp_binned_counts: K[%d] = %d outside [1, 65536]", q, K[q]);
    MP_CHECK_ARG(m_lo[q] >= 0, MP_ERR_ARG, "mp_binned_counts: m_lo[%d] = %d < 0", q, m_lo[q]);
  }
  MP_CHECK_ARG(mode != MP_JOINT || d <= 4, MP_ERR_UNSUPPORTED,
               "mp_binned_counts: joint distributions need d <= 4");
  MP_CHECK_ARG(aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_binned_counts: workspace must be 256-byte aligned");
  return binned_counts_launch(M, E, C, n, prec, est, d, bin_of_mode, mode, m_lo, K, n_sub,
                              samples_per_sub, e0, acc, workspace, ws_bytes, (hipStream_t)stream);
}

// Shared argument checks of the fused and unfused counting calls.
static mp_status counts_args(const char* who, int32_t M, int64_t E, mp_estimator est, int32_t d,
                             const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                             const int32_t* K, int32_t n_sub, int64_t samples_per_sub,
                             int64_t e0) {
  MP_CHECK_ARG(M >= 1 && E >= 1, MP_ERR_ARG, "%s: M and E must be >= 1", who);
  MP_CHECK_ARG(est == MP_MATRIX_P || est == MP_PLUS_P, MP_ERR_ARG, "%s: unknown estimator %d", who,
               (int)est);
  MP_CHECK_ARG(d >= 1 && d <= MP_MAX_BINS, MP_ERR_ARG, "%s: d = %d outside [1, %d]", who, d,
               MP_MAX_BINS);
  MP_CHECK_ARG(mode >= MP_JOINT && mode <= MP_MARGINALS_AND_TOTAL, MP_ERR_ARG,
               "%s: unknown bin mode %d", who, (int)mode);
  MP_CHECK_ARG(bin_of_mode && m_lo && K, MP_ERR_ARG, "%s: null pointer argument", who);
  MP_CHECK_ARG(n_sub >= 1 && samples_per_sub >= 1 && e0 >= 0, MP_ERR_ARG,
               "%s: n_sub, samples_per_sub must be >= 1 and e0 >= 0", who);
  for (int j = 0; j < M; ++j)
    MP_CHECK_ARG(bin_of_mode[j] >= -1 && bin_of_mode[j] < d, MP_ERR_ARG,
                 "%s: bin_of_mode[%d] = %d outside [-1, %d)", who, j, bin_of_mode[j], d);
  const int nd = n_dist_of(d, mode);
  for (int q = 0; q < nd; ++q) {
    MP_CHECK_ARG(K[q] >= 1 && K[q] <= 65536, MP_ERR_ARG, "%s: K[%d] = %d outside [1, 65536]", who,
                 q, K[q]);
    MP_CHECK_ARG(m_lo[q] >= 0, MP_ERR_ARG, "%s: m_lo[%d] = %d < 0", who, q, m_lo[q]);
  }
  return MP_OK;
}

size_t mp_propagate_counts_workspace(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                                     mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                                     int64_t samples_per_sub, int64_t e0) {
  std::vector<int32_t> m_lo(MP_MAX_BINS + 1, 0);
  if (counts_args("mp_propagate_counts_workspace", M, E, MP_MATRIX_P, d, bin_of_mode, mode,
                  m_lo.data(), K, n_sub, samples_per_sub, e0) != MP_OK ||
      (mode == MP_JOINT && d > 4))
    return 0;
  return propagate_counts_workspace(M, E, d, bin_of_mode, mode, K, n_sub, samples_per_sub, e0);
}

mp_status mp_propagate_counts(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                              const void* ab, const double* n, const void* packed,
                              size_t packed_bytes, int32_t d, const int32_t* bin_of_mode,
                              mp_bin_mode mode, const int32_t* m_lo, const int32_t* K,
                              int32_t n_sub, int64_t samples_per_sub, int64_t e0, double* acc,
                              void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  const mp_status st = counts_args("mp_propagate_counts", M, E, est, d, bin_of_mode, mode, m_lo, K,
                                   n_sub, samples_per_sub, e0);
  if (st != MP_OK) return st;
  MP_CHECK_ARG(prec == MP_FP32 || prec == MP_SPLIT_BF16 || prec == MP_SPLIT_FP16 ||
                   prec == MP_SPLIT1_FP16 || pair_columns(prec),
               MP_ERR_UNSUPPORTED,
               "mp_propagate_counts: precision %d is not fused (FP32 and split precisions are)",
               (int)prec);
  MP_CHECK_ARG(mode != MP_JOINT || d <= 4, MP_ERR_UNSUPPORTED,
               "mp_propagate_counts: joint distributions need d <= 4");
  MP_CHECK_ARG(ab && n && packed && acc, MP_ERR_ARG, "mp_propagate_counts: null pointer argument");
  MP_CHECK_ARG(aligned(ab, 16), MP_ERR_ARG, "mp_propagate_counts: ab must be 16-byte aligned");
  const size_t need_packed = propagate_workspace(M, prec);
  MP_CHECK_ARG(packed_bytes >= need_packed && aligned(packed, 256), MP_ERR_WORKSPACE,
               "mp_propagate_counts: packed operand of %zu bytes (256-aligned) needed, %zu given",
               need_packed, packed_bytes);
  MP_CHECK_ARG(aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_propagate_counts: workspace must be 256-byte aligned");
  return propagate_counts_launch(M, E, prec, est, ab, n, packed, d, bin_of_mode, mode, m_lo, K,
                                 n_sub, samples_per_sub, e0, acc, workspace, ws_bytes,
                                 (hipStream_t)stream);
}

size_t mp_bilinear_workspace(int32_t M) { return M >= 1 ? bilinear_workspace(M) : 0; }

size_t mp_bilinear_packed_bytes(int32_t M) {
  return M >= 1 ? bilinear_packed_bytes(M, MP_SPLIT1T_F8) : 0;
}

mp_status mp_pack_bilinear(int32_t M, const double* T, const int32_t* bin_of_mode,
                           mp_precision prec, void* packed, size_t packed_bytes, void* scratch,
                           size_t scratch_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1, MP_ERR_ARG, "mp_pack_bilinear: M must be >= 1");
  MP_CHECK_ARG(prec == MP_SPLIT1T_F8, MP_ERR_UNSUPPORTED,
               "mp_pack_bilinear: precision %d (MP_SPLIT1T_F8 only)", (int)prec);
  MP_CHECK_ARG(T && bin_of_mode && packed && scratch, MP_ERR_ARG,
               "mp_pack_bilinear: null pointer argument");
  for (int j = 0; j < M; ++j)
    MP_CHECK_ARG(bin_of_mode[j] == 0 || bin_of_mode[j] == -1, MP_ERR_ARG,
                 "mp_pack_bilinear: bin_of_mode[%d] = %d (0: in the set, -1: not)", j,
                 bin_of_mode[j]);
  const size_t need_packed = bilinear_packed_bytes(M, prec);
  MP_CHECK_ARG(packed_bytes >= need_packed && aligned(packed, 256), MP_ERR_WORKSPACE,
               "mp_pack_bilinear: packed operand of %zu bytes (256-aligned) needed, %zu given",
               need_packed, packed_bytes);
  const size_t need_scratch = bilinear_workspace(M);
  MP_CHECK_ARG(scratch_bytes >= need_scratch && aligned(scratch, 256), MP_ERR_WORKSPACE,
               "mp_pack_bilinear: scratch of %zu bytes (256-aligned) needed, %zu given",
               need_scratch, scratch_bytes);
  const mp_status st =
      bilinear_pack_launch(M, T, bin_of_mode, prec, packed, scratch, (hipStream_t)stream);
  if (st != MP_OK) return st;
  // the mode set is copied from host memory on the stream: return only once
  // the stream has passed the packing, whatever memory the caller's array is
  const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    set_error("mp_pack_bilinear: %s", hipGetErrorString(e));
    return MP_ERR_HIP;
  }
  return MP_OK;
}

mp_status mp_propagate_counts_bilinear(int32_t M, int64_t E, mp_precision prec,
                                       mp_estimator est, const void* ab, const double* n,
                                       const void* packed, size_t packed_bytes,
                                       const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                       int64_t samples_per_sub, int64_t e0, double* acc,
                                       void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1, MP_ERR_ARG, "mp_propagate_counts_bilinear: M must be >= 1");
  const std::vector<int32_t> all(M, 0);
  const mp_status st = counts_args("mp_propagate_counts_bilinear", M, E, est, 1, all.data(),
                                   MP_JOINT, m_lo, K, n_sub, samples_per_sub, e0);
  if (st != MP_OK) return st;
  MP_CHECK_ARG(prec == MP_SPLIT1T_F8, MP_ERR_UNSUPPORTED,
               "mp_propagate_counts_bilinear: precision %d (MP_SPLIT1T_F8 only)", (int)prec);
  MP_CHECK_ARG(ab && n && packed && acc, MP_ERR_ARG,
               "mp_propagate_counts_bilinear: null pointer argument");
  MP_CHECK_ARG(aligned(ab, 16), MP_ERR_ARG, "mp_propagate_counts_bilinear: ab must be 16-byte aligned");
  const size_t need_packed = bilinear_packed_bytes(M, prec);
  MP_CHECK_ARG(packed_bytes >= need_packed && aligned(packed, 256), MP_ERR_WORKSPACE,
               "mp_propagate_counts_bilinear: packed operand of %zu bytes (256-aligned) needed, "
               "%zu given", need_packed, packed_bytes);
  MP_CHECK_ARG(aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_propagate_counts_bilinear: workspace must be 256-byte aligned");
  return propagate_counts_bilinear_launch(M, E, prec, est, ab, n, packed, m_lo, K, n_sub,
                                          samples_per_sub, e0, acc, workspace, ws_bytes,
                                          (hipStream_t)stream);
}

mp_status mp_propagate_counts_noalloc(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                                      const void* ab, const double* n, const void* packed,
                                      size_t packed_bytes, int32_t d, const int32_t* bin_of_mode,
                                      mp_bin_mode mode, const int32_t* m_lo, const int32_t* K,
                                      int32_t n_sub, int64_t samples_per_sub, int64_t e0,
                                      double* acc, void* stream) {
  clear_error();
  const mp_status st = counts_args("mp_propagate_counts_noalloc", M, E, est, d, bin_of_mode, mode,
                                   m_lo, K, n_sub, samples_per_sub, e0);
  if (st != MP_OK) return st;
  MP_CHECK_ARG(prec == MP_FP32 || prec == MP_SPLIT_BF16 || prec == MP_SPLIT_FP16 ||
                   prec == MP_SPLIT1_FP16 || pair_columns(prec),
               MP_ERR_UNSUPPORTED,
               "mp_propagate_counts_noalloc: precision %d is not fused (FP32 and split "
               "precisions are)", (int)prec);
  MP_CHECK_ARG(ab && n && packed && acc, MP_ERR_ARG,
               "mp_propagate_counts_noalloc: null pointer argument");
  MP_CHECK_ARG(aligned(ab, 16), MP_ERR_ARG, "mp_propagate_counts_noalloc: ab must be 16-byte aligned");
  const size_t need_packed = propagate_workspace(M, prec);
  MP_CHECK_ARG(packed_bytes >= need_packed && aligned(packed, 256), MP_ERR_WORKSPACE,
               "mp_propagate_counts_noalloc: packed operand of %zu bytes (256-aligned) needed, "
               "%zu given", need_packed, packed_bytes);
  return propagate_counts_noalloc_launch(M, E, prec, est, ab, n, packed, d, bin_of_mode, mode,
                                         m_lo, K, n_sub, samples_per_sub, e0, acc,
                                         (hipStream_t)stream);
}

size_t mp_finalize_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub) {
  if (mp_acc_entries(d, mode, K) < 0 || n_sub < 1) return 0;
  return finalize_workspace(d, mode, K, n_sub);
}

mp_status mp_counts_finalize(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                             int64_t samples_per_sub, const double* acc, double* P_re,
                             double* P_im, double* sigma, void* workspace, size_t ws_bytes,
                             void* stream) {
  clear_error();
  MP_CHECK_ARG(mp_acc_entries(d, mode, K) > 0, MP_ERR_ARG,
               "mp_counts_finalize: invalid bin layout (d = %d, mode = %d)", d, (int)mode);
  MP_CHECK_ARG(n_sub >= 1 && samples_per_sub >= 1, MP_ERR_ARG,
               "mp_counts_finalize: n_sub and samples_per_sub must be >= 1");
  MP_CHECK_ARG(acc && P_re && sigma, MP_ERR_ARG, "mp_counts_finalize: null pointer argument");
  MP_CHECK_ARG(workspace == nullptr || aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_counts_finalize: workspace must be 256-byte aligned");
  return counts_finalize_launch(d, mode, K, n_sub, samples_per_sub, acc, P_re, P_im, sigma,
                                workspace, ws_bytes, (hipStream_t)stream);
}

mp_status mp_occupations(int32_t M, int64_t E, const void* C, mp_precision prec, int32_t d,
                         const int32_t* bin_of_mode, mp_bin_mode mode, double* nq, void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1 && E >= 1, MP_ERR_ARG, "mp_occupations: M and E must be >= 1");
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_occupations: unknown precision %d", (int)prec);
  MP_CHECK_ARG(d >= 1 && d <= MP_MAX_BINS, MP_ERR_ARG, "mp_occupations: d = %d outside [1, %d]", d,
               MP_MAX_BINS);
  MP_CHECK_ARG(mode == MP_MARGINALS || mode == MP_MARGINALS_AND_TOTAL, MP_ERR_ARG,
               "mp_occupations: mode must be MP_MARGINALS or MP_MARGINALS_AND_TOTAL");
  MP_CHECK_ARG(C && bin_of_mode && nq, MP_ERR_ARG, "mp_occupations: null pointer argument");
  MP_CHECK_ARG(aligned(C, 16) && aligned(nq, 8), MP_ERR_ARG,
               "mp_occupations: C must be 16-byte and nq 8-byte aligned");
  for (int j = 0; j < M; ++j)
    MP_CHECK_ARG(bin_of_mode[j] >= -1 && bin_of_mode[j] < d, MP_ERR_ARG,
                 "mp_occupations: bin_of_mode[%d] = %d outside [-1, %d)", j, bin_of_mode[j], d);
  return occupations_launch(M, E, C, prec, d, bin_of_mode, mode, nq, (hipStream_t)stream);
}

// Shared checks of the per-sample statistics calls.
static bool sample_stat_args(const char* who, int64_t E, const double* n, const double* nq,
                             int32_t n_dist, mp_estimator est, int32_t n_sub, int64_t ns,
                             int64_t e0, const double* out) {
  if (E < 1 || !n || !nq || !out) {
    set_error("%s: E must be >= 1 and pointers non-null", who);
    return false;
  }
  if (n_dist < 1 || n_dist > MP_MAX_BINS + 1) {
    set_error("%s: n_dist = %d outside [1, %d]", who, n_dist, MP_MAX_BINS + 1);
    return false;
  }
  if (est != MP_MATRIX_P && est != MP_PLUS_P) {
    set_error("%s: unknown estimator %d", who, (int)est);
    return false;
  }
  if (n_sub < 1 || ns < 1 || e0 < 0 || (e0 + E - 1) / ns >= n_sub) {
    set_error("%s: samples [%lld, %lld) do not fit n_sub = %d sub-ensembles of %lld", who,
              (long long)e0, (long long)(e0 + E), n_sub, (long long)ns);
    return false;
  }
  return true;
}

mp_status mp_moments_accumulate(int64_t E, const double* n, const double* nq, int32_t n_dist,
                                int32_t kmax, mp_estimator est, int32_t n_sub,
                                int64_t samples_per_sub, int64_t e0, double* acc, void* stream) {
  clear_error();
  if (!sample_stat_args("mp_moments_accumulate", E, n, nq, n_dist, est, n_sub, samples_per_sub, e0,
                        acc))
    return MP_ERR_ARG;
  MP_CHECK_ARG(kmax >= 1 && kmax <= MP_MAX_MOMENTS, MP_ERR_ARG,
               "mp_moments_accumulate: kmax = %d outside [1, %d]", kmax, MP_MAX_MOMENTS);
  return moments_launch(E, n, nq, n_dist, kmax, est, samples_per_sub, e0, acc, (hipStream_t)stream);
}

mp_status mp_observable_histogram(int64_t E, const double* n, const double* nq, int32_t n_dist,
                                  int32_t q, int32_t m, mp_estimator est, double o_min,
                                  double width, int32_t n_bins, int32_t n_sub,
                                  int64_t samples_per_sub, int64_t e0, double* hist,
                                  void* stream) {
  clear_error();
  if (!sample_stat_args("mp_observable_histogram", E, n, nq, n_dist, est, n_sub, samples_per_sub,
                        e0, hist))
    return MP_ERR_ARG;
  MP_CHECK_ARG(q >= 0 && q < n_dist && m >= 0, MP_ERR_ARG,
               "mp_observable_histogram: q = %d outside [0, %d) or m = %d < 0", q, n_dist, m);
  MP_CHECK_ARG(n_bins >= 1 && width > 0.0 && std::isfinite(width) && std::isfinite(o_min),
               MP_ERR_ARG, "mp_observable_histogram: need n_bins >= 1 and finite o_min, width > 0");
  return histogram_launch(E, n, nq, n_dist, q, m, est, o_min, width, n_bins, samples_per_sub, e0,
                          hist, (hipStream_t)stream);
}

mp_status mp_subensemble_stats(int32_t n_sub, int64_t samples_per_sub, int64_t n_vals,
                               int32_t ncomp, double scale, const double* acc, double* mean,
                               double* sigma, void* stream) {
  clear_error();
  MP_CHECK_ARG(n_sub >= 1 && samples_per_sub >= 1 && n_vals >= 1, MP_ERR_ARG,
               "mp_subensemble_stats: n_sub, samples_per_sub and n_vals must be >= 1");
  MP_CHECK_ARG(ncomp == 1 || ncomp == 2, MP_ERR_ARG, "mp_subensemble_stats: ncomp = %d not 1 or 2",
               ncomp);
  MP_CHECK_ARG(acc && mean && sigma && std::isfinite(scale), MP_ERR_ARG,
               "mp_subensemble_stats: null pointer or non-finite scale");
  return subensemble_stats_launch(n_sub, samples_per_sub, n_vals, ncomp, scale, acc, mean, sigma,
                                  (hipStream_t)stream);
}

mp_status mp_check_finite(const double* x, int64_t n, int64_t* scratch, int64_t* n_bad,
                          void* stream) {
  clear_error();
  MP_CHECK_ARG(x && scratch && n >= 1, MP_ERR_ARG,
               "mp_check_finite: x and scratch must be non-null and n >= 1");
  MP_CHECK_ARG(aligned(x, 8) && aligned(scratch, 8), MP_ERR_ARG,
               "mp_check_finite: x and scratch must be 8-byte aligned");
  return check_finite_launch(x, n, scratch, n_bad, (hipStream_t)stream);
}

size_t mp_mode_occupations_bytes(int32_t M, int64_t E, mp_precision prec) {
  return (M >= 1 && E >= 1 && valid_prec(prec)) ? mode_occupations_bytes(M, E, prec) : 0;
}

mp_status mp_mode_occupations(int32_t M, int64_t E, const void* C, mp_precision prec, void* X,
                              void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1 && E >= 1, MP_ERR_ARG, "mp_mode_occupations: M and E must be >= 1");
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_mode_occupations: unknown precision %d",
               (int)prec);
  MP_CHECK_ARG(C && X, MP_ERR_ARG, "mp_mode_occupations: null pointer argument");
  MP_CHECK_ARG(aligned(C, 32) && aligned(X, 32), MP_ERR_ARG,
               "mp_mode_occupations: C and X must be 32-byte aligned");
  return mode_occupations_launch(M, E, C, prec, X, (hipStream_t)stream);
}

size_t mp_pair_correlations_workspace(int32_t M, int64_t E, mp_precision prec,
                                      int64_t samples_per_sub, int64_t e0) {
  if (M < 1 || E < 1 || !valid_prec(prec) || samples_per_sub < 1 || e0 < 0) return 0;
  return pair_corr_workspace(M, E, prec, samples_per_sub, e0);
}

mp_status mp_pair_correlations_accumulate(int32_t M, int64_t E, const void* X, mp_precision prec,
                                          int32_t n_sub, int64_t samples_per_sub, int64_t e0,
                                          double* acc, void* workspace, size_t ws_bytes,
                                          void* stream) {
  clear_error();
  MP_CHECK_ARG(M >= 1 && E >= 1, MP_ERR_ARG,
               "mp_pair_correlations_accumulate: M and E must be >= 1");
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG,
               "mp_pair_correlations_accumulate: unknown precision %d", (int)prec);
  MP_CHECK_ARG(X && acc, MP_ERR_ARG, "mp_pair_correlations_accumulate: null pointer argument");
  MP_CHECK_ARG(aligned(X, 32) && aligned(acc, 16), MP_ERR_ARG,
               "mp_pair_correlations_accumulate: X must be 32-byte and acc 16-byte aligned");
  MP_CHECK_ARG(n_sub >= 1 && samples_per_sub >= 1 && e0 >= 0 &&
                   (e0 + E - 1) / samples_per_sub < n_sub,
               MP_ERR_ARG,
               "mp_pair_correlations_accumulate: samples [%lld, %lld) do not fit n_sub = %d "
               "sub-ensembles of %lld",
               (long long)e0, (long long)(e0 + E), n_sub, (long long)samples_per_sub);
  MP_CHECK_ARG(workspace == nullptr || aligned(workspace, 256), MP_ERR_WORKSPACE,
               "mp_pair_correlations_accumulate: workspace must be 256-byte aligned");
  return pair_corr_launch(M, E, X, prec, samples_per_sub, e0, acc, workspace, ws_bytes,
                          (hipStream_t)stream);
}

int64_t mp_mlp_param_count(const mp_mlp_shape* shape) {
  return valid_shape(shape) ? mlp_param_count(shape) : -1;
}

size_t mp_mlp_workspace(const mp_mlp_shape* shape, int32_t batch) {
  return (valid_shape(shape) && batch >= 1) ? mlp_workspace(shape, batch) : 0;
}

mp_status mp_mlp_round(const mp_mlp_shape* shape, const float* params, uint16_t* w16,
                       void* stream) {
  clear_error();
  MP_CHECK_ARG(valid_shape(shape), MP_ERR_ARG, "mp_mlp_round: invalid shape");
  MP_CHECK_ARG(params && w16, MP_ERR_ARG, "mp_mlp_round: null pointer argument");
  return mlp_round_launch(mlp_param_count(shape), params, w16, (hipStream_t)stream);
}

mp_status mp_mlp_forward(const mp_mlp_shape* shape, const uint16_t* w16, const float* params,
                         const float* X, int32_t batch, float* Y, void* workspace,
                         size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(valid_shape(shape), MP_ERR_ARG, "mp_mlp_forward: invalid shape");
  MP_CHECK_ARG(batch >= 1, MP_ERR_ARG, "mp_mlp_forward: batch must be >= 1");
  MP_CHECK_ARG(w16 && params && X && Y, MP_ERR_ARG, "mp_mlp_forward: null pointer argument");
  MP_CHECK_ARG(workspace && ws_bytes >= mlp_workspace(shape, batch), MP_ERR_WORKSPACE,
               "mp_mlp_forward: workspace of %zu bytes needed", mlp_workspace(shape, batch));
  return mlp_forward(shape, w16, params, X, batch, Y, workspace, (hipStream_t)stream);
}

mp_status mp_mlp_loss_grad(const mp_mlp_shape* shape, const uint16_t* w16, const float* params,
                           const float* X, const float* Y, int32_t batch, float* grads,
                           float* loss, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  MP_CHECK_ARG(valid_shape(shape), MP_ERR_ARG, "mp_mlp_loss_grad: invalid shape");
  MP_CHECK_ARG(batch >= 1, MP_ERR_ARG, "mp_mlp_loss_grad: batch must be >= 1");
  MP_CHECK_ARG(w16 && params && X && Y && grads && loss, MP_ERR_ARG,
               "mp_mlp_loss_grad: null pointer argument");
  MP_CHECK_ARG(workspace && ws_bytes >= mlp_workspace(shape, batch), MP_ERR_WORKSPACE,
               "mp_mlp_loss_grad: workspace of %zu bytes needed", mlp_workspace(shape, batch));
  return mlp_loss_grad(shape, w16, params, X, Y, batch, grads, loss, workspace,
                       (hipStream_t)stream);
}

mp_status mp_mlp_adam(const mp_mlp_shape* shape, float* params, const float* grads, float* m,
                      float* v, uint16_t* w16, float lr, float beta1, float beta2, float eps,
                      float weight_decay, int32_t step, void* stream) {
  clear_error();
  MP_CHECK_ARG(valid_shape(shape), MP_ERR_ARG, "mp_mlp_adam: invalid shape");
  MP_CHECK_ARG(params && grads && m && v && w16, MP_ERR_ARG, "mp_mlp_adam: null pointer argument");
  MP_CHECK_ARG(step >= 1 && lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f &&
                   beta2 < 1.0f && eps > 0.0f && weight_decay >= 0.0f,
               MP_ERR_ARG, "mp_mlp_adam: invalid hyper-parameters");
  return mlp_adam_launch(mlp_param_count(shape), params, grads, m, v, w16, lr, beta1, beta2, eps,
                         weight_decay, step, (hipStream_t)stream);
}

const char* mp_last_error(void) { return g_err; }

const char* mp_version(void) { return "mpgbs 0.1 (gfx950)"; }

}  // extern "C"
