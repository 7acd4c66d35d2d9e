// Host-side self-check of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (python -m paper_2503_12749_amd.build --host-check).
// It links the library's sources (host code sanitized, device code built as
// usual) and drives every entry point through its size queries and its
// argument validation: each call below fails, or returns a size, before any
// HIP call, so no GPU is needed.
// The sanitizers then watch the validation, the bin-run and tiling arithmetic
// and the error-message formatting for out-of-bounds accesses, overflow and
// undefined behaviour.  Prints "host check ok" and exits 0 on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/mpgbs.h"

static int g_fail = 0;

#define EXPECT(cond)                                                           \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "host check: %s:%d: %s (last error: %s)\n", __FILE__, \
                   __LINE__, #cond, mp_last_error());                          \
      ++g_fail;                                                                \
    }                                                                          \
  } while (0)

static void* P(uintptr_t v) { return (void*)v; }  // fake aligned device pointers

static void sizes() {
  EXPECT(mp_ld_modes(1) == 128 && mp_ld_modes(8000) == 8064 && mp_ld_modes(0) == -1);
  const mp_precision precs[] = {MP_FP64, MP_FP32, MP_SPLIT_BF16, MP_SPLIT_FP16, MP_SPLIT1_FP16,
                                MP_SPLIT1T_FP16, MP_SPLIT1T_F8};
  for (mp_precision p : precs) {
    EXPECT(mp_ab_bytes(16, 10, p) > 0 && mp_c_bytes(16, 10, p) > 0);
    EXPECT(mp_propagate_workspace(8000, p) > 0);
    EXPECT(mp_mode_occupations_bytes(333, 1000, p) > 0);
  }
  EXPECT(mp_ab_bytes(16, 0, MP_FP32) == 0 && mp_ab_bytes(16, 10, (mp_precision)9) == 0);
  EXPECT(mp_propagate_workspace(8000, MP_SPLIT1_FP16) * 2 == mp_propagate_workspace(8000, MP_SPLIT_BF16));
  EXPECT(mp_propagate_workspace(8000, MP_SPLIT1T_FP16) == mp_propagate_workspace(8000, MP_SPLIT_FP16));
  // T-split samples: one FP16 value, columns rounded up to even per half
  EXPECT(mp_ab_bytes(16, 10, MP_SPLIT1T_FP16) == 128u * 20 * 2);
  EXPECT(mp_ab_bytes(16, 11, MP_SPLIT1T_FP16) == 128u * 24 * 2);
  // FP8-correction form: the T-split operand plus one e4m3 byte per entry; T as
  // FP16 plus its e4m3 remainder
  EXPECT(mp_ab_bytes(16, 10, MP_SPLIT1T_F8) == 128u * 20 * 3);
  EXPECT(mp_ab_bytes(16, 11, MP_SPLIT1T_F8) == 128u * 24 * 3);
  EXPECT(mp_propagate_workspace(8000, MP_SPLIT1T_F8) == 2u * 8064 * 8064 * 3);
  EXPECT(mp_ab_bytes(16, 10, (mp_precision)(MP_SPLIT1T_F8 + 1)) == 0);
  const int32_t K1[] = {128}, K3[] = {8, 9, 10}, K4[] = {4, 5, 6, 7}, K5[] = {4, 4, 4, 4, 4};
  EXPECT(mp_acc_entries(1, MP_JOINT, K1) == 128);
  EXPECT(mp_acc_entries(3, MP_JOINT, K3) == 720);
  EXPECT(mp_acc_entries(3, MP_MARGINALS_AND_TOTAL, K4) == 22);
  EXPECT(mp_acc_entries(5, MP_JOINT, K5) == -1);
  EXPECT(mp_acc_entries(0, MP_JOINT, K1) == -1 && mp_acc_entries(1, MP_JOINT, nullptr) == -1);
  // 1000 samples from e0 = 500, N_S = 300: 100 + 300 + 300 + 300 in tiles of 64
  EXPECT(mp_binned_workspace(1, MP_JOINT, K1, 1000, 10, 300, 500) == (2 + 5 + 5 + 5) * 128 * 16);
  EXPECT(mp_binned_workspace(3, MP_JOINT, K3, 100, 1, 100, 0) > 0);
  EXPECT(mp_finalize_workspace(3, MP_JOINT, K3, 2) >= 2 * 720 * 16);
  // bin layouts of the fused path: contiguous runs, gaps, the run limit
  std::vector<int32_t> bins(8000, 0);
  const int32_t Kt[] = {3840};
  EXPECT(mp_propagate_counts_workspace(8000, 65536, 1, bins.data(), MP_JOINT, Kt, 8, 8192, 0) >
         (size_t)MP_NOALLOC_SCRATCH_BYTES);
  for (int j = 0; j < 8000; ++j) bins[j] = (j / 1000) % 4 - (j % 1000 < 10 ? 5 : 0);
  for (int j = 0; j < 8000; ++j) bins[j] = bins[j] < 0 ? -1 : bins[j];
  const int32_t K4b[] = {1536, 1536, 1536, 1536, 4096};
  EXPECT(mp_propagate_counts_workspace(8000, 4096, 4, bins.data(), MP_MARGINALS_AND_TOTAL, K4b, 2,
                                       4096, 0) > 0);
  for (int j = 0; j < 8000; ++j) bins[j] = j % 2;  // 8000 runs
  const int32_t K2[] = {64, 64};
  EXPECT(mp_propagate_counts_workspace(8000, 4096, 2, bins.data(), MP_MARGINALS, K2, 1, 4096, 0) ==
         0);
  EXPECT(mp_pair_correlations_workspace(1000, 100000, MP_FP32, 10000, 0) ==
         (size_t)10 * 36 * 6 * 128 * 128 * 8);
  mp_mlp_shape sh{};
  sh.n_layers = 4;
  const int w[] = {5, 256, 256, 256, 8};
  for (int l = 0; l <= 4; ++l) sh.width[l] = w[l];
  EXPECT(mp_mlp_param_count(&sh) == 5 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 8 + 8);
  EXPECT(mp_mlp_workspace(&sh, 64) > 0 && mp_mlp_workspace(&sh, 0) == 0);
  sh.width[2] = 2000;
  EXPECT(mp_mlp_param_count(&sh) == -1);
  EXPECT(std::strlen(mp_version()) > 0);
}

static void validation() {
  const double* r = (const double*)P(256);
  // sampling
  EXPECT(mp_sample(0, 0, 8, r, 1, 0, MP_FP64, P(256), (double*)P(256), nullptr) == MP_ERR_ARG);
  EXPECT(std::strstr(mp_last_error(), "M = 0") != nullptr);
  EXPECT(mp_sample(4, -5, 8, r, 1, 0, MP_FP64, P(256), (double*)P(256), nullptr) == MP_ERR_ARG);
  EXPECT(mp_sample(4, 0, 8, r, 1, 0, (mp_precision)7, P(256), (double*)P(256), nullptr) ==
         MP_ERR_ARG);
  EXPECT(mp_sample(4, 0, 8, nullptr, 1, 0, MP_FP64, P(256), (double*)P(256), nullptr) ==
         MP_ERR_ARG);
  EXPECT(mp_sample(4, 0, 8, r, 1, 0, MP_FP64, P(257), (double*)P(256), nullptr) == MP_ERR_ARG);
  // propagation: workspace missing or short
  EXPECT(mp_propagate(16, 4, r, MP_FP64, P(256), P(256), nullptr, 0, nullptr) == MP_ERR_WORKSPACE);
  EXPECT(mp_propagate(16, 4, r, MP_FP64, P(256), P(256), P(256), 10, nullptr) == MP_ERR_WORKSPACE);
  EXPECT(mp_pack_transmission(16, r, MP_SPLIT1_FP16, P(256), 10, nullptr) == MP_ERR_WORKSPACE);
  // grouped counts: bin index, run limit, window, sub-ensembles, workspace
  const int32_t b4[] = {0, 1, 5, 0}, lo2[] = {0, 0}, K8[] = {8, 8};
  EXPECT(mp_binned_counts(4, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 2, b4,
                          MP_MARGINALS, lo2, K8, 1, 8, 0, (double*)P(256), P(256), 1 << 20,
                          nullptr) == MP_ERR_ARG);
  EXPECT(std::strstr(mp_last_error(), "bin_of_mode[2]") != nullptr);
  std::vector<int32_t> alt(40);
  for (int j = 0; j < 40; ++j) alt[j] = j % 2;
  EXPECT(mp_binned_counts(40, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 2,
                          alt.data(), MP_MARGINALS, lo2, K8, 1, 8, 0, (double*)P(256), P(256),
                          1 << 20, nullptr) == MP_ERR_UNSUPPORTED);
  const int32_t z4[] = {0, 0, 0, 0}, lo1[] = {0}, K0[] = {0}, Kk[] = {8};
  EXPECT(mp_binned_counts(4, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 1, z4,
                          MP_JOINT, lo1, K0, 1, 8, 0, (double*)P(256), P(256), 1 << 20,
                          nullptr) == MP_ERR_ARG);
  EXPECT(mp_binned_counts(4, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 1, z4,
                          MP_JOINT, lo1, Kk, 1, 4, 0, (double*)P(256), P(256), 1 << 20,
                          nullptr) == MP_ERR_SHAPE);
  EXPECT(mp_binned_counts(4, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 1, z4,
                          MP_JOINT, lo1, Kk, 1, 8, 0, (double*)P(256), P(256), 16, nullptr) ==
         MP_ERR_WORKSPACE);
  const int32_t b5[] = {0, 1, 2, 3}, lo5[] = {0, 0, 0, 0, 0}, K5[] = {4, 4, 4, 4, 4};
  EXPECT(mp_binned_counts(4, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 5, b5,
                          MP_JOINT, lo5, K5, 1, 8, 0, (double*)P(256), P(256), 1 << 20,
                          nullptr) == MP_ERR_UNSUPPORTED);
  // the fused call: precision, joint limit, null and short buffers
  const int32_t z8[] = {0, 0, 0, 0, 0, 0, 0, 0};
  EXPECT(mp_propagate_counts(8, 8, MP_FP64, MP_MATRIX_P, P(256), (const double*)P(256), P(256),
                             1 << 20, 1, z8, MP_JOINT, lo1, Kk, 1, 8, 0, (double*)P(256), P(256),
                             1 << 20, nullptr) == MP_ERR_UNSUPPORTED);
  EXPECT(mp_propagate_counts(8, 8, MP_SPLIT1_FP16, MP_MATRIX_P, P(256), (const double*)P(256),
                             P(256), 16, 1, z8, MP_JOINT, lo1, Kk, 1, 8, 0, (double*)P(256),
                             P(256), 1 << 20, nullptr) == MP_ERR_WORKSPACE);
  EXPECT(mp_propagate_counts_noalloc(8, 8, MP_SPLIT1_FP16, MP_MATRIX_P, P(256),
                                     (const double*)P(256), nullptr, 1 << 20, 1, z8, MP_JOINT,
                                     lo1, Kk, 1, 8, 0, (double*)P(256), nullptr) == MP_ERR_ARG);
  std::vector<int32_t> all(8000, 0);
  const int32_t lot[] = {8083}, Kt[] = {3840};
  EXPECT(mp_propagate_counts_noalloc(8000, 65536, MP_SPLIT1_FP16, MP_MATRIX_P, P(256),
                                     (const double*)P(256), P(256),
                                     mp_propagate_workspace(8000, MP_SPLIT1_FP16), 1, all.data(),
                                     MP_JOINT, lot, Kt, 8, 8192, 0, (double*)P(256),
                                     nullptr) == MP_ERR_WORKSPACE);
  // the bilinear form: sizes, precision, mode set, buffers, windows
  EXPECT(mp_bilinear_workspace(0) == 0 && mp_bilinear_packed_bytes(0) == 0);
  EXPECT(mp_bilinear_packed_bytes(8000) == mp_propagate_workspace(8000, MP_SPLIT1T_F8) + 4 * 8064);
  EXPECT(mp_bilinear_workspace(8000) > (size_t)96 * 8000 * 8000 - (size_t)200000000);
  {
    const size_t pb = mp_bilinear_packed_bytes(8000), sb = mp_bilinear_workspace(8000);
    std::vector<int32_t> bad(all);
    bad[7999] = 1;
    EXPECT(mp_pack_bilinear(8000, (const double*)P(256), all.data(), MP_SPLIT1T_FP16, P(256), pb,
                            P(512), sb, nullptr) == MP_ERR_UNSUPPORTED);
    EXPECT(mp_pack_bilinear(8000, (const double*)P(256), bad.data(), MP_SPLIT1T_F8, P(256), pb,
                            P(512), sb, nullptr) == MP_ERR_ARG);
    EXPECT(mp_pack_bilinear(8000, nullptr, all.data(), MP_SPLIT1T_F8, P(256), pb, P(512), sb,
                            nullptr) == MP_ERR_ARG);
    EXPECT(mp_pack_bilinear(8000, (const double*)P(256), all.data(), MP_SPLIT1T_F8, P(256), pb - 1,
                            P(512), sb, nullptr) == MP_ERR_WORKSPACE);
    EXPECT(mp_pack_bilinear(8000, (const double*)P(256), all.data(), MP_SPLIT1T_F8, P(256), pb,
                            P(520), sb, nullptr) == MP_ERR_WORKSPACE);
    EXPECT(mp_propagate_counts_bilinear(8000, 65536, MP_FP32, MP_MATRIX_P, P(256),
                                        (const double*)P(256), P(256), pb, lot, Kt, 8, 8192, 0,
                                        (double*)P(256), P(256), 1 << 30,
                                        nullptr) == MP_ERR_UNSUPPORTED);
    EXPECT(mp_propagate_counts_bilinear(8000, 65536, MP_SPLIT1T_F8, MP_MATRIX_P, P(256),
                                        (const double*)P(256), P(256), pb - 1, lot, Kt, 8, 8192, 0,
                                        (double*)P(256), P(256), 1 << 30,
                                        nullptr) == MP_ERR_WORKSPACE);
    EXPECT(mp_propagate_counts_bilinear(8000, 65536, MP_SPLIT1T_F8, MP_MATRIX_P, P(256),
                                        (const double*)P(256), P(256), pb, lot, Kt, 4, 8192, 0,
                                        (double*)P(256), P(256), 1 << 30,
                                        nullptr) == MP_ERR_SHAPE);
  }
  // finalize, observables, statistics, finiteness
  EXPECT(mp_counts_finalize(1, MP_JOINT, Kk, 0, 8, (const double*)P(256), (double*)P(256),
                            (double*)P(256), (double*)P(256), nullptr, 0, nullptr) == MP_ERR_ARG);
  const int32_t K168[] = {16, 8};
  EXPECT(mp_counts_finalize(2, MP_JOINT, K168, 3, 8, (const double*)P(256), (double*)P(256),
                            (double*)P(256), (double*)P(256), nullptr, 0, nullptr) ==
         MP_ERR_WORKSPACE);
  EXPECT(mp_occupations(4, 8, P(256), MP_FP32, 1, z4, MP_JOINT, (double*)P(256), nullptr) ==
         MP_ERR_ARG);
  EXPECT(mp_moments_accumulate(8, (const double*)P(256), (const double*)P(256), 1, 9, MP_MATRIX_P,
                               2, 4, 0, (double*)P(256), nullptr) == MP_ERR_ARG);
  EXPECT(mp_observable_histogram(8, (const double*)P(256), (const double*)P(256), 2, 0, 4,
                                 MP_MATRIX_P, 0.0, 0.0, 10, 2, 4, 0, (double*)P(256), nullptr) ==
         MP_ERR_ARG);
  EXPECT(mp_subensemble_stats(1, 1, 4, 3, 1.0, (const double*)P(256), (double*)P(256),
                              (double*)P(256), nullptr) == MP_ERR_ARG);
  EXPECT(mp_subensemble_stats(1, 1, 4, 1, NAN, (const double*)P(256), (double*)P(256),
                              (double*)P(256), nullptr) == MP_ERR_ARG);
  int64_t bad = -1;
  EXPECT(mp_check_finite(nullptr, 4, (int64_t*)P(256), &bad, nullptr) == MP_ERR_ARG);
  EXPECT(mp_mode_occupations(8, 10, P(256), MP_FP32, P(48), nullptr) == MP_ERR_ARG);
  EXPECT(mp_pair_correlations_accumulate(8, 10, P(256), MP_FP32, 2, 4, 0, (double*)P(256),
                                         nullptr, 0, nullptr) == MP_ERR_ARG);
  // plans: every network is validated before any allocation
  void* plan = nullptr;
  mp_net_desc nd{};
  nd.M = 64;
  nd.T = r;
  nd.r = r;
  nd.E = 1000;
  nd.n_sub = 3;
  nd.K = 64;
  EXPECT(mp_plan_create(&plan, 1, &nd, MP_SPLIT_FP16, MP_MATRIX_P, 1000, nullptr) == MP_ERR_SHAPE);
  nd.n_sub = 4;
  nd.K = 0;
  EXPECT(mp_plan_create(&plan, 1, &nd, MP_SPLIT_FP16, MP_MATRIX_P, 1000, nullptr) == MP_ERR_ARG);
  EXPECT(mp_plan_create(&plan, 0, &nd, MP_SPLIT_FP16, MP_MATRIX_P, 1000, nullptr) == MP_ERR_ARG);
  // binned networks: bins in range, windows per distribution, supported modes
  std::vector<int32_t> bins64(64, 0);
  bins64[10] = 1;
  bins64[20] = 2;  // outside [-1, 2) for d = 2
  const int32_t mlo3[3] = {0, 0, 0}, k3[3] = {64, 64, 128};
  nd.K = 64;
  nd.d = 2;
  nd.mode = MP_MARGINALS_AND_TOTAL;
  nd.bin_of_mode = bins64.data();
  nd.m_lo_b = mlo3;
  nd.K_b = k3;
  EXPECT(mp_plan_create(&plan, 1, &nd, MP_SPLIT_FP16, MP_MATRIX_P, 1000, nullptr) == MP_ERR_ARG);
  EXPECT(std::strstr(mp_last_error(), "bin_of_mode[20]") != nullptr);
  bins64[20] = 1;
  nd.bin_of_mode = nullptr;
  EXPECT(mp_plan_create(&plan, 1, &nd, MP_SPLIT_FP16, MP_MATRIX_P, 1000, nullptr) == MP_ERR_ARG);
  nd.bin_of_mode = bins64.data();
  nd.d = 5;
  nd.mode = MP_JOINT;  // joint grids of more than 4 bins are not supported
  EXPECT(mp_plan_create(&plan, 1, &nd, MP_SPLIT_FP16, MP_MATRIX_P, 1000, nullptr) == MP_ERR_ARG);
  nd.d = 0;
  EXPECT(mp_plan_launch(nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_plan_info(nullptr, nullptr, nullptr, nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_plan_tile(nullptr, 0, nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_mfma_sustained(4, 10, (double*)P(256), 1 << 20, nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_mfma_sustained(-1, 10, (double*)P(256), 1 << 20, nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_mfma_sustained(0, 0, (double*)P(256), 1 << 20, nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_mfma_sustained(1, 10, nullptr, 1 << 20, nullptr, nullptr) == MP_ERR_ARG);
  EXPECT(mp_plan_destroy(nullptr) == MP_OK);
  // the surrogate's calls
  mp_mlp_shape sh{};
  sh.n_layers = 2;
  sh.width[0] = 5;
  sh.width[1] = 16;
  sh.width[2] = 8;
  EXPECT(mp_mlp_forward(&sh, (const uint16_t*)P(256), (const float*)P(256), (const float*)P(256),
                        0, (float*)P(256), P(256), 1 << 20, nullptr) == MP_ERR_ARG);
  EXPECT(mp_mlp_loss_grad(&sh, (const uint16_t*)P(256), (const float*)P(256),
                          (const float*)P(256), (const float*)P(256), 4, (float*)P(256),
                          (float*)P(256), nullptr, 0, nullptr) == MP_ERR_WORKSPACE);
  EXPECT(mp_mlp_adam(&sh, (float*)P(256), (const float*)P(256), (float*)P(256), (float*)P(256),
                     (uint16_t*)P(256), 1e-3f, 0.9f, 1.5f, 1e-8f, 0.0f, 1, nullptr) == MP_ERR_ARG);
  sh.n_layers = 0;
  EXPECT(mp_mlp_round(&sh, (const float*)P(256), (uint16_t*)P(256), nullptr) == MP_ERR_ARG);
  // a long message is cut at the buffer, not past it
  std::vector<int32_t> many(20000);
  for (int j = 0; j < 20000; ++j) many[j] = j % 2;
  EXPECT(mp_binned_counts(20000, 8, P(256), (const double*)P(256), MP_FP64, MP_MATRIX_P, 2,
                          many.data(), MP_MARGINALS, lo2, K8, 1, 8, 0, (double*)P(256), P(256),
                          1 << 20, nullptr) == MP_ERR_UNSUPPORTED);
  EXPECT(std::strlen(mp_last_error()) < 512);
}

int main() {
  sizes();
  validation();
  if (g_fail) {
    std::fprintf(stderr, "host check: %d failure(s)\n", g_fail);
    return 1;
  }
  std::printf("host check ok\n");
  return 0;
}
