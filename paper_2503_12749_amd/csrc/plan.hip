// Batched plans: many independent networks (uneven M) run as one pass that is
// captured once in a hipGraph and replayed.  The pass is
//   zero accumulators (fill kernels; no memset nodes) -> sample every network
//   -> one persistent grouped split-precision GEMM launch over all networks'
//   tiles -> occupations/characteristic function per network -> inverse DFT
// (FP32 plans: the occupation-fused GEMM per network; FP64: GEMM writing C,
// then the counts from C, per network).
// A plan owns all of its device memory (allocated in mp_plan_create).
//
// Autotuning: the grouped launch's work-list order decides which tiles share
// an XCD's L2 at the same time, and each network's tile shape (128 modes by
// 128 or by 64 samples; three-product split precisions) trades operand reuse against the number of tiles a
// small network offers the 256 compute units.  Candidate orders (with and
// without the L2 prefetch) are timed on the plan's own data at creation, then
// the narrower shape per size class of networks (equal M), largest first,
// kept where it is faster; results are cached in a small JSON file keyed by
// precision and the networks' (M, samples per chunk).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "common.h"

namespace mp {


mp_status sample_launch(int32_t M, int64_t g0, int64_t E, const double* r, uint64_t seed,
                        uint32_t net, mp_precision prec, void* ab, double* n_out,
                        hipStream_t stream);
size_t propagate_workspace(int32_t M, mp_precision prec);
int split_scale_exp(int32_t M, mp_precision prec);
int f8_scale_a(int32_t M);
mp_status pack_launch(int32_t M, const double* T, mp_precision prec, void* packed,
                      hipStream_t stream);
mp_status gemm_packed_launch(int32_t M, int64_t E, const void* packed, mp_precision prec,
                             const void* ab, void* C, hipStream_t stream);
mp_status grouped_launch(const GroupNet* d_nets, const int4* d_items, int n_items, int grid,
                         mp_precision prec, bool prefetch, hipStream_t stream);
size_t propagate_counts_workspace(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                                  mp_bin_mode mode, const int32_t* K, int32_t n_sub, int64_t ns,
                                  int64_t e0);
mp_status propagate_counts_launch(int32_t M, int64_t E, mp_precision prec, mp_estimator est,
                                  const void* ab, const double* n, const void* packed, int32_t d,
                                  const int32_t* bin_of_mode, mp_bin_mode mode,
                                  const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                  int64_t ns, int64_t e0, double* acc, void* ws, size_t ws_bytes,
                                  hipStream_t stream);
mp_status fused_out_setup(int32_t M, int64_t E, int32_t d, const int32_t* bin_of_mode,
                          mp_bin_mode mode, const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                          int64_t ns, int64_t e0, mp_estimator est, void* ws, size_t ws_bytes,
                          FusedOut& fo);
mp_status counts_from_partials_launch(int32_t M, int64_t E, const double* n, mp_estimator est,
                                      int32_t d, const int32_t* bin_of_mode, mp_bin_mode mode,
                                      const int32_t* m_lo, const int32_t* K, int32_t n_sub,
                                      int64_t ns, int64_t e0, double* acc, void* ws,
                                      size_t ws_bytes, hipStream_t stream);
bool split_prefetch(int64_t ldm);
size_t binned_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int64_t E, int32_t n_sub,
                        int64_t ns, int64_t e0);
mp_status binned_counts_launch(int32_t M, int64_t E, const void* C, const double* n,
                               mp_precision prec, mp_estimator est, int32_t d,
                               const int32_t* bin_of_mode, mp_bin_mode mode, const int32_t* m_lo,
                               const int32_t* K, int32_t n_sub, int64_t ns, int64_t e0,
                               double* acc, void* ws, size_t ws_bytes, hipStream_t stream);
size_t finalize_workspace(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub);
mp_status counts_finalize_launch(int32_t d, mp_bin_mode mode, const int32_t* K, int32_t n_sub,
                                 int64_t ns, const double* acc, double* P_re, double* P_im,
                                 double* sigma, void* ws, size_t ws_bytes, hipStream_t stream);

__global__ void fill_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

constexpr int kOrders = 3;  // autotuner candidates
constexpr int kXcdsPlan = 8;
constexpr int kTileModes = 128;  // per grouped work item; samples: 32 x (4 or 2)

struct PlanNet {
  mp_net_desc d;
  int64_t ldm = 0, chunk = 0;
  double* r = nullptr;
  double* n = nullptr;
  double* acc = nullptr;
  double* P_re = nullptr;
  double* P_im = nullptr;
  double* sigma = nullptr;
  void* ab = nullptr;
  void* C = nullptr;  // FP64 plans only; the others never materialise C
  void* packed = nullptr;
  void* ws_counts = nullptr;  // FP64: counts partials; else fused partials + counts partials
  size_t ws_counts_bytes = 0;
  // distributions: d bins by `bins` with `mode`, one window per
  // distribution (the total count of all modes on one window when the
  // descriptor's d is 0)
  std::vector<int32_t> bins;
  int32_t nb = 1;
  mp_bin_mode mode = MP_JOINT;
  std::vector<int32_t> m_lo, K;
  int64_t entries = 0;     // accumulator / result entries per sub-ensemble
  void* ws_fin = nullptr;  // inverse DFT workspace (joint grids of d >= 2)
  size_t ws_fin_bytes = 0;
  int nj = 4;  // grouped tile: 128 modes x 32 nj samples (nj 4 or 2)
};

// Side streams of a plan: the per-network kernels (sampling, counts, inverse
// DFT) of different networks are independent, so the captured graph holds
// them as parallel branches, network i on branch i % kBranches, joined
// before and after each grouped GEMM.  With small ensembles these kernels
// fill a fraction of the chip each, and the branches let them overlap.
constexpr int kBranches = 4;

struct Plan {
  std::vector<PlanNet> nets;
  mp_precision prec;
  mp_estimator est;
  int64_t chunk = 0;
  int passes = 0;
  hipStream_t stream = nullptr;
  hipStream_t side[kBranches] = {};
  std::vector<hipEvent_t> events;  // fork and join points (created as needed)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void*> allocs;
  // grouped launch, one per pass
  std::vector<GroupNet*> d_nets;
  std::vector<int4*> d_items;
  std::vector<int> n_items;
  int grid = 0;
  int order = 0;
  bool prefetch = true;  // the split GEMM's L2 prefetch (autotuned with the order)
  double tuned_ms = 0.0;
  size_t bytes = 0;
};

static void* plan_alloc(Plan* p, size_t bytes) {
  void* ptr = nullptr;
  if (bytes == 0) bytes = 256;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return nullptr;
  p->allocs.push_back(ptr);
  p->bytes += bytes;
  return ptr;
}

static void plan_free(Plan* p) {
  // teardown: errors here have nowhere to go (a failed creation already set one)
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (hipStream_t s : p->side)
    if (s) (void)hipStreamSynchronize(s);
  for (void* a : p->allocs) (void)hipFree(a);
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  for (hipStream_t s : p->side)
    if (s) (void)hipStreamDestroy(s);
  if (p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// The split precisions run one grouped GEMM per pass; the three-product ones
// offer two tile widths (the one-sided split kernel has the 128-sample tile only).
static bool split(mp_precision p) {
  return p == MP_SPLIT_BF16 || p == MP_SPLIT_FP16 || p == MP_SPLIT1_FP16 || p == MP_SPLIT1T_FP16 ||
         p == MP_SPLIT1T_F8;
}
static bool two_widths(mp_precision p) { return p == MP_SPLIT_BF16 || p == MP_SPLIT_FP16; }

// Work list of one pass in the given order.  Slot it * grid + w is processed
// by workgroup w (on XCD w % 8) in its it-th round.
static std::vector<int4> build_items(const Plan* p, int pass, int order, int grid) {
  struct T4 { int net, tm, tn, nj; };
  std::vector<T4> seq;
  std::vector<int> idx(p->nets.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return p->nets[a].d.M > p->nets[b].d.M; });
  const int gm = order == 1 ? 4 : 8;  // group rows x cols: 8 x 4 or 4 x 8
  const int gn = 32 / gm;
  for (int i : idx) {
    const PlanNet& n = p->nets[i];
    const int64_t e_this = std::min<int64_t>(n.chunk, n.d.E - (int64_t)pass * n.chunk);
    if (e_this <= 0) continue;
    const int tiles_m = (int)(n.ldm / kTileModes);
    const int nj = two_widths(p->prec) ? n.nj : 4;
    const int tiles_n = (int)((e_this + 32 * nj - 1) / (32 * nj));
    if (order == 2) {
      for (int tn = 0; tn < tiles_n; ++tn)
        for (int tm = 0; tm < tiles_m; ++tm) seq.push_back({i, tm, tn, nj});
    } else {
      for (int bm = 0; bm < tiles_m; bm += gm)
        for (int bn = 0; bn < tiles_n; bn += gn)
          for (int tn = bn; tn < std::min(bn + gn, tiles_n); ++tn)
            for (int tm = bm; tm < std::min(bm + gm, tiles_m); ++tm) seq.push_back({i, tm, tn, nj});
    }
  }
  const int n = (int)seq.size();
  const int rounds = (n + grid - 1) / grid;
  std::vector<int4> items((size_t)rounds * grid, int4{-1, 0, 0, 0});
  if (order == 2) {
    for (int q = 0; q < n; ++q) items[q] = int4{seq[q].net, seq[q].tm, seq[q].tn, seq[q].nj};
    return items;
  }
  // groups of consecutive sequence entries go to the workgroups of one XCD:
  // round it, XCD x, slot j (j-th workgroup of that XCD) <- seq[(it*8 + x)*per + j]
  const int per = grid / kXcdsPlan;
  for (int q = 0; q < n; ++q) {
    const int g = q / per, j = q % per;
    const int it = g / kXcdsPlan, x = g % kXcdsPlan;
    const int slot = it * grid + x + kXcdsPlan * j;
    items[slot] = int4{seq[q].net, seq[q].tm, seq[q].tn, seq[q].nj};
  }
  return items;
}


// ---------------------------------------------------------------- tuning cache

static std::string tune_key(const Plan* p) {
  std::string k = "prec" + std::to_string((int)p->prec) + ":";
  for (const PlanNet& n : p->nets)
    k += std::to_string(n.d.M) + "x" + std::to_string(n.chunk) + ",";
  return k;
}

// The cache is a flat JSON object
//   {"<key>": {"order": o, "prefetch": f, "ms": t, "nj": "4,2,..."}, ...}
// with one tile width per network ("nj" absent: 4 for every network).
static bool cache_lookup(const char* path, const std::string& key, int& order, int& prefetch,
                         double& ms, std::vector<int>& nj) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  fclose(f);
  // the last entry of this key that parses (an older entry may lack a field)
  const std::string pat = "\"" + key + "\": {\"order\": ";
  bool found = false;
  for (size_t at = text.find(pat); at != std::string::npos; at = text.find(pat, at + 1)) {
    int o = 0, f = 0;
    double t = 0.0;
    if (sscanf(text.c_str() + at + pat.size(), "%d, \"prefetch\": %d, \"ms\": %lf", &o, &f, &t) !=
        3)
      continue;
    if (o < 0 || o >= kOrders || (f != 0 && f != 1)) continue;
    // tile widths: inside this entry, one per network, each 4 or 2
    std::vector<int> w(nj.size(), 4);
    const size_t close = text.find('}', at + pat.size());
    const size_t q = text.find("\"nj\": \"", at + pat.size());
    if (q != std::string::npos && q < close) {
      const char* c = text.c_str() + q + 7;
      size_t k = 0;
      bool ok = true;
      while (ok && k < w.size()) {
        if (*c != '4' && *c != '2') ok = false;
        else w[k++] = *c++ - '0';
        if (ok && k < w.size()) ok = *c++ == ',';
      }
      if (!ok || *c != '"') continue;
    }
    order = o;
    prefetch = f;
    ms = t;
    nj = w;
    found = true;
  }
  return found;
}

static void cache_store(const char* path, const std::string& key, int order, int prefetch,
                        double ms, const std::vector<int>& nj) {
  if (!path) return;
  std::string text;
  if (FILE* f = fopen(path, "r")) {
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
  }
  size_t end = text.rfind('}');
  std::string body = end == std::string::npos ? "" : text.substr(text.find('{') + 1, end - text.find('{') - 1);
  while (!body.empty() && (body.back() == '\n' || body.back() == ' ')) body.pop_back();
  char head[128];
  snprintf(head, sizeof(head), "{\"order\": %d, \"prefetch\": %d, \"ms\": %.4f, \"nj\": \"", order,
           prefetch, ms);
  std::string entry = "\"" + key + "\": " + head;
  for (size_t i = 0; i < nj.size(); ++i) entry += (i ? "," : "") + std::to_string(nj[i]);
  entry += "\"}";
  const std::string out = "{" + body + (body.empty() ? "\n  " : ",\n  ") + entry + "\n}\n";
  const std::string tmp = std::string(path) + ".tmp";
  if (FILE* f = fopen(tmp.c_str(), "w")) {
    fwrite(out.data(), 1, out.size(), f);
    fclose(f);
    rename(tmp.c_str(), path);
  }
}

// ---------------------------------------------------------------- pass

static mp_status upload_items(Plan* p, int order) {
  for (int pass = 0; pass < p->passes; ++pass) {
    std::vector<int4> items = build_items(p, pass, order, p->grid);
    const size_t bytes = items.size() * sizeof(int4);
    if ((int)items.size() > p->n_items[pass]) {
      set_error("mp_plan: work list grew between orders");
      return MP_ERR_HIP;
    }
    std::vector<int4> padded = items;
    padded.resize(p->n_items[pass], int4{-1, 0, 0, 0});
    if (hipMemcpy(p->d_items[pass], padded.data(), padded.size() * sizeof(int4),
                  hipMemcpyHostToDevice) != hipSuccess) {
      set_error("mp_plan: work list upload failed");
      return MP_ERR_HIP;
    }
    (void)bytes;
  }
  return MP_OK;
}

// Every precision but FP64 runs the occupation-fused GEMM epilogue.
static bool fused(mp_precision p) { return p != MP_FP64; }

static mp_status plan_event(Plan* p, hipEvent_t& e) {
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    set_error("mp_plan: event creation failed");
    return MP_ERR_HIP;
  }
  p->events.push_back(e);
  return MP_OK;
}

// The side streams continue from the work queued on the plan stream so far.
static mp_status branch_fork(Plan* p) {
  hipEvent_t e;
  mp_status st = plan_event(p, e);
  if (st != MP_OK) return st;
  hipError_t h = hipEventRecord(e, p->stream);
  for (int b = 0; b < kBranches && h == hipSuccess; ++b) h = hipStreamWaitEvent(p->side[b], e, 0);
  if (h != hipSuccess) {
    set_error("mp_plan: fork: %s", hipGetErrorString(h));
    return MP_ERR_HIP;
  }
  return MP_OK;
}

// The plan stream waits for everything queued on the side streams.
static mp_status branch_join(Plan* p) {
  for (int b = 0; b < kBranches; ++b) {
    hipEvent_t e;
    mp_status st = plan_event(p, e);
    if (st != MP_OK) return st;
    hipError_t h = hipEventRecord(e, p->side[b]);
    if (h == hipSuccess) h = hipStreamWaitEvent(p->stream, e, 0);
    if (h != hipSuccess) {
      set_error("mp_plan: join: %s", hipGetErrorString(h));
      return MP_ERR_HIP;
    }
  }
  return MP_OK;
}

// Enqueues one full pass of every network: per-network kernels on the side
// streams (network i on side[i % kBranches]) between fork and join points,
// the grouped GEMM on the plan stream.  gemm_only: the GEMMs alone (timing).
static mp_status enqueue_pass(Plan* p, bool gemm_only = false) {
  mp_status st;
  const bool grouped = split(p->prec);
  if (!gemm_only && (st = branch_fork(p)) != MP_OK) return st;
  for (int pass = 0; pass < p->passes; ++pass) {
    if (!gemm_only) {
      for (size_t i = 0; i < p->nets.size(); ++i) {
        PlanNet& n = p->nets[i];
        hipStream_t s = p->side[i % kBranches];
        if (pass == 0) {
          const int64_t cnt = (int64_t)n.d.n_sub * n.entries * 2;
          hipLaunchKernelGGL(fill_zero_f64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                             n.acc, cnt);
        }
        const int64_t g0 = (int64_t)pass * n.chunk, e = std::min<int64_t>(n.chunk, n.d.E - g0);
        if (e <= 0) continue;
        if ((st = sample_launch(n.d.M, g0, e, n.r, n.d.seed, n.d.net, p->prec, n.ab, n.n, s)) !=
            MP_OK)
          return st;
      }
    }
    if (grouped) {
      // one grouped launch with the occupation epilogue, then counts from
      // each network's partials
      if (!gemm_only && (st = branch_join(p)) != MP_OK) return st;
      if ((st = grouped_launch(p->d_nets[pass], p->d_items[pass], p->n_items[pass], p->grid,
                               p->prec, p->prefetch, p->stream)) != MP_OK)
        return st;
      if (gemm_only) continue;
      if ((st = branch_fork(p)) != MP_OK) return st;
      for (size_t i = 0; i < p->nets.size(); ++i) {
        PlanNet& n = p->nets[i];
        const int64_t g0 = (int64_t)pass * n.chunk, e = std::min<int64_t>(n.chunk, n.d.E - g0);
        if (e <= 0) continue;
        if ((st = counts_from_partials_launch(n.d.M, e, n.n, p->est, n.nb, n.bins.data(), n.mode,
                                              n.m_lo.data(), n.K.data(), n.d.n_sub,
                                              n.d.E / n.d.n_sub, g0, n.acc,
                                              n.ws_counts, n.ws_counts_bytes,
                                              p->side[i % kBranches])) != MP_OK)
          return st;
      }
      continue;
    }
    // one GEMM per network, each on its network's branch (gemm_only: all on
    // the plan stream)
    for (size_t i = 0; i < p->nets.size(); ++i) {
      PlanNet& n = p->nets[i];
      hipStream_t s = gemm_only ? p->stream : p->side[i % kBranches];
      const int64_t g0 = (int64_t)pass * n.chunk, e = std::min<int64_t>(n.chunk, n.d.E - g0);
      if (e <= 0) continue;
      if (fused(p->prec)) {  // FP32: the fused GEMM and its counts
        if ((st = propagate_counts_launch(n.d.M, e, p->prec, p->est, n.ab, n.n, n.packed, n.nb,
                                          n.bins.data(), n.mode, n.m_lo.data(), n.K.data(),
                                          n.d.n_sub,
                                          n.d.E / n.d.n_sub, g0, n.acc, n.ws_counts,
                                          n.ws_counts_bytes, s)) != MP_OK)
          return st;
        continue;
      }
      if ((st = gemm_packed_launch(n.d.M, e, n.packed, p->prec, n.ab, n.C, s)) != MP_OK) return st;
      if (gemm_only) continue;
      if ((st = binned_counts_launch(n.d.M, e, n.C, n.n, p->prec, p->est, n.nb, n.bins.data(),
                                     n.mode, n.m_lo.data(), n.K.data(), n.d.n_sub,
                                     n.d.E / n.d.n_sub, g0, n.acc,
                                     n.ws_counts, n.ws_counts_bytes, s)) != MP_OK)
        return st;
    }
  }
  if (gemm_only) return MP_OK;
  for (size_t i = 0; i < p->nets.size(); ++i) {
    PlanNet& n = p->nets[i];
    if ((st = counts_finalize_launch(n.nb, n.mode, n.K.data(), n.d.n_sub, n.d.E / n.d.n_sub, n.acc,
                                     n.P_re, n.P_im, n.sigma, n.ws_fin, n.ws_fin_bytes,
                                     p->side[i % kBranches])) != MP_OK)
      return st;
  }
  return branch_join(p);
}

}  // namespace mp

using namespace mp;

extern "C" {

mp_status mp_plan_create(void** plan, int32_t n_net, const mp_net_desc* nets, mp_precision prec,
                         mp_estimator est, int64_t chunk, const char* tune_cache) {
  clear_error();
  MP_CHECK_ARG(plan && nets && n_net >= 1, MP_ERR_ARG, "mp_plan_create: null argument or n_net < 1");
  MP_CHECK_ARG(valid_prec(prec), MP_ERR_ARG, "mp_plan_create: unknown precision %d", (int)prec);
  MP_CHECK_ARG(est == MP_MATRIX_P || est == MP_PLUS_P, MP_ERR_ARG, "mp_plan_create: unknown estimator");
  MP_CHECK_ARG(chunk >= 1, MP_ERR_ARG, "mp_plan_create: chunk must be >= 1");
  *plan = nullptr;
  for (int i = 0; i < n_net; ++i) {
    const mp_net_desc& d = nets[i];
    MP_CHECK_ARG(d.M >= 1 && d.T && d.r && d.E >= 1 && d.n_sub >= 1, MP_ERR_ARG,
                 "mp_plan_create: network %d has an invalid size or a null pointer", i);
    MP_CHECK_ARG(d.E % d.n_sub == 0, MP_ERR_SHAPE,
                 "mp_plan_create: network %d: E = %lld not a multiple of n_sub = %d", i,
                 (long long)d.E, d.n_sub);
    MP_CHECK_ARG(d.E <= chunk || d.E % chunk == 0, MP_ERR_SHAPE,
                 "mp_plan_create: network %d: E = %lld must be <= chunk or a multiple of it", i,
                 (long long)d.E);
    if (d.d == 0) {
      MP_CHECK_ARG(d.K >= 1 && d.K <= 65536 && d.m_lo >= 0, MP_ERR_ARG,
                   "mp_plan_create: network %d: window K in [1, 65536] and m_lo >= 0 required", i);
    } else {
      MP_CHECK_ARG(d.d >= 1 && d.d <= MP_MAX_BINS && d.bin_of_mode && d.m_lo_b && d.K_b,
                   MP_ERR_ARG,
                   "mp_plan_create: network %d: d in [1, %d] with bin_of_mode, m_lo_b, K_b", i,
                   MP_MAX_BINS);
      MP_CHECK_ARG(mp_acc_entries(d.d, d.mode, d.K_b) > 0, MP_ERR_ARG,
                   "mp_plan_create: network %d: unsupported bin mode or window sizes", i);
      for (int j = 0; j < d.M; ++j)
        MP_CHECK_ARG(d.bin_of_mode[j] >= -1 && d.bin_of_mode[j] < d.d, MP_ERR_ARG,
                     "mp_plan_create: network %d: bin_of_mode[%d] = %d outside [-1, %d)", i, j,
                     d.bin_of_mode[j], d.d);
      const int nd = d.mode == MP_JOINT ? d.d : (d.mode == MP_MARGINALS ? d.d : d.d + 1);
      for (int q = 0; q < nd; ++q)
        MP_CHECK_ARG(d.m_lo_b[q] >= 0, MP_ERR_ARG, "mp_plan_create: network %d: m_lo_b[%d] < 0",
                     i, q);
    }
  }
  Plan* p = new Plan();
  p->prec = prec;
  p->est = est;
  p->chunk = chunk;
  if (hipStreamCreate(&p->stream) != hipSuccess) {
    delete p;
    set_error("mp_plan_create: hipStreamCreate failed");
    return MP_ERR_HIP;
  }
  for (hipStream_t& s : p->side)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      s = nullptr;
      plan_free(p);
      set_error("mp_plan_create: hipStreamCreate failed");
      return MP_ERR_HIP;
    }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    plan_free(p);
    set_error("mp_plan_create: device query failed");
    return MP_ERR_HIP;
  }
  p->grid = std::max(kXcdsPlan, (cus / kXcdsPlan) * kXcdsPlan);
  const size_t eb = (prec == MP_FP64) ? 8 : 4;
  int64_t max_e = 0;
  for (int i = 0; i < n_net; ++i) {
    PlanNet n;
    n.d = nets[i];
    n.ldm = ld_modes(n.d.M);
    n.chunk = std::min<int64_t>(chunk, n.d.E);
    if (n.d.d == 0) {  // total count of all modes on one window
      n.bins.assign(n.d.M, 0);
      n.nb = 1;
      n.mode = MP_JOINT;
      n.m_lo.assign(1, n.d.m_lo);
      n.K.assign(1, n.d.K);
    } else {
      n.bins.assign(n.d.bin_of_mode, n.d.bin_of_mode + n.d.M);
      n.nb = n.d.d;
      n.mode = n.d.mode;
      const int nd = n.mode == MP_MARGINALS_AND_TOTAL ? n.nb + 1 : n.nb;
      n.m_lo.assign(n.d.m_lo_b, n.d.m_lo_b + nd);
      n.K.assign(n.d.K_b, n.d.K_b + nd);
    }
    n.entries = mp_acc_entries(n.nb, n.mode, n.K.data());
    // the descriptor's pointers need not outlive creation
    n.d.bin_of_mode = nullptr;
    n.d.m_lo_b = nullptr;
    n.d.K_b = nullptr;
    max_e = std::max<int64_t>(max_e, n.d.E);
    n.r = (double*)plan_alloc(p, (size_t)n.d.M * 8);
    n.n = (double*)plan_alloc(p, (size_t)n.chunk * 8);
    n.acc = (double*)plan_alloc(p, (size_t)n.d.n_sub * n.entries * 16);
    n.P_re = (double*)plan_alloc(p, (size_t)n.entries * 8);
    n.P_im = (double*)plan_alloc(p, (size_t)n.entries * 8);
    n.sigma = (double*)plan_alloc(p, (size_t)n.entries * 8);
    n.ws_fin_bytes = finalize_workspace(n.nb, n.mode, n.K.data(), n.d.n_sub);
    if (n.ws_fin_bytes) n.ws_fin = plan_alloc(p, n.ws_fin_bytes);
    n.ab = plan_alloc(p, (size_t)n.ldm * ab_columns(n.chunk, prec) * elem_bytes_ab(prec));
    if (!fused(prec)) n.C = plan_alloc(p, (size_t)2 * n.ldm * 2 * n.chunk * eb);
    n.packed = plan_alloc(p, propagate_workspace(n.d.M, prec));
    const int64_t ns = n.d.E / n.d.n_sub;
    size_t wsb = 0;
    for (int64_t g0 = 0; g0 < n.d.E; g0 += n.chunk) {
      const int64_t e = std::min<int64_t>(n.chunk, n.d.E - g0);
      wsb = std::max(wsb, fused(prec) ? propagate_counts_workspace(n.d.M, e, n.nb, n.bins.data(),
                                                                   n.mode, n.K.data(), n.d.n_sub,
                                                                   ns, g0)
                                      : binned_workspace(n.nb, n.mode, n.K.data(), e, n.d.n_sub,
                                                         ns, g0));
    }
    n.ws_counts_bytes = wsb;
    n.ws_counts = plan_alloc(p, wsb);
    if (!n.r || !n.n || !n.acc || !n.P_re || !n.P_im || !n.sigma || !n.ab ||
        (!fused(prec) && !n.C) || !n.packed || !n.ws_counts || (n.ws_fin_bytes && !n.ws_fin)) {
      plan_free(p);
      set_error("mp_plan_create: device allocation failed (network %d)", i);
      return MP_ERR_HIP;
    }
    if (hipMemcpyAsync(n.r, n.d.r, (size_t)n.d.M * 8, hipMemcpyDeviceToDevice, p->stream) !=
        hipSuccess) {
      plan_free(p);
      set_error("mp_plan_create: copy of r failed (network %d)", i);
      return MP_ERR_HIP;
    }
    mp_status st = pack_launch(n.d.M, n.d.T, prec, n.packed, p->stream);
    if (st != MP_OK) {
      plan_free(p);
      return st;
    }
    p->nets.push_back(n);
  }
  p->passes = (int)((max_e + chunk - 1) / chunk);
  // grouped launch tables, one per pass
  if (split(prec)) {
    for (int pass = 0; pass < p->passes; ++pass) {
      std::vector<GroupNet> g(p->nets.size());
      for (size_t i = 0; i < p->nets.size(); ++i) {
        PlanNet& n = p->nets[i];
        const int64_t e = std::max<int64_t>(0, std::min<int64_t>(n.chunk, n.d.E - (int64_t)pass * n.chunk));
        const float sc = ldexpf(1.0f, -split_scale_exp(n.d.M, prec));
        // the T-split sample operand's storage columns: beta from E2 on
        const int64_t cols = ab_columns(e, prec);
        g[i] = GroupNet{(const uint16_t*)n.packed, (const uint16_t*)n.ab, nullptr, n.ldm, cols, sc,
                        prec == MP_SPLIT1T_F8 ? f8_scale_a(n.d.M) : 0, FusedOut{}};
        if (e > 0) {
          const mp_status st = fused_out_setup(n.d.M, e, n.nb, n.bins.data(), n.mode,
                                               n.m_lo.data(), n.K.data(),
                                               n.d.n_sub, n.d.E / n.d.n_sub, (int64_t)pass * n.chunk,
                                               est, n.ws_counts, n.ws_counts_bytes, g[i].fo);
          if (st != MP_OK) {
            plan_free(p);
            return st;
          }
        }
      }
      GroupNet* dn = (GroupNet*)plan_alloc(p, g.size() * sizeof(GroupNet));
      // room for the longest work list over orders and tile widths (the
      // narrower tile has at least as many items per network)
      size_t max_items = 0;
      for (PlanNet& n : p->nets) n.nj = 2;
      for (int o = 0; o < kOrders; ++o) max_items = std::max(max_items, build_items(p, pass, o, p->grid).size());
      for (PlanNet& n : p->nets) n.nj = 4;
      int4* di = (int4*)plan_alloc(p, max_items * sizeof(int4));
      if (!dn || !di) {
        plan_free(p);
        set_error("mp_plan_create: device allocation failed (work lists)");
        return MP_ERR_HIP;
      }
      if (hipMemcpy(dn, g.data(), g.size() * sizeof(GroupNet), hipMemcpyHostToDevice) != hipSuccess) {
        plan_free(p);
        set_error("mp_plan_create: upload of the network table failed");
        return MP_ERR_HIP;
      }
      p->d_nets.push_back(dn);
      p->d_items.push_back(di);
      p->n_items.push_back((int)max_items);
    }
    // autotune the work-list order and the L2 prefetch on this plan's data;
    // the prefetch is a candidate only when no network's operand rows are a
    // multiple of 32 KB apart (there it slowed the GEMM)
    bool prefetch_allowed = true;
    for (const PlanNet& n : p->nets) prefetch_allowed = prefetch_allowed && split_prefetch(n.ldm);
    const std::string key = tune_key(p);
    int order = 0, prefetch = prefetch_allowed ? 1 : 0;
    double ms = 0.0;
    std::vector<int> nj(p->nets.size(), 4);
    if (!cache_lookup(tune_cache, key, order, prefetch, ms, nj) || (prefetch && !prefetch_allowed)) {
      // a valid work list must be on the device before the first grouped launch
      p->prefetch = prefetch_allowed;
      mp_status st = upload_items(p, 0);
      if (st == MP_OK) st = enqueue_pass(p);  // real data in every buffer
      if (st != MP_OK) {
        plan_free(p);
        return st;
      }
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        plan_free(p);
        set_error("mp_plan_create: event creation failed");
        return MP_ERR_HIP;
      }
      // mean time of the grouped launches of one pass under the current
      // order, prefetch and tile widths (a warm pass, then two timed)
      auto time_pass = [&](int o, float& ms_out) -> mp_status {
        mp_status s2 = upload_items(p, o);
        if (s2 == MP_OK) s2 = enqueue_pass(p, true);
        float t = 0.f;
        bool ok = s2 == MP_OK && hipEventRecord(a, p->stream) == hipSuccess;
        for (int rep = 0; rep < 2 && ok && s2 == MP_OK; ++rep) s2 = enqueue_pass(p, true);
        ok = ok && s2 == MP_OK && hipEventRecord(b, p->stream) == hipSuccess &&
             hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&t, a, b) == hipSuccess;
        if (!ok && s2 == MP_OK) {
          set_error("mp_plan_create: timing the grouped launch failed");
          s2 = MP_ERR_HIP;
        }
        ms_out = t / 2;
        return s2;
      };
      double best = 1e30;
      for (int c = 0; c < 2 * kOrders && st == MP_OK; ++c) {
        const int o = c % kOrders, f = c < kOrders ? 1 : 0;
        if (f && !prefetch_allowed) continue;
        p->prefetch = f != 0;
        float t = 0.f;
        if ((st = time_pass(o, t)) != MP_OK) break;
        if (t < best) {
          best = t;
          order = o;
          prefetch = f;
        }
      }
      // tile width per size class, largest networks first, under the chosen
      // order and prefetch
      p->prefetch = prefetch != 0;
      std::vector<int32_t> sizes;
      for (const PlanNet& n : p->nets) sizes.push_back(n.d.M);
      std::sort(sizes.begin(), sizes.end(), std::greater<int32_t>());
      sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
      for (size_t c = 0; c < sizes.size() && st == MP_OK && two_widths(prec); ++c) {
        for (PlanNet& n : p->nets)
          if (n.d.M == sizes[c]) n.nj = 2;
        float t = 0.f;
        if ((st = time_pass(order, t)) != MP_OK) break;
        if (t < best) {
          best = t;
        } else {
          for (PlanNet& n : p->nets)
            if (n.d.M == sizes[c]) n.nj = 4;
        }
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      if (st != MP_OK) {
        plan_free(p);
        return st;
      }
      ms = best;
      for (size_t i = 0; i < p->nets.size(); ++i) nj[i] = p->nets[i].nj;
      cache_store(tune_cache, key, order, prefetch, ms, nj);
    }
    for (size_t i = 0; i < p->nets.size(); ++i) p->nets[i].nj = two_widths(prec) ? nj[i] : 4;
    p->order = order;
    p->prefetch = prefetch != 0;
    p->tuned_ms = ms;
    mp_status st = upload_items(p, order);
    if (st != MP_OK) {
      plan_free(p);
      return st;
    }
  }
  // capture the full pass once
  if (hipStreamSynchronize(p->stream) != hipSuccess ||
      hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    plan_free(p);
    set_error("mp_plan_create: stream capture could not start");
    return MP_ERR_HIP;
  }
  mp_status st = enqueue_pass(p);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(p->stream, &graph);
  if (st != MP_OK || ce != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    plan_free(p);
    if (st == MP_OK) set_error("mp_plan_create: stream capture failed: %s", hipGetErrorString(ce));
    return st == MP_OK ? MP_ERR_HIP : st;
  }
  p->graph = graph;
  if (hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    plan_free(p);
    set_error("mp_plan_create: graph instantiation failed");
    return MP_ERR_HIP;
  }
  *plan = p;
  return MP_OK;
}

mp_status mp_plan_launch(void* plan, void* stream) {
  clear_error();
  MP_CHECK_ARG(plan, MP_ERR_ARG, "mp_plan_launch: null plan");
  Plan* p = (Plan*)plan;
  // order the replay after the caller's stream and make the caller wait for it
  hipEvent_t ev;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    set_error("mp_plan_launch: event creation failed");
    return MP_ERR_HIP;
  }
  hipStream_t s = (hipStream_t)stream;
  // each step runs only if the previous ones succeeded; the first error is reported
  hipError_t e = hipEventRecord(ev, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, ev, 0);
  if (e == hipSuccess) e = hipGraphLaunch(p->exec, p->stream);
  if (e == hipSuccess) e = hipEventRecord(ev, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
  (void)hipEventDestroy(ev);
  if (e != hipSuccess) {
    set_error("mp_plan_launch: %s", hipGetErrorString(e));
    return MP_ERR_HIP;
  }
  return MP_OK;
}

mp_status mp_plan_result(void* plan, int32_t i, const double** P_re, const double** P_im,
                         const double** sigma) {
  clear_error();
  MP_CHECK_ARG(plan, MP_ERR_ARG, "mp_plan_result: null plan");
  Plan* p = (Plan*)plan;
  MP_CHECK_ARG(i >= 0 && i < (int)p->nets.size(), MP_ERR_ARG, "mp_plan_result: network %d", i);
  if (P_re) *P_re = p->nets[i].P_re;
  if (P_im) *P_im = p->nets[i].P_im;
  if (sigma) *sigma = p->nets[i].sigma;
  return MP_OK;
}

mp_status mp_plan_info(void* plan, int32_t* order, int32_t* prefetch, double* tuned_ms,
                       size_t* device_bytes) {
  clear_error();
  MP_CHECK_ARG(plan, MP_ERR_ARG, "mp_plan_info: null plan");
  Plan* p = (Plan*)plan;
  if (order) *order = p->order;
  if (prefetch) *prefetch = p->prefetch ? 1 : 0;
  if (tuned_ms) *tuned_ms = p->tuned_ms;
  if (device_bytes) *device_bytes = p->bytes;
  return MP_OK;
}

mp_status mp_plan_tile(void* plan, int32_t i, int32_t* modes, int32_t* samples) {
  clear_error();
  MP_CHECK_ARG(plan, MP_ERR_ARG, "mp_plan_tile: null plan");
  Plan* p = (Plan*)plan;
  MP_CHECK_ARG(i >= 0 && i < (int)p->nets.size(), MP_ERR_ARG, "mp_plan_tile: network %d", i);
  const bool grouped = split(p->prec);
  if (modes) *modes = grouped ? kTileModes : 0;
  if (samples) *samples = grouped ? 32 * (two_widths(p->prec) ? p->nets[i].nj : 4) : 0;
  return MP_OK;
}

mp_status mp_plan_destroy(void* plan) {
  clear_error();
  if (plan) plan_free((Plan*)plan);
  return MP_OK;
}

}  // extern "C"
