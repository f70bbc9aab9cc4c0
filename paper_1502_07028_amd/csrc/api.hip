// C ABI of libtca.so (declared in include/tca.h): argument checking, device
// memory owned by a context, and the host-side block schedule of a sweep.
//
// A sweep (Sec. II(c), Fig. 2) is issued as the four quadrant blocks of the
// parallel scheme (Sec. III(a), Fig. 3/4): for each block one batched launch
// solves every cluster (old and new matrix) and one launch makes the block's
// Metropolis decisions; the kernel boundary plays the role of the broadcast of
// the updated spin array between blocks.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <mutex>
#include <vector>

#include "ctx.hpp"
#include "internal.hpp"

using namespace tca;

namespace tca {
thread_local char g_err[512] = "";
}

namespace {

bool is_fin(double v) { return isfinite(v) != 0; }

bool unit_spins(const double* s, long n) {
  for (long p = 0; p < n; ++p) {
    const double x = s[3 * p], y = s[3 * p + 1], z = s[3 * p + 2];
    const double r = x * x + y * y + z * z;
    if (!is_fin(r) || fabs(sqrt(r) - 1.0) > 1e-12) return false;
  }
  return true;
}

}  // namespace

// Event pairs bracketing launches when profiling: pairs [2i, 2i+1].
struct ProfRec {
  tca_ctx* c;
  bool on;
  size_t used = 0;
  std::vector<int> kind;  // 0 reduce, 1 eigenvalues, 2 decide, 3 surrogate stage
  hipError_t begin() {
    if (!on) return hipSuccess;
    while (c->prof.size() < 2 * (used + 1)) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      c->prof.push_back(e);
    }
    return hipEventRecord(c->prof[2 * used], c->stream);
  }
  hipError_t end(int k) {
    if (!on) return hipSuccess;
    kind.push_back(k);
    return hipEventRecord(c->prof[2 * used++ + 1], c->stream);
  }
};

static int check_Lc(int Lc, int L) { return Lc >= 2 && Lc <= kMaxLc && Lc <= L / 2 + 1; }

static void free_ctx(tca_ctx* c) {
  if (!c) return;
  if (c->S) (void)hipFree(c->S);
  if (c->F) (void)hipFree(c->F);
  if (c->D) (void)hipFree(c->D);
  if (c->E2) (void)hipFree(c->E2);
  if (c->nmat) (void)hipFree(c->nmat);
  if (c->cls_count) (void)hipFree(c->cls_count);
  if (c->cls_list) (void)hipFree(c->cls_list);
  if (c->counters) (void)hipFree(c->counters);
  if (c->prep) (void)hipFree(c->prep);
  if (c->sq_work) (void)hipFree(c->sq_work);
  if (c->sq_out) (void)hipFree(c->sq_out);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->prof) (void)hipEventDestroy(e);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->sched_base) (void)hipFree(c->sched_base);
  if (c->sched_idx) (void)hipFree(c->sched_idx);
  if (c->sched_T) (void)hipFree(c->sched_T);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

static ModelParams model_of(const tca_ctx* c) {
  const double gap = (c->p.flags & TCA_FLAG_EXACT_METROPOLIS) ? HUGE_VAL : kDecideGap;
  return ModelParams{c->p.t, c->p.JH, c->p.JAF, c->p.mu, c->p.seed, gap};
}

// ---------------------------------------------------------------- autotuner
// Reducer variants are timed once per process and (dimension class,
// precision), on the clusters of block 0 of the first context that needs
// them: one warm-up launch and three timed launches of every variant, the
// fastest recorded for the process.
static std::mutex g_tune_mu;
static bool g_tuned[2][kNumReducerClasses];
static std::atomic<int> g_tune_gen{0};
static std::string g_tune_log[2][kNumReducerClasses];

int tca::tuning_generation() { return g_tune_gen.load(); }

static int autotune(tca_ctx* c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int sizes[4], ns = 0;
  if (c->p.n_classes == 0) {
    sizes[ns++] = c->p.Lc;
  } else {
    for (int k = 0; k < c->p.n_classes; ++k) sizes[ns++] = c->p.Lc_classes[k];
  }
  const int prec = c->p.precision == TCA_MIXED ? 1 : 0;
  const int hh = c->h * c->h;
  const BlockGeom g{c->p.L, c->h, 0, 0};
  const ReduceOut ro{c->D, c->E2, c->ld, c->nmat};
  const ModelParams m = model_of(c);
  std::string rep;
  for (int q = 0; q < ns; ++q) {
    const int n = 2 * sizes[q] * sizes[q];
    const int cls = reducer_class(n);
    const int nv = reducer_variants(cls, c->p.precision);
    if (!g_tuned[prec][cls] && nv > 1) {
      char buf[160];
      snprintf(buf, sizeof(buf), "n=%d %s (%d matrices):", n, prec ? "mixed" : "fp64", 2 * hh);
      std::string line = buf;
      double best_ms = 1e300;
      int best = 0;
      for (int v = 0; v < nv; ++v) {
        TCA_CK(launch_cluster_block_reduce(c->p.precision, sizes[q], c->S, g, m,
                                           fixed_sweep(0, 1.0), nullptr, nullptr, hh, ro,
                                           c->stream, v));
        TCA_CK(hipEventRecord(c->ev0, c->stream));
        for (int r = 0; r < 3; ++r)
          TCA_CK(launch_cluster_block_reduce(c->p.precision, sizes[q], c->S, g, m,
                                             fixed_sweep(0, 1.0), nullptr, nullptr, hh, ro,
                                             c->stream, v));
        TCA_CK(hipEventRecord(c->ev1, c->stream));
        TCA_CK(hipStreamSynchronize(c->stream));
        float ms = 0.f;
        TCA_CK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const double per = ms / 3.0;
        snprintf(buf, sizeof(buf), " %s %.3f ms;", reducer_name(cls, c->p.precision, v), per);
        line += buf;
        if (per < best_ms) {
          best_ms = per;
          best = v;
        }
      }
      line += " -> ";
      line += reducer_name(cls, c->p.precision, best);
      set_reducer_choice(cls, c->p.precision, best);
      g_tuned[prec][cls] = true;
      g_tune_log[prec][cls] = line;
      g_tune_gen.fetch_add(1);
    } else if (!g_tuned[prec][cls]) {
      g_tune_log[prec][cls] = "n=" + std::to_string(n) + (prec ? " mixed" : " fp64") +
                              ": single variant " + reducer_name(cls, c->p.precision, 0);
    }
    rep += g_tune_log[prec][cls] + "\n";
  }
  c->tune_report = rep;
  return TCA_OK;
}

extern "C" {

int tca_reducer_variants(int32_t n, int32_t precision, int32_t variant, int32_t* count,
                         const char** name) {
  g_err[0] = 0;
  if (!count) TCA_INVAL("count is NULL");
  if (!supported_n(n)) TCA_INVAL("n must satisfy 2 <= n <= 200");
  if (precision != TCA_FP64 && precision != TCA_MIXED) TCA_INVAL("bad precision");
  const int cls = reducer_class(n);
  *count = reducer_variants(cls, precision);
  if (name) *name = (variant >= 0 && variant < *count) ? reducer_name(cls, precision, variant) : nullptr;
  return TCA_OK;
}

int tca_select_reducer_variant(int32_t n, int32_t precision, int32_t variant) {
  g_err[0] = 0;
  if (!supported_n(n)) TCA_INVAL("n must satisfy 2 <= n <= 200");
  if (precision != TCA_FP64 && precision != TCA_MIXED) TCA_INVAL("bad precision");
  const int cls = reducer_class(n);
  if (variant < 0 || variant >= reducer_variants(cls, precision)) TCA_INVAL("variant out of range");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  set_reducer_choice(cls, precision, variant);
  const int prec = precision == TCA_MIXED ? 1 : 0;
  g_tuned[prec][cls] = true;
  g_tune_log[prec][cls] = "n=" + std::to_string(n) + (prec ? " mixed" : " fp64") + ": selected " +
                          reducer_name(cls, precision, variant);
  g_tune_gen.fetch_add(1);
  return TCA_OK;
}

int tca_tuning_report(tca_ctx* c, char* buf, int32_t len) {
  g_err[0] = 0;
  if (!c || !buf || len < 1) TCA_INVAL("NULL argument or len < 1");
  const size_t n = c->tune_report.size() < (size_t)(len - 1) ? c->tune_report.size() : (size_t)(len - 1);
  memcpy(buf, c->tune_report.data(), n);
  buf[n] = 0;
  return TCA_OK;
}

const char* tca_strerror(int s) {
  switch (s) {
    case TCA_OK: return "ok";
    case TCA_E_INVAL: return "invalid argument";
    case TCA_E_NOMEM: return "out of memory";
    case TCA_E_DEVICE: return "HIP device error";
    case TCA_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* tca_last_error(void) { return g_err; }

int tca_abi_sizes(int32_t* out3) {
  if (!out3) return TCA_E_INVAL;
  out3[0] = (int32_t)sizeof(tca_params);
  out3[1] = (int32_t)sizeof(tca_update_record);
  out3[2] = (int32_t)sizeof(tca_sweep_stats);
  return TCA_OK;
}

int tca_init_lattice(const tca_params* p, const double* spins_xyz, void* hip_stream,
                     tca_ctx** out) {
  g_err[0] = 0;
  if (!out) TCA_INVAL("out is NULL");
  *out = nullptr;
  if (!p) TCA_INVAL("params is NULL");
  if (p->abi_version != TCA_ABI_VERSION) TCA_INVAL("abi_version mismatch");
  if (p->L < 2 || (p->L & 1) || p->L > 4096) TCA_INVAL("L must be even, 2 <= L <= 4096");
  if (p->n_classes < 0 || p->n_classes > 4) TCA_INVAL("n_classes must be 0..4");
  if (p->n_classes == 0 && !check_Lc(p->Lc, p->L))
    TCA_INVAL("Lc must satisfy 2 <= Lc <= min(10, L/2+1)");
  for (int k = 0; k < p->n_classes; ++k)
    if (!check_Lc(p->Lc_classes[k], p->L))
      TCA_INVAL("every size class must satisfy 2 <= Lc <= min(10, L/2+1)");
  if (p->precision != TCA_FP64 && p->precision != TCA_MIXED) TCA_INVAL("bad precision");
  if (p->init < TCA_INIT_RANDOM || p->init > TCA_INIT_USER) TCA_INVAL("bad init");
  if (p->flags & ~(TCA_FLAG_PROFILE | TCA_FLAG_NO_GRAPH | TCA_FLAG_NO_AUTOTUNE | TCA_FLAG_EXACT_METROPOLIS))
    TCA_INVAL("unknown flag bits");
  if (!is_fin(p->t) || !is_fin(p->JH) || !is_fin(p->JAF) || !is_fin(p->mu))
    TCA_INVAL("model parameters must be finite");
  const int N = p->L * p->L;
  if (p->init == TCA_INIT_USER) {
    if (!spins_xyz) TCA_INVAL("TCA_INIT_USER needs spins_xyz");
    if (!unit_spins(spins_xyz, N)) TCA_INVAL("spins must have unit norm within 1e-12");
  }
  tca_ctx* c = new (std::nothrow) tca_ctx;
  if (!c) {
    set_err("host allocation failed");
    return TCA_E_NOMEM;
  }
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  if (c->stream == nullptr) {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      set_err("stream creation failed");
      delete c;
      return TCA_E_DEVICE;
    }
    c->own_stream = true;
  }
  c->N = N;
  c->h = p->L / 2;
  const size_t hh = (size_t)c->h * c->h;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void**)&c->S, sizeof(double) * 3 * N);
  int maxLc = p->Lc;
  for (int k = 0; k < p->n_classes; ++k) maxLc = k == 0 ? p->Lc_classes[0] : std::max(maxLc, p->Lc_classes[k]);
  c->ld = 2 * maxLc * maxLc;
  if (e == hipSuccess) e = hipMalloc((void**)&c->F, sizeof(double) * 2 * hh);
  if (e == hipSuccess) e = hipMalloc((void**)&c->D, sizeof(double) * 2 * hh * c->ld);
  if (e == hipSuccess) e = hipMalloc((void**)&c->E2, sizeof(double) * 2 * hh * c->ld);
  if (e == hipSuccess) e = hipMalloc((void**)&c->nmat, sizeof(int32_t) * 2 * hh);
  if (e == hipSuccess) e = hipMalloc((void**)&c->cls_count, sizeof(int32_t) * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&c->cls_list, sizeof(int32_t) * 4 * hh);
  if (e == hipSuccess) e = hipMalloc((void**)&c->counters, sizeof(unsigned long long) * 4);
  if (e == hipSuccess) e = hipMalloc(&c->prep, decide_prep_bytes((int)hh));
  if (e == hipSuccess) e = hipMalloc((void**)&c->sched_base, sizeof(uint64_t));
  if (e == hipSuccess) e = hipMalloc((void**)&c->sched_idx, sizeof(int32_t));
  if (e == hipSuccess) e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e != hipSuccess) {
    set_err("device allocation failed: %s", hipGetErrorString(e));
    free_ctx(c);
    return e == hipErrorOutOfMemory ? TCA_E_NOMEM : TCA_E_DEVICE;
  }
  if (p->init == TCA_INIT_USER) {
    e = hipMemcpyAsync(c->S, spins_xyz, sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->stream);
  } else {
    e = launch_init_spins(c->S, p->L, p->init, p->seed, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    set_err("initialization failed: %s", hipGetErrorString(e));
    free_ctx(c);
    return TCA_E_DEVICE;
  }
  if (!(p->flags & TCA_FLAG_NO_AUTOTUNE)) {
    const int rc = autotune(c);
    if (rc != TCA_OK) {
      free_ctx(c);
      return rc;
    }
  }
  *out = c;
  return TCA_OK;
}

int tca_destroy(tca_ctx* c) {
  free_ctx(c);
  return TCA_OK;
}

int tca_set_state(tca_ctx* c, const double* spins_xyz, uint64_t sweep_counter) {
  g_err[0] = 0;
  if (!c || !spins_xyz) TCA_INVAL("NULL argument");
  if (!unit_spins(spins_xyz, c->N)) TCA_INVAL("spins must have unit norm within 1e-12");
  TCA_CK(hipMemcpyAsync(c->S, spins_xyz, sizeof(double) * 3 * c->N, hipMemcpyHostToDevice,
                        c->stream));
  TCA_CK(hipStreamSynchronize(c->stream));
  c->sweep_counter = sweep_counter;
  return TCA_OK;
}

int tca_get_sweep_counter(tca_ctx* c, uint64_t* sc) {
  g_err[0] = 0;
  if (!c || !sc) TCA_INVAL("NULL argument");
  *sc = c->sweep_counter;
  return TCA_OK;
}

}  // extern "C"

// Issue one sweep on the context's stream (no synchronization), reading the
// sweep counter and temperature through `sr`.  With a surrogate attached, each
// block first runs the delayed-acceptance stage 1 (features of the forward and
// reverse moves, BF16 MLP, pass flags and the compacted list of survivors) and
// only the survivors are solved exactly.  With `collect`, every update's
// (features, dF) row is appended to the surrogate's dataset from row `row0` on
// (plain sweeps only).  The call ends by advancing the device sweep index.
static int issue_sweep(tca_ctx* c, SweepRef sr, int32_t* idx, tca_update_record* dlog,
                       ProfRec& pr, tca_surrogate* collect, int64_t row0) {
  const int L = c->p.L, h = c->h, hh = h * h;
  const ModelParams m = model_of(c);
  tca_surrogate* sg = collect ? nullptr : c->sg;
  for (int K = 0; K < 4; ++K) {
    const BlockGeom g{L, h, h * (K & 1), h * (K >> 1)};
    const ReduceOut ro{c->D, c->E2, c->ld, c->nmat};
    const int32_t* list = nullptr;
    const int32_t* count = nullptr;
    if (sg) {
      TCA_CK(pr.begin());
      TCA_CK(sg_block_features(c->S, g, c->p.Lc, m, sr, sg->dm, c->da.Fin.p, c->stream));
      TCA_CK(sg_infer_bf16(c->da.Fin.p, 2 * hh, sg->W.p, sg->W1b.p, sg->W2b.p, sg->dm,
                           SgInferBufs{c->da.H1.p, c->da.H2.p}, c->da.dS.p, c->stream));
      TCA_CK(sg_stage1(c->da.dS.p, g, m, sr, c->da.pass.p, c->da.count.p, c->da.list.p,
                       c->stream));
      TCA_CK(pr.end(3));
      list = c->da.list.p;
      count = c->da.count.p;
    }
    TCA_CK(pr.begin());
    if (c->p.n_classes == 0) {
      TCA_CK(launch_cluster_block_reduce(c->p.precision, c->p.Lc, c->S, g, m, sr, list, count,
                                         hh, ro, c->stream));
    } else {
      const ClassLists cl{c->cls_count, c->cls_list};
      TCA_CK(launch_classify(c->p.Lc_classes, c->p.n_classes, g, c->p.seed, sr, cl, c->stream));
      // largest clusters first so the longest workgroups start earliest
      int order[4] = {0, 1, 2, 3};
      for (int a = 0; a < c->p.n_classes; ++a)
        for (int b = a + 1; b < c->p.n_classes; ++b)
          if (c->p.Lc_classes[order[b]] > c->p.Lc_classes[order[a]]) std::swap(order[a], order[b]);
      for (int a = 0; a < c->p.n_classes; ++a) {
        const int k = order[a];
        TCA_CK(launch_cluster_block_reduce(c->p.precision, c->p.Lc_classes[k], c->S, g, m, sr,
                                           c->cls_list + (size_t)k * hh, c->cls_count + k, hh, ro,
                                           c->stream));
      }
    }
    TCA_CK(pr.end(0));
    TCA_CK(pr.begin());
    TCA_CK(launch_tridiag_eig(c->ld, 2 * hh, ro, sr, c->p.mu, c->F, nullptr, 0, c->stream, list,
                              count));
    TCA_CK(pr.end(1));
    if (collect)
      TCA_CK(sg_block_collect(c->S, g, K, c->p.Lc, m, sr, collect->dm, c->F, collect->X.p,
                              collect->y.p, row0, c->stream));
    TCA_CK(pr.begin());
    TCA_CK(launch_decide(c->S, c->F, g, m, sr, c->p.Lc, c->p.Lc_classes, c->p.n_classes, K,
                         sg ? c->da.pass.p : nullptr, sg ? c->da.dS.p : nullptr, c->prep, dlog,
                         c->counters, c->stream));
    TCA_CK(pr.end(2));
  }
  TCA_CK(launch_advance(idx, c->stream));
  return TCA_OK;
}

// Totals of a finished call into st (host).
static int fill_stats(tca_ctx* c, ProfRec& pr, tca_sweep_stats* st) {
  unsigned long long cnt[4];
  TCA_CK(hipMemcpy(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost));
  float ms = 0.f;
  TCA_CK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  memset(st, 0, sizeof(*st));
  st->accepted = (int64_t)cnt[0];
  st->near_threshold = (int64_t)cnt[1];
  st->updates = (int64_t)cnt[2];
  st->stage1_passed = (int64_t)cnt[3];
  st->elapsed_ms = ms;
  for (size_t i = 0; i < pr.used; ++i) {
    float e = 0.f;
    TCA_CK(hipEventElapsedTime(&e, c->prof[2 * i], c->prof[2 * i + 1]));
    switch (pr.kind[i]) {
      case 0: st->reduce_ms += e; st->reduce_launches += 1; break;
      case 1: st->eig_ms += e; st->eig_launches += 1; break;
      case 2: st->decide_ms += e; st->decide_launches += 1; break;
      default: st->surrogate_ms += e; st->surrogate_launches += 1; break;
    }
  }
  return TCA_OK;
}

// Key of the captured sweep graph: everything a captured launch depends on.
static void graph_key(const tca_ctx* c, uintptr_t key[4]) {
  key[0] = (uintptr_t)c->sg;
  key[1] = (uintptr_t)c->sched_T;
  key[2] = (uintptr_t)tuning_generation();
  key[3] = c->sg ? (uintptr_t)c->da.H1.p : 0;
}

int tca::run_sweeps(tca_ctx* c, const double* T, int32_t nsweeps, tca_update_record* log,
                    tca_sweep_stats* st, tca_surrogate* collect, int64_t row0) {
  DevBuf<tca_update_record> dlog;
  if (log && nsweeps > 0) {
    hipError_t e = dlog.alloc((size_t)nsweeps * c->N);
    if (e != hipSuccess) {
      set_err("log allocation failed: %s", hipGetErrorString(e));
      return TCA_E_NOMEM;
    }
  }
  if (nsweeps > c->sched_cap) {
    TCA_CK(hipStreamSynchronize(c->stream));
    if (c->sched_T) TCA_CK(hipFree(c->sched_T));
    c->sched_T = nullptr;
    c->sched_cap = 0;
    TCA_CK(hipMalloc((void**)&c->sched_T, sizeof(double) * (size_t)nsweeps));
    c->sched_cap = nsweeps;
  }
  tca_surrogate* sg = collect ? nullptr : c->sg;
  if (sg && sg->bf16_stale) {
    TCA_CK(sg_to_bf16(sg->W.p, sg->dm, sg->W1b.p, sg->W2b.p, c->stream));
    sg->bf16_stale = false;
  }
  ProfRec pr{c, (c->p.flags & TCA_FLAG_PROFILE) != 0};
  if (nsweeps > 0) {
    TCA_CK(hipMemcpyAsync(c->sched_T, T, sizeof(double) * (size_t)nsweeps, hipMemcpyHostToDevice,
                          c->stream));
    c->sched_host_base = c->sweep_counter;
    TCA_CK(hipMemcpyAsync(c->sched_base, &c->sched_host_base, sizeof(uint64_t),
                          hipMemcpyHostToDevice, c->stream));
  }
  TCA_CK(launch_zero_i32(c->sched_idx, 1, c->stream));
  TCA_CK(launch_zero_u64(c->counters, 4, c->stream));
  const SweepRef sr{c->sched_base, c->sched_idx, c->sched_T, 0, 0.0};
  const bool graph = !log && !collect && !pr.on && !(c->p.flags & TCA_FLAG_NO_GRAPH);
  if (graph && nsweeps > 0) {
    uintptr_t key[4];
    graph_key(c, key);
    if (!c->graph_exec || memcmp(key, c->graph_key, sizeof(key)) != 0) {
      if (c->graph_exec) TCA_CK(hipGraphExecDestroy(c->graph_exec));
      c->graph_exec = nullptr;
      TCA_CK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
      const int rc = issue_sweep(c, sr, c->sched_idx, nullptr, pr, nullptr, 0);
      hipGraph_t gr = nullptr;
      const hipError_t ec = hipStreamEndCapture(c->stream, &gr);
      if (rc != TCA_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      TCA_CK(ec);
      const hipError_t ei = hipGraphInstantiate(&c->graph_exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      TCA_CK(ei);
      memcpy(c->graph_key, key, sizeof(key));
      c->graph_captures += 1;
    }
  }
  TCA_CK(hipEventRecord(c->ev0, c->stream));
  for (int s = 0; s < nsweeps; ++s) {
    if (graph) {
      TCA_CK(hipGraphLaunch(c->graph_exec, c->stream));
    } else {
      const int rc = issue_sweep(c, sr, c->sched_idx, dlog.p, pr, collect, row0);
      if (rc != TCA_OK) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
      }
    }
  }
  TCA_CK(hipEventRecord(c->ev1, c->stream));
  TCA_CK(hipStreamSynchronize(c->stream));
  c->sweep_counter += (uint64_t)nsweeps;
  if (log && nsweeps > 0)
    TCA_CK(hipMemcpy(log, dlog.p, sizeof(tca_update_record) * (size_t)nsweeps * c->N,
                     hipMemcpyDeviceToHost));
  if (st) return fill_stats(c, pr, st);
  return TCA_OK;
}

int tca::check_temps(const double* T, int32_t nsweeps) {
  if (!T) TCA_INVAL("T is NULL");
  if (nsweeps < 0) TCA_INVAL("nsweeps < 0");
  for (int s = 0; s < nsweeps; ++s)
    if (!is_fin(T[s]) || T[s] <= 0.0) TCA_INVAL("temperatures must be finite and > 0");
  return TCA_OK;
}

extern "C" {

int tca_sweep(tca_ctx* c, const double* T, int32_t nsweeps, tca_update_record* log,
              tca_sweep_stats* st) {
  g_err[0] = 0;
  if (!c) TCA_INVAL("NULL context");
  const int rc = check_temps(T, nsweeps);
  if (rc != TCA_OK) return rc;
  return run_sweeps(c, T, nsweeps, log, st, nullptr, 0);
}

int tca_cluster_eigvals(tca_ctx* c, const int32_t* sites, const int32_t* Lc,
                        const double* proposed_xyz, int32_t count, double* eig, int32_t ld) {
  g_err[0] = 0;
  if (!c || !sites || !eig) TCA_INVAL("NULL argument");
  if (count < 0) TCA_INVAL("count < 0");
  if (count == 0) return TCA_OK;
  const int L = c->p.L;
  std::vector<int> lcs(count);
  for (int r = 0; r < count; ++r) {
    if (sites[r] < 0 || sites[r] >= c->N) TCA_INVAL("site out of range");
    lcs[r] = Lc ? Lc[r] : c->p.Lc;
    if (!check_Lc(lcs[r], L)) TCA_INVAL("cluster size out of range");
    if (ld < 2 * lcs[r] * lcs[r]) TCA_INVAL("ld < 2*Lc^2");
  }
  if (proposed_xyz && !unit_spins(proposed_xyz, count))
    TCA_INVAL("proposed spins must have unit norm within 1e-12");
  DevBuf<int32_t> dsites, dn;
  DevBuf<double> dprop, dev, dD, dE;
  TCA_CK(dsites.alloc(count));
  TCA_CK(dprop.alloc((size_t)3 * count));
  TCA_CK(dev.alloc((size_t)count * ld));
  TCA_CK(dD.alloc((size_t)count * kMaxN));
  TCA_CK(dE.alloc((size_t)count * kMaxN));
  TCA_CK(dn.alloc((size_t)count));
  const ReduceOut ro{dD.p, dE.p, kMaxN, dn.p};
  const ModelParams m = model_of(c);
  std::vector<int32_t> hs(count);
  std::vector<double> hp(3 * (size_t)count);
  for (int Lv = 2; Lv <= kMaxLc; ++Lv) {
    int k = 0;
    std::vector<int> rows;
    for (int r = 0; r < count; ++r)
      if (lcs[r] == Lv) {
        rows.push_back(r);
        hs[k] = sites[r];
        if (proposed_xyz)
          for (int a = 0; a < 3; ++a) hp[3 * k + a] = proposed_xyz[3 * r + a];
        ++k;
      }
    if (k == 0) continue;
    TCA_CK(hipMemcpy(dsites.p, hs.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice));
    if (proposed_xyz)
      TCA_CK(hipMemcpy(dprop.p, hp.data(), sizeof(double) * 3 * k, hipMemcpyHostToDevice));
    TCA_CK(launch_cluster_sites_reduce(c->p.precision, Lv, c->S, L, m, dsites.p,
                                       proposed_xyz ? dprop.p : nullptr, k, ro, c->stream));
    TCA_CK(launch_tridiag_eig(2 * Lv * Lv, k, ro, fixed_sweep(0, 1.0), 0.0, nullptr, dev.p, ld,
                              c->stream));
    TCA_CK(hipStreamSynchronize(c->stream));
    std::vector<double> tmp((size_t)k * ld);
    TCA_CK(hipMemcpy(tmp.data(), dev.p, sizeof(double) * k * ld, hipMemcpyDeviceToHost));
    for (int q = 0; q < k; ++q)
      memcpy(eig + (size_t)rows[q] * ld, tmp.data() + (size_t)q * ld,
             sizeof(double) * 2 * Lv * Lv);
  }
  return TCA_OK;
}

int tca_observables(tca_ctx* c, double* spins_out, double* Sq, double* m) {
  g_err[0] = 0;
  if (!c) TCA_INVAL("NULL context");
  const int N = c->N, L = c->p.L;
  if (Sq) {
    if (!c->sq_work) TCA_CK(hipMalloc((void**)&c->sq_work, sizeof(double) * 6 * N));
    if (!c->sq_out) TCA_CK(hipMalloc((void**)&c->sq_out, sizeof(double) * N));
    TCA_CK(launch_sq(c->S, L, c->sq_work, c->sq_out, c->stream));
  }
  TCA_CK(hipStreamSynchronize(c->stream));
  if (Sq) TCA_CK(hipMemcpy(Sq, c->sq_out, sizeof(double) * N, hipMemcpyDeviceToHost));
  if (spins_out || m) {
    std::vector<double> tmp;
    double* dst = spins_out;
    if (!dst) {
      tmp.resize(3 * (size_t)N);
      dst = tmp.data();
    }
    TCA_CK(hipMemcpy(dst, c->S, sizeof(double) * 3 * N, hipMemcpyDeviceToHost));
    if (m) {
      double a[3] = {0, 0, 0};
      for (int p = 0; p < N; ++p)
        for (int k = 0; k < 3; ++k) a[k] += dst[3 * p + k];
      for (int k = 0; k < 3; ++k) m[k] = a[k] / N;
    }
  }
  return TCA_OK;
}

static int heevals_checks(const double* A, int32_t n, int32_t batch, int32_t precision) {
  if (!A) TCA_INVAL("A is NULL");
  if (!supported_n(n)) TCA_INVAL("n must satisfy 2 <= n <= 200");
  if (batch < 0) TCA_INVAL("batch < 0");
  if (precision != TCA_FP64 && precision != TCA_MIXED) TCA_INVAL("bad precision");
  return TCA_OK;
}

// Grow-only device workspace of the device-pointer entry point.
static std::mutex g_ws_mu;
static double* g_ws = nullptr;
static size_t g_ws_bytes = 0;

int tca_heevals_batched_dev(const double* A, int32_t n, int32_t batch, int32_t precision,
                            double T, double mu, double* w, double* F, void* hip_stream) {
  g_err[0] = 0;
  int s = heevals_checks(A, n, batch, precision);
  if (s != TCA_OK) return s;
  if (F && (!is_fin(T) || T <= 0.0 || !is_fin(mu))) TCA_INVAL("T must be > 0 and mu finite");
  if (batch == 0) return TCA_OK;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  const size_t need = (size_t)batch * (2 * n * sizeof(double) + sizeof(int32_t)) + 256;
  if (need > g_ws_bytes) {
    if (g_ws) TCA_CK(hipFree(g_ws));
    g_ws = nullptr;
    g_ws_bytes = 0;
    TCA_CK(hipMalloc((void**)&g_ws, need));
    g_ws_bytes = need;
  }
  const ReduceOut ro{g_ws, g_ws + (size_t)batch * n, n, (int32_t*)(g_ws + (size_t)2 * batch * n)};
  hipStream_t st = (hipStream_t)hip_stream;
  TCA_CK(launch_heevals_reduce(precision, n, A, batch, ro, st));
  TCA_CK(launch_tridiag_eig(n, batch, ro, fixed_sweep(0, F ? T : 1.0), mu, F, w, n, st));
  return TCA_OK;
}

int tca_heevals_batched(const double* A, int32_t n, int32_t batch, int32_t precision, double T,
                        double mu, double* w, double* F) {
  g_err[0] = 0;
  int s = heevals_checks(A, n, batch, precision);
  if (s != TCA_OK) return s;
  if (!w && !F) TCA_INVAL("w and F are both NULL");
  if (F && (!is_fin(T) || T <= 0.0 || !is_fin(mu))) TCA_INVAL("T must be > 0 and mu finite");
  if (batch == 0) return TCA_OK;
  const size_t nA = (size_t)batch * n * n * 2;
  DevBuf<double> dA, dw, dF, dD, dE;
  DevBuf<int32_t> dn;
  TCA_CK(dA.alloc(nA));
  TCA_CK(dw.alloc((size_t)batch * n));
  TCA_CK(dF.alloc((size_t)batch));
  TCA_CK(dD.alloc((size_t)batch * n));
  TCA_CK(dE.alloc((size_t)batch * n));
  TCA_CK(dn.alloc((size_t)batch));
  TCA_CK(hipMemcpy(dA.p, A, sizeof(double) * nA, hipMemcpyHostToDevice));
  const ReduceOut ro{dD.p, dE.p, n, dn.p};
  TCA_CK(launch_heevals_reduce(precision, n, dA.p, batch, ro, nullptr));
  TCA_CK(launch_tridiag_eig(n, batch, ro, fixed_sweep(0, F ? T : 1.0), mu, F ? dF.p : nullptr,
                            w ? dw.p : nullptr,
                            n, nullptr));
  TCA_CK(hipDeviceSynchronize());
  if (w) TCA_CK(hipMemcpy(w, dw.p, sizeof(double) * batch * n, hipMemcpyDeviceToHost));
  if (F) TCA_CK(hipMemcpy(F, dF.p, sizeof(double) * batch, hipMemcpyDeviceToHost));
  return TCA_OK;
}

}  // extern "C"
