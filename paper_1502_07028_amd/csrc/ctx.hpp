// Host-side objects behind the opaque handles of the C ABI (include/tca.h),
// shared by api.hip (lattice contexts) and api_surrogate.hip (the learned
// first stage), plus the error-reporting helpers of both.
#pragma once
#include <hip/hip_runtime.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "internal.hpp"
#include "surrogate.hpp"

namespace tca {

extern thread_local char g_err[512];

inline void set_err(const char* fmt, const char* a = "", int line = 0) {
  snprintf(g_err, sizeof(g_err), fmt, a, line);
}

#define TCA_CK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::tca::set_err("HIP error %s at line %d", hipGetErrorString(e_), __LINE__); \
      return TCA_E_DEVICE;                                                        \
    }                                                                             \
  } while (0)

#define TCA_INVAL(msg)          \
  do {                          \
    ::tca::set_err("%s", msg);  \
    return TCA_E_INVAL;         \
  } while (0)

// Device buffer freed on scope exit.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  hipError_t alloc(size_t n) {
    reset();
    return hipMalloc((void**)&p, n * sizeof(T) + 16);
  }
};

// Buffers of delayed acceptance inside a sweep (sized for one block).
struct DaBufs {
  int rows = 0;           // 2 * clusters per block
  DevBuf<uint16_t> Fin;   // rows x kpad BF16 features
  DevBuf<uint16_t> H1;    // rows x H BF16
  DevBuf<uint16_t> H2;    // rows x H BF16
  DevBuf<float> dS;       // rows surrogate values (2c forward, 2c+1 reverse)
  DevBuf<uint8_t> pass;   // clusters
  DevBuf<int32_t> count;  // 1
  DevBuf<int32_t> list;   // clusters
};

}  // namespace tca

struct tca_surrogate {
  int Lc = 0;
  tca::SurrogateDims dm{};
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  int64_t capacity = 0, rows = 0;
  int64_t adam_t = 0;                          // Adam steps taken
  tca::DevBuf<float> W, G, m, v;               // nparam each
  tca::DevBuf<uint16_t> W1b, W2b;              // BF16 copies for inference
  bool bf16_stale = true;                      // W changed since the BF16 copies were made
  tca::DevBuf<float> X, y;                     // dataset: capacity x n_in, capacity
  int tb_rows = 0;                             // capacity of the training buffers
  tca::DevBuf<float> Xb, yb, z1, h1, z2, h2, out, dout, dz1, dz2, dh;
  tca::DevBuf<double> loss;                    // per-step losses of the last train call
  int64_t loss_cap = 0;
};

struct tca_ctx {
  tca_params p;
  hipStream_t stream = nullptr;
  int N = 0, h = 0;
  double* S = nullptr;           // N x 3
  double* F = nullptr;           // 2 * h*h grand potentials (old, new per cluster)
  double* D = nullptr;           // 2 * h*h * ld tridiagonal diagonals
  double* E2 = nullptr;          // 2 * h*h * ld squared off-diagonals
  int32_t* nmat = nullptr;       // 2 * h*h matrix dimensions
  int ld = 0;                    // 2 * (largest Lc)^2
  int32_t* cls_count = nullptr;  // 4
  int32_t* cls_list = nullptr;   // 4 * h*h
  unsigned long long* counters = nullptr;  // 4: accepted, near-threshold, updates, stage-1 passes
  void* prep = nullptr;          // per-cluster decision records of one block
  double* sq_work = nullptr;     // 6 N
  double* sq_out = nullptr;      // N
  uint64_t sweep_counter = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> prof;  // event pool for TCA_FLAG_PROFILE
  tca_surrogate* sg = nullptr;   // first stage of delayed acceptance, or none
  tca::DaBufs da;
  bool own_stream = false;       // stream created by the context (none was given)
  // device-side sweep schedule of the current call: sweep counter base, index
  // of the sweep being run, temperatures
  uint64_t* sched_base = nullptr;
  int32_t* sched_idx = nullptr;
  double* sched_T = nullptr;
  int sched_cap = 0;
  uint64_t sched_host_base = 0;
  hipGraphExec_t graph_exec = nullptr;  // one captured sweep, replayed per sweep
  uintptr_t graph_key[4] = {0, 0, 0, 0};
  int64_t graph_captures = 0;
  std::string tune_report;
};

namespace tca {
// nsweeps sweeps of a context, synchronized; `collect` appends (features, dF)
// rows of every update to that surrogate's dataset from row `row0` on.
int run_sweeps(tca_ctx* c, const double* T, int32_t nsweeps, tca_update_record* log,
               tca_sweep_stats* st, tca_surrogate* collect, int64_t row0);
// TCA_E_INVAL unless T holds nsweeps finite positive temperatures.
int check_temps(const double* T, int32_t nsweeps);
// Changes whenever the autotuner records a new reducer choice (captured
// graphs depending on the old choice are then re-captured).
int tuning_generation();
}  // namespace tca
