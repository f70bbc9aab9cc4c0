// Internal interface between the C ABI (api.hip) and the kernels
// (cluster_kernels.hip, sweep_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tca.h"

namespace tca {

constexpr int kMaxLc = 10;
constexpr int kMaxN = 2 * kMaxLc * kMaxLc;  // 200

// One parallel block of the sweep: the (L/2) x (L/2) quadrant with origin
// (x0, y0); cluster c of the block is anchored at (x0 + c % h, y0 + c / h).
struct BlockGeom {
  int L;
  int h;
  int x0, y0;
};

struct ModelParams {
  double t, JH, JAF, mu;
  uint64_t seed;
  double decide_gap;  // relative band around the Metropolis threshold decided by the exact form
};

// Default band: outside it ln u and -dE/T differ by far more than the rounding
// of log, exp and the quotient, so the comparison of logarithms decides.
constexpr double kDecideGap = 1e-10;

// Size classes of one block, filled on the device: list[k][*] holds the
// cluster indices c whose drawn size is class k.
struct ClassLists {
  int32_t* count;  // [4]
  int32_t* list;   // [4][h*h]
};

// Tridiagonal output of the reduction kernels: matrix m has diagonal
// D[m*ld .. m*ld+n), squared off-diagonal E2[m*ld .. m*ld+n-1), n = nmat[m].
struct ReduceOut {
  double* D;
  double* E2;
  int ld;
  int32_t* nmat;
};

// Sweep counter and temperature of the sweep being run.  Inside tca_sweep the
// kernels read them from device memory (sweep = *base + *idx, T = Ts[*idx]) so
// that one captured sweep graph can be replayed for every sweep of a call;
// elsewhere they are fixed values (base == nullptr).
struct SweepRef {
  const uint64_t* base;
  const int32_t* idx;
  const double* Ts;
  uint64_t sweep0;
  double T0;
  __device__ __forceinline__ uint64_t sweep() const {
    return base != nullptr ? *base + (uint64_t)*idx : sweep0;
  }
  __device__ __forceinline__ double T() const { return base != nullptr ? Ts[*idx] : T0; }
  __device__ __forceinline__ int s() const { return base != nullptr ? *idx : 0; }
};
inline SweepRef fixed_sweep(uint64_t sweep, double T) {
  return SweepRef{nullptr, nullptr, nullptr, sweep, T};
}

bool supported_n(int n);

// Reducer variants: dimension classes n <= 32, 64, 80, 128, 176, 208; the
// autotuner records the fastest variant of each (class, precision).
constexpr int kNumReducerClasses = 6;
int reducer_class(int n);  // -1 if n is too large
int reducer_variants(int cls, int precision);
const char* reducer_name(int cls, int precision, int variant);
int reducer_choice(int cls, int precision);
void set_reducer_choice(int cls, int precision, int variant);

// matrices 2c (old) and 2c+1 (new, proposal at the corner) of every cluster c
// of a block (or of the clusters listed for one size class)
// (variant -1: the recorded choice)
hipError_t launch_cluster_block_reduce(int precision, int Lc, const double* S, BlockGeom g,
                                       ModelParams m, SweepRef sr, const int32_t* list,
                                       const int32_t* count, int max_clusters, ReduceOut out,
                                       hipStream_t st, int variant = -1);

hipError_t launch_cluster_sites_reduce(int precision, int Lc, const double* S, int L,
                                       ModelParams m, const int32_t* sites, const double* prop,
                                       int count, ReduceOut out, hipStream_t st);

hipError_t launch_heevals_reduce(int precision, int n, const double* A, int batch, ReduceOut out,
                                 hipStream_t st, int variant = -1);

// eigenvalues (optional) and grand potential F (optional) of nmats tridiagonals;
// with list/count, only matrices 2*list[i] and 2*list[i]+1, i < *count
hipError_t launch_tridiag_eig(int nmax, int nmats, ReduceOut in, SweepRef sr, double mu,
                              double* F, double* ev, int ev_ld, hipStream_t st,
                              const int32_t* list = nullptr, const int32_t* count = nullptr);

hipError_t launch_classify(const int32_t* classes_Lc, int n_classes, BlockGeom g, uint64_t seed,
                           SweepRef sr, ClassLists cl, hipStream_t st);

// pass/dS: stage-1 flags and surrogate values of delayed acceptance, or nullptr
// log_base: records of the whole call (sweep s of the call at log_base + s*L*L), or nullptr;
// prep: decide_prep_bytes(h*h) bytes of device scratch
hipError_t launch_decide(double* S, const double* Fpair, BlockGeom g, ModelParams m, SweepRef sr,
                         int Lc_fixed, const int32_t* classes_Lc, int n_classes, int K,
                         const uint8_t* pass, const float* dS, void* prep,
                         tca_update_record* log_base, unsigned long long* counters,
                         hipStream_t st);
size_t decide_prep_bytes(int clusters);

// *idx += 1 (end of a sweep inside a call)
hipError_t launch_advance(int32_t* idx, hipStream_t st);

hipError_t launch_init_spins(double* S, int L, int kind, uint64_t seed, hipStream_t st);

hipError_t launch_sq(const double* S, int L, double* work /* L*L*6 */, double* Sq,
                     hipStream_t st);

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st);

}  // namespace tca
