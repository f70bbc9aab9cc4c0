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
};

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

bool supported_n(int n);

// matrices 2c (old) and 2c+1 (new, proposal at the corner) of every cluster c
// of a block (or of the clusters listed for one size class)
hipError_t launch_cluster_block_reduce(int precision, int Lc, const double* S, BlockGeom g,
                                       ModelParams m, uint64_t sweep, const int32_t* list,
                                       const int32_t* count, int max_clusters, ReduceOut out,
                                       hipStream_t st);

hipError_t launch_cluster_sites_reduce(int precision, int Lc, const double* S, int L,
                                       ModelParams m, const int32_t* sites, const double* prop,
                                       int count, ReduceOut out, hipStream_t st);

hipError_t launch_heevals_reduce(int precision, int n, const double* A, int batch, ReduceOut out,
                                 hipStream_t st);

// eigenvalues (optional) and grand potential F (optional) of nmats tridiagonals;
// with list/count, only matrices 2*list[i] and 2*list[i]+1, i < *count
hipError_t launch_tridiag_eig(int nmax, int nmats, ReduceOut in, double T, double mu, double* F,
                              double* ev, int ev_ld, hipStream_t st,
                              const int32_t* list = nullptr, const int32_t* count = nullptr);

hipError_t launch_classify(const int32_t* classes_Lc, int n_classes, BlockGeom g, uint64_t seed,
                           uint64_t sweep, ClassLists cl, hipStream_t st);

// pass/dS: stage-1 flags and surrogate values of delayed acceptance, or nullptr
hipError_t launch_decide(double* S, const double* Fpair, BlockGeom g, ModelParams m,
                         uint64_t sweep, double T, int Lc_fixed, const int32_t* classes_Lc,
                         int n_classes, int K, const uint8_t* pass, const float* dS,
                         tca_update_record* log_dev, unsigned long long* counters,
                         hipStream_t st);

hipError_t launch_init_spins(double* S, int L, int kind, uint64_t seed, hipStream_t st);

hipError_t launch_sq(const double* S, int L, double* work /* L*L*6 */, double* Sq,
                     hipStream_t st);

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);

}  // namespace tca
