// Internal interface between the C ABI (api.hip) and the kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tca.h"

namespace tca {

constexpr int kMaxLc = 10;
constexpr int kMaxN = 2 * kMaxLc * kMaxLc;  // 200

// Which cluster of a block a workgroup pair works on.
struct BlockGeom {
  int L;      // lattice size
  int h;      // block side L/2
  int x0, y0; // block origin
};

struct ModelParams {
  double t, JH, JAF, mu;
  uint64_t seed;
};

// Size classes of one block, filled on the device: list[k][*] holds cluster
// indices (c = i + h*j within the block) whose drawn size is class k.
struct ClassLists {
  int32_t* count;   // [4]
  int32_t* list;    // [4][h*h]
};

hipError_t launch_cluster_block(int precision, int Lc, const double* S, BlockGeom g,
                                ModelParams m, uint64_t sweep, double T, const int32_t* list,
                                const int32_t* count, int max_clusters, double* Fpair,
                                hipStream_t st);

hipError_t launch_cluster_eig(int precision, int Lc, const double* S, int L, ModelParams m,
                              const int32_t* sites, const double* prop, int count, double* ev,
                              int ld, hipStream_t st);

hipError_t launch_heevals(int precision, int n, const double* A, int batch, double T, double mu,
                          double* w, double* F, hipStream_t st);

hipError_t launch_classify(const int32_t* classes_Lc, int n_classes, BlockGeom g, uint64_t seed,
                           uint64_t sweep, ClassLists cl, hipStream_t st);

hipError_t launch_decide(double* S, const double* Fpair, BlockGeom g, ModelParams m,
                         uint64_t sweep, double T, int Lc_fixed, const int32_t* classes_Lc,
                         int n_classes, int K, tca_update_record* log_dev,
                         unsigned long long* counters, hipStream_t st);

hipError_t launch_init_spins(double* S, int L, int kind, uint64_t seed, hipStream_t st);

hipError_t launch_sq(const double* S, int L, double* work /* L*L*6 */, double* Sq,
                     hipStream_t st);

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);

bool supported_n(int n);

}  // namespace tca
