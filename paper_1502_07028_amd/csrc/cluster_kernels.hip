// Cluster solves of the traveling cluster approximation on gfx950.
//
// The paper diagonalizes the cluster Hamiltonian before and after the proposed
// change of the update-site spin (Sec. II(c), Fig. 2 steps (b) and (d)), for
// every cluster of a parallel block at once (Sec. III(a)).  Here each matrix is
// one workgroup of the reduction kernel (build or load -> Householder
// tridiagonalization in registers -> (d, e^2) to global memory); a second,
// high-occupancy kernel finds all eigenvalues of every tridiagonal and sums the
// grand potential.
//
//  cluster_block_reduce  matrices (old, new) of every cluster of one block
//  cluster_sites_reduce  matrices around given sites (eigenvalue queries)
//  heevals_reduce        raw Hermitian matrices from global memory
//  tridiag_eig_kernel    eigenvalues + F = sum_i [min(x,0) - T log1p(e^{-|x|/T})]
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <unordered_map>
#include <type_traits>

#include "internal.hpp"
#include "reduce_full.hpp"
#include "reduce_fused.hpp"
#include "reduce_lower.hpp"
#include "reduce_split.hpp"
#include "rng.hpp"
#include "tridiag.hpp"

namespace tca {

// -------------------------------------------------------------------------
// Cluster Hamiltonian entry (i >= j) of the double-exchange model:
//   hopping -t for each of the four periodic cluster directions linking the
//   two sites (so -2t when Lc == 2), same spin;
//   on-site block -(J_H/2) [[Sz, Sx - i Sy], [Sx + i Sy, -Sz]].
// Basis index 2*l + s, cluster site l = a + Lc*b.
template <typename R>
__device__ __forceinline__ cx<R> h_elem(int i, int j, int Lc, double t, double JH,
                                        const double* sp) {
  const int li = i >> 1, si = i & 1, lj = j >> 1, sj = j & 1;
  double re = 0.0, im = 0.0;
  if (li == lj) {
    const double h = -0.5 * JH;
    const double* s = sp + 3 * li;
    if (si == sj) {
      re = (si == 0) ? h * s[2] : -h * s[2];
    } else {  // (2l+1, 2l): h (Sx + i Sy)
      re = h * s[0];
      im = h * s[1];
    }
  } else if (si == sj) {
    const int a = li % Lc, b = li / Lc;
    const int cnt = (lj == (a + 1) % Lc + Lc * b) + (lj == (a + Lc - 1) % Lc + Lc * b) +
                    (lj == a + Lc * ((b + 1) % Lc)) + (lj == a + Lc * ((b + Lc - 1) % Lc));
    re = -t * (double)cnt;
  }
  return {(R)re, (R)im};
}

// Cluster spins (cluster order l = a + Lc*b) of the cluster anchored at (px, py).
__device__ __forceinline__ void gather_spins(const double* __restrict__ S, int L, int px, int py,
                                             int Lc, double* sp) {
  const int Nc = Lc * Lc;
  for (int q = threadIdx.x; q < 3 * Nc; q += blockDim.x) {
    const int l = q / 3, comp = q % 3;
    const int a = l % Lc, b = l / Lc;
    const int sx = (px + a) % L, sy = (py + b) % L;
    sp[q] = S[3 * (sx + L * sy) + comp];
  }
}

template <class Red, typename R>
__device__ __forceinline__ void solve_cluster(const double* sp, int Lc, const ModelParams& m,
                                              typename Red::Smem& sm, double* d, double* e2) {
  const int n = 2 * Lc * Lc;
  typename Red::Regs A;
  Red::load(A, n, [&](int i, int j) { return h_elem<R>(i, j, Lc, m.t, m.JH, sp); });
  Red::run(n, A, sm, d, e2);
}

// One workgroup per matrix: matrix 2c is the old and 2c+1 the new cluster c.
// With a compacted work list (survivors of the first stage, or one size
// class) the bound is read on the device; the listed items occupy the first
// workgroups and the rest exit at once.  (A persistent loop around the
// register-resident reduction makes the compiler spill the matrix, so the
// reduction kernels keep one item per workgroup.)
template <class Red, typename R>
__global__ __launch_bounds__(Red::NT, Red::MINW) void cluster_block_reduce(
    const double* __restrict__ S, BlockGeom g, int Lc, ModelParams m, SweepRef sr,
    const int32_t* __restrict__ list, const int32_t* __restrict__ count, int max_clusters,
    ReduceOut out) {
  __shared__ typename Red::Smem sm;
  __shared__ double sp[3 * kMaxLc * kMaxLc];
  const int w = blockIdx.x;
  if (w >= 2 * (list != nullptr ? *count : max_clusters)) return;
  const int ci = w >> 1, which = w & 1;
  const int c = list != nullptr ? list[ci] : ci;
  const int px = g.x0 + c % g.h, py = g.y0 + c / g.h;
  const int site = px + g.L * py;
  gather_spins(S, g.L, px, py, Lc, sp);
  __syncthreads();
  if (which == 1 && threadIdx.x == 0) sphere_point(m.seed, sr.sweep(), site, kStreamProposal, sp);
  __syncthreads();
  const int mat = 2 * c + which;
  solve_cluster<Red, R>(sp, Lc, m, sm, out.D + (size_t)mat * out.ld,
                        out.E2 + (size_t)mat * out.ld);
  if (threadIdx.x == 0) out.nmat[mat] = 2 * Lc * Lc;
}

template <class Red, typename R>
__global__ __launch_bounds__(Red::NT, Red::MINW) void cluster_sites_reduce(
    const double* __restrict__ S, int L, int Lc, ModelParams m, const int32_t* __restrict__ sites,
    const double* __restrict__ prop, ReduceOut out) {
  __shared__ typename Red::Smem sm;
  __shared__ double sp[3 * kMaxLc * kMaxLc];
  const int w = blockIdx.x;
  const int site = sites[w];
  gather_spins(S, L, site % L, site / L, Lc, sp);
  __syncthreads();
  if (prop != nullptr && threadIdx.x < 3) sp[threadIdx.x] = prop[3 * w + threadIdx.x];
  __syncthreads();
  solve_cluster<Red, R>(sp, Lc, m, sm, out.D + (size_t)w * out.ld, out.E2 + (size_t)w * out.ld);
  if (threadIdx.x == 0) out.nmat[w] = 2 * Lc * Lc;
}

template <class Red, typename R>
__global__ __launch_bounds__(Red::NT, Red::MINW) void heevals_reduce(const double* __restrict__ Ag,
                                                                     int n, ReduceOut out) {
  __shared__ typename Red::Smem sm;
  const int b = blockIdx.x;
  const double* M = Ag + (size_t)b * n * n * 2;
  typename Red::Regs A;
  Red::load(A, n, [&](int i, int j) -> cx<R> {
    const size_t o = 2 * ((size_t)i * n + j);
    return {(R)M[o], i == j ? R(0) : (R)M[o + 1]};
  });
  Red::run(n, A, sm, out.D + (size_t)b * out.ld, out.E2 + (size_t)b * out.ld);
  if (threadIdx.x == 0) out.nmat[b] = n;
}

// One workgroup per tridiagonal (persistent over the matrices).  The matrix is
// staged in LDS as (d_i, e2_{i-1}) pairs.  A first pass slices the spectrum:
// the threads count the eigenvalues below 4 NTHR evenly spaced points of the
// Gershgorin interval (four interleaved counts per thread), which brackets
// every eigenvalue to one slice; then thread j finishes eigenvalues j,
// j + NTHR, ... from their slices (bisection until isolated, then safeguarded
// Laguerre steps), and the grand potential is reduced in a fixed order.
template <int NTHR>
__global__ __launch_bounds__(NTHR) void tridiag_eig_kernel(const double* __restrict__ D,
                                                           const double* __restrict__ E2, int ld,
                                                           const int32_t* __restrict__ nmat,
                                                           int nmats, SweepRef sr, double mu,
                                                           double* __restrict__ F,
                                                           double* __restrict__ ev, int ev_ld,
                                                           const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ count) {
  constexpr int NW = NTHR / 64;
  constexpr int SPT = 4;             // slice points per thread
  constexpr int NS = SPT * NTHR;     // slice points
  __shared__ double2 de[kMaxN];
  __shared__ int cnt[NS];
  __shared__ double red[NW], wlo[NW], whi[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double T = sr.T();
  const int limit = list != nullptr ? 2 * *count : nmats;
  for (int w = blockIdx.x; w < limit; w += gridDim.x) {
    const int mat = list != nullptr ? 2 * list[w >> 1] + (w & 1) : w;
    const int n = nmat[mat];
    const double* d = D + (size_t)mat * ld;
    const double* e2 = E2 + (size_t)mat * ld;
    // stage the pairs and the Gershgorin bounds
    double lo = DBL_MAX, hi = -DBL_MAX;
    for (int i = tid; i < n; i += NTHR) {
      const double el = i > 0 ? e2[i - 1] : 0.0, er = i < n - 1 ? e2[i] : 0.0;
      const double di = d[i];
      de[i] = make_double2(di, el);
      const double r = sqrt(el) + sqrt(er);
      lo = fmin(lo, di - r);
      hi = fmax(hi, di + r);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) {
      wlo[wave] = lo;
      whi[wave] = hi;
    }
    __syncthreads();
    lo = wlo[0];
    hi = whi[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      lo = fmin(lo, wlo[q]);
      hi = fmax(hi, whi[q]);
    }
    const double span = fmax(fmax(fabs(lo), fabs(hi)), DBL_MIN);
    const double widen = 2.0 * DBL_EPSILON * span * (double)n;
    lo -= widen;
    hi += widen;
    const double tol = 2.0 * DBL_EPSILON * span;
    // slice the spectrum at x_t = lo + (t + 1) (hi - lo) / (NS + 1), SPT points
    // per thread counted together
    const double h = (hi - lo) / (double)(NS + 1);
    {
      double xs[SPT];
      int cs[SPT];
#pragma unroll
      for (int m = 0; m < SPT; ++m) xs[m] = fma((double)(tid + m * NTHR + 1), h, lo);
      sturm_count_pairs_multi<SPT>(n, xs, de, cs);
#pragma unroll
      for (int m = 0; m < SPT; ++m) cnt[tid + m * NTHR] = cs[m];
    }
    __syncthreads();
    double acc = 0.0;
    for (int j = tid; j < n; j += NTHR) {
      // last slice point with count <= j (counts are nondecreasing in x)
      int lo_t = -1, hi_t = NS;  // cnt[lo_t] <= j < cnt[hi_t] (virtual ends 0 and n)
      while (hi_t - lo_t > 1) {
        const int mid = (lo_t + hi_t) >> 1;
        if (cnt[mid] <= j)
          lo_t = mid;
        else
          hi_t = mid;
      }
      double a = lo_t < 0 ? lo : fma((double)(lo_t + 1), h, lo);
      double b = hi_t >= NS ? hi : fma((double)(hi_t + 1), h, lo);
      int ca = lo_t < 0 ? 0 : cnt[lo_t];
      int cb = hi_t >= NS ? n : cnt[hi_t];
      if (!(ca <= j && j < cb)) {  // a count that broke monotonicity: full interval
        a = lo;
        b = hi;
        ca = 0;
        cb = n;
      }
      const double lam = tri_eigenvalue_pairs(n, j, de, a, b, ca, cb, tol);
      if (ev != nullptr) ev[(size_t)mat * ev_ld + j] = lam;
      if (F != nullptr) acc += omega_term(lam, T, mu);
    }
    if (F != nullptr) {
      acc = wave_total(acc);
      if (lane == 0) red[wave] = acc;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += red[q];
        F[mat] = s;
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------------
// Reducer variants per (dimension class, precision); the autotuner times them
// and records the fastest in a process-wide table.  Class k covers
// n <= kClassMaxN[k].  Full storage on a TR x TC grid where the matrix fits
// the register file (fused or two-pass step), lower-triangle storage above
// dimension 128 in FP64.
constexpr int kClassMaxN[kNumReducerClasses] = {32, 64, 80, 128, 176, 208};

template <typename F>
static hipError_t dispatch_variant(int cls, int precision, int v, F&& f) {
  if (precision == TCA_MIXED) {
    using R = float;
    switch (cls) {
      case 0: return v == 0 ? f(ReduceFused<8, 8, 4, 4, R>{}, R{}) : f(ReduceFull<8, 8, 4, 4, R>{}, R{});
      case 1:
        return v == 0   ? f(ReduceFused<16, 16, 4, 4, R>{}, R{})
               : v == 1 ? f(ReduceFull<16, 16, 4, 4, R>{}, R{})
                        : f(ReduceSplit<16, 16, 4, 4, R>{}, R{});
      case 2:
        return v == 0   ? f(ReduceFused<16, 16, 5, 5, R>{}, R{})
               : v == 1 ? f(ReduceFull<16, 16, 5, 5, R>{}, R{})
                        : f(ReduceSplit<16, 16, 5, 5, R>{}, R{});
      case 3:
        return v == 0   ? f(ReduceFused<32, 16, 4, 8, R>{}, R{})
               : v == 1 ? f(ReduceFused<32, 16, 4, 8, R, 2>{}, R{})
               : v == 2 ? f(ReduceFull<32, 16, 4, 8, R>{}, R{})
               : v == 3 ? f(ReduceFused<32, 16, 4, 8, R, 0, true>{}, R{})
               : v == 4 ? f(ReduceFused<32, 16, 4, 8, R, 2, true>{}, R{})
               : v == 5 ? f(ReduceSplit<32, 16, 4, 8, R, 2>{}, R{})
               : v == 6 ? f(ReduceSplit<32, 16, 4, 8, R, 2, true>{}, R{})
               : v == 7 ? f(ReduceSplit<16, 16, 8, 8, R, 2>{}, R{})
               : v == 8 ? f(ReduceFused<16, 16, 8, 8, R, 2>{}, R{})
               : v == 9 ? f(ReduceSplit<16, 16, 8, 8, R, 2, true>{}, R{})
                        : f(ReduceSplit<32, 8, 4, 16, R, 2>{}, R{});
      case 4:
        return v == 0   ? f(ReduceFused<32, 16, 6, 11, R, 2>{}, R{})
               : v == 1 ? f(ReduceFull<32, 16, 6, 11, R>{}, R{})
               : v == 2 ? f(ReduceLower<32, 6, R>{}, R{})
                        : f(ReduceSplit<32, 16, 6, 11, R, 2>{}, R{});
      case 5:
        return v == 0   ? f(ReduceFused<32, 16, 7, 13, R, 2>{}, R{})
               : v == 1 ? f(ReduceFull<32, 16, 7, 13, R>{}, R{})
               : v == 2 ? f(ReduceLower<32, 7, R>{}, R{})
                        : f(ReduceSplit<32, 16, 7, 13, R, 2>{}, R{});
    }
  } else {
    using R = double;
    switch (cls) {
      case 0: return v == 0 ? f(ReduceFused<8, 8, 4, 4, R>{}, R{}) : f(ReduceFull<8, 8, 4, 4, R>{}, R{});
      case 1:
        return v == 0   ? f(ReduceFused<16, 16, 4, 4, R>{}, R{})
               : v == 1 ? f(ReduceFull<16, 16, 4, 4, R>{}, R{})
                        : f(ReduceSplit<16, 16, 4, 4, R>{}, R{});
      case 2:
        return v == 0   ? f(ReduceFused<16, 16, 5, 5, R>{}, R{})
               : v == 1 ? f(ReduceFull<16, 16, 5, 5, R>{}, R{})
                        : f(ReduceSplit<16, 16, 5, 5, R>{}, R{});
      case 3:
        return v == 0   ? f(ReduceFused<32, 16, 4, 8, R>{}, R{})
               : v == 1 ? f(ReduceFull<32, 16, 4, 8, R>{}, R{})
               : v == 2 ? f(ReduceFused<32, 16, 4, 8, R, 0, true>{}, R{})
               : v == 3 ? f(ReduceSplit<32, 16, 4, 8, R>{}, R{})
               : v == 4 ? f(ReduceSplit<32, 16, 4, 8, R, 0, true>{}, R{})
               : v == 5 ? f(ReduceSplit<32, 16, 4, 8, R, 0, true, 3>{}, R{})
               : v == 6 ? f(ReduceSplit<32, 16, 4, 8, R, 0, true, 0, true>{}, R{})
                        : f(ReduceSplit<32, 16, 4, 8, R, 0, false, 0, true>{}, R{});
      case 4: return f(ReduceLower<16, 11, R>{}, R{});
      case 5: return f(ReduceLower<16, 13, R>{}, R{});
    }
  }
  return hipErrorInvalidValue;
}

constexpr int kMaxVariants = 11;
static const char* const kVariantNames[2][kNumReducerClasses][kMaxVariants] = {
    {{"fused 8x8 grid", "two-pass 8x8 grid"},
     {"fused 16x16 grid", "two-pass 16x16 grid", "split 16x16 grid"},
     {"fused 16x16 grid", "two-pass 16x16 grid", "split 16x16 grid"},
     {"fused 32x16 grid", "two-pass 32x16 grid", "fused 32x16 grid, rank-2 update on MFMA",
      "split 32x16 grid", "split 32x16 grid, rank-2 update on MFMA",
      "split 32x16 grid, rank-2 update on MFMA and vector ALUs",
      "split 32x16 grid, rank-2 update on MFMA, reflector on half the wavefronts",
      "split 32x16 grid, reflector on half the wavefronts"},
     {"lower-triangle 16x16 grid"},
     {"lower-triangle 16x16 grid"}},
    {{"fused 8x8 grid", "two-pass 8x8 grid"},
     {"fused 16x16 grid", "two-pass 16x16 grid", "split 16x16 grid"},
     {"fused 16x16 grid", "two-pass 16x16 grid", "split 16x16 grid"},
     {"fused 32x16 grid, 2 workgroups/CU", "fused 32x16 grid, 1 workgroup/CU",
      "two-pass 32x16 grid", "fused 32x16 grid, rank-2 update on MFMA, 2 workgroups/CU",
      "fused 32x16 grid, rank-2 update on MFMA, 1 workgroup/CU",
      "split 32x16 grid, 2 workgroups/CU",
      "split 32x16 grid, rank-2 update on MFMA, 2 workgroups/CU",
      "split 16x16 grid, 2 workgroups/CU", "fused 16x16 grid, 2 workgroups/CU",
      "split 16x16 grid, rank-2 update on MFMA, 2 workgroups/CU",
      "split 32x8 grid, 2 workgroups/CU"},
     {"fused 32x16 grid", "two-pass 32x16 grid", "lower-triangle 32x32 grid", "split 32x16 grid"},
     {"fused 32x16 grid", "two-pass 32x16 grid", "lower-triangle 32x32 grid", "split 32x16 grid"}}};

static std::atomic<int> g_choice[2][kNumReducerClasses];

int reducer_class(int n) {
  for (int k = 0; k < kNumReducerClasses; ++k)
    if (n <= kClassMaxN[k]) return k;
  return -1;
}

int reducer_variants(int cls, int precision) {
  int v = 0;
  while (v < kMaxVariants && kVariantNames[precision == TCA_MIXED][cls][v] != nullptr) ++v;
  return v;
}

const char* reducer_name(int cls, int precision, int variant) {
  return kVariantNames[precision == TCA_MIXED][cls][variant];
}

int reducer_choice(int cls, int precision) { return g_choice[precision == TCA_MIXED][cls].load(); }

void set_reducer_choice(int cls, int precision, int variant) {
  g_choice[precision == TCA_MIXED][cls].store(variant);
}

template <typename F>
static hipError_t dispatch_reducer(int n, int precision, int variant, F&& f) {
  const int cls = reducer_class(n);
  if (cls < 0) return hipErrorInvalidValue;
  int v = variant >= 0 ? variant : reducer_choice(cls, precision);
  if (v >= reducer_variants(cls, precision)) v = 0;
  return dispatch_variant(cls, precision, v, f);
}

bool supported_n(int n) { return n >= 2 && n <= kMaxN; }

// Resident workgroups of a kernel on the current device (cached per kernel).
static int resident_grid(const void* kernel, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  cache[kernel] = cus * per_cu;
  return cus * per_cu;
}

static dim3 persistent(int items, int resident) {
  return dim3((unsigned)(items < resident ? (items > 0 ? items : 1) : resident));
}

hipError_t launch_cluster_block_reduce(int precision, int Lc, const double* S, BlockGeom g,
                                       ModelParams m, SweepRef sr, const int32_t* list,
                                       const int32_t* count, int max_clusters, ReduceOut out,
                                       hipStream_t st, int variant) {
  if (max_clusters <= 0) return hipSuccess;
  return dispatch_reducer(2 * Lc * Lc, precision, variant, [&](auto red, auto r) -> hipError_t {
    using Red = decltype(red);
    using R = decltype(r);
    hipLaunchKernelGGL((cluster_block_reduce<Red, R>), dim3(2 * max_clusters), dim3(Red::NT), 0,
                       st, S, g, Lc, m, sr, list, count, max_clusters, out);
    return hipGetLastError();
  });
}

hipError_t launch_cluster_sites_reduce(int precision, int Lc, const double* S, int L,
                                       ModelParams m, const int32_t* sites, const double* prop,
                                       int count, ReduceOut out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  return dispatch_reducer(2 * Lc * Lc, precision, -1, [&](auto red, auto r) -> hipError_t {
    using Red = decltype(red);
    using R = decltype(r);
    hipLaunchKernelGGL((cluster_sites_reduce<Red, R>), dim3(count), dim3(Red::NT), 0, st, S, L,
                       Lc, m, sites, prop, out);
    return hipGetLastError();
  });
}

hipError_t launch_heevals_reduce(int precision, int n, const double* A, int batch, ReduceOut out,
                                 hipStream_t st, int variant) {
  if (batch <= 0) return hipSuccess;
  return dispatch_reducer(n, precision, variant, [&](auto red, auto r) -> hipError_t {
    using Red = decltype(red);
    using R = decltype(r);
    hipLaunchKernelGGL((heevals_reduce<Red, R>), dim3(batch), dim3(Red::NT), 0, st, A, n, out);
    return hipGetLastError();
  });
}

template <int NTHR>
static hipError_t eig_launch(int nmats, ReduceOut in, SweepRef sr, double mu, double* F,
                             double* ev, int ev_ld, hipStream_t st, const int32_t* list,
                             const int32_t* count) {
  auto kern = tridiag_eig_kernel<NTHR>;
  hipLaunchKernelGGL(kern, persistent(nmats, resident_grid((const void*)kern, NTHR)), dim3(NTHR), 0, st,
                     in.D, in.E2, in.ld, in.nmat, nmats, sr, mu, F, ev, ev_ld, list, count);
  return hipGetLastError();
}

hipError_t launch_tridiag_eig(int nmax, int nmats, ReduceOut in, SweepRef sr, double mu,
                              double* F, double* ev, int ev_ld, hipStream_t st,
                              const int32_t* list, const int32_t* count) {
  if (nmats <= 0) return hipSuccess;
  if (nmax <= 64) return eig_launch<64>(nmats, in, sr, mu, F, ev, ev_ld, st, list, count);
  if (nmax <= 128) return eig_launch<128>(nmats, in, sr, mu, F, ev, ev_ld, st, list, count);
  if (nmax <= 256) return eig_launch<256>(nmats, in, sr, mu, F, ev, ev_ld, st, list, count);
  return hipErrorInvalidValue;
}

}  // namespace tca
