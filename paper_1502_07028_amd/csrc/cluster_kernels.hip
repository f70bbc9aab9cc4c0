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

#include <type_traits>

#include "internal.hpp"
#include "reduce_full.hpp"
#include "reduce_lower.hpp"
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
  cx<R> A[Red::NLOC];
  Red::load(A, n, [&](int i, int j) { return h_elem<R>(i, j, Lc, m.t, m.JH, sp); });
  Red::run(n, A, sm, d, e2);
}

template <class Red, typename R>
__global__ __launch_bounds__(Red::NT, Red::MINW) void cluster_block_reduce(
    const double* __restrict__ S, BlockGeom g, int Lc, ModelParams m, uint64_t sweep,
    const int32_t* __restrict__ list, const int32_t* __restrict__ count, ReduceOut out) {
  __shared__ typename Red::Smem sm;
  __shared__ double sp[3 * kMaxLc * kMaxLc];
  const int ci = blockIdx.x >> 1, which = blockIdx.x & 1;
  int c = ci;
  if (list != nullptr) {
    if (ci >= *count) return;
    c = list[ci];
  }
  const int px = g.x0 + c % g.h, py = g.y0 + c / g.h;
  const int site = px + g.L * py;
  gather_spins(S, g.L, px, py, Lc, sp);
  __syncthreads();
  if (which == 1 && threadIdx.x == 0) sphere_point(m.seed, sweep, site, kStreamProposal, sp);
  __syncthreads();
  const int mat = 2 * c + which;
  solve_cluster<Red, R>(sp, Lc, m, sm, out.D + (size_t)mat * out.ld, out.E2 + (size_t)mat * out.ld);
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
__global__ __launch_bounds__(Red::NT, Red::MINW) void heevals_reduce(const double* __restrict__ Ag, int n,
                                                          ReduceOut out) {
  __shared__ typename Red::Smem sm;
  const int b = blockIdx.x;
  const double* M = Ag + (size_t)b * n * n * 2;
  cx<R> A[Red::NLOC];
  Red::load(A, n, [&](int i, int j) -> cx<R> {
    const size_t o = 2 * ((size_t)i * n + j);
    return {(R)M[o], i == j ? R(0) : (R)M[o + 1]};
  });
  Red::run(n, A, sm, out.D + (size_t)b * out.ld, out.E2 + (size_t)b * out.ld);
  if (threadIdx.x == 0) out.nmat[b] = n;
}

// One workgroup per tridiagonal: thread j finds eigenvalue j; then the grand
// potential is reduced in a fixed order.  Every lane of a wavefront walks the
// same (d, e2) with the same index, so the Sturm loops read them through the
// scalar cache straight from global memory (read-only in this kernel) and use
// them as scalar operands.
template <int NTHR>
__global__ __launch_bounds__(NTHR) void tridiag_eig_kernel(const double* __restrict__ D,
                                                           const double* __restrict__ E2, int ld,
                                                           const int32_t* __restrict__ nmat,
                                                           double T, double mu,
                                                           double* __restrict__ F,
                                                           double* __restrict__ ev, int ev_ld,
                                                           const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ count) {
  __shared__ double red[NTHR / 64];
  const int tid = threadIdx.x;
  int mat = blockIdx.x;
  if (list != nullptr) {
    if ((int)(blockIdx.x >> 1) >= *count) return;
    mat = 2 * list[blockIdx.x >> 1] + (blockIdx.x & 1);
  }
  const int n = nmat[mat];
  const double* d = D + (size_t)mat * ld;
  const double* e2 = E2 + (size_t)mat * ld;
  const TriBounds B = tri_bounds(n, d, e2);
  double acc = 0.0;
  for (int j = tid; j < n; j += NTHR) {
    const double lam = tri_eigenvalue(n, j, d, e2, B);
    if (ev != nullptr) ev[(size_t)mat * ev_ld + j] = lam;
    if (F != nullptr) acc += omega_term(lam, T, mu);
  }
  if (F == nullptr) return;
  acc = wave_total(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < NTHR / 64; ++w) s += red[w];
    F[mat] = s;
  }
}

// -------------------------------------------------------------------------
// Reducer per (dimension, precision).  Full storage on a TR x TC grid where
// the whole matrix fits the register file; lower-triangle storage above
// dimension 128 in FP64.
template <typename F>
static hipError_t dispatch_reducer(int n, int precision, F&& f) {
  if (precision == TCA_MIXED) {
    using R = float;
    if (n <= 32) return f(ReduceFull<8, 8, 4, 4, R>{}, R{});
    if (n <= 64) return f(ReduceFull<16, 16, 4, 4, R>{}, R{});
    if (n <= 80) return f(ReduceFull<16, 16, 5, 5, R>{}, R{});
    if (n <= 128) return f(ReduceFull<32, 16, 4, 8, R>{}, R{});
    if (n <= 176) return f(ReduceFull<32, 16, 6, 11, R>{}, R{});
    if (n <= 208) return f(ReduceFull<32, 16, 7, 13, R>{}, R{});
  } else {
    using R = double;
    if (n <= 32) return f(ReduceFull<8, 8, 4, 4, R>{}, R{});
    if (n <= 64) return f(ReduceFull<16, 16, 4, 4, R>{}, R{});
    if (n <= 80) return f(ReduceFull<16, 16, 5, 5, R>{}, R{});
    if (n <= 128) return f(ReduceFull<32, 16, 4, 8, R>{}, R{});
    if (n <= 176) return f(ReduceLower<16, 11, R>{}, R{});
    if (n <= 208) return f(ReduceLower<16, 13, R>{}, R{});
  }
  return hipErrorInvalidValue;
}

bool supported_n(int n) { return n >= 2 && n <= kMaxN; }

hipError_t launch_cluster_block_reduce(int precision, int Lc, const double* S, BlockGeom g,
                                       ModelParams m, uint64_t sweep, const int32_t* list,
                                       const int32_t* count, int max_clusters, ReduceOut out,
                                       hipStream_t st) {
  return dispatch_reducer(2 * Lc * Lc, precision, [&](auto red, auto r) -> hipError_t {
    using Red = decltype(red);
    using R = decltype(r);
    hipLaunchKernelGGL((cluster_block_reduce<Red, R>), dim3(2 * max_clusters), dim3(Red::NT), 0,
                       st, S, g, Lc, m, sweep, list, count, out);
    return hipGetLastError();
  });
}

hipError_t launch_cluster_sites_reduce(int precision, int Lc, const double* S, int L,
                                       ModelParams m, const int32_t* sites, const double* prop,
                                       int count, ReduceOut out, hipStream_t st) {
  return dispatch_reducer(2 * Lc * Lc, precision, [&](auto red, auto r) -> hipError_t {
    using Red = decltype(red);
    using R = decltype(r);
    hipLaunchKernelGGL((cluster_sites_reduce<Red, R>), dim3(count), dim3(Red::NT), 0, st, S, L, Lc,
                       m, sites, prop, out);
    return hipGetLastError();
  });
}

hipError_t launch_heevals_reduce(int precision, int n, const double* A, int batch, ReduceOut out,
                                 hipStream_t st) {
  return dispatch_reducer(n, precision, [&](auto red, auto r) -> hipError_t {
    using Red = decltype(red);
    using R = decltype(r);
    hipLaunchKernelGGL((heevals_reduce<Red, R>), dim3(batch), dim3(Red::NT), 0, st, A, n, out);
    return hipGetLastError();
  });
}

hipError_t launch_tridiag_eig(int nmax, int nmats, ReduceOut in, double T, double mu, double* F,
                              double* ev, int ev_ld, hipStream_t st, const int32_t* list,
                              const int32_t* count) {
  if (nmats <= 0) return hipSuccess;
  if (nmax <= 64)
    hipLaunchKernelGGL(tridiag_eig_kernel<64>, dim3(nmats), dim3(64), 0, st, in.D, in.E2, in.ld,
                       in.nmat, T, mu, F, ev, ev_ld, list, count);
  else if (nmax <= 128)
    hipLaunchKernelGGL(tridiag_eig_kernel<128>, dim3(nmats), dim3(128), 0, st, in.D, in.E2, in.ld,
                       in.nmat, T, mu, F, ev, ev_ld, list, count);
  else if (nmax <= 256)
    hipLaunchKernelGGL(tridiag_eig_kernel<256>, dim3(nmats), dim3(256), 0, st, in.D, in.E2, in.ld,
                       in.nmat, T, mu, F, ev, ev_ld, list, count);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tca
