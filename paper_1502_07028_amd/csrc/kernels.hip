// Kernels of the traveling-cluster Monte Carlo sweep on gfx950.
//
//  cluster_block_kernel  one workgroup per (cluster, old|new) of a parallel
//                        block (Sec. III(a)): gather the cluster spins, build the
//                        cluster Hamiltonian in registers, tridiagonalize, find
//                        all eigenvalues, sum the grand potential -> F.
//  decide_kernel         Metropolis decisions of the block in an order
//                        equivalent to the sequential sweep (Sec. II(c) step
//                        (e)-(f)), committing accepted spins.
//  cluster_eig_kernel    eigenvalues of chosen clusters (same solver).
//  heevals_kernel        eigenvalues of raw Hermitian matrices (same solver).
//  init / S(q) kernels   initial state and the structure factor of Eq. (2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "rng.hpp"
#include "solver.hpp"

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

template <int G, int LR, typename R>
__device__ __forceinline__ void build_cluster(cx<R> (&A)[LR * (LR + 1) / 2], int n, int Lc,
                                              double t, double JH, const double* sp) {
  const int tr = threadIdx.x / G, tc = threadIdx.x % G;
#pragma unroll
  for (int li = 0; li < LR; ++li) {
#pragma unroll
    for (int lj = 0; lj <= li; ++lj) {
      const int i = tr + G * li, j = tc + G * lj;
      cx<R> v = {R(0), R(0)};
      if (i < n && (li > lj || tr >= tc)) v = h_elem<R>(i, j, Lc, t, JH, sp);
      A[Solver<G, LR, R>::idx(li, lj)] = v;
    }
  }
}

// Cluster spins (cluster order) into LDS; the corner optionally replaced.
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

template <int G, int LR, typename R>
__global__ __launch_bounds__(G* G) void cluster_block_kernel(
    const double* __restrict__ S, BlockGeom g, int Lc, ModelParams m, uint64_t sweep, double T,
    const int32_t* __restrict__ list, const int32_t* __restrict__ count, double* __restrict__ Fpair) {
  using Sv = Solver<G, LR, R>;
  __shared__ typename Sv::Smem sm;
  __shared__ double sp[3 * kMaxLc * kMaxLc];
  const int ci = blockIdx.x >> 1, which = blockIdx.x & 1;
  int c = ci;
  if (list != nullptr) {
    if (ci >= *count) return;
    c = list[ci];
  }
  const int px = g.x0 + c % g.h, py = g.y0 + c / g.h;
  const int site = px + g.L * py;
  const int n = 2 * Lc * Lc;
  gather_spins(S, g.L, px, py, Lc, sp);
  __syncthreads();
  if (which == 1 && threadIdx.x == 0) sphere_point(m.seed, sweep, site, kStreamProposal, sp);
  __syncthreads();
  cx<R> A[Sv::NLOC];
  build_cluster<G, LR, R>(A, n, Lc, m.t, m.JH, sp);
  Sv::tridiagonalize(n, A, sm);
  Sv::eigenvalues(n, sm);
  const double F = Sv::free_energy(n, T, m.mu, sm);
  if (threadIdx.x == 0) Fpair[2 * c + which] = F;
}

template <int G, int LR, typename R>
__global__ __launch_bounds__(G* G) void cluster_eig_kernel(const double* __restrict__ S, int L,
                                                           int Lc, ModelParams m,
                                                           const int32_t* __restrict__ sites,
                                                           const double* __restrict__ prop,
                                                           double* __restrict__ ev, int ld) {
  using Sv = Solver<G, LR, R>;
  __shared__ typename Sv::Smem sm;
  __shared__ double sp[3 * kMaxLc * kMaxLc];
  const int w = blockIdx.x;
  const int site = sites[w];
  const int px = site % L, py = site / L;
  const int n = 2 * Lc * Lc;
  gather_spins(S, L, px, py, Lc, sp);
  __syncthreads();
  if (prop != nullptr && threadIdx.x < 3) sp[threadIdx.x] = prop[3 * w + threadIdx.x];
  __syncthreads();
  cx<R> A[Sv::NLOC];
  build_cluster<G, LR, R>(A, n, Lc, m.t, m.JH, sp);
  Sv::tridiagonalize(n, A, sm);
  Sv::eigenvalues(n, sm);
  for (int j = threadIdx.x; j < n; j += blockDim.x) ev[(size_t)w * ld + j] = sm.ev[j];
}

template <int G, int LR, typename R>
__global__ __launch_bounds__(G* G) void heevals_kernel(const double* __restrict__ Ag, int n,
                                                       double T, double mu,
                                                       double* __restrict__ w,
                                                       double* __restrict__ F) {
  using Sv = Solver<G, LR, R>;
  __shared__ typename Sv::Smem sm;
  const int b = blockIdx.x;
  const int tr = threadIdx.x / G, tc = threadIdx.x % G;
  const double* M = Ag + (size_t)b * n * n * 2;
  cx<R> A[Sv::NLOC];
#pragma unroll
  for (int li = 0; li < LR; ++li) {
#pragma unroll
    for (int lj = 0; lj <= li; ++lj) {
      const int i = tr + G * li, j = tc + G * lj;
      cx<R> v = {R(0), R(0)};
      if (i < n && (li > lj || tr >= tc)) {
        const size_t o = 2 * ((size_t)i * n + j);
        v.re = (R)M[o];
        v.im = (i == j) ? R(0) : (R)M[o + 1];
      }
      A[Sv::idx(li, lj)] = v;
    }
  }
  Sv::tridiagonalize(n, A, sm);
  Sv::eigenvalues(n, sm);
  if (w != nullptr)
    for (int j = threadIdx.x; j < n; j += blockDim.x) w[(size_t)b * n + j] = sm.ev[j];
  if (F != nullptr) {
    const double f = Sv::free_energy(n, T, mu, sm);
    if (threadIdx.x == 0) F[b] = f;
  }
}

// -------------------------------------------------------------------------
// Change of the classical superexchange energy, evaluated one rounded
// operation at a time: neighbour sum (-x, +x, -y, +y), difference, dot.
__device__ __attribute__((noinline)) double classical_delta(const double* S, int L,
                                                            int px, int py, const double* sn,
                                                            double JAF) {
#pragma clang fp contract(off)
  const int xm = (px + L - 1) % L, xp = (px + 1) % L, ym = (py + L - 1) % L, yp = (py + 1) % L;
  const double* a = S + 3 * (xm + L * py);
  const double* b = S + 3 * (xp + L * py);
  const double* c = S + 3 * (px + L * ym);
  const double* d = S + 3 * (px + L * yp);
  const double* s = S + 3 * (px + L * py);
  double acc[3], df[3];
  for (int k = 0; k < 3; ++k) {
    acc[k] = ((a[k] + b[k]) + c[k]) + d[k];
    df[k] = sn[k] - s[k];
  }
  double dot = df[0] * acc[0];
  dot = dot + df[1] * acc[1];
  dot = dot + df[2] * acc[2];
  return JAF * dot;
}

// Metropolis decisions of block K.  Each cluster's dF came from the
// block-start state, which equals the state the sequential sweep would have
// shown it (no cluster of a block contains a site visited earlier in that
// block).  The classical term reads the -x and -y lattice neighbours, which
// may belong to the same block and be decided earlier in raster order, so with
// J_AF != 0 the sites are processed by anti-diagonals i + j = const of the
// block: every site is decided after both of those neighbours, exactly as in
// the sequential order.  With J_AF == 0 all decisions are independent.
__global__ __launch_bounds__(1024) void decide_kernel(double* S,
                                                      const double* __restrict__ Fpair,
                                                      BlockGeom g, ModelParams m, uint64_t sweep,
                                                      double T, int Lc_fixed, int4 classes,
                                                      int n_classes, int K,
                                                      tca_update_record* __restrict__ logbuf,
                                                      unsigned long long* __restrict__ counters) {
  const int h = g.h, L = g.L;
  const bool wave = (m.JAF != 0.0);
  const int ndiag = wave ? 2 * h - 1 : 1;
  unsigned long long nacc = 0, nnear = 0;
  for (int dd = 0; dd < ndiag; ++dd) {
    const int lo = wave ? max(0, dd - (h - 1)) : 0;
    const int cnt = wave ? (min(dd, h - 1) - lo + 1) : h * h;
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
      int i, j;
      if (wave) {
        i = lo + q;
        j = dd - i;
      } else {
        i = q % h;
        j = q / h;
      }
      const int c = i + h * j;
      const int px = g.x0 + i, py = g.y0 + j, site = px + L * py;
      double sn[3];
      sphere_point(m.seed, sweep, site, kStreamProposal, sn);
      const double dF = Fpair[2 * c + 1] - Fpair[2 * c];
      const double dE = dF + classical_delta(S, L, px, py, sn, m.JAF);
      const U64x4 r = philox4x64_10(m.seed, 0, sweep, site, kStreamMetropolis, 0);
      const double u = u53(r.w0);
      const bool acc = (dE <= 0.0) || (u < exp(-dE / T));
      bool near = false;
      if (u > 0.0) near = fabs(dE + T * log(u)) <= 1e-9 * fmax(fabs(dE), 1e-3);
      if (acc) {
        S[3 * site + 0] = sn[0];
        S[3 * site + 1] = sn[1];
        S[3 * site + 2] = sn[2];
      }
      nacc += acc;
      nnear += near;
      if (logbuf != nullptr) {
        int Lc = Lc_fixed;
        if (n_classes > 0) {
          const int k = size_class(m.seed, sweep, site, n_classes);
          Lc = k == 0 ? classes.x : k == 1 ? classes.y : k == 2 ? classes.z : classes.w;
        }
        tca_update_record rec;
        rec.site = site;
        rec.Lc = (int16_t)Lc;
        rec.accept = acc ? 1 : 0;
        rec.flags = near ? 1 : 0;
        rec.dF = dF;
        rec.dE = dE;
        rec.u = u;
        logbuf[(size_t)K * h * h + c] = rec;
      }
    }
    if (wave) __syncthreads();
  }
  if (nacc) atomicAdd(&counters[0], nacc);
  if (nnear) atomicAdd(&counters[1], nnear);
  if (threadIdx.x == 0) atomicAdd(&counters[2], (unsigned long long)(h * h));
}

__global__ void classify_kernel(int4 classes, int n_classes, BlockGeom g, uint64_t seed,
                                uint64_t sweep, int32_t* __restrict__ count,
                                int32_t* __restrict__ list) {
  const int hh = g.h * g.h;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= hh) return;
  const int site = (g.x0 + c % g.h) + g.L * (g.y0 + c / g.h);
  const int k = size_class(seed, sweep, site, n_classes);
  const int pos = atomicAdd(&count[k], 1);
  list[k * hh + pos] = c;
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void init_spins_kernel(double* S, int L, int kind, uint64_t seed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L * L) return;
  double s[3] = {0.0, 0.0, 1.0};
  if (kind == TCA_INIT_RANDOM) {
    sphere_point(seed, kInitSweep, (uint64_t)p, kStreamInit, s);
  } else if (kind == TCA_INIT_NEEL) {
    const int x = p % L, y = p / L;
    s[2] = ((x + y) & 1) ? -1.0 : 1.0;
  }
  S[3 * p + 0] = s[0];
  S[3 * p + 1] = s[1];
  S[3 * p + 2] = s[2];
}

// S(q) by a separable DFT: rows first (x -> qx), then columns (y -> qy).
__global__ void sq_rows_kernel(const double* __restrict__ S, int L, double* __restrict__ W) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;  // o = qx + L*y
  if (o >= L * L) return;
  const int qx = o % L, y = o / L;
  double re[3] = {0, 0, 0}, im[3] = {0, 0, 0};
  for (int x = 0; x < L; ++x) {
    const int ph = (int)(((long long)qx * x) % L);
    double sn, cs;
    sincospi(2.0 * ph / L, &sn, &cs);
    const double* s = S + 3 * (x + L * y);
    for (int a = 0; a < 3; ++a) {
      re[a] += s[a] * cs;
      im[a] -= s[a] * sn;
    }
  }
  for (int a = 0; a < 3; ++a) {
    W[6 * o + 2 * a] = re[a];
    W[6 * o + 2 * a + 1] = im[a];
  }
}

__global__ void sq_cols_kernel(const double* __restrict__ W, int L, double* __restrict__ Sq) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;  // o = qx + L*qy
  if (o >= L * L) return;
  const int qx = o % L, qy = o / L;
  double tot = 0.0;
  for (int a = 0; a < 3; ++a) {
    double re = 0.0, im = 0.0;
    for (int y = 0; y < L; ++y) {
      const int ph = (int)(((long long)qy * y) % L);
      double sn, cs;
      sincospi(2.0 * ph / L, &sn, &cs);
      const double wr = W[6 * (qx + L * y) + 2 * a], wi = W[6 * (qx + L * y) + 2 * a + 1];
      re += wr * cs + wi * sn;
      im += wi * cs - wr * sn;
    }
    tot += re * re + im * im;
  }
  const double N = (double)L * L;
  Sq[o] = tot / (N * N);
}

// -------------------------------------------------------------------------
// Compile-time (G, LR) for a matrix dimension n.
template <typename F>
static hipError_t dispatch_n(int n, F&& f) {
  using std::integral_constant;
  if (n <= 32) return f(integral_constant<int, 8>{}, integral_constant<int, 4>{});
  if (n <= 64) return f(integral_constant<int, 16>{}, integral_constant<int, 4>{});
  if (n <= 80) return f(integral_constant<int, 16>{}, integral_constant<int, 5>{});
  if (n <= 112) return f(integral_constant<int, 16>{}, integral_constant<int, 7>{});
  if (n <= 128) return f(integral_constant<int, 16>{}, integral_constant<int, 8>{});
  if (n <= 176) return f(integral_constant<int, 16>{}, integral_constant<int, 11>{});
  if (n <= 208) return f(integral_constant<int, 16>{}, integral_constant<int, 13>{});
  return hipErrorInvalidValue;
}

bool supported_n(int n) { return n >= 2 && n <= kMaxN; }

hipError_t launch_cluster_block(int precision, int Lc, const double* S, BlockGeom g,
                                ModelParams m, uint64_t sweep, double T, const int32_t* list,
                                const int32_t* count, int max_clusters, double* Fpair,
                                hipStream_t st) {
  const int n = 2 * Lc * Lc;
  return dispatch_n(n, [&](auto Gc, auto LRc) -> hipError_t {
    constexpr int G = decltype(Gc)::value, LR = decltype(LRc)::value;
    const dim3 grid(2 * max_clusters), block(G * G);
    if (precision == TCA_MIXED)
      hipLaunchKernelGGL((cluster_block_kernel<G, LR, float>), grid, block, 0, st, S, g, Lc, m,
                         sweep, T, list, count, Fpair);
    else
      hipLaunchKernelGGL((cluster_block_kernel<G, LR, double>), grid, block, 0, st, S, g, Lc, m,
                         sweep, T, list, count, Fpair);
    return hipGetLastError();
  });
}

hipError_t launch_cluster_eig(int precision, int Lc, const double* S, int L, ModelParams m,
                              const int32_t* sites, const double* prop, int count, double* ev,
                              int ld, hipStream_t st) {
  const int n = 2 * Lc * Lc;
  return dispatch_n(n, [&](auto Gc, auto LRc) -> hipError_t {
    constexpr int G = decltype(Gc)::value, LR = decltype(LRc)::value;
    if (precision == TCA_MIXED)
      hipLaunchKernelGGL((cluster_eig_kernel<G, LR, float>), dim3(count), dim3(G * G), 0, st, S,
                         L, Lc, m, sites, prop, ev, ld);
    else
      hipLaunchKernelGGL((cluster_eig_kernel<G, LR, double>), dim3(count), dim3(G * G), 0, st, S,
                         L, Lc, m, sites, prop, ev, ld);
    return hipGetLastError();
  });
}

hipError_t launch_heevals(int precision, int n, const double* A, int batch, double T, double mu,
                          double* w, double* F, hipStream_t st) {
  return dispatch_n(n, [&](auto Gc, auto LRc) -> hipError_t {
    constexpr int G = decltype(Gc)::value, LR = decltype(LRc)::value;
    if (precision == TCA_MIXED)
      hipLaunchKernelGGL((heevals_kernel<G, LR, float>), dim3(batch), dim3(G * G), 0, st, A, n, T,
                         mu, w, F);
    else
      hipLaunchKernelGGL((heevals_kernel<G, LR, double>), dim3(batch), dim3(G * G), 0, st, A, n,
                         T, mu, w, F);
    return hipGetLastError();
  });
}

static int4 pack_classes(const int32_t* c, int n) {
  int4 r = make_int4(0, 0, 0, 0);
  if (n > 0) r.x = c[0];
  if (n > 1) r.y = c[1];
  if (n > 2) r.z = c[2];
  if (n > 3) r.w = c[3];
  return r;
}

hipError_t launch_classify(const int32_t* classes_Lc, int n_classes, BlockGeom g, uint64_t seed,
                           uint64_t sweep, ClassLists cl, hipStream_t st) {
  const int hh = g.h * g.h;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, cl.count, 4);
  hipLaunchKernelGGL(classify_kernel, dim3((hh + 255) / 256), dim3(256), 0, st,
                     pack_classes(classes_Lc, n_classes), n_classes, g, seed, sweep, cl.count,
                     cl.list);
  return hipGetLastError();
}

hipError_t launch_decide(double* S, const double* Fpair, BlockGeom g, ModelParams m,
                         uint64_t sweep, double T, int Lc_fixed, const int32_t* classes_Lc,
                         int n_classes, int K, tca_update_record* log_dev,
                         unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(1024), 0, st, S, Fpair, g, m, sweep, T,
                     Lc_fixed, pack_classes(classes_Lc, n_classes), n_classes, K, log_dev,
                     counters);
  return hipGetLastError();
}

hipError_t launch_init_spins(double* S, int L, int kind, uint64_t seed, hipStream_t st) {
  const int N = L * L;
  hipLaunchKernelGGL(init_spins_kernel, dim3((N + 255) / 256), dim3(256), 0, st, S, L, kind, seed);
  return hipGetLastError();
}

hipError_t launch_sq(const double* S, int L, double* work, double* Sq, hipStream_t st) {
  const int N = L * L;
  hipLaunchKernelGGL(sq_rows_kernel, dim3((N + 255) / 256), dim3(256), 0, st, S, L, work);
  hipLaunchKernelGGL(sq_cols_kernel, dim3((N + 255) / 256), dim3(256), 0, st, work, L, Sq);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace tca
