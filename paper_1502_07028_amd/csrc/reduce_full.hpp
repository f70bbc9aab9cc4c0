// Householder reduction of one dense complex Hermitian matrix per workgroup to
// real symmetric tridiagonal form, the full matrix held in registers.
//
// Layout: a TR x TC thread grid; thread (tr, tc) = (tid / TC, tid % TC) owns
// rows i = tr + TR*li (li < LR) and columns j = tc + TC*lj (lj < LC), both
// triangles stored.  The TC threads sharing a row group are consecutive lanes
// of one wavefront (TC divides 64), so the row sums of A*v are DPP exchanges
// inside the wavefront.  The current column, y = A*v and the reflector
// vectors pass through LDS; every wavefront keeps its own copy of v and w, so
// building them needs no workgroup barrier.
//
// Step k (trailing block B = A[k+1:, k+1:], column x = A[k+1:, k]):
//   reflector  beta = -sign(Re x_0) ||x||, tau = (beta - x_0)/beta,
//              v = (1, x_1.., / (x_0 - beta))   so that (I - tau v v^H)^H x = beta e_1
//   y = B v,   w = tau y - (|tau|^2/2) Re(v^H y) v,   B <- B - v w^H - w v^H
// The tridiagonal is d_k = Re A[k][k], e_k = beta (only e_k^2 is kept).
// Two workgroup barriers per step: after the column is written and after y.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cplx.hpp"

namespace tca {

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// DPP controls: lane pairings that are involutions inside a row of 16 lanes
constexpr int kDppRowMirror = 0x140;      // l <-> 15 - l
constexpr int kDppRowHalfMirror = 0x141;  // l <-> 7 - l   (within 8)
constexpr int kDppQuadReverse = 0x1B;     // l <-> 3 - l   (within 4)
constexpr int kDppQuadSwap1 = 0xB1;       // l <-> l ^ 1
constexpr int kDppQuadSwap2 = 0x4E;       // l <-> l ^ 2

// Sum over the TC consecutive lanes of a row group (TC in {4, 8, 16}); every
// lane of the group receives the same total.
template <int TC, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(TC == 4 || TC == 8 || TC == 16, "row group must be 4, 8 or 16 lanes");
  v += dpp_mov<kDppQuadSwap1>(v);
  v += dpp_mov<kDppQuadSwap2>(v);
  if constexpr (TC >= 8) v += dpp_mov<kDppRowHalfMirror>(v);
  if constexpr (TC >= 16) v += dpp_mov<kDppRowMirror>(v);
  return v;
}

// Sum over the 64 lanes of a wavefront, identical in every lane and every
// wavefront that holds the same data.
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
  v = group_sum<16>(v);
  return (readlane_t(v, 0) + readlane_t(v, 16)) + (readlane_t(v, 32) + readlane_t(v, 48));
}

// One reduce-scatter stage: each lane keeps one half of its NV values and adds
// the partner's copy of that half; `upper` selects the half kept.
template <int CTRL, int NV, typename T>
__device__ __forceinline__ void rs_stage(const T (&a)[NV], T (&b)[NV / 2], const bool upper) {
#pragma unroll
  for (int q = 0; q < NV / 2; ++q) {
    const T send = upper ? a[q] : a[q + NV / 2];
    const T keep = upper ? a[q + NV / 2] : a[q];
    b[q] = keep + dpp_mov<CTRL>(send);
  }
}

// Reduce-scatter of P values (P a power of two, P <= TC) over the TC lanes of
// a row group: lane l ends with the group total of value index
// `reduce_scatter_index<TC, P>(l)`; lanes that duplicate a value are told apart
// by `reduce_scatter_writer<TC, P>(l)`.
template <int TC, int P>
__device__ __forceinline__ int reduce_scatter_index(int l) {
  int q = 0, half = P / 2;
  int bit = TC / 2;
  for (; half >= 1; half /= 2, bit /= 2) q += (l & bit) ? half : 0;
  return q;
}
template <int TC, int P>
__device__ __forceinline__ bool reduce_scatter_writer(int l) {
  int bit = TC / 2;
  for (int half = P / 2; half >= 1; half /= 2) bit /= 2;  // skip the halving stages
  const int dup_mask = (bit > 0) ? (2 * bit - 1) : 0;      // remaining all-reduce bits
  return (l & dup_mask) == 0;
}

template <int TC, int P, typename T>
__device__ __forceinline__ T reduce_scatter(const T (&v)[P], const int l) {
  static_assert((P & (P - 1)) == 0 && P <= TC, "P must be a power of two <= TC");
  static_assert(TC == 8 || TC == 16, "row group of 8 or 16 lanes");
  T a16[16], a8[8], a4[4], a2[2], a1[1];
  T r;
  if constexpr (P == 16) {
#pragma unroll
    for (int q = 0; q < 16; ++q) a16[q] = v[q];
    rs_stage<kDppRowMirror>(a16, a8, (l & 8) != 0);
    rs_stage<kDppRowHalfMirror>(a8, a4, (l & 4) != 0);
    rs_stage<kDppQuadReverse>(a4, a2, (l & 2) != 0);
    rs_stage<kDppQuadSwap1>(a2, a1, (l & 1) != 0);
    r = a1[0];
  } else if constexpr (P == 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a8[q] = v[q];
    if constexpr (TC == 16) {
      rs_stage<kDppRowMirror>(a8, a4, (l & 8) != 0);
      rs_stage<kDppRowHalfMirror>(a4, a2, (l & 4) != 0);
      rs_stage<kDppQuadReverse>(a2, a1, (l & 2) != 0);
      r = a1[0];
      r += dpp_mov<kDppQuadSwap1>(r);
    } else {
      rs_stage<kDppRowHalfMirror>(a8, a4, (l & 4) != 0);
      rs_stage<kDppQuadReverse>(a4, a2, (l & 2) != 0);
      rs_stage<kDppQuadSwap1>(a2, a1, (l & 1) != 0);
      r = a1[0];
    }
  } else {
    static_assert(P == 8 || P == 16, "reduce-scatter width must be 8 or 16");
  }
  return r;
}

// The LDS writes of this wavefront become visible to its own later reads.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
struct pow2_ceil {
  static constexpr int value = N <= 1 ? 1 : 2 * pow2_ceil<(N + 1) / 2>::value;
};
template <>
struct pow2_ceil<1> {
  static constexpr int value = 1;
};

template <int TR, int TC, int LR, int LC, typename R>
struct ReduceFull {
  static constexpr int NT = TR * TC;
  static constexpr int NW = NT / 64;
  static constexpr int NPR = TR * LR;   // padded row extent
  static constexpr int NPC = TC * LC;   // padded column extent
  static constexpr int NP = NPR > NPC ? NPR : NPC;
  static constexpr int NLOC = LR * LC;
  typedef cx<R> Regs[NLOC];
  static constexpr int NV = 2 * LR;                       // row-sum values per lane
  static constexpr int PV = pow2_ceil<NV>::value < 8 ? 8 : pow2_ceil<NV>::value;
  // minimum wavefronts per SIMD to compile for (launch bounds): four when the
  // FP32 matrix leaves room for two workgroups per CU, else no constraint
  static constexpr int MINW = (sizeof(R) == 4 && NLOC <= 48) ? 4 : 1;
  static_assert(NT % 64 == 0 && 64 % TC == 0, "bad thread grid");
  static_assert(PV <= TC, "row group too narrow for the reduce-scatter");

  struct Smem {
    cx<R> x[2][NP];   // current column, double-buffered
    R yr[NP], yi[NP]; // y = B v
    cx<R> vb[NW][NP]; // per-wavefront v (zero outside the trailing range)
    cx<R> wb[NW][NP]; // per-wavefront w
    double d[NP];     // tridiagonal, staged here and written out at the end
    double e2[NP];
  };

  static __device__ __forceinline__ int idx(int li, int lj) { return li * LC + lj; }

  // Fill the registers from lower(i, j) (i >= j), mirroring the upper triangle.
  template <class F>
  static __device__ __forceinline__ void load(cx<R> (&A)[NLOC], const int n, F&& lower) {
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
#pragma unroll
    for (int li = 0; li < LR; ++li) {
#pragma unroll
      for (int lj = 0; lj < LC; ++lj) {
        const int i = tr + TR * li, j = tc + TC * lj;
        cx<R> v = {R(0), R(0)};
        if (i < n && j < n) {
          if (i >= j) {
            v = lower(i, j);
          } else {
            v = lower(j, i);
            v.im = -v.im;
          }
        }
        A[idx(li, lj)] = v;
      }
    }
  }

  // Column k (rows > k) of the register matrix -> xb; d[k] and, at k = n-2,
  // the last off-diagonal entry.
  static __device__ __forceinline__ void write_col(const int n, const int k, const cx<R> (&A)[NLOC],
                                                   cx<R>* xb, double* d, double* e2) {
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
    const int lj0 = k / TC;  // wavefront-uniform
#pragma unroll
    for (int lj = 0; lj < LC; ++lj) {
      if (lj != lj0) continue;
      if (tc == k % TC) {
#pragma unroll
        for (int li = 0; li < LR; ++li) {
          const int i = tr + TR * li;
          const cx<R> a = A[idx(li, lj)];
          if (i > k && i < n) xb[i] = a;
          if (i == k) d[k] = (double)a.re;
          if (k == n - 2 && i == n - 1)
            e2[k] = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
        }
      }
    }
  }

  static __device__ __forceinline__ void write_last_diag(const int n, const cx<R> (&A)[NLOC],
                                                         double* d) {
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
    const int k = n - 1;
    if (tc != k % TC || tr != k % TR) return;
#pragma unroll
    for (int li = 0; li < LR; ++li)
#pragma unroll
      for (int lj = 0; lj < LC; ++lj)
        if (tr + TR * li == k && tc + TC * lj == k) d[k] = (double)A[idx(li, lj)].re;
  }

  // Reduce A (registers) to (d, e2) in global memory.
  static __device__ __forceinline__ void run(const int n, cx<R> (&A)[NLOC], Smem& sm,
                                             double* __restrict__ dg, double* __restrict__ e2g) {
    const int tid = threadIdx.x, tr = tid / TC, tc = tid % TC, lane = tid & 63, wave = tid >> 6;
    const int lg = tid % TC;  // lane within the row group
    double* d = sm.d;
    double* e2 = sm.e2;
    cx<R>* vw = sm.vb[wave];
    cx<R>* ww = sm.wb[wave];
    if (n == 1) {
      if (tid == 0) dg[0] = (double)A[0].re;
      return;
    }
    write_col(n, 0, A, sm.x[0], d, e2);
    if (n == 2) write_last_diag(n, A, d);
    __syncthreads();
    const int q_rs = reduce_scatter_index<TC, PV>(lg);
    const bool w_rs = reduce_scatter_writer<TC, PV>(lg);
    int buf = 0;
    for (int k = 0; k < n - 2; ++k) {
      const cx<R>* xk = sm.x[buf];
      // ---- reflector (identical in every wavefront)
      R s2 = R(0);
      for (int i = k + 2 + lane; i < n; i += 64) {
        const cx<R> v = xk[i];
        s2 += v.re * v.re + v.im * v.im;
      }
      s2 = wave_total(s2);
      const cx<R> al = xk[k + 1];
      R beta, tre, tim, scr, sci;
      if (s2 == R(0) && al.im == R(0)) {
        beta = al.re;
        tre = tim = scr = sci = R(0);
      } else {
        const R nrm = sqrt(al.re * al.re + al.im * al.im + s2);
        beta = al.re >= R(0) ? -nrm : nrm;
        const R rb = R(1) / beta;
        tre = (beta - al.re) * rb;
        tim = -al.im * rb;
        const R dr = al.re - beta, di = al.im;
        const R rden = R(1) / (dr * dr + di * di);
        scr = dr * rden;
        sci = -di * rden;
      }
      if (tid == 0) e2[k] = (double)beta * (double)beta;
      // ---- this wavefront's copy of v (zeros outside k+1 .. n-1)
      for (int i = lane; i < NP; i += 64) {
        cx<R> v = {R(0), R(0)};
        if (i == k + 1) {
          v.re = R(1);
        } else if (i > k + 1 && i < n) {
          const cx<R> x = xk[i];
          v = {x.re * scr - x.im * sci, x.re * sci + x.im * scr};
        }
        vw[i] = v;
      }
      wave_lds_fence();
      const int kr = (k + 1) / TR, kc = (k + 1) / TC;  // first local blocks touching the trailing part
      // ---- y = B v: per-lane row partials, then a reduce-scatter over the row group
      cx<R> vc[LC];
#pragma unroll
      for (int lj = 0; lj < LC; ++lj) vc[lj] = (lj >= kc) ? vw[tc + TC * lj] : cx<R>{R(0), R(0)};
      R part[PV];
#pragma unroll
      for (int q = 0; q < PV; ++q) part[q] = R(0);
#pragma unroll
      for (int lj = 0; lj < LC; ++lj) {
        if (lj < kc) continue;
        const cx<R> v = vc[lj];
#pragma unroll
        for (int li = 0; li < LR; ++li) {
          if (li < kr) continue;
          const cx<R> a = A[idx(li, lj)];
          part[2 * li] += a.re * v.re - a.im * v.im;
          part[2 * li + 1] += a.re * v.im + a.im * v.re;
        }
      }
      const R ysum = reduce_scatter<TC, PV>(part, lg);
      {
        const int li = q_rs >> 1;
        const int i = tr + TR * li;
        if (w_rs && q_rs < NV && li >= kr && i > k && i < n) {
          if (q_rs & 1)
            sm.yi[i] = ysum;
          else
            sm.yr[i] = ysum;
        }
      }
      __syncthreads();
      // ---- c = Re(v^H y), then this wavefront's copy of w = tau y - (|tau|^2/2) c v
      R c = R(0);
      for (int i = k + 1 + lane; i < n; i += 64) {
        const cx<R> v = vw[i];
        c += v.re * sm.yr[i] + v.im * sm.yi[i];
      }
      c = wave_total(c);
      const R a2 = R(0.5) * (tre * tre + tim * tim) * c;
      for (int i = lane; i < NP; i += 64) {
        cx<R> w = {R(0), R(0)};
        if (i > k && i < n) {
          const cx<R> v = vw[i];
          const R yr = sm.yr[i], yi = sm.yi[i];
          w = {tre * yr - tim * yi - a2 * v.re, tre * yi + tim * yr - a2 * v.im};
        }
        ww[i] = w;
      }
      wave_lds_fence();
      // ---- B <- B - v w^H - w v^H
      cx<R> wc[LC];
#pragma unroll
      for (int lj = 0; lj < LC; ++lj) wc[lj] = (lj >= kc) ? ww[tc + TC * lj] : cx<R>{R(0), R(0)};
      cx<R> vr[LR], wr[LR];
#pragma unroll
      for (int li = 0; li < LR; ++li) {
        const int i = tr + TR * li;
        vr[li] = (li >= kr) ? vw[i] : cx<R>{R(0), R(0)};
        wr[li] = (li >= kr) ? ww[i] : cx<R>{R(0), R(0)};
      }
#pragma unroll
      for (int li = 0; li < LR; ++li) {
        if (li < kr) continue;
        const cx<R> vi = vr[li], wi = wr[li];
#pragma unroll
        for (int lj = 0; lj < LC; ++lj) {
          if (lj < kc) continue;
          cx<R>& a = A[idx(li, lj)];
          a.re -= vi.re * wc[lj].re + vi.im * wc[lj].im + wi.re * vc[lj].re + wi.im * vc[lj].im;
          a.im -= vi.im * wc[lj].re - vi.re * wc[lj].im + wi.im * vc[lj].re - wi.re * vc[lj].im;
        }
      }
      write_col(n, k + 1, A, sm.x[buf ^ 1], d, e2);
      if (k + 1 == n - 2) write_last_diag(n, A, d);
      buf ^= 1;
      __syncthreads();
    }
    if (n == 2) __syncthreads();
    for (int i = tid; i < n; i += NT) {
      dg[i] = d[i];
      if (i < n - 1) e2g[i] = e2[i];
    }
  }
};

}  // namespace tca
