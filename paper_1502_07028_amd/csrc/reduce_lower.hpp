// Householder reduction of one dense complex Hermitian matrix per workgroup to
// real symmetric tridiagonal form, storing only the lower triangle in
// registers.  Used where the full matrix does not fit the register file
// (FP64 matrices above dimension 128); the full-storage reducer is preferred
// elsewhere because it needs no column partial sums.
//
// Data layout.  Element (i, j) of the n x n matrix lives in thread
// (tr, tc) = (i mod G, j mod G), local block (li, lj) = (i / G, j / G); only the
// lower triangle is stored (li >= lj, and inside a diagonal local block only
// tr >= tc carries data, the rest stays zero).  y = A v is assembled from row
// partials (lower part) and column partials (upper part, via conj(A_ji)) that
// are summed through LDS.  The step algebra is that of reduce_full.hpp.  The
// product takes the row partials and the column partials in two passes over
// the stored blocks, and the rank-2 update walks them column block by column
// block, all reading the entries of v and w from LDS, so that beside the
// matrix only one accumulator lives in registers (the matrix takes most of the
// register file at n = 200 in FP64).
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "cplx.hpp"
#include "reduce_split.hpp"  // wave_total_rows, rsqrt_nr, fast_rcp

namespace tca {

template <int G, int LR, typename R>
struct ReduceLower {
  static constexpr int NT = G * G;            // threads per workgroup
  static constexpr int NW = NT / 64;          // wavefronts per workgroup
  static constexpr int NP = G * LR;           // padded dimension
  static constexpr int NLOC = LR * (LR + 1) / 2;
  typedef cx<R> Regs[NLOC];
  static constexpr int PITCH = NP + 1;        // LDS row pitch of partial sums
  static_assert(NT % 64 == 0, "workgroup must be whole wavefronts");

  static constexpr int MINW = 1;  // minimum wavefronts per SIMD (launch bounds)
  // copies of v and w in LDS: one per wavefront (no barrier after writing
  // them) up to four wavefronts, else one shared copy behind a barrier
  static constexpr int NVC = NW <= 4 ? NW : 1;

  struct Smem {
    double d[NP];
    double e2[NP];
    cx<R> x[2][NP];      // current column (double-buffered)
    cx<R> y[NP];         // B v
    cx<R> pr[G * PITCH]; // row partials   [tc][i]
    cx<R> pc[G * PITCH]; // column partials [tr][j]
    cx<R> vw[NVC][NP];   // v of the step (one copy per wavefront when they fit)
    cx<R> ww[NVC][NP];   // w of the step
  };

  static __device__ __forceinline__ constexpr int idx(int li, int lj) { return li * (li + 1) / 2 + lj; }

  // Fill the registers from lower(i, j) (i >= j).
  template <class F>
  static __device__ __forceinline__ void load(cx<R> (&A)[NLOC], const int n, F&& lower) {
    const int tr = threadIdx.x / G, tc = threadIdx.x % G;
#pragma unroll
    for (int li = 0; li < LR; ++li) {
#pragma unroll
      for (int lj = 0; lj <= li; ++lj) {
        const int i = tr + G * li, j = tc + G * lj;
        cx<R> v = {R(0), R(0)};
        if (i < n && (li > lj || tr >= tc)) v = lower(i, j);
        A[idx(li, lj)] = v;
      }
    }
  }

  // Copy column k (rows k+1..n-1) of the register matrix to LDS; also write
  // the diagonal entry d[k] and, at the last column, the final 2x2 entries.
  // The column block is tested once per block (a uniform branch) and the
  // lanes of column k once inside it, instead of once per register entry.
  static __device__ __forceinline__ void write_col(int n, int k, const cx<R> (&A)[NLOC],
                                                   cx<R>* xb, double* d, double* e2) {
    const int tid = threadIdx.x, tr = tid / G, tc = tid % G;
    const int kb = k / G, kc = k % G;
#pragma unroll
    for (int lj = 0; lj < LR; ++lj) {
      if (lj == kb) {
        if (tc == kc) {
#pragma unroll
          for (int li = lj; li < LR; ++li) {
            const int i = tr + G * li;
            const cx<R> a = A[idx(li, lj)];
            if (i > k && i < n) xb[i] = a;
            if (i == k) d[k] = (double)a.re;
            if (k == n - 2 && i == n - 1) {
              const double ar = (double)a.re, ai = (double)a.im;
              e2[k] = ar * ar + ai * ai;
            }
          }
        }
      }
    }
    if (k == n - 2) {
      const int lb = (n - 1) / G;
      if (tr == (n - 1) % G && tc == (n - 1) % G) {
#pragma unroll
        for (int lj = 0; lj < LR; ++lj)
          if (lj == lb) d[n - 1] = (double)A[idx(lj, lj)].re;
      }
    }
  }

  // Householder reduction to (d, e2); leaves them in LDS.
  static __device__ __forceinline__ void run(const int n, cx<R> (&A)[NLOC], Smem& sm,
                                             double* __restrict__ dg, double* __restrict__ e2g) {
    double* d = sm.d;
    double* e2 = sm.e2;
    const int tid = threadIdx.x, tr = tid / G, tc = tid % G, lane = tid & 63;
    if (n == 1) {
      if (tid == 0) dg[0] = (double)A[0].re;
      return;
    }
    write_col(n, 0, A, sm.x[0], d, e2);
    __syncthreads();
    int buf = 0;
    for (int k = 0; k < n - 2; ++k) {
      const cx<R>* xk = sm.x[buf];
      // ---- reflector, computed redundantly and identically by every wavefront
      R s2 = R(0);
      for (int i = k + 2 + lane; i < n; i += 64) {
        const cx<R> v = xk[i];
        s2 += v.re * v.re + v.im * v.im;
      }
      s2 = wave_total_rows(s2);
      const cx<R> al = xk[k + 1];
      R beta, tre, tim, scr, sci;
      if (s2 == R(0) && al.im == R(0)) {
        beta = al.re;
        tre = tim = scr = sci = R(0);
      } else {
        // one reciprocal square root and one reciprocal (the algebra of the
        // split reducer's reflector): r = 1/|x|, sg = sign(Re alpha),
        // beta = -sg |x|, tau = 1 + |Re alpha| r + i sg Im alpha r,
        // 1/(alpha - beta) = (sg (|Re alpha| + |x|) - i Im alpha) / den
        const R s = fma(al.re, al.re, fma(al.im, al.im, s2));
        const R r = rsqrt_nr(s), nrm = s * r;
        const R sg = al.re >= R(0) ? R(1) : R(-1), are = fabs(al.re), dr = are + nrm;
        const R rden = fast_rcp(fma(dr, dr, al.im * al.im));
        beta = -sg * nrm;
        tre = fma(are, r, R(1));
        tim = sg * al.im * r;
        scr = sg * dr * rden;
        sci = -al.im * rden;
      }
      if (tid == 0) {
        e2[k] = (double)beta * (double)beta;
      }
      auto vget = [&](int i) -> cx<R> {
        if (i == k + 1) return {R(1), R(0)};
        if (i > k + 1 && i < n) {
          const cx<R> v = xk[i];
          return {v.re * scr - v.im * sci, v.re * sci + v.im * scr};
        }
        return {R(0), R(0)};
      };
      const int kb = (k + 1) / G;
      // ---- y = B v : row partials (lower part) and column partials (upper part),
      // column block by column block with v read from LDS, so that only the
      // row partials stay in registers beside the matrix
      cx<R>* vs = sm.vw[NVC == 1 ? 0 : tid >> 6];
      if constexpr (NVC == 1) {
        for (int i = kb * G + tid; i < NP; i += NT) vs[i] = vget(i);
        __syncthreads();
      } else {
        for (int i = kb * G + lane; i < NP; i += 64) vs[i] = vget(i);
      }
      const R ms = (tr > tc) ? R(1) : R(0);
      // row partials, one accumulator per row block
#pragma unroll
      for (int li = 0; li < LR; ++li) {
        if (li < kb) continue;
        cx<R> yr = {R(0), R(0)};
#pragma unroll
        for (int lj = 0; lj <= li; ++lj) {
          if (lj < kb) continue;
          const cx<R> vc = vs[tc + G * lj];
          const cx<R> a = A[idx(li, lj)];
          yr.re += a.re * vc.re - a.im * vc.im;
          yr.im += a.re * vc.im + a.im * vc.re;
        }
        const int i = tr + G * li;
        if (i > k && i < n) sm.pr[tc * PITCH + i] = yr;
      }
      // column partials, one accumulator per column block
#pragma unroll
      for (int lj = 0; lj < LR; ++lj) {
        if (lj < kb) continue;
        cx<R> yc = {R(0), R(0)};
#pragma unroll
        for (int li = lj; li < LR; ++li) {
          const cx<R> vi = vs[tr + G * li];
          const cx<R> a = A[idx(li, lj)];
          if (li == lj) {  // diagonal block: strictly lower entries only
            yc.re += ms * (a.re * vi.re + a.im * vi.im);
            yc.im += ms * (a.re * vi.im - a.im * vi.re);
          } else {
            yc.re += a.re * vi.re + a.im * vi.im;
            yc.im += a.re * vi.im - a.im * vi.re;
          }
        }
        const int j = tc + G * lj;
        if (j > k && j < n) sm.pc[tr * PITCH + j] = yc;
      }
      __syncthreads();
      for (int i = k + 1 + tid; i < n; i += NT) {
        cx<R> s = {R(0), R(0)};
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const cx<R> a = sm.pr[t * PITCH + i], b = sm.pc[t * PITCH + i];
          s.re += a.re + b.re;
          s.im += a.im + b.im;
        }
        sm.y[i] = s;
      }
      __syncthreads();
      // ---- w = tau y - (|tau|^2/2) Re(v^H y) v
      R c = R(0);
      for (int i = k + 1 + lane; i < n; i += 64) {
        const cx<R> v = vget(i), yy = sm.y[i];
        c += v.re * yy.re + v.im * yy.im;
      }
      c = wave_total_rows(c);
      const R a2 = R(0.5) * (tre * tre + tim * tim) * c;
      auto wget = [&](int i, cx<R> v) -> cx<R> {
        if (i <= k || i >= n) return {R(0), R(0)};
        const cx<R> yy = sm.y[i];
        return {tre * yy.re - tim * yy.im - a2 * v.re, tre * yy.im + tim * yy.re - a2 * v.im};
      };
      cx<R>* ws = sm.ww[NVC == 1 ? 0 : tid >> 6];
      if constexpr (NVC == 1) {
        for (int i = kb * G + tid; i < NP; i += NT) ws[i] = wget(i, vs[i]);
        __syncthreads();
      } else {
        for (int i = kb * G + lane; i < NP; i += 64) ws[i] = wget(i, vs[i]);
      }
      // ---- B <- B - v w^H - w v^H on the stored lower triangle
      const R mr = (tr >= tc) ? R(1) : R(0);
#pragma unroll
      for (int lj = 0; lj < LR; ++lj) {
        if (lj < kb) continue;
        const cx<R> vc = vs[tc + G * lj], wc = ws[tc + G * lj];
#pragma unroll
        for (int li = lj; li < LR; ++li) {
          const cx<R> vi = vs[tr + G * li], wi = ws[tr + G * li];
          cx<R>& a = A[idx(li, lj)];
          if (li > lj) {
            a.re -= vi.re * wc.re + vi.im * wc.im + wi.re * vc.re + wi.im * vc.im;
            a.im -= vi.im * wc.re - vi.re * wc.im + wi.im * vc.re - wi.re * vc.im;
          } else {
            const R ur = vi.re * wc.re + vi.im * wc.im + wi.re * vc.re + wi.im * vc.im;
            const R ui = vi.im * wc.re - vi.re * wc.im + wi.im * vc.re - wi.re * vc.im;
            a.re -= mr * ur;
            a.im -= ms * ui;
          }
        }
      }
      write_col(n, k + 1, A, sm.x[buf ^ 1], d, e2);
      buf ^= 1;
      __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += NT) {
      dg[i] = d[i];
      if (i < n - 1) e2g[i] = e2[i];
    }
  }

};

}  // namespace tca
