// Householder reduction of one dense complex Hermitian matrix per workgroup to
// real symmetric tridiagonal form, full matrix in registers, with the rank-2
// update of step k and the Hermitian matrix-vector product of step k+1 fused
// into one pass over the registers and one workgroup barrier per step.
//
// Layout as in reduce_full.hpp: thread (tr, tc) = (tid / TC, tid % TC) owns
// rows i = tr + TR*li (li < LR) and columns j = tc + TC*lj (lj < LC); the TC
// lanes of a row group sum their row partials with a DPP reduce-scatter.
//
// Step algebra (reflector k acts on rows k+1..n-1 of column k):
//   alpha = x_0, s2 = sum_{i>0} |x_i|^2, beta = -sign(Re alpha) sqrt(|alpha|^2 + s2),
//   tau = (beta - alpha)/beta, v = (1, x_1/(alpha - beta), ...),
//   y = A v,  w = tau y - (|tau|^2/2) Re(v^H y) v,  A <- A - v w^H - w v^H,
//   d_k = Re A_kk, e_k^2 = beta^2.
// Fusion.  Before the register pass of step k the next reflector v_{k+1} must
// be known.  Its column is A^{(k+1)}[:, k+1] = A^{(k)}[:, k+1]
// - v_k conj(w_k[k+1]) - w_k conj(v_k[k+1]); the owners of column k+1 wrote
// A^{(k)}[:, k+1] to LDS during the previous pass, so every wavefront applies
// this rank-2 correction to one column itself, builds v_{k+1}, and then the
// pass updates each register entry with (v_k, w_k) and immediately
// accumulates it into y_{k+1} = A^{(k+1)} v_{k+1}.
//
// Work skipping.  The pass of step k only touches local blocks whose rows and
// columns reach the trailing part (>= k+1).  The block bounds change every TC
// steps, so the pass is compiled once per phase P = (k+1)/TC with the bounds
// as constants: no per-element selects or branches in the FMA stream, and
// every complex update is written as explicit fused multiply-adds (8 for the
// rank-2 update, 4 for the product).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "cplx.hpp"
#include "reduce_full.hpp"

namespace tca {

// 1/x to full precision for normal, finite x: hardware reciprocal and two
// Newton steps (no scaling for denormals or overflow, which the reflector
// never produces for a nonzero column).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// f(integral_constant<int, I>) for I = B .. E-1
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <typename R>
struct Vec4Of;
template <>
struct Vec4Of<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4Of<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};

// MF = true: the rank-2 update of each 16 x 16 tile runs on the matrix cores.
// With the 32 x 16 grid and LR = 4, the four registers (li = 0..3) of one
// column block lj held by the 16-lane group g of wavefront w are exactly an
// MFMA 16 x 16 accumulator tile: rows 4w + g + 32 li, columns 16 lj + (lane
// % 16).  The real and imaginary parts of A - v w^H - w v^H are each one
// K = 4 product (operands: the row components of v and w, negated, times the
// column components of w and v), i.e. two v_mfma_*_16x16x4 per tile per step;
// the matrix-vector product stays on the vector ALUs.
template <int TR, int TC, int LR, int LC, typename R, int MW = 0, bool MF = false>
struct ReduceFused {
  static constexpr int NT = TR * TC;
  static constexpr int NW = NT / 64;
  static constexpr int NPR = TR * LR;
  static constexpr int NPC = TC * LC;
  static constexpr int NP = NPR > NPC ? NPR : NPC;
  static constexpr int NLOC = LR * LC;
  static constexpr int NV = 2 * LR;
  static constexpr int PV = pow2_ceil<NV>::value < 8 ? 8 : pow2_ceil<NV>::value;
  static constexpr int RATIO = TR / TC;  // phase P covers row blocks li >= P / RATIO
  // minimum wavefronts per SIMD for the launch bounds (MW overrides)
  static constexpr int MINW = MW > 0 ? MW : ((sizeof(R) == 4 && NLOC <= 48) ? 4 : 1);
  static_assert(NT % 64 == 0 && 64 % TC == 0, "bad thread grid");
  static_assert(TR % TC == 0, "row groups must be a multiple of the column groups");
  static_assert(PV <= TC, "row group too narrow for the reduce-scatter");
  static_assert(!MF || (TR == 32 && TC == 16 && LR == 4), "matrix-core tiles need the 32x16 grid");
  typedef typename Vec4Of<R>::type R4;

  // Register storage: per (li, lj) complex entries, or per column block one
  // accumulator tile of real parts and one of imaginary parts.
  struct TileRegs {
    R4 re[LC], im[LC];
  };
  typedef typename std::conditional<MF, TileRegs, cx<R>[NLOC]>::type Regs;

  static __device__ __forceinline__ cx<R> get(const Regs& A, int li, int lj) {
    if constexpr (MF)
      return {A.re[lj][li], A.im[lj][li]};
    else
      return A[li * LC + lj];
  }
  static __device__ __forceinline__ void set(Regs& A, int li, int lj, cx<R> v) {
    if constexpr (MF) {
      A.re[lj][li] = v.re;
      A.im[lj][li] = v.im;
    } else {
      A[li * LC + lj] = v;
    }
  }

  struct Smem {
    cx<R> col[2][NP];    // column k+1 of A^{(k)} (double-buffered by column parity)
    cx<R> y[2][NP];      // y_k = A^{(k)} v_k (double-buffered by step parity)
    cx<R> vb[NW][2][NP]; // per-wavefront reflector vectors v_k, v_{k+1} (by parity)
    cx<R> wb[NW][NP];    // per-wavefront w_k
    double d[NP];
    double e2[NP];
  };

  static __device__ __forceinline__ int idx(int li, int lj) { return li * LC + lj; }

  static constexpr int NQ = (NP + 63) / 64;  // LDS vector entries per lane

  // Entry i of a lane-strided vector (entry i sits in lane i % 64, slot i / 64),
  // the same value in every lane; i must be wavefront-uniform.
  static __device__ __forceinline__ cx<R> bcast(const cx<R> (&v)[NQ], const int i) {
    cx<R> s = v[0];
#pragma unroll
    for (int q = 1; q < NQ; ++q)
      if ((i >> 6) == q) s = v[q];
    return {readlane_t(s.re, i & 63), readlane_t(s.im, i & 63)};
  }

  template <class F>
  static __device__ __forceinline__ void load(Regs& A, const int n, F&& lower) {
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
        set(A, li, lj, v);
      }
    }
  }

  // Column `wc` of the registers -> colbuf (all owned rows; only rows >= wc
  // are read later).
  static __device__ __forceinline__ void store_col(const Regs& A, const int wc, cx<R>* colbuf) {
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
    if (tc != wc % TC) return;
    const int lw = wc / TC;
#pragma unroll
    for (int lj = 0; lj < LC; ++lj) {
      if (lj != lw) continue;
#pragma unroll
      for (int li = 0; li < LR; ++li) colbuf[tr + TR * li] = get(A, li, lj);
    }
  }

  // One register pass of phase P: A <- A - vk wk^H - wk vk^H on the blocks
  // that reach the trailing part, part += A * vn (row partials).
  template <int P>
  static __device__ __forceinline__ void pass(Regs& A, const cx<R>* __restrict__ vk,
                                              const cx<R>* __restrict__ wk,
                                              const cx<R>* __restrict__ vn, R (&part)[PV]) {
    constexpr int KR = P / RATIO;
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
#pragma unroll
    for (int q = 0; q < PV; ++q) part[q] = R(0);
    if constexpr (MF) {
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, ii = lane & 15;
      // global row of accumulator row ii of this wavefront's tiles
      const int row = sizeof(R) == 8 ? 4 * wave + (ii & 3) + 32 * (ii >> 2)
                                     : 4 * wave + (ii >> 2) + 32 * (ii & 3);
      // A operand (row ii, k = g): -(vr, vi, wr, wi)[g] for the real part,
      // -(vi, -vr, wi, -wr)[g] for the imaginary part
      const R* ra = reinterpret_cast<const R*>(g < 2 ? vk : wk) + 2 * row;
      const R aop_re = -ra[g & 1];
      const R aop_im = (g & 1) ? ra[0] : -ra[1];
      // B operand (k = g, column of this lane): (wr, wi, vr, vi)[g]
      const R* rb = reinterpret_cast<const R*>(g < 2 ? wk : vk) + 2 * tc + (g & 1);
      // tile lj + 1 goes to the matrix cores while the vector ALUs form the
      // product of tile lj
      auto update = [&](auto LJ) {
        constexpr int lj = decltype(LJ)::value;
        const R bop = rb[2 * TC * lj];
        if constexpr (sizeof(R) == 8) {
          A.re[lj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop_re, bop, A.re[lj], 0, 0, 0);
          A.im[lj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop_im, bop, A.im[lj], 0, 0, 0);
        } else {
          A.re[lj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop_re, bop, A.re[lj], 0, 0, 0);
          A.im[lj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop_im, bop, A.im[lj], 0, 0, 0);
        }
      };
      auto product = [&](auto LJ) {
        constexpr int lj = decltype(LJ)::value;
        const cx<R> xc = vn[tc + TC * lj];
#pragma unroll
        for (int li = KR; li < LR; ++li) {
          const R are = A.re[lj][li], aim = A.im[lj][li];
          part[2 * li] = fma(are, xc.re, part[2 * li]);
          part[2 * li] = fma(-aim, xc.im, part[2 * li]);
          part[2 * li + 1] = fma(are, xc.im, part[2 * li + 1]);
          part[2 * li + 1] = fma(aim, xc.re, part[2 * li + 1]);
        }
      };
      update(std::integral_constant<int, P>{});
      static_for<P, LC>([&](auto LJ) {
        constexpr int lj = decltype(LJ)::value;
        if constexpr (lj + 1 < LC) update(std::integral_constant<int, lj + 1>{});
        product(LJ);
      });
    } else {
      cx<R> vr[LR], wr[LR];
#pragma unroll
      for (int li = KR; li < LR; ++li) {
        vr[li] = vk[tr + TR * li];
        wr[li] = wk[tr + TR * li];
      }
#pragma unroll
      for (int lj = P; lj < LC; ++lj) {
        const int j = tc + TC * lj;
        const cx<R> vc = vk[j], wc = wk[j], xc = vn[j];
#pragma unroll
        for (int li = KR; li < LR; ++li) {
          cx<R> a = get(A, li, lj);
          // a -= v_i conj(w_j) + w_i conj(v_j)
          a.re = fma(-vr[li].re, wc.re, a.re);
          a.re = fma(-vr[li].im, wc.im, a.re);
          a.re = fma(-wr[li].re, vc.re, a.re);
          a.re = fma(-wr[li].im, vc.im, a.re);
          a.im = fma(-vr[li].im, wc.re, a.im);
          a.im = fma(vr[li].re, wc.im, a.im);
          a.im = fma(-wr[li].im, vc.re, a.im);
          a.im = fma(wr[li].re, vc.im, a.im);
          set(A, li, lj, a);
          // (A v)_i += a x_j
          part[2 * li] = fma(a.re, xc.re, part[2 * li]);
          part[2 * li] = fma(-a.im, xc.im, part[2 * li]);
          part[2 * li + 1] = fma(a.re, xc.im, part[2 * li + 1]);
          part[2 * li + 1] = fma(a.im, xc.re, part[2 * li + 1]);
        }
      }
    }
  }

  // Step k (-1 <= k <= n-3) in phase P = (k+1)/TC: w_k, column k+1 of
  // A^{(k+1)}, reflector k+1, the fused register pass, y_{k+1}; one barrier.
  template <int P>
  static __device__ __forceinline__ void step(const int n, const int k, Regs& A, Smem& sm, R& tre,
                                              R& tim) {
    const int tid = threadIdx.x, tr = tid / TC, lane = tid & 63, wave = tid >> 6;
    const int lg = tid % TC;
    const int q_rs = reduce_scatter_index<TC, PV>(lg);
    const bool w_rs = reduce_scatter_writer<TC, PV>(lg);
    cx<R>* wb = sm.wb[wave];
    {
      const int kb = k & 1, nb = (k + 1) & 1, k1 = k + 1;
      const cx<R>* vk = sm.vb[wave][kb];
      cx<R>* vn = sm.vb[wave][nb];
      const cx<R>* yk = sm.y[kb];
      const cx<R>* colk = sm.col[nb];
      // Every LDS operand of the vector phase is read once, up front; entries
      // outside rows k+1..n-1 are masked with selects (rows <= k of y_k and of
      // the column buffer hold stale data), so the phase has no branches and
      // a single LDS round trip.  For k = -1 the v_k buffer holds zeros.
      cx<R> vv[NQ], yv[NQ];
      bool ok[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        const int ic = i < NP ? i : NP - 1;
        vv[q] = vk[ic];
        yv[q] = yk[ic];
        ok[q] = i > k && i < n;
      }
      // ---- w_k = tau y_k - (|tau|^2/2) Re(v_k^H y_k) v_k   (rows k+1..n-1)
      cx<R> wreg[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) wreg[q] = {R(0), R(0)};
      cx<R> wk1 = {R(0), R(0)};  // w_k[k+1], the same in every lane
      if (k >= 0) {
        R c = R(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const R t = fma(vv[q].re, yv[q].re, vv[q].im * yv[q].im);
          c += ok[q] ? t : R(0);
        }
        c = wave_total(c);
        const R a2 = R(0.5) * (tre * tre + tim * tim) * c;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const R wr_ = fma(tre, yv[q].re, fma(-tim, yv[q].im, -a2 * vv[q].re));
          const R wi_ = fma(tre, yv[q].im, fma(tim, yv[q].re, -a2 * vv[q].im));
          wreg[q] = {ok[q] ? wr_ : R(0), ok[q] ? wi_ : R(0)};
          const int i = lane + 64 * q;
          if (NP % 64 == 0 || i < NP) wb[i] = wreg[q];
        }
        wk1 = bcast(wreg, k1);
      }
      // ---- column k+1 of A^{(k+1)}: x_i = col_i - v_k[i] conj(w_k[k+1]) - w_k[i]  (v_k[k+1] = 1)
      cx<R> xreg[NQ];
      R s2 = R(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int ic = lane + 64 * q < NP ? lane + 64 * q : NP - 1;
        const cx<R> v = vv[q], w = wreg[q], c = colk[ic];
        const R xr = fma(-v.re, wk1.re, fma(-v.im, wk1.im, c.re - w.re));
        const R xi = fma(-v.im, wk1.re, fma(v.re, wk1.im, c.im - w.im));
        xreg[q] = {ok[q] ? xr : R(0), ok[q] ? xi : R(0)};
        const int i = lane + 64 * q;
        const R t = fma(xreg[q].re, xreg[q].re, xreg[q].im * xreg[q].im);
        s2 += i > k + 2 ? t : R(0);
      }
      s2 = wave_total(s2);
      const cx<R> x1 = bcast(xreg, k1);
      if (tid == 0) sm.d[k1] = (double)x1.re;
      cx<R> al = {R(0), R(0)};
      if (k1 + 1 < n) al = bcast(xreg, k1 + 1);
      // ---- reflector k+1 from x[k+2..n-1] (none for the last column pair)
      R scr = R(0), sci = R(0);
      const bool refl = (k1 <= n - 3);
      if (refl) {
        R beta;
        if (s2 == R(0) && al.im == R(0)) {
          beta = al.re;
          tre = tim = R(0);
        } else {
          const R nrm = sqrt(fma(al.re, al.re, fma(al.im, al.im, s2)));
          beta = al.re >= R(0) ? -nrm : nrm;
          const R rb = fast_rcp(beta);
          tre = (beta - al.re) * rb;
          tim = -al.im * rb;
          const R dr = al.re - beta, di = al.im;
          const R rden = fast_rcp(fma(dr, dr, di * di));
          scr = dr * rden;
          sci = -di * rden;
        }
        if (tid == 0) sm.e2[k1] = (double)beta * (double)beta;
      } else if (k1 == n - 2) {
        if (tid == 0) sm.e2[k1] = (double)al.re * (double)al.re + (double)al.im * (double)al.im;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        const cx<R> x = xreg[q];
        const R sr_ = fma(x.re, scr, -x.im * sci), si_ = fma(x.re, sci, x.im * scr);
        const bool head = refl && i == k1 + 1, tail = refl && i > k1 + 1 && i < n;
        const cx<R> v = {head ? R(1) : (tail ? sr_ : R(0)), tail ? si_ : R(0)};
        if (NP % 64 == 0 || i < NP) vn[i] = v;
      }
      wave_lds_fence();
      // ---- fused pass: A^{(k+1)} = A^{(k)} - v_k w_k^H - w_k v_k^H,  part = A^{(k+1)} v_{k+1}
      R part[PV];
      pass<P>(A, vk, wb, vn, part);
      if (k1 + 1 < n) store_col(A, k1 + 1, sm.col[kb]);  // column k+2 of A^{(k+1)}
      // ---- y_{k+1} rows by the reduce-scatter of the row partials
      const R ysum = reduce_scatter<TC, PV>(part, lg);
      if (refl) {
        const int li = q_rs >> 1;
        const int i = tr + TR * li;
        if (w_rs && q_rs < NV && i > k1 && i < n) {
          if (q_rs & 1)
            sm.y[nb][i].im = ysum;
          else
            sm.y[nb][i].re = ysum;
        }
      }
      __syncthreads();
    }
  }

  // Steps of phase P and every later phase; k advances to n-2.
  template <int P>
  static __device__ __forceinline__ void phases(const int n, int& k, Regs& A, Smem& sm, R& tre,
                                                R& tim) {
    if constexpr (P < LC) {
      const int kend = (P + 1) * TC - 2 < n - 3 ? (P + 1) * TC - 2 : n - 3;  // last k of phase P
      for (; k <= kend; ++k) step<P>(n, k, A, sm, tre, tim);
      phases<P + 1>(n, k, A, sm, tre, tim);
    }
  }

  static __device__ __forceinline__ void run(const int n, Regs& A, Smem& sm,
                                             double* __restrict__ dg, double* __restrict__ e2g) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // v_{-1} = w_{-1} = 0
    for (int i = lane; i < NP; i += 64) {
      sm.vb[wave][1][i] = {R(0), R(0)};
      sm.wb[wave][i] = {R(0), R(0)};
    }
    store_col(A, 0, sm.col[0]);
    __syncthreads();
    R tre = R(0), tim = R(0);  // tau of the current reflector
    int k = -1;
    phases<0>(n, k, A, sm, tre, tim);
    if (tid == 0) sm.d[n - 1] = (double)sm.col[(n - 1) & 1][n - 1].re;
    __syncthreads();
    for (int i = tid; i < n; i += NT) {
      dg[i] = sm.d[i];
      if (i < n - 1) e2g[i] = sm.e2[i];
    }
  }
};

}  // namespace tca
