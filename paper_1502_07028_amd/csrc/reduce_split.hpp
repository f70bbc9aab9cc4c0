// Householder reduction of one dense complex Hermitian matrix per workgroup to
// real symmetric tridiagonal form, full matrix in registers, one workgroup
// barrier per step, with the per-step vector work cut down and the rank-2
// update separated from the matrix-vector product so that the serial part of
// a step can overlap register work.
//
// Register layout, LDS buffers and step algebra are those of reduce_fused.hpp
// (32 x 16 or 16 x 16 thread grid, thread (tr, tc) owns rows tr + TR*li and
// columns tc + TC*lj).  What changes:
//
// Step order.  Step k is
//   (1) c = Re(v_k^H y_k), w_k = tau_k y_k - (|tau_k|^2/2) c v_k;
//   (2) column k+1 of A^{(k+1)}, its norm, reflector v_{k+1}      (vector work)
//   (3) update  A^{(k+1)} = A^{(k)} - v_k w_k^H - w_k v_k^H       (registers)
//   (4) product y_{k+1} = A^{(k+1)} v_{k+1}, row reduce-scatter, barrier.
// (2) and (3) are independent.  With MF the update is a pair of MFMA
// products per 16 x 16 tile (but for the last VT column blocks, which the
// vector ALUs update after (2): FP64 matrix cores and vector ALUs have the
// same peak, so the two share the work), all operands read from LDS first and the MFMAs
// issued before (2), so that the matrix cores work while the vector ALUs
// build the reflector (issuing them in groups between the parts of (2),
// pinned by scheduling barriers, measured slower); otherwise (2) runs first,
// which keeps the register update and the product together.
//
// With LD, only the lower half of the wavefronts (one per SIMD) builds the
// reflector; the other half issues its update and waits at a second barrier,
// then takes v_{k+1} and tau from the leaders' LDS copies.
//
// Less vector work per step.
//  - Buffers are cleared once, so v_k vanishes outside rows k+1..n-1 and y_k
//    is finite everywhere: c needs no row mask, and w_k may hold nonzero
//    values in rows <= k.  Those only reach register entries of rows or
//    columns <= k, which later steps multiply by zero entries of v and never
//    store, and they stay finite (each step adds bounded terms).
//  - w_k[k+1], w_k[k+2] and x[k+1], x[k+2] come from a few uniform LDS reads
//    (v_k[k+1] = 1 whenever tau_k != 0) instead of lane broadcasts.
//  - The reflector takes one reciprocal square root and one reciprocal:
//    with s = |alpha|^2 + s2, r = 1/sqrt(s), sg = sign(Re alpha):
//      beta = -sg s r,  tau = 1 + |Re alpha| r + i sg Im alpha r,
//      1/(alpha - beta) = (sg (|Re alpha| + s r) - i Im alpha) / den,
//      den = (|Re alpha| + s r)^2 + (Im alpha)^2.
//  - Wavefront sums finish with DPP row broadcasts; the row reduce-scatter
//    only carries the row blocks that are still active in the phase.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "reduce_fused.hpp"

namespace tca {

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_rows(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_rows(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

// Sum over the 64 lanes, returned as a wavefront-uniform value: row sums,
// then row 1 += row 0 and row 3 += row 2 (row_bcast:15), then row 3 += row 1
// (row_bcast:31); lane 63 holds the total.
template <typename T>
__device__ __forceinline__ T wave_total_rows(T v) {
  v = group_sum<16>(v);
  v += dpp_rows<0x142, 0xA>(v);
  v += dpp_rows<0x143, 0xC>(v);
  return readlane_t(v, 63);
}

// Reduce-scatter of P values (P a power of two, 2 <= P <= TC) over a row
// group of TC = 8 or 16 lanes; lane l ends with the group total of value
// reduce_scatter_index<TC, P>(l), and the lanes of a duplicate group all hold
// it.
template <int TC, int P, typename T>
__device__ __forceinline__ T rs_group(const T (&v)[P], const int l) {
  static_assert((TC == 8 || TC == 16) && P >= 2 && P <= TC && (P & (P - 1)) == 0, "bad width");
  if constexpr (P == TC || (TC == 16 && P == 8)) {
    return reduce_scatter<TC, P>(v, l);
  } else if constexpr (TC == 16 && P == 4) {
    T a2[2], a1[1];
    rs_stage<kDppRowMirror>(v, a2, (l & 8) != 0);
    rs_stage<kDppRowHalfMirror>(a2, a1, (l & 4) != 0);
    T r = a1[0];
    r += dpp_mov<kDppQuadReverse>(r);
    r += dpp_mov<kDppQuadSwap1>(r);
    return r;
  } else if constexpr (TC == 16) {  // P == 2
    T a1[1];
    rs_stage<kDppRowMirror>(v, a1, (l & 8) != 0);
    T r = a1[0];
    r += dpp_mov<kDppRowHalfMirror>(r);
    r += dpp_mov<kDppQuadReverse>(r);
    r += dpp_mov<kDppQuadSwap1>(r);
    return r;
  } else if constexpr (P == 4) {  // TC == 8
    T a2[2], a1[1];
    rs_stage<kDppRowHalfMirror>(v, a2, (l & 4) != 0);
    rs_stage<kDppQuadReverse>(a2, a1, (l & 2) != 0);
    T r = a1[0];
    r += dpp_mov<kDppQuadSwap1>(r);
    return r;
  } else {  // TC == 8, P == 2
    T a1[1];
    rs_stage<kDppRowHalfMirror>(v, a1, (l & 4) != 0);
    T r = a1[0];
    r += dpp_mov<kDppQuadReverse>(r);
    r += dpp_mov<kDppQuadSwap1>(r);
    return r;
  }
}

__device__ __forceinline__ double rsqrt_nr(double s) {
  double r = __builtin_amdgcn_rsq(s);
  double t = s * r;
  double e = fma(-t, r, 1.0);
  r = fma(0.5 * r, e, r);
  t = s * r;
  e = fma(-t, r, 1.0);
  return fma(0.5 * r, e, r);
}
__device__ __forceinline__ float rsqrt_nr(float s) {
  float r = __builtin_amdgcn_rsqf(s);
  const float t = s * r;
  const float e = fmaf(-t, r, 1.0f);
  return fmaf(0.5f * r, e, r);
}

// The operands of the reflector of step k that are ready when the step
// begins: column k+1 of A^{(k)} (rows lane + 64 q) and the entries k+1, k+2
// of that column, of y_k and of v_k.
template <int NQ, typename R>
struct ReflectIn {
  cx<R> cv[NQ];
  cx<R> c1, c2, y1, y2, v2;
};
template <int NP, int NQ, typename R, class Smem>
__device__ __forceinline__ ReflectIn<NQ, R> reflect_in(const int k, const Smem& sm,
                                                       const cx<R>* __restrict__ vk) {
  const int lane = threadIdx.x & 63, k1 = k + 1;
  const cx<R>* colk = sm.col[(k + 1) & 1];
  const cx<R>* yk = sm.y[k & 1];
  ReflectIn<NQ, R> o;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    o.cv[q] = colk[i < NP ? i : NP - 1];
  }
  o.c1 = colk[k1];
  o.c2 = colk[k1 + 1];
  o.y1 = yk[k1];
  o.y2 = yk[k1 + 1];
  o.v2 = vk[k1 + 1];
  return o;
}

// Column k+1 of A^{(k+1)}, d_{k+1}, e_{k+1}^2, reflector k+1 into this
// wavefront's copy of v_{k+1} and (tre, tim), from the operands read when the
// step began and this wavefront's rows of v_k and w_k (vv, wv) in registers.
template <int NP, int NQ, typename R, class Smem>
__device__ __forceinline__ void split_reflect(const int n, const int k, Smem& sm, const R a2, R& tre,
                                            R& tim, const ReflectIn<NQ, R>& in,
                                            const cx<R> (&vv)[NQ], const cx<R> (&wv)[NQ]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, k1 = k + 1;
  cx<R>* vn = sm.vb[wave][(k + 1) & 1];
  const cx<R> c1 = in.c1, c2 = in.c2, y1 = in.y1, y2 = in.y2, v2 = in.v2;
  // w_k[k+1] (v_k[k+1] = 1 whenever tau_k != 0) and w_k[k+2]
  const cx<R> wk1 = {fma(tre, y1.re, fma(-tim, y1.im, -a2)), fma(tre, y1.im, tim * y1.re)};
  const cx<R> wk2 = {fma(tre, y2.re, fma(-tim, y2.im, -a2 * v2.re)),
                     fma(tre, y2.im, fma(tim, y2.re, -a2 * v2.im))};
  const cx<R>(&cv)[NQ] = in.cv;
  // x_i = col_i - v_k[i] conj(w_k[k+1]) - w_k[i]
  cx<R> xreg[NQ];
  R s2 = R(0);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + 64 * q;
    const cx<R> c = cv[q], v = vv[q], w = wv[q];
    xreg[q].re = fma(-v.re, wk1.re, fma(-v.im, wk1.im, c.re - w.re));
    xreg[q].im = fma(-v.im, wk1.re, fma(v.re, wk1.im, c.im - w.im));
    const R t = fma(xreg[q].re, xreg[q].re, xreg[q].im * xreg[q].im);
    s2 += (i > k1 + 1 && i < n) ? t : R(0);
  }
  // x[k+1] (v_k[k+1] = 1 or w_k = 0) and x[k+2]
  const R d1 = fma(R(-2), wk1.re, c1.re);
  cx<R> al;
  al.re = fma(-v2.re, wk1.re, fma(-v2.im, wk1.im, c2.re - wk2.re));
  al.im = fma(-v2.im, wk1.re, fma(v2.re, wk1.im, c2.im - wk2.im));
  s2 = wave_total_rows(s2);
  if (tid == 0) sm.d[k1] = (double)d1;
  const bool refl = (k1 <= n - 3);
  const bool triv = (s2 == R(0) && al.im == R(0));
  const bool act = refl && !triv;
  const R s = act ? fma(al.re, al.re, fma(al.im, al.im, s2)) : R(1);
  const R r = rsqrt_nr(s);
  const R nrm = s * r;
  const R sg = al.re >= R(0) ? R(1) : R(-1);
  const R are = fabs(al.re);
  const R dr = are + nrm;
  const R rden = fast_rcp(fma(dr, dr, al.im * al.im));
  const R scr = act ? sg * dr * rden : R(0);
  const R sci = act ? -al.im * rden : R(0);
  tre = act ? fma(are, r, R(1)) : R(0);
  tim = act ? sg * al.im * r : R(0);
  if (tid == 0) {
    if (refl) {
      const double beta = act ? -(double)sg * (double)nrm : (double)al.re;
      sm.e2[k1] = beta * beta;
    } else if (k1 == n - 2) {
      sm.e2[k1] = (double)al.re * (double)al.re + (double)al.im * (double)al.im;
    }
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
}

template <int TR, int TC, int LR, int LC, typename R, int MW = 0, bool MF = false, int VT = 0,
          bool LD = false>
struct ReduceSplit : ReduceFused<TR, TC, LR, LC, R, MW, false> {
  typedef ReduceFused<TR, TC, LR, LC, R, MW, false> Base;
  struct Smem : Base::Smem {
    R tau[2][2];  // tau of the newest reflector (by step parity), for the followers
  };
  typedef typename Base::R4 R4;
  static constexpr int NT = Base::NT;
  static constexpr int NW = Base::NW;
  static constexpr int NP = Base::NP;
  static constexpr int NQ = Base::NQ;
  static constexpr int NLOC = Base::NLOC;
  static constexpr int RATIO = Base::RATIO;
  static constexpr int MINW = Base::MINW;
  static constexpr int NRT = LR / 4;  // MFMA row tiles per column block
  static_assert(TC == 8 || TC == 16, "row groups of 8 or 16 lanes");
  static_assert(2 * LR <= TC, "at most TC row values per lane");
  static_assert(!MF || TC == 16, "matrix-core tiles need 16-lane row groups");
  static_assert(!MF || (LR % 4 == 0 && TR == 4 * NW), "matrix-core tiles need LR = 4a");

  // Register storage.  With MF, the registers of column block lj and row
  // blocks 4a .. 4a+3 of wavefront w form one MFMA 16 x 16 accumulator tile
  // (real and imaginary parts apart): register r of lane l holds row
  // 4w + l/16 + TR (4a + r), column 16 lj + l % 16, which is where the FP32
  // (row 4 (l/16) + r) and the FP64 (row l/16 + 4r) accumulator layouts put
  // tile row l/16 + 4r resp. 4 (l/16) + r.
  struct TileRegs {
    R4 re[LC][NRT > 0 ? NRT : 1], im[LC][NRT > 0 ? NRT : 1];
  };
  typedef typename std::conditional<MF, TileRegs, cx<R>[NLOC]>::type Regs;

  static __device__ __forceinline__ cx<R> get(const Regs& A, int li, int lj) {
    if constexpr (MF)
      return {A.re[lj][li >> 2][li & 3], A.im[lj][li >> 2][li & 3]};
    else
      return A[li * LC + lj];
  }
  static __device__ __forceinline__ void set(Regs& A, int li, int lj, cx<R> v) {
    if constexpr (MF) {
      A.re[lj][li >> 2][li & 3] = v.re;
      A.im[lj][li >> 2][li & 3] = v.im;
    } else {
      A[li * LC + lj] = v;
    }
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

  // MFMA operands of the rank-2 update of phase P: row components of v and w
  // (A operand, negated) of every active row tile and the column components
  // of w and v of every active column block (B operand), read from LDS once.
  struct MfOps {
    R aop_re[NRT > 0 ? NRT : 1], aop_im[NRT > 0 ? NRT : 1];
    R bop[LC];
  };
  template <int P>
  static __device__ __forceinline__ MfOps mf_ops(const cx<R>* __restrict__ vk,
                                                 const cx<R>* __restrict__ wk) {
    constexpr int A0 = (P / RATIO) / 4;
    const int tc = threadIdx.x % TC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, ii = lane & 15;
    // tile row ii -> (group, register) -> matrix row
    const int rg = sizeof(R) == 8 ? (ii & 3) : (ii >> 2), rr = sizeof(R) == 8 ? (ii >> 2) : (ii & 3);
    const R* rb = reinterpret_cast<const R*>(g < 2 ? wk : vk) + 2 * tc + (g & 1);
    MfOps o;
#pragma unroll
    for (int a = A0; a < NRT; ++a) {
      const int row = 4 * wave + rg + TR * (4 * a + rr);
      const R* ra = reinterpret_cast<const R*>(g < 2 ? vk : wk) + 2 * row;
      o.aop_re[a] = -ra[g & 1];
      o.aop_im[a] = (g & 1) ? ra[0] : -ra[1];
    }
#pragma unroll
    for (int lj = P; lj < LC; ++lj) o.bop[lj] = rb[2 * TC * lj];
    return o;
  }
  // Issue the update MFMAs of the active tiles of phase P in column blocks
  // below JE.
  template <int P, int JE>
  static __device__ __forceinline__ void mf_tiles(Regs& A, const MfOps& o) {
    constexpr int A0 = (P / RATIO) / 4;
    static_for<P, JE>([&](auto LJ) {
      constexpr int lj = decltype(LJ)::value;
      static_for<A0, NRT>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        if constexpr (sizeof(R) == 8) {
          A.re[lj][a] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(o.aop_re[a], o.bop[lj], A.re[lj][a], 0, 0, 0);
          A.im[lj][a] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(o.aop_im[a], o.bop[lj], A.im[lj][a], 0, 0, 0);
        } else {
          A.re[lj][a] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(o.aop_re[a], o.bop[lj], A.re[lj][a], 0, 0, 0);
          A.im[lj][a] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(o.aop_im[a], o.bop[lj], A.im[lj][a], 0, 0, 0);
        }
      });
    });
  }

  // A <- A - vk wk^H - wk vk^H on the vector ALUs, row blocks from KR and
  // column blocks from J0.
  template <int KR, int J0>
  static __device__ __forceinline__ void valu_update(Regs& A, const cx<R>* __restrict__ vk,
                                                     const cx<R>* __restrict__ wk) {
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
    cx<R> vr[LR], wr[LR];
#pragma unroll
    for (int li = KR; li < LR; ++li) {
      vr[li] = vk[tr + TR * li];
      wr[li] = wk[tr + TR * li];
    }
#pragma unroll
    for (int lj = J0; lj < LC; ++lj) {
      const int j = tc + TC * lj;
      const cx<R> vc = vk[j], wc = wk[j];
#pragma unroll
      for (int li = KR; li < LR; ++li) {
        cx<R> a = get(A, li, lj);
        a.re = fma(-vr[li].re, wc.re, a.re);
        a.re = fma(-vr[li].im, wc.im, a.re);
        a.re = fma(-wr[li].re, vc.re, a.re);
        a.re = fma(-wr[li].im, vc.im, a.re);
        a.im = fma(-vr[li].im, wc.re, a.im);
        a.im = fma(vr[li].re, wc.im, a.im);
        a.im = fma(-wr[li].im, vc.re, a.im);
        a.im = fma(wr[li].re, vc.im, a.im);
        set(A, li, lj, a);
      }
    }
  }

  // Column wc (= k+2) of the registers -> colbuf.  In phase P it lies in
  // column block P, or in block P+1 at the phase's last step: the two
  // candidates are selected, so register indices stay static.
  template <int P>
  static __device__ __forceinline__ void store_next_col(const Regs& A, const int wc,
                                                        cx<R>* __restrict__ colbuf) {
    constexpr int P1 = P + 1 < LC ? P + 1 : P;
    const int tr = threadIdx.x / TC, tc = threadIdx.x % TC;
    const bool in_p = wc < TC * (P + 1);
    if (tc == wc % TC) {
#pragma unroll
      for (int li = 0; li < LR; ++li) {
        const cx<R> a = get(A, li, P), b = get(A, li, P1);
        colbuf[tr + TR * li] = {in_p ? a.re : b.re, in_p ? a.im : b.im};
      }
    }
  }

  // part[2 li + {0,1}] = row partials of A x over the blocks of phase P.
  template <int P>
  static __device__ __forceinline__ void product(const Regs& A, const cx<R>* __restrict__ x,
                                                 R (&part)[2 * LR]) {
    constexpr int KR = P / RATIO;
    const int tc = threadIdx.x % TC;
#pragma unroll
    for (int q = 0; q < 2 * LR; ++q) part[q] = R(0);
#pragma unroll
    for (int lj = P; lj < LC; ++lj) {
      const cx<R> xc = x[tc + TC * lj];
#pragma unroll
      for (int li = KR; li < LR; ++li) {
        const cx<R> a = get(A, li, lj);
        part[2 * li] = fma(a.re, xc.re, part[2 * li]);
        part[2 * li] = fma(-a.im, xc.im, part[2 * li]);
        part[2 * li + 1] = fma(a.re, xc.im, part[2 * li + 1]);
        part[2 * li + 1] = fma(a.im, xc.re, part[2 * li + 1]);
      }
    }
  }

  static __device__ __forceinline__ void reflect(const int n, const int k, Smem& sm, const R a2,
                                                 R& tre, R& tim, const ReflectIn<NQ, R>& in,
                                                 const cx<R> (&vv)[NQ], const cx<R> (&wv)[NQ]) {
    split_reflect<NP, NQ>(n, k, sm, a2, tre, tim, in, vv, wv);
  }

  template <int P>
  static __device__ __forceinline__ void step(const int n, const int k, Regs& A, Smem& sm, R& tre,
                                              R& tim) {
    constexpr int KR = P / RATIO;
    constexpr int NA = 2 * (LR - KR);  // row values still active
    constexpr int PA = NA <= 2 ? 2 : NA <= 4 ? 4 : NA <= 8 ? 8 : 16;
    static_assert(PA <= TC, "row values exceed the row group");
    const int tid = threadIdx.x, tr = tid / TC, lane = tid & 63;
    // with LD the wavefront index is made scalar, so the role test is a
    // uniform branch
    const int wave = LD ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
    const int lg = tid % TC;
    const int kb = k & 1, nb = (k + 1) & 1, k1 = k + 1;
    // with LD the lower half of the wavefronts (one per SIMD) builds the
    // reflector and the upper half uses their copies
    const bool leader = !LD || wave < NW / 2;
    const int lead = LD ? wave % (NW / 2) : wave;
    const cx<R>* vk = sm.vb[lead][kb];
    const cx<R>* vn = sm.vb[lead][nb];
    cx<R>* wb = sm.wb[wave];
    const cx<R>* yk = sm.y[kb];
    // ---- (1) w_k
    cx<R> vv[NQ], yv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      const int ic = i < NP ? i : NP - 1;
      vv[q] = vk[ic];
      yv[q] = yk[ic];
    }
    // the reflector's LDS operands are read with these (with LD after the
    // leaders' matrix-core issue, which measured faster there)
    ReflectIn<NQ, R> rin;
    if (!LD) rin = reflect_in<NP, NQ>(k, sm, vk);
    R c = R(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      const R t = fma(vv[q].re, yv[q].re, vv[q].im * yv[q].im);
      c += (NP % 64 == 0 || i < NP) ? t : R(0);  // lanes past NP read row NP-1 again
    }
    c = wave_total_rows(c);
    const R a2 = R(0.5) * (tre * tre + tim * tim) * c;
    cx<R> wv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      wv[q].re = fma(tre, yv[q].re, fma(-tim, yv[q].im, -a2 * vv[q].re));
      wv[q].im = fma(tre, yv[q].im, fma(tim, yv[q].re, -a2 * vv[q].im));
      const int i = lane + 64 * q;
      if (NP % 64 == 0 || i < NP) wb[i] = wv[q];
    }
    wave_lds_fence();
    // ---- (2) reflector and (3) update
    if constexpr (LD) {
      // followers: the update only, while the leaders build the reflector
      if constexpr (MF) {
        mf_tiles<P, LC>(A, mf_ops<P>(vk, wb));
        if (leader) {
          rin = reflect_in<NP, NQ>(k, sm, vk);
          reflect(n, k, sm, a2, tre, tim, rin, vv, wv);
        }
      } else {
        if (leader) {
          rin = reflect_in<NP, NQ>(k, sm, vk);
          reflect(n, k, sm, a2, tre, tim, rin, vv, wv);
        }
        valu_update<P / RATIO, P>(A, vk, wb);
      }
      if (tid == 0) {
        sm.tau[nb][0] = tre;
        sm.tau[nb][1] = tim;
      }
      __syncthreads();
      if (!leader) {
        tre = sm.tau[nb][0];
        tim = sm.tau[nb][1];
      }
    } else if constexpr (MF) {
      // the last VT column blocks of the update on the vector ALUs, after (2)
      constexpr int JE = LC - VT > P ? LC - VT : P;
      mf_tiles<P, JE>(A, mf_ops<P>(vk, wb));
      reflect(n, k, sm, a2, tre, tim, rin, vv, wv);
      if constexpr (JE < LC) valu_update<P / RATIO, JE>(A, vk, wb);
      wave_lds_fence();
    } else {
      reflect(n, k, sm, a2, tre, tim, rin, vv, wv);
      valu_update<P / RATIO, P>(A, vk, wb);
      wave_lds_fence();
    }
    if (k1 + 1 < n) store_next_col<P>(A, k1 + 1, sm.col[kb]);  // column k+2 of A^{(k+1)}
    // ---- (4) y_{k+1}
    R part[2 * LR];
    product<P>(A, vn, part);
    R pa[PA];
#pragma unroll
    for (int q = 0; q < PA; ++q) pa[q] = q < NA ? part[2 * KR + q] : R(0);
    const R ysum = rs_group<TC, PA>(pa, lg);
    if (k1 <= n - 3) {
      const int q = reduce_scatter_index<TC, PA>(lg);
      const int i = tr + TR * (KR + (q >> 1));
      if (reduce_scatter_writer<TC, PA>(lg) && q < NA && i > k1 && i < n) {
        if (q & 1)
          sm.y[nb][i].im = ysum;
        else
          sm.y[nb][i].re = ysum;
      }
    }
    __syncthreads();
  }

  template <int P>
  static __device__ __forceinline__ void phases(const int n, int& k, Regs& A, Smem& sm, R& tre,
                                                R& tim) {
    if constexpr (P < LC) {
      const int kend = (P + 1) * TC - 2 < n - 3 ? (P + 1) * TC - 2 : n - 3;
      for (; k <= kend; ++k) step<P>(n, k, A, sm, tre, tim);
      phases<P + 1>(n, k, A, sm, tre, tim);
    }
  }

  static __device__ __forceinline__ void run(const int n, Regs& A, Smem& sm,
                                             double* __restrict__ dg, double* __restrict__ e2g) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // v_{-1} = w_{-1} = 0; y buffers cleared (rows never written stay zero)
    for (int i = lane; i < NP; i += 64) {
      sm.vb[wave][1][i] = {R(0), R(0)};
      sm.wb[wave][i] = {R(0), R(0)};
    }
    for (int i = tid; i < 2 * NP; i += NT) sm.y[i / NP][i % NP] = {R(0), R(0)};
    {
      const int tr = tid / TC, tc = tid % TC;
      if (tc == 0) {
#pragma unroll
        for (int li = 0; li < LR; ++li) sm.col[0][tr + TR * li] = get(A, li, 0);
      }
    }
    __syncthreads();
    R tre = R(0), tim = R(0);
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
