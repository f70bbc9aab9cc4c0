// Eigenvalues of a real symmetric tridiagonal matrix T (diagonal d, squared
// off-diagonal e2) and the fermionic grand potential of its spectrum, FP64.
//
// Sturm sequence.  The leading principal minors of T - x,
//   P_0 = 1,  P_1 = d_0 - x,  P_{i+1} = (d_i - x) P_i - e2_{i-1} P_{i-1},
// change sign exactly as often as T has eigenvalues below x (their ratios
// P_{i+1}/P_i are the pivots of the LDL^T factorization of T - x).  Each step
// costs one FMA on the critical path (the division of the pivot form is
// avoided); every eight steps the pair (P_i, P_{i-1}) is rescaled by an exact
// power of two so that it stays far from overflow and underflow, which changes
// no sign.  An exactly zero minor takes the sign of its zero bit, which yields
// the same total count as replacing a zero pivot by a tiny negative one.
//
// Search.  Eigenvalue j (ascending) is bracketed by bisection only until
// [a, b] holds eigenvalue j alone; then Laguerre steps on det(T - x) = P_n(x)
// finish it, P_n' and P_n'' coming from the recurrence differentiated once and
// twice.  Every evaluation also gives the Sturm count that keeps the bracket;
// an iterate leaving the bracket is replaced by the midpoint.  The iteration
// stops when its step is below the tolerance, or is small and fails to halve
// or leaves the bracket (the rounding noise of det(T - x) is reached); an
// eigenvalue that cannot be isolated (a cluster narrower than the tolerance)
// is finished by plain bisection.
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>

namespace tca {

__device__ __forceinline__ unsigned sign_change(double a, double b) {
  return (unsigned)(__double2hiint(a) ^ __double2hiint(b)) >> 31;
}

// power-of-two factor bringing a magnitude m >= 0 back into [2^-200, 2^200]
__device__ __forceinline__ double rescale_factor(double m) {
  return m > 0x1p200 ? 0x1p-200 : (m < 0x1p-200 && m > 0.0 ? 0x1p200 : 1.0);
}

constexpr int kSturmGroup = 8;  // steps between rescalings

// The sign bits of the minors enter a shift register, one funnel shift per
// step: bits = bits << 1 | sign(P_i).  The sign changes of a group of G steps
// are then the set bits of bits ^ (bits >> 1) in its low G positions (bit G
// holds the sign before the group).
__device__ __forceinline__ unsigned push_sign(unsigned bits, double p) {
  return __builtin_amdgcn_alignbit(bits, (unsigned)__double2hiint(p), 31);
}
template <int G>
__device__ __forceinline__ unsigned group_changes(unsigned bits) {
  return (unsigned)__builtin_popcount((bits ^ (bits >> 1)) & ((1u << G) - 1u));
}

// ---------------------------------------------------------------------------
// The same recurrences with the matrix staged in LDS as pairs
// de[i] = (d_i, e2_{i-1}) (e2_{-1} = 0): every lane reads the same pair, a
// broadcast LDS read that the compiler issues ahead of the dependent chain.
__device__ __forceinline__ int sturm_count_pairs(const int n, const double x,
                                                 const double2* de) {
  double pm = 1.0, p = de[0].x - x;
  unsigned bits = push_sign(0u, p);  // P_0 = 1 is positive
  unsigned c = bits & 1u;
  int i = 1;
  for (; i + kSturmGroup - 1 < n; i += kSturmGroup) {
    double2 q[kSturmGroup];
#pragma unroll
    for (int u = 0; u < kSturmGroup; ++u) q[u] = de[i + u];
#pragma unroll
    for (int u = 0; u < kSturmGroup; ++u) {
      const double pn = fma(q[u].x - x, p, -q[u].y * pm);
      bits = push_sign(bits, pn);
      pm = p;
      p = pn;
    }
    c += group_changes<kSturmGroup>(bits);
    const double f = rescale_factor(fmax(fabs(p), fabs(pm)));
    p *= f;
    pm *= f;
  }
  for (; i < n; ++i) {
    const double2 q = de[i];
    const double pn = fma(q.x - x, p, -q.y * pm);
    c += sign_change(pn, p);
    pm = p;
    p = pn;
  }
  return (int)c;
}

// Counts at M points at once: M independent chains interleaved step by step,
// which fills the latency of each chain's FMA with the others'.
template <int M>
__device__ __forceinline__ void sturm_count_pairs_multi(const int n, const double (&x)[M],
                                                        const double2* de, int (&cnt)[M]) {
  double pm[M], p[M];
  unsigned bits[M], c[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    pm[m] = 1.0;
    p[m] = de[0].x - x[m];
    bits[m] = push_sign(0u, p[m]);
    c[m] = bits[m] & 1u;
  }
  int i = 1;
  for (; i + kSturmGroup - 1 < n; i += kSturmGroup) {
    double2 q[kSturmGroup];
#pragma unroll
    for (int u = 0; u < kSturmGroup; ++u) q[u] = de[i + u];
#pragma unroll
    for (int u = 0; u < kSturmGroup; ++u) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const double pn = fma(q[u].x - x[m], p[m], -q[u].y * pm[m]);
        bits[m] = push_sign(bits[m], pn);
        pm[m] = p[m];
        p[m] = pn;
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      c[m] += group_changes<kSturmGroup>(bits[m]);
      const double f = rescale_factor(fmax(fabs(p[m]), fabs(pm[m])));
      p[m] *= f;
      pm[m] *= f;
    }
  }
  for (; i < n; ++i) {
    const double2 q = de[i];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const double pn = fma(q.x - x[m], p[m], -q.y * pm[m]);
      c[m] += sign_change(pn, p[m]);
      pm[m] = p[m];
      p[m] = pn;
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) cnt[m] = (int)c[m];
}

// Sturm count at x and the Laguerre step for det(T - x) = P_n(x), from P_n,
// P_n' and P_n'' (the recurrence differentiated twice:
// P''_{i+1} = -2 P'_i + (d_i - x) P''_i - e2_{i-1} P''_{i-1}).  With
// G = P'/P and H = G^2 - P''/P the step is n / (G +- sqrt((n-1)(n H - G^2))),
// the sign taken to make the denominator larger.  For a polynomial with real
// roots only the iteration converges from any start and cubically near a
// simple root, where the step tends to the Newton step P/P'.
__device__ __forceinline__ int sturm_laguerre_pairs(const int n, const double x,
                                                    const double2* de, double* step) {
  double pm = 1.0, p = de[0].x - x;
  double qm = 0.0, q = -1.0;  // first derivatives
  double rm = 0.0, r = 0.0;   // second derivatives
  unsigned bits = push_sign(0u, p);
  unsigned c = bits & 1u;
  int i = 1;
  for (; i + kSturmGroup - 1 < n; i += kSturmGroup) {
    double2 v[kSturmGroup];
#pragma unroll
    for (int u = 0; u < kSturmGroup; ++u) v[u] = de[i + u];
#pragma unroll
    for (int u = 0; u < kSturmGroup; ++u) {
      const double dx = v[u].x - x, e = v[u].y;
      const double pn = fma(dx, p, -e * pm);
      const double qn = fma(dx, q, -fma(e, qm, p));
      const double rn = fma(dx, r, -fma(e, rm, 2.0 * q));
      bits = push_sign(bits, pn);
      pm = p;
      p = pn;
      qm = q;
      q = qn;
      rm = r;
      r = rn;
    }
    c += group_changes<kSturmGroup>(bits);
    const double f = rescale_factor(fmax(fmax(fmax(fabs(p), fabs(pm)), fmax(fabs(q), fabs(qm))),
                                         fmax(fabs(r), fabs(rm))));
    p *= f;
    pm *= f;
    q *= f;
    qm *= f;
    r *= f;
    rm *= f;
  }
  for (; i < n; ++i) {
    const double dx = de[i].x - x, e = de[i].y;
    const double pn = fma(dx, p, -e * pm);
    const double qn = fma(dx, q, -fma(e, qm, p));
    const double rn = fma(dx, r, -fma(e, rm, 2.0 * q));
    c += sign_change(pn, p);
    pm = p;
    p = pn;
    qm = q;
    q = qn;
    rm = r;
    r = rn;
  }
  if (p == 0.0) {
    *step = 0.0;  // x is an eigenvalue
  } else {
    const double nd = (double)n, G = q / p, H = G * G - r / p;
    const double s = sqrt(fmax((nd - 1.0) * (nd * H - G * G), 0.0));
    const double den = fabs(G + s) >= fabs(G - s) ? G + s : G - s;
    *step = nd / den;  // den == 0 gives an infinite step, which the bracket rejects
  }
  return (int)c;
}

constexpr double kLastStep = 2.25e6;  // ~1e-9 / (2 eps)

// Eigenvalue j of T from a bracket [a, b] with counts ca <= j < cb.
__device__ inline double tri_eigenvalue_pairs(const int n, const int j, const double2* de,
                                              double a, double b, int ca, int cb,
                                              const double tol) {
  while (b - a > tol) {
    if (ca == j && cb == j + 1) break;
    const double mid = 0.5 * (a + b);
    if (mid <= a || mid >= b) break;
    const int c = sturm_count_pairs(n, mid, de);
    if (c > j) {
      b = mid;
      cb = c;
    } else {
      a = mid;
      ca = c;
    }
  }
  if (b - a <= tol) return 0.5 * (a + b);
  double x = 0.5 * (a + b);
  double last = b - a;
  for (int it = 0; it < 12; ++it) {
    double step;
    const int c = sturm_laguerre_pairs(n, x, de, &step);
    if (c > j)
      b = x;
    else
      a = x;
    if (b - a <= tol) return 0.5 * (a + b);
    double xn = x - step;
    const bool inside = xn > a && xn < b;
    const double st = fabs(step);
    if (st <= tol) return xn;
    // near a simple root the error after a step of size st is of order
    // st^3 / (root spacing)^2 (at most st^2 / spacing, as for Newton): a step
    // below ~1e-9 of the spectral scale (tol is 2 eps of it) leaves an error
    // far below tol, so it is the last one
    if (inside && st <= kLastStep * tol) return xn;
    if (st <= 1e5 * tol && (st > 0.5 * last || !inside)) return x;
    if (!inside) xn = 0.5 * (a + b);
    last = inside ? st : b - a;
    x = xn;
  }
  while (b - a > tol) {
    const double mid = 0.5 * (a + b);
    if (mid <= a || mid >= b) break;
    if (sturm_count_pairs(n, mid, de) > j)
      b = mid;
    else
      a = mid;
  }
  return 0.5 * (a + b);
}

// Grand potential term of one level: min(x,0) - T log1p(exp(-|x|/T)), x = eps - mu.
__device__ __forceinline__ double omega_term(const double eps, const double T, const double mu) {
  const double x = eps - mu;
  return fmin(x, 0.0) - T * log1p(exp(-fabs(x) / T));
}

}  // namespace tca
