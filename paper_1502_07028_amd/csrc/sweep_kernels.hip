// Kernels of a sweep around the cluster solves:
//  decide_kernel,
//  decide_wave_kernel  Metropolis decisions of one parallel block in an order
//                    equivalent to the sequential sweep (Sec. II(c) steps
//                    (e)-(f)), committing accepted spins;
//  classify_kernel   per-update cluster size classes of one block;
//  init / S(q)       initial spins and the structure factor of Eq. (2).
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "rng.hpp"

namespace tca {

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

// Metropolis decisions of block K, in two kernels.
//
// decide_prep_kernel (one thread per cluster, fully parallel): everything of
// an update that does not depend on earlier decisions of the block -- the
// Metropolis uniforms, the proposal, dF = F_new - F_old, ln u and the
// surrogate terms -- into one record per cluster.
//
// decide_kernel (one workgroup): the decisions themselves.  Each cluster's dF
// came from the block-start state, which equals the state the sequential
// sweep would have shown it (no cluster of a block contains a site visited
// earlier in that block).  The classical term reads the -x and -y lattice
// neighbours, which may belong to the same block and be decided earlier in
// raster order, so with J_AF != 0 the sites are processed by anti-diagonals
// i + j = const of the block: every site is decided after both of those
// neighbours, exactly as in the sequential order.  With J_AF == 0 all
// decisions are independent.
//
// With delayed acceptance (pass != nullptr) only clusters that passed the
// surrogate stage were solved exactly; the others are rejected, and a passing
// one is accepted iff ln u < -dE/T + min(0, -dS_r/T) - min(0, -dS_f/T)
// (Christen & Fox), dS_f/dS_r the surrogate on the move and its reverse.
struct DecidePrep {
  double sn[3];     // proposal
  double dF;        // F_new - F_old (NaN when stage 1 rejected)
  double u, lnu;    // Metropolis uniform and its logarithm (lnu unused when u == 0)
  double sa, sb;    // min(0, -dS_r/T), min(0, -dS_f/T)
  float dSf, dSr;
  int16_t Lc;
  uint8_t flags;    // bit 1: reached the exact stage; bit 2: stage 1 near threshold
  uint8_t pad[5];
};

__global__ __launch_bounds__(256) void decide_prep_kernel(const double* __restrict__ Fpair,
                                                          BlockGeom g, ModelParams m, SweepRef sr,
                                                          int Lc_fixed, int4 classes,
                                                          int n_classes,
                                                          const uint8_t* __restrict__ pass,
                                                          const float* __restrict__ dS,
                                                          DecidePrep* __restrict__ prep) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.h * g.h) return;
  const uint64_t sweep = sr.sweep();
  const double T = sr.T();
  const int site = (g.x0 + c % g.h) + g.L * (g.y0 + c / g.h);
  const U64x4 r = philox4x64_10(m.seed, 0, sweep, site, kStreamMetropolis, 0);
  DecidePrep q;
  q.u = u53(r.w0);
  q.lnu = q.u > 0.0 ? log(q.u) : 0.0;
  const bool stage1 = (pass == nullptr) || (pass[c] != 0);
  bool near1 = false;
  q.dSf = q.dSr = 0.0f;
  q.sa = q.sb = 0.0;
  if (pass != nullptr) {
    q.dSf = dS[2 * c];
    q.dSr = dS[2 * c + 1];
    q.sa = fmin(0.0, -(double)q.dSr / T);
    q.sb = fmin(0.0, -(double)q.dSf / T);
    const double u1 = u53(r.w1);
    if (u1 > 0.0)
      near1 = fabs(T * (log(u1) - fmin(0.0, -(double)q.dSf / T))) <=
              1e-9 * fmax(fabs((double)q.dSf), 1e-3);
  }
  q.dF = __builtin_nan("");
  q.sn[0] = q.sn[1] = 0.0;
  q.sn[2] = 1.0;
  if (stage1) {
    sphere_point(m.seed, sweep, site, kStreamProposal, q.sn);
    q.dF = Fpair[2 * c + 1] - Fpair[2 * c];
  }
  int Lc = Lc_fixed;
  if (n_classes > 0) {
    const int k = size_class(m.seed, sweep, site, n_classes);
    Lc = k == 0 ? classes.x : k == 1 ? classes.y : k == 2 ? classes.z : classes.w;
  }
  q.Lc = (int16_t)Lc;
  q.flags = (uint8_t)((stage1 ? 2 : 0) | (near1 ? 4 : 0));
  prep[c] = q;
}

// Metropolis decision from the energy change dE of a stage-1 survivor.
// Plain chain: accept iff dE <= 0 or u < exp(-dE/T).  Delayed acceptance:
// accept iff ln u < -dE/T + sa - sb (the second-stage ratio).  Away from the
// threshold the decision is taken from ln u against -dE * (1/T): the two sides
// then differ by far more than the rounding of the logarithm, the exponential
// and the quotient, so the result is the one of the exact form, which is
// evaluated only within a relative band gap (kDecideGap = 1e-10; infinite
// with TCA_FLAG_EXACT_METROPOLIS) of the threshold.
__device__ __forceinline__ bool metropolis_accept(const double u, const double lnu,
                                                  const double sa, const double sb,
                                                  const double dE, const double T,
                                                  const double invT, const bool da,
                                                  const double gap_rel) {
  if (!da) {
    if (dE <= 0.0) return true;
    if (!(u > 0.0)) return u < exp(-dE / T);
    const double z = -dE * invT;
    const double gap = lnu - z, tol = gap_rel * (1.0 + fabs(z));
    return gap < -tol ? true : (gap > tol ? false : u < exp(-dE / T));
  }
  if (u <= 0.0) return true;
  const double z = fma(-dE, invT, sa - sb);
  const double gap = lnu - z;
  const double tol = gap_rel * (1.0 + fabs(dE * invT) + fabs(sa) + fabs(sb));
  return gap < -tol ? true : (gap > tol ? false : lnu < -dE / T + sa - sb);
}

// Near-threshold flag: |T ln u + dE| (delayed acceptance: T |ln u - rhs|)
// below 1e-9 of max(|dE|, 1e-3).
__device__ __forceinline__ bool metropolis_near(const double u, const double lnu,
                                                const double sa, const double sb,
                                                const double dE, const double T,
                                                const bool da) {
  if (!(u > 0.0)) return false;
  if (!da) return fabs(dE + T * lnu) <= 1e-9 * fmax(fabs(dE), 1e-3);
  const double rhs = -dE / T + sa - sb;
  return fabs(T * (lnu - rhs)) <= 1e-9 * fmax(fabs(dE), 1e-3);
}

__device__ __forceinline__ bool metropolis_decide(const DecidePrep& pr, const double dE,
                                                  const double T, const double invT,
                                                  const bool da, const double gap_rel, bool& near) {
  near = metropolis_near(pr.u, pr.lnu, pr.sa, pr.sb, dE, T, da);
  return metropolis_accept(pr.u, pr.lnu, pr.sa, pr.sb, dE, T, invT, da, gap_rel);
}

// Adds the wavefront total of a per-thread count to *p with one atomic from
// lane 0 (every lane of the wavefront takes part).
__device__ __forceinline__ void add_wave_total(unsigned long long* p, unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v != 0u) atomicAdd(p, (unsigned long long)v);
}

__global__ __launch_bounds__(1024) void decide_kernel(double* S, BlockGeom g, ModelParams m,
                                                      SweepRef sr, int K, bool da,
                                                      const DecidePrep* __restrict__ prep,
                                                      tca_update_record* __restrict__ log_base,
                                                      unsigned long long* __restrict__ counters) {
  const int h = g.h, L = g.L;
  const double T = sr.T(), invT = 1.0 / T;
  tca_update_record* logbuf =
      log_base != nullptr ? log_base + (size_t)sr.s() * (size_t)L * (size_t)L : nullptr;
  const bool wave = (m.JAF != 0.0);
  const int ndiag = wave ? 2 * h - 1 : 1;
  unsigned nacc = 0, nnear = 0, npass = 0;
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
      const DecidePrep pr = prep[c];
      const bool stage1 = (pr.flags & 2) != 0;
      double dE = __builtin_nan("");
      bool acc = false, near = false;
      if (stage1) {
        dE = pr.dF + classical_delta(S, L, px, py, pr.sn, m.JAF);
        acc = metropolis_decide(pr, dE, T, invT, da, m.decide_gap, near);
        if (acc) {
          S[3 * site + 0] = pr.sn[0];
          S[3 * site + 1] = pr.sn[1];
          S[3 * site + 2] = pr.sn[2];
        }
      }
      nacc += acc;
      nnear += near;
      npass += stage1;
      if (logbuf != nullptr) {
        tca_update_record rec;
        rec.site = site;
        rec.Lc = pr.Lc;
        rec.accept = acc ? 1 : 0;
        rec.flags = (uint8_t)((near ? 1 : 0) | pr.flags);
        rec.dF = pr.dF;
        rec.dE = dE;
        rec.u = pr.u;
        rec.dS_f = pr.dSf;
        rec.dS_r = pr.dSr;
        logbuf[(size_t)K * h * h + c] = rec;
      }
    }
    if (wave) __syncthreads();
  }
  add_wave_total(&counters[0], nacc);
  add_wave_total(&counters[1], nnear);
  add_wave_total(&counters[3], npass);
  if (threadIdx.x == 0) atomicAdd(&counters[2], (unsigned long long)(h * h));
}

// The classical term from the four neighbour spins (-x, +x, -y, +y), the
// site's spin s and the proposal sn, in the operation order of
// classical_delta (every operation rounded on its own).
__device__ __forceinline__ double classical_term(const double* a, const double* b, const double* c,
                                                 const double* d, const double* s,
                                                 const double* sn, double JAF) {
#pragma clang fp contract(off)
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

// Anti-diagonal decision pass for J_AF != 0 and blocks of side h <= 512:
// the same decisions as decide_kernel, with the state the pass creates kept
// on chip.  Site (i, j) of anti-diagonal d = i + j needs the final spins of
// (i-1, j) and (i, j-1), both on anti-diagonal d-1, which the previous
// iteration left in LDS; its own spin, the +x and +y neighbours (decided only
// later) and neighbours outside the block still hold their block-start values
// and, with the per-cluster record, are read from memory one anti-diagonal
// ahead, so the global-memory latency stays off the sequential chain.
constexpr int kWaveMaxH = 512;  // one thread per site of an anti-diagonal

struct WaveSite {
  DecidePrep pr;
  double s[3], xm[3], xp[3], ym[3], yp[3];
  int i, j, c, site;
  bool valid;
};

__device__ __forceinline__ void wave_fetch(const double* S, const BlockGeom& g,
                                           const DecidePrep* __restrict__ prep, int dd,
                                           WaveSite& w) {
  const int h = g.h, L = g.L;
  const int lo = max(0, dd - (h - 1));
  const int cnt = min(dd, h - 1) - lo + 1;
  w.valid = (int)threadIdx.x < cnt;
  if (!w.valid) return;
  w.i = lo + (int)threadIdx.x;
  w.j = dd - w.i;
  w.c = w.i + h * w.j;
  const int px = g.x0 + w.i, py = g.y0 + w.j;
  w.site = px + L * py;
  w.pr = prep[w.c];
  const int xm = (px + L - 1) % L, xp = (px + 1) % L, ym = (py + L - 1) % L, yp = (py + 1) % L;
  for (int k = 0; k < 3; ++k) {
    w.s[k] = S[3 * w.site + k];
    w.xp[k] = S[3 * (xp + L * py) + k];
    w.yp[k] = S[3 * (px + L * yp) + k];
    w.xm[k] = w.i == 0 ? S[3 * (xm + L * py) + k] : 0.0;
    w.ym[k] = w.j == 0 ? S[3 * (px + L * ym) + k] : 0.0;
  }
}

__global__ __launch_bounds__(kWaveMaxH) void decide_wave_kernel(
    double* S, BlockGeom g, ModelParams m, SweepRef sr, int K, bool da,
    const DecidePrep* __restrict__ prep, tca_update_record* __restrict__ log_base,
    unsigned long long* __restrict__ counters) {
  __shared__ double fin[2][kWaveMaxH][3];  // final spins of an anti-diagonal, by row i
  const int h = g.h, L = g.L;
  const double T = sr.T(), invT = 1.0 / T;
  tca_update_record* logbuf =
      log_base != nullptr ? log_base + (size_t)sr.s() * (size_t)L * (size_t)L : nullptr;
  unsigned nacc = 0, nnear = 0, npass = 0;
  const int nd = 2 * h - 1;
  // anti-diagonal dd from cur, while the loads of dd + 1 into nxt are in flight
  auto diagonal = [&](const int dd, const WaveSite& cur, WaveSite& nxt) {
    if (dd + 1 < nd) wave_fetch(S, g, prep, dd + 1, nxt);
    if (cur.valid) {
      const double(*prev)[3] = fin[(dd + 1) & 1];  // anti-diagonal dd - 1
      double a[3], c[3];
      for (int k = 0; k < 3; ++k) {
        a[k] = cur.i > 0 ? prev[cur.i - 1][k] : cur.xm[k];
        c[k] = cur.j > 0 ? prev[cur.i][k] : cur.ym[k];
      }
      const DecidePrep& pr = cur.pr;
      const bool stage1 = (pr.flags & 2) != 0;
      double dE = __builtin_nan("");
      bool acc = false, near = false;
      if (stage1) {
        dE = pr.dF + classical_term(a, cur.xp, c, cur.yp, cur.s, pr.sn, m.JAF);
        acc = metropolis_decide(pr, dE, T, invT, da, m.decide_gap, near);
      }
      for (int k = 0; k < 3; ++k) fin[dd & 1][cur.i][k] = acc ? pr.sn[k] : cur.s[k];
      if (acc) {
        S[3 * cur.site + 0] = pr.sn[0];
        S[3 * cur.site + 1] = pr.sn[1];
        S[3 * cur.site + 2] = pr.sn[2];
      }
      nacc += acc;
      nnear += near;
      npass += stage1;
      if (logbuf != nullptr) {
        tca_update_record rec;
        rec.site = cur.site;
        rec.Lc = pr.Lc;
        rec.accept = acc ? 1 : 0;
        rec.flags = (uint8_t)((near ? 1 : 0) | pr.flags);
        rec.dF = pr.dF;
        rec.dE = dE;
        rec.u = pr.u;
        rec.dS_f = pr.dSf;
        rec.dS_r = pr.dSr;
        logbuf[(size_t)K * h * h + cur.c] = rec;
      }
    }
    // a barrier that orders the LDS only: the global loads of the next
    // anti-diagonal stay in flight (no global location is written and read
    // within the pass)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  };
  // two site buffers used alternately, so no copy waits for loads in flight
  WaveSite w0, w1;
  wave_fetch(S, g, prep, 0, w0);
  for (int dd = 0; dd < nd; dd += 2) {
    diagonal(dd, w0, w1);
    if (dd + 1 < nd) diagonal(dd + 1, w1, w0);
  }
  add_wave_total(&counters[0], nacc);
  add_wave_total(&counters[1], nnear);
  add_wave_total(&counters[3], npass);
  if (threadIdx.x == 0) atomicAdd(&counters[2], (unsigned long long)(h * h));
}

// The same pass for blocks of side h <= kStageMaxH, by one wavefront with the
// whole block staged in LDS first: the per-cluster records and the spins of
// the block and its one-site frame, (h + 2)^2 sites read once with every load
// in flight together.  The staged spins are then the state of the pass: site
// (i, j) sits at frame position (i + 1, j + 1), its decision overwrites it, and
// its four neighbours are read from the frame, where the -x and -y ones (or
// the frame's fixed edge) already hold their final values and the +x and +y
// ones still hold their block-start values, which is the order of the
// sequential sweep.  The sequential loop carries only what the next
// anti-diagonal needs (the operands of anti-diagonal d + 1 that the pass does
// not change are read while d is decided); decisions and dE go to LDS, and the
// spin writes, flags, records and counters follow in a parallel pass over the
// block.  No global memory is read after the staging.
constexpr int kStageMaxH = 24;  // 80 h^2 + 24 (h + 2)^2 + 9 h^2 bytes of LDS <= 66 KB

static size_t decide_stage_lds_bytes(int h) {
  const size_t hh = (size_t)h * h, hf2 = (size_t)(h + 2) * (h + 2);
  return sizeof(DecidePrep) * hh + 3 * sizeof(double) * hf2 + sizeof(double) * hh + hh;
}

// Operands of one site of an anti-diagonal that the pass leaves unchanged.
struct StageSite {
  double dF, u, lnu, sa, sb, sn[3], s0[3], xp[3], yp[3];
  int f, c;
  bool on, stage1;
};

__global__ __launch_bounds__(64) void decide_stage_kernel(
    double* S, BlockGeom g, ModelParams m, SweepRef sr, int K, bool da,
    const DecidePrep* __restrict__ prep, tca_update_record* __restrict__ log_base,
    unsigned long long* __restrict__ counters) {
  extern __shared__ double stage_lds[];
  constexpr int PW = (int)(sizeof(DecidePrep) / sizeof(double));
  static_assert(sizeof(DecidePrep) % sizeof(double) == 0, "records are whole doubles");
  const int h = g.h, L = g.L, hf = h + 2, hh = h * h, lane = threadIdx.x;
  DecidePrep* pl = reinterpret_cast<DecidePrep*>(stage_lds);
  double* fr = stage_lds + PW * hh;     // frame spins, 3 per site
  double* dEs = fr + 3 * hf * hf;       // dE per site
  uint8_t* accb = reinterpret_cast<uint8_t*>(dEs + hh);  // decision per site
  {
    // batches of loads issued together, so the staging costs a few memory
    // latencies rather than one per element
    constexpr int BF = 8, BP = 16;
    for (int f0 = 0; f0 < hf * hf; f0 += 64 * BF) {
      double v[BF][3];
#pragma unroll
      for (int u = 0; u < BF; ++u) {
        const int f = f0 + lane + 64 * u;
        const int px = (g.x0 + f % hf - 1 + L) % L, py = (g.y0 + f / hf - 1 + L) % L;
        const double* sp = S + 3 * (px + L * py);
#pragma unroll
        for (int k = 0; k < 3; ++k) v[u][k] = f < hf * hf ? sp[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BF; ++u) {
        const int f = f0 + lane + 64 * u;
        if (f < hf * hf) {
#pragma unroll
          for (int k = 0; k < 3; ++k) fr[3 * f + k] = v[u][k];
        }
      }
    }
    const double* src = reinterpret_cast<const double*>(prep);
    const int nw = PW * hh;
    for (int w0 = 0; w0 < nw; w0 += 64 * BP) {
      double v[BP];
#pragma unroll
      for (int u = 0; u < BP; ++u) {
        const int w = w0 + lane + 64 * u;
        v[u] = w < nw ? src[w] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BP; ++u) {
        const int w = w0 + lane + 64 * u;
        if (w < nw) stage_lds[w] = v[u];
      }
    }
  }
  __syncthreads();
  const double T = sr.T(), invT = 1.0 / T;
  const int nd = 2 * h - 1;
  auto fetch = [&](const int dd, StageSite& st) {
    const int lo = max(0, dd - (h - 1));
    const int cnt = min(dd, h - 1) - lo + 1;
    st.on = dd < nd && lane < cnt;
    if (!st.on) return;
    const int i = lo + lane, j = dd - i;
    st.c = i + h * j;
    st.f = (i + 1) + hf * (j + 1);
    const DecidePrep& pr = pl[st.c];
    st.stage1 = (pr.flags & 2) != 0;
    st.dF = pr.dF;
    st.u = pr.u;
    st.lnu = pr.lnu;
    st.sa = pr.sa;
    st.sb = pr.sb;
    for (int k = 0; k < 3; ++k) {
      st.sn[k] = pr.sn[k];
      st.s0[k] = fr[3 * st.f + k];
      st.xp[k] = fr[3 * (st.f + 1) + k];
      st.yp[k] = fr[3 * (st.f + hf) + k];
    }
  };
  // anti-diagonal dd from cur; the unchanged operands of dd + 1 go to nxt
  auto diagonal = [&](const int dd, const StageSite& cur, StageSite& nxt) {
    if (cur.on) {
      double a[3], b[3];
      for (int k = 0; k < 3; ++k) {
        a[k] = fr[3 * (cur.f - 1) + k];
        b[k] = fr[3 * (cur.f - hf) + k];
      }
      double dE = __builtin_nan("");
      bool acc = false;
      if (cur.stage1) {
        dE = cur.dF + classical_term(a, cur.xp, b, cur.yp, cur.s0, cur.sn, m.JAF);
        acc = metropolis_accept(cur.u, cur.lnu, cur.sa, cur.sb, dE, T, invT, da, m.decide_gap);
      }
      if (acc) {
        for (int k = 0; k < 3; ++k) fr[3 * cur.f + k] = cur.sn[k];
      }
      dEs[cur.c] = dE;
      accb[cur.c] = acc ? 1 : 0;
    }
    fetch(dd + 1, nxt);
    // the next anti-diagonal reads this one's frame entries: order the LDS only
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  };
  StageSite w0, w1;
  fetch(0, w0);
  for (int dd = 0; dd < nd; dd += 2) {
    diagonal(dd, w0, w1);
    if (dd + 1 < nd) diagonal(dd + 1, w1, w0);
  }
  // spins, flags, records and counters of the whole block
  tca_update_record* logbuf =
      log_base != nullptr ? log_base + (size_t)sr.s() * (size_t)L * (size_t)L : nullptr;
  unsigned nacc = 0, nnear = 0, npass = 0;
  for (int c = lane; c < hh; c += 64) {
    const DecidePrep& pr = pl[c];
    const bool stage1 = (pr.flags & 2) != 0, acc = accb[c] != 0;
    const double dE = dEs[c];
    const bool near = stage1 && metropolis_near(pr.u, pr.lnu, pr.sa, pr.sb, dE, T, da);
    const int site = (g.x0 + c % h) + L * (g.y0 + c / h);
    if (acc) {
      for (int k = 0; k < 3; ++k) S[3 * site + k] = pr.sn[k];
    }
    nacc += acc;
    nnear += near;
    npass += stage1;
    if (logbuf != nullptr) {
      tca_update_record rec;
      rec.site = site;
      rec.Lc = pr.Lc;
      rec.accept = acc ? 1 : 0;
      rec.flags = (uint8_t)((near ? 1 : 0) | pr.flags);
      rec.dF = pr.dF;
      rec.dE = dE;
      rec.u = pr.u;
      rec.dS_f = pr.dSf;
      rec.dS_r = pr.dSr;
      logbuf[(size_t)K * h * h + c] = rec;
    }
  }
  add_wave_total(&counters[0], nacc);
  add_wave_total(&counters[1], nnear);
  add_wave_total(&counters[3], npass);
  if (lane == 0) atomicAdd(&counters[2], (unsigned long long)(h * h));
}

__global__ void classify_kernel(int4 classes, int n_classes, BlockGeom g, uint64_t seed,
                                SweepRef sr, int32_t* __restrict__ count,
                                int32_t* __restrict__ list) {
  const int hh = g.h * g.h;
  const uint64_t sweep = sr.sweep();
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

static int4 pack_classes(const int32_t* c, int n) {
  int4 r = make_int4(0, 0, 0, 0);
  if (n > 0) r.x = c[0];
  if (n > 1) r.y = c[1];
  if (n > 2) r.z = c[2];
  if (n > 3) r.w = c[3];
  return r;
}

hipError_t launch_classify(const int32_t* classes_Lc, int n_classes, BlockGeom g, uint64_t seed,
                           SweepRef sr, ClassLists cl, hipStream_t st) {
  const int hh = g.h * g.h;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, cl.count, 4);
  hipLaunchKernelGGL(classify_kernel, dim3((hh + 255) / 256), dim3(256), 0, st,
                     pack_classes(classes_Lc, n_classes), n_classes, g, seed, sr, cl.count,
                     cl.list);
  return hipGetLastError();
}

hipError_t launch_decide(double* S, const double* Fpair, BlockGeom g, ModelParams m, SweepRef sr,
                         int Lc_fixed, const int32_t* classes_Lc, int n_classes, int K,
                         const uint8_t* pass, const float* dS, void* prep_buf,
                         tca_update_record* log_base, unsigned long long* counters,
                         hipStream_t st) {
  DecidePrep* prep = (DecidePrep*)prep_buf;
  const int hh = g.h * g.h;
  hipLaunchKernelGGL(decide_prep_kernel, dim3((hh + 255) / 256), dim3(256), 0, st, Fpair, g, m, sr,
                     Lc_fixed, pack_classes(classes_Lc, n_classes), n_classes, pass, dS, prep);
  if (m.JAF != 0.0 && g.h <= kStageMaxH)
    hipLaunchKernelGGL(decide_stage_kernel, dim3(1), dim3(64), decide_stage_lds_bytes(g.h), st, S,
                       g, m, sr, K, pass != nullptr, (const DecidePrep*)prep, log_base, counters);
  else if (m.JAF != 0.0 && g.h <= kWaveMaxH)
    hipLaunchKernelGGL(decide_wave_kernel, dim3(1), dim3(kWaveMaxH), 0, st, S, g, m, sr, K,
                       pass != nullptr, (const DecidePrep*)prep, log_base, counters);
  else
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(1024), 0, st, S, g, m, sr, K, pass != nullptr,
                       (const DecidePrep*)prep, log_base, counters);
  return hipGetLastError();
}

size_t decide_prep_bytes(int clusters) { return sizeof(DecidePrep) * (size_t)clusters; }

__global__ void advance_kernel(int32_t* idx) { *idx += 1; }

hipError_t launch_advance(int32_t* idx, hipStream_t st) {
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(1), 0, st, idx);
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

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace tca
