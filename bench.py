"""Throughput of the traveling-cluster Monte Carlo sweep on one MI355X.

Headline workload: double-exchange model on a 32x32 periodic lattice (1,024
sites), 8x8 traveling cluster (128x128 complex Hermitian matrices), t = 1,
J_H = 8, J_AF = 0.05, mu = 0, T = 0.05, seed 11, random start, plain FP64 TCA.
A step is one Monte Carlo sweep: 1,024 updates in four quadrant blocks, each
block one batched cluster-solve launch (2 x 256 matrices), one eigenvalue
launch and the decision launches; sweeps are replayed from one captured HIP
graph.  The same workload is then run in mixed precision (FP32 reduction,
FP64 eigenvalues and log-sum), and the dF error of both against the FP64
oracle is measured at T = 0.02, 0.05 and 0.1.

Full form (printed under "full_form"): a 320x320 lattice (102,400 sites),
8x8 cluster, J_AF = 0.03, T annealed geometrically from 0.1 to 0.01 over 200
sweeps, delayed acceptance with the learned first stage and the mixed
reduction, against the plain FP64 sweep of the same lattice.  The surrogate
is trained first by the library's own kernels on exact dF data from annealing
chains of a 100x100 lattice.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (and matrix): 256 CU x 2.4 GHz x 128 flop/clk/CU
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector: 256 CU x 2.4 GHz x 256 flop/clk/CU
# HBM bytes per launch of each FP64 reduction variant the autotuner may pick at the headline
# workload, from the FETCH_SIZE / WRITE_SIZE counters of `bench.py --counter-run` (every
# variant runs there) scaled by the calibration transfers (FETCH_SIZE x 1.996, WRITE_SIZE x
# 1.0); re-measure whenever a kernel changes.
TRAFFIC_BYTES_FP64_REDUCE = {
    "fused 32x16 grid": 2.465e6,
    "two-pass 32x16 grid": 2.008e6,
    "fused 32x16 grid, rank-2 update on MFMA": 5.049e6,
    "split 32x16 grid": 2.334e6,
    "split 32x16 grid, rank-2 update on MFMA": 2.240e6,
    "split 32x16 grid, rank-2 update on MFMA and vector ALUs": 2.298e6,
    "split 32x16 grid, rank-2 update on MFMA, reflector on half the wavefronts": 2.266e6,
    "split 32x16 grid, reflector on half the wavefronts": 2.320e6,
}


def reduce_flops(n):
    """Algorithmic flops of reducing one n x n complex Hermitian matrix to
    real tridiagonal form: (16/3) n^3 (Hermitian matrix-vector product and
    rank-2 update, 8 real flops per complex multiply-add)."""
    return 16.0 / 3.0 * n ** 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=8)
    ap.add_argument("--no-full-form", action="store_true")
    ap.add_argument("--full-sweeps", type=int, default=200)
    ap.add_argument("--counter-run", action="store_true",
                    help="for hardware-counter runs: two FP64 sweeps of the headline workload, then "
                         "a 64 MiB fill and a 64 MiB sum whose byte counts calibrate FETCH_SIZE and "
                         "WRITE_SIZE; prints no JSON")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--sq-check-sweeps", type=int, default=40,
                    help="anneal length of the S(q) comparison of the two chains (0 = skip)")
    return ap.parse_args()


def dF_error(tca, otca, L, Lc, JAF, seed, T, precision, nsample=24):
    """Max relative/absolute dF error of the HIP path vs the FP64 oracle on a
    sample of one logged sweep (updates followed in order, sampled ones
    recomputed by the oracle), and the count of unflagged decision
    mismatches."""
    import numpy as np
    lat = tca.Lattice(L, Lc, seed=seed, JH=8.0, JAF=JAF, precision=precision)
    S0 = lat.spins()
    recs, _ = lat.sweep([T], log=True)
    lat.close()
    rng = np.random.default_rng(0)
    check = set(rng.choice(L * L, nsample, replace=False).tolist())
    prm = otca.Params(L=L, Lc=Lc, JH=8.0, JAF=JAF, seed=seed)
    log = [dict(site=int(r["site"]), dF=float(r["dF"]), accept=bool(r["accept"]),
                near=bool(r["flags"] & 1)) for r in recs]
    _, st = otca.replay_sweep(S0, prm, T, 0, log, check=check)
    return st["max_rel"], st["max_abs"], st["bad"]


def cpu_baseline(otca, L, Lc, JAF, seed, T, nsweeps):
    """The FP64 oracle's sequential sweep, single thread, on the same input."""
    from threadpoolctl import threadpool_limits
    prm = otca.Params(L=L, Lc=Lc, JH=8.0, JAF=JAF, seed=seed)
    S = otca.initial_spins(L, seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for sw in range(nsweeps):
            S, _ = otca.sweep_sequential(S, prm, T, sw)
        dt = time.perf_counter() - t0
    return L * L * nsweeps / dt, dt


def batched_uneven(tca, stream):
    """Uneven cluster sizes: 100x100 lattice, sizes drawn per update from
    {6x6, 8x8, 10x10} (n = 72, 128, 200), J_AF = 0.05, T = 0.05; one reduction
    launch per size class per block (largest first), graph-replayed sweeps."""
    out = {"workload": "100x100 lattice, cluster sizes {6,8,10} drawn per update, J_AF=0.05, T=0.05"}
    for name, prec in (("fp64", tca.TCA_FP64), ("mixed", tca.TCA_MIXED)):
        lat = tca.Lattice(100, 8, seed=21, JAF=0.05, precision=prec, Lc_classes=(6, 8, 10),
                          stream=stream)
        lat.sweep([0.05])
        t0 = time.perf_counter()
        _, st = lat.sweep([0.05] * 4)
        dt = time.perf_counter() - t0
        rep = lat.tuning_report()
        lat.close()
        prof = tca.Lattice(100, 8, seed=21, JAF=0.05, precision=prec, Lc_classes=(6, 8, 10),
                           flags=tca.TCA_FLAG_PROFILE, stream=stream)
        _, sp = prof.sweep([0.05] * 2)
        prof.close()
        out[name] = {"updates_per_s": st["updates"] / dt,
                     "ms_per_sweep": {"reduce_all_classes": sp["reduce_ms"] / 2,
                                      "eigenvalues": sp["eig_ms"] / 2, "decide": sp["decide_ms"] / 2},
                     "autotuner": rep.strip().splitlines()}
    return out


def full_form(tca, a, stream):
    """Surrogate + delayed acceptance + mixed precision vs plain FP64 on the
    320x320 annealing workload."""
    import numpy as np
    Lc, JAF, seed = 8, 0.03, 5
    t0 = time.perf_counter()
    # training data: exact dF of two annealing chains on a 100x100 lattice, T 0.2 -> 0.01
    nanneal = 60
    Ttrain = 0.2 * (0.01 / 0.2) ** (np.arange(nanneal) / (nanneal - 1))
    sg = tca.Surrogate(Lc, 256, seed=1, capacity=2 * nanneal * 100 * 100, stream=stream)
    for r in range(2):
        lat = tca.Lattice(100, Lc, seed=seed + r, JAF=JAF, precision=tca.TCA_MIXED, stream=stream)
        sg.collect(lat, Ttrain)
        lat.close()
    untrained = sg.train(0, holdout=0.1)
    for rep in range(4):
        res = sg.train(1000, batch=1024, lr=1e-3 if rep < 3 else 2e-4, holdout=0.1)
    t_train = time.perf_counter() - t0

    K = a.full_sweeps
    Ts = 0.1 * 10.0 ** (-np.arange(K) / max(1, K - 1))
    # delayed acceptance + mixed, the whole anneal (graph-replayed sweeps)
    da = tca.Lattice(320, Lc, seed=seed + 9, JAF=JAF, precision=tca.TCA_MIXED, stream=stream)
    da.attach(sg)
    t1 = time.perf_counter()
    _, st = da.sweep(Ts)
    dt_da = time.perf_counter() - t1
    upd_da = st["updates"] / dt_da
    # the same anneal once more with per-phase timing (not the timed run)
    prof = tca.Lattice(320, Lc, seed=seed + 9, JAF=JAF, precision=tca.TCA_MIXED,
                       flags=tca.TCA_FLAG_PROFILE, stream=stream)
    prof.attach(sg)
    _, sp = prof.sweep(Ts)
    prof.close()
    # plain FP64 throughput on the same lattice (every update solved exactly)
    plain = tca.Lattice(320, Lc, seed=seed + 9, JAF=JAF, stream=stream)
    plain.sweep([Ts[0]])
    t2 = time.perf_counter()
    _, sp64 = plain.sweep(Ts[:5])
    dt_plain = time.perf_counter() - t2
    upd_plain = sp64["updates"] / dt_plain
    plain.close()
    mixed = tca.Lattice(320, Lc, seed=seed + 9, JAF=JAF, precision=tca.TCA_MIXED, stream=stream)
    mixed.sweep([Ts[0]])
    t3 = time.perf_counter()
    _, spm = mixed.sweep(Ts[:5])
    upd_mixed = spm["updates"] / (time.perf_counter() - t3)
    mixed.close()
    out = {
        "workload": f"320x320 lattice, 8x8 cluster, J_AF={JAF}, T geometric 0.1 -> 0.01 over {K} sweeps",
        "updates_per_s_surrogate_mixed": upd_da,
        "updates_per_s_plain_fp64": upd_plain,
        "updates_per_s_plain_mixed": upd_mixed,
        "ratio_vs_plain_fp64": upd_da / upd_plain,
        "stage1_pass_rate": st["stage1_passed"] / st["updates"],
        "accept_rate": st["accepted"] / st["updates"],
        "stage2_reject_rate": 1.0 - st["accepted"] / max(1, st["stage1_passed"]),
        "phase_ms": {"surrogate": sp["surrogate_ms"], "reduce": sp["reduce_ms"],
                     "eigenvalues": sp["eig_ms"], "decide": sp["decide_ms"],
                     "total": sp["elapsed_ms"]},
        "surrogate": {"train_rows": sg.rows, "holdout_rmse_fp32": res["holdout_rmse_fp32"],
                      "holdout_rmse_bf16": res["holdout_rmse_bf16"],
                      "untrained_rmse_bf16": untrained["holdout_rmse_bf16"],
                      "collect_and_train_s": t_train},
    }
    # the second coupling of the workload, with the same surrogate (it predicts the
    # fermionic dF only, which J_AF does not enter)
    JAF2 = 0.08
    da2 = tca.Lattice(320, Lc, seed=seed + 10, JAF=JAF2, precision=tca.TCA_MIXED, stream=stream)
    da2.attach(sg)
    t4 = time.perf_counter()
    _, st2 = da2.sweep(Ts)
    upd_da2 = st2["updates"] / (time.perf_counter() - t4)
    da2.close()
    plain2 = tca.Lattice(320, Lc, seed=seed + 10, JAF=JAF2, stream=stream)
    plain2.sweep([Ts[0]])
    t5 = time.perf_counter()
    _, sp2 = plain2.sweep(Ts[:5])
    upd_plain2 = sp2["updates"] / (time.perf_counter() - t5)
    plain2.close()
    out["jaf_0.08"] = {"updates_per_s_surrogate_mixed": upd_da2,
                       "updates_per_s_plain_fp64": upd_plain2,
                       "ratio_vs_plain_fp64": upd_da2 / upd_plain2,
                       "stage1_pass_rate": st2["stage1_passed"] / st2["updates"],
                       "accept_rate": st2["accepted"] / st2["updates"]}
    # S(q) of the two chains after the same (shortened) anneal from the same start
    if a.sq_check_sweeps > 0:
        Kq = a.sq_check_sweeps
        Tq = 0.1 * 10.0 ** (-np.arange(Kq) / max(1, Kq - 1))
        ref = tca.Lattice(320, Lc, seed=seed + 11, JAF=JAF, stream=stream)
        ref.sweep(Tq)
        _, sq_ref, m_ref = ref.observables()
        ref.close()
        alt = tca.Lattice(320, Lc, seed=seed + 11, JAF=JAF, precision=tca.TCA_MIXED,
                          stream=stream)
        alt.attach(sg)
        alt.sweep(Tq)
        _, sq_alt, m_alt = alt.observables()
        alt.close()
        ia = np.unravel_index(np.argmax(sq_ref), sq_ref.shape)
        ib = np.unravel_index(np.argmax(sq_alt), sq_alt.shape)
        out["sq_check"] = {"anneal_sweeps": Kq,
                           "peak_q_plain_fp64": [int(ia[1]), int(ia[0])],
                           "peak_q_surrogate_mixed": [int(ib[1]), int(ib[0])],
                           "S_peak_plain_fp64": float(sq_ref.max()),
                           "S_peak_surrogate_mixed": float(sq_alt.max()),
                           "max_abs_dS_q": float(np.max(np.abs(sq_ref - sq_alt))),
                           "abs_m_plain_fp64": float(np.linalg.norm(m_ref)),
                           "abs_m_surrogate_mixed": float(np.linalg.norm(m_alt))}
    da.close()
    sg.close()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU "
              "sharding of the sweep is a design, not a build, here.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1502_07028_amd as tca
    from oracle import tca as otca

    L, Lc, JAF, T, seed = 32, 8, 0.05, 0.05, 11
    n = 2 * Lc * Lc
    h = L // 2
    torch.cuda.set_device(0)
    if a.counter_run:
        lat = tca.Lattice(L, Lc, seed=seed, JH=8.0, JAF=JAF)   # autotuned, as in the bench
        lat.sweep([T, T])
        lat.close()
        x = torch.ones(16 * 1024 * 1024, dtype=torch.float32, device="cuda")  # elementwise fill
        s = x.sum()
        torch.cuda.synchronize()
        print(f"counter run done ({float(s):.0f})", file=sys.stderr)
        return
    stream_obj = torch.cuda.Stream()
    stream = stream_obj.cuda_stream

    def timed(precision):
        lat = tca.Lattice(L, Lc, seed=seed, JH=8.0, JAF=JAF, precision=precision, stream=stream)
        lat.sweep([T] * a.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = lat.sweep([T] * a.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        report = lat.tuning_report()
        lat.close()
        # kernel durations: the same sweeps once more with HIP events around
        # every launch (on the library's stream)
        lat = tca.Lattice(L, Lc, seed=seed, JH=8.0, JAF=JAF, precision=precision,
                          flags=tca.TCA_FLAG_PROFILE, stream=stream)
        lat.sweep([T] * a.warmup)
        _, sp = lat.sweep([T] * min(a.steps, 50))
        lat.close()
        return dt, st, sp, report

    dt, st, sp, report = timed(tca.TCA_FP64)
    updates = a.steps * L * L
    value = updates / dt
    avg_reduce_s = sp["reduce_ms"] / max(1, sp["reduce_launches"]) * 1e-3
    flops_per_launch = 2 * h * h * reduce_flops(n)
    achieved = flops_per_launch / avg_reduce_s / 1e12

    dtm, stm, spm, report_m = timed(tca.TCA_MIXED)
    avg_reduce_m = spm["reduce_ms"] / max(1, spm["reduce_launches"]) * 1e-3
    errs = {}
    for Te in (0.02, 0.05, 0.1):
        r64 = dF_error(tca, otca, L, Lc, JAF, seed, Te, tca.TCA_FP64)
        rm = dF_error(tca, otca, L, Lc, JAF, seed, Te, tca.TCA_MIXED)
        errs[str(Te)] = {"fp64_rel": r64[0], "fp64_abs": r64[1], "fp64_decision_mismatches": r64[2],
                         "mixed_rel": rm[0], "mixed_abs": rm[1]}

    cpu = None
    if not a.no_cpu_baseline:
        v, secs = cpu_baseline(otca, L, Lc, JAF, seed, T, a.cpu_sweeps)
        cpu = {"value": v, "unit": "updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{a.cpu_sweeps} sequential sweep(s) ({a.cpu_sweeps * L * L} updates) of the "
                         f"same 32x32 / 8x8 workload from the same start, FP64 oracle with LAPACK "
                         f"eigenvalues, one thread, {secs:.1f} s"}

    ff = None if a.no_full_form else full_form(tca, a, stream)
    un = None if a.no_uneven else batched_uneven(tca, stream)

    chosen = report.strip().splitlines()[0].split("-> ")[-1]
    out = {
        "metric": "cluster diagonalizations & exact-equivalent MC updates/sec at 8×8 cluster; ΔF err",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "double-exchange 32x32 lattice, 8x8 traveling cluster (128x128 complex "
                               "Hermitian), t=1, J_H=8, J_AF=0.05, mu=0, T=0.05, plain FP64 TCA sweep",
                   "lattice": L, "cluster": Lc, "matrix_dim": n, "clusters_per_launch": h * h,
                   "parallelism": "single GPU, one workgroup per cluster matrix"},
        "diagonalizations_per_s": 2 * value,
        "dF_error": errs,
        "mixed": {"updates_per_s": updates / dtm,
                  "diagonalizations_per_s": 2 * updates / dtm,
                  "reduce_kernel_ms": avg_reduce_m * 1e3,
                  "eig_kernel_ms": spm["eig_ms"] / max(1, spm["eig_launches"]),
                  "reduce_roofline_frac_fp32_valu":
                      flops_per_launch / avg_reduce_m / 1e12 / PEAK_FP32_VALU_TFLOPS},
        "kernel_ms": {"reduce": avg_reduce_s * 1e3,
                      "eig": sp["eig_ms"] / max(1, sp["eig_launches"]),
                      "decide": sp["decide_ms"] / max(1, sp["decide_launches"])},
        "autotuner": report.strip().splitlines() + report_m.strip().splitlines(),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": TRAFFIC_BYTES_FP64_REDUCE.get(chosen),
                     "kernel": "cluster_block_reduce, n=128 FP64, autotuned: " + chosen,
                     "flops_per_launch": flops_per_launch},
        "cpu_baseline": cpu,
        "full_form": ff,
        "batched_uneven": un,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
