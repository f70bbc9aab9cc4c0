"""Sequential TCA Monte Carlo sweep, its block-batched equivalent, and the
replay used to check a logged GPU trajectory update by update.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. II(c) (Fig. 2 flowchart): for each update site, read the cluster
spins from S, build and diagonalize the cluster Hamiltonian, randomly modify
the spin at the update site, rebuild and re-diagonalize, decide by Metropolis,
and write the new spin into S if accepted.  Sites are visited in the order of
the parallel scheme of Sec. III(a): the four quadrant blocks in turn, raster
order inside each block.

Readings of what the paper leaves open:
* Energy of a cluster (the paper speaks of energy differences, Sec. II(a), and
  of a grand-canonical cluster, Sec. II(b)): the fermionic grand potential
  F = -T sum_i ln(1 + exp(-(eps_i - mu)/T)), evaluated in the overflow-free
  form  sum_i [min(x_i, 0) - T log1p(exp(-|x_i|/T))],  x_i = eps_i - mu.
  The Monte Carlo temperature and the fermion temperature are the same T.
* Two diagonalizations per update (old and new cluster matrix).
* dE = (F_new - F_old) + J_AF (s' - S_p) . (sum of the four lattice
  neighbours of p in the current state).
* Metropolis: accept iff dE <= 0 or u < exp(-dE/T).
* Near-threshold flag: |dE - (-T ln u)| <= tau, tau = rel_tau*max(|dE|, 1e-3)
  (rel_tau = 1e-9 for FP64 parity).  A flagged update is one whose decision
  may legitimately differ between two correct implementations.
* Error measure for dF: |dF_a - dF_b| / max(|dF_b|, 1e-3 t).

Pinned by: closed-form F of the ferromagnet, antisymmetry dF(C->C') =
-dF(C'->C), rotation invariance, dF == 0 exactly when t == 0 or J_H == 0
(reduction to the classical Heisenberg Metropolis), sequential == block-batched
(bitwise), and exact enumeration of the stationary law on a 2x2 lattice with
flip-only proposals.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import model, sampling
from .eigen import eigvals_lapack


@dataclass
class Params:
    L: int
    Lc: int
    t: float = 1.0
    JH: float = 8.0
    JAF: float = 0.0
    mu: float = 0.0
    seed: int = 1
    Lc_classes: tuple = field(default_factory=tuple)   # non-empty -> size drawn per update

    def cluster_size(self, sweep: int, site: int) -> int:
        if self.Lc_classes:
            k = sampling.size_class(self.seed, sweep, site, len(self.Lc_classes))
            return int(self.Lc_classes[k])
        return int(self.Lc)


def free_energy(eigs, T: float, mu: float) -> float:
    """Fermionic grand potential of one spectrum, plain left-to-right sum over
    the ascending eigenvalues."""
    F = 0.0
    for e in np.asarray(eigs, dtype=np.float64):
        x = float(e) - mu
        F += min(x, 0.0) - T * math.log1p(math.exp(-abs(x) / T))
    return F


def near_threshold(dE: float, u: float, T: float, rel_tau: float) -> bool:
    if u <= 0.0:
        return False
    thr = -T * math.log(u)
    return abs(dE - thr) <= rel_tau * max(abs(dE), 1e-3)


def metropolis_accept(dE: float, u: float, T: float) -> bool:
    return dE <= 0.0 or u < math.exp(-dE / T)


def initial_spins(L: int, seed: int, kind: str = "random"):
    N = L * L
    if kind == "random":
        return np.array([sampling.initial_spin(seed, p) for p in range(N)])
    if kind == "ferro":
        S = np.zeros((N, 3)); S[:, 2] = 1.0
        return S
    if kind == "neel":
        S = np.zeros((N, 3))
        for p in range(N):
            x, y = model.site_xy(L, p)
            S[p, 2] = 1.0 if (x + y) % 2 == 0 else -1.0
        return S
    raise ValueError(kind)


def cluster_dF(S, prm: Params, p: int, s_new, T: float, Lc: int, eig=eigvals_lapack):
    """F_new - F_old of the cluster around p when S_p -> s_new."""
    C = model.gather_cluster(S, prm.L, Lc, p)
    e_old = eig(model.cluster_hamiltonian(C, Lc, prm.t, prm.JH))
    C2 = C.copy()
    C2[0] = s_new
    e_new = eig(model.cluster_hamiltonian(C2, Lc, prm.t, prm.JH))
    return free_energy(e_new, T, prm.mu) - free_energy(e_old, T, prm.mu)


def update_record(S, prm: Params, T: float, sweep: int, p: int, eig, rel_tau):
    Lc = prm.cluster_size(sweep, p)
    s_new = sampling.proposal(prm.seed, sweep, p)
    dF = cluster_dF(S, prm, p, s_new, T, Lc, eig)
    dE = dF + model.classical_delta(S, prm.L, p, s_new, prm.JAF)
    u, _ = sampling.metropolis_uniforms(prm.seed, sweep, p)
    acc = metropolis_accept(dE, u, T)
    return dict(site=p, Lc=Lc, dF=dF, dE=dE, u=u, accept=acc,
                near=near_threshold(dE, u, T, rel_tau), s_new=s_new)


def sweep_sequential(S, prm: Params, T: float, sweep: int, eig=eigvals_lapack,
                     rel_tau=1e-9):
    """One sequential TCA sweep (Fig. 2) in block-major raster order.
    Returns (new state, list of per-update records)."""
    model.validate(prm.L, max((prm.Lc,) + tuple(prm.Lc_classes)))
    S = np.array(S, dtype=np.float64, copy=True)
    recs = []
    for p in model.sweep_order(prm.L):
        r = update_record(S, prm, T, sweep, p, eig, rel_tau)
        if r["accept"]:
            S[p] = r["s_new"]
        recs.append(r)
    return S, recs


def sweep_block_batched(S, prm: Params, T: float, sweep: int, eig=eigvals_lapack,
                        rel_tau=1e-9):
    """The parallel scheme of Sec. III: for each block, every cluster's dF is
    taken from the block-start snapshot (all clusters of a block are
    independent), then the decisions are made in raster order with the
    classical term read from the current state.  Must equal
    ``sweep_sequential`` bit for bit."""
    S = np.array(S, dtype=np.float64, copy=True)
    recs = []
    for K in range(4):
        sites = model.block_sites(prm.L, K)
        snap = S.copy()
        dFs = {}
        for p in sites:
            Lc = prm.cluster_size(sweep, p)
            s_new = sampling.proposal(prm.seed, sweep, p)
            dFs[p] = (cluster_dF(snap, prm, p, s_new, T, Lc, eig), s_new, Lc)
        for p in sites:
            dF, s_new, Lc = dFs[p]
            dE = dF + model.classical_delta(S, prm.L, p, s_new, prm.JAF)
            u, _ = sampling.metropolis_uniforms(prm.seed, sweep, p)
            acc = metropolis_accept(dE, u, T)
            if acc:
                S[p] = s_new
            recs.append(dict(site=p, Lc=Lc, dF=dF, dE=dE, u=u, accept=acc,
                             near=near_threshold(dE, u, T, rel_tau), s_new=s_new))
    return S, recs


def rel_err(a: float, b: float, t: float = 1.0) -> float:
    return abs(a - b) / max(abs(b), 1e-3 * t)


def _logged_near(g) -> bool:
    """Near-threshold flag of a logged update: a dict with key 'near', or a
    record with bit 0 of 'flags'."""
    if isinstance(g, dict):
        return bool(g.get("near", False))
    names = getattr(getattr(g, "dtype", None), "names", None) or ()
    return bool(int(g["flags"]) & 1) if "flags" in names else False


def replay_sweep(S, prm: Params, T: float, sweep: int, gpu_log, eig=eigvals_lapack,
                 rel_tau=1e-9, check=None):
    """Re-run one sweep update by update next to a logged trajectory.

    ``gpu_log`` lists, in visiting order, dicts with keys site, dF, accept
    (and optionally near).  For each update the oracle recomputes dF from the
    same pre-update state.  When the two decisions differ and either side
    flags the update as near-threshold, the logged decision is adopted (so the
    two states stay identical); an unflagged disagreement is counted as a
    failure.  ``check`` (optional set of visit positions) restricts the
    expensive dF recomputation to a sample; unchecked updates take the logged
    decision.  Returns (state, stats dict)."""
    S = np.array(S, dtype=np.float64, copy=True)
    order = model.sweep_order(prm.L)
    stats = dict(n=0, checked=0, max_rel=0.0, max_abs=0.0, flagged=0,
                 flagged_disagree=0, bad=0, bad_sites=[], rels=[])
    for pos, p in enumerate(order):
        g = gpu_log[pos]
        if int(g["site"]) != p:
            raise AssertionError(f"visit order differs at position {pos}: {g['site']} != {p}")
        stats["n"] += 1
        s_new = sampling.proposal(prm.seed, sweep, p)
        if check is None or pos in check:
            r = update_record(S, prm, T, sweep, p, eig, rel_tau)
            e = rel_err(float(g["dF"]), r["dF"], prm.t)
            stats["checked"] += 1
            stats["rels"].append(e)
            stats["max_rel"] = max(stats["max_rel"], e)
            stats["max_abs"] = max(stats["max_abs"], abs(float(g["dF"]) - r["dF"]))
            flag = r["near"] or _logged_near(g)
            stats["flagged"] += int(flag)
            if bool(g["accept"]) != r["accept"]:
                if flag:
                    stats["flagged_disagree"] += 1
                else:
                    stats["bad"] += 1
                    stats["bad_sites"].append(p)
        if bool(g["accept"]):
            S[p] = s_new
    return S, stats
