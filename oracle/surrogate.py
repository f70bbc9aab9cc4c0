"""Learned first-stage filter and delayed-acceptance Metropolis, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper has no learned component.  This module follows the
delayed-acceptance scheme of Christen & Fox (J. Comput. Graph. Stat. 14, 795
(2005)) with the exact TCA energy of Sec. II as the second stage, so the
chain's stationary law is the plain TCA one for *any* surrogate.

Surrogate f: n_in inputs -> H -> H -> 1 with SiLU (z * sigmoid(z)) after the
first two layers (three Linear layers).  Inputs of a move, in this order: the
L_c^2 cluster spins in cluster order (x, y, z each), the proposed spin (3),
and T / T_REF (T_REF = 0.1); output: predicted fermionic dF of the move.
All inputs are cluster spins at or after the update site in raster order, so
they are the same in the block-start snapshot and in the sequential state
(the -x/-y lattice neighbours used by the classical term are not inputs).
For L_c = 8, n_in = 196; H = 256.

Delayed acceptance of a move x -> y with a symmetric proposal:
  stage 1: accept with a1(x->y) = min(1, exp(-dS(x->y)/T))
  stage 2: accept with a2 = min(1, exp(-dE/T) a1(y->x) / a1(x->y)),
where dS(y->x) is the surrogate on the reverse move (corner spin = proposal,
proposing the old spin).  In logarithms, with u1, u the two uniforms of the
update (words 1 and 0 of its Metropolis Philox block):
  stage 1 passes iff  u1 == 0 or ln u1 < min(0, -dS_f/T)
  stage 2 accepts iff u  == 0 or ln u  < -dE/T + min(0, -dS_r/T) - min(0, -dS_f/T).

Inference in BF16 is defined here as: inputs, W1 and W2 rounded to bfloat16
(round to nearest, ties to even), exact products summed, bias added, SiLU,
activation rounded to bfloat16; the output layer takes the rounded second
activation with W3 and b3 as given.  ``forward_bf16`` evaluates exactly that
in FP64.

Pinned by (tests/test_oracle_pins.py): central finite differences of the loss
(backward pass); Adam's first step moving each parameter by lr * sign(g); the
bfloat16 rounding at hand-computed values; SiLU identities; detailed balance
of the delayed-acceptance kernel computed from the decision functions
themselves on a 2x2 lattice; the visit histogram of a 2x2 flip chain with
delayed acceptance and a deliberately wrong surrogate against exact
enumeration.
"""
import math

import numpy as np

from . import model, sampling
from .eigen import eigvals_lapack

T_REF = 0.1
HIDDEN = 256


def n_inputs(Lc: int) -> int:
    return 3 * Lc * Lc + 4


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed, n_in, hidden=HIDDEN):
    """Uniform(-a, a) with a = sqrt(6/(fan_in + fan_out)), biases zero."""
    rng = np.random.default_rng(seed)

    def u(fo, fi):
        a = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))

    return {"W1": u(hidden, n_in), "b1": np.zeros(hidden),
            "W2": u(hidden, hidden), "b2": np.zeros(hidden),
            "W3": u(1, hidden), "b3": np.zeros(1)}


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(p):
    """Flat parameter vector in the order W1 (H x n_in, row-major), b1, W2
    (H x H), b2, W3 (H), b3 (1)."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unflatten(v, n_in, hidden):
    v = np.asarray(v, dtype=np.float64)
    shapes = {"W1": (hidden, n_in), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (1, hidden), "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = v[o:o + n].reshape(shapes[k]).copy()
        o += n
    assert o == v.size, (o, v.size)
    return out


def features(cluster_spins, proposal, T):
    """Input row of one move: flattened cluster spins, proposal, T/T_REF."""
    c = np.asarray(cluster_spins, dtype=np.float64).reshape(-1)
    return np.concatenate([c, np.asarray(proposal, dtype=np.float64), [float(T) / T_REF]])


def reverse_features(cluster_spins, proposal, T):
    """Input row of the reverse move: corner spin replaced by the proposal,
    proposing the old corner spin."""
    c = np.array(cluster_spins, dtype=np.float64, copy=True).reshape(-1, 3)
    old = c[0].copy()
    c[0] = proposal
    return features(c, old, T)


def forward(p, X):
    """Returns (out[B], cache)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    z1 = X @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    out = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return out, (X, z1, h1, z2, h2)


def round_bf16(x):
    """Round to bfloat16 (8 significant bits), nearest with ties to even, via
    the float32 bit pattern (finite inputs; the value is first rounded to
    float32)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, X):
    """BF16 inference as defined in the module docstring."""
    X = round_bf16(np.atleast_2d(np.asarray(X, dtype=np.float64)))
    h1 = round_bf16(silu(X @ round_bf16(p["W1"]).T + p["b1"]))
    h2 = round_bf16(silu(h1 @ round_bf16(p["W2"]).T + p["b2"]))
    return (h2 @ p["W3"].T + p["b3"])[:, 0]


def mse_loss(p, X, y):
    out, _ = forward(p, X)
    return float(np.mean((out - np.asarray(y)) ** 2))


def backward(p, X, y):
    """Loss = mean((f(X) - y)^2); returns (loss, grads dict) by the chain rule."""
    out, (X, z1, h1, z2, h2) = forward(p, X)
    B = X.shape[0]
    r = out - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    dout = (2.0 / B) * r[:, None]                 # [B, 1]
    g = {"W3": dout.T @ h2, "b3": dout.sum(0)}
    dh2 = dout @ p["W3"]                           # [B, H]
    dz2 = dh2 * silu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * silu_grad(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every parameter; t counts from 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** t)
        vh = v[k] / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


# ---------------------------------------------------------------- decisions
def stage1_pass(dS_f, u1, T):
    return math.log(u1) < min(0.0, -dS_f / T) if u1 > 0.0 else True


def stage2_rhs(dE, dS_f, dS_r, T):
    return -dE / T + min(0.0, -dS_r / T) - min(0.0, -dS_f / T)


def stage2_accept(dE, dS_f, dS_r, u, T):
    return math.log(u) < stage2_rhs(dE, dS_f, dS_r, T) if u > 0.0 else True


def da_decide(dE, dS_f, dS_r, u1, u, T):
    """(stage-1 passed, accepted) of one delayed-acceptance update."""
    if not stage1_pass(dS_f, u1, T):
        return False, False
    return True, stage2_accept(dE, dS_f, dS_r, u, T)


def near_stage1(dS_f, u1, T, rel_tau=1e-9):
    """Stage-1 test within rel_tau of its threshold (decision may differ
    between two correct evaluations)."""
    if u1 <= 0.0:
        return False
    return abs(T * (math.log(u1) - min(0.0, -dS_f / T))) <= rel_tau * max(abs(dS_f), 1e-3)


def near_stage2(dE, dS_f, dS_r, u, T, rel_tau=1e-9):
    if u <= 0.0:
        return False
    return abs(T * (math.log(u) - stage2_rhs(dE, dS_f, dS_r, T))) <= rel_tau * max(abs(dE), 1e-3)


# ---------------------------------------------------------------- sweeps
def net_fn(p, bf16=False):
    """dS(features row) of a parameter dict."""
    f = forward_bf16 if bf16 else (lambda q, X: forward(q, X)[0])
    return lambda row: float(f(p, row)[0])


def sweep_da_sequential(S, prm, T, sweep, dS, eig=eigvals_lapack, rel_tau=1e-9):
    """One sequential TCA sweep with delayed acceptance.  ``dS`` maps a
    feature row to the surrogate dF (any function).  Returns (state, records);
    a record has stage1, accept, dS_f, dS_r and, for stage-1 survivors, dF/dE."""
    from . import tca
    S = np.array(S, dtype=np.float64, copy=True)
    recs = []
    for p in model.sweep_order(prm.L):
        Lc = prm.cluster_size(sweep, p)
        s_new = sampling.proposal(prm.seed, sweep, p)
        C = model.gather_cluster(S, prm.L, Lc, p)
        dSf = dS(features(C, s_new, T))
        dSr = dS(reverse_features(C, s_new, T))
        u, u1 = sampling.metropolis_uniforms(prm.seed, sweep, p)
        r = dict(site=p, Lc=Lc, dS_f=dSf, dS_r=dSr, u=u, dF=math.nan, dE=math.nan,
                 stage1=stage1_pass(dSf, u1, T), accept=False,
                 near1=near_stage1(dSf, u1, T, rel_tau), near=False)
        if r["stage1"]:
            dF = tca.cluster_dF(S, prm, p, s_new, T, Lc, eig)
            dE = dF + model.classical_delta(S, prm.L, p, s_new, prm.JAF)
            r.update(dF=dF, dE=dE, accept=stage2_accept(dE, dSf, dSr, u, T),
                     near=near_stage2(dE, dSf, dSr, u, T, rel_tau))
            if r["accept"]:
                S[p] = s_new
        recs.append(r)
    return S, recs


def replay_da_sweep(S, prm, T, sweep, gpu_log, eig=eigvals_lapack, rel_tau=1e-9, p=None,
                    check=None):
    """Re-run one delayed-acceptance sweep next to a logged trajectory.

    Each logged record carries site, flags (bit 1: passed stage 1, bit 0 /
    bit 2: near-threshold at stage 2 / stage 1), accept, dF and the surrogate
    values dS_f, dS_r that the logged run used.  The oracle takes both stage
    decisions from those logged surrogate values with its own FP64 rules
    (the chain is exact for any surrogate), recomputes dF exactly for every
    stage-1 survivor (or for the positions in ``check``), and, when the
    parameter dict ``p`` is given, evaluates its own BF16-defined surrogate on
    the same state to bound the logged dS values.  A decision that differs
    and is not flagged near-threshold by either side is counted as bad; a
    flagged one adopts the logged decision.  Returns (state, stats)."""
    from . import tca
    S = np.array(S, dtype=np.float64, copy=True)
    order = model.sweep_order(prm.L)
    st = dict(n=0, passed=0, checked=0, max_rel=0.0, max_abs=0.0, bad=0, bad_sites=[],
              flagged=0, dS_max_abs=0.0, dS_checked=0)
    for pos, site in enumerate(order):
        g = gpu_log[pos]
        if int(g["site"]) != site:
            raise AssertionError(f"visit order differs at position {pos}")
        st["n"] += 1
        flags = int(g["flags"])
        Lc = prm.cluster_size(sweep, site)
        s_new = sampling.proposal(prm.seed, sweep, site)
        u, u1 = sampling.metropolis_uniforms(prm.seed, sweep, site)
        dSf, dSr = float(g["dS_f"]), float(g["dS_r"])
        if p is not None and (check is None or pos in check):
            C = model.gather_cluster(S, prm.L, Lc, site)
            ref = forward_bf16(p, np.stack([features(C, s_new, T),
                                            reverse_features(C, s_new, T)]))
            st["dS_max_abs"] = max(st["dS_max_abs"], abs(ref[0] - dSf), abs(ref[1] - dSr))
            st["dS_checked"] += 1
        pass_o = stage1_pass(dSf, u1, T)
        pass_g = bool(flags & 2)
        near1 = near_stage1(dSf, u1, T, rel_tau) or bool(flags & 4)
        if pass_o != pass_g:
            if near1:
                st["flagged"] += 1
            else:
                st["bad"] += 1
                st["bad_sites"].append(site)
        st["passed"] += int(pass_g)
        if pass_g and (check is None or pos in check):
            dF = tca.cluster_dF(S, prm, site, s_new, T, Lc, eig)
            dE = dF + model.classical_delta(S, prm.L, site, s_new, prm.JAF)
            e = tca.rel_err(float(g["dF"]), dF, prm.t)
            st["checked"] += 1
            st["max_rel"] = max(st["max_rel"], e)
            st["max_abs"] = max(st["max_abs"], abs(float(g["dF"]) - dF))
            acc_o = stage2_accept(dE, dSf, dSr, u, T)
            if acc_o != bool(g["accept"]):
                if near_stage2(dE, dSf, dSr, u, T, rel_tau) or bool(flags & 1):
                    st["flagged"] += 1
                else:
                    st["bad"] += 1
                    st["bad_sites"].append(site)
        if not pass_g and bool(g["accept"]):
            st["bad"] += 1
            st["bad_sites"].append(site)
        if bool(g["accept"]):
            S[site] = s_new
    return S, st
