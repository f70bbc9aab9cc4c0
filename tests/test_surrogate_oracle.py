"""Pins of the delayed-acceptance oracle (oracle/surrogate.py) against
mathematics that does not depend on how the oracle is written: finite
differences, Adam's closed-form first step, hand-computed bfloat16 roundings,
detailed balance of the two-stage kernel and exact enumeration of a small
chain's stationary law."""
import math

import numpy as np
import pytest

from oracle import model, sampling, surrogate as sg, tca


def small_net(seed, n_in, hidden=8, scale=1.0):
    p = sg.init_params(seed, n_in, hidden)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(scale=0.3, size=p[k].shape)
    p["W3"] = p["W3"] * scale
    return p


# ---------------------------------------------------------------- arithmetic
def test_bf16_rounding_hand_values():
    x = [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 2 ** -7 + 2 ** -8, -3.14159, 0.0, 2.0 ** -130,
         65504.0]
    want = [1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -6, -3.140625, 0.0, 2.0 ** -130, 65536.0]
    assert list(sg.round_bf16(x)) == want


def test_silu_identities():
    z = np.linspace(-20, 20, 81)
    assert sg.silu(np.array([0.0]))[0] == 0.0
    assert np.allclose(sg.silu(z) - sg.silu(-z), z, atol=1e-12)
    h = 1e-6
    fd = (sg.silu(z + h) - sg.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - sg.silu_grad(z))) < 1e-8


def test_backward_matches_central_differences():
    n_in, H, B = 16, 8, 7
    p = small_net(3, n_in, H)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(B, n_in))
    y = rng.normal(size=B)
    _, g = sg.backward(p, X, y)
    h = 1e-6
    worst = 0.0
    for k in sg.PARAM_ORDER:
        flat = p[k].reshape(-1)
        gk = g[k].reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp = sg.mse_loss(p, X, y)
            flat[i] = old - h
            lm = sg.mse_loss(p, X, y)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            worst = max(worst, abs(fd - gk[i]) / max(1e-6, abs(fd)))
    assert worst < 1e-6


def test_adam_first_step_is_lr_times_sign():
    """With m0 = v0 = 0 the bias-corrected first moments are g and g^2, so
    the first Adam step moves each parameter by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = {"a": rng.normal(size=50)}
    g = {"a": rng.normal(size=50)}
    m = {"a": np.zeros(50)}
    v = {"a": np.zeros(50)}
    before = p["a"].copy()
    sg.adam_step(p, g, m, v, 1, 0.01)
    step = before - p["a"]
    dev = np.abs(step - 0.01 * np.sign(g["a"]))
    assert np.all(dev <= 0.01 * 1e-8 / np.abs(g["a"]) + 1e-15)


def test_flatten_roundtrip():
    p = small_net(2, 10, 6)
    v = sg.flatten(p)
    assert v.size == 6 * 10 + 6 + 36 + 6 + 6 + 1
    q = sg.unflatten(v, 10, 6)
    for k in sg.PARAM_ORDER:
        assert np.array_equal(p[k], q[k])


def test_features_layout():
    C = np.arange(12, dtype=float).reshape(4, 3) / 20
    s = np.array([0.0, 0.6, 0.8])
    f = sg.features(C, s, 0.05)
    assert f.size == sg.n_inputs(2)
    assert np.array_equal(f[:12], C.ravel()) and np.array_equal(f[12:15], s)
    assert f[15] == 0.05 / sg.T_REF
    r = sg.reverse_features(C, s, 0.05)
    assert np.array_equal(r[:3], s) and np.array_equal(r[3:12], C[1:].ravel())
    assert np.array_equal(r[12:15], C[0])


def test_bf16_forward_close_to_fp64():
    p = sg.init_params(5, sg.n_inputs(8))
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, size=(40, sg.n_inputs(8)))
    a = sg.forward(p, X)[0]
    b = sg.forward_bf16(p, X)
    # a few bfloat16 roundings (relative 2^-9 each) per layer
    assert np.max(np.abs(a - b)) < 0.05 * (np.max(np.abs(a)) + 0.1)
    assert not np.array_equal(a, b)


# ---------------------------------------------------------------- the chain
L2_T, L2_JAF = 1.0, 0.3


def _flip_setup(seed_net, scale):
    L, Lc = 2, 2
    prm = tca.Params(L=L, Lc=Lc, JAF=L2_JAF, seed=11)
    p = small_net(seed_net, sg.n_inputs(Lc), 8, scale=scale)
    dS = sg.net_fn(p)

    def state(bits):
        S = np.zeros((4, 3))
        S[:, 2] = [1 - 2 * ((bits >> i) & 1) for i in range(4)]
        return S

    def energy(bits):
        S = state(bits)
        e = np.linalg.eigvalsh(model.cluster_hamiltonian(S, Lc, 1.0, 8.0))
        return tca.free_energy(e, L2_T, 0.0) + model.classical_energy(S, L, L2_JAF)

    E = np.array([energy(b) for b in range(16)])
    w = np.exp(-(E - E.min()) / L2_T)
    w /= w.sum()
    return prm, dS, state, w


def _threshold(accepts):
    """Lebesgue measure of {u in (0,1): accepts(u)} for a decision that holds
    for small u and fails above a threshold (bisection on the decision)."""
    if accepts(1.0 - 2 ** -53):
        return 1.0
    lo, hi = 0.0, 1.0 - 2 ** -53
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        if accepts(mid):
            lo = mid
        else:
            hi = mid
    return lo


def test_delayed_acceptance_detailed_balance_2x2():
    """pi(x) P(x->y) = pi(y) P(y->x) for every single-site flip of the 2x2
    flip chain, with P built from the stage decision functions alone (their
    acceptance regions measured by bisection in u1 and u) and a surrogate
    that is wrong by construction."""
    prm, dS, state, w = _flip_setup(21, 3.0)
    T = L2_T

    def prob(bits, p):
        S = state(bits)
        s_new = -S[p]
        C = model.gather_cluster(S, 2, 2, p)
        dSf = dS(sg.features(C, s_new, T))
        dSr = dS(sg.reverse_features(C, s_new, T))
        dE = tca.cluster_dF(S, prm, p, s_new, T, 2) + model.classical_delta(S, 2, p, s_new, L2_JAF)
        m1 = _threshold(lambda u1: sg.stage1_pass(dSf, u1, T))
        m2 = _threshold(lambda u: sg.stage2_accept(dE, dSf, dSr, u, T))
        return m1 * m2, dSf

    worst, spread = 0.0, []
    for x in range(16):
        for p in range(4):
            y = x ^ (1 << p)
            pxy, dSf = prob(x, p)
            pyx, _ = prob(y, p)
            spread.append(dSf)
            worst = max(worst, abs(w[x] * pxy - w[y] * pyx) / (w[x] * pxy + w[y] * pyx))
    assert worst < 1e-9
    assert np.std(spread) > 0.1     # the surrogate is far from constant


def test_delayed_acceptance_chain_matches_enumeration_2x2():
    """Visit histogram of the 2x2 flip chain driven by the oracle's
    delayed-acceptance decisions (Philox uniforms, wrong surrogate) against
    exp(-(F + E_cl)/T)/Z.  The surrogate is a random network whose output
    (about 0.9 +- 0.05) does not follow dE at all; a harsher one still leaves
    the law exact (detailed-balance test above) but mixes too slowly for a
    histogram of this length."""
    prm, dS, state, w = _flip_setup(22, 0.3)
    T = L2_T
    S = state(0)
    counts = np.zeros(16)
    nsw, passed, total = 6000, 0, 0
    for sw in range(nsw):
        for p in model.sweep_order(2):
            s_new = -S[p]
            C = model.gather_cluster(S, 2, 2, p)
            dSf = dS(sg.features(C, s_new, T))
            dSr = dS(sg.reverse_features(C, s_new, T))
            u, u1 = sampling.metropolis_uniforms(prm.seed, sw, p)
            total += 1
            if not sg.stage1_pass(dSf, u1, T):
                continue
            passed += 1
            dE = tca.cluster_dF(S, prm, p, s_new, T, 2) + model.classical_delta(S, 2, p, s_new,
                                                                                 L2_JAF)
            if sg.stage2_accept(dE, dSf, dSr, u, T):
                S[p] = s_new
        counts[sum(int(S[i, 2] < 0) << i for i in range(4))] += 1
    emp = counts / nsw
    assert 0.5 * np.sum(np.abs(emp - w)) < 0.04
    assert passed < 0.95 * total      # stage 1 really filters


def test_zero_surrogate_reduces_to_plain_metropolis():
    """dS == 0: stage 1 always passes and stage 2 is the plain Metropolis
    test, so the delayed-acceptance sweep reproduces the plain sweep."""
    prm = tca.Params(L=6, Lc=3, JAF=0.05, seed=4)
    S0 = tca.initial_spins(6, 4)
    Sa, ra = tca.sweep_sequential(S0, prm, 0.05, 0)
    Sb, rb = sg.sweep_da_sequential(S0, prm, 0.05, 0, lambda row: 0.0)
    assert all(r["stage1"] for r in rb)
    assert [r["accept"] for r in ra] == [r["accept"] for r in rb]
    assert np.array_equal(Sa, Sb)
    assert [r["dF"] for r in ra] == [r["dF"] for r in rb]


def test_replay_accepts_own_log_and_catches_planted_error():
    prm = tca.Params(L=6, Lc=3, JAF=0.05, seed=5)
    S0 = tca.initial_spins(6, 5)
    p = small_net(7, sg.n_inputs(3), 8, scale=0.3)
    dS = sg.net_fn(p, bf16=True)
    S1, recs = sg.sweep_da_sequential(S0, prm, 0.05, 0, dS)
    log = [dict(site=r["site"], flags=(int(r["near"]) | 2 * int(r["stage1"]) | 4 * int(r["near1"])),
                accept=r["accept"], dF=r["dF"], dS_f=r["dS_f"], dS_r=r["dS_r"]) for r in recs]
    S2, st = sg.replay_da_sweep(S0, prm, 0.05, 0, log, p=p)
    assert st["bad"] == 0 and np.array_equal(S1, S2)
    assert st["dS_max_abs"] < 1e-12 and st["max_rel"] == 0.0
    assert 0 < st["passed"] < st["n"]
    # plant: flip the first stage-1 decision
    k = 0
    log[k] = dict(log[k], flags=log[k]["flags"] ^ 2, accept=False, dF=math.nan)
    _, st2 = sg.replay_da_sweep(S0, prm, 0.05, 0, log, p=p)
    assert st2["bad"] >= 1
