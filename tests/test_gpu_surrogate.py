"""Parity of the learned first stage (hand-written FP32 training kernels,
BF16 MFMA inference, delayed-acceptance sweep) with the FP64 oracle, through
the C ABI.

Tolerances: gradients and FP32 predictions within 1e-4 of the largest entry
(FP32 accumulation over at most a few hundred terms); BF16 predictions
against the oracle's BF16 definition (same rounding points) within 1e-2 of
the output scale at worst and 1e-4 at the median (only an activation that
FP32 accumulation order pushes across a bfloat16 rounding boundary differs,
by one bfloat16 ulp); exact-stage dF within 1e-9 relative; delayed-acceptance
decisions identical except near-threshold updates; states bit for bit."""
import math

import numpy as np
import pytest

from oracle import model, sampling, surrogate as osg, tca as otca

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    import paper_1502_07028_amd as tca
    return tca


def oracle_params(sg):
    return osg.unflatten(sg.params().astype(np.float64), sg.n_in, sg.hidden)


def rand_rows(n, n_in, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, n_in)).astype(np.float32)
    y = rng.normal(scale=0.5, size=n).astype(np.float32)
    return X, y


def randomize(lib_sg, seed, bias=0.2, out=None):
    """Random weights with non-zero biases (the library initializes biases to 0);
    out = (w3 scale, b3) sets the output layer's spread and offset."""
    p = oracle_params(lib_sg)
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(scale=bias, size=p[k].shape)
    if out is not None:
        p["W3"] = p["W3"] * out[0]
        p["b3"] = np.array([out[1]])
    lib_sg.load(osg.flatten(p).astype(np.float32))
    return oracle_params(lib_sg)


@pytest.mark.parametrize("Lc,hidden,rows", [(4, 64, 200), (3, 80, 65), (8, 256, 130)])
def test_gradient_matches_oracle(lib, Lc, hidden, rows):
    sg = lib.Surrogate(Lc, hidden, seed=3)
    p = randomize(sg, 4)
    X, y = rand_rows(rows, sg.n_in, 5)
    loss, g = sg.grad(X, y)
    ref_loss, ref = osg.backward(p, X.astype(np.float64), y.astype(np.float64))
    ref = osg.flatten(ref)
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    for k, sl in zip(osg.PARAM_ORDER, np.split(np.arange(ref.size), np.cumsum(
            [p[q].size for q in osg.PARAM_ORDER])[:-1])):
        assert np.max(np.abs(g[sl] - ref[sl])) <= 1e-4 * np.max(np.abs(ref[sl])) + 1e-7, k
    sg.close()


def test_adam_steps_match_oracle(lib):
    sg = lib.Surrogate(3, 32, seed=6)
    p = oracle_params(sg)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    rng = np.random.default_rng(7)
    for t in (1, 2, 3):
        g = rng.normal(size=sg.n_params).astype(np.float32)
        sg.adam_step(g, 1e-2)
        osg.adam_step(p, osg.unflatten(g.astype(np.float64), sg.n_in, 32), m, v, t, 1e-2)
    got = sg.params().astype(np.float64)
    want = osg.flatten(p)
    assert np.max(np.abs(got - want)) <= 1e-6


@pytest.mark.parametrize("rows", [1, 63, 64, 300])
def test_fp32_and_bf16_predictions(lib, rows):
    sg = lib.Surrogate(8, 256, seed=8)
    p = randomize(sg, 9)
    X, _ = rand_rows(rows, sg.n_in, 10)
    out32 = sg.eval(X, bf16=False)
    ref = osg.forward(p, X.astype(np.float64))[0]
    scale = np.max(np.abs(ref)) + 1e-3
    assert np.max(np.abs(out32 - ref)) <= 1e-4 * scale
    out16 = sg.eval(X, bf16=True)
    ref16 = osg.forward_bf16(p, X.astype(np.float64))
    err = np.abs(out16 - ref16)
    assert np.max(err) <= 1e-2 * scale
    assert np.median(err) <= 1e-4 * scale
    sg.close()


def test_empty_eval_and_bad_arguments(lib):
    sg = lib.Surrogate(4, 32)
    assert sg.eval(np.zeros((0, sg.n_in), np.float32)).size == 0
    with pytest.raises(lib.TCAError):
        sg.train(1)                          # no rows
    with pytest.raises(lib.TCAError):
        sg.add_rows(np.zeros((1, sg.n_in)), np.zeros(1))   # capacity 0
    sg.close()


def test_collected_rows_match_oracle(lib):
    """Dataset rows of two exact sweeps: features of every proposed move in
    the state the sequential sweep sees, and its exact dF."""
    L, Lc, seed, T = 8, 4, 2, 0.05
    lat = lib.Lattice(L, Lc, seed=seed, JAF=0.05)
    S0 = lat.spins()
    sg = lib.Surrogate(Lc, 32, capacity=2 * L * L)
    st = sg.collect(lat, [T, T])
    assert st["updates"] == 2 * L * L and sg.rows == 2 * L * L
    X, y = sg.get_rows(0, 2 * L * L)
    prm = otca.Params(L=L, Lc=Lc, JAF=0.05, seed=seed)
    S = S0.copy()
    r = 0
    for sw in range(2):
        for K in range(4):
            for p in model.block_sites(L, K):
                rec = otca.update_record(S, prm, T, sw, p, otca.eigvals_lapack, 1e-9)
                C = model.gather_cluster(S, L, Lc, p)
                assert np.array_equal(X[r], osg.features(C, rec["s_new"], T).astype(np.float32))
                assert abs(float(y[r]) - rec["dF"]) <= 2 ** -23 * abs(rec["dF"]) + 1e-9
                if rec["accept"]:
                    S[p] = rec["s_new"]
                r += 1
    assert np.array_equal(S, lat.spins())
    lat.close()
    sg.close()


def _da_log(recs):
    return [dict(site=int(r["site"]), flags=int(r["flags"]), accept=bool(r["accept"]),
                 dF=float(r["dF"]), dS_f=float(r["dS_f"]), dS_r=float(r["dS_r"])) for r in recs]


@pytest.mark.parametrize("JAF,seed", [(0.0, 1), (0.05, 2)])
def test_delayed_acceptance_lockstep(lib, JAF, seed):
    L, Lc, T = 8, 4, 0.05
    lat = lib.Lattice(L, Lc, seed=seed, JAF=JAF)
    sg = lib.Surrogate(Lc, 64, seed=seed)
    # dS of about 0.05 +- 0.05 at T = 0.05: stage 1 passes roughly half the moves
    p = randomize(sg, seed + 10, bias=0.5, out=(0.1, 0.05))
    lat.attach(sg)
    prm = otca.Params(L=L, Lc=Lc, JAF=JAF, seed=seed)
    passed = 0
    for sw in range(2):
        S0 = lat.spins()
        recs, st = lat.sweep([T], log=True)
        S_or, rs = osg.replay_da_sweep(S0, prm, T, sw, _da_log(recs), p=p)
        assert rs["bad"] == 0, rs["bad_sites"]
        assert rs["max_rel"] <= 1e-9
        assert rs["dS_max_abs"] <= 1e-2 * (np.max(np.abs(recs["dS_f"])) + 1e-3)
        assert np.array_equal(S_or, lat.spins())
        assert st["stage1_passed"] == rs["passed"]
        passed += rs["passed"]
        nan = ~(recs["flags"] & 2).astype(bool)
        assert np.all(np.isnan(recs["dF"][nan]))
    assert 0 < passed < 2 * L * L
    lat.close()
    sg.close()


@pytest.mark.parametrize("JAF", [0.0, 0.05])
def test_delayed_acceptance_exact_form_flag(lib, JAF):
    """Second-stage decisions from ln u against the quotient equal the exact
    form's (TCA_FLAG_EXACT_METROPOLIS) bitwise, with a surrogate attached."""
    L, Lc, T = 8, 4, 0.05
    out = []
    for flags in (0, lib.TCA_FLAG_EXACT_METROPOLIS):
        lat = lib.Lattice(L, Lc, seed=6, JAF=JAF, flags=flags)
        sg = lib.Surrogate(Lc, 64, seed=6)
        randomize(sg, 16, bias=0.5, out=(0.1, 0.05))
        lat.attach(sg)
        recs = [lat.sweep([T], log=True)[0] for _ in range(2)]
        out.append((lat.spins(), recs))
        lat.close()
        sg.close()
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1], out[1][1]):
        assert a.tobytes() == b.tobytes()


def test_zero_surrogate_equals_plain_sweep(lib):
    L, Lc, T, seed = 12, 5, 0.05, 4
    a = lib.Lattice(L, Lc, seed=seed, JAF=0.05)
    b = lib.Lattice(L, Lc, seed=seed, JAF=0.05)
    sg = lib.Surrogate(Lc, 32)
    sg.load(np.zeros(sg.n_params, np.float32))
    b.attach(sg)
    ra, _ = a.sweep([T, T], log=True)
    rb, st = b.sweep([T, T], log=True)
    assert st["stage1_passed"] == st["updates"]
    assert np.array_equal(ra["accept"], rb["accept"])
    assert np.array_equal(ra["dF"], rb["dF"])
    assert np.array_equal(a.spins(), b.spins())
    for x in (a, b):
        x.close()
    sg.close()


def test_attach_rejects_mismatch(lib):
    lat = lib.Lattice(8, 4)
    sg = lib.Surrogate(3, 32)
    with pytest.raises(lib.TCAError):
        lat.attach(sg)
    lat.close()
    lat = lib.Lattice(8, 4, Lc_classes=(3, 4))
    with pytest.raises(lib.TCAError) as e:
        lat.attach(lib.Surrogate(4, 32))
    assert e.value.status == lib.TCA_E_UNSUPPORTED
    lat.close()
    sg.close()


def test_trained_filter_cuts_exact_work(lib):
    """What the trained network gains: a surrogate trained by the library on
    dF data of exact sweeps filters most rejected proposals before the exact
    stage, so the delayed-acceptance chain solves far fewer cluster matrices
    per proposal than the plain chain while accepting nearly as often."""
    L, Lc, JAF, seed = 16, 4, 0.05, 5
    Ts = [0.03, 0.05, 0.08]
    nwarm, ncol = 6, 16
    sg = lib.Surrogate(Lc, 128, seed=1, capacity=len(Ts) * ncol * L * L)
    for k, T in enumerate(Ts):
        lat = lib.Lattice(L, Lc, seed=seed + k, JAF=JAF)
        lat.sweep([T] * nwarm)
        sg.collect(lat, [T] * ncol)
        lat.close()
    untrained = sg.train(0, holdout=0.15)
    res = sg.train(3000, batch=256, lr=1e-3, holdout=0.15)
    print("surrogate", untrained, res)
    assert res["holdout_rmse_bf16"] < 0.5 * untrained["holdout_rmse_bf16"]

    T = 0.05
    plain = lib.Lattice(L, Lc, seed=seed + 1, JAF=JAF)
    plain.sweep([T] * nwarm)
    S = plain.spins()
    da = lib.Lattice(L, Lc, spins=S, seed=seed + 1, JAF=JAF)
    da.set_state(S, plain.sweep_counter)
    da.attach(sg)
    _, sp = plain.sweep([T] * 8)
    _, sd = da.sweep([T] * 8)
    acc_p = sp["accepted"] / sp["updates"]
    acc_d = sd["accepted"] / sd["updates"]
    pass_rate = sd["stage1_passed"] / sd["updates"]
    print(f"plain accept {acc_p:.3f}; delayed acceptance: stage-1 pass {pass_rate:.3f}, "
          f"accept {acc_d:.3f}, stage-2 reject {1 - acc_d / max(pass_rate, 1e-9):.3f}")
    assert pass_rate < 0.6
    assert acc_d > 0.5 * acc_p
    for x in (plain, da):
        x.close()
    sg.close()
