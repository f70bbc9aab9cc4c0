"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Floating-point tolerance: in FP64 mode dF must agree to 1e-9 relative with
the denominator floored at 1e-3 t; decisions must agree except for updates
flagged near-threshold by either side; states must agree bit for bit."""
import numpy as np
import pytest

from oracle import eigen, model, observables, sampling, tca as otca

pytestmark = pytest.mark.gpu

REL_TOL = 1e-9


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    import paper_1502_07028_amd as tca
    return tca


def recs_to_dicts(recs):
    return [dict(site=int(r["site"]), dF=float(r["dF"]), accept=bool(r["accept"]),
                 near=bool(r["flags"] & 1), Lc=int(r["Lc"])) for r in recs]


def rand_hermitian(n, seed, kind="gauss"):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        return (A + A.conj().T) / 2
    if kind == "zero":
        return np.zeros((n, n), complex)
    if kind == "scalar":
        return 2.5 * np.eye(n, dtype=complex)
    if kind == "diag":
        return np.diag(rng.normal(size=n)).astype(complex)
    if kind == "degenerate":
        q, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
        d = np.repeat([-1.0, 0.5, 3.0], (n + 2) // 3)[:n]
        return (q * d) @ q.conj().T
    if kind == "tridiag":
        A = np.diag(rng.normal(size=n)).astype(complex)
        off = rng.normal(size=n - 1) + 1j * rng.normal(size=n - 1)
        A += np.diag(off, -1) + np.diag(off.conj(), 1)
        return A
    raise ValueError(kind)


# ------------------------------------------------------------------ sampler
def test_initial_spins_bitwise(lib):
    L, seed = 16, 7
    lat = lib.Lattice(L, 4, seed=seed)
    S = lat.spins()
    ref = otca.initial_spins(L, seed)
    lat.close()
    assert np.array_equal(S, ref)


def test_accepted_proposals_bitwise(lib):
    """At very high T nearly every proposal is accepted; every accepted spin
    must equal the oracle's Marsaglia sample bit for bit."""
    L, seed = 8, 3
    lat = lib.Lattice(L, 4, seed=seed)
    recs, _ = lat.sweep([1e6], log=True)
    S = lat.spins()
    lat.close()
    n_acc = 0
    for r in recs:
        if r["accept"]:
            n_acc += 1
            assert tuple(S[r["site"]]) == sampling.proposal(seed, 0, int(r["site"]))
    assert n_acc > 50


# ------------------------------------------------------------------ eigenvalues
NS = [2, 3, 8, 17, 32, 33, 50, 64, 72, 100, 128, 162, 200]


@pytest.mark.parametrize("n", NS)
def test_heevals_random_fp64(lib, n):
    A = np.stack([rand_hermitian(n, 100 * n + b) for b in range(3)])
    w, F = lib.tca_heevals_batched(A, lib.TCA_FP64, T=0.3, mu=0.1)
    for b in range(3):
        ref = eigen.eigvals_lapack(A[b])
        scale = max(1.0, np.max(np.abs(ref)))
        assert np.max(np.abs(w[b] - ref)) <= 1e-12 * scale * max(1.0, n / 32)
        Fref = otca.free_energy(ref, 0.3, 0.1)
        assert abs(F[b] - Fref) <= 1e-11 * max(1.0, abs(Fref))


@pytest.mark.parametrize("kind", ["zero", "scalar", "diag", "degenerate", "tridiag"])
@pytest.mark.parametrize("n", [2, 31, 128])
def test_heevals_special_matrices(lib, kind, n):
    A = rand_hermitian(n, n, kind)[None]
    w, _ = lib.tca_heevals_batched(A, lib.TCA_FP64)
    ref = eigen.eigvals_lapack(A[0])
    assert np.max(np.abs(w[0] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))) * max(1.0, n / 32)


@pytest.mark.parametrize("n", [32, 72, 128, 200])
def test_heevals_mixed_precision(lib, n):
    A = np.stack([rand_hermitian(n, 7 * n + b) for b in range(2)])
    w, _ = lib.tca_heevals_batched(A, lib.TCA_MIXED)
    for b in range(2):
        ref = eigen.eigvals_lapack(A[b])
        assert np.max(np.abs(w[b] - ref)) <= 2e-5 * np.max(np.abs(ref)) * np.sqrt(n)


def test_heevals_empty_batch(lib):
    w, _ = lib.tca_heevals_batched(np.zeros((0, 8, 8), complex))
    assert w.shape == (0, 8)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("Lc,d", [(4, 2), (2, 3), (4, 3)])
def test_hubbard_mf_cluster_spectra(lib, Lc, d, precision):
    """Cluster matrices of the paper's Hubbard mean-field benchmark model
    (Eq. (1); the 3D 4^3 cluster gives n = 128) through the batched solver:
    eigenvalues against LAPACK and grand potentials against the oracle, for
    random fields of random length, a uniform field and m = 0 (degenerate)."""
    from oracle import hubbard_mf as hmf
    rng = np.random.default_rng(10 * Lc + d)
    Nc, U = Lc ** d, 8.0
    fields = []
    for _ in range(4):
        v = rng.normal(size=(Nc, 3))
        fields.append(v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.0, 1.2, (Nc, 1)))
    fields += [np.tile([0.0, 0.0, 0.8], (Nc, 1)), np.zeros((Nc, 3))]
    A = np.stack([hmf.cluster_hamiltonian(m, Lc, d, 1.0, U) for m in fields])
    n = A.shape[1]
    T, mu = 0.1, U / 2
    w, F = lib.tca_heevals_batched(A, precision, T=T, mu=mu)
    for b in range(len(A)):
        ref = eigen.eigvals_lapack(A[b])
        scale = max(1.0, np.max(np.abs(ref)))
        tol = 1e-12 * scale * max(1.0, n / 32) if precision == 0 else 2e-5 * scale * np.sqrt(n)
        assert np.max(np.abs(w[b] - ref)) <= tol
        Fref = otca.free_energy(ref, T, mu)
        ftol = 1e-11 * max(1.0, abs(Fref)) if precision == 0 else n * tol
        assert abs(F[b] - Fref) <= ftol


@pytest.mark.parametrize("Lc", [2, 3, 4, 5, 6, 8, 10])
def test_cluster_eigvals_ferro_closed_form(lib, Lc):
    lat = lib.Lattice(20, Lc, init=lib.TCA_INIT_FERRO)
    ev = lat.eigvals([0, 37, 399], Lc)
    lat.close()
    ref = model.band_closed_form(Lc, 1.0, 8.0, "ferro")
    n = 2 * Lc * Lc
    assert np.max(np.abs(ev[:, :n] - ref)) < 1e-12


@pytest.mark.parametrize("Lc", [2, 4, 6, 8, 10])
def test_cluster_eigvals_neel_closed_form(lib, Lc):
    lat = lib.Lattice(20, Lc, init=lib.TCA_INIT_NEEL)
    ev = lat.eigvals([0, 21, 398], Lc)
    lat.close()
    ref = model.band_closed_form(Lc, 1.0, 8.0, "neel")
    n = 2 * Lc * Lc
    assert np.max(np.abs(ev[:, :n] - ref)) < 1e-12


@pytest.mark.parametrize("Lc", [3, 4, 7, 8, 10])
def test_cluster_eigvals_random_state(lib, Lc):
    L, seed = 20, 5
    lat = lib.Lattice(L, Lc, seed=seed)
    S = lat.spins()
    sites = [0, 19, 205, 399]
    prop = np.array([sampling.proposal(99, 0, s) for s in sites])
    ev0 = lat.eigvals(sites, Lc)
    ev1 = lat.eigvals(sites, Lc, proposed=prop)
    lat.close()
    n = 2 * Lc * Lc
    for r, p in enumerate(sites):
        C = model.gather_cluster(S, L, Lc, p)
        ref0 = eigen.eigvals_lapack(model.cluster_hamiltonian(C, Lc, 1.0, 8.0))
        C[0] = prop[r]
        ref1 = eigen.eigvals_lapack(model.cluster_hamiltonian(C, Lc, 1.0, 8.0))
        assert np.max(np.abs(ev0[r, :n] - ref0)) < 1e-12
        assert np.max(np.abs(ev1[r, :n] - ref1)) < 1e-12


# ------------------------------------------------------------------ sweeps
def run_lockstep(lib, L, Lc, JAF, seed, T, nsweeps, check=None, precision=0, classes=()):
    lat = lib.Lattice(L, Lc, seed=seed, JH=8.0, JAF=JAF, precision=precision, Lc_classes=classes)
    prm = otca.Params(L=L, Lc=Lc, JH=8.0, JAF=JAF, seed=seed, Lc_classes=tuple(classes))
    out = []
    for sw in range(nsweeps):
        S0 = lat.spins()
        recs, st = lat.sweep([T], log=True)
        S1 = lat.spins()
        Sor, stats = otca.replay_sweep(S0, prm, T, sw, recs_to_dicts(recs), check=check)
        assert np.array_equal(Sor, S1), f"state differs after sweep {sw}"
        assert st["updates"] == L * L
        out.append((recs, stats, st))
    lat.close()
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_sweep_lockstep_c1(lib, seed):
    """8x8 lattice, 4x4 cluster, J_AF = 0, T = 0.05, 10 sweeps: every update
    replayed by the oracle."""
    res = run_lockstep(lib, 8, 4, 0.0, seed, 0.05, 10)
    nacc = 0
    for recs, stats, st in res:
        assert stats["bad"] == 0
        assert stats["max_rel"] <= REL_TOL, stats["max_rel"]
        nacc += st["accepted"]
    assert 0 < nacc < 640


def test_sweep_lockstep_c1_superexchange(lib):
    """Same with J_AF = 0.05: exercises the anti-diagonal decision pass."""
    res = run_lockstep(lib, 8, 4, 0.05, 4, 0.05, 6)
    for recs, stats, st in res:
        assert stats["bad"] == 0
        assert stats["max_rel"] <= REL_TOL


@pytest.mark.parametrize("T", [0.02, 0.05, 0.1])
def test_sweep_c2_sampled(lib, T):
    """32x32 lattice, 8x8 cluster (128x128 complex), J_AF = 0.05: two sweeps,
    every decision followed and a sample of updates recomputed."""
    rng = np.random.default_rng(int(T * 1000))
    check = set(rng.choice(1024, 40, replace=False).tolist()) | {0, 255, 256, 1023}
    res = run_lockstep(lib, 32, 8, 0.05, 11, T, 2, check=check)
    for recs, stats, st in res:
        assert stats["bad"] == 0
        assert stats["max_rel"] <= REL_TOL, stats["max_rel"]


def test_sweep_mixed_precision_error(lib):
    """FP32 reduction, FP64 eigenvalues and log-sum: dF error vs the FP64
    oracle is reported; bounded loosely (parity unpinned beyond the bound)."""
    rng = np.random.default_rng(5)
    check = set(rng.choice(1024, 48, replace=False).tolist())
    res = run_lockstep(lib, 32, 8, 0.05, 12, 0.05, 1, check=check, precision=1)
    recs, stats, st = res[0]
    rels = np.array(stats["rels"])
    print(f"mixed dF err: max abs {stats['max_abs']:.3e}, rel max {rels.max():.3e} "
          f"p50 {np.median(rels):.3e}")
    # FP32 reduction: backward error ~ n eps32 ||H|| per eigenvalue (n = 128,
    # ||H||_2 <= 8); dF inherits a few times that in absolute terms
    assert stats["max_abs"] < 128 * 2.0 ** -24 * 8.0


def test_sweep_uneven_classes(lib):
    """Cluster size drawn per update from {6, 8, 10} (72, 128, 200)."""
    rng = np.random.default_rng(9)
    check = set(rng.choice(400, 24, replace=False).tolist())
    res = run_lockstep(lib, 20, 8, 0.05, 13, 0.05, 1, check=check, classes=(6, 8, 10))
    recs, stats, st = res[0]
    assert stats["bad"] == 0 and stats["max_rel"] <= REL_TOL
    lcs = [int(r["Lc"]) for r in recs]
    prm = otca.Params(L=20, Lc=8, seed=13, Lc_classes=(6, 8, 10))
    assert lcs == [prm.cluster_size(0, int(r["site"])) for r in recs]
    assert set(lcs) == {6, 8, 10}


def test_sweep_large_lattice_sampled(lib):
    """320x320 lattice (25,600 clusters per block): one sweep, sampled."""
    L = 320
    rng = np.random.default_rng(2)
    check = set(rng.choice(L * L, 16, replace=False).tolist())
    res = run_lockstep(lib, L, 8, 0.03, 21, 0.1, 1, check=check)
    recs, stats, st = res[0]
    assert stats["bad"] == 0 and stats["max_rel"] <= REL_TOL


def test_sweep_wide_block_decisions(lib):
    """Blocks wider than 512 sites (1028x1028 lattice, 2x2 cluster, J_AF != 0)
    take the decision kernel that reads every neighbour from memory: one sweep,
    every decision replayed by the oracle from the logged dF, a few dF recomputed."""
    L = 1028
    rng = np.random.default_rng(4)
    check = set(rng.choice(L * L, 8, replace=False).tolist())
    res = run_lockstep(lib, L, 2, 0.05, 23, 0.1, 1, check=check)
    recs, stats, st = res[0]
    assert stats["bad"] == 0 and stats["max_rel"] <= REL_TOL


@pytest.mark.parametrize("L", [48, 50])
def test_decision_pass_at_staging_limit(lib, L):
    """Blocks of side 24 (staged whole in LDS) and 25 (read one anti-diagonal
    ahead from memory), J_AF != 0: every decision replayed by the oracle."""
    rng = np.random.default_rng(L)
    check = set(rng.choice(L * L, 8, replace=False).tolist())
    res = run_lockstep(lib, L, 2, 0.05, 31, 0.1, 2, check=check)
    for recs, stats, st in res:
        assert stats["bad"] == 0 and stats["max_rel"] <= REL_TOL
        assert 0 < st["accepted"] < L * L


@pytest.mark.parametrize("L,Lc,JAF", [(8, 4, 0.05), (8, 4, 0.0), (50, 2, 0.05)])
def test_metropolis_fast_path_equals_exact_form(lib, L, Lc, JAF):
    """Decisions taken from ln u away from the threshold equal those of the
    exact form (u < exp(-dE/T) for every update, TCA_FLAG_EXACT_METROPOLIS):
    spins and update records bitwise, for the staged (side 4), memory-fed
    (side 25) and independent (J_AF = 0) decision kernels."""
    out = []
    for flags in (0, lib.TCA_FLAG_EXACT_METROPOLIS):
        lat = lib.Lattice(L, Lc, seed=41, JH=8.0, JAF=JAF, flags=flags)
        recs = [lat.sweep([0.05], log=True)[0] for _ in range(2)]
        out.append((lat.spins(), recs))
        lat.close()
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1], out[1][1]):
        assert a.tobytes() == b.tobytes()
    assert 0 < int(sum(r["accept"].sum() for r in out[0][1])) < 2 * L * L


def test_zero_sweeps_is_noop(lib):
    lat = lib.Lattice(8, 4, seed=1)
    S0 = lat.spins()
    recs, st = lat.sweep(np.zeros(0), log=False)
    assert np.array_equal(lat.spins(), S0) and lat.sweep_counter == 0
    lat.close()


def test_resume_is_bitwise(lib):
    L, Lc, T = 16, 4, 0.05
    a = lib.Lattice(L, Lc, seed=8, JAF=0.05)
    a.sweep([T] * 4)
    Sa = a.spins()
    b = lib.Lattice(L, Lc, seed=8, JAF=0.05)
    b.sweep([T] * 2)
    ck, sc = b.spins(), b.sweep_counter
    b.close()
    c = lib.Lattice(L, Lc, seed=8, JAF=0.05, spins=ck)
    c.set_state(ck, sc)
    c.sweep([T] * 2)
    assert np.array_equal(c.spins(), Sa)
    a.close()
    c.close()


def test_determinism(lib):
    outs = []
    for _ in range(2):
        lat = lib.Lattice(16, 8, seed=4, JAF=0.05)
        recs, _ = lat.sweep([0.05, 0.05], log=True)
        outs.append((recs.copy(), lat.spins()))
        lat.close()
    assert outs[0][0].tobytes() == outs[1][0].tobytes()
    assert np.array_equal(outs[0][1], outs[1][1])


# ------------------------------------------------------------------ S(q)
def test_structure_factor(lib):
    for init, L in [(lib.TCA_INIT_RANDOM, 12), (lib.TCA_INIT_NEEL, 10), (lib.TCA_INIT_FERRO, 6)]:
        lat = lib.Lattice(L, 2, seed=3, init=init)
        S, sq, m = lat.observables()
        lat.close()
        ref = observables.sq_dft(S, L)
        assert np.max(np.abs(sq - ref)) < 1e-13
        assert abs(sq.sum() - 1.0) < 1e-12
        assert np.allclose(m, S.mean(0), atol=1e-15)


def test_graph_replay_matches_direct_launches(lib):
    """Sweeps replayed from one captured graph (sweep counter and T read on the
    device) equal directly issued sweeps, call after call, with an annealed
    temperature schedule and host work between the calls."""
    L, Lc, seed = 16, 4, 9
    a = lib.Lattice(L, Lc, seed=seed, JAF=0.05)
    b = lib.Lattice(L, Lc, seed=seed, JAF=0.05, flags=lib.TCA_FLAG_NO_GRAPH)
    for Ts in ([0.1, 0.08], [0.06], [0.05, 0.04, 0.03]):
        _, sa = a.sweep(Ts)
        _, sb = b.sweep(Ts)
        assert sa["accepted"] == sb["accepted"] and sa["updates"] == sb["updates"]
        assert np.array_equal(a.spins(), b.spins())
    # a logged (direct) call after graph replays continues the same chain
    ra, _ = a.sweep([0.05], log=True)
    rb, _ = b.sweep([0.05], log=True)
    assert np.array_equal(ra["accept"], rb["accept"]) and np.array_equal(ra["dF"], rb["dF"])
    assert a.sweep_counter == b.sweep_counter == 7
    a.close()
    b.close()


def test_autotuner_reports_choices(lib):
    lat = lib.Lattice(16, 8, seed=1)
    rep = lat.tuning_report()
    assert "n=128" in rep and "fp64" in rep
    lat.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [32, 50, 64, 72, 80, 128, 129, 162, 176, 177, 200])
def test_every_reducer_variant(lib, n, precision):
    """Each reducer variant the autotuner may pick gives the LAPACK spectrum
    (FP64 to 1e-12 of the spectral scale, mixed to the FP32 bound), on random
    Hermitian matrices of ragged dimensions and of each class's padded size and
    minimum."""
    names = lib.tca_reducer_variants(n, precision)
    A = np.stack([rand_hermitian(n, 40 + s) for s in range(3)])
    ref = np.stack([np.linalg.eigvalsh(a) for a in A])
    scale = np.max(np.abs(ref))
    # FP64 as test_heevals_random_fp64; FP32 as test_heevals_mixed_precision
    tol = 1e-12 * max(1.0, n / 32) if precision == 0 else 2e-5 * np.sqrt(n)
    try:
        for v, name in enumerate(names):
            lib.tca_select_reducer_variant(n, precision, v)
            w, _ = lib.tca_heevals_batched(A, precision=precision)
            assert np.max(np.abs(np.sort(w, axis=1) - ref)) <= tol * max(1.0, scale), name
    finally:
        lib.tca_select_reducer_variant(n, precision, 0)


def _cluster_matrices(Lc):
    rng = np.random.default_rng(Lc)
    Nc = Lc * Lc
    mats = []
    for _ in range(2):
        sp = rng.normal(size=(Nc, 3))
        mats.append(sp / np.linalg.norm(sp, axis=1, keepdims=True))
    mats.append(np.tile([0.0, 0.0, 1.0], (Nc, 1)))                       # ferromagnet
    sgn = np.array([(-1) ** ((l % Lc) + (l // Lc)) for l in range(Nc)], float)
    mats.append(np.outer(sgn, [0.0, 0.0, 1.0]))                           # Neel
    mats.append(np.tile([0.6, 0.0, 0.8], (Nc, 1)))                        # tilted ferromagnet
    return np.stack([model.cluster_hamiltonian(sp, Lc, 1.0, 8.0) for sp in mats])


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("Lc", [5, 6, 8, 10])
def test_every_reducer_variant_cluster_matrices(lib, Lc, precision):
    """Each reducer variant on cluster Hamiltonians (sparse columns with exact
    zeros, degenerate spectra: random, ferromagnetic, Neel and tilted spins)."""
    n = 2 * Lc * Lc
    names = lib.tca_reducer_variants(n, precision)
    A = _cluster_matrices(Lc)
    ref = np.stack([np.linalg.eigvalsh(a) for a in A])
    tol = (1e-12 * max(1.0, n / 32) if precision == 0 else 2e-5 * np.sqrt(n)) * np.max(np.abs(ref))
    bad = []
    try:
        for v, name in enumerate(names):
            lib.tca_select_reducer_variant(n, precision, v)
            w, _ = lib.tca_heevals_batched(A, precision=precision)
            err = np.max(np.abs(np.sort(w, axis=1) - ref), axis=1)
            if not np.all(err <= tol):
                bad.append((name, err.tolist()))
        assert not bad, bad
    finally:
        lib.tca_select_reducer_variant(n, precision, 0)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_reducer_variants_lockstep_8x8_cluster(lib, variant):
    """Sampled lockstep replay of a 32x32 / 8x8 sweep with each FP64 reducer variant."""
    names = lib.tca_reducer_variants(128, 0)
    if variant >= len(names):
        pytest.skip("no such variant")
    lib.tca_select_reducer_variant(128, 0, variant)
    try:
        L, Lc, T, seed = 32, 8, 0.05, 3
        lat = lib.Lattice(L, Lc, seed=seed, JAF=0.05)
        S0 = lat.spins()
        recs, _ = lat.sweep([T], log=True)
        S1 = lat.spins()
        lat.close()
        prm = otca.Params(L=L, Lc=Lc, JAF=0.05, seed=seed)
        rng = np.random.default_rng(variant)
        check = set(rng.choice(L * L, 16, replace=False).tolist())
        S_or, st = otca.replay_sweep(S0, prm, T, 0, recs_to_dicts(recs), check=check)
        assert st["bad"] == 0 and st["max_rel"] <= REL_TOL, names[variant]
        assert np.array_equal(S_or, S1)
    finally:
        lib.tca_select_reducer_variant(128, 0, 0)
