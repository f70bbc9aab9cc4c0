"""Pins of the FP64 oracle against things other than itself: an independent
Philox implementation, closed-form spectra, invariants, an unrelated
eigensolver, exact enumeration and the paper's Fig. 3 worked example."""
import json
import math
import os

import numpy as np
import pytest

from oracle import eigen, model, observables, philox, sampling, tca

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- RNG
@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((12345, 0), (7, 11, 2, 3)),
                                     ((2**64 - 1, 99), (2**64 - 1, 5, 1, 0)),
                                     ((42, 0), (3, 1023, 0, 17))])
def test_philox_matches_numpy(key, ctr):
    ours = philox.philox4x64(key, ctr)
    c = list(ctr)
    # numpy advances the 256-bit counter before producing a block
    v = c[0] + (c[1] << 64) + (c[2] << 128) + (c[3] << 192) - 1
    v %= 1 << 256
    c = [(v >> (64 * i)) & philox.MASK64 for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    assert [int(x) for x in bg.random_raw(4)] == list(ours)


def test_uniform_ranges():
    assert sampling.u53(0) == 0.0
    assert sampling.u53(2**64 - 1) == 1.0 - 2.0 ** -53
    assert sampling.v52(0) == -1.0
    assert sampling.v52(2**64 - 1) == 1.0 - 2.0 ** -52


def test_sphere_sampler_moments():
    pts = np.array([sampling.sphere_point(7, 3, i, 0) for i in range(20000)])
    assert np.max(np.abs(np.linalg.norm(pts, axis=1) - 1.0)) < 4e-16
    se = math.sqrt(1.0 / 3.0 / len(pts))
    assert np.all(np.abs(pts.mean(0)) < 5 * se)
    m2 = (pts ** 2).mean(0)
    assert np.all(np.abs(m2 - 1.0 / 3.0) < 0.015)
    # z is uniform on [-1, 1] for a uniform point on S^2 (Archimedes)
    h, _ = np.histogram(pts[:, 2], bins=10, range=(-1, 1))
    assert np.all(np.abs(h / len(pts) - 0.1) < 0.012)


def test_size_class_uniform():
    ks = [sampling.size_class(5, 1, i, 3) for i in range(6000)]
    c = np.bincount(ks, minlength=3) / 6000
    assert np.all(np.abs(c - 1 / 3) < 0.03)


# ---------------------------------------------------------------- Hamiltonian
def _rand_spins(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("Lc", [2, 3, 4, 5, 8])
def test_hamiltonian_invariants(Lc):
    Nc = Lc * Lc
    t, JH = 1.0, 8.0
    S = _rand_spins(Nc, Lc)
    H = model.cluster_hamiltonian(S, Lc, t, JH)
    assert np.array_equal(H, H.conj().T)
    assert abs(np.trace(H)) < 1e-14
    hop = (16 if Lc == 2 else 8) * Nc * t * t
    assert abs(np.linalg.norm(H) ** 2 - (hop + Nc * JH * JH / 2)) < 1e-10
    S2 = S.copy(); S2[0] = _rand_spins(1, 99)[0]
    D = model.cluster_hamiltonian(S2, Lc, t, JH) - H
    nz = np.argwhere(np.abs(D) > 0)
    assert nz.size and nz.max() <= 1               # only site 0's 2x2 block
    assert np.linalg.matrix_rank(D) <= 2


@pytest.mark.parametrize("Lc", [2, 3, 4, 8])
def test_ferromagnet_closed_form(Lc):
    d = _rand_spins(1, Lc + 10)[0]
    S = np.tile(d, (Lc * Lc, 1))
    H = model.cluster_hamiltonian(S, Lc, 1.0, 8.0)
    ref = model.band_closed_form(Lc, 1.0, 8.0, "ferro")
    assert np.max(np.abs(eigen.eigvals_lapack(H) - ref)) < 1e-12
    if Lc <= 4:
        assert np.max(np.abs(eigen.eigvals_jacobi(H) - ref)) < 1e-12


@pytest.mark.parametrize("Lc", [2, 4, 6, 8])
def test_neel_closed_form(Lc):
    d = _rand_spins(1, Lc + 20)[0]
    S = np.array([d if ((l % Lc) + (l // Lc)) % 2 == 0 else -d for l in range(Lc * Lc)])
    H = model.cluster_hamiltonian(S, Lc, 1.0, 8.0)
    ref = model.band_closed_form(Lc, 1.0, 8.0, "neel")
    assert np.max(np.abs(eigen.eigvals_lapack(H) - ref)) < 1e-12


def test_limits_t0_and_jh0():
    Lc = 4
    S = _rand_spins(16, 3)
    e = eigen.eigvals_lapack(model.cluster_hamiltonian(S, Lc, 0.0, 8.0))
    assert np.max(np.abs(e - np.repeat([-4.0, 4.0], 16))) < 1e-13
    e = eigen.eigvals_lapack(model.cluster_hamiltonian(S, Lc, 1.0, 0.0))
    k = 2 * np.pi * np.arange(Lc) / Lc
    band = np.sort(np.repeat((-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel(), 2))
    assert np.max(np.abs(e - band)) < 1e-13


@pytest.mark.parametrize("Lc", [4, 8])
def test_spectral_invariants_random(Lc):
    S = _rand_spins(Lc * Lc, 50 + Lc)
    H = model.cluster_hamiltonian(S, Lc, 1.0, 8.0)
    e = eigen.eigvals_lapack(H)
    assert np.max(np.abs(e + e[::-1])) < 1e-12             # bipartite: eps <-> -eps
    assert np.max(np.abs(e)) <= 4.0 + 4.0 + 1e-12
    assert abs(np.sum(e ** 2) - np.linalg.norm(H) ** 2) < 1e-9
    # global rotation and J_H -> -J_H leave the spectrum unchanged
    q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    e_rot = eigen.eigvals_lapack(model.cluster_hamiltonian(S @ q.T, Lc, 1.0, 8.0))
    e_neg = eigen.eigvals_lapack(model.cluster_hamiltonian(S, Lc, 1.0, -8.0))
    assert np.max(np.abs(e_rot - e)) < 1e-12
    assert np.max(np.abs(e_neg - e)) < 1e-12


def test_odd_cluster_breaks_symmetry():
    S = _rand_spins(9, 4)
    e = eigen.eigvals_lapack(model.cluster_hamiltonian(S, 3, 1.0, 8.0))
    assert np.max(np.abs(e + e[::-1])) > 1e-3


@pytest.mark.parametrize("n,seed", [(6, 0), (17, 1), (32, 2)])
def test_jacobi_vs_lapack_random_hermitian(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A = A + A.conj().T
    assert np.max(np.abs(eigen.eigvals_jacobi(A) - eigen.eigvals_lapack(A))) < 1e-12


def test_jacobi_vs_lapack_cluster_8x8():
    S = _rand_spins(64, 77)
    H = model.cluster_hamiltonian(S, 8, 1.0, 8.0)
    assert np.max(np.abs(eigen.eigvals_jacobi(H) - eigen.eigvals_lapack(H))) < 1e-12


# ---------------------------------------------------------------- free energy
def test_free_energy_matches_naive_definition():
    e = np.linspace(-6, 6, 41)
    for T, mu in [(1.0, 0.0), (0.5, 0.3), (2.0, -1.0)]:
        naive = -T * np.sum(np.log(1.0 + np.exp(-(e - mu) / T)))
        assert abs(tca.free_energy(e, T, mu) - naive) < 1e-12 * max(1, abs(naive))


def test_free_energy_low_T_limit():
    e = np.array([-3.0, -1.0, -0.5, 0.5, 2.0])
    F = tca.free_energy(e, 1e-3, 0.0)
    assert abs(F - (-4.5)) < 1e-100 + 5 * 1e-3 * math.exp(-0.5 / 1e-3)


def test_ferro_free_energy_closed_form():
    Lc, T, mu = 4, 0.05, 0.0
    S = np.tile([0.0, 0.0, 1.0], (16, 1))
    e = eigen.eigvals_lapack(model.cluster_hamiltonian(S, Lc, 1.0, 8.0))
    k = 2 * np.pi * np.arange(Lc) / Lc
    eps = (-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel()
    ref = 0.0
    for x in np.concatenate([eps - 4, eps + 4]):
        ref += -T * np.logaddexp(0.0, -x / T)
    assert abs(tca.free_energy(e, T, mu) - ref) < 1e-11


def _cluster_dF(C, s_new, T, Lc=4, t=1.0, JH=8.0, mu=0.0):
    e0 = eigen.eigvals_lapack(model.cluster_hamiltonian(C, Lc, t, JH))
    C2 = C.copy(); C2[0] = s_new
    e1 = eigen.eigvals_lapack(model.cluster_hamiltonian(C2, Lc, t, JH))
    return tca.free_energy(e1, T, mu) - tca.free_energy(e0, T, mu)


def test_dF_antisymmetric_and_rotation_invariant():
    C = _rand_spins(16, 8)
    s = _rand_spins(1, 9)[0]
    d1 = _cluster_dF(C, s, 0.05)
    C2 = C.copy(); C2[0] = s
    d2 = _cluster_dF(C2, C[0], 0.05)
    assert abs(d1 + d2) < 1e-11
    q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    d3 = _cluster_dF(C @ q.T, q @ s, 0.05)
    assert abs(d3 - d1) < 1e-11
    assert abs(d1) > 1e-4


def test_dF_vanishes_without_coupling():
    C = _rand_spins(16, 10)
    s = _rand_spins(1, 11)[0]
    assert _cluster_dF(C, s, 0.05, JH=0.0) == 0.0
    assert abs(_cluster_dF(C, s, 0.05, t=0.0)) < 1e-12


# ---------------------------------------------------------------- schedule
def test_fig3_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "fig3_boundary_clusters.json")))
    N, Nc = g["N"], g["Nc"]
    deps = {}
    for r in range(1, N + 1):                      # 1-based update site, sweep left to right
        cl = [((r - 1 + a) % N) + 1 for a in range(Nc)]
        deps[r] = sorted(s for s in cl if s < r)
    indep = [r for r in deps if not deps[r]]
    assert indep == g["independent_rows"]
    assert {str(r): deps[r] for r in deps if deps[r]} == g["row_dependencies"]
    assert len(indep) == N - Nc + 1 == g["n_independent"]
    assert N - len(indep) == Nc - 1 == g["n_boundary"]
    # the two-block split: no cluster of a block contains a site of the same
    # block that is visited earlier
    for blk in g["blocks"]:
        for r in blk:
            assert not [s for s in deps[r] if s in blk]


@pytest.mark.parametrize("L,Lc,ok", [(8, 4, True), (8, 5, True), (32, 8, True), (100, 6, True),
                                     (100, 10, True), (8, 6, False), (6, 4, True)])
def test_block_independence(L, Lc, ok):
    bad = 0
    for K in range(4):
        sites = model.block_sites(L, K)
        seen = set()
        for p in sites:
            bad += len(seen.intersection(model.cluster_sites(L, Lc, p)))
            seen.add(p)
    assert (bad == 0) == ok


def test_sweep_order_covers_lattice():
    o = model.sweep_order(10)
    assert sorted(o) == list(range(100))


def test_sequential_equals_block_batched():
    prm = tca.Params(L=8, Lc=4, JAF=0.05, seed=3)
    S0 = tca.initial_spins(8, 3)
    Sa, ra = tca.sweep_sequential(S0, prm, 0.05, 0)
    Sb, rb = tca.sweep_block_batched(S0, prm, 0.05, 0)
    assert np.array_equal(Sa, Sb)
    assert [(r["site"], r["dF"], r["accept"]) for r in ra] == [(r["site"], r["dF"], r["accept"]) for r in rb]
    assert 0 < sum(r["accept"] for r in ra) < 64


def test_heisenberg_limit_matches_textbook_metropolis():
    """J_H = 0: dF == 0 exactly and the chain is the classical Heisenberg
    Metropolis with coupling J_AF; compare with an independent vectorized
    implementation of that textbook algorithm."""
    L, seed, T, J = 8, 5, 0.3, 1.0
    prm = tca.Params(L=L, Lc=4, JH=0.0, JAF=J, seed=seed)
    S = tca.initial_spins(L, seed)
    Sref = S.reshape(L, L, 3).copy()                   # [y, x]
    for sw in range(2):
        S, recs = tca.sweep_sequential(S, prm, T, sw)
        assert all(r["dF"] == 0.0 for r in recs)
        for K in range(4):
            x0, y0 = (L // 2) * (K & 1), (L // 2) * (K >> 1)
            for j in range(L // 2):
                for i in range(L // 2):
                    x, y = x0 + i, y0 + j
                    s_new = np.array(sampling.proposal(seed, sw, x + L * y))
                    nb = Sref[y, (x - 1) % L] + Sref[y, (x + 1) % L] + Sref[(y - 1) % L, x] + Sref[(y + 1) % L, x]
                    dE = J * np.dot(s_new - Sref[y, x], nb)
                    u = sampling.metropolis_uniforms(seed, sw, x + L * y)[0]
                    if dE <= 0 or u < np.exp(-dE / T):
                        Sref[y, x] = s_new
        assert np.array_equal(S, Sref.reshape(L * L, 3))


def test_exact_enumeration_2x2_flip_chain():
    """Lc = L = 2 (the traveling cluster is the whole lattice: ED+MC limit),
    spins restricted to +-z with flip proposals: the empirical distribution of
    the chain matches exp(-(F + E_cl)/T)/Z over the 16 states."""
    L, Lc, T, JAF, seed = 2, 2, 1.0, 0.3, 11
    prm = tca.Params(L=L, Lc=Lc, JAF=JAF, seed=seed)

    def energy(bits):
        S = np.zeros((4, 3)); S[:, 2] = [1 - 2 * ((bits >> i) & 1) for i in range(4)]
        e = eigen.eigvals_lapack(model.cluster_hamiltonian(S, Lc, 1.0, 8.0))
        return tca.free_energy(e, T, 0.0) + model.classical_energy(S, L, JAF)

    E = np.array([energy(b) for b in range(16)])
    w = np.exp(-(E - E.min()) / T); w /= w.sum()
    S = np.zeros((4, 3)); S[:, 2] = 1.0
    counts = np.zeros(16)
    nsw = 6000
    for sw in range(nsw):
        for p in model.sweep_order(L):
            s_new = -S[p]
            dF = tca.cluster_dF(S, prm, p, s_new, T, Lc)
            dE = dF + model.classical_delta(S, L, p, s_new, JAF)
            u = sampling.metropolis_uniforms(seed, sw, p)[0]
            if tca.metropolis_accept(dE, u, T):
                S[p] = s_new
        bits = sum(int(S[i, 2] < 0) << i for i in range(4))
        counts[bits] += 1
    emp = counts / nsw
    assert 0.5 * np.sum(np.abs(emp - w)) < 0.04
    assert w.max() > 2 * w.min()          # the law is far from uniform


# ---------------------------------------------------------------- S(q)
def test_structure_factor_pins():
    L = 6
    S = np.tile([0.0, 1.0, 0.0], (L * L, 1))
    sq = observables.sq_dft(S, L)
    assert abs(sq[0, 0] - 1.0) < 1e-14 and abs(sq.sum() - 1.0) < 1e-13
    S = tca.initial_spins(L, 1, "neel")
    sq = observables.sq_dft(S, L)
    assert abs(sq[L // 2, L // 2] - 1.0) < 1e-14
    S = tca.initial_spins(L, 4)
    a = observables.sq_dft(S, L)
    b = observables.sq_double_sum(S, L)
    assert np.max(np.abs(a - b)) < 1e-14
    assert abs(a.sum() - 1.0) < 1e-13
