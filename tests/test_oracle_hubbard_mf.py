"""Pins of the Hubbard mean-field cluster model (Eq. (1)) in the oracle:
closed forms, limits and invariants (CPU)."""
import numpy as np
import pytest

from oracle import eigen, hubbard_mf as hmf, model
from oracle import tca as otca

CASES = [(2, 2), (3, 2), (4, 2), (2, 3), (3, 3), (4, 3)]  # (Lc, d)


def _random_fields(Nc, seed, lo=0.0, hi=1.5):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(Nc, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * rng.uniform(lo, hi, size=(Nc, 1))


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


@pytest.mark.parametrize("Lc,d", CASES)
def test_hermitian_of_dimension_2_Nc(Lc, d):
    H = hmf.cluster_hamiltonian(_random_fields(Lc ** d, 1), Lc, d, 1.0, 8.0)
    assert H.shape == (2 * Lc ** d, 2 * Lc ** d)
    assert np.array_equal(H, H.conj().T)


def test_paper_benchmark_cluster_is_128():
    """The 3D benchmark cluster N_c = 4^3 gives 128 x 128 matrices."""
    H = hmf.cluster_hamiltonian(np.zeros((64, 3)), 4, 3, 1.0, 8.0)
    assert H.shape == (128, 128)


@pytest.mark.parametrize("Lc,d", CASES)
def test_zero_field_is_band_plus_half_U(Lc, d):
    U = 6.0
    w = eigen.eigvals_lapack(hmf.cluster_hamiltonian(np.zeros((Lc ** d, 3)), Lc, d, 1.0, U))
    b = hmf.band(Lc, d, 1.0) + U / 2
    assert np.allclose(w, np.sort(np.concatenate([b, b])), atol=1e-12)


@pytest.mark.parametrize("Lc,d", CASES)
def test_uniform_field_splits_the_band(Lc, d):
    U, M = 8.0, 0.7
    nhat = np.array([0.3, -0.5, 0.81])
    nhat /= np.linalg.norm(nhat)
    m = np.tile(M * nhat, (Lc ** d, 1))
    w = eigen.eigvals_lapack(hmf.cluster_hamiltonian(m, Lc, d, 1.0, U))
    b = hmf.band(Lc, d, 1.0) + U / 2
    ref = np.sort(np.concatenate([b - U * M / 2, b + U * M / 2]))
    assert np.allclose(w, ref, atol=1e-12)


@pytest.mark.parametrize("Lc,d", CASES)
def test_atomic_limit(Lc, d):
    U = 5.0
    m = _random_fields(Lc ** d, 3)
    w = eigen.eigvals_lapack(hmf.cluster_hamiltonian(m, Lc, d, 0.0, U))
    r = np.linalg.norm(m, axis=1)
    ref = np.sort(np.concatenate([U / 2 - U * r / 2, U / 2 + U * r / 2]))
    assert np.allclose(w, ref, atol=1e-12)


@pytest.mark.parametrize("Lc,d", CASES)
def test_global_rotation_leaves_the_spectrum(Lc, d):
    m = _random_fields(Lc ** d, 4)
    R = _rotation(5)
    w1 = eigen.eigvals_lapack(hmf.cluster_hamiltonian(m, Lc, d, 1.0, 8.0))
    w2 = eigen.eigvals_lapack(hmf.cluster_hamiltonian(m @ R.T, Lc, d, 1.0, 8.0))
    assert np.allclose(w1, w2, atol=1e-11)


@pytest.mark.parametrize("Lc,d", [(3, 2), (4, 2), (3, 3), (4, 3)])
def test_trace_and_frobenius_norm(Lc, d):
    """tr H = U Nc (the Pauli part is traceless); |H|_F^2 = sum of the on-site
    blocks (U/2)^2 (2 + 2|m_i|^2) plus 2 * 2d * Nc t^2 of hopping (Lc >= 3, where
    the 2d neighbours are distinct)."""
    U, t = 7.0, 1.3
    Nc = Lc ** d
    m = _random_fields(Nc, 6)
    H = hmf.cluster_hamiltonian(m, Lc, d, t, U)
    assert abs(np.trace(H).real - U * Nc) < 1e-12 * U * Nc
    onsite = np.sum((U / 2) ** 2 * (2.0 + 2.0 * np.sum(m * m, axis=1)))
    assert abs(np.sum(np.abs(H) ** 2) - (onsite + 2 * 2 * d * Nc * t * t)) < 1e-10 * onsite


@pytest.mark.parametrize("Lc", [2, 3, 4])
def test_unit_fields_give_the_double_exchange_matrix(Lc):
    """For unit vectors the on-site block is the double-exchange one with
    J_H = U plus (U/2) I."""
    U = 8.0
    S = _random_fields(Lc * Lc, 7, 1.0, 1.0)
    H = hmf.cluster_hamiltonian(S, Lc, 2, 1.0, U)
    ref = model.cluster_hamiltonian(S, Lc, 1.0, U) + (U / 2) * np.eye(2 * Lc * Lc)
    assert np.allclose(H, ref, atol=1e-14, rtol=0)


def test_classical_energy_and_delta():
    U = 8.0
    m = _random_fields(9, 8)
    e = hmf.classical_energy(m, U)
    assert abs(e - 0.25 * U * sum(float(np.dot(x, x)) - 1.0 for x in m)) < 1e-12
    m2 = m.copy()
    m2[4] = [0.1, 0.2, -0.3]
    assert abs(hmf.classical_energy(m2, U) - e - hmf.classical_delta(m[4], m2[4], U)) < 1e-12


@pytest.mark.parametrize("Lc,d", [(2, 2), (4, 2), (2, 3)])
def test_delta_energy_zero_antisymmetric_rotation_invariant(Lc, d):
    U, T, mu = 8.0, 0.1, 0.3
    m = _random_fields(Lc ** d, 9)
    mnew = np.array([0.2, -0.9, 0.4])
    f = dict(free_energy=otca.free_energy, eigvals=eigen.eigvals_lapack)
    assert hmf.delta_energy(m, m[0], Lc, d, 1.0, U, T, mu, **f) == 0.0
    fwd = hmf.delta_energy(m, mnew, Lc, d, 1.0, U, T, mu, **f)
    m2 = m.copy()
    m2[0] = mnew
    back = hmf.delta_energy(m2, m[0], Lc, d, 1.0, U, T, mu, **f)
    assert abs(fwd + back) < 1e-10 * max(1.0, abs(fwd))
    R = _rotation(10)
    rot = hmf.delta_energy(m @ R.T, R @ mnew, Lc, d, 1.0, U, T, mu, **f)
    assert abs(rot - fwd) < 1e-9 * max(1.0, abs(fwd))
