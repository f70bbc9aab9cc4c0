"""Cluster Hamiltonian and classical energy of the Hubbard mean-field
spin-fermion model the paper benchmarks (Sec. IV, Eq. (1)), in two or three
dimensions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  First step of widening the
batched path to the paper's own model: the GPU path does not implement it yet.

Model (Eq. (1), SU(2)-invariant Hartree-Fock decoupling of the Hubbard model
with the mean fields m_i treated as classical vectors of free length, and
<n_i> = 1 at half filling as the paper sets):
    H = -t sum_<ij>,s c+_is c_js + (U/2) sum_i (n_i - m_i . sigma_i)
        + (U/4) sum_i (|m_i|^2 - 1) - mu sum_i n_i.
The fermionic on-site 2x2 block of site i is therefore
    (U/2) I - (U/2) [[m_z, m_x - i m_y], [m_x + i m_y, -m_z]]
and the c-number (U/4)(|m_i|^2 - 1) is the classical energy.  As for the
double-exchange model in ``model.py``, mu enters the grand potential
(eigenvalue minus mu), not the matrix.

Geometry: an Lc^d cluster (d = 2 or 3) anchored at its corner, index
l = a + Lc b (+ Lc^2 c), periodic in itself; each of the 2d directions adds -t,
so the band is -2t sum_dims cos(k) on the Lc^d momentum grid for every Lc >= 2
(the paper's 3D benchmark uses Lc = 4, n = 2 * 4^3 = 128).  Basis index 2l + s.

Pinned by the closed forms m = 0 (band + U/2, each level twice), uniform m
(band + U/2 -+ U|m|/2), t = 0 (U/2 -+ U|m_i|/2 per site), invariance of the
spectrum under a global rotation of the m_i, trace and Frobenius norm, and the
reduction to the double-exchange cluster matrix for unit vectors (J_H = U, the
shift U/2 aside).
"""
import numpy as np


def cluster_size(Lc: int, d: int) -> int:
    assert d in (2, 3) and Lc >= 2
    return Lc ** d


def cluster_coords(Lc: int, d: int, l: int):
    return [(l // Lc ** k) % Lc for k in range(d)]


def cluster_index(Lc: int, coords) -> int:
    return sum((c % Lc) * Lc ** k for k, c in enumerate(coords))


def cluster_neighbours(Lc: int, d: int, l: int):
    """The 2d periodic neighbours of cluster site l (+e_k, -e_k for k = 0..d-1)."""
    x = cluster_coords(Lc, d, l)
    out = []
    for k in range(d):
        for step in (1, -1):
            y = list(x)
            y[k] += step
            out.append(cluster_index(Lc, y))
    return out


def cluster_hamiltonian(m, Lc: int, d: int, t: float, U: float):
    """Dense 2Nc x 2Nc complex Hermitian cluster matrix for the mean fields
    ``m`` (Nc x 3, cluster order) of Eq. (1)."""
    m = np.asarray(m, dtype=np.float64)
    Nc = cluster_size(Lc, d)
    assert m.shape == (Nc, 3)
    H = np.zeros((2 * Nc, 2 * Nc), dtype=np.complex128)
    for l in range(Nc):
        for q in cluster_neighbours(Lc, d, l):
            for s in range(2):
                H[2 * l + s, 2 * q + s] += -t
        mx, my, mz = m[l]
        h = 0.5 * U
        H[2 * l, 2 * l] += h - h * mz
        H[2 * l + 1, 2 * l + 1] += h + h * mz
        H[2 * l, 2 * l + 1] += -h * complex(mx, -my)
        H[2 * l + 1, 2 * l] += -h * complex(mx, my)
    return H


def band(Lc: int, d: int, t: float):
    """Cluster band -2t sum_k cos(2 pi n_k / Lc) over the Lc^d momentum grid."""
    ks = 2.0 * np.pi * np.arange(Lc) / Lc
    grids = np.meshgrid(*([ks] * d), indexing="ij")
    return (-2.0 * t * sum(np.cos(g) for g in grids)).ravel()


def classical_energy(m, U: float) -> float:
    """(U/4) sum_i (|m_i|^2 - 1)."""
    m = np.asarray(m, dtype=np.float64)
    return 0.25 * U * float(np.sum(np.sum(m * m, axis=1) - 1.0))


def classical_delta(m_old, m_new, U: float) -> float:
    """Change of the classical energy when one mean field m_old -> m_new."""
    a = float(np.dot(m_old, m_old))
    b = float(np.dot(m_new, m_new))
    return 0.25 * U * (b - a)


def delta_energy(m_cluster, m_new0, Lc: int, d: int, t: float, U: float, T: float, mu: float,
                 free_energy, eigvals):
    """Energy change of replacing the update site's field (cluster site 0) by
    m_new0: grand-potential difference of the two cluster matrices plus the
    classical term.  ``free_energy(eigs, T, mu)`` and ``eigvals(H)`` are the
    oracle's own routines."""
    m_cluster = np.asarray(m_cluster, dtype=np.float64)
    m_new = m_cluster.copy()
    m_new[0] = m_new0
    F_old = free_energy(eigvals(cluster_hamiltonian(m_cluster, Lc, d, t, U)), T, mu)
    F_new = free_energy(eigvals(cluster_hamiltonian(m_new, Lc, d, t, U)), T, mu)
    return (F_new - F_old) + classical_delta(m_cluster[0], m_new0, U)
