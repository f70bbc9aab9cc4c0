"""Lattice, traveling cluster and Hamiltonian of the double-exchange
spin-fermion model.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Geometry (Sec. II(b), Sec. II(c); Fig. 1; cluster of the same geometry as the
lattice with its own periodic boundary conditions):
* L x L periodic square lattice, site index p = x + L*y.
* The traveling cluster of update site p = (x, y) is the Lc x Lc patch of
  sites ((x + a) mod L, (y + b) mod L), a, b in [0, Lc), with cluster index
  l = a + Lc*b.  The update site is the cluster's corner l = 0 (the "leftmost"
  choice of Sec. III(a) and Sec. VII(b)).
* The cluster is periodic in itself: its hopping links l to the four sites
  (a +- 1 mod Lc, b) and (a, b +- 1 mod Lc).  Each of the four directions adds
  -t, so when Lc == 2 the +x and -x neighbours coincide and the link carries
  -2t; this keeps the cluster band equal to -2t(cos kx + cos ky) on the
  Lc x Lc momentum grid for every Lc >= 2.

Hamiltonian (the paper benchmarks the Hubbard mean-field model, Eq. (1), and
cites spin-fermion models for manganites without writing them; reading used
here, the double-exchange model with classical unit spins S_i):
    H = -t sum_<ij>,s c+_is c_js  -  (J_H/2) sum_i S_i . (c+_i sigma c_i)
        + J_AF sum_<ij> S_i . S_j
Basis index 2*l + s (s = 0 up, 1 down).  The on-site 2x2 block is
    -(J_H/2) [[S_z, S_x - i S_y], [S_x + i S_y, -S_z]].
The chemical potential enters only the free energy, not H.  The classical
superexchange term is a c-number: it is evaluated on the full lattice (the four
true neighbours of the update site, with sequential semantics), each bond once,
and never enters the cluster matrix.

Parallel blocks (Sec. III(a): 2^d blocks, four in two dimensions): quadrant
K = 0: [0,L/2)x[0,L/2), 1: [L/2,L)x[0,L/2), 2: [0,L/2)x[L/2,L),
3: [L/2,L)x[L/2,L); a sweep visits K = 0..3 in turn, raster order (y outer,
x inner) inside a block.  L must be even and 2 <= Lc <= L/2 + 1, which makes
every cluster of a block free of sites updated earlier in the same block.

Pinned by: closed-form ferromagnet and Neel spectra, t = 0 and J_H = 0
limits, trace and Frobenius invariants, Hermiticity, rank-2 support of
H_new - H_old, and a brute-force check of the block independence property.
"""
import numpy as np


def site_index(L: int, x: int, y: int) -> int:
    return (x % L) + L * (y % L)


def site_xy(L: int, p: int):
    return p % L, p // L


def cluster_sites(L: int, Lc: int, p: int):
    """Lattice sites of the cluster anchored at p, in cluster order l = a + Lc*b."""
    x, y = site_xy(L, p)
    return [site_index(L, x + a, y + b) for b in range(Lc) for a in range(Lc)]


def cluster_neighbours(Lc: int, l: int):
    """The four periodic cluster neighbours of cluster site l (+x, -x, +y, -y)."""
    a, b = l % Lc, l // Lc
    return [((a + 1) % Lc) + Lc * b, ((a - 1) % Lc) + Lc * b,
            a + Lc * ((b + 1) % Lc), a + Lc * ((b - 1) % Lc)]


def cluster_hamiltonian(spins, Lc: int, t: float, JH: float):
    """Dense 2Nc x 2Nc complex Hermitian cluster matrix for cluster spins
    ``spins`` (Nc x 3, cluster order)."""
    spins = np.asarray(spins, dtype=np.float64)
    Nc = Lc * Lc
    assert spins.shape == (Nc, 3)
    n = 2 * Nc
    H = np.zeros((n, n), dtype=np.complex128)
    for l in range(Nc):
        for m in cluster_neighbours(Lc, l):
            for s in range(2):
                H[2 * l + s, 2 * m + s] += -t
        sx, sy, sz = spins[l]
        h = -0.5 * JH
        H[2 * l, 2 * l] += h * sz
        H[2 * l + 1, 2 * l + 1] += -h * sz
        H[2 * l, 2 * l + 1] += h * complex(sx, -sy)
        H[2 * l + 1, 2 * l] += h * complex(sx, sy)
    return H


def gather_cluster(S, L: int, Lc: int, p: int):
    """C[p] of the flowchart: the classical spins of the cluster around p."""
    return np.array([S[q] for q in cluster_sites(L, Lc, p)], dtype=np.float64)


def lattice_neighbours(L: int, p: int):
    x, y = site_xy(L, p)
    return [site_index(L, x - 1, y), site_index(L, x + 1, y),
            site_index(L, x, y - 1), site_index(L, x, y + 1)]


def classical_delta(S, L: int, p: int, s_new, JAF: float) -> float:
    """Change of J_AF sum_<ij> S_i.S_j when S_p -> s_new, from the current
    state S.  Order of operations: neighbour sum (-x, +x, -y, +y), difference,
    dot product, scale."""
    nb = lattice_neighbours(L, p)
    acc = [0.0, 0.0, 0.0]
    for q in nb:
        for c in range(3):
            acc[c] = acc[c] + float(S[q][c])
    d = [float(s_new[c]) - float(S[p][c]) for c in range(3)]
    dot = d[0] * acc[0]
    dot = dot + d[1] * acc[1]
    dot = dot + d[2] * acc[2]
    return JAF * dot


def classical_energy(S, L: int, JAF: float) -> float:
    """J_AF sum over the +x and +y bond of every site of S_i . S_j."""
    S = np.asarray(S, dtype=np.float64)
    e = 0.0
    for p in range(L * L):
        x, y = site_xy(L, p)
        for q in (site_index(L, x + 1, y), site_index(L, x, y + 1)):
            e += float(np.dot(S[p], S[q]))
    return JAF * e


def block_sites(L: int, K: int):
    """Update sites of parallel block K in raster order."""
    h = L // 2
    x0 = h * (K & 1)
    y0 = h * (K >> 1)
    return [site_index(L, x0 + i, y0 + j) for j in range(h) for i in range(h)]


def sweep_order(L: int):
    """Block-major, raster-within-block visiting order of one sweep."""
    order = []
    for K in range(4):
        order.extend(block_sites(L, K))
    return order


def validate(L: int, Lc: int):
    if L < 2 or L % 2:
        raise ValueError("L must be even and >= 2")
    if Lc < 2 or Lc > L // 2 + 1:
        raise ValueError("cluster size must satisfy 2 <= Lc <= L/2 + 1")


def band_closed_form(Lc: int, t: float, JH: float, kind: str):
    """Closed-form cluster spectrum for uniform spin textures.

    kind == 'ferro': all spins equal -> eps_k -+ J_H/2 with
        eps_k = -2t(cos kx + cos ky), k = 2 pi n / Lc.
    kind == 'neel' (even Lc): staggered spins -> +-sqrt(eps_k^2 + J_H^2/4),
        each k counted once (the magnetic zone doubles the cell).
    """
    k = 2.0 * np.pi * np.arange(Lc) / Lc
    eps = (-2.0 * t * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel()
    if kind == "ferro":
        ev = np.concatenate([eps - 0.5 * JH, eps + 0.5 * JH])
    elif kind == "neel":
        r = np.sqrt(eps * eps + 0.25 * JH * JH)
        ev = np.concatenate([-r, r])
    else:
        raise ValueError(kind)
    return np.sort(ev)
