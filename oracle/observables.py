"""Spin structure factor, Eq. (2) of the paper.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

S(q) = (1/N^2) sum_{i,j} exp(i q.(r_i - r_j)) <m_i . m_j>, here for one
configuration (the thermal average is the caller's mean over stored
configurations), on the L x L grid q = 2 pi (nx, ny)/L.

``sq_double_sum`` is the definition written out (O(N^2) per q, small
lattices).  ``sq_dft`` uses the identity
sum_{ij} e^{iq(ri-rj)} S_i.S_j = sum_a |sum_i S_i^a e^{iq ri}|^2 with a
library FFT as one step.  Pinned by: ferromagnet S(0) = 1, Neel
S(pi,pi) = 1, sum_q S(q) = 1 for unit spins (Parseval), and
double-sum == DFT.
"""
import numpy as np


def sq_double_sum(S, L: int):
    S = np.asarray(S, dtype=np.float64)
    N = L * L
    xs = np.arange(N) % L
    ys = np.arange(N) // L
    G = S @ S.T                                  # m_i . m_j
    out = np.zeros((L, L))
    for ny in range(L):
        for nx in range(L):
            qx, qy = 2 * np.pi * nx / L, 2 * np.pi * ny / L
            ph = np.exp(1j * (qx * xs + qy * ys))
            out[ny, nx] = np.real(ph @ G @ np.conj(ph)) / (N * N)
    return out


def sq_dft(S, L: int):
    S = np.asarray(S, dtype=np.float64)
    N = L * L
    tot = np.zeros((L, L))
    for a in range(3):
        f = S[:, a].reshape(L, L)                 # [y, x]
        F = np.fft.fft2(f)                        # sum e^{-iq r}; |.|^2 is sign-free
        tot += np.abs(F) ** 2
    return tot / (N * N)
