"""Eigenvalues of a dense complex Hermitian matrix.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper diagonalizes each cluster Hamiltonian exactly (Sec. II(b), Fig. 2
steps (b) and (d)) and does not name its solver.  The eigenvalues have a plain
definition, so the oracle uses two unrelated routes:

* ``eigvals_lapack``: LAPACK's divide-and-conquer Hermitian solver through
  ``numpy.linalg.eigvalsh`` (a library primitive);
* ``eigvals_jacobi``: a cyclic two-sided complex Jacobi iteration written
  here from the textbook method (Golub & Van Loan, Matrix Computations,
  Sec. 8.5: each rotation first removes the phase of a_pq with a diagonal
  unitary and then applies the real symmetric 2x2 Schur rotation).

Both return eigenvalues in ascending order.  Pinned by: closed-form spectra
of ``oracle.model``, trace/Frobenius invariants, and agreement of the two
routes with each other on random Hermitian matrices.
"""
import numpy as np


def eigvals_lapack(H):
    return np.linalg.eigvalsh(np.asarray(H, dtype=np.complex128))


def eigvals_jacobi(H, tol=1e-15, max_sweeps=60):
    A = np.array(H, dtype=np.complex128, copy=True)
    n = A.shape[0]
    scale = np.linalg.norm(A)
    if scale == 0.0:
        return np.zeros(n)
    for _ in range(max_sweeps):
        off = np.sqrt(max(np.linalg.norm(A) ** 2 - np.sum(np.abs(np.diag(A)) ** 2), 0.0))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                r = abs(apq)
                if r <= 1e-300:
                    continue
                ph = apq / r                       # e^{i phi}
                app, aqq = A[p, p].real, A[q, q].real
                tau = (aqq - app) / (2.0 * r)
                sgn = 1.0 if tau >= 0.0 else -1.0
                tt = sgn / (abs(tau) + np.sqrt(1.0 + tau * tau))
                c = 1.0 / np.sqrt(1.0 + tt * tt)
                s = tt * c
                # G = diag(1, conj(ph)) @ [[c, s], [-s, c]]
                g00, g01 = c, s
                g10, g11 = -s * np.conj(ph), c * np.conj(ph)
                cp = A[:, p].copy()
                cq = A[:, q].copy()
                A[:, p] = cp * g00 + cq * g10
                A[:, q] = cp * g01 + cq * g11
                rp = A[p, :].copy()
                rq = A[q, :].copy()
                A[p, :] = np.conj(g00) * rp + np.conj(g10) * rq
                A[q, :] = np.conj(g01) * rp + np.conj(g11) * rq
                A[p, q] = 0.0
                A[q, p] = 0.0
                A[p, p] = A[p, p].real
                A[q, q] = A[q, q].real
    return np.sort(np.diag(A).real)
