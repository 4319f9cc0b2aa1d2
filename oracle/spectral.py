"""The paper's complex-energy diagonalisation route (oracle).

Sec. II.C, Eqs. 8-13: right eigenvectors U of the complex symmetric
H_op = H - iW (Eq. 8) are complex orthogonal, so after normalising each
column to U_i^T U_i = 1 the inverse is U^T.  Then G(E) = U diag(1/(E-eps)) U^T
(Eqs. 9-10) and
    T(E) = sum_{i,j} Gt_L,ij Gt_R,ji / ((E - eps_j)(E - eps_i^*))      (Eq. 13)
with Gt_L = U^+ Gamma_L U and Gt_R = U^T Gamma_R U^* (Eq. 12).  Here all
eigenpairs are kept (the fraction p of Sec. II.C equal to 1), so the route is
exact; Gamma = 2W as in the real-space route.
"""

from __future__ import annotations

import numpy as np

from .operator import cap_diagonals, hamiltonian


def _complex_orthonormalise(eps, U, cluster_tol=1e-8):
    """Make U^T U = 1 (no conjugation).

    Eigenvectors of distinct eigenvalues of a complex symmetric matrix are
    already complex orthogonal; inside a cluster of (numerically) equal
    eigenvalues any basis is returned, so it is re-orthogonalised there with
    the factorisation M = U_c^T U_c = L L^T (Cholesky without conjugation),
    U_c <- U_c L^-T.
    """
    U = U.copy()
    order = np.argsort(eps.real + 1e-3 * eps.imag)
    scale = max(1.0, float(np.max(np.abs(eps))))
    start = 0
    while start < len(order):
        stop = start + 1
        while stop < len(order) and abs(eps[order[stop]] - eps[order[start]]) < cluster_tol * scale:
            stop += 1
        idx = order[start:stop]
        M = U[:, idx].T @ U[:, idx]
        n = len(idx)
        L = np.zeros((n, n), complex)
        for j in range(n):
            d = M[j, j] - np.dot(L[j, :j], L[j, :j])
            L[j, j] = np.sqrt(d)
            for i in range(j + 1, n):
                L[i, j] = (M[i, j] - np.dot(L[i, :j], L[j, :j])) / L[j, j]
        U[:, idx] = np.linalg.solve(L, U[:, idx].T).T  # U_c L^-T
        start = stop
    return U


def transmission_spectral(wire, energies=None, keep=None):
    """T(E) from the complex eigenpairs of H - iW.

    keep: optional fraction p in (0, 1]; keeps the eigenpairs with real parts
    closest to the middle of the energy window (the truncation of Sec. II.C).
    """
    if energies is None:
        energies = wire.energies
    H = hamiltonian(wire).toarray()
    wl, wr = cap_diagonals(wire)
    Hop = H - 1j * np.diag(wl + wr)  # Eq. 4
    eps, U = np.linalg.eig(Hop)  # Eq. 8
    U = _complex_orthonormalise(eps, U)
    if keep is not None and keep < 1.0:
        mid = 0.5 * (np.min(energies) + np.max(energies))
        n_keep = max(1, int(round(keep * len(eps))))
        order = np.argsort(np.abs(eps.real - mid))[:n_keep]
        eps, U = eps[order], U[:, order]
    gl = 2.0 * wl
    gr = 2.0 * wr
    GtL = U.conj().T @ (gl[:, None] * U)  # Eq. 12
    GtR = U.T @ (gr[:, None] * U.conj())
    M = GtL * GtR.T  # M_ij = GtL_ij GtR_ji
    out = []
    for E in energies:
        a = 1.0 / (E - eps)  # 1/(E - eps_j)
        b = 1.0 / (E - eps.conj())  # 1/(E - eps_i^*)
        # Eq. 13: sum_ij GtL_ij GtR_ji a_j b_i
        out.append(np.real(b @ M @ a))
    return np.array(out)
