"""Green's function columns and the real-space transmission (oracle).

Eq. 7: with diagonal coupling matrices only the block of G between the left
and the right absorbing regions is needed,
    T(E) = sum_{i in L, j in R} |G_ij(E)|^2 Gamma_R,jj Gamma_L,ii .
The absorbing potential W enters the operator as +iW (Eq. 4), i.e. as the
anti-Hermitian part -Im(Sigma) of a self-energy, whose coupling matrix is
Gamma = i(Sigma - Sigma^+) = 2W.  Substituting Gamma = 2W gives the factor 4
used throughout: T(E) = 4 sum W_L,i W_R,j |G_ij|^2.  (The exact 1-D lead pin
in the tests fixes this factor.)

Three interchangeable routes compute the same columns g_j = A(E)^-1 e_j:
dense inversion (numpy), sparse LU (scipy splu) and a Krylov solve from
scipy whose true residual ||b - A x|| / ||b|| is checked afterwards.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import cap_diagonals, hamiltonian, operator_A


def _support(wire, side):
    planes = wire.cap_left if side == "L" else wire.cap_right
    per = wire.nx * wire.ny
    idx = [np.arange(z * per, (z + 1) * per) for z in range(wire.nz) if planes[z] > 0]
    return np.concatenate(idx).astype(np.int64)


def solve_iterative(A, b, tol=1e-12, maxiter=200000):
    """x = A^-1 b by scipy Krylov solvers; raises unless the TRUE relative
    residual ||b - A x||_2 / ||b||_2 <= tol."""
    nb = np.linalg.norm(b)
    x = None
    for method in ("bicgstab", "gmres"):
        x0 = x
        if method == "bicgstab":
            x, _ = spla.bicgstab(A, b, x0=x0, rtol=tol * 0.1, atol=0.0, maxiter=maxiter)
        else:
            x, _ = spla.gmres(A, b, x0=x0, rtol=tol * 0.1, atol=0.0, restart=300,
                              maxiter=maxiter // 300 + 1)
        res = np.linalg.norm(b - A @ x) / nb
        if res <= tol:
            return x, res
    raise RuntimeError(f"oracle iterative solve missed tol: residual {res:.3e}")


def green_columns(wire, E, cols, rows=None, method="auto", H=None, tol=1e-12):
    """G(E)[rows, cols] (complex128), columns g_j = A(E)^-1 e_j."""
    cols = np.asarray(cols, dtype=np.int64)
    A = operator_A(wire, E, H)
    N = wire.N
    if method == "auto":
        method = "dense" if N <= 4096 else ("splu" if N <= 70000 else "iterative")
    if method == "dense":
        B = np.zeros((N, len(cols)), complex)
        B[cols, np.arange(len(cols))] = 1.0
        X = np.linalg.solve(A.toarray(), B)
    elif method == "splu":
        lu = spla.splu(A)
        B = np.zeros((N, len(cols)), complex)
        B[cols, np.arange(len(cols))] = 1.0
        X = lu.solve(B)
    elif method == "iterative":
        A = A.tocsr()
        X = np.empty((N, len(cols)), complex)
        for k, j in enumerate(cols):
            b = np.zeros(N, complex)
            b[j] = 1.0
            X[:, k], _ = solve_iterative(A, b, tol)
    else:
        raise ValueError(method)
    return X if rows is None else X[np.asarray(rows, dtype=np.int64)]


def column_transmissions(wire, E, cols=None, method="auto", H=None, direction="RL"):
    """Per-column t_j(E) = 4 W_R,j sum_{i in L} W_L,i |G_ij|^2 (Eq. 7).

    direction "RL": columns j on the right CAP, rows i on the left CAP;
    direction "LR": the roles swapped (reciprocity check).
    """
    wl, wr = cap_diagonals(wire)
    src, dst = ("R", "L") if direction == "RL" else ("L", "R")
    w_src = wr if src == "R" else wl
    w_dst = wl if dst == "L" else wr
    if cols is None:
        cols = _support(wire, src)
    rows = _support(wire, dst)
    G = green_columns(wire, E, cols, rows=rows, method=method, H=H)
    return 4.0 * w_src[cols] * (w_dst[rows][:, None] * np.abs(G) ** 2).sum(axis=0)


def transmission(wire, energies=None, method="auto", direction="RL"):
    """T(E) for every energy (Eq. 7 with the factor 4)."""
    if energies is None:
        energies = wire.energies
    H = hamiltonian(wire)
    return np.array([column_transmissions(wire, E, method=method, H=H,
                                          direction=direction).sum()
                     for E in energies])
