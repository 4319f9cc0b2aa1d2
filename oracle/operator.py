"""Real-space operator assembly (oracle; test infrastructure only).

Sec. II.C: in real space the Kohn-Sham matrix is sparse; its only off-diagonal
elements come from the high-order finite-difference Laplacian and from the
non-local pseudopotential inside a cutoff radius.  Sec. II.B, Eqs. 4-5: the
open-system operator adds -i*Gamma with Gamma diagonal and depending on z.

Readings of what the paper leaves open (Sec. II.C gives no stencil details):
* central difference of order 2R along each axis (star stencil), weights from
  the Taylor moment conditions (solved here in exact rational arithmetic);
* Dirichlet walls one spacing outside the first and last grid points: ghost
  values are zero, which keeps H symmetric;
* the separable projector term is sum_p E_p b_p b_p^T with real b_p.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.sparse as sp


def fd_second_derivative_weights(R: int):
    """Weights c_0..c_R of the order-2R central second derivative.

    f''(0) h^2 ~= c_0 f(0) + sum_m c_m (f(mh) + f(-mh)).  The weights are the
    unique symmetric solution of the moment conditions
    sum_{m=-R..R} c_|m| m^(2k) = 2*delta_{k,1}, k = 0..R, solved exactly with
    fractions (Gauss-Jordan elimination).  Returns a list of Fractions.
    """
    if not (1 <= R <= 12):
        raise ValueError("R out of range")
    n = R + 1
    # row k: coefficient of c_0 is m^(2k) at m=0 (1 if k==0 else 0);
    # coefficient of c_m (m>=1) is 2*m^(2k)
    A = []
    for k in range(n):
        row = [Fraction(1 if k == 0 else 0)]
        row += [Fraction(2 * m ** (2 * k)) for m in range(1, n)]
        row.append(Fraction(2 if k == 1 else 0))
        A.append(row)
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [a / pv for a in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return [A[k][n] for k in range(n)]


def second_difference_1d(n: int, R: int) -> sp.csr_matrix:
    """n x n matrix of h^2 * d^2/dx^2 with zero ghosts beyond both walls."""
    c = [float(v) for v in fd_second_derivative_weights(R)]
    diags = [np.full(n, c[0])]
    offsets = [0]
    for m in range(1, R + 1):
        if m >= n:
            break
        diags += [np.full(n - m, c[m]), np.full(n - m, c[m])]
        offsets += [m, -m]
    return sp.diags(diags, offsets, shape=(n, n), format="csr")


def kinetic_operator(nx: int, ny: int, nz: int, h: float, R: int) -> sp.csr_matrix:
    """-1/2 Laplacian on the grid; index i = ix + nx*(iy + ny*iz)."""
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    Dx = second_difference_1d(nx, R)
    Dy = second_difference_1d(ny, R)
    Dz = second_difference_1d(nz, R)
    # Kronecker order: the last factor runs fastest (x).
    lap = (sp.kron(Iz, sp.kron(Iy, Dx)) + sp.kron(Iz, sp.kron(Dy, Ix))
           + sp.kron(Dz, sp.kron(Iy, Ix)))
    return (-0.5 / (h * h) * lap).tocsr()


def kb_matrix(wire) -> sp.csr_matrix:
    """B (N x n_p) with column p = projector b_p on the grid."""
    n_p = wire.n_proj
    if n_p == 0:
        return sp.csr_matrix((wire.N, 0))
    cols = np.repeat(np.arange(n_p), np.diff(wire.kb_offsets))
    return sp.csr_matrix((wire.kb_val, (wire.kb_idx.astype(np.int64), cols)),
                         shape=(wire.N, n_p))


def hamiltonian(wire, v_local=None) -> sp.csr_matrix:
    """Real symmetric H = -1/2 Lap_h + diag(V) + sum_p E_p b_p b_p^T."""
    v = wire.v_local if v_local is None else v_local
    H = kinetic_operator(wire.nx, wire.ny, wire.nz, wire.h, wire.R) + sp.diags(v)
    if wire.n_proj:
        B = kb_matrix(wire)
        H = H + B @ sp.diags(wire.kb_energy) @ B.T
    return H.tocsr()


def cap_diagonals(wire):
    """Diagonals (W_L, W_R), each (N,): per-plane profiles broadcast over x, y."""
    per = wire.nx * wire.ny
    return np.repeat(wire.cap_left, per), np.repeat(wire.cap_right, per)


def operator_A(wire, E: float, H=None) -> sp.csc_matrix:
    """A(E) = E*1 - H + i(W_L + W_R) = (G^r)^-1 (Eqs. 3-4 with eta -> 0)."""
    if H is None:
        H = hamiltonian(wire)
    wl, wr = cap_diagonals(wire)
    N = wire.N
    return (E * sp.identity(N, dtype=complex) - H.astype(complex)
            + 1j * sp.diags(wl + wr)).tocsc()
