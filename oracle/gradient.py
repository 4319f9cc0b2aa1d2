"""Derivatives of T(E) with respect to the local potential (oracle).

With A(E) = E - H + iW and dA/dV_r = -e_r e_r^T, dG = -G dA G gives
dG_ij/dV_r = G_ir G_rj.  Differentiating Eq. 7 (with the factor 4):
    dT/dV_r = 8 Re sum_{i in L, j in R} W_L,i W_R,j conj(G_ij) G_ir G_rj .
The finite-difference routes perturb V (or the well depths) and call the
transmission routes again.
"""

from __future__ import annotations

import numpy as np

from .operator import cap_diagonals, operator_A
from .solve import _support, transmission


def grad_T_dense(wire, E):
    """dT(E)/dV_r for every grid point r, by dense inversion (small N)."""
    wl, wr = cap_diagonals(wire)
    L = _support(wire, "L")
    Rs = _support(wire, "R")
    G = np.linalg.inv(operator_A(wire, E).toarray())
    D = (wl[L][:, None] * wr[Rs][None, :]) * np.conj(G[np.ix_(L, Rs)])
    # sum_ij G_ri D_ij G_rj for every r
    return 8.0 * np.real(np.sum((G[:, L] @ D) * G[:, Rs], axis=1))


def grad_T_fd(wire, E, points, step=1e-5, method="auto"):
    """Central differences of T(E) in V at the given grid points."""
    out = []
    v0 = wire.v_local.copy()
    for r in points:
        vals = []
        for s in (+step, -step):
            wire.v_local = v0.copy()
            wire.v_local[r] += s
            vals.append(transmission(wire, [E], method=method)[0])
        out.append((vals[0] - vals[1]) / (2 * step))
    wire.v_local = v0
    return np.array(out)


def grad_T_amplitudes_fd(wire, energies, weights, step=1e-5, method="auto"):
    """Central differences of L = sum_E w_E T(E) in the well depths U_a."""
    from workloads import potential_from_amplitudes

    v0 = wire.v_local.copy()
    d0 = wire.well_depths.copy()
    out = []
    for a in range(len(d0)):
        vals = []
        for s in (+step, -step):
            d = d0.copy()
            d[a] += s
            wire.v_local = potential_from_amplitudes(wire, d)
            vals.append(float(np.dot(weights, transmission(wire, energies, method=method))))
        out.append((vals[0] - vals[1]) / (2 * step))
    wire.v_local = v0
    return np.array(out)

