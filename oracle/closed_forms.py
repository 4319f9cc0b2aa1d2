"""Closed forms used to pin the oracle (test infrastructure only).

They are independent of the transmission routes: textbook results for a
uniform nearest-neighbour chain and for the transverse modes of a box.
"""

from __future__ import annotations

import numpy as np

from .operator import second_difference_1d


def chain_self_energy(E: float, h: float) -> complex:
    """Retarded self-energy of a semi-infinite chain with on-site 2t and
    hopping -t, t = 1/(2h^2) (the R=1 discretisation of -1/2 d^2/dz^2):
    Sigma = -t exp(ikh) with cos(kh) = 1 - E/(2t), valid inside (0, 4t)."""
    t = 1.0 / (2.0 * h * h)
    c = 1.0 - E / (2.0 * t)
    if not (-1.0 < c < 1.0):
        raise ValueError("energy outside the chain band")
    s = np.sqrt(1.0 - c * c)  # sin(kh) > 0 for the retarded branch
    return -t * (c + 1j * s)


def chain_transmission_exact(n_sites, h, E, v_onsite=None):
    """Build a 1-D wire whose end sites carry the exact lead self-energy.

    E is the longitudinal (1-D) energy.  Returns (wire, E3) for the
    transmission routes: nx = ny = 1, nz = n_sites, R = 1, V = v_onsite +
    Re(Sigma) on the two end sites and W_L = W_R = -Im(Sigma) on the end
    planes.  On the 3-D grid a 1 x 1 cross-section adds the transverse
    zero-point energy 2/h^2 (one 1/h^2 per wall-bounded axis), so the
    operator must be evaluated at E3 = E + 2/h^2.  Through Eq. 7 the perfect
    chain must give T = 1 inside the band.
    """
    from workloads import make_custom

    sig = chain_self_energy(E, h)
    e3 = E + 2.0 / (h * h)
    w = make_custom(1, 1, n_sites, h, 1, 1, [e3], name="chain")
    v = np.zeros(n_sites) if v_onsite is None else np.asarray(v_onsite, float).copy()
    v[0] += sig.real
    v[-1] += sig.real
    w.v_local = v
    w.cap_left = np.zeros(n_sites)
    w.cap_right = np.zeros(n_sites)
    w.cap_left[0] = -sig.imag
    w.cap_right[-1] = -sig.imag
    return w, e3


def impurity_transmission_closed_form(E, h, v0):
    """Single on-site impurity v0 in the infinite chain:
    T = 1 / (1 + (v0 / (2 t sin kh))^2), t = 1/(2h^2)."""
    t = 1.0 / (2.0 * h * h)
    c = 1.0 - E / (2.0 * t)
    s = np.sqrt(1.0 - c * c)
    return 1.0 / (1.0 + (v0 / (2.0 * t * s)) ** 2)


def transverse_thresholds(nx, ny, h, R):
    """Sorted channel thresholds lambda_a + lambda_b of an empty wire: the
    eigenvalues of the 1-D zero-ghost operator -1/2 h^-2 D2 in x and in y."""
    lx = np.linalg.eigvalsh(-0.5 / h ** 2 * second_difference_1d(nx, R).toarray())
    ly = np.linalg.eigvalsh(-0.5 / h ** 2 * second_difference_1d(ny, R).toarray())
    return np.sort((lx[:, None] + ly[None, :]).ravel())
