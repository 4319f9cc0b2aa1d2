"""Eigenpairs of H - iW on the device (negf_eigenpairs) against numpy's
dense eigen-solver, and the spectral route of Eqs. 8-13 fed with them against
the oracle's transmission."""

import numpy as np
import pytest

import oracle as O
from workloads import make_custom

pytestmark = pytest.mark.gpu


def _wire(nz=30, R=2):
    h = 0.5
    th = O.transverse_thresholds(3, 3, h, R)[0]
    return make_custom(3, 3, nz, h, R, 6, th + np.linspace(0.1, 0.9, 7),
                       wells=[(1.0, 1.1, 6.0, 0.4), (1.1, 0.9, 9.0, 0.3)],
                       atoms_kb=[(0.8, 0.3, 0.1), (0.7, 0.2, 0.12)], name="eig3x3")


def _dense_eigs(w):
    wl, wr = O.cap_diagonals(w)
    return np.linalg.eigvals(O.hamiltonian(w).toarray() - 1j * np.diag(wl + wr))


def _match(found, ref):
    """Distance from each found eigenvalue to the nearest reference one."""
    return np.array([np.min(np.abs(ref - f)) for f in found])


def test_full_krylov_space_finds_every_eigenpair(gpu_lib):
    """K = N: every eigenvalue of the 270-point operator, each to 1e-9 of
    numpy's, with U_i^T U_i = 1 and residual <= 1e-8; Eq. 13 with all of them
    equals the oracle's T(E) (dense inversion)."""
    import paper_1401_0782_amd as P

    w = _wire()
    op = P.operator_from_wire(w)
    ref = _dense_eigs(w)
    lo, hi = ref.real.min() - 1.0, ref.real.max() + 1.0
    eps, U, res = P.negf_eigenpairs(op, lo, hi, n_lanczos=w.N, resid_tol=1e-8)
    assert len(eps) == w.N, len(eps)
    assert _match(eps, ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    # no eigenvalue twice: the matching is one to one
    assert len(np.unique(np.round(eps, 8))) == w.N
    assert np.all(res <= 1e-8)
    norms = np.einsum("ij,ij->i", U, U)
    assert np.abs(norms - 1.0).max() <= 1e-9
    T = P.negf_spectral_transmission(op, eps, U, w.energies)
    Tref = O.transmission(w, method="dense")
    assert np.max(np.abs(T - Tref)) <= 1e-8 * max(1.0, Tref.max())


def test_partial_space_low_end_converges_first(gpu_lib):
    """K = 640 < N = 900: the eigenpairs returned from the window [lowest,
    lowest + 1 Ha] (residual <= 1e-8) are eigenpairs of numpy's dense solve,
    and every eigenvalue numpy finds in its lower 70 % is among them (the
    low end of the spectrum converges first; a single start vector resolves
    close pairs late, so at K = 400 one of the lowest was still missing)."""
    import paper_1401_0782_amd as P

    w = _wire(nz=100)
    op = P.operator_from_wire(w)
    ref = _dense_eigs(w)
    lo = ref.real.min()
    eps, U, res = P.negf_eigenpairs(op, lo, lo + 1.0, margin=0.0, n_lanczos=640,
                                    resid_tol=1e-8)
    assert len(eps) > 0
    assert _match(eps, ref).max() <= 1e-8
    inwin = ref[(ref.real >= lo) & (ref.real <= lo + 1.0)]
    missing = inwin[_match(inwin, eps) > 1e-8]
    print(f"{len(eps)} of {len(inwin)} window eigenvalues found; missing: {np.sort_complex(missing)}")
    want = ref[(ref.real >= lo) & (ref.real <= lo + 0.7)]
    assert _match(want, eps).max() <= 1e-8, (len(want), len(eps))
    assert np.all(res <= 1e-8)
    assert np.abs(np.einsum("ij,ij->i", U, U) - 1.0).max() <= 1e-9
