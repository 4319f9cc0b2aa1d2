"""The spectral route (Eqs. 8-13) on the device, from eigenpairs computed in
the test with the oracle's complex normalisation."""

import numpy as np
import pytest

import oracle as O
from oracle.spectral import _complex_orthonormalise
from workloads import make_custom

pytestmark = pytest.mark.gpu


def _eigenpairs(wire):
    wl, wr = O.cap_diagonals(wire)
    Hop = O.hamiltonian(wire).toarray() - 1j * np.diag(wl + wr)  # Eq. 4
    eps, U = np.linalg.eig(Hop)
    U = _complex_orthonormalise(eps, U)
    return eps, np.ascontiguousarray(U.T)  # rows are eigenvectors


@pytest.fixture(scope="module")
def kb_wire():
    # energies across the first transverse thresholds (~1.3 Ha for this
    # cross-section): T from 1e-10 to ~0.95
    return make_custom(5, 4, 24, 0.5, 3, 4, np.linspace(1.0, 2.6, 9),
                       wells=[(1.4, 1.1, 5.0, 0.5), (1.7, 1.3, 7.5, 0.3)],
                       atoms_kb=[(0.8, 0.3, 0.1), (0.7, 0.2, 0.12)])


def test_spectral_route_all_eigenpairs(gpu_lib, kb_wire):
    import paper_1401_0782_amd as P

    eps, U = _eigenpairs(kb_wire)
    op = P.operator_from_wire(kb_wire)
    E = kb_wire.energies
    T = P.negf_spectral_transmission(op, eps, U, E)
    T_sp = O.transmission_spectral(kb_wire, E)
    T_ls = O.transmission(kb_wire, E, method="dense")
    assert T_ls.max() > 0.5
    np.testing.assert_allclose(T, T_sp, rtol=1e-9, atol=1e-12)
    assert np.max(np.abs(T - T_ls)) <= 1e-8
    # the same route through the real-space solver of this library
    T_gpu = P.negf_transmission(op, E, tol=1e-12)
    assert np.max(np.abs(T - T_gpu)) <= 1e-8


@pytest.mark.parametrize("keep", [0.75, 0.4, 0.1])
def test_spectral_route_truncated(gpu_lib, kb_wire, keep):
    """Fraction-p truncation keeps the eigenpairs nearest the window; the
    oracle's truncated route gives the same T(E), missing poles included."""
    import paper_1401_0782_amd as P

    eps, U = _eigenpairs(kb_wire)
    op = P.operator_from_wire(kb_wire)
    E = kb_wire.energies
    T = P.negf_spectral_transmission(op, eps, U, E, keep=keep)
    T_sp = O.transmission_spectral(kb_wire, E, keep=keep)
    np.testing.assert_allclose(T, T_sp, rtol=1e-9, atol=1e-12)


def test_spectral_route_degenerate_wire_device_eigenvectors(gpu_lib):
    """A square, symmetric wire (degenerate transverse modes); eigenvectors
    handed over in device memory."""
    import torch

    import paper_1401_0782_amd as P

    w = make_custom(4, 4, 20, 0.5, 2, 5, np.linspace(0.5, 2.0, 7))
    eps, U = _eigenpairs(w)
    op = P.operator_from_wire(w)
    dU = torch.tensor(U, device="cuda")
    T = P.negf_spectral_transmission(op, eps, dU, w.energies)
    T_ls = O.transmission(w, w.energies, method="dense")
    assert np.max(np.abs(T - T_ls)) <= 1e-8


def test_spectral_rejects_pole_on_grid(gpu_lib, kb_wire):
    import paper_1401_0782_amd as P

    eps, U = _eigenpairs(kb_wire)
    op = P.operator_from_wire(kb_wire)
    eps = eps.copy()
    eps[3] = 0.5 + 0.0j
    with pytest.raises(P.NegfError):
        P.negf_spectral_transmission(op, eps, U, np.array([0.4, 0.5]))
