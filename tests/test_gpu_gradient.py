"""Adjoint gradients through the C ABI and torch.autograd against the oracle."""

import numpy as np
import pytest

import oracle as O
from workloads import make_custom, well_basis

pytestmark = pytest.mark.gpu


def _wire():
    h = 0.5
    cx, cy = 3.5 * h, 3.0 * h
    return make_custom(6, 5, 28, h, 2, 5, [0.35, 0.7, 1.1],
                       wells=[(cx, cy, 5.5, 0.45), (cx + 0.3, cy - 0.2, 8.0, 0.3),
                              (cx - 0.2, cy + 0.1, 10.0, 0.5)], name="gradwire")


def test_grad_field_matches_dense_oracle(gpu_lib):
    import paper_1401_0782_amd as P

    w = _wire()
    op = P.operator_from_wire(w)
    weights = np.array([1.0, -0.5, 0.25])
    dV, T = P.negf_transmission_grad(op, w.energies, weights, tol=1e-13)
    ref = sum(wt * O.grad_T_dense(w, E) for wt, E in zip(weights, w.energies))
    Tref = O.transmission(w, method="dense")
    assert np.max(np.abs(T - Tref)) < 1e-9
    err = np.linalg.norm(dV - ref) / np.linalg.norm(ref)
    assert err < 1e-7, err


def test_autograd_amplitudes_match_finite_differences(gpu_lib):
    import torch

    from paper_1401_0782_amd.autograd import transmission

    w = _wire()
    phi = torch.as_tensor(well_basis(w))
    U = torch.tensor(w.well_depths.copy(), dtype=torch.float64, requires_grad=True)
    V = -(phi @ U)
    T = transmission(V, w, w.energies, tol=1e-13)
    weights = torch.tensor([1.0, 0.5, 2.0], dtype=torch.float64)
    L = (weights * T).sum()
    L.backward()
    fd = O.grad_T_amplitudes_fd(w, w.energies, weights.numpy(), step=1e-5, method="dense")
    g = U.grad.numpy()
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-5, (g, fd)
    for a in range(len(g)):
        assert abs(g[a] - fd[a]) <= 1e-5 * max(abs(fd[a]), 1e-3 * np.abs(fd).max())
