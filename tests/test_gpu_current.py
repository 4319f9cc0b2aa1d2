"""Landauer current (Eq. 1) on the device against the oracle."""

import numpy as np
import pytest

import oracle as O
from workloads import make_wire

pytestmark = pytest.mark.gpu


def test_current_matches_oracle_on_wire_transmission(gpu_lib):
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    E = np.linspace(0.05, 0.65, 61)
    T = O.transmission(wire, energies=E, method="dense")
    bias = np.linspace(-0.3, 0.3, 13)
    for kT in (0.0, 0.005, 0.05):
        I = P.negf_current(E, T, bias, e_fermi=0.35, kT=kT)
        ref = np.array([O.landauer_current(E, T, bias=v, e_fermi=0.35, kT=kT) for v in bias])
        np.testing.assert_allclose(I, ref, rtol=1e-13, atol=1e-17)


def test_current_nonuniform_grid_and_device_arrays(gpu_lib):
    import torch

    import paper_1401_0782_amd as P

    rng = np.random.default_rng(11)
    E = np.sort(rng.uniform(-1.0, 1.0, 3000))
    T = 2.0 + np.sin(7 * E) + 0.3 * rng.standard_normal(E.size) ** 2
    bias = rng.uniform(-0.5, 0.5, 40)
    I = P.negf_current(E, T, bias, e_fermi=0.05, kT=0.01)
    ref = np.array([O.landauer_current(E, T, bias=v, e_fermi=0.05, kT=0.01) for v in bias])
    np.testing.assert_allclose(I, ref, rtol=1e-12, atol=1e-16)
    # device inputs and output through the C ABI
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    de = torch.tensor(E, device="cuda")
    dt = torch.tensor(T, device="cuda")
    db = torch.tensor(bias, device="cuda")
    dout = torch.zeros(bias.size, dtype=torch.float64, device="cuda")
    st = lib.negf_current(E.size, de.data_ptr(), dt.data_ptr(), bias.size, db.data_ptr(), 0.05,
                          0.01, dout.data_ptr(), None)
    assert st == 0
    np.testing.assert_allclose(dout.cpu().numpy(), ref, rtol=1e-12, atol=1e-16)
