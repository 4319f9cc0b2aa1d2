"""The launch-shape autotuner (negf_tune) through the C ABI."""

import numpy as np
import pytest

import oracle as O
from workloads import make_wire

pytestmark = pytest.mark.gpu


def test_tune_picks_fastest_candidate_and_keeps_results(gpu_lib):
    import paper_1401_0782_amd as P

    wire = make_wire(1)  # 8x8x32, R=2, 384 source columns, 8 energies
    op = P.operator_from_wire(wire)
    T_default = P.negf_transmission(op, wire.energies, tol=1e-12)
    res = P.negf_tune(op, wire.energies)
    tried = res["tried"]
    # 5 widths x 2 stencil kernels (the 64-point plane fits one work-group) x 5 targets
    assert len(tried) == 50
    assert {t[0] for t in tried} == {16, 32, 64, 128, 256}
    assert {t[2] for t in tried} == {0, 1}
    assert all(t[3] > 0 for t in tried)
    best = min(tried, key=lambda t: t[3])
    assert (res["block_width"], res["wg_target"], res["plane_kernel"]) == best[:3]
    # later calls run with the tuned shape: same T up to rounding, and the oracle's
    T_tuned = P.negf_transmission(op, wire.energies, tol=1e-12)
    assert np.max(np.abs(T_tuned - T_default)) <= 1e-12
    T_ref = O.transmission(wire, method="dense")
    assert np.max(np.abs(T_tuned - T_ref)) <= 1e-8


@pytest.mark.parametrize("plane", [0, 1])
def test_every_tuned_shape_matches_oracle(gpu_lib, plane):
    """A fixed block width tunes only z-chunking and kernel; each probe shape,
    forced in turn, gives the oracle's T(E)."""
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    res = P.negf_tune(op, wire.energies, block_width=32)
    assert {t[0] for t in res["tried"]} == {32}
    T_ref = O.transmission(wire, method="dense")
    for target in (128, 1024):
        P.negf_set_launch_shape(op, 32, target, plane)
        T, d = P.negf_transmission(op, wire.energies, n_cols=384, tol=1e-12, block_width=32)
        assert d.status == 0
        assert np.max(np.abs(T - T_ref)) <= 1e-8, (target, plane)
