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


def test_tune_cache_round_trip(gpu_lib, tmp_path):
    """negf_tune_cached: the first call tunes and appends one line to the
    cache; a second operator of the same shape then gets the same choice from
    the file without probes (n_tried = 0, the stored timing), and its T is
    the oracle's; another request (a fixed block width) is a new key; a line
    that does not parse is skipped."""
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    cache = tmp_path / "tune.txt"
    cache.write_text("garbage without separator\n")
    op = P.operator_from_wire(wire)
    first = P.negf_tune(op, wire.energies, cache=str(cache))
    assert len(first["tried"]) == 50
    lines = [ln for ln in cache.read_text().splitlines() if " => " in ln]
    assert len(lines) == 1 and "grid8x8x32" in lines[0] and "|R2|" in lines[0]
    op2 = P.operator_from_wire(wire)
    second = P.negf_tune(op2, wire.energies, cache=str(cache))
    assert second["tried"] == []
    key = ("block_width", "wg_target", "plane_kernel")
    assert tuple(second[k] for k in key) == tuple(first[k] for k in key)
    T = P.negf_transmission(op2, wire.energies, tol=1e-12)
    assert np.max(np.abs(T - O.transmission(wire, method="dense"))) <= 1e-8
    third = P.negf_tune(op2, wire.energies, cache=str(cache), block_width=32)
    assert {t[0] for t in third["tried"]} == {32}
    assert len([ln for ln in cache.read_text().splitlines() if " => " in ln]) == 2


def test_tune_cache_rejects_empty_path(gpu_lib):
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    with pytest.raises(P.NegfError, match="cache path"):
        P.negf_tune(op, wire.energies, cache="")


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



@pytest.mark.parametrize("shape", [(9, 7), (13, 40), (1, 1)])
def test_both_stencil_kernels_on_planes_off_the_wave_size(gpu_lib, shape):
    """Planes of 63, 520 and 1 points: the whole-plane kernel pads its block
    to whole waves (1, 56 and 63 padding lanes), the row-tiled kernel runs
    each as one tile.  Both give the oracle's partial T(E) over 16 source
    columns in the middle of the right CAP."""
    import paper_1401_0782_amd as P
    from workloads import make_custom, rhs_columns

    nx, ny = shape
    h = 0.5
    if nx > 1:
        n_cap = 6
        w = make_custom(nx, ny, 24, h, 2, n_cap, np.linspace(0.3, 1.1, 2),
                        wells=[((nx + 1) * h / 2, (ny + 1) * h / 2, 25 * h / 2, 0.5)])
    else:  # a chain: its band starts at 10 Ha
        n_cap = 40
        w = make_custom(1, 1, 120, h, 2, n_cap, np.linspace(10.3, 13.0, 2), w0=0.5)
    op = P.operator_from_wire(w)
    c0 = (n_cap // 2) * nx * ny
    src = rhs_columns(w)[c0:c0 + 16]
    T_ref = np.array([O.column_transmissions(w, E, src).sum() for E in w.energies])
    assert T_ref.max() > 1e-3
    for plane in (1, 0):
        P.negf_set_launch_shape(op, 16, 256, plane)
        T, d = P.negf_transmission(op, w.energies, n_cols=16, col_begin=c0, col_count=16,
                                   tol=1e-12, block_width=16)
        assert d.status == 0
        assert np.max(np.abs(T - T_ref)) <= 1e-8, (plane, T, T_ref)
