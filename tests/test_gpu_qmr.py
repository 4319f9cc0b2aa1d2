"""The simplified QMR solver option of the per-energy core (FP64 and mixed)."""

import numpy as np
import pytest

import oracle as O
from workloads import make_custom, make_wire, rhs_columns, left_support

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_qmr_transmission_matches_oracle(gpu_lib, prec, bound):
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    pr = P.NEGF_FP64 if prec == "fp64" else P.NEGF_MIXED
    T, d = P.negf_transmission(op, wire.energies, n_cols=384, precision=pr,
                               solver=P.NEGF_SOLVER_QMR, tol=1e-12)
    assert d.status == 0
    T_ref = O.transmission(wire, method="dense")
    assert np.max(np.abs(T - T_ref)) <= bound
    # the same Lanczos process and stopping rule as COCG: in FP64 the same
    # iteration counts (mixed precision refines from each solver's own FP32
    # iterate, so its refinement steps may differ)
    Tc, dc = P.negf_transmission(op, wire.energies, n_cols=384, precision=pr,
                                 core=P.NEGF_CORE_PER_ENERGY, tol=1e-12)
    if prec == "fp64":
        assert np.array_equal(d.iters, dc.iters)
    assert np.max(np.abs(T - Tc)) <= bound


def test_qmr_solve_columns_projector_wire(gpu_lib):
    import paper_1401_0782_amd as P

    nx, ny, nz, h = 9, 7, 40, 0.5
    cx, cy = (nx + 1) * h / 2, (ny + 1) * h / 2
    wire = make_custom(nx, ny, nz, h, 3, 6, np.linspace(0.2, 1.2, 6),
                       wells=[(cx + 0.3, cy - 0.2, 7.5, 0.4), (cx - 0.4, cy + 0.3, 12.0, 0.5)],
                       atoms_kb=[(0.8, 0.3, 0.1), (0.7, 0.2, 0.15)])
    op = P.operator_from_wire(wire)
    cols = rhs_columns(wire)[:24].astype(np.int32)
    rows = left_support(wire).astype(np.int32)
    E = wire.energies[[0, 3, 5]]
    G, status = P.negf_solve_columns(op, E, rhs_idx=cols, row_idx=rows,
                                     solver=P.NEGF_SOLVER_QMR, tol=1e-12)
    assert (status == 0).all()
    for k, e in enumerate(E):
        Gfull = O.green_columns(wire, e, cols, method="dense")
        # error on the scale of each column (its largest entry, the diagonal):
        # a relative residual tol bounds it by ||A^-1|| tol
        err = (np.abs(G[k].T - Gfull[rows]) / np.abs(Gfull).max(axis=0)).max()
        assert err <= 1e-9, (e, err)


def test_qmr_with_multishift_rejected(gpu_lib):
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    with pytest.raises(P.NegfError, match="per-energy"):
        P.negf_transmission(op, wire.energies, core=P.NEGF_CORE_MULTISHIFT,
                            solver=P.NEGF_SOLVER_QMR)
