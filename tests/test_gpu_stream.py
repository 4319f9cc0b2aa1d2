"""Column streaming: slots of a multi-shift block restart on queued source
columns; every column's arithmetic is that of a block of its own."""

import os

import numpy as np
import pytest

import oracle as O
from workloads import make_wire

pytestmark = pytest.mark.gpu


def _run(op, wire, n_cols, stream, **kw):
    import paper_1401_0782_amd as P

    old = os.environ.get("NEGF_NO_COLUMN_STREAM")
    os.environ["NEGF_NO_COLUMN_STREAM"] = "0" if stream else "1"
    try:
        return P.negf_transmission(op, wire.energies, n_cols=n_cols, **kw)
    finally:
        if old is None:
            del os.environ["NEGF_NO_COLUMN_STREAM"]
        else:
            os.environ["NEGF_NO_COLUMN_STREAM"] = old


@pytest.mark.parametrize("block_width", [16, 64, 100])
def test_streaming_equals_blockwise_bit_for_bit(gpu_lib, block_width):
    import paper_1401_0782_amd as P

    wire = make_wire(1)  # 384 source columns, 8 energies
    op = P.operator_from_wire(wire)
    kw = dict(tol=1e-12, block_width=block_width)
    T_s, d_s = _run(op, wire, 384, True, **kw)
    T_b, d_b = _run(op, wire, 384, False, **kw)
    assert d_s.status == 0 and d_b.status == 0
    # block-wise, a last partial block runs narrower, and the stencil's
    # z-chunking (so its partial-sum order) depends on the width: those
    # columns agree to rounding, all others bit for bit
    full = (384 // block_width) * block_width
    assert np.array_equal(d_s.t_col[:, :full], d_b.t_col[:, :full])
    assert np.array_equal(d_s.iters[:, :full], d_b.iters[:, :full])
    assert np.array_equal(d_s.resid[:, :full], d_b.resid[:, :full])
    np.testing.assert_allclose(d_s.t_col[:, full:], d_b.t_col[:, full:], rtol=1e-9, atol=1e-20)
    if full == 384:
        assert d_s.total_iters == d_b.total_iters
    T_ref = O.transmission(wire, method="dense")
    assert np.max(np.abs(T_s - T_ref)) <= 1e-8


def test_streaming_shard_and_max_iter(gpu_lib):
    """A column shard streams too, and columns that hit max_iter hand over
    their partial results with the max-iter status."""
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    kw = dict(tol=1e-12, block_width=40, col_begin=40, col_count=200, check=False)
    T_s, d_s = _run(op, wire, 200, True, **kw)
    T_b, d_b = _run(op, wire, 200, False, **kw)
    assert d_s.status == 0
    assert np.array_equal(d_s.t_col, d_b.t_col)
    short = dict(kw, max_iter=20)
    T_s, d_s = _run(op, wire, 200, True, **short)
    T_b, d_b = _run(op, wire, 200, False, **short)
    assert d_s.status == 4 and d_b.status == 4  # NOT_CONVERGED
    assert np.array_equal(d_s.t_col, d_b.t_col)
    assert np.array_equal(d_s.item_status, d_b.item_status)
    assert (d_s.iters <= 20).all()


def test_mfma_and_valu_shift_accumulation_agree(gpu_lib):
    """The blocked shift accumulation on the matrix cores and on the vector
    ALUs give the same T(E) to rounding, and both the oracle's."""
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    old = os.environ.get("NEGF_GEMM_VALU")
    try:
        os.environ["NEGF_GEMM_VALU"] = "0"
        T_m, d_m = P.negf_transmission(op, wire.energies, n_cols=384, tol=1e-12)
        os.environ["NEGF_GEMM_VALU"] = "1"
        T_v, d_v = P.negf_transmission(op, wire.energies, n_cols=384, tol=1e-12)
    finally:
        if old is None:
            del os.environ["NEGF_GEMM_VALU"]
        else:
            os.environ["NEGF_GEMM_VALU"] = old
    assert np.array_equal(d_m.iters, d_v.iters)
    np.testing.assert_allclose(d_m.t_col, d_v.t_col, rtol=1e-11, atol=1e-24)
    T_ref = O.transmission(wire, method="dense")
    assert np.max(np.abs(T_m - T_ref)) <= 1e-8
    assert np.max(np.abs(T_v - T_ref)) <= 1e-8


def test_live_energy_compaction_is_bit_identical(gpu_lib):
    """The matrix-core GEMM tiles only the energies that still move; with
    every energy listed instead, the frozen ones get zero coefficients and
    T(E) per column comes out bit for bit the same."""
    import paper_1401_0782_amd as P

    wire = make_wire(1)
    op = P.operator_from_wire(wire)
    old = os.environ.get("NEGF_GEMM_NO_COMPACT")
    try:
        os.environ["NEGF_GEMM_NO_COMPACT"] = "0"
        T_c, d_c = P.negf_transmission(op, wire.energies, n_cols=384, tol=1e-12)
        os.environ["NEGF_GEMM_NO_COMPACT"] = "1"
        T_a, d_a = P.negf_transmission(op, wire.energies, n_cols=384, tol=1e-12)
    finally:
        if old is None:
            del os.environ["NEGF_GEMM_NO_COMPACT"]
        else:
            os.environ["NEGF_GEMM_NO_COMPACT"] = old
    assert np.array_equal(d_c.t_col, d_a.t_col)
    assert np.array_equal(d_c.iters, d_a.iters)
