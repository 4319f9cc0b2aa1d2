"""Graph-replayed iteration chunks give the same results as eager launches."""

import os

import numpy as np
import pytest

from workloads import make_wire, rhs_columns

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("core", ["multishift", "per_energy_mixed"])
def test_graph_replay_equals_eager(gpu_lib, core):
    import paper_1401_0782_amd as P

    w = make_wire(1)
    op = P.operator_from_wire(w)
    kw = dict(core=P.NEGF_CORE_MULTISHIFT) if core == "multishift" else \
        dict(core=P.NEGF_CORE_PER_ENERGY, precision=P.NEGF_MIXED)
    runs = []
    for flag in ("0", "1", "0", "1"):
        os.environ["NEGF_NO_GRAPH"] = flag
        try:
            T, d = P.negf_transmission(op, w.energies, n_cols=len(rhs_columns(w)), tol=1e-11, **kw)
        finally:
            os.environ.pop("NEGF_NO_GRAPH", None)
        runs.append((T, d.t_col.copy(), d.iters.copy()))
    for T, tc, it in runs[1:]:
        assert np.array_equal(T, runs[0][0])
        assert np.array_equal(tc, runs[0][1])
        assert np.array_equal(it, runs[0][2])
