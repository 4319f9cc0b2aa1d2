"""Batched junctions: negf_transmission_batch equals per-junction calls bit for
bit, and matches the oracle on the small ones."""

import numpy as np
import pytest

import oracle as O
from workloads import make_custom, make_junctions

pytestmark = pytest.mark.gpu


def _junctions():
    out = []
    for k, (n, nz, R, ncap, ne) in enumerate([(8, 28, 2, 6, 5), (10, 36, 3, 6, 9), (9, 30, 4, 7, 3),
                                                (12, 40, 2, 8, 7), (8, 24, 1, 5, 6)]):
        h = 0.5
        c = (n + 1) * h / 2
        wells = [(c + 0.2 * k, c - 0.1, 5.0 + k, 0.3 + 0.05 * k), (c, c, nz * h * 0.6, 0.4)]
        out.append(make_custom(n, n, nz, h, R, ncap, np.linspace(0.2, 1.0, ne), wells=wells,
                               name=f"j{k}"))
    return out


def test_batch_matches_single_calls_and_oracle(gpu_lib):
    import paper_1401_0782_amd as P

    js = _junctions()
    ops = [P.operator_from_wire(j) for j in js]
    Tb, st = P.negf_transmission_batch(ops, [j.energies for j in js], max_concurrent=3, tol=1e-12)
    assert np.all(st == 0)
    for j, op, T in zip(js, ops, Tb):
        Ts = P.negf_transmission(op, j.energies, tol=1e-12)
        assert np.array_equal(T, Ts)
    for j, T in zip(js[:3], Tb[:3]):
        assert np.max(np.abs(T - O.transmission(j, method="dense"))) <= 1e-8


def test_batch_uneven_wire_junctions(gpu_lib):
    """Eight junctions of the batched workload (16^2 x 64 .. 40^2 x 160), first
    8 source columns each, every energy: batch equals single calls."""
    import paper_1401_0782_amd as P

    js = make_junctions(64)[:8]
    ops = [P.operator_from_wire(j) for j in js]
    kw = dict(tol=1e-10, col_begin=0, col_count=8, block_width=8)
    Tb, st = P.negf_transmission_batch(ops, [j.energies for j in js], max_concurrent=4, **kw)
    assert np.all(st == 0)
    for j, op, T in zip(js, ops, Tb):
        assert np.all(T >= 0)
        assert np.array_equal(T, P.negf_transmission(op, j.energies, **kw))


def test_batch_shards_per_junction(gpu_lib):
    """negf_transmission_batch_shards: each junction sums over its own column
    shard (here 8 columns in the middle of its right absorbing region, and
    its last 5 with col_count 0 meaning to the end); the per-junction T are
    bit-identical to negf_transmission on the same shard, and for the small
    junctions the shards of all columns add up to the oracle's T."""
    import paper_1401_0782_amd as P
    from workloads import rhs_columns

    js = _junctions()
    ops = [P.operator_from_wire(j) for j in js]
    n_src = [len(rhs_columns(j)) for j in js]
    es = [j.energies for j in js]
    mid = [(n // 2 - 4, 8) for n in n_src]
    Tm, st = P.negf_transmission_batch(ops, es, max_concurrent=3, tol=1e-12, shards=mid)
    assert np.all(st == 0)
    for j, op, T, (c0, cn) in zip(js, ops, Tm, mid):
        assert np.array_equal(T, P.negf_transmission(op, j.energies, tol=1e-12, col_begin=c0,
                                                     col_count=cn))
    # three shards per junction: [0, c), [c, n - 5), [n - 5, end) add up to T
    parts = []
    for cut in ([(0, n // 3) for n in n_src], [(n // 3, n - 5 - n // 3) for n in n_src],
                [(n - 5, 0) for n in n_src]):
        T, st = P.negf_transmission_batch(ops, es, max_concurrent=3, tol=1e-12, shards=cut)
        assert np.all(st == 0)
        parts.append(T)
    for k, j in enumerate(js[:3]):
        total = parts[0][k] + parts[1][k] + parts[2][k]
        assert np.max(np.abs(total - O.transmission(j, method="dense"))) <= 1e-8


def test_batch_shards_reject_negative_ranges(gpu_lib):
    import paper_1401_0782_amd as P
    from paper_1401_0782_amd import NegfError

    js = _junctions()[:2]
    ops = [P.operator_from_wire(j) for j in js]
    with pytest.raises(NegfError, match="negative column range"):
        P.negf_transmission_batch(ops, [j.energies for j in js], shards=[(0, 4), (-1, 4)])


def test_batch_unconverged_and_mixed_paths(gpu_lib):
    """A batch whose junctions all stop at max_iter reports NOT_CONVERGED per
    junction with the same T as single calls; mixed precision (the per-energy
    core, run junction by junction inside the batch) equals single calls."""
    import paper_1401_0782_amd as P
    from paper_1401_0782_amd import _abi

    js = _junctions()
    ops = [P.operator_from_wire(j) for j in js]
    es = [j.energies for j in js]
    kw = dict(tol=1e-12, max_iter=6)
    Tb, st = P.negf_transmission_batch(ops, es, max_concurrent=2, check=False, **kw)
    assert np.all(st == _abi.NEGF_E_NOT_CONVERGED)
    for j, op, T in zip(js, ops, Tb):
        assert np.array_equal(T, P.negf_transmission(op, j.energies, check=False, **kw))
    km = dict(tol=1e-10, precision=P.NEGF_MIXED)
    Tm, st = P.negf_transmission_batch(ops[:3], es[:3], **km)
    assert np.all(st == 0)
    for j, op, T in zip(js[:3], ops[:3], Tm):
        assert np.array_equal(T, P.negf_transmission(op, j.energies, **km))


def test_batch_rejects_shared_operator(gpu_lib):
    import paper_1401_0782_amd as P
    from paper_1401_0782_amd import NegfError

    j = _junctions()[0]
    op = P.operator_from_wire(j)
    with pytest.raises(NegfError, match="share"):
        P.negf_transmission_batch([op, op], [j.energies, j.energies])
