"""Parity of the HIP path (through the C ABI) against the CPU oracle."""

import numpy as np
import pytest

import oracle as O
from workloads import make_custom, make_wire, rhs_columns, left_support

pytestmark = pytest.mark.gpu


def _op(wire):
    import paper_1401_0782_amd as P

    return P.operator_from_wire(wire)


def _small_kb_wire(nx=9, ny=7, nz=40, R=3, h=0.5):
    # two atoms with s+p projectors, away from the 6-plane CAPs
    cx, cy = (nx + 1) * h / 2, (ny + 1) * h / 2
    wells = [(cx + 0.3, cy - 0.2, 7.5, 0.4), (cx - 0.4, cy + 0.3, 12.0, 0.5)]
    return make_custom(nx, ny, nz, h, R, 6, np.linspace(0.2, 1.2, 6), wells=wells,
                       atoms_kb=[(0.8, 0.3, 0.1), (0.7, 0.2, 0.15)], name="kbwire")


@pytest.mark.parametrize("R,shape", [(1, (5, 3, 12)), (2, (8, 8, 32)), (3, (13, 6, 20)),
                                     (4, (24, 5, 30)), (5, (7, 40, 22)), (6, (32, 9, 26))])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_apply_matches_oracle(gpu_lib, R, shape, prec):
    import paper_1401_0782_amd as P

    nx, ny, nz = shape
    rng = np.random.default_rng([7, R, nx])
    wire = make_custom(nx, ny, nz, 0.45, R, max(R, 3), [0.3],
                       wells=[((nx + 1) * 0.225, (ny + 1) * 0.225, (nz + 1) * 0.225, 0.5)])
    op = _op(wire)
    H = O.hamiltonian(wire)
    n_vec = 5
    shifts = rng.uniform(-1, 1, n_vec)
    X = rng.standard_normal((n_vec, wire.N)) + 1j * rng.standard_normal((n_vec, wire.N))
    Y = P.negf_apply_operator(op, shifts, X, precision=P.NEGF_FP64 if prec == "fp64" else P.NEGF_MIXED)
    for c in range(n_vec):
        A = O.operator_A(wire, shifts[c], H)
        ref = A @ X[c]
        err = np.linalg.norm(Y[c] - ref) / np.linalg.norm(ref)
        assert err <= (1e-13 if prec == "fp64" else 2e-6), (c, err)


def test_apply_with_projectors(gpu_lib):
    import paper_1401_0782_amd as P

    wire = _small_kb_wire()
    op = _op(wire)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, wire.N)) + 1j * rng.standard_normal((3, wire.N))
    sh = np.array([0.1, 0.5, 0.9])
    Y = P.negf_apply_operator(op, sh, X)
    H = O.hamiltonian(wire)
    for c in range(3):
        ref = O.operator_A(wire, sh[c], H) @ X[c]
        assert np.linalg.norm(Y[c] - ref) / np.linalg.norm(ref) < 1e-13


@pytest.fixture(scope="module")
def cfg1():
    w = make_wire(1)
    return w, O.transmission(w, method="dense")


@pytest.mark.parametrize("core", ["multishift", "per_energy"])
def test_cfg1_fp64(gpu_lib, cfg1, core):
    import paper_1401_0782_amd as P

    w, Tref = cfg1
    op = _op(w)
    c = P.NEGF_CORE_MULTISHIFT if core == "multishift" else P.NEGF_CORE_PER_ENERGY
    T, diag = P.negf_transmission(op, w.energies, n_cols=len(rhs_columns(w)), core=c, tol=1e-12)
    print(core, T, Tref, diag.total_iters)
    assert np.max(np.abs(T - Tref)) <= 1e-8


def test_cfg1_mixed(gpu_lib, cfg1):
    import paper_1401_0782_amd as P

    w, Tref = cfg1
    op = _op(w)
    T, diag = P.negf_transmission(op, w.energies, n_cols=len(rhs_columns(w)),
                                  precision=P.NEGF_MIXED, tol=1e-10)
    print("mixed", T, Tref, diag.total_iters)
    assert np.max(np.abs(T - Tref)) <= 1e-6
    assert np.all(diag.resid <= 1e-10)


def test_kb_wire_transmission(gpu_lib):
    import paper_1401_0782_amd as P

    w = _small_kb_wire()
    Tref = O.transmission(w, method="dense")
    op = _op(w)
    T = P.negf_transmission(op, w.energies, tol=1e-12)
    print(T, Tref)
    assert np.max(np.abs(T - Tref)) <= 1e-8


def test_solve_columns_match_oracle(gpu_lib):
    import paper_1401_0782_amd as P

    w = _small_kb_wire()
    op = _op(w)
    cols = rhs_columns(w)[[0, 17, 100]]
    rows = left_support(w)[::7]
    for core in (P.NEGF_CORE_MULTISHIFT, P.NEGF_CORE_PER_ENERGY):
        out, st = P.negf_solve_columns(op, w.energies[:4], rhs_idx=cols, row_idx=rows, core=core,
                                       tol=1e-12)
        assert np.all(st == 0)
        for e, E in enumerate(w.energies[:4]):
            Gfull = O.green_columns(w, E, cols, method="dense")
            G = Gfull[rows]
            # error on the scale of each column (its largest entry, the diagonal):
            # a relative residual tol bounds it by ||A^-1|| tol
            err = (np.abs(out[e].T - G) / np.abs(Gfull).max(axis=0)).max()
            assert err < 1e-9, (core, e, err)


def test_row_tiled_planes_with_y_halo(gpu_lib):
    """Planes of 8 x 132 points (above the whole-plane kernel's 1024) split
    into two y-tiles of the row-tiled stencil kernel, each reading R rows of
    its neighbour: columns of G on both sides of the tile boundary against
    the oracle."""
    import paper_1401_0782_amd as P

    nx, ny, nz, h = 8, 132, 24, 0.5
    w = make_custom(nx, ny, nz, h, 2, 5, np.linspace(0.4, 1.0, 2),
                    wells=[((nx + 1) * h / 2, (ny + 1) * h / 2, (nz + 1) * h / 2, 0.6)])
    op = _op(w)
    # row 128 starts the second tile of 1024 / nx rows
    cols = rhs_columns(w)[[0, 127 * nx + 3, 128 * nx + 5, 777]]
    rows = np.concatenate([left_support(w)[::29], np.arange(w.N - 3 * nx * ny, w.N, 41)])
    out, st = P.negf_solve_columns(op, w.energies, rhs_idx=cols, row_idx=rows, tol=1e-12)
    assert np.all(st == 0)
    for e, E in enumerate(w.energies):
        Gfull = O.green_columns(w, E, cols)
        err = (np.abs(out[e].T - Gfull[rows]) / np.abs(Gfull).max(axis=0)).max()
        assert err < 1e-9, (e, err)


def test_chain_one_point_planes(gpu_lib):
    """The degenerate 1 x 1 x nz grid (a chain; planes of one point, so the
    whole-plane kernel's block is one point and 63 padding lanes) with long
    CAPs: both cores against the oracle.  The band of this chain starts at
    10 Ha (the two transverse second differences of the one-point planes add
    5 Ha each at h = 0.5, R = 2), so the energies sit inside it, where the
    long CAPs give T close to 1."""
    import paper_1401_0782_amd as P

    w = make_custom(1, 1, 120, 0.5, 2, 40, np.linspace(10.3, 13.0, 6), w0=0.5)
    op = _op(w)
    T_ref = O.transmission(w, method="dense")
    assert T_ref.min() > 0.9
    for core in (P.NEGF_CORE_MULTISHIFT, P.NEGF_CORE_PER_ENERGY):
        T = P.negf_transmission(op, w.energies, tol=1e-12, core=core)
        assert np.max(np.abs(T - T_ref)) <= 1e-8, (core, T, T_ref)


def test_multishift_single_energy_single_column_and_duplicates(gpu_lib):
    """Degenerate shift sets of the multi-shift core: one energy (the seed
    alone), one source column, and repeated energies (zero relative shift),
    each against the oracle; repeated energies give identical columns."""
    import paper_1401_0782_amd as P

    w = make_wire(1)
    op = _op(w)
    col = rhs_columns(w)[[5]]
    rows = left_support(w)
    for E in (np.array([0.35]), np.array([0.3, 0.45, 0.3, 0.45])):
        out, st = P.negf_solve_columns(op, E, rhs_idx=col, row_idx=rows, tol=1e-12,
                                       core=P.NEGF_CORE_MULTISHIFT)
        assert np.all(st == 0)
        for e, En in enumerate(E):
            G = O.green_columns(w, En, col, method="dense")
            err = np.abs(out[e, 0] - G[rows, 0]).max() / np.abs(G).max()
            assert err < 1e-9, (En, err)
    assert np.array_equal(out[0], out[2]) and np.array_equal(out[1], out[3])
    T = P.negf_transmission(op, np.array([0.4]), tol=1e-12)
    assert abs(T[0] - O.transmission(w, np.array([0.4]), method="dense")[0]) <= 1e-8


def test_out_of_memory_is_reported_and_recoverable(gpu_lib):
    """A failed device allocation (forced by the library's test hook on the
    k-th allocation of a fresh process) surfaces as NEGF_E_OUT_OF_MEMORY with
    a message, and the process can build and run an operator afterwards."""
    import os
    import subprocess
    import sys

    code = (
        "import numpy as np, paper_1401_0782_amd as P\n"
        "from workloads import make_wire\n"
        "w = make_wire(1)\n"
        "try:\n"
        "    P.operator_from_wire(w)\n"
        "    print('NO-ERROR')\n"
        "except P.NegfError as e:\n"
        "    print('STATUS', e.status, str(e))\n"
        "op = P.operator_from_wire(w)\n"
        "T = P.negf_transmission(op, w.energies, tol=1e-12)\n"
        "print('T-OK', bool(np.all(np.isfinite(T))))\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, NEGF_TEST_FAIL_ALLOC="2", PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    from paper_1401_0782_amd import _abi

    assert f"STATUS {_abi.NEGF_E_OUT_OF_MEMORY}" in out.stdout, out.stdout
    assert "test hook" in out.stdout
    assert "T-OK True" in out.stdout


def test_invalid_calls_rejected(gpu_lib):
    """Empty energy lists, out-of-range shards and null outputs are errors,
    not launches."""
    import paper_1401_0782_amd as P

    w = make_wire(1)
    op = _op(w)
    with pytest.raises(P.NegfError):
        P.negf_transmission(op, np.zeros(0))
    with pytest.raises(P.NegfError):
        P.negf_transmission(op, w.energies, col_begin=380, col_count=10)
    with pytest.raises(P.NegfError):
        P.negf_transmission(op, np.array([0.3, np.nan]))
    # the operator still works afterwards
    T = P.negf_transmission(op, w.energies, tol=1e-12)
    assert np.max(np.abs(T - O.transmission(w, method="dense"))) <= 1e-8
