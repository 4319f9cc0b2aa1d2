"""Oracle parity of the fused COCG stencil step at every radius and on every
tiling the kernels take, in both solver cores and in the mixed (FP32 inner)
form, with projectors.

* whole-plane kernel (planes of at most 1024 points): T(E) over every source
  column at R = 1..6 on planes off the wave size, with projectors at R = 5, 6;
* row-tiled kernel (planes above 1024 points, split into y-tiles whose
  radius-R halo crosses the tile boundary): columns of G on both sides of the
  boundary at R = 3..6 on 8 x 132 planes (tiles of 128 + 4 rows), on 130 x 8
  planes (tiles of 7 + 1 rows, 910 of 1024 threads owning a point), and on
  64 x 64 planes at R = 6 with projectors (tiles of 16 rows; the cross-section
  of the largest workload) against stored oracle solves;
* the operator apply with projectors at R = 6 in FP64 and FP32;
* the adjoint gradient at R = 4 with projectors against the dense oracle.

Bars: FP64 |dT| <= 1e-8 and mixed |dT| <= 1e-6 (the two parity targets);
columns of G within 1e-9 of the column's scale (largest entry) at a true
relative residual of 1e-12, as in the other parity tests.
"""

import json
import pathlib

import numpy as np
import pytest

import oracle as O
from workloads import left_support, make_custom, rhs_columns

pytestmark = pytest.mark.gpu
GOLDEN64 = pathlib.Path(__file__).parent / "golden" / "plane64x64x25_samples.json"

CORES = [("multishift", "fp64"), ("per_energy", "fp64"), ("per_energy", "mixed")]


def _opts(P, core, prec):
    return dict(core=P.NEGF_CORE_MULTISHIFT if core == "multishift" else P.NEGF_CORE_PER_ENERGY,
                precision=P.NEGF_FP64 if prec == "fp64" else P.NEGF_MIXED)


def _in_band(nx, ny, h, R, offsets=(0.2, 0.8)):
    """Energies above the lowest transverse threshold (open channels, T of order 1)."""
    return O.transverse_thresholds(nx, ny, h, R)[0] + np.asarray(offsets)


def _kb_wire(nx, ny, R, h=0.5, energies=None):
    """nx x ny planes, R-plane CAPs and one atom with s+p projectors whose
    2-bohr sphere stays one plane clear of both CAPs (nz = 2R + 11 at h = 0.5)."""
    nz = 2 * R + 11
    energies = _in_band(nx, ny, h, R) if energies is None else energies
    cx, cy, cz = (nx + 1) * h / 2, (ny + 1) * h / 2, (nz + 1) * h / 2
    return make_custom(nx, ny, nz, h, R, R, np.asarray(energies),
                       wells=[(cx + 0.2, cy - 0.1, cz, 0.45)], atoms_kb=[(0.8, 0.3, 0.12)],
                       name=f"kb{nx}x{ny}R{R}")


@pytest.mark.parametrize("R,nx,ny", [(1, 5, 3), (2, 9, 7), (3, 13, 6), (4, 12, 10),
                                     (5, 7, 11), (6, 10, 9)])
@pytest.mark.parametrize("core,prec", CORES)
def test_whole_plane_every_radius_T(gpu_lib, R, nx, ny, core, prec):
    """T(E) over every source column through the whole-plane fused kernel
    (blocks padded to whole waves), projectors from R = 5 on."""
    import paper_1401_0782_amd as P

    h = 0.5
    if R >= 5:
        w = _kb_wire(nx, ny, R, h)
    else:
        nz = 2 * R + 8
        w = make_custom(nx, ny, nz, h, R, R, _in_band(nx, ny, h, R),
                        wells=[((nx + 1) * h / 2, (ny + 1) * h / 2, (nz + 1) * h / 2, 0.5)])
    Tref = O.transmission(w, method="dense")
    op = P.operator_from_wire(w)
    T = P.negf_transmission(op, w.energies, tol=1e-12 if prec == "fp64" else 1e-11,
                            **_opts(P, core, prec))
    bar = 1e-8 if prec == "fp64" else 1e-6
    assert np.max(np.abs(T - Tref)) <= bar, (T, Tref)


def _boundary_columns(w, y_rows, xs):
    """Grid indices on the innermost right-CAP plane at the given rows."""
    zs = int(np.nonzero(w.cap_right > 0)[0][0])
    per = w.nx * w.ny
    return np.array([zs * per + y * w.nx + x for y, x in zip(y_rows, xs)], np.int64)


def _rows_near(w, y_lo, y_hi):
    """Every 11th left-CAP point, plus the innermost left plane and the source
    plane between rows y_lo and y_hi (the tile boundary) at three x."""
    per = w.nx * w.ny
    zl = int(np.nonzero(w.cap_left > 0)[0][-1])
    zs = int(np.nonzero(w.cap_right > 0)[0][0])
    xs = sorted({0, w.nx // 2, w.nx - 1})
    near = [z * per + y * w.nx + x for z in (zl, zs) for y in range(y_lo, y_hi) for x in xs]
    return np.unique(np.concatenate([left_support(w)[::11], near])).astype(np.int64)


_ORACLE = {}


def _oracle_columns(w, cols, rows):
    """Oracle G[rows, cols] and each column's scale, per energy (sparse LU),
    computed once per wire for the three solver forms."""
    key = (w.name, tuple(cols), tuple(rows))
    if key not in _ORACLE:
        res = []
        for E in w.energies:
            Gfull = O.green_columns(w, E, cols, method="splu")
            res.append((Gfull[rows], np.abs(Gfull).max(axis=0)))
        _ORACLE[key] = res
    return _ORACLE[key]


def _compare_columns(P, op, w, cols, rows, core, prec, bar=1e-9):
    out, st = P.negf_solve_columns(op, w.energies, rhs_idx=cols, row_idx=rows, tol=1e-12,
                                   **_opts(P, core, prec))
    assert np.all(st == 0)
    for e, (G, scale) in enumerate(_oracle_columns(w, cols, rows)):
        err = (np.abs(out[e].T - G) / scale).max()
        assert err < bar, (core, prec, w.energies[e], err)


@pytest.mark.parametrize("R", [3, 4, 5, 6])
@pytest.mark.parametrize("core,prec", CORES)
def test_row_tiled_8x132_every_radius(gpu_lib, R, core, prec):
    """8 x 132 planes: y-tiles of 128 and 4 rows; the second tile's halo
    reaches R rows into the first.  Columns at y = 0, 127, 128 and 131."""
    import paper_1401_0782_amd as P

    nx, ny, h = 8, 132, 0.4
    nz = 2 * R + 4
    w = make_custom(nx, ny, nz, h, R, R, np.array([0.6, 1.0]),
                    wells=[((nx + 1) * h / 2, (ny + 1) * h / 2, (nz + 1) * h / 2, 0.6)],
                    name=f"rows8x132R{R}")
    op = P.operator_from_wire(w)
    cols = _boundary_columns(w, [0, 127, 128, 131], [3, 5, 2, 7])
    rows = _rows_near(w, 120, 132)
    _compare_columns(P, op, w, cols, rows, core, prec)


@pytest.mark.parametrize("core,prec", CORES)
def test_row_tiled_130x8_ragged_threads(gpu_lib, core, prec):
    """130 x 8 planes at R = 6: 7 rows per tile (910 of the 1024 threads own a
    point), so the second tile is one row whose halo is six rows of the first."""
    import paper_1401_0782_amd as P

    nx, ny, nz, h = 130, 8, 14, 0.4
    w = make_custom(nx, ny, nz, h, 6, 6, np.array([0.7]),
                    wells=[((nx + 1) * h / 2, (ny + 1) * h / 2, (nz + 1) * h / 2, 0.5)],
                    name="rows130x8R6")
    op = P.operator_from_wire(w)
    cols = _boundary_columns(w, [6, 7, 0], [64, 129, 0])
    rows = _rows_near(w, 0, 8)
    _compare_columns(P, op, w, cols, rows, core, prec)


@pytest.mark.skipif(not GOLDEN64.exists(), reason="oracle samples not generated")
@pytest.mark.parametrize("core,prec", CORES)
def test_row_tiled_64x64_projectors_golden(gpu_lib, core, prec):
    """64 x 64 planes at R = 6 with projectors (16-row tiles, halo across three
    tile boundaries) against stored oracle solves (true residual 1e-12):
    G at the stored rows within 1e-9 of the column scale, and t_j(E) from the
    transmission call on a one-column shard within 1e-12 (absolute)."""
    import paper_1401_0782_amd as P
    import sys

    sys.path.insert(0, str(GOLDEN64.parent))
    import make_plane64_samples as M

    data = json.loads(GOLDEN64.read_text())
    w = M.make()
    rows = np.asarray(data["rows"], np.int64)
    assert np.array_equal(rows, M.rows_of(w))
    op = P.operator_from_wire(w)
    srcs = sorted({s["grid_index"] for s in data["samples"]})
    out, st = P.negf_solve_columns(op, w.energies, rhs_idx=srcs, row_idx=rows, tol=1e-12,
                                   **_opts(P, core, prec))
    assert np.all(st == 0)
    rc = rhs_columns(w)
    for s in data["samples"]:
        k = srcs.index(s["grid_index"])
        ref = np.array([complex(a, b) for a, b in s["g_rows"]])
        err = np.abs(out[s["e_index"], k] - ref).max() / s["g_scale"]
        assert err < 1e-9, (core, prec, s["source"], s["energy"], err)
        c = int(np.nonzero(rc == s["grid_index"])[0][0])
        T, d = P.negf_transmission(op, w.energies, n_cols=1, col_begin=c, col_count=1,
                                   tol=1e-12, **_opts(P, core, prec))
        assert abs(d.t_col[s["e_index"], 0] - s["t_col"]) <= 1e-12 + 1e-9 * s["t_col"], s


def test_apply_with_projectors_radius6_both_precisions(gpu_lib):
    """A(E) X with the radius-6 stencil and projectors, on planes of both
    kernels' sizes, in FP64 (1e-13) and FP32 arithmetic (2e-6)."""
    import paper_1401_0782_amd as P

    rng = np.random.default_rng(11)
    for nx, ny in ((10, 9), (40, 30)):
        w = _kb_wire(nx, ny, 6)
        op = P.operator_from_wire(w)
        H = O.hamiltonian(w)
        X = rng.standard_normal((3, w.N)) + 1j * rng.standard_normal((3, w.N))
        sh = np.array([0.2, 0.7, 1.3])
        for prec, bar in ((P.NEGF_FP64, 1e-13), (P.NEGF_MIXED, 2e-6)):
            Y = P.negf_apply_operator(op, sh, X, precision=prec)
            for c in range(3):
                ref = O.operator_A(w, sh[c], H) @ X[c]
                err = np.linalg.norm(Y[c] - ref) / np.linalg.norm(ref)
                assert err <= bar, (nx, ny, prec, c, err)


def test_adjoint_radius4_projectors_dense(gpu_lib):
    """dL/dV for L = sum_E w_E T(E) at R = 4 with projectors, against the
    dense oracle gradient 8 Re sum W_L W_R conj(G_ij) G_ir G_rj."""
    import paper_1401_0782_amd as P

    w = _kb_wire(6, 6, 4, energies=_in_band(6, 6, 0.5, 4, (0.1, 0.5, 0.9)))
    op = P.operator_from_wire(w)
    weights = np.array([1.0, -0.5, 0.25])
    dV, T = P.negf_transmission_grad(op, w.energies, weights, tol=1e-13)
    ref = sum(wt * O.grad_T_dense(w, E) for wt, E in zip(weights, w.energies))
    assert np.max(np.abs(T - O.transmission(w, method="dense"))) < 1e-9
    err = np.linalg.norm(dV - ref) / np.linalg.norm(ref)
    assert err < 1e-7, err
