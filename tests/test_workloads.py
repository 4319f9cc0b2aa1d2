"""The seeded input generator: determinism, shapes and stated conventions."""

import numpy as np

from workloads import (make_junctions, make_wire, quartic_cap, rhs_columns, left_support,
                       well_basis, potential_from_amplitudes)


def test_deterministic():
    a, b = make_wire(2), make_wire(2)
    assert np.array_equal(a.v_local, b.v_local)
    assert np.array_equal(a.kb_val, b.kb_val) and np.array_equal(a.kb_idx, b.kb_idx)


def test_cfg_shapes():
    w1 = make_wire(1)
    assert (w1.nx, w1.ny, w1.nz, w1.R, w1.N) == (8, 8, 32, 2, 2048)
    assert len(rhs_columns(w1)) == 384 and len(w1.energies) == 8
    w2 = make_wire(2)
    assert w2.N == 196608 and w2.n_proj == 80 and len(rhs_columns(w2)) == 16384
    assert len(w2.energies) == 256
    w4 = make_wire(4)
    assert w4.N == 55296 and len(rhs_columns(w4)) == 6912 and len(w4.energies) == 64


def test_quartic_cap_convention():
    l, r = quartic_cap(20, 4, 0.5)
    assert l[0] == 0.5 and r[-1] == 0.5  # outermost planes carry W0
    assert np.allclose(l[:4], 0.5 * (np.array([4, 3, 2, 1]) / 4) ** 4)
    assert np.all(l[4:] == 0) and np.all(r[:-4] == 0)


def test_kb_projectors_normalised_and_clear_of_caps():
    w = make_wire(2)
    per = w.nx * w.ny
    for p in range(w.n_proj):
        v = w.kb_val[w.kb_offsets[p]:w.kb_offsets[p + 1]]
        assert abs(np.sum(v * v) - 1.0) < 1e-12
    z = w.kb_idx // per
    assert z.min() > w.n_cap and z.max() < w.nz - w.n_cap - 1


def test_supports_and_well_basis():
    w = make_wire(4)
    L, R = left_support(w), rhs_columns(w)
    assert np.all(np.repeat(w.cap_left, w.nx * w.ny)[L] > 0)
    assert np.all(np.repeat(w.cap_right, w.nx * w.ny)[R] > 0)
    assert np.allclose(-well_basis(w) @ w.well_depths, w.v_local)
    assert np.allclose(potential_from_amplitudes(w, w.well_depths), w.v_local)


def test_junctions():
    js = make_junctions(8)
    for j in js:
        assert 16 <= j.nx <= 40 and j.nz == 4 * j.nx and 8 <= j.n_cap <= 16
        assert 32 <= len(j.energies) <= 256 and j.n_proj == 0
