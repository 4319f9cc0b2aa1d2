"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign, a transposed index, a missing factor) fails it:

* finite-difference weights: exactness on polynomials and the closed form;
* 3-D assembly: separability of the kinetic spectrum into 1-D spectra;
* projector term: Sherman-Morrison update of G for one projector;
* factor 4 and operator sign: exact 1-D lead self-energy gives T = 1;
* local potential: on-site impurity closed form;
* absorbing potentials: a long CAP on a chain absorbs (T ~ 1), and an empty
  wire counts its open transverse modes;
* exact identities of Eq. 6/7: G = G^T, reciprocity, optical theorem,
  0 <= T <= sum_j 4 W_R,j (-Im G_jj);
* route independence: dense, sparse LU, iterative and the spectral route of
  Eqs. 8-13 agree;
* gradient: the dG = G dA G formula against central differences;
* Landauer current (Eq. 1) for a constant transmission.
"""

from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle as O
from workloads import make_custom, rhs_columns


# ---------------------------------------------------------------- weights
@pytest.mark.parametrize("R", range(1, 7))
def test_fd_weights_exact_on_polynomials(R):
    c = O.fd_second_derivative_weights(R)
    for deg in range(0, 2 * R + 2):
        # sum_m c_|m| m^deg equals d^2/dx^2 x^deg at 0 times h^2 (= 2 for deg 2)
        s = sum(c[abs(m)] * Fraction(m) ** deg for m in range(-R, R + 1)) if deg else \
            sum(c[abs(m)] for m in range(-R, R + 1))
        assert s == (2 if deg == 2 else 0), (R, deg, s)


@pytest.mark.parametrize("R", range(1, 7))
def test_fd_weights_closed_form(R):
    c = O.fd_second_derivative_weights(R)
    for m in range(1, R + 1):
        cf = Fraction(2 * (-1) ** (m + 1) * factorial(R) ** 2,
                      m * m * factorial(R - m) * factorial(R + m))
        assert c[m] == cf
    assert c[0] == -2 * sum(c[1:])


@pytest.mark.parametrize("R", [1, 3, 6])
def test_second_difference_interior_rows_exact(R):
    n, h = 30, 0.3
    D = O.second_difference_1d(n, R).toarray()
    x = (np.arange(n) + 1) * h
    f = 0.3 * x ** 3 - x ** 2 + 2.0 * x + 1.0
    f2 = 1.8 * x - 2.0
    inner = slice(R, n - R)
    assert np.allclose((D @ f)[inner] / h ** 2, f2[inner], rtol=0, atol=1e-9)


def test_kinetic_is_separable():
    nx, ny, nz, h, R = 4, 3, 5, 0.5, 2
    K = O.kinetic_operator(nx, ny, nz, h, R).toarray()
    assert np.allclose(K, K.T)
    ev = np.sort(np.linalg.eigvalsh(K))
    l1 = [np.linalg.eigvalsh(-0.5 / h ** 2 * O.second_difference_1d(n, R).toarray())
          for n in (nx, ny, nz)]
    sums = np.sort((l1[0][:, None, None] + l1[1][None, :, None] + l1[2][None, None, :]).ravel())
    assert np.allclose(ev, sums, atol=1e-10)
    # the x direction is the fastest index: a function of x only stays one
    f = np.tile(np.sin(np.arange(nx) + 0.5), ny * nz)
    Kx = -0.5 / h ** 2 * O.second_difference_1d(nx, R).toarray()
    ky = -0.5 / h ** 2 * O.second_difference_1d(ny, R).toarray().sum(axis=1)
    kz = -0.5 / h ** 2 * O.second_difference_1d(nz, R).toarray().sum(axis=1)
    expect = (np.tile(Kx @ f[:nx], ny * nz)
              + np.tile(np.repeat(ky, nx), nz) * f
              + np.repeat(kz, nx * ny) * f)
    assert np.allclose(K @ f, expect, atol=1e-10)


# ---------------------------------------------------------------- projectors
def test_projector_term_sherman_morrison():
    h = 0.5
    base = make_custom(5, 4, 20, h, 2, 4, [0.4], wells=[(1.5, 1.2, 5.0, 0.3)])
    kbw = make_custom(5, 4, 20, h, 2, 4, [0.4], wells=[(1.5, 1.2, 5.0, 0.3)],
                      atoms_kb=[(0.8, 0.3, 0.12)])
    # keep only the s projector
    p = 0
    sel = slice(kbw.kb_offsets[p], kbw.kb_offsets[p + 1])
    kbw.kb_offsets = np.array([0, sel.stop - sel.start], np.int64)
    kbw.kb_idx, kbw.kb_val = kbw.kb_idx[sel], kbw.kb_val[sel]
    kbw.kb_energy = kbw.kb_energy[:1]
    b = np.zeros(base.N)
    b[kbw.kb_idx] = kbw.kb_val
    E = 0.4
    G0 = np.linalg.inv(O.operator_A(base, E).toarray())
    G1 = np.linalg.inv(O.operator_A(kbw, E).toarray())
    # A1 = A0 - e b b^T  =>  G1 = G0 + e G0 b b^T G0 / (1 - e b^T G0 b)
    e = kbw.kb_energy[0]
    u = G0 @ b
    G_sm = G0 + e * np.outer(u, u) / (1.0 - e * b @ u)
    assert np.abs(G1 - G_sm).max() < 1e-10 * np.abs(G1).max()


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("E", [0.05, 0.6, 1.9, 3.2, 3.95])
def test_chain_exact_self_energy_gives_unit_transmission(E):
    w, e3 = O.chain_transmission_exact(25, 0.5, E)
    T = O.transmission(w, [e3], method="dense")[0]
    assert abs(T - 1.0) < 1e-12


@pytest.mark.parametrize("E", [0.2, 1.0, 2.7])
@pytest.mark.parametrize("v0", [0.3, -0.8])
def test_impurity_closed_form(E, v0):
    h, n = 0.5, 31
    v = np.zeros(n)
    v[n // 2] = v0
    w, e3 = O.chain_transmission_exact(n, h, E, v)
    T = O.transmission(w, [e3], method="dense")[0]
    assert abs(T - O.impurity_transmission_closed_form(E, h, v0)) < 1e-12


def test_impurity_tends_to_delta_barrier():
    # V0 = alpha/h on one site: T -> 2E / (2E + alpha^2) as h -> 0
    E, alpha = 0.5, 0.4
    errs = []
    for h in (0.2, 0.1, 0.05):
        T = O.impurity_transmission_closed_form(E, h, alpha / h)
        errs.append(abs(T - 2 * E / (2 * E + alpha ** 2)))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 2e-3


def test_long_cap_chain_absorbs():
    # R = 2 chain with an 80-plane quartic CAP on each end: T ~ 1 in band
    h, ncap = 0.5, 80
    nz = 2 * ncap + 20
    w = make_custom(1, 1, nz, h, 2, ncap, [0.0])
    e_perp = 2 * (-0.5 / h ** 2) * float(O.fd_second_derivative_weights(2)[0])
    for E in (0.3, 1.0, 2.0):
        T = O.transmission(w, [E + e_perp], method="splu")[0]
        # the residual CAP reflection (~4e-5 at the top energy) is the only deviation
        assert abs(1.0 - T) < 1e-4, (E, T)


def test_empty_wire_counts_open_modes():
    nx = ny = 4
    h, R, ncap = 0.5, 2, 40
    thr = O.transverse_thresholds(nx, ny, h, R)
    # energies midway between distinct thresholds
    uniq = np.unique(np.round(thr, 10))
    mids = 0.5 * (uniq[:-1] + uniq[1:])[:3]
    w = make_custom(nx, ny, 2 * ncap + 10, h, R, ncap, mids, w0=2.0)
    T = O.transmission(w, mids, method="splu")
    expect = [np.count_nonzero(thr < E) for E in mids]
    assert expect == [1, 3, 4]
    assert np.max(np.abs(T - expect)) < 1e-4, (T, expect)


def test_cap_calibration_plateau_on_empty_wire():
    """The paper's CAP calibration (Sec. III.A): on a long empty lead the
    transmission stays at the open-mode count while the Gaussian CAP of Eq. 5
    changes by 100 % in height and 23 % in width, and for monomial ramps."""
    from workloads import end_gaussian_cap, power_cap, with_caps

    nx = ny = 4
    h, R, ncap = 0.5, 2, 40
    thr = O.transverse_thresholds(nx, ny, h, R)
    uniq = np.unique(np.round(thr, 10))
    mids = 0.5 * (uniq[:-1] + uniq[1:])[:3]
    expect = np.array([np.count_nonzero(thr < E) for E in mids])
    nz = 2 * ncap + 10
    base = make_custom(nx, ny, nz, h, R, ncap, mids)
    caps = [end_gaussian_cap(nz, h, ncap, s, w0) for w0 in (1.0, 2.0) for s in (8.0, 8.0 * 1.23)]
    caps += [power_cap(nz, ncap, 2.0, order) for order in (2, 4)]
    for left, right in caps:
        T = O.transmission(with_caps(base, left, right), mids, method="dense")
        assert np.max(np.abs(T - expect)) < 5e-4, T
    # a CAP far too weak for this lead reflects: the plateau has an edge
    T = O.transmission(with_caps(base, *end_gaussian_cap(nz, h, ncap, 6.0, 0.25)), mids, method="dense")
    assert np.max(np.abs(T - expect)) > 0.1


# ---------------------------------------------------------------- identities
@pytest.fixture(scope="module")
def small_wire():
    return make_custom(5, 4, 24, 0.5, 3, 4, [0.35, 0.8],
                       wells=[(1.4, 1.1, 5.0, 0.5), (1.7, 1.3, 7.5, 0.3)],
                       atoms_kb=[(0.8, 0.3, 0.1), (0.7, 0.2, 0.12)])


def test_green_function_symmetric(small_wire):
    G = np.linalg.inv(O.operator_A(small_wire, 0.35).toarray())
    assert np.abs(G - G.T).max() < 1e-12 * np.abs(G).max()


def test_reciprocity(small_wire):
    for E in small_wire.energies:
        a = O.transmission(small_wire, [E], method="dense", direction="RL")[0]
        b = O.transmission(small_wire, [E], method="dense", direction="LR")[0]
        assert abs(a - b) <= 1e-12 * max(1.0, a)


def test_optical_theorem_per_column(small_wire):
    wl, wr = O.cap_diagonals(small_wire)
    cols = rhs_columns(small_wire)[::9]
    G = O.green_columns(small_wire, 0.8, cols, method="dense")
    for k, j in enumerate(cols):
        g = G[:, k]
        lhs = np.sum((wl + wr) * np.abs(g) ** 2)
        assert abs(lhs + g[j].imag) < 1e-12 * abs(g[j])


def test_transmission_bounds(small_wire):
    wl, wr = O.cap_diagonals(small_wire)
    cols = rhs_columns(small_wire)
    for E in small_wire.energies:
        t = O.column_transmissions(small_wire, E, method="dense")
        G = O.green_columns(small_wire, E, cols, method="dense")
        upper = np.sum(4 * wr[cols] * (-np.diag(G[cols, :]).imag))
        assert np.all(t >= 0) and t.sum() <= upper * (1 + 1e-12)


def test_routes_agree(small_wire):
    Td = O.transmission(small_wire, method="dense")
    Ts = O.transmission(small_wire, method="splu")
    Ti = O.transmission(small_wire, method="iterative")
    Tsp = O.transmission_spectral(small_wire)
    assert np.max(np.abs(Td - Ts)) < 1e-12
    assert np.max(np.abs(Td - Ti)) < 1e-9
    assert np.max(np.abs(Td - Tsp)) < 1e-10


def test_spectral_route_degenerate_wire():
    # square cross-section with on-axis wells: x <-> y degenerate eigenvalues
    c = 2.5 * 0.5
    w = make_custom(4, 4, 20, 0.5, 2, 4, [0.4, 1.1, 2.0],
                    wells=[(c, c, 4.0, 0.5), (c, c, 7.0, 0.3)])
    Td = O.transmission(w, method="dense")
    Tsp = O.transmission_spectral(w)
    assert np.max(np.abs(Td - Tsp)) < 1e-10


@pytest.fixture(scope="module")
def band_wire():
    """A 2 x 2 x 60 wire with one shallow well and 20-plane CAPs (W0 = 0.5 Ha),
    its energy window inside the first transverse band (T close to 1), the
    full T from dense inversion, and the eigenvalues of H - iW."""
    nx, ny, h, R = 2, 2, 0.5, 2
    th = O.transverse_thresholds(nx, ny, h, R)[0]
    w = make_custom(nx, ny, 60, h, R, 20, np.linspace(th + 0.3, th + 0.8, 6),
                    wells=[(0.75, 0.75, 15.25, 0.5)], w0=0.5)
    Tfull = O.transmission(w, method="dense")
    wl, wr = O.cap_diagonals(w)
    eps = np.linalg.eigvals(O.hamiltonian(w).toarray() - 1j * np.diag(wl + wr))
    return w, Tfull, eps


def _window_distance(w, eps):
    lo, hi = w.energies.min(), w.energies.max()
    return np.maximum(np.maximum(lo - eps.real, eps.real - hi), 0.0)


def test_spectral_truncation_paper_criterion(band_wire):
    """Sec. II.C after Eq. 13: eigenpairs with |E - eps_j|^2 >> Gamma_0^2 may be
    dropped.  Keeping every pole within 4 W0 of the window (|E - eps|^2 >= 16
    W0^2 dropped) must reproduce the full T inside the window (dense route)
    to 2e-3 of T ~ 1 (measured 6.7e-4); the fraction keep = n/N_r keeps exactly
    those poles, since nearness to the window's middle orders them the same
    way.  A selection by the wrong end (farthest poles), or a dropped pole
    near the window, fails the bound."""
    w, Tfull, eps = band_wire
    assert Tfull.min() > 0.9
    W0 = 0.5
    d = _window_distance(w, eps)
    n = int(np.sum(d <= 4 * W0))
    assert 0 < n < len(eps) // 4
    Tp = O.transmission_spectral(w, keep=n / len(eps))
    assert np.max(np.abs(Tp - Tfull)) < 2e-3


def test_spectral_truncation_drops_near_poles_fail(band_wire):
    """The pole-like artefacts the paper warns of: keeping only the poles
    inside the window, or within W0/2 of it, misses T by more than 0.1."""
    w, Tfull, eps = band_wire
    d = _window_distance(w, eps)
    for radius in (0.0, 0.25):
        n = int(np.sum(d <= radius))
        Tp = O.transmission_spectral(w, keep=n / len(eps))
        assert np.max(np.abs(Tp - Tfull)) > 0.1, radius


def test_spectral_truncation_converges_as_p_to_1(band_wire):
    """T_p -> T as the kept fraction p -> 1: within 1e-4 at p = 0.9, and the
    route is exact (to rounding) at p = 1."""
    w, Tfull, _ = band_wire
    assert np.max(np.abs(O.transmission_spectral(w, keep=0.9) - Tfull)) < 1e-4
    assert np.max(np.abs(O.transmission_spectral(w, keep=1.0) - Tfull)) < 1e-10


# ---------------------------------------------------------------- gradient
def test_gradient_dense_matches_fd(small_wire):
    E = 0.8
    g = O.grad_T_dense(small_wire, E)
    pts = [30, 250, 400]
    fd = O.grad_T_fd(small_wire, E, pts, step=1e-5, method="dense")
    assert np.allclose(g[pts], fd, rtol=1e-6, atol=1e-12)


def test_gradient_amplitudes_chain_rule(small_wire):
    from workloads import well_basis

    energies = np.array([0.35, 0.8])
    weights = np.array([1.0, 0.5])
    gV = sum(wt * O.grad_T_dense(small_wire, E) for wt, E in zip(weights, energies))
    dU = -well_basis(small_wire).T @ gV  # V = -sum_a U_a phi_a
    fd = O.grad_T_amplitudes_fd(small_wire, energies, weights, step=1e-5, method="dense")
    assert np.allclose(dU, fd, rtol=1e-6, atol=1e-10)


# ---------------------------------------------------------------- Landauer
def test_landauer_constant_transmission():
    E = np.linspace(-1, 1, 2001)
    T = np.full_like(E, 0.7)
    I = O.landauer_current(E, T, bias=0.2, e_fermi=0.0, kT=0.0)
    assert abs(I - 0.7 * 0.2 / np.pi) < 1e-12
    assert abs(O.landauer_current(E, T, bias=0.2, e_fermi=0.0, kT=0.01) - 0.7 * 0.2 / np.pi) < 1e-6
    assert O.landauer_current(E, T, bias=-0.2, e_fermi=0.0) == pytest.approx(-0.7 * 0.2 / np.pi)


def test_landauer_linear_transmission_closed_form():
    """T(E) = a + b E, zero temperature, bias window on grid points: the
    trapezoid rule is exact, I = (1/pi) [a V + b (mu_L^2 - mu_R^2) / 2]."""
    E = np.arange(-256, 257) / 256.0  # binary spacing: every chemical potential below is a grid point
    a, b = 0.3, 1.7
    T = a + b * E
    for ef, V in [(0.125, 0.25), (-0.25, 0.5), (0.0, -0.375)]:
        mu_l, mu_r = ef + V / 2, ef - V / 2
        exact = (a * V + b * (mu_l ** 2 - mu_r ** 2) / 2) / np.pi
        assert O.landauer_current(E, T, bias=V, e_fermi=ef, kT=0.0) == pytest.approx(exact, abs=1e-14)
    # at finite temperature the window integrates to V for any E_F deep inside the grid
    assert O.landauer_current(E, np.ones_like(E), bias=0.1, e_fermi=0.0, kT=0.02) == \
        pytest.approx(0.1 / np.pi, rel=1e-9)
