"""The Riss-Meyer-tuned monomial CAP (the more efficient absorber the paper
points to among its future work, Sec. III.E) on an empty 1-D chain, where
the exact transmission of the single channel is 1 at every energy of the
band: the oracle's T(E) (dense inversion of Eq. 7) then measures the CAP's
own error.

* with the strength the estimates pick for a window of kinetic energies,
  max |T - 1| over the window stays within twice the estimated amplitude
  error sqrt(|r|^2 + round trip) at the window's ends;
* three times weaker or stronger, the error is larger (the pick sits near
  the optimum of the reflection / transmission trade-off);
* longer CAPs and higher orders absorb better at the balanced strength.
"""

import math

import numpy as np
import pytest

import oracle as O
from workloads import make_custom, power_cap, riss_meyer_error, riss_meyer_strength, with_caps

H, R = 0.4, 2
EKIN = np.linspace(0.3, 1.5, 25)


def _chain_error(n_cap, order, eta):
    nz = 2 * n_cap + 20
    thr = O.transverse_thresholds(1, 1, H, R)[0]
    E = thr + EKIN
    base = make_custom(1, 1, nz, H, R, n_cap, E)
    wire = with_caps(base, *power_cap(nz, n_cap, eta, order))
    return np.abs(O.transmission(wire, E, method="dense") - 1.0).max()


@pytest.mark.parametrize("n_cap,order", [(12, 2), (20, 2), (30, 3)])
def test_tuned_strength_is_near_the_optimum(n_cap, order):
    L = n_cap * H
    eta = riss_meyer_strength(L, order, EKIN[0], EKIN[-1])
    # at the balance the two worst-case estimates are equal
    k_lo, k_hi = math.sqrt(2 * EKIN[0]), math.sqrt(2 * EKIN[-1])
    r_lo = eta * math.factorial(order) / (k_lo * L ** order * (2 * k_lo) ** (order + 1))
    t_hi = math.exp(-4 * eta * L / ((order + 1) * k_hi))
    assert r_lo ** 2 == pytest.approx(t_hi, rel=1e-9)
    bound = 2.0 * math.sqrt(max(riss_meyer_error(L, order, eta, EKIN[0]),
                                riss_meyer_error(L, order, eta, EKIN[-1])))
    err = _chain_error(n_cap, order, eta)
    print(f"n_cap {n_cap} order {order}: eta {eta:.4f}, max|T-1| {err:.2e} (bound {bound:.2e})")
    assert err <= bound
    for f in (1 / 3, 3.0):
        assert _chain_error(n_cap, order, eta * f) > err


def test_longer_and_higher_order_absorb_better():
    errs = [_chain_error(n, o, riss_meyer_strength(n * H, o, EKIN[0], EKIN[-1]))
            for n, o in [(12, 2), (20, 2), (30, 3)]]
    assert errs[0] > errs[1] > errs[2]


def test_strength_rejects_bad_windows():
    with pytest.raises(ValueError):
        riss_meyer_strength(4.0, 2, 1.0, 0.5)
    with pytest.raises(ValueError):
        riss_meyer_strength(0.0, 2, 0.5, 1.0)
