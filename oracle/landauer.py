"""Landauer current, Eq. 1 (oracle).

I = (2e/h) int T(E) [f(E - mu_L) - f(E - mu_R)] dE with mu_{L,R} = E_F +- V/2.
Atomic units: e = hbar = 1, so 2e/h = 1/pi (current in a.u.).  The integral is
the trapezoid rule on the supplied energy grid.
"""

from __future__ import annotations

import numpy as np


def fermi(x, kT):
    if kT == 0.0:
        return np.where(x < 0, 1.0, np.where(x > 0, 0.0, 0.5))
    return 0.5 * (1.0 - np.tanh(0.5 * np.asarray(x) / kT))


def landauer_current(energies, T, bias, e_fermi, kT=0.0):
    energies = np.asarray(energies, float)
    T = np.asarray(T, float)
    mu_l, mu_r = e_fermi + 0.5 * bias, e_fermi - 0.5 * bias
    window = fermi(energies - mu_l, kT) - fermi(energies - mu_r, kT)
    return float(np.trapezoid(T * window, energies) / np.pi)
