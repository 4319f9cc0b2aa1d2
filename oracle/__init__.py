"""CPU FP64 oracle for the real-space NEGF transmission path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package; only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.
It shares no code with the GPU path: the only common module is ``workloads``,
which draws seeded inputs and contains none of the method's arithmetic.

What it computes (each function cites the passage it follows):

* the real-space Kohn-Sham-like operator: high-order finite-difference
  kinetic term, local potential and separable non-local projectors
  (Sec. II.C), with z-only absorbing potentials (Sec. II.B, Eqs. 4-5);
* the retarded Green's function columns G = (E - H + iW)^-1 e_j (Eq. 3 with
  the absorbing potential playing the anti-Hermitian self-energy, Eq. 4) by
  dense inversion, sparse LU or an iterative solve with a checked true
  residual;
* the transmission T(E) = 4 sum_{i in L, j in R} W_L,i W_R,j |G_ij|^2
  (Eq. 7, with the factor 4 that relates the absorbing potential W to the
  coupling matrix Gamma = 2W of Eq. 2);
* the paper's own spectral route, Eqs. 8-13, with all eigenpairs;
* closed forms used as pins (exact 1-D lead self-energy, on-site impurity,
  transverse mode counting);
* the gradient dT/dV(r) from dG = G dA G, and central finite differences;
* the Landauer current, Eq. 1.

Pins for every function live in tests/test_oracle_*.py (run with
-m "not gpu").  Functions without an independent pin say "parity unpinned".
"""

from .operator import (  # noqa: F401
    fd_second_derivative_weights,
    second_difference_1d,
    kinetic_operator,
    kb_matrix,
    hamiltonian,
    cap_diagonals,
    operator_A,
)
from .solve import (  # noqa: F401
    green_columns,
    transmission,
    column_transmissions,
    solve_iterative,
)
from .spectral import transmission_spectral  # noqa: F401
from .closed_forms import (  # noqa: F401
    chain_self_energy,
    chain_transmission_exact,
    impurity_transmission_closed_form,
    transverse_thresholds,
)
from .gradient import grad_T_dense, grad_T_fd, grad_T_amplitudes_fd  # noqa: F401
from .landauer import landauer_current  # noqa: F401
