"""Seeded synthetic wire junctions.

The paper's workloads are DFT junctions (Au chains, Au(111) nanowires with an
atom, BDT or C60 between them; Sec. III).  Their Kohn-Sham potentials and
pseudopotentials are not available, so these generators stand in for them with
the same structure: a uniform real-space grid of spacing h (Sec. II.D), a local
potential made of attractive Gaussian wells, short-ranged separable (KB) s+p
projectors inside a cutoff sphere (the non-local pseudopotential part named in
Sec. II.C), and absorbing potentials that depend on z only (Sec. II.B, Eq. 5).

Conventions (all stated once here, used everywhere):

* grid point (ix, iy, iz), 0-based, sits at ((ix+1)h, (iy+1)h, (iz+1)h);
  linear index i = ix + nx*(iy + ny*iz) (x fastest);
* the CAP on each end is a quartic ramp W_q = W0 (q/n_cap)^4, q = 1..n_cap
  counted from the inner edge outward, so the outermost plane carries W0;
* wells: V(r) = -sum_a U_a exp(-|r - R_a|^2 / w_a^2);
* KB projectors: s: exp(-d^2/r_a^2); p_x,p_y,p_z: (x-X) exp(-d^2/r_a^2) etc.,
  kept where d <= 2 bohr, normalised to unit 2-norm over grid points;
* energies are inclusive linspace grids;
* random draws use numpy.random.default_rng([14010782, cfg_id, junction_id])
  in the order: well depths, well positions, KB radii, KB s energies,
  KB p energies.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 14010782
KB_CUTOFF = 2.0  # bohr
WELL_WIDTH = 1.0  # bohr
CAP_PEAK = 0.5  # Ha


@dataclasses.dataclass
class Wire:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    R: int
    v_local: np.ndarray  # (N,) float64
    cap_left: np.ndarray  # (nz,) float64
    cap_right: np.ndarray  # (nz,) float64
    energies: np.ndarray  # (n_e,) float64
    n_cap: int
    well_centers: np.ndarray  # (n_a, 3)
    well_widths: np.ndarray  # (n_a,)
    well_depths: np.ndarray  # (n_a,)  U_a > 0 (attractive)
    kb_offsets: Optional[np.ndarray] = None  # (n_p+1,) int64
    kb_idx: Optional[np.ndarray] = None  # (nnz,) int32
    kb_val: Optional[np.ndarray] = None  # (nnz,) float64
    kb_energy: Optional[np.ndarray] = None  # (n_p,) float64
    block_width: int = 64

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_proj(self) -> int:
        return 0 if self.kb_energy is None else int(self.kb_energy.shape[0])

    def coords(self):
        """Physical coordinates (x, y, z) of every grid point, each (N,)."""
        iz, iy, ix = np.meshgrid(np.arange(self.nz), np.arange(self.ny),
                                 np.arange(self.nx), indexing="ij")
        return ((ix.ravel() + 1) * self.h, (iy.ravel() + 1) * self.h,
                (iz.ravel() + 1) * self.h)


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def power_cap(nz: int, n_cap: int, w0: float = CAP_PEAK, order: int = 4):
    """Monomial ramp CAP W_q = w0 (q / n_cap)^order on the n_cap end planes
    (q = 1 innermost .. n_cap outermost); per-plane (left, right), each (nz,)."""
    left = np.zeros(nz)
    right = np.zeros(nz)
    for q in range(1, n_cap + 1):
        val = w0 * (q / n_cap) ** order
        left[n_cap - q] = val  # q = n_cap -> plane 0 (outermost)
        right[nz - n_cap - 1 + q] = val  # q = n_cap -> plane nz-1
    return left, right


def quartic_cap(nz: int, n_cap: int, w0: float = CAP_PEAK):
    """Per-plane CAP profiles (left, right), each (nz,): the order-4 ramp."""
    return power_cap(nz, n_cap, w0, 4)


def end_gaussian_cap(nz: int, h: float, n_cap: int, sigma: float, w0: float):
    """Gaussian CAP of Eq. (5) centred on the outermost plane of each end and
    kept on the n_cap end planes (zero further in, where it has decayed below
    w0 exp(-(n_cap h / sigma)^2)), so that the two absorbing regions stay
    disjoint."""
    z = np.arange(nz)
    left = np.where(z < n_cap, w0 * np.exp(-((z * h) ** 2) / sigma ** 2), 0.0)
    right = np.where(z >= nz - n_cap, w0 * np.exp(-(((nz - 1 - z) * h) ** 2) / sigma ** 2), 0.0)
    return left, right


def riss_meyer_strength(length: float, order: int, e_kin_lo: float, e_kin_hi: float) -> float:
    """Strength eta of a monomial CAP W(z) = eta (z / length)^order, 0 <= z <=
    length, tuned to a window of longitudinal kinetic energies in the way
    Riss and Meyer analyse such CAPs (the reference the paper gives, in
    Sec. III.E, for a more efficient absorber than Eq. 5): in atomic units,
    a wave of wavenumber k is
      * reflected at the CAP's onset with the first-order (Born) amplitude
        |r| = eta order! / (k length^order (2k)^(order+1)), largest at the
        low end of the window;
      * transmitted through the CAP, reflected by the box end and returned
        with weight exp(-4 eta length / ((order + 1) k)) (WKB), largest at
        the high end.
    eta balances the two worst cases, |r(k_lo)|^2 = exp(...)(k_hi), which
    minimises the larger of them (one rises with eta, the other falls)."""
    if not (length > 0 and order >= 1 and 0 < e_kin_lo < e_kin_hi):
        raise ValueError("need length > 0, order >= 1 and 0 < e_kin_lo < e_kin_hi")
    k_lo, k_hi = math.sqrt(2.0 * e_kin_lo), math.sqrt(2.0 * e_kin_hi)
    fact = math.factorial(order)

    def gap(log_eta):  # log reflection(k_lo) - log round trip(k_hi)
        eta = math.exp(log_eta)
        log_r2 = 2.0 * (math.log(eta * fact) - math.log(k_lo) - order * math.log(length)
                        - (order + 1) * math.log(2.0 * k_lo))
        log_t = -4.0 * eta * length / ((order + 1) * k_hi)
        return log_r2 - log_t

    lo, hi = math.log(1e-12), math.log(1e12)
    for _ in range(200):  # bisection: gap rises monotonically with eta
        mid = 0.5 * (lo + hi)
        if gap(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    return math.exp(0.5 * (lo + hi))


def riss_meyer_error(length: float, order: int, eta: float, e_kin: float) -> float:
    """The two estimates above at one kinetic energy, summed: |r|^2 + round trip."""
    k = math.sqrt(2.0 * e_kin)
    r = eta * math.factorial(order) / (k * length ** order * (2.0 * k) ** (order + 1))
    return r * r + math.exp(-4.0 * eta * length / ((order + 1) * k))


def riss_meyer_cap(nz: int, h: float, n_cap: int, e_kin_lo: float, e_kin_hi: float,
                   order: int = 2):
    """Monomial CAP on the n_cap end planes (onset one plane inside, length
    n_cap h) with the strength riss_meyer_strength picks for the window;
    returns (left, right, eta)."""
    eta = riss_meyer_strength(n_cap * h, order, e_kin_lo, e_kin_hi)
    left, right = power_cap(nz, n_cap, eta, order)
    return left, right, eta


def with_caps(wire, left, right, name=None):
    """A copy of wire with other per-plane CAP profiles."""
    import dataclasses

    return dataclasses.replace(wire, cap_left=np.asarray(left, float),
                               cap_right=np.asarray(right, float),
                               name=name or wire.name)


def gaussian_cap(nz: int, h: float, z_left: float, z_right: float,
                 sigma: float, w0: float):
    """Gaussian CAP of Eq. (5), centred at z_left / z_right (bohr)."""
    z = (np.arange(nz) + 1) * h
    left = w0 * np.exp(-((z - z_left) ** 2) / sigma ** 2)
    right = w0 * np.exp(-((z - z_right) ** 2) / sigma ** 2)
    return left, right


def _wells_potential(coords, centers, widths, depths):
    x, y, z = coords
    v = np.zeros_like(x)
    for c, w, u in zip(centers, widths, depths):
        d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        v -= u * np.exp(-d2 / w ** 2)
    return v


def _kb_projectors(coords, centers, radii, e_s, e_p):
    x, y, z = coords
    offsets = [0]
    idx_list, val_list, energies = [], [], []
    for c, ra, es, ep in zip(centers, radii, e_s, e_p):
        dx, dy, dz = x - c[0], y - c[1], z - c[2]
        d2 = dx * dx + dy * dy + dz * dz
        sel = np.nonzero(d2 <= KB_CUTOFF ** 2)[0]
        g = np.exp(-d2[sel] / ra ** 2)
        for shape, en in ((g, es), (dx[sel] * g, ep), (dy[sel] * g, ep),
                          (dz[sel] * g, ep)):
            nrm = np.sqrt(np.sum(shape * shape))
            keep = shape != 0.0
            idx_list.append(sel[keep].astype(np.int32))
            val_list.append(shape[keep] / nrm)
            energies.append(en)
            offsets.append(offsets[-1] + int(keep.sum()))
    return (np.asarray(offsets, dtype=np.int64),
            np.concatenate(idx_list).astype(np.int32),
            np.concatenate(val_list).astype(np.float64),
            np.asarray(energies, dtype=np.float64))


def _finish(name, nx, ny, nz, h, R, n_cap, energies, centers, depths,
            kb=None, block_width=64, w0=CAP_PEAK):
    widths = np.full(len(depths), WELL_WIDTH)
    tmp = Wire(name, nx, ny, nz, h, R, np.zeros(0), np.zeros(0), np.zeros(0),
               np.asarray(energies, float), n_cap, np.asarray(centers, float).reshape(-1, 3),
               widths, np.asarray(depths, float), block_width=block_width)
    crd = tmp.coords()
    tmp.v_local = _wells_potential(crd, tmp.well_centers, widths, tmp.well_depths)
    tmp.cap_left, tmp.cap_right = quartic_cap(nz, n_cap, w0)
    if kb is not None:
        radii, e_s, e_p = kb
        (tmp.kb_offsets, tmp.kb_idx, tmp.kb_val,
         tmp.kb_energy) = _kb_projectors(crd, tmp.well_centers, radii, e_s, e_p)
    return tmp


def _axis_wells(rng, n, nx, ny, nz, h, n_cap):
    depths = rng.uniform(0.2, 0.6, size=n)
    zlo = (n_cap + 1) * h + WELL_WIDTH
    zhi = (nz - n_cap) * h - WELL_WIDTH
    zs = rng.uniform(zlo, zhi, size=n)
    cx, cy = (nx + 1) * h / 2.0, (ny + 1) * h / 2.0
    centers = np.stack([np.full(n, cx), np.full(n, cy), zs], axis=1)
    return centers, depths


def _atoms(rng, n, nx, ny, nz, h, n_cap):
    depths = rng.uniform(0.2, 0.6, size=n)
    xs = rng.uniform(h, nx * h, size=n)
    ys = rng.uniform(h, ny * h, size=n)
    # KB spheres stay at least one plane clear of the CAP planes
    zlo = (n_cap + 2) * h + KB_CUTOFF
    zhi = (nz - n_cap - 1) * h - KB_CUTOFF
    zs = rng.uniform(zlo, zhi, size=n)
    return np.stack([xs, ys, zs], axis=1), depths


def _kb_draws(rng, n):
    radii = rng.uniform(0.6, 1.0, size=n)
    e_s = rng.uniform(0.1, 0.5, size=n)
    e_p = rng.uniform(0.05, 0.25, size=n)
    return radii, e_s, e_p


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    1: "wire 8x8x32 h=0.5 R=2, 4 axis wells, CAP 6, 384 columns x 8 energies",
    2: "wire 32x32x192 h=0.4 R=6, 20 atoms + s,p KB, CAP 16, 16384 columns x 256 energies",
    3: "64 junctions 16^2x64 .. 40^2x160 h=0.4 R=6, 4-30 atoms, CAP 8-16, 32-256 energies",
    4: "wire 24x24x96 h=0.5 R=4, 10 axis wells, CAP 12, 6912 columns x 64 energies",
    5: "wire 64x64x256 h=0.35 R=6, 80 atoms + s,p KB, CAP 20, 81920 columns x 1024 energies",
}


def make_wire(cfg_id: int, junction_id: int = 0) -> Wire:
    """Return the seeded workload `cfg_id` (1, 2, 4 or 5; 3 via make_junctions)."""
    rng = np.random.default_rng([SEED_BASE, cfg_id, junction_id])
    if cfg_id == 1:
        nx, ny, nz, h, R, n_cap = 8, 8, 32, 0.5, 2, 6
        c, d = _axis_wells(rng, 4, nx, ny, nz, h, n_cap)
        return _finish("wire-8x8x32-R2", nx, ny, nz, h, R, n_cap,
                       np.linspace(0.1, 0.6, 8), c, d, block_width=64)
    if cfg_id == 2:
        nx, ny, nz, h, R, n_cap = 32, 32, 192, 0.4, 6, 16
        c, d = _atoms(rng, 20, nx, ny, nz, h, n_cap)
        kb = _kb_draws(rng, 20)
        return _finish("wire-32x32x192-R6-kb", nx, ny, nz, h, R, n_cap,
                       np.linspace(0.05, 0.8, 256), c, d, kb=kb, block_width=64)
    if cfg_id == 4:
        nx, ny, nz, h, R, n_cap = 24, 24, 96, 0.5, 4, 12
        c, d = _axis_wells(rng, 10, nx, ny, nz, h, n_cap)
        return _finish("wire-24x24x96-R4", nx, ny, nz, h, R, n_cap,
                       np.linspace(0.1, 0.6, 64), c, d, block_width=64)
    if cfg_id == 5:
        nx, ny, nz, h, R, n_cap = 64, 64, 256, 0.35, 6, 20
        c, d = _atoms(rng, 80, nx, ny, nz, h, n_cap)
        kb = _kb_draws(rng, 80)
        return _finish("wire-64x64x256-R6-kb", nx, ny, nz, h, R, n_cap,
                       np.linspace(0.0, 1.0, 1024), c, d, kb=kb, block_width=128)
    raise ValueError(f"unknown workload {cfg_id}")


def make_junctions(n_junctions: int = 64):
    """The batched workload: uneven junctions (local potentials only)."""
    rng = np.random.default_rng([SEED_BASE, 3])
    n_perp = rng.integers(16, 41, size=n_junctions)
    n_atoms = rng.integers(4, 31, size=n_junctions)
    n_caps = rng.integers(8, 17, size=n_junctions)
    n_es = rng.integers(32, 257, size=n_junctions)
    out = []
    for j in range(n_junctions):
        jr = np.random.default_rng([SEED_BASE, 3, j + 1])
        nx = ny = int(n_perp[j])
        nz = 4 * nx
        h, R, n_cap = 0.4, 6, int(n_caps[j])
        c, d = _atoms(jr, int(n_atoms[j]), nx, ny, nz, h, n_cap)
        out.append(_finish(f"junction{j}-{nx}x{ny}x{nz}", nx, ny, nz, h, R, n_cap,
                           np.linspace(0.05, 0.8, int(n_es[j])), c, d, block_width=64))
    return out


def make_custom(nx, ny, nz, h, R, n_cap, energies, wells=(), atoms_kb=None,
                w0=CAP_PEAK, name="custom", block_width=64):
    """Small hand-specified wire.

    wells: iterable of (x, y, z, depth); width WELL_WIDTH.
    atoms_kb: optional iterable of (r_a, E_s, E_p), one per well, adds KB
    projectors centred on the wells.
    """
    wells = list(wells)
    centers = np.array([[w[0], w[1], w[2]] for w in wells], float).reshape(-1, 3)
    depths = np.array([w[3] for w in wells], float)
    kb = None
    if atoms_kb is not None:
        a = np.asarray(list(atoms_kb), float).reshape(-1, 3)
        kb = (a[:, 0], a[:, 1], a[:, 2])
    return _finish(name, nx, ny, nz, h, R, n_cap, np.asarray(energies, float),
                   centers, depths, kb=kb, block_width=block_width, w0=w0)


# ----------------------------------------------------------------------------
# index sets and well basis
# ----------------------------------------------------------------------------

def _plane_points(wire: Wire, planes):
    per = wire.nx * wire.ny
    return np.concatenate([np.arange(z * per, (z + 1) * per) for z in planes]).astype(np.int64)


def rhs_columns(wire: Wire) -> np.ndarray:
    """Grid indices j with W_R(j) > 0, ascending (z-major)."""
    planes = [z for z in range(wire.nz) if wire.cap_right[z] > 0]
    return _plane_points(wire, planes)


def left_support(wire: Wire) -> np.ndarray:
    """Grid indices i with W_L(i) > 0, ascending."""
    planes = [z for z in range(wire.nz) if wire.cap_left[z] > 0]
    return _plane_points(wire, planes)


def well_basis(wire: Wire) -> np.ndarray:
    """phi_a(r) = exp(-|r-R_a|^2/w_a^2), (N, n_a); V = -phi @ U."""
    x, y, z = wire.coords()
    out = np.empty((wire.N, len(wire.well_depths)))
    for a, (c, w) in enumerate(zip(wire.well_centers, wire.well_widths)):
        d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        out[:, a] = np.exp(-d2 / w ** 2)
    return out


def potential_from_amplitudes(wire: Wire, depths) -> np.ndarray:
    return _wells_potential(wire.coords(), wire.well_centers, wire.well_widths,
                            np.asarray(depths, float))
