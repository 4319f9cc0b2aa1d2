"""Python binding of libnegf: same names as the C ABI, argument marshalling only.

Arrays may be numpy arrays (host) or torch tensors; device tensors are passed
to the library as device pointers (it asks the HIP runtime which kind each
pointer is).  Every computation happens in libnegf's HIP kernels.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (NEGF_CORE_AUTO, NEGF_CORE_MULTISHIFT, NEGF_CORE_PER_ENERGY,  # noqa: F401
                   NEGF_DIR_LR, NEGF_DIR_RL, NEGF_FP64, NEGF_MIXED, NEGF_RECOVER_OFF,
                   NEGF_RECOVER_RESTART, NEGF_SOLVER_COCG, NEGF_SOLVER_QMR)


class NegfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"negf {_abi.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _lib():
    return _abi.load()


def _check(status: int, allow=()):
    if status != _abi.NEGF_OK and status not in allow:
        raise NegfError(status, _lib().negf_last_error().decode())
    return status


def _ptr(a):
    """Raw pointer of a numpy array or torch tensor (kept alive by the caller)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    raise TypeError(type(a))


def _c64(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


class Operator:
    """Owning handle of a negf_op."""

    def __init__(self, handle, N, nx, ny, nz):
        self._h = handle
        self.N, self.nx, self.ny, self.nz = N, nx, ny, nz

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("operator destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            _lib().negf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def negf_version() -> str:
    return _lib().negf_version().decode()


def negf_build_operator(nx, ny, nz, h, stencil_radius, v_local, cap_left_z, cap_right_z,
                        kb_offsets=None, kb_idx=None, kb_val=None, kb_energy=None) -> Operator:
    lib = _lib()
    g = _abi.negf_grid(int(nx), int(ny), int(nz), float(h))
    v = np.ascontiguousarray(v_local, dtype=np.float64)
    cl = np.ascontiguousarray(cap_left_z, dtype=np.float64)
    cr = np.ascontiguousarray(cap_right_z, dtype=np.float64)
    if v.size != int(nx) * int(ny) * int(nz) or cl.size != nz or cr.size != nz:
        raise ValueError("array sizes do not match the grid")
    kbp = None
    keep = []
    if kb_energy is not None and len(kb_energy) > 0:
        off = np.ascontiguousarray(kb_offsets, dtype=np.int64)
        idx = np.ascontiguousarray(kb_idx, dtype=np.int32)
        val = np.ascontiguousarray(kb_val, dtype=np.float64)
        ekb = np.ascontiguousarray(kb_energy, dtype=np.float64)
        keep = [off, idx, val, ekb]
        kb = _abi.negf_kb(len(ekb), off.ctypes.data_as(C.POINTER(C.c_int64)),
                          idx.ctypes.data_as(C.POINTER(C.c_int32)),
                          val.ctypes.data_as(C.POINTER(C.c_double)),
                          ekb.ctypes.data_as(C.POINTER(C.c_double)))
        kbp = C.byref(kb)
    out = C.c_void_p()
    _check(lib.negf_build_operator(C.byref(g), int(stencil_radius), _ptr(v), kbp, _ptr(cl),
                                   _ptr(cr), C.byref(out)))
    del keep
    return Operator(out, v.size, int(nx), int(ny), int(nz))


def operator_from_wire(wire) -> Operator:
    """Convenience: build from any object with the wire attributes
    (nx, ny, nz, h, R, v_local, cap_left, cap_right, kb_*)."""
    return negf_build_operator(wire.nx, wire.ny, wire.nz, wire.h, wire.R, wire.v_local,
                               wire.cap_left, wire.cap_right, wire.kb_offsets, wire.kb_idx,
                               wire.kb_val, wire.kb_energy)


def _opts(precision=NEGF_FP64, core=NEGF_CORE_AUTO, direction=NEGF_DIR_RL, tol=0.0,
          max_iter=0, block_width=0, shift_group=0, max_refine=0, col_begin=0, col_count=0,
          stream=None, solver=0, recover=False):
    return _abi.negf_opts(int(precision), int(core), int(solver), int(direction), float(tol),
                          int(max_iter),
                          int(block_width), int(shift_group), int(max_refine), int(col_begin),
                          int(col_count), C.c_void_p(stream) if stream else None,
                          NEGF_RECOVER_RESTART if recover else NEGF_RECOVER_OFF)


def negf_apply_operator(op: Operator, shifts, x, precision=NEGF_FP64):
    """Y = A(E_c) X for X of shape (n_vec, N) (numpy complex128 or torch complex128)."""
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    if isinstance(x, np.ndarray):
        x = _c64(x)
        y = np.empty_like(x)
    else:
        y = x.new_empty(x.shape)
    n_vec = shifts.size
    if x.shape[0] != n_vec or x.shape[1] != op.N:
        raise ValueError("x must be (n_vec, N)")
    _check(_lib().negf_apply_operator(op.handle, int(precision), n_vec, _ptr(shifts), _ptr(x),
                                      _ptr(y)))
    return y


@dataclass
class Diagnostics:
    iters: np.ndarray
    resid: np.ndarray
    t_col: np.ndarray
    item_status: np.ndarray
    total_iters: int = 0
    n_not_converged: int = 0
    seconds: float = 0.0
    status: int = 0
    extra: dict = field(default_factory=dict)
    refine_steps: Optional[np.ndarray] = None
    optical_err: Optional[np.ndarray] = None


def n_source_columns(op: Operator, cap_src) -> int:
    return int(np.count_nonzero(np.asarray(cap_src) > 0)) * op.nx * op.ny


def negf_transmission(op: Operator, energies, n_cols: Optional[int] = None, check=True,
                      time_matvec=False, optical=False, **opts):
    """T(E) (FP64) for the given energies.  n_cols (number of source columns
    in the shard, see col_begin/col_count) enables the per-item diagnostics
    (optical=True adds the per-item optical-theorem error); time_matvec
    brackets the stencil launches with HIP events (an int n > 1 times every
    n-th chunk of the multi-shift core)."""
    energies = np.ascontiguousarray(energies, dtype=np.float64)
    n_e = energies.size
    T = np.zeros(n_e)
    o = _opts(**opts)
    d = None
    arrays = None
    if n_cols or time_matvec:
        nc = max(1, n_cols or 0)
        arrays = (np.zeros((n_e, nc), np.int32), np.zeros((n_e, nc)),
                  np.zeros((n_e, nc)), np.zeros((n_e, nc), np.int32),
                  np.full((n_e, nc), np.nan), np.zeros((n_e, nc), np.int32))
        ptrs = [None] * 4
        extra = [None, None]
        if n_cols:
            ptrs = [arrays[0].ctypes.data_as(C.POINTER(C.c_int32)),
                    arrays[1].ctypes.data_as(C.POINTER(C.c_double)),
                    arrays[2].ctypes.data_as(C.POINTER(C.c_double)),
                    arrays[3].ctypes.data_as(C.POINTER(C.c_int32))]
            extra = [arrays[4].ctypes.data_as(C.POINTER(C.c_double)) if optical else None,
                     arrays[5].ctypes.data_as(C.POINTER(C.c_int32))]
        d = _abi.negf_diag(*ptrs, 0, 0, 0.0, int(time_matvec), 0.0, 0, 0.0, *extra)
    st = _lib().negf_transmission(op.handle, C.byref(o), n_e, _ptr(energies), _ptr(T),
                                  C.byref(d) if d is not None else None)
    if check:
        _check(st)
    if d is None:
        return T
    diag = Diagnostics(arrays[0], arrays[1], arrays[2], arrays[3], int(d.total_iters),
                       int(d.n_not_converged), float(d.seconds), int(st))
    diag.extra.update(matvec_seconds=float(d.matvec_seconds),
                      matvec_launches=int(d.matvec_launches), matvec_bytes=float(d.matvec_bytes))
    diag.refine_steps = arrays[5]
    diag.optical_err = arrays[4] if optical else None
    return T, diag


def negf_solve_columns(op: Operator, energies, rhs_idx=None, rhs_dense=None, row_idx=None,
                       out=None, check=True, **opts):
    """out[e, r, k] = (A(E_e)^-1 b_r)[row_idx[k]]; returns (out, item_status)."""
    energies = np.ascontiguousarray(energies, dtype=np.float64)
    n_e = energies.size
    ridx = None if rhs_idx is None else np.ascontiguousarray(rhs_idx, dtype=np.int32)
    rd = None
    if rhs_dense is not None:
        rd = _c64(rhs_dense) if isinstance(rhs_dense, np.ndarray) else rhs_dense
    n_rhs = ridx.size if ridx is not None else rd.shape[0]
    rows = None if row_idx is None else np.ascontiguousarray(row_idx, dtype=np.int32)
    n_rows = op.N if rows is None else rows.size
    if out is None:
        out = np.zeros((n_e, n_rhs, n_rows), np.complex128)
    status = np.zeros((n_e, n_rhs), np.int32)
    o = _opts(**opts)
    st = _lib().negf_solve_columns(op.handle, C.byref(o), n_e, _ptr(energies), n_rhs, _ptr(ridx),
                                   _ptr(rd), n_rows, _ptr(rows), _ptr(out), _ptr(status))
    if check:
        _check(st)
    return out, status


def negf_transmission_grad(op: Operator, energies, weights, dL_dV=None, want_T=True, **opts):
    """dL/dV for L = sum_e weights[e] T(E_e); returns (dL_dV, T)."""
    energies = np.ascontiguousarray(energies, dtype=np.float64)
    weights = np.ascontiguousarray(weights, dtype=np.float64)
    if dL_dV is None:
        dL_dV = np.zeros(op.N)
    T = np.zeros(energies.size) if want_T else None
    o = _opts(**opts)
    _check(_lib().negf_transmission_grad(op.handle, C.byref(o), energies.size, _ptr(energies),
                                         _ptr(weights), _ptr(dL_dV), _ptr(T)))
    return dL_dV, T


def negf_tune(op: Operator, energies, probe_iters: int = 0, cache: Optional[str] = None,
              **opts) -> dict:
    """Autotune the multi-shift launch shape of op (block width, stencil
    z-chunking, stencil kernel) by timing short probe runs; later calls with
    block_width=0 use the choice.  With cache (a file path) a choice stored
    there for the same operator shape, request and device is used without
    probes (an empty "tried" table), and a new one is appended.  Returns the
    choice and the timing table."""
    e = np.ascontiguousarray(energies, dtype=np.float64)
    o = _opts(**opts)
    res = _abi.negf_tune_result()
    if cache is not None:
        _check(_lib().negf_tune_cached(op.handle, C.byref(o), e.size, _ptr(e), int(probe_iters),
                                       str(cache).encode(), C.byref(res)))
    else:
        _check(_lib().negf_tune(op.handle, C.byref(o), e.size, _ptr(e), int(probe_iters),
                                C.byref(res)))
    n = res.n_tried
    return {
        "block_width": res.block_width,
        "wg_target": res.wg_target,
        "plane_kernel": res.plane_kernel,
        "tried": [(res.tried_block_width[i], res.tried_wg_target[i], res.tried_plane_kernel[i],
                   res.us_per_column_iteration[i]) for i in range(n)],
    }


def negf_set_launch_shape(op: Operator, block_width: int = 0, wg_target: int = 0,
                          plane_kernel: int = -1) -> None:
    """Set op's multi-shift launch shape (e.g. a cached negf_tune choice)."""
    _check(_lib().negf_set_launch_shape(op.handle, int(block_width), int(wg_target),
                                        int(plane_kernel)))


def negf_spectral_transmission(op: Operator, eps, U, energies, keep: float = 1.0):
    """T(E) by the complex-energy diagonalisation route (Eqs. 8-13) from
    eigenpairs of H - iW: eps (n_r,), U (n_r, N) with each row an eigenvector
    normalised to U_i^T U_i = 1 (numpy or a torch device tensor).  keep in
    (0, 1) truncates to the eigenpairs nearest the window."""
    e = np.ascontiguousarray(energies, dtype=np.float64)
    ev = _c64(np.asarray(eps))
    if isinstance(U, np.ndarray):
        U = _c64(U)
    if tuple(U.shape) != (ev.size, op.N):
        raise ValueError("U must be (n_r, N)")
    T = np.zeros(e.size)
    _check(_lib().negf_spectral_transmission(op.handle, ev.size, _ptr(ev), _ptr(U), float(keep),
                                             e.size, _ptr(e), _ptr(T)))
    return T


def negf_eigenpairs(op: Operator, e_lo: float, e_hi: float, margin: float = 0.0,
                    n_lanczos: int = 0, resid_tol: float = 1e-8, max_pairs: int = 0, U=None):
    """Eigenpairs of H - iW near [e_lo, e_hi] by complex-symmetric Lanczos on
    the device (see include/negf.h).  Returns (eps, U, resid) with U of shape
    (n_found, N), each row normalised to U_i^T U_i = 1; U may be a
    preallocated (max_pairs, N) torch device tensor."""
    n_lanczos = int(n_lanczos) if n_lanczos else op.N
    max_pairs = int(max_pairs) if max_pairs else n_lanczos
    eps = np.zeros(max_pairs, np.complex128)
    res = np.zeros(max_pairs)
    if U is None:
        U = np.zeros((max_pairs, op.N), np.complex128)
    n = C.c_int32(0)
    _check(_lib().negf_eigenpairs(op.handle, float(e_lo), float(e_hi), float(margin), n_lanczos,
                                  float(resid_tol), max_pairs, _ptr(eps), _ptr(U), _ptr(res),
                                  C.byref(n)))
    k = n.value
    return eps[:k], U[:k], res[:k]


def negf_current(energies, T, bias, e_fermi: float, kT: float = 0.0, stream=None):
    """Landauer current I(V) (Eq. 1, atomic units) for each bias in `bias`
    from T(E) on the energy grid, computed on the device."""
    e = np.ascontiguousarray(energies, dtype=np.float64)
    t = np.ascontiguousarray(T, dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_1d(bias), dtype=np.float64)
    if t.shape != e.shape:
        raise ValueError("T must match energies")
    out = np.zeros(b.size)
    _check(_lib().negf_current(e.size, _ptr(e), _ptr(t), b.size, _ptr(b), float(e_fermi),
                               float(kT), _ptr(out), C.c_void_p(stream) if stream else None))
    return out


def negf_transmission_batch(ops, energies_list, max_concurrent=0, check=True, shards=None,
                            **opts):
    """T(E) for many junctions at once; returns (list of T arrays, statuses).
    shards: optional per-junction (col_begin, col_count) pairs (each
    junction's own source-column shard, negf_transmission_batch_shards)."""
    n = len(ops)
    es = [np.ascontiguousarray(e, dtype=np.float64) for e in energies_list]
    Ts = [np.zeros(e.size) for e in es]
    n_e = np.array([e.size for e in es], np.int32)
    handles = (C.c_void_p * n)(*[op.handle.value if hasattr(op.handle, "value") else op.handle
                                 for op in ops])
    e_ptrs = (C.c_void_p * n)(*[e.ctypes.data for e in es])
    t_ptrs = (C.c_void_p * n)(*[t.ctypes.data for t in Ts])
    status = np.zeros(n, np.int32)
    o = _opts(**opts)
    if shards is not None:
        sh = np.asarray(shards, np.int32).reshape(n, 2)
        cb, cc = np.ascontiguousarray(sh[:, 0]), np.ascontiguousarray(sh[:, 1])
        st = _lib().negf_transmission_batch_shards(n, handles, C.byref(o), _ptr(n_e), e_ptrs,
                                                   _ptr(cb), _ptr(cc), t_ptrs, _ptr(status),
                                                   int(max_concurrent))
    else:
        st = _lib().negf_transmission_batch(n, handles, C.byref(o), _ptr(n_e), e_ptrs, t_ptrs,
                                            _ptr(status), int(max_concurrent))
    if check:
        _check(st)
    return Ts, status
