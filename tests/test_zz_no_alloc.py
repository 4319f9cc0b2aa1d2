"""The operator apply that allocates nothing (negf_apply_operator_noalloc),
through the C ABI, against negf_apply_operator on the same inputs: two calls
in a row, the second on a smaller input, and the size limit of its scratch
array."""

import ctypes as C

import numpy as np
import pytest

from workloads import make_custom, make_wire

pytestmark = pytest.mark.gpu


def _noalloc(lib, op, shifts, x, y, stream=None):
    fn = lib.negf_apply_operator_noalloc
    fn.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    fn.restype = C.c_int
    sh = np.ascontiguousarray(shifts, dtype=np.float64)
    st = fn(op.handle, sh.size, sh.ctypes.data_as(C.c_void_p), C.c_void_p(x.data_ptr()),
            C.c_void_p(y.data_ptr()), C.c_void_p(stream) if stream else None)
    return st


def test_noalloc_apply_matches_apply(gpu_lib):
    import torch

    import paper_1401_0782_amd as P
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    g = torch.Generator(device="cuda").manual_seed(7)
    big = make_wire(2)  # 32x32x192, R = 6, 80 projectors
    h = 0.5
    small = make_custom(9, 7, 40, h, 3, 6, [0.5],
                        wells=[(2.5, 2.0, 10.0, 0.4)], atoms_kb=[(0.8, 0.3, 0.1)])
    for wire, n_vec in ((big, 5), (small, 2)):
        op = P.operator_from_wire(wire)
        x = torch.randn(n_vec, wire.N, dtype=torch.complex128, device="cuda", generator=g)
        shifts = np.linspace(-0.3, 0.9, n_vec)
        y = torch.empty_like(x)
        assert _noalloc(lib, op, shifts, x, y) == _abi.NEGF_OK, lib.negf_last_error()
        torch.cuda.synchronize()
        ref = P.negf_apply_operator(op, shifts, x)
        torch.cuda.synchronize()
        err = ((y - ref).abs().max() / ref.abs().max()).item()
        assert err <= 1e-13, (wire.name, n_vec, err)
        # a device array of shifts on a caller's stream gives the same result
        s = torch.cuda.Stream()
        d_sh = torch.tensor(shifts, device="cuda")
        y2 = torch.empty_like(x)
        fn = lib.negf_apply_operator_noalloc
        st = fn(op.handle, n_vec, C.c_void_p(d_sh.data_ptr()), C.c_void_p(x.data_ptr()),
                C.c_void_p(y2.data_ptr()), C.c_void_p(s.cuda_stream))
        assert st == _abi.NEGF_OK
        s.synchronize()
        assert torch.equal(y2, y)
        op.close()


def test_noalloc_rejects_oversized_and_host_arrays(gpu_lib):
    import torch

    import paper_1401_0782_amd as P
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    wire = make_wire(2)  # 80 projectors: 16 * 80 bytes of coefficients per vector
    op = P.operator_from_wire(wire)
    n_vec = (1 << 20) // (16 * 80) + 1
    x = torch.zeros(n_vec, wire.N, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    assert _noalloc(lib, op, np.zeros(n_vec), x, y) == _abi.NEGF_E_INVALID_ARG
    assert b"scratch" in lib.negf_last_error()
    del x, y
    xh = np.zeros((1, wire.N), np.complex128)
    fn = lib.negf_apply_operator_noalloc
    sh = np.zeros(1)
    yd = torch.empty(1, wire.N, dtype=torch.complex128, device="cuda")
    st = fn(op.handle, 1, sh.ctypes.data_as(C.c_void_p), xh.ctypes.data_as(C.c_void_p),
            C.c_void_p(yd.data_ptr()), None)
    assert st == _abi.NEGF_E_INVALID_ARG
    op.close()
