"""Host-side checks of the C ABI library (no GPU needed)."""

import ctypes as C
import pathlib
import re

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]


def _header_functions():
    text = (ROOT / "include" / "negf.h").read_text()
    return sorted(set(re.findall(r"\b(negf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    declared = _header_functions()
    assert set(declared) == set(_abi.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.negf_version().decode().startswith("libnegf")


def _build(**kw):
    import paper_1401_0782_amd as P
    from workloads import make_wire

    w = make_wire(1)
    args = dict(nx=w.nx, ny=w.ny, nz=w.nz, h=w.h, stencil_radius=w.R, v_local=w.v_local,
                cap_left_z=w.cap_left, cap_right_z=w.cap_right)
    args.update(kw)
    return P.negf_build_operator(**args)


@pytest.mark.parametrize("bad,msg", [
    (dict(stencil_radius=0), "radius"),
    (dict(stencil_radius=7), "radius"),
    (dict(h=0.0), "grid"),
    (dict(h=-1.0), "grid"),
])
def test_invalid_operator_arguments_rejected_before_device(bad, msg):
    from paper_1401_0782_amd import NegfError
    from paper_1401_0782_amd._abi import NEGF_E_INVALID_ARG

    with pytest.raises(NegfError) as ei:
        _build(**bad)
    assert ei.value.status == NEGF_E_INVALID_ARG and msg in str(ei.value)


def test_invalid_caps_rejected():
    from paper_1401_0782_amd import NegfError
    from workloads import make_wire

    w = make_wire(1)
    bad = w.cap_left.copy()
    bad[3] = -0.1
    for kw in (dict(cap_left_z=bad),
               dict(cap_left_z=np.zeros(w.nz)),
               dict(cap_left_z=np.r_[w.cap_left[:1] * 0, w.cap_left[1:]]),  # not touching wall
               dict(cap_left_z=np.r_[[0.5] * 20, [0.0] * 12], cap_right_z=np.r_[[0.0] * 12, [0.5] * 20]),
               dict(cap_left_z=np.r_[[0.5], [0.0] * 31]),  # fewer than R planes
               ):
        with pytest.raises(NegfError):
            _build(**kw)


def test_nan_potential_rejected():
    from paper_1401_0782_amd import NegfError
    from workloads import make_wire

    v = make_wire(1).v_local.copy()
    v[5] = np.nan
    with pytest.raises(NegfError, match="not finite"):
        _build(v_local=v)


def test_projector_on_cap_plane_rejected():
    from paper_1401_0782_amd import NegfError

    with pytest.raises(NegfError, match="CAP plane"):
        _build(kb_offsets=np.array([0, 1]), kb_idx=np.array([3]), kb_val=np.array([1.0]),
               kb_energy=np.array([0.2]))


def test_null_output_rejected():
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    g = _abi.negf_grid(4, 4, 8, 0.5)
    assert lib.negf_build_operator(C.byref(g), 2, None, None, None, None, None) == _abi.NEGF_E_INVALID_ARG
    assert b"null" in lib.negf_last_error()
    lib.negf_destroy(None)  # no-op


def test_tune_rejects_null_operator():
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    e = np.array([0.3])
    assert lib.negf_tune(None, None, 1, e.ctypes.data, 0, None) == _abi.NEGF_E_INVALID_ARG
    assert b"null op" in lib.negf_last_error()


def test_tune_result_layout_matches_header():
    """The ctypes mirror of negf_tune_result has the header's field order and size."""
    from paper_1401_0782_amd import _abi

    text = (ROOT / "include" / "negf.h").read_text()
    body = re.search(r"typedef struct \{((?:(?!typedef).)*?)\} negf_tune_result;", text, re.S).group(1)
    fields = re.findall(r"\b(int32_t|double)\s+([a-z_]+)(\[NEGF_TUNE_MAX\])?;", body)
    assert [f[1] for f in fields] == [f[0] for f in _abi.negf_tune_result._fields_]
    n_max = int(re.search(r"#define NEGF_TUNE_MAX (\d+)", text).group(1))
    assert n_max == _abi.NEGF_TUNE_MAX
    size = sum((4 if t == "int32_t" else 8) * (n_max if arr else 1) for t, _, arr in fields)
    assert C.sizeof(_abi.negf_tune_result) == size


def test_set_launch_shape_validates_without_device():
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    assert lib.negf_set_launch_shape(None, 64, 256, 1) == _abi.NEGF_E_INVALID_ARG
    assert b"null op" in lib.negf_last_error()


def test_current_validates_before_device():
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    e = np.array([0.1, 0.3, 0.2])  # not increasing
    t = np.ones(3)
    b = np.array([0.1])
    out = np.zeros(1)
    args = (e.ctypes.data, t.ctypes.data, 1, b.ctypes.data, 0.2, 0.0, out.ctypes.data, None)
    assert lib.negf_current(3, *args) == _abi.NEGF_E_INVALID_ARG
    assert b"increasing" in lib.negf_last_error()
    assert lib.negf_current(1, *args) == _abi.NEGF_E_INVALID_ARG
    e2 = np.array([0.1, 0.2, 0.3])
    assert lib.negf_current(3, e2.ctypes.data, t.ctypes.data, 1, b.ctypes.data, 0.2, -1.0,
                            out.ctypes.data, None) == _abi.NEGF_E_INVALID_ARG


def test_spectral_rejects_null_operator():
    from paper_1401_0782_amd import _abi

    lib = _abi.load()
    e = np.array([0.3])
    assert lib.negf_spectral_transmission(None, 1, None, None, 1.0, 1, e.ctypes.data,
                                          None) == _abi.NEGF_E_INVALID_ARG


def test_opts_layout_matches_header():
    """The ctypes mirror of negf_opts has the header's field order."""
    from paper_1401_0782_amd import _abi

    text = (ROOT / "include" / "negf.h").read_text()
    body = re.search(r"typedef struct \{((?:(?!typedef).)*?)\} negf_opts;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(int32_t|double|void\*)\s+([a-z_]+);", body)
    assert [f[1] for f in fields] == [f[0] for f in _abi.negf_opts._fields_]


@pytest.mark.parametrize("R,max_nx", [(1, 1024), (2, 1020), (3, 725), (4, 560), (5, 455), (6, 381)])
def test_x_rows_wider_than_the_stencil_tile_rejected(R, max_nx):
    """One x-row with its radius-R halo must fit the double-buffered FP64 LDS
    tile (160 KB), one thread per point: wider grids are refused by the
    build, before any device work; the widest admitted row passes that
    check."""
    from paper_1401_0782_amd import NegfError
    from paper_1401_0782_amd._abi import NEGF_E_INVALID_ARG

    assert max_nx == min(1024, 163840 // (32 * (2 * R + 1)) - 2 * R)
    nz = 2 * R + 4
    cap_l = np.zeros(nz)
    cap_l[:R] = 0.1
    cap_r = cap_l[::-1].copy()
    kw = dict(ny=1, nz=nz, stencil_radius=R, cap_left_z=cap_l, cap_right_z=cap_r)
    with pytest.raises(NegfError) as ei:
        _build(nx=max_nx + 1, v_local=np.zeros((max_nx + 1) * nz), **kw)
    assert ei.value.status == NEGF_E_INVALID_ARG and "widest x-row" in str(ei.value)
    try:  # without a device this fails later, for another reason
        _build(nx=max_nx, v_local=np.zeros(max_nx * nz), **kw)
    except NegfError as e:
        assert "widest x-row" not in str(e)


@pytest.mark.parametrize("nx,ny,ok", [(2, 512, False), (3, 400, False), (4, 256, True),
                                      (32, 32, True), (40, 40, True), (64, 64, True)])
def test_planes_whose_stencil_tile_overflows_lds_rejected(nx, ny, ok):
    """At R = 6 the tile of a narrow, tall plane (whole plane, or 1024 / nx
    rows) with its halo exceeds 160 KB of LDS: refused before device work.
    Square cross-sections pass the check."""
    from paper_1401_0782_amd import NegfError
    from paper_1401_0782_amd._abi import NEGF_E_INVALID_ARG

    R, nz = 6, 16
    cap_l = np.zeros(nz)
    cap_l[:R] = 0.1
    kw = dict(nx=nx, ny=ny, nz=nz, stencil_radius=R, v_local=np.zeros(nx * ny * nz),
              cap_left_z=cap_l, cap_right_z=cap_l[::-1].copy())
    if not ok:
        with pytest.raises(NegfError) as ei:
            _build(**kw)
        assert ei.value.status == NEGF_E_INVALID_ARG and "stencil tile in LDS" in str(ei.value)
        return
    try:  # without a device this fails later, for another reason
        _build(**kw)
    except NegfError as e:
        assert "stencil tile" not in str(e) and "widest x-row" not in str(e)


def test_enum_constants_match_header():
    """Every enumerator of include/negf.h has the same value in the binding."""
    from paper_1401_0782_amd import _abi

    text = re.sub(r"/\*.*?\*/", "", (ROOT / "include" / "negf.h").read_text(), flags=re.S)
    found = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", text, re.S):
        for name, val in re.findall(r"\b(NEGF_[A-Z0-9_]+)\s*=\s*(\d+)", body):
            found[name] = int(val)
    assert len(found) >= 21
    for name, val in found.items():
        assert getattr(_abi, name) == val, name


def test_header_is_plain_c_and_links_from_c(tmp_path):
    """include/negf.h compiles as C99 and C++17 without warnings, and a plain
    C program links against libnegf.so and calls an entry point that needs
    no GPU (the version string) and one that rejects its arguments before any
    device work."""
    import shutil
    import subprocess

    from paper_1401_0782_amd import _abi

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    inc = ROOT / "include"
    for lang, std in (("c", "-std=c99"), ("c++", "-std=c++17")):
        r = subprocess.run([gcc if lang == "c" else (shutil.which("g++") or gcc), std, "-Wall",
                            "-Wextra", "-Werror", "-fsyntax-only", "-x", lang,
                            str(inc / "negf.h")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
    src = tmp_path / "use.c"
    src.write_text(
        '#include <stdio.h>\n#include <string.h>\n#include "negf.h"\n'
        "int main(void) {\n"
        "    const char* v = negf_version();\n"
        "    negf_op* op = 0;\n"
        "    negf_status s = negf_build_operator(0, 2, 0, 0, 0, 0, &op);\n"
        '    printf("%s|%d|%d\\n", v, (int)s, op == 0);\n'
        "    return strlen(v) > 0 ? 0 : 1;\n}\n")
    exe = tmp_path / "use"
    lib = _abi.LIB_PATH
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", f"-I{inc}", str(src), "-o", str(exe),
                        f"-L{lib.parent}", "-lnegf", f"-Wl,-rpath,{lib.parent}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    version, status, untouched = r.stdout.strip().split("|")
    assert version.startswith("libnegf")
    assert int(status) == _abi.NEGF_E_INVALID_ARG and untouched == "1"
