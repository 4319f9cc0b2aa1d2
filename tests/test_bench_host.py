"""Host logic of bench.py that needs no GPU: the counter summary is used only
for the kernel source, kernel and launch shape it was taken on, and runs on
more than one GPU are refused."""

import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402

KERNEL = "k_cocg_plane<6,double,true,true>"


def _fields():
    out = {}
    for line in bench.COUNTERS.read_text().splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            out[k.strip()] = v.strip()
    return out


def test_committed_counters_are_used_only_for_their_source():
    f = _fields()
    ratio, why = bench._traffic_from_profile(KERNEL, (192, 1))
    if f["kernel_src_sha256_16"] != bench.kernel_source_hash(KERNEL):
        # the source changed after the counters were taken: no traffic figure
        assert ratio is None and "predate" in why
        return
    assert why is None, why
    assert f["launch_shape"] == "192,1"
    assert ratio == pytest.approx(float(f["traffic_over_algorithmic"]))
    # HBM bytes are at least the algorithmic bytes, and not wildly above
    assert 1.0 <= ratio < 1.3


STAND_IN = """// stand-in source
template <int RAD, typename R, bool FUSED, bool NTH>
__global__ void k_cocg_plane(const R* r) {
    body();
}

template <int RAD, typename R>
FusedGeom plane_geom(const negf_op* op, int w) {
    return FusedGeom{};
}
"""


@pytest.fixture
def matched(monkeypatch, tmp_path):
    """The committed counter summary, re-keyed to a stand-in kernel source so
    that the checks below hold whatever the source is now."""
    src = tmp_path / "stencil.hip"
    src.write_text(STAND_IN)
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "KERNEL_HELPERS", tmp_path / "none.h")
    old_hash = _fields()["kernel_src_sha256_16"]
    counters = tmp_path / "counters.txt"
    counters.write_text(bench.COUNTERS.read_text().replace(old_hash,
                                                           bench.kernel_source_hash(KERNEL)))
    monkeypatch.setattr(bench, "COUNTERS", counters)
    return src


def test_ratio_follows_the_tuned_shape(matched):
    f = _fields()
    r192, why = bench._traffic_from_profile(KERNEL, (192, 1))
    assert why is None and r192 == pytest.approx(float(f["traffic_over_algorithmic"]))
    # HBM bytes are at least the algorithmic bytes, and not wildly above
    assert 1.0 <= r192 < 1.3
    # the shape bench.py launches by default has counters
    assert f["launch_shape"] == "%d,%d" % bench.LAUNCH_SHAPE
    # a shape without counters gives none
    r, why = bench._traffic_from_profile(KERNEL, (128, 1))
    assert r is None and "128,1" in why


def test_other_kernel_or_source_gives_no_traffic(matched):
    r, why = bench._traffic_from_profile("k_cocg_apply<6,double,1024,true>", (192, 1))
    assert r is None and "k_cocg_plane" in why
    # edits outside the kernel, its geometry and its helpers keep the figure
    matched.write_text(matched.read_text() + "// changed elsewhere\nvoid other() {\n}\n")
    r, why = bench._traffic_from_profile(KERNEL, (192, 1))
    assert why is None and r is not None
    # an edit of the kernel drops it
    matched.write_text(matched.read_text().replace("body();", "body(); more();"))
    r, why = bench._traffic_from_profile(KERNEL, (192, 1))
    assert r is None and "predate" in why
    # so does an edit of the launch geometry
    matched.write_text(STAND_IN.replace("return FusedGeom{};", "return FusedGeom{1};"))
    r, why = bench._traffic_from_profile(KERNEL, (192, 1))
    assert r is None and "predate" in why


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_unknown_rows_are_refused_before_any_device_work():
    p = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--rows", "small,bogus"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "bogus" in p.stderr and "spectral" in p.stderr
