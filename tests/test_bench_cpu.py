"""bench.py host logic: the roofline's measured-traffic figure is reported only while the
counter summary it comes from was taken on the current kernel sources, headers and build
flags."""
import importlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench():
    return importlib.import_module("bench")


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    bench = _bench()
    f = tmp_path / "counters.txt"
    h = bench.kernel_source_hash()
    f.write_text(f"hbm_bytes_per_launch: 1234567\nkernel_source_sha256_16: {h}\n")
    monkeypatch.setattr(bench, "COUNTERS", str(f))
    assert bench.measured_traffic() == 1234567.0
    f.write_text("hbm_bytes_per_launch: 1234567\nkernel_source_sha256_16: 0000000000000000\n")
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    import subprocess

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_three_dimensional_traffic_follows_its_own_source(tmp_path):
    bench = _bench()
    f = tmp_path / "counters3.txt"
    h3 = bench.kernel_source_hash(bench.KERNEL3_FILES)
    f.write_text(f"hbm_bytes_per_launch: 7654321\nkernel_source_sha256_16: {h3}\n")
    assert bench.measured_traffic(str(f), bench.KERNEL3_FILES) == 7654321.0
    # the 2-D source's hash does not validate the 3-D summary
    if bench.kernel_source_hash() != h3:
        assert bench.measured_traffic(str(f)) is None


def test_hash_covers_headers_and_build_flags(tmp_path, monkeypatch):
    """A change to a header the kernels include (or to the build flags) changes the digest,
    so counters taken before it are no longer reported."""
    bench = _bench()
    files = []
    for path in bench.KERNEL_FILES:
        q = tmp_path / os.path.basename(path)
        q.write_bytes(open(path, "rb").read())
        files.append(str(q))
    h0 = bench.kernel_source_hash(files)
    for q in files:
        old = open(q, "rb").read()
        open(q, "ab").write(b"\n// changed\n")
        assert bench.kernel_source_hash(files) != h0, q
        open(q, "wb").write(old)
    assert bench.kernel_source_hash(files) == h0
    names = {os.path.basename(p) for p in bench.KERNEL_FILES}
    assert {"kernels.hip", "dilbm_internal.h", "device_common.h", "build.py"} <= names
