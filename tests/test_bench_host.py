"""Host-side logic of bench.py (no GPU): the one-GPU guard, the output
fingerprints that compare served and plain results, the host record of
the oracle's timing, and the gate that reports counter-measured traffic
only for the sources it was measured on."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_host_fingerprint_tells_outputs_apart():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 256, 4099, dtype=np.uint8).tobytes()
    assert bench.host_fingerprint(a) == bench.host_fingerprint(bytes(a))
    # the same bytes as a numpy view (the in-place read of host outputs)
    assert bench.host_fingerprint(np.frombuffer(a, dtype=np.uint8)) == bench.host_fingerprint(a)
    for at in (0, 8, 4095, 4098):  # a flip in a word, in an odd word, in the tail
        b = bytearray(a)
        b[at] ^= 1
        assert bench.host_fingerprint(bytes(b)) != bench.host_fingerprint(a), at
    assert bench.host_fingerprint(a[:-1]) != bench.host_fingerprint(a)


def test_host_info_names_the_cores():
    h = bench.host_info()
    assert h["nproc"] == os.cpu_count() and isinstance(h["cpu_model"], str)


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(tmp_path):
    """measured_traffic gives the committed per-launch bytes while the
    encoder's sources hash to the recorded sha256, and None for another
    hash, another kernel or a missing file."""
    import hashlib
    csrc = os.path.join(os.path.dirname(bench.__file__), "paper_2004_03054_amd", "csrc")
    h = hashlib.sha256()
    for f in bench.TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    good = tmp_path / "good.md"
    good.write_text(f"notes\n\ntraffic k_encode bytes_per_launch=12345 sources_sha256={h.hexdigest()}\n")
    assert bench.measured_traffic("k_encode", str(good)) == 12345.0
    assert bench.measured_traffic("k_gaps", str(good)) is None
    stale = tmp_path / "stale.md"
    stale.write_text("traffic k_encode bytes_per_launch=12345 sources_sha256=" + "0" * 64 + "\n")
    assert bench.measured_traffic("k_encode", str(stale)) is None
    assert bench.measured_traffic("k_encode", str(tmp_path / "missing.md")) is None
