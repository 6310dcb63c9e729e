"""Host logic of bench.py (no GPU): the algorithmic byte model of the step's
kernel groups, the measured-traffic lookup that is void once the kernel
sources change, and the refusal of more than one GPU."""
import json
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def _stats():
    return {"kernel_particles": [1000, 1000, 0, 5000, 0], "event_particles": [300, 40],
            "n_emit": 4000, "n_pair": 40}


def test_byte_model():
    st, n_main = _stats(), [200, 200, 100]
    # leptons: 1000 particles in the launches, 400 of them main, 300 with events
    assert bench.kernel_bytes("count_lepton", st, n_main, 1) == 1000 * 56 + 600 * 8 + 700 * 8
    assert bench.kernel_bytes("count_lepton", st, n_main, 1, push=True) == 1000 * 56 + 600 * 8 + 700 * 20
    assert bench.kernel_bytes("scan", st, n_main, 1) == 1000 * 4 + 300 * 12
    assert bench.kernel_bytes("scan", st, n_main, 1, merged=False) == 1000 * 4 + 340 * 12
    assert bench.kernel_bytes("write_lepton", st, n_main, 1) == 300 * 88 + 4000 * 48
    # photons: 5000 in the launches, 100 main, 40 with an event
    assert bench.kernel_bytes("count_photon", st, n_main, 1) == 5000 * 52 + 4900 * 8 + 4960 * 33 + 40 * 12
    assert bench.kernel_bytes("count_photon", st, n_main, 1, merged=False) == 5000 * 56 + 4900 * 8 + 4960 * 8
    assert bench.kernel_bytes("write_photon", st, n_main, 1) == 40 * 69 + 2 * 40 * 48
    with pytest.raises(KeyError):
        bench.kernel_bytes("nope", st, n_main, 1)


def test_measured_traffic_is_void_once_sources_change(tmp_path, monkeypatch):
    import hashlib
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    (tmp_path / "profiles").mkdir()
    rec = {"kernels": {"count_photon": {"traffic_bytes_per_launch": 123.0}}, "sources": ["k.hip"],
           "sources_sha256": hashlib.sha256(src.read_bytes()).hexdigest()}
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    assert bench.measured_traffic("count_photon") == 123.0
    assert bench.measured_traffic("write_lepton") is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("count_photon") is None


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err
