"""Host model of the lepton count pass's event log and its replay (CPU).

``event_log_model.cpp`` writes the log of one wave over random particles
with the count kernel's lane discipline (a queue of shuffled chunks, one
chunk per trip) and the format of csrc/event_log.h, reads it back as the
replay kernel does, and requires every particle with events to get its launch
index, its events in order and its final optical depth back, across block
jumps, trips on which every lane takes a new particle, and fresh lanes whose
particle has no event.  It must also find two variants wrong: a reader that
ranks a new lane among the fresh lanes with an event only, and a writer whose
queue serves a trip from two chunks.
"""
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent


def test_event_log_model(tmp_path):
    exe = tmp_path / "event_log_model"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", str(HERE / "event_log_model.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe), "400"], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("reader: 0/")
