"""Host model of the lepton write kernel's child-record staging (CPU).

The kernel stages each lane's child records in a line buffer and writes a line
out when a record reaches its end or the parent finishes (csrc/line_rule.h).
``line_rule_model.cpp`` runs that rule on the host over random parents, child
counts, buffer alignments and capacities, for 48- and 64-byte records and
half or whole lines, and requires the buffer to equal direct stores byte for
byte with nothing written past the capacity.  The same model must find the
earlier rule (write a line only when all its pieces are set) wrong: under it
a parent whose range starts mid-line stages its next record into the wrong
line, which is how misplaced records once reached the GPU.
"""
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent


def test_line_rule_model(tmp_path):
    exe = tmp_path / "line_rule_model"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", str(HERE / "line_rule_model.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe), "20000"], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for line in r.stdout.splitlines():
        assert ": current rule 0/" in line, line
