"""Philox4x32-10 of the oracle against rocRAND's independent implementation
(the counter-based generator of Salmon et al., SC'11, which both sides use for
the draws of the event generator), plus structural checks."""
import shutil
import subprocess

import numpy as np
import pytest


def _rocrand_blocks(tmp_path, rows):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not shutil.which(hipcc) and not __import__("os").path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = __import__("pathlib").Path(__file__).with_name("philox_rocrand_check.cpp")
    exe = tmp_path / "philox_check"
    subprocess.run([hipcc, "-O1", str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    inp = "\n".join(f"{s} {i} {st} {j}" for s, i, st, j in rows) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand(orc, tmp_path):
    rng = np.random.default_rng(7)
    rows = [(0, 0, 0, 0), (0, 1, 0, 0), (1, 0, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
            (2**64 - 1, 2**62 - 1, 2**32 - 1, 2**32 - 1), (0, 2**40 + 5, 3, 0xFFFFFFFF),
            (12345, 99, 7, 0x80000003)]
    for _ in range(200):
        rows.append((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**62)),
                     int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))))
    # the harness maps the counter through rocRAND's offset = 4 id, so ids stay below 2^62
    ref = _rocrand_blocks(tmp_path, rows)
    for (s, i, st, j), r in zip(rows, ref):
        got = orc.philox_stream(s, [i], st, j)[0].astype(np.uint64)
        assert np.array_equal(got, r), (s, i, st, j)


def test_philox_key_and_counter_all_matter(orc):
    base = orc.philox_stream(5, [10], 3, 4)[0]
    for args in [(6, 10, 3, 4), (5, 11, 3, 4), (5, 10, 4, 4), (5, 10, 3, 5), (5 + 2**32, 10, 3, 4),
                 (5, 10 + 2**32, 3, 4)]:
        assert not np.array_equal(orc.philox_stream(args[0], [args[1]], args[2], args[3])[0], base)


def test_philox_uniformity(orc):
    # 2^16 blocks -> 2^18 words; chi-square over 256 bins of the top byte
    ids = np.arange(1 << 16, dtype=np.uint64)
    words = orc.philox_stream(1, ids, 0, 0).ravel()
    counts = np.bincount((words >> 24).astype(np.int64), minlength=256)
    e = words.size / 256
    chi2 = ((counts - e) ** 2 / e).sum()
    assert 180 < chi2 < 340  # 255 dof, ~ +-3.5 sigma
    # avalanche: flipping one counter bit changes about half the output bits
    a = orc.philox_stream(1, ids[:4096], 0, 0)
    b = orc.philox_stream(1, ids[:4096] ^ np.uint64(1 << 17), 0, 0)
    flips = np.unpackbits((a ^ b).view(np.uint8)).mean()
    assert abs(flips - 0.5) < 0.01
