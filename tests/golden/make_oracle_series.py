"""Writes tests/golden/oracle_rotating_series.json: a series of 100 cascades
of the FP64 oracle (Sec. 5.2's validation: the same problem run 100 times with
different random numbers), the rotating-field workload at reduced scale.

Each run: 200 seed electrons (synth.rotating_e, indices 0..199), 20 steps of
synth's dt, push on, merge after every step, Philox seed = run index (0..99).
Stored per run: the counts of e-, e+ and photons after every step, and the
growth rate Gamma (least-squares slope of ln N over steps 5..20).  Calls only
oracle/ and synth; run from the repository root:

    python tests/golden/make_oracle_series.py
"""
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import synth  # noqa: E402
from oracle import cascade as oc  # noqa: E402

SEEDS, STEPS, RUNS = 200, 20, 100


def main():
    wl = synth.rotating_e(1_000_000, indices=np.arange(SEEDS))
    counts, gammas = [], []
    t0 = time.time()
    for run in range(RUNS):
        c = oc.run(wl, STEPS, seed=run)
        counts.append(c.tolist())
        gammas.append(oc.growth_rate(c, wl.dt, first=5))
        print(f"run {run}: N = {int(c[-1].sum())}, Gamma = {gammas[-1]:.6e} ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "rotating_e", "seed_electrons": SEEDS, "steps": STEPS, "runs": RUNS,
           "philox_seeds": list(range(RUNS)), "dt": wl.dt, "growth_rate_first_step": 5,
           "script": "tests/golden/make_oracle_series.py", "counts": counts, "gamma": gammas}
    (Path(__file__).resolve().parent / "oracle_rotating_series.json").write_text(json.dumps(out))


if __name__ == "__main__":
    main()
