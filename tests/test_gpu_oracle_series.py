"""Sec. 5.2's validation with the oracle on one side: the paper runs its
problem 100 times with each implementation and compares the growth rate
(eta_Gamma < 0.5%) and the spread of the results over the runs.

tests/golden/oracle_rotating_series.json holds the FP64 oracle's 100 runs of
the rotating-field cascade at reduced scale (200 seed electrons, 20 steps,
push on, merge after every step, Philox seeds 0..99), written by
tests/golden/make_oracle_series.py, which calls only the oracle.  Here the
GPU's FP32 path runs the same problem 100 times on independent streams
(seeds 1000..1099); its mean growth rate must agree with the oracle's to
eta_Gamma < 0.5% and within three standard errors, its mean count after every
step within three standard errors of the oracle's, and its runs must fall
inside the oracle's mean +- 3 sigma band but for a few outliers."""
import json
from pathlib import Path

import numpy as np
import pytest

import synth
from oracle import cascade as ocascade

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
GOLDEN = Path(__file__).resolve().parent / "golden" / "oracle_rotating_series.json"


def test_fp32_series_against_oracle_series():
    torch, sf = need_gpu()
    from paper_2409_17299_amd import cascade
    g = json.loads(GOLDEN.read_text())
    seeds, steps, runs = g["seed_electrons"], g["steps"], g["runs"]
    assert (seeds, steps, runs) == (200, 20, 100)
    wl = synth.rotating_e(1_000_000, indices=np.arange(seeds))
    assert abs(wl.dt - g["dt"]) <= 1e-12 * g["dt"]
    e0, wdt = wl.flags["e0"], wl.flags["omega_dt"]
    sp = [(s.p, s.w, s.tau, s.id) for s in wl.species]
    tabs = sf.Tables()
    gam, tot = [], []
    for run in range(runs):
        counts, _, _, _, _ = cascade.run(tabs, sp, wl.dt, steps, lambda k: synth.rotating_field(e0, wdt, k),
                                         [seeds * 200, seeds * 200, seeds * 800], [seeds * 60, seeds * 60, seeds * 250],
                                         dtype=torch.float32, seed=1000 + run)
        gam.append(ocascade.growth_rate(counts, wl.dt, first=g["growth_rate_first_step"]))
        tot.append(counts.sum(axis=1))
    g32, n32 = np.array(gam), np.array(tot, dtype=np.float64)
    go, no = np.array(g["gamma"]), np.array(g["counts"], dtype=np.float64).sum(axis=2)
    mo, so = go.mean(), go.std(ddof=1)
    m32, s32 = g32.mean(), g32.std(ddof=1)
    se = np.sqrt(so ** 2 / runs + s32 ** 2 / runs)
    eta = abs(m32 - mo) / mo
    mu, sd = no.mean(axis=0), no.std(axis=0, ddof=1)
    se_n = np.sqrt(sd ** 2 / runs + n32.std(axis=0, ddof=1) ** 2 / runs)
    z_n = np.abs(n32.mean(axis=0)[1:] - mu[1:]) / se_n[1:]
    outside = np.abs(n32[:, 1:] - mu[1:]) > 3 * sd[1:]
    print(f"Gamma over {runs} runs of {seeds} seeds: oracle {mo:.5e} (spread {so / mo:.2%} per run), "
          f"GPU FP32 {m32:.5e} (spread {s32 / m32:.2%}); eta_Gamma {eta:.2e} = {abs(m32 - mo) / se:.1f} standard "
          f"errors; mean counts per step at most {z_n.max():.1f} standard errors apart; GPU counts outside the "
          f"oracle's mean +- 3 sigma: {outside.sum()} of {outside.size}")
    assert eta < 5e-3                      # Sec. 5.2's criterion
    assert abs(m32 - mo) < 3 * se
    assert z_n.max() < 3.5                 # 20 steps: the largest of 20 correlated |z| values
    assert outside.mean() < 0.02
