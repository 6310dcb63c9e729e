"""Statistical validation in the manner of Sec. 5.2: a series of 100 cascades
with different seeds (the rotating-field cascade, 2000 seed electrons, 20
steps, merge after every step) gives the sample mean and standard deviation
of the growth rate Gamma and of the particle counts per step.

The FP64 path reproduces the oracle particle for particle on the same stream
(test_gpu_cascade.py), so its series stands for the oracle's.  The FP32 path
differs from it only by rare decision flips; over 100 seeds its mean growth
rate must agree with the FP64 series' to eta_Gamma < 0.5% (the paper's
criterion) and within three standard errors, and at every step the FP32
counts must lie inside the FP64 series' mean +- 3 sigma (the paper's band),
up to the expected one in a few hundred outliers."""
import numpy as np
import pytest

import synth
from oracle import cascade as ocascade

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
SEEDS, STEPS, RUNS = 2000, 20, 100


def series(torch, sf, tabs, wl, dtype):
    from paper_2409_17299_amd import cascade
    e0, wdt = wl.flags["e0"], wl.flags["omega_dt"]
    sp = [(s.p, s.w, s.tau, s.id) for s in wl.species]
    cap = [SEEDS * 200, SEEDS * 200, SEEDS * 800]
    gam, tot = [], []
    for seed in range(RUNS):
        counts, _, _, _, _ = cascade.run(tabs, sp, wl.dt, STEPS, lambda k: synth.rotating_field(e0, wdt, k), cap,
                                         [SEEDS * 60, SEEDS * 60, SEEDS * 250], dtype=dtype, seed=1000 + seed)
        gam.append(ocascade.growth_rate(counts, wl.dt, first=5))
        tot.append(counts.sum(axis=1))
    return np.array(gam), np.array(tot, dtype=np.float64)


def test_hundred_seed_series():
    torch, sf = need_gpu()
    tabs = sf.Tables()
    wl = synth.rotating_e(1_000_000, indices=np.arange(SEEDS))
    g64, n64 = series(torch, sf, tabs, wl, torch.float64)
    g32, n32 = series(torch, sf, tabs, wl, torch.float32)
    m64, s64 = g64.mean(), g64.std(ddof=1)
    m32, s32 = g32.mean(), g32.std(ddof=1)
    se = np.sqrt(s64 ** 2 / RUNS + s32 ** 2 / RUNS)
    eta = abs(m32 - m64) / m64
    mu, sd = n64.mean(axis=0), n64.std(axis=0, ddof=1)
    outside = np.abs(n32[:, 1:] - mu[1:]) > 3 * sd[1:]
    print(f"Gamma over {RUNS} seeds: FP64 {m64:.5e} +- {s64 / m64:.2%} (per run), FP32 {m32:.5e} +- {s32 / m32:.2%}; "
          f"eta_Gamma {eta:.2e} ({abs(m32 - m64) / se:.1f} standard errors); FP32 counts outside the FP64 "
          f"mean +- 3 sigma: {outside.sum()} of {outside.size}; relative sigma of N at step {STEPS}: "
          f"{sd[-1] / mu[-1]:.2%}")
    assert s64 / m64 < 0.02                 # the seed-to-seed spread the series resolves
    assert eta < 5e-3                       # Sec. 5.2's criterion
    assert abs(m32 - m64) < 3 * se
    assert outside.mean() < 0.02
