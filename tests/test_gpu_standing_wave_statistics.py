"""Statistical validation on the paper's own test problem (Sec. 5.1 and 5.2):
series of 100 cascades from rest in the standing wave on its grid, 2000 seeds
(half e-, half e+) per run, 1.5 T (300 steps), photons below the pair
threshold dropped after every merge, one series per precision, each run with
its own seed for the positions and for the random stream.

The paper compares two implementations by the growth rate Gamma of the
number of electrons (eta_Gamma < 0.5%) and by the particle densities along x
at the end, which scatter by 5-10% from run to run (mean +- 3 sigma bands).
Here FP64 stands for the oracle (it reproduces the oracle's cascade on the
same stream, test_gpu_grid.py) and FP32 is compared with it:
* mean Gamma of the two series within 0.5% and three standard errors;
* the FP32 mean density in every bin within three standard errors of the
  FP64 mean (with a Bonferroni margin for the number of bins);
* individual FP32 densities outside the FP64 mean +- 3 sigma in no more than
  2% of (run, bin) pairs;
* the densities symmetric under x -> -x (the wave's E is even and B odd about
  the antinode), within the same statistics."""
import numpy as np
import pytest

import synth
from oracle import cascade as ocascade

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
SEEDS, STEPS, RUNS, BINS, FIRST = 2000, 300, 100, 32, 150


def series(torch, sf, tabs, dtype):
    from paper_2409_17299_amd import cascade
    gam, dens_e, dens_g = [], [], []
    for r in range(RUNS):
        wl = synth.standing_wave(SEEDS, seed=100 + r)
        prm = wl.flags
        grid = cascade.standing_wave_grid(prm, wl.dt, dtype)
        sp = [(s.p, s.w, s.tau, s.id, s.x) for s in wl.species]
        counts, _, _, main, _ = cascade.run(tabs, sp, wl.dt, STEPS, None, [SEEDS * 400, SEEDS * 400, SEEDS * 3000],
                                            [SEEDS * 40, SEEDS * 40, SEEDS * 400], dtype=dtype, seed=100 + r,
                                            grid=grid, resample=dict(photon_energy_min=2.0))
        gam.append(ocascade.growth_rate(counts[:, :1], wl.dt, first=FIRST) * prm["period"])
        L, x0 = prm["length"], prm["x0"]
        edges = np.linspace(x0, x0 + L, BINS + 1)
        def wrapped(m):   # the last step's positions, folded back into the box
            return x0 + np.mod(m.x[:m.count].double().cpu().numpy() - x0, L)
        dens_e.append(np.histogram(wrapped(main[0]), edges)[0])
        dens_g.append(np.histogram(wrapped(main[2]), edges)[0])
    return np.array(gam), np.array(dens_e, np.float64), np.array(dens_g, np.float64)


def compare(name, d64, d32):
    mu, sd = d64.mean(0), d64.std(0, ddof=1)
    se = np.sqrt(d64.var(0, ddof=1) / RUNS + d32.var(0, ddof=1) / RUNS)
    z = np.abs(d32.mean(0) - mu) / np.maximum(se, 1e-12)
    outside = np.abs(d32 - mu) > 3 * sd
    sym = np.abs(mu - mu[::-1]) / np.maximum(np.sqrt(2) * sd / np.sqrt(RUNS), 1e-12)
    print(f"{name}: run-to-run spread {np.median(sd / mu):.1%} of the mean; max |z| of the FP32 mean {z.max():.2f}; "
          f"FP32 values outside the FP64 mean +- 3 sigma {outside.mean():.2%}; max asymmetry {sym.max():.2f} sigma")
    assert z.max() < 4.0                    # 3 sigma with a margin for 32 bins
    assert outside.mean() < 0.02
    assert sym.max() < 4.5


def test_standing_wave_series():
    torch, sf = need_gpu()
    tabs = sf.Tables()
    g64, e64, p64 = series(torch, sf, tabs, torch.float64)
    g32, e32, p32 = series(torch, sf, tabs, torch.float32)
    m64, m32 = g64.mean(), g32.mean()
    se = np.sqrt(g64.var(ddof=1) / RUNS + g32.var(ddof=1) / RUNS)
    eta = abs(m32 - m64) / m64
    print(f"Gamma T over {RUNS} runs: FP64 {m64:.4f} +- {g64.std(ddof=1) / m64:.2%} (per run), FP32 {m32:.4f}; "
          f"eta_Gamma {eta:.2e} ({abs(m32 - m64) / se:.1f} standard errors); electrons at {STEPS} steps "
          f"{e64.sum(1).mean():.0f}, photons {p64.sum(1).mean():.0f}")
    assert eta < 5e-3 and abs(m32 - m64) < 3 * se
    compare("electron density", e64, e32)
    compare("photon density", p64, p32)
