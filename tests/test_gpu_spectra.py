"""Emitted spectra of the FP32 GPU generator against the FP64 oracle with
independent random streams (GPU seed 1, oracle seed 2): unpaired two-sample
Kolmogorov-Smirnov tests must not reject at the 1% level.  With a shared
stream the two sides draw the same numbers and KS is trivially passed, hence
different seeds.

* photon emission: energies of the photons emitted by the 1e5-electron
  static-B workload (every 5th electron);
* pair production: the electron's energy fraction xi of the pairs made by the
  photons of the crossed-field workload (every 200th photon, emission off).
"""
import numpy as np
import pytest
from scipy import stats

import synth
from gpu_util import cast_inputs, need_gpu, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, sf = need_gpu()
    return torch, sf, sf.Tables()


def test_emission_spectrum_ks(env):
    torch, sf, tabs = env
    wl = synth.emission_static_b(100_000, indices=np.arange(0, 100_000, 5))
    inp = cast_inputs(wl, np.float32)
    n = inp[0]["id"].size
    cap = [1, 1, n * 40]
    cfg = sf.step_cfg(pair=False, push=False)
    rc, st, _, _, ga = run_gpu(sf, torch, tabs, wl, inp, torch.float32, cap, cfg, seed=1)
    assert rc == 0
    orc_rc, ost, _, oa = run_oracle(wl, inp, cap, seed=2, emission=1, pair=0, push=0)
    assert orc_rc == 0
    kg = np.linalg.norm(ga[2].host()["p"], axis=1)
    ko = np.linalg.norm(oa[2].p[:oa[2].count], axis=1)
    assert kg.size > 50_000 and ko.size > 50_000
    # event counts are Poisson: the totals agree within a few standard deviations
    assert abs(kg.size - ko.size) < 5 * np.sqrt(ko.size)
    res = stats.ks_2samp(np.log(kg), np.log(ko))
    print(f"emission: {kg.size} vs {ko.size} photons, KS D={res.statistic:.2e} p={res.pvalue:.3f}")
    assert res.pvalue > 0.01


def test_pair_spectrum_ks(env):
    torch, sf, tabs = env
    n_all = 10_000_000
    idx = [np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.arange(0, 2_000_000, 200)]
    wl = synth.crossed_field(n_all, indices=idx)
    inp = cast_inputs(wl, np.float32)
    n = inp[2]["id"].size
    cap = [n, n, n]
    cfg = sf.step_cfg(emission=False, push=False)
    rc, st, _, _, ga = run_gpu(sf, torch, tabs, wl, inp, torch.float32, cap, cfg, seed=1)
    assert rc == 0
    orc_rc, ost, _, oa = run_oracle(wl, inp, cap, seed=2, emission=0, pair=1, push=0)
    assert orc_rc == 0

    def xi(ge, gp):
        a, b = np.linalg.norm(ge, axis=1), np.linalg.norm(gp, axis=1)
        return a / (a + b)

    xg = xi(ga[0].host()["p"], ga[1].host()["p"])
    xo = xi(oa[0].p[:oa[0].count], oa[1].p[:oa[1].count])
    assert xg.size > 1000 and xo.size > 1000
    assert abs(xg.size - xo.size) < 5 * np.sqrt(xo.size)
    res = stats.ks_2samp(xg, xo)
    print(f"pairs: {xg.size} vs {xo.size}, KS D={res.statistic:.2e} p={res.pvalue:.3f}")
    assert res.pvalue > 0.01
