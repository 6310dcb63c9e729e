"""Precision sweep over chi in [1e-3, 1e3] (1e8 electrons and 1e8 photons in a
static B field; every 1000th particle of each species here, regenerated
exactly by index): the FP64 GPU path, the FP32 table path and the BF16
surrogate against the FP64 oracle, on one shared stream of 32-bit uniforms.

* chi: FP64 within 1e-13 of the oracle's chi at the same rounded inputs;
  FP32 leptons within 2e-6, FP32 photons (chi evaluated in FP64 and rounded
  once) within half an ulp, 2^-24;
* rates (where the rate exceeds 1e-30; pair rates below chi ~ 0.04 are
  smaller), FP64 <= 1e-12 and FP32 <= 1e-5 relative, both at the path's own
  chi and end to end: the path's rate against the oracle's rate at the
  oracle's chi of the same inputs (for pairs the FP32 chi rounding enters
  amplified by up to 8/(3 chi) ~ 70);
* first-event energy fraction at the particle's chi: FP64 table within 1e-7,
  FP32 table within 5e-5 (at the chi of the FP32-rounded inputs);
* surrogate (emission, trained range [1e-2, 1e2]): per-draw |d ln delta|
  median < 1e-3, 99% < 5e-3; the table outside.  (The paired-L1 statistic is
  not used at this size: with ~6e4 draws the few hundred that change bin give
  it a counting floor near 4e-3, falling as 1/sqrt(N); the 4e6-draw test and
  the 1e8-event bench hold the surrogate to L1 <= 1e-3.)
"""
import numpy as np
import pytest

import oracle
import synth

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
N_TOTAL = 200_000_000


@pytest.fixture(scope="module")
def sweep():
    torch, sf = need_gpu()
    idx = np.arange(0, N_TOTAL // 2, 1000)
    wl = synth.static_b_sweep(N_TOTAL, indices=[idx, idx, idx])
    return torch, sf, sf.Tables(), wl


def oracle_chi(sp, photon, np_dtype=np.float64):
    """chi and energy of every particle from its inputs rounded to np_dtype."""
    p = sp.p.astype(np_dtype).astype(np.float64)
    f = sp.fields.astype(np_dtype).astype(np.float64)
    e = np.linalg.norm(p, axis=1) if photon else np.sqrt(1.0 + np.einsum("ij,ij->i", p, p))
    chi = np.array([oracle.chi(p[i], e[i], f[i, :3], f[i, 3:]) for i in range(sp.n)])
    return chi, e


def oracle_rates_at(chi, e, s):
    if s == 0:
        return oracle.ALPHA / e * oracle.rate_rad_reduced_many(chi)
    return np.where(e >= 2.0, oracle.ALPHA / e * oracle.rate_pair_reduced_many(chi), 0.0)


@pytest.mark.parametrize("s", [0, 2])
def test_rates(sweep, s):
    """chi of each path against the oracle's chi at that path's rounded inputs,
    and the rate against the oracle's rate at the path's own chi (the rate
    bounds are properties of the rate approximation; a pair rate near chi ~ 0.04
    turns a chi error of a few FP32 ulp into 2e-5 by its e^(-8/(3 chi)) factor)."""
    torch, sf, tabs, wl = sweep
    sp = wl.species[s]
    half_ulp = 2.0 ** -24
    for dt, np_dt, tol_chi, tol in ((torch.float64, np.float64, 1e-13, 1e-12),
                                    (torch.float32, np.float32, half_ulp * (1 + 1e-9) if s == 2 else 2e-6, 1e-5)):
        chi_o, e = oracle_chi(sp, s == 2, np_dt)
        st = sf.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, dtype=dt, photon=s == 2)
        chi_g, w_g = sf.eval_particles(tabs, s, st, sf.Fields.from_array(sp.fields, dt))
        chi_g = chi_g.double().cpu().numpy()
        w_g = w_g.double().cpu().numpy()
        ce = np.abs(chi_g - chi_o) / chi_o
        assert ce.max() <= tol_chi, ce.max()
        w_o = oracle_rates_at(chi_g, e, s)
        if s == 2:
            w_g = np.where(e >= 2.0, w_g, 0.0)
        floor = 1e-300 if dt == torch.float64 else 1e-30
        ok = (w_o > floor) & (w_g > floor)
        assert (w_g[w_o == 0] == 0).all()
        rel = np.abs(w_g[ok] - w_o[ok]) / w_o[ok]
        w_e2e = oracle_rates_at(chi_o, e, s)  # the oracle's rate at its own chi
        ok2 = (w_e2e > floor) & (w_g > floor)
        rel2 = np.abs(w_g[ok2] - w_e2e[ok2]) / w_e2e[ok2]
        worst = int(np.argmax(np.where(ok2, np.abs(w_g - w_e2e) / np.where(ok2, w_e2e, 1.0), 0.0)))
        print(f"species {s} {dt}: chi max rel err {ce.max():.2e}; {ok.sum()} rates, max rel err {rel.max():.2e}, "
              f"median {np.median(rel):.2e}; end to end max {rel2.max():.2e} (at chi {chi_o[worst]:.3g})")
        assert rel.max() <= tol, rel.max()
        assert rel2.max() <= tol, rel2.max()
        assert ok.sum() > 0.3 * sp.n


@pytest.mark.parametrize("s", [0, 2])
def test_first_event_samples(sweep, s):
    torch, sf, tabs, wl = sweep
    sp = wl.species[s]
    proc = 0 if s == 0 else 1
    chi_o, _ = oracle_chi(sp, s == 2)
    k = synth.bits32(0, 56 + s, sp.id)
    kt = torch.tensor(k.view(np.int32), device="cuda")
    st64 = sf.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, dtype=torch.float64, photon=s == 2)
    st32 = sf.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, dtype=torch.float32, photon=s == 2)
    c64, _ = sf.eval_particles(tabs, s, st64, sf.Fields.from_array(sp.fields, torch.float64))
    c32, _ = sf.eval_particles(tabs, s, st32, sf.Fields.from_array(sp.fields, torch.float32))
    d64 = sf.sample(tabs, proc, c64, kt).cpu().numpy()
    d32 = sf.sample(tabs, proc, c32, kt).double().cpu().numpy()
    c32h = c32.double().cpu().numpy()
    if proc == 0:
        sel = np.ones(sp.n, bool)
        ref64, _ = oracle.sample_rad(chi_o, k)
        ref32, _ = oracle.sample_rad(c32h, k)
    else:
        sel = chi_o >= 1e-2          # pair events below chi ~ 0.03 have rates under e^-90
        ref64, _ = oracle.sample_pair(chi_o[sel], k[sel])
        ref32, _ = oracle.sample_pair(c32h[sel], k[sel])
        d64, d32 = d64[sel], d32[sel]
    e64 = np.abs(d64 - ref64) / ref64
    e32 = np.abs(d32 - ref32) / ref32
    print(f"species {s}: sampler FP64 max {e64.max():.2e}, FP32 max {e32.max():.2e} median {np.median(e32):.2e}")
    assert e64.max() < 1e-7
    assert e32.max() < 5e-5
    if proc == 0:
        net = sf.Mlp(sf.load_surrogate())
        dm = net.sample(tabs, c32, kt).double().cpu().numpy()
        inside = (c32h >= np.float32(1e-2)) & (c32h <= np.float32(1e2))
        assert np.array_equal(dm[~inside], d32[~inside])
        e = np.abs(np.log(dm[inside]) - np.log(ref32[inside]))
        print(f"surrogate in range: {inside.sum()} draws, |d ln delta| median {np.median(e):.2e}, "
              f"99% {np.quantile(e, 0.99):.2e}, max {e.max():.2e}")
        assert np.median(e) < 1e-3 and np.quantile(e, 0.99) < 5e-3 and e.max() < 0.2
