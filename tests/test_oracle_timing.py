"""Pins of the oracle's event timing where the particle does not start at t = 0,
and of the photon's pair event (Sec. 3 and Algorithms 1 and 2 of
arXiv:2409.17299).

Algorithm 2 advances every particle created during the step from its birth
time to the end of the step, and the pair process runs "the same scheme" as
emission with the photon removed at its event (Sec. 3).  The oracle's step
loop starts each particle at its stored start time (state column 8), so
particles of the input ensemble placed at t0 > 0 exercise exactly the code
that children run from their birth time.

Pins, each independent of the oracle's step loop:
* closed forms of the optical-depth scheme (Sec. 3): with the rate frozen, the
  first event happens at t0 + tau0 / W; without an event the optical depth
  left at the end is tau0 - W (dt - t0); a photon dies iff tau0 <= W (dt - t0);
* a brute-force generator in the style the paper contrasts with inverse
  sampling: small time steps from t0 with an event probability per step and
  rejection sampling of the energy fraction from the spectrum; event counts,
  event-time and energy-fraction distributions must agree with the oracle's;
* the random stream: children's optical depths and ids from the counter of
  the event (Philox4x32-10, checked against rocRAND elsewhere).

``test_pins_catch_planted_mistakes`` builds copies of the oracle with one
plausible mistake planted in the step loop (start time ignored, remaining
interval taken as the whole step, photon optical depth not carried, wrong
event time) and shows that one of these pins fails for every copy.
"""
import math
import os
import subprocess
import sys
from pathlib import Path

import numpy as np
import pytest
import scipy.stats as st

import synth

ROOT = Path(__file__).resolve().parent.parent


def _photons(orc, n):
    """Photons in a static B perpendicular to k (E = 0), chi* in [0.5, 20]."""
    wl = synth.static_b_sweep(2 * n, indices=[np.arange(0), None, np.arange(n)], chi_range=(0.5, 20.0),
                              energy_range=(1e2, 1e3))
    ph = wl.species[2]
    eps = np.linalg.norm(ph.p, axis=1)
    chi = eps * np.linalg.norm(ph.fields[:, 3:], axis=1)  # |k x B| with k perpendicular to B
    W = orc.ALPHA / eps * orc.rate_pair_reduced_many(chi)
    return ph, eps, chi, W


def _rejection(rng, spec, chi, lo=1e-9):
    """One draw per chi of a variable on (0, 1) with density proportional to spec(chi, v)."""
    out = np.empty(chi.size)
    grid = (np.arange(400) + 0.5) / 400
    for i, c in enumerate(chi):
        env = 1.3 * spec(np.full(grid.size, c), grid).max()
        while True:
            v = np.clip(rng.random(256), lo, 1 - lo)
            acc = rng.random(256) * env < spec(np.full(v.size, c), v)
            if acc.any():
                out[i] = v[np.argmax(acc)]
                break
    return out


# ----------------------------------------------------------------------------- photons
def test_photon_pair_timing_from_t0(orc):
    n = 3000
    ph, eps, chi, W = _photons(orc, n)
    dt = 2.0 / np.median(W)
    n_sub = 2000
    h = dt / n_sub
    rng = np.random.default_rng(5)
    t0 = rng.integers(0, int(0.7 * n_sub), n) * h  # start times on the brute force's grid
    seed, step = 7, 3
    main = [orc.Store(1), orc.Store(1), orc.Store.from_arrays(ph.p, ph.w, ph.tau, ph.id)]
    main[2].state[:n, 8] = t0
    app = [orc.Store(n), orc.Store(n), orc.Store(1)]
    rc, stats = orc.step(main, [np.zeros((1, 6)), np.zeros((1, 6)), ph.fields], app, dt, seed, step,
                         emission=0, pair=1, push=0)
    assert rc == 0
    tau0, rem = ph.tau, dt - t0
    dead = main[2].alive[:n] == 0
    # the decision in closed form: an event iff tau0 <= W (dt - t0)
    np.testing.assert_array_equal(dead, tau0 <= W * rem)
    k = np.nonzero(dead)[0]
    assert app[0].count == app[1].count == k.size == stats.n_pair and 0 < k.size < n
    # one e- and one e+ per dead photon, in photon order, born at t0 + tau0 / W
    np.testing.assert_allclose(app[0].t_birth, t0[k] + tau0[k] / W[k], rtol=1e-12)
    np.testing.assert_array_equal(app[0].t_birth, app[1].t_birth)
    # survivors keep tau0 - W (dt - t0) and their momentum
    s = ~dead
    np.testing.assert_allclose(main[2].tau[s], tau0[s] - W[s] * rem[s], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(main[2].p[s], ph.p[s])
    # the pair shares the photon momentum collinearly (e- + e+ = k)
    np.testing.assert_allclose(app[0].p + app[1].p, ph.p[k], rtol=1e-14, atol=0)
    xi = np.linalg.norm(app[0].p, axis=1) / eps[k]
    cos = np.einsum("ij,ij->i", app[0].p, ph.p[k]) / (np.linalg.norm(app[0].p, axis=1) * eps[k])
    assert np.all(cos > 1 - 1e-14)
    # children's optical depths and ids from the photon's counter j = 0 (and j | 2^31)
    u = orc.philox_stream(seed, ph.id[k], step, 0)
    v = orc.philox_stream(seed, ph.id[k], step, 0x80000000)
    # (the C library's and numpy's logarithms may differ in the last place)
    np.testing.assert_allclose(app[0].tau, -np.log((u[:, 2] + 0.5) * 2.0 ** -32), rtol=5e-16, atol=0)
    np.testing.assert_allclose(app[1].tau, -np.log((u[:, 3] + 0.5) * 2.0 ** -32), rtol=5e-16, atol=0)
    np.testing.assert_array_equal(app[0].id[:k.size], v[:, 0].astype(np.uint64) | (v[:, 1].astype(np.uint64) << 32))
    np.testing.assert_array_equal(app[1].id[:k.size], v[:, 2].astype(np.uint64) | (v[:, 3].astype(np.uint64) << 32))

    # the number of pairs: sum of Bernoulli(1 - exp(-W (dt - t0)))
    p_ev = -np.expm1(-W * rem)
    sd = math.sqrt(np.sum(p_ev * (1 - p_ev)))
    assert abs(k.size - p_ev.sum()) < 4 * sd, (k.size, p_ev.sum(), sd)
    # brute force: steps of h from t0, event probability 1 - exp(-W h) per step
    alive = np.ones(n, dtype=bool)
    t_ev = np.full(n, np.nan)
    for i in range(n_sub):
        act = alive & (t0 <= i * h + 1e-9 * h)
        hit = act & (rng.random(n) < -np.expm1(-W * h))
        t_ev[hit] = i * h + h * rng.random(int(hit.sum()))
        alive &= ~hit
    kb = np.nonzero(~alive)[0]
    assert abs(kb.size - k.size) < 4 * math.sqrt(2) * sd, (kb.size, k.size)
    # event times after t0, in units of the rate: Exp(1) truncated at W (dt - t0) on both sides
    a = (app[0].t_birth - t0[k]) * W[k]
    b = (t_ev[kb] - t0[kb]) * W[kb]
    assert st.ks_2samp(a, b).pvalue > 1e-3
    # the electron's share xi against rejection sampling from the pair spectrum at the same chi
    xb = _rejection(rng, orc.spec_pair_many, chi[kb])
    assert st.ks_2samp(xi, xb).pvalue > 1e-3
    assert abs(xi.mean() - 0.5) < 4 * xi.std() / math.sqrt(xi.size)  # symmetric spectrum


# ----------------------------------------------------------------------------- leptons
def _naive_emission_from(orc, p0, bmag, t0, dt, rng, n_sub):
    """Small-step Monte Carlo from t0 (push off, static B perpendicular to p)."""
    n = p0.shape[0]
    P = np.linalg.norm(p0, axis=1)
    nev = np.zeros(n, dtype=np.int64)
    h = dt / n_sub
    grid = (np.arange(400) + 0.5) / 400

    def rate(P, b):
        return orc.ALPHA / np.sqrt(1 + P * P) * orc.rate_rad_reduced_many(P * b)

    W = rate(P, bmag)
    for i in range(n_sub):
        act = t0 <= i * h + 1e-9 * h
        hit = np.nonzero(act & (rng.random(n) < -np.expm1(-W * h)))[0]
        for j in hit:
            chi = P[j] * bmag[j]
            g = 3 * grid ** 2 * orc.spec_rad_many(np.full(grid.size, chi), grid ** 3)
            env = 1.5 * g.max()
            while True:
                u = rng.random(64)
                acc = rng.random(64) * env < 3 * u ** 2 * orc.spec_rad_many(np.full(64, chi), u ** 3)
                if acc.any():
                    d = u[np.argmax(acc)] ** 3
                    break
            P[j] *= 1 - d
            nev[j] += 1
        if hit.size:
            W[hit] = rate(P[hit], bmag[hit])
    return nev, P


def test_lepton_subcycles_from_t0(orc):
    wl = synth.emission_static_b(100_000, indices=np.arange(0, 100_000, 125), chi_range=(0.3, 3.0))
    e = wl.species[0]
    n = e.n
    n_sub = 1500
    dt = wl.dt
    h = dt / n_sub
    rng = np.random.default_rng(17)
    t0 = rng.integers(0, int(0.8 * n_sub), n) * h
    main = [orc.Store.from_arrays(e.p, e.w, e.tau, e.id), orc.Store(1), orc.Store(1)]
    main[0].state[:n, 8] = t0
    app = [orc.Store(1), orc.Store(1), orc.Store(n * 60)]
    rc, stats = orc.step(main, [e.fields, np.zeros((1, 6)), np.zeros((1, 6))], app, dt, 0, 0, emission=1, pair=0,
                         push=0)
    assert rc == 0
    nev = main[0].nev[:n].astype(np.int64)
    bmag = np.linalg.norm(e.fields[:, 3:], axis=1)
    P0 = np.linalg.norm(e.p, axis=1)
    W0 = orc.ALPHA / np.sqrt(1 + P0 * P0) * orc.rate_rad_reduced_many(P0 * bmag)
    rem = dt - t0
    # first event at t0 + tau0 / W0; without an event tau0 - W0 (dt - t0) is left
    first = np.r_[0, np.cumsum(nev)[:-1]][nev > 0]
    np.testing.assert_allclose(app[2].t_birth[first], (t0 + e.tau / W0)[nev > 0], rtol=1e-12)
    z = nev == 0
    assert np.all(e.tau[z] > W0[z] * rem[z]) and np.all(e.tau[nev > 0] <= W0[nev > 0] * rem[nev > 0])
    np.testing.assert_allclose(main[0].tau[z], e.tau[z] - W0[z] * rem[z], rtol=1e-12, atol=1e-12)
    # every child is born inside [t0, dt] of its parent, in time order
    par = np.repeat(np.arange(n), nev)
    tb = app[2].t_birth
    assert np.all(tb >= t0[par]) and np.all(tb <= dt)
    assert np.all(np.diff(tb)[np.diff(par) == 0] >= 0)
    # against the brute force from the same start times
    nev_b, P_b = _naive_emission_from(orc, e.p, bmag, t0, dt, rng, n_sub)
    se = math.sqrt(nev.var() / n + nev_b.var() / n)
    assert abs(nev.mean() - nev_b.mean()) < 4 * se, (nev.mean(), nev_b.mean(), se)
    bins = np.array([0, 1, 2, 3, 4, 6, 9, 1000])
    a, _ = np.histogram(nev, bins)
    b, _ = np.histogram(nev_b, bins)
    assert st.chi2_contingency(np.stack([a, b]))[1] > 1e-3
    P_o = np.linalg.norm(main[0].p, axis=1)
    assert st.ks_2samp(P_o / P0, P_b / P0).pvalue > 1e-3


# ----------------------------------------------------------------------------- planted mistakes
# (test, occurrence of the statement in the source, replacement): occurrence 0
# is in the lepton loop, 1 in the photon loop
_MUTANTS = [
    ("lepton start time ignored", "double t = s[8];", 0, "double t = 0.0;", "test_lepton_subcycles_from_t0"),
    ("lepton interval taken as the whole step", "const double rem = dt - t;", 0, "const double rem = dt;",
     "test_lepton_subcycles_from_t0"),
    ("photon start time ignored", "double t = s[8];", 1, "double t = 0.0;", "test_photon_pair_timing_from_t0"),
    ("photon interval taken as the whole step", "const double rem = dt - t;", 1, "const double rem = dt;",
     "test_photon_pair_timing_from_t0"),
    ("photon optical depth not carried", "tau -= W * rem;", 1, "tau -= 0.0 * rem;",
     "test_photon_pair_timing_from_t0"),
    ("photon event time off", "double h = tau / W;", 1, "double h = (tau + 0.5) / W;",
     "test_photon_pair_timing_from_t0"),
]


def _plant(src: str, stmt: str, occurrence: int, repl: str) -> str:
    pos = -1
    for _ in range(occurrence + 1):
        pos = src.index(stmt, pos + 1)
    return src[:pos] + repl + src[pos + len(stmt):]


def test_pins_catch_planted_mistakes(tmp_path):
    src = (ROOT / "oracle" / "sfqed_oracle.cpp").read_text()
    # each statement sits once in the lepton loop and once in the photon loop
    for _, stmt, _, _, _ in _MUTANTS:
        assert src.count(stmt) == 2, stmt
    failed = []
    for i, (name, stmt, occ, repl, test) in enumerate(_MUTANTS):
        cpp = tmp_path / f"mutant{i}.cpp"
        so = tmp_path / f"mutant{i}.so"
        cpp.write_text(_plant(src, stmt, occ, repl))
        subprocess.run(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", str(cpp),
                        "-o", str(so)], check=True)
        env = dict(os.environ, SFQED_ORACLE_LIB=str(so), OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "8"))
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            f"{Path(__file__).resolve()}::{test}"], cwd=ROOT, env=env, capture_output=True, text=True)
        print(f"{name}: {test} -> {'fails (caught)' if r.returncode == 1 else 'rc ' + str(r.returncode)}")
        if r.returncode != 1:  # 1 = a test failed; anything else is a missed mistake or a broken run
            failed.append((name, r.returncode, r.stdout[-800:]))
    assert not failed, failed
