"""Pins of the oracle's ensemble step (Alg. 1 and 2 of arXiv:2409.17299).

* a brute-force generator in the style the paper contrasts with inverse
  sampling (Sec. 3): small time steps with an event probability per step and
  rejection sampling of the photon energy from the spectrum; its event counts
  and final momenta must agree in distribution with the oracle's optical-depth
  sub-cycling;
* momentum conservation per event (collinear recoil) through whole cascades;
* Boris push invariants; closed forms of chi; merge and capacity behaviour;
  the append order of Alg. 2.
"""
import math

import numpy as np
import pytest
import scipy.stats as st

import synth


def _stores(orc, wl, cap_factor=50, positions=False):
    main, fields = [], []
    for sp in wl.species:
        main.append(orc.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, capacity=max(sp.n, 1)))
        fields.append(sp.fields if sp.fields.shape[0] else np.zeros((1, 6)))
    tot = max(1, sum(wl.counts))
    app = [orc.Store(tot * cap_factor) for _ in range(3)]
    return main, fields, app


# ----------------------------------------------------------------------------- brute force
def _naive_emission(orc, p0, bmag, dt, rng, n_sub=4000):
    """Small-step Monte Carlo with rejection sampling (push off, static B perpendicular to p)."""
    n = p0.shape[0]
    P = np.linalg.norm(p0, axis=1)
    nev = np.zeros(n, dtype=np.int64)
    h = dt / n_sub
    ugrid = (np.arange(400) + 0.5) / 400

    def rate(P, b):
        g = np.sqrt(1 + P * P)
        return orc.ALPHA / g * orc.rate_rad_reduced_many(P * b)

    W = rate(P, bmag)
    for _ in range(n_sub):
        hit = np.nonzero(rng.random(n) < -np.expm1(-W * h))[0]
        for i in hit:
            chi = P[i] * bmag[i]
            g = 3 * ugrid ** 2 * orc.spec_rad_many(np.full(ugrid.size, chi), ugrid ** 3)
            env = 1.5 * g.max()
            while True:
                u = rng.random(64)
                acc = rng.random(64) * env < 3 * u ** 2 * orc.spec_rad_many(np.full(64, chi), u ** 3)
                if acc.any():
                    d = u[np.argmax(acc)] ** 3
                    break
            P[i] *= 1 - d
            nev[i] += 1
        if hit.size:
            W[hit] = rate(P[hit], bmag[hit])
    return nev, P


@pytest.mark.slow
def test_event_statistics_vs_bruteforce(orc):
    wl = synth.emission_static_b(100_000, indices=np.arange(0, 100_000, 100))
    main, fields, app = _stores(orc, wl)
    p0 = wl.species[0].p.copy()
    rc, stats = orc.step(main, fields, app, wl.dt, 0, 0, emission=1, pair=0, push=0)
    assert rc == 0
    nev_o = main[0].nev[:main[0].count].astype(np.int64)
    P_o = np.linalg.norm(main[0].p, axis=1)
    bmag = np.linalg.norm(wl.species[0].fields[:, 3:], axis=1)
    nev_n, P_n = _naive_emission(orc, p0, bmag, wl.dt, np.random.default_rng(11))
    # mean number of events: agree within 4 standard errors
    se = math.sqrt(nev_o.var() / nev_o.size + nev_n.var() / nev_n.size)
    assert abs(nev_o.mean() - nev_n.mean()) < 4 * se
    # distributions of the event count and of the final momentum
    assert st.ks_2samp(P_o / np.linalg.norm(p0, axis=1), P_n / np.linalg.norm(p0, axis=1)).pvalue > 1e-3
    bins = np.array([0, 1, 2, 3, 5, 8, 13, 1000])
    a, _ = np.histogram(nev_o, bins)
    b, _ = np.histogram(nev_n, bins)
    assert st.chi2_contingency(np.stack([a, b]))[1] > 1e-3
    # the first event happens after tau0 / W0 (the optical depth is used up)
    first = app[2].t_birth[np.r_[0, np.cumsum(nev_o)[:-1]][nev_o > 0]]
    g0 = np.sqrt(1 + np.einsum("ij,ij->i", p0, p0))
    w0 = orc.ALPHA / g0 * orc.rate_rad_reduced_many(np.linalg.norm(p0, axis=1) * bmag)
    tau0 = wl.species[0].tau
    np.testing.assert_allclose(first, (tau0 / w0)[nev_o > 0], rtol=1e-13)
    # particles with no event: tau0 > W0 dt and the remaining depth is tau0 - W0 dt
    z = nev_o == 0
    assert np.all(tau0[z] > w0[z] * wl.dt)
    np.testing.assert_allclose(main[0].tau[z], tau0[z] - w0[z] * wl.dt, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------------------- conservation
def test_momentum_conserved_through_cascade(orc):
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 40_000)] * 2 + [np.arange(0, 2_000_000, 20_000)])
    main, fields, app = _stores(orc, wl, cap_factor=400)
    p_in = [sp.p.copy() for sp in wl.species]
    rc, stats = orc.step(main, fields, app, wl.dt, 3, 0, emission=1, pair=1, push=0, gamma_min=2.0)
    assert rc == 0 and stats.n_pair > 0 and stats.n_rounds > 2
    total = {}
    for s in range(3):
        for i in range(main[s].count):
            if s == 2 and not main[s].alive[i]:
                continue
            total.setdefault((s, i), np.zeros(3))
            total[(s, i)] += main[s].p[i]
        for i in range(app[s].count):
            if s == 2 and not app[s].alive[i]:
                continue
            r = int(app[s].root[i]) & 0xFFFFFFFF
            key = (r >> 30, r & 0x3FFFFFFF)
            total.setdefault(key, np.zeros(3))
            total[key] += app[s].p[i]
    for (s, i), tot in total.items():
        ref = p_in[s][i]
        assert np.linalg.norm(tot - ref) <= 1e-12 * np.linalg.norm(ref), (s, i)


# ----------------------------------------------------------------------------- Boris, chi
def test_boris_invariants(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        p = rng.normal(size=3) * 100
        B = rng.normal(size=3)
        h = rng.uniform(0.1, 1e3)
        q = rng.choice([-1.0, 1.0])
        p1 = orc.boris(p, q, np.zeros(3), B, h)
        assert abs(np.linalg.norm(p1) / np.linalg.norm(p) - 1) < 1e-14
        # rotation about B by 2 atan(|B| h / (2 gamma)) (Boris 1970)
        g = math.sqrt(1 + p @ p)
        bn = B / np.linalg.norm(B)
        pp0, pp1 = p - (p @ bn) * bn, p1 - (p1 @ bn) * bn
        ang = math.atan2(np.linalg.norm(np.cross(pp0, pp1)), pp0 @ pp1)
        assert abs(ang - 2 * math.atan(np.linalg.norm(B) * h / (2 * g))) < 1e-10
        assert abs(p1 @ bn - p @ bn) < 1e-12 * np.linalg.norm(p)
    # pure E along p: exact kick q E h
    p = np.array([0.0, 0.0, 5.0])
    E = np.array([0.0, 0.0, 0.3])
    np.testing.assert_allclose(orc.boris(p, -1.0, E, np.zeros(3), 2.0), p - 0.6 * np.array([0, 0, 1.0]), rtol=0, atol=1e-15)


def test_chi_closed_forms(orc):
    rng = np.random.default_rng(1)
    for _ in range(100):
        Ed = synth.direction(rng.random(1), rng.random(1))[0]
        Bd = synth.perpendicular(Ed[None, :], rng.random(1))[0]
        n = np.cross(Ed, Bd)
        Em = 10 ** rng.uniform(-4, 0)
        p = rng.normal(size=3) * 10 ** rng.uniform(0, 4)
        g = math.sqrt(1 + p @ p)
        # crossed field |E| = |B|: chi = |E| (gamma - n.p)
        assert abs(orc.chi(p, g, Ed * Em, Bd * Em) / (Em * (g - n @ p)) - 1) < 1e-9
        # photon in crossed field: chi = |E| (eps - n.k)
        eps = np.linalg.norm(p)
        assert abs(orc.chi(p, eps, Ed * Em, Bd * Em) / (Em * (eps - n @ p)) - 1) < 1e-8
        # pure magnetic field: chi = |p x B|
        assert abs(orc.chi(p, g, np.zeros(3), Bd * Em) / np.linalg.norm(np.cross(p, Bd * Em)) - 1) < 1e-12
        # pure electric field: chi = sqrt(gamma^2 E^2 - (p.E)^2)
        E = Ed * Em
        assert abs(orc.chi(p, g, E, np.zeros(3)) / math.sqrt(g * g * (E @ E) - (p @ E) ** 2) - 1) < 1e-9


# ----------------------------------------------------------------------------- order, merge, capacity
def test_append_order_alg2(orc):
    wl = synth.emission_static_b(100_000, indices=np.arange(0, 100_000, 500))
    main, fields, app = _stores(orc, wl)
    rc, stats = orc.step(main, fields, app, wl.dt, 0, 0, emission=1, pair=0, push=0)
    nev = main[0].nev[:main[0].count]
    roots = app[2].root[:app[2].count].view(np.uint32) & 0x3FFFFFFF
    # children of a parent are contiguous, parents in index order, events in time order
    np.testing.assert_array_equal(roots, np.repeat(np.arange(nev.size), nev))
    tb = app[2].t_birth
    for i0, k in zip(np.r_[0, np.cumsum(nev)[:-1]], nev):
        assert np.all(np.diff(tb[i0:i0 + k]) >= 0)
    assert np.all(tb <= wl.dt)
    assert stats.n_emit == nev.sum() == app[2].count
    # ids of children are distinct and differ from the parents'
    ids = np.concatenate([app[2].id[:app[2].count], main[0].id[:main[0].count]])
    assert np.unique(ids).size == ids.size


def test_merge_drops_dead_photons_stably(orc):
    main = [orc.Store(10), orc.Store(10), orc.Store(20)]
    app = [orc.Store(5), orc.Store(5), orc.Store(5)]
    for s in range(3):
        main[s].count = 4
        main[s].id[:4] = np.arange(4) + 10 * s
        main[s].state[:4, 0] = np.arange(4) + 10 * s
        app[s].count = 3
        app[s].id[:3] = np.arange(3) + 100 + 10 * s
        app[s].state[:3, 0] = np.arange(3) + 100 + 10 * s
    main[2].alive[:4] = [1, 0, 1, 0]
    app[2].alive[:3] = [0, 1, 1]
    assert orc.merge(main, app) == 0
    np.testing.assert_array_equal(main[0].id[:main[0].count], [0, 1, 2, 3, 100, 101, 102])
    np.testing.assert_array_equal(main[2].id[:main[2].count], [20, 22, 121, 122])
    np.testing.assert_array_equal(main[2].p[:, 0], [20, 22, 121, 122])


def test_capacity_overflow_reports_and_writes_nothing_past_end(orc):
    wl = synth.emission_static_b(100_000, indices=np.arange(0, 100_000, 1000))
    main, fields, app = _stores(orc, wl)
    small = [orc.Store(8) for _ in range(3)]
    for s in small:
        s.state[:] = np.nan  # sentinel; capacity 8 of a larger buffer
        s.capacity = 5
    rc, stats = orc.step(main, fields, small, wl.dt, 0, 0, emission=1, pair=0, push=0)
    assert rc == 2 and stats.overflow == 1
    assert small[2].count > 5
    assert np.all(np.isnan(small[2].state[5:8]))


def test_init_tau_reserved_counter(orc):
    s = orc.Store.from_arrays(np.zeros((5, 3)), np.ones(5), np.array([-1.0, 2.0, -1.0, -1.0, 0.5]),
                              np.arange(5, dtype=np.uint64) + 7)
    orc.init_tau(s, 9, 4)
    blocks = orc.philox_stream(9, np.arange(5, dtype=np.uint64) + 7, 4, 0xFFFFFFFF)
    ref = -np.log((blocks[:, 0].astype(np.float64) + 0.5) * 2.0 ** -32)
    np.testing.assert_array_equal(s.tau[[0, 2, 3]], ref[[0, 2, 3]])
    np.testing.assert_array_equal(s.tau[[1, 4]], [2.0, 0.5])


# ----------------------------------------------------------------------------- event cap
def test_event_cap(orc):
    """max_events: once a particle has had max_events events in the step it has
    no more (its rate is taken as zero), and the step reports it (status 5).
    The first events are those of the uncapped step (same draws), so the
    capped counts are min(uncapped, cap) and the children are the first ones
    of each parent in the uncapped step."""
    wl = synth.emission_static_b(100_000, indices=np.arange(0, 100_000, 500))
    runs = []
    for cap in (1 << 20, 3):
        main, fields, app = _stores(orc, wl)
        rc, stats = orc.step(main, fields, app, wl.dt, 0, 0, emission=1, pair=0, push=0, max_events=cap)
        runs.append((rc, stats, main[0].nev[:main[0].count].copy(), app[2]))
    (rc_f, st_f, nev_f, app_f), (rc_c, st_c, nev_c, app_c) = runs
    assert rc_f == 0 and rc_c == 5 and st_c.capped == 1
    assert nev_f.max() > 3
    np.testing.assert_array_equal(nev_c, np.minimum(nev_f, 3))
    first = np.concatenate([np.arange(o, o + k) for o, k in zip(np.r_[0, np.cumsum(nev_f)[:-1]], nev_c)])
    np.testing.assert_array_equal(app_c.id[:app_c.count], app_f.id[first])
    np.testing.assert_array_equal(app_c.p, app_f.p[first])
