"""Pins of the oracle's resampling (global leveling and the photon energy
filter, Sec. 4.2 and Sec. 5.1): closed forms of the threshold weight, the
defining equation at random weights, and the two expectations leveling must
keep (count at the target, total weight unchanged) over many draws."""
import numpy as np
import pytest

from oracle import resample as rs


def test_threshold_equal_weights():
    # N equal weights w0 thinned to n_t: every particle stays with probability
    # n_t / N, so w_th = w0 N / n_t
    for n, nt, w0 in ((1000, 250, 0.5), (7, 3, 2.0), (10, 9, 1e-3)):
        assert rs.leveling_threshold(np.full(n, w0), nt) == pytest.approx(w0 * n / nt, rel=1e-15)


def test_threshold_two_classes():
    # 600 particles of weight 1 and 400 of weight 10 thinned to 500: the heavy
    # ones all stay (10 > w_th), the light ones fill the remaining 100 on
    # average: 600 / w_th = 100, so w_th = 6
    w = np.concatenate([np.ones(600), np.full(400, 10.0)])
    np.random.default_rng(0).shuffle(w)
    assert rs.leveling_threshold(w, 500) == pytest.approx(6.0, rel=1e-15)
    # target below the heavy class: everything is thinned, w_th = sum / n_t
    assert rs.leveling_threshold(w, 200) == pytest.approx(4600.0 / 200, rel=1e-15)


def test_threshold_solves_definition():
    rng = np.random.default_rng(1)
    for n, nt in ((5000, 1234), (3000, 2999), (100, 1)):
        w = np.exp(rng.normal(0.0, 2.0, n))
        wth = rs.leveling_threshold(w, nt)
        assert np.minimum(1.0, w / wth).sum() == pytest.approx(nt, rel=1e-10)
    assert rs.leveling_threshold(np.ones(10), 10) is None
    assert rs.leveling_threshold(np.ones(10), 20) is None


def test_leveling_expectations():
    # over many seeds: mean survivor count -> n_t and mean total weight -> sum w
    rng = np.random.default_rng(2)
    n, nt, runs = 2000, 500, 200
    w = np.exp(rng.normal(0.0, 1.0, n)).astype(np.float32).astype(np.float64)
    ids = np.arange(n, dtype=np.uint64) * 7919 + 11
    p = np.ones((n, 3))
    counts, weights = [], []
    for seed in range(runs):
        keep, wn, wth, _ = rs.resample(p, w, ids, seed, 3, n_target=nt)
        counts.append(keep.sum())
        weights.append(wn[keep].sum())
    counts, weights = np.array(counts), np.array(weights)
    se_c = counts.std(ddof=1) / np.sqrt(runs)
    se_w = weights.std(ddof=1) / np.sqrt(runs)
    assert abs(counts.mean() - nt) < 5 * se_c + 1e-9
    assert abs(weights.mean() - w.sum()) < 5 * se_w
    # heavy particles are never touched
    keep, wn, wth, _ = rs.resample(p, w, ids, 0, 3, n_target=nt)
    heavy = w >= wth
    assert keep[heavy].all() and np.array_equal(wn[heavy], w[heavy])
    assert np.all(wn[keep & ~heavy] == wth)


def test_energy_filter_and_determinism():
    rng = np.random.default_rng(3)
    n = 1000
    p = rng.normal(0.0, 3.0, (n, 3))
    w = np.ones(n)
    ids = np.arange(n, dtype=np.uint64)
    keep, wn, wth, nf = rs.resample(p, w, ids, 5, 1, e_min=2.0, photon=True)
    e = np.linalg.norm(p, axis=1)
    assert np.array_equal(keep, e >= 2.0) and nf == int((e < 2.0).sum()) and wth is None
    # leptons are not filtered
    keep_l, _, _, nf_l = rs.resample(p, w, ids, 5, 1, e_min=2.0, photon=False)
    assert keep_l.all() and nf_l == 0
    # the same seed and step give the same survivors; another step other ones
    a = rs.resample(p, w, ids, 5, 1, n_target=300)[0]
    b = rs.resample(p, w, ids, 5, 1, n_target=300)[0]
    c = rs.resample(p, w, ids, 5, 2, n_target=300)[0]
    assert np.array_equal(a, b) and not np.array_equal(a, c)
