"""qed_resample (photon energy filter and global leveling after the merge,
Sec. 4.2 and Sec. 5.1) against the oracle.

The threshold weight is a root found by two different algorithms (the oracle
sorts the weights; the library runs Newton's method on sums), so it is
compared to 1e-12 relative.  Given the library's threshold, the survivors,
their order and every stored value must equal the oracle's bit for bit."""
import numpy as np
import pytest

from oracle import resample as ors

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def ensemble(n, seed, positions=False):
    """Three species with log-normal weights (FP32) and a few equal-weight
    groups (the ties a cascade produces)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(3):
        m = n[s]
        p = rng.normal(0.0, 3.0, (m, 3))
        w = np.exp(rng.normal(0.0, 1.0, m)).astype(np.float32)
        w[: m // 4] = np.float32(0.75)
        rng.shuffle(w)
        tau = rng.exponential(1.0, m)
        ids = rng.integers(0, 2**63, m, dtype=np.uint64)
        x = rng.normal(0.0, 1.0, (m, 3)) if positions else None
        out.append((p, w, tau, ids, x))
    return out


def run(torch, sf, data, dtype, cfg_kw, capacity_extra=5):
    main, fields = [], []
    for s, (p, w, tau, ids, x) in enumerate(data):
        main.append(sf.Store.from_arrays(p, w, tau, ids, dtype=dtype, photon=s == 2, x=x,
                                         capacity=len(ids) + capacity_extra))
        fields.append(sf.Fields.from_array(np.zeros((1, 6)), dtype))
    st = sf.resample(main, fields, sf.resample_cfg(**cfg_kw))
    torch.cuda.synchronize()
    return main, st


def check_species(sf, store, data, s, st, cfg_kw, dtype_np):
    p, w, tau, ids, x = data
    # the inputs as the device holds them
    pr = p.astype(dtype_np).astype(np.float64)
    wr = w.astype(np.float64)
    target = cfg_kw.get("target", (0, 0, 0))[s]
    e_min = cfg_kw.get("photon_energy_min", 0.0)
    keep_f, _, wth_o, nf = ors.resample(pr, wr, ids, cfg_kw.get("seed", 0), cfg_kw.get("step", 0),
                                        n_target=target, e_min=e_min, photon=s == 2)
    wth_g = st.w_threshold[s]
    if wth_o is None:
        assert wth_g == 0.0
    else:
        assert abs(wth_g - wth_o) <= 1e-12 * wth_o, (wth_g, wth_o)
    # decisions with the library's threshold
    keep, wn, _, _ = ors.resample(pr, wr, ids, cfg_kw.get("seed", 0), cfg_kw.get("step", 0),
                                  e_min=e_min, photon=s == 2, w_th=(wth_g if wth_g > 0 else None))
    h = store.host()
    assert store.count == int(keep.sum()) == st.count_after[s]
    assert np.array_equal(h["id"], ids[keep])
    assert np.array_equal(h["p"], pr[keep])
    assert np.array_equal(h["tau"], tau[keep])
    assert np.array_equal(h["w"], wn[keep].astype(np.float32))
    if x is not None:
        assert np.array_equal(h["x"], x.astype(dtype_np).astype(np.float64)[keep])
    if s == 2:
        assert np.all(h["alive"] == 1)
        assert st.filtered == nf
    return wth_g


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_leveling_and_filter_parity(dtype_name):
    torch, sf = need_gpu()
    dtype = getattr(torch, dtype_name)
    dnp = np.float32 if dtype_name == "float32" else np.float64
    n = (70001, 5003, 123457)
    data = ensemble(n, 11)
    cfg = dict(photon_energy_min=2.0, target=(20000, 6000, 40000), seed=7, step=3)
    main, st = run(torch, sf, data, dtype, cfg)
    print(f"{dtype_name}: counts {list(st.count_before)} -> {list(st.count_after)}, w_th {list(st.w_threshold)}, "
          f"iterations {list(st.iterations)}, photons filtered {st.filtered}")
    for s in range(3):
        check_species(sf, main[s], data[s], s, st, cfg, dnp)
    assert st.w_threshold[1] == 0.0 and st.count_after[1] == n[1]   # below its target: untouched
    assert st.iterations[0] < 40 and st.iterations[2] < 40


def test_filter_only_positions_and_determinism():
    torch, sf = need_gpu()
    data = ensemble((1000, 1000, 50000), 12, positions=True)
    cfg = dict(photon_energy_min=3.0, seed=1, step=9)
    main, st = run(torch, sf, data, torch.float32, cfg)
    for s in range(3):
        check_species(sf, main[s], data[s], s, st, cfg, np.float32)
    assert st.count_after[0] == 1000 and st.count_after[1] == 1000
    # the same call again gives the same survivors
    main2, st2 = run(torch, sf, data, torch.float32, cfg)
    assert np.array_equal(main[2].host()["id"], main2[2].host()["id"])
    # a different step changes the draws of a thinning
    cfg_a = dict(target=(0, 0, 10000), seed=1, step=9)
    cfg_b = dict(target=(0, 0, 10000), seed=1, step=10)
    ma, _ = run(torch, sf, data, torch.float32, cfg_a)
    mb, _ = run(torch, sf, data, torch.float32, cfg_b)
    assert not np.array_equal(ma[2].host()["id"], mb[2].host()["id"])


def test_edge_cases():
    torch, sf = need_gpu()
    # empty species, a species exactly at its target, a target of 1
    data = ensemble((0, 300, 4096), 13)
    cfg = dict(target=(5, 300, 1), seed=2, step=0)
    main, st = run(torch, sf, data, torch.float32, cfg)
    assert st.count_after[0] == 0 and st.count_after[1] == 300 and st.w_threshold[1] == 0.0
    check_species(sf, main[2], data[2], 2, st, cfg, np.float32)
    with pytest.raises(sf.SfqedError):
        sf.resample(main, [sf.Fields.from_array(np.zeros((1, 6)), torch.float32)] * 3,
                    sf.resample_cfg(photon_energy_min=-1.0))


def test_queued_passes_follow_the_last_solve():
    """The Newton passes queued without waiting for the host follow the last
    solve's count (plus one).  A solve that needs more finishes pass by pass on
    the host and must give the same threshold and survivors as one that had
    enough passes queued."""
    torch, sf = need_gpu()
    # equal weights: w_0 = total / target is already the root, one pass confirms it
    flat = [(p, np.full_like(w, 0.75), tau, ids, x) for (p, w, tau, ids, x) in ensemble((4000, 4000, 4000), 14)]
    _, st0 = run(torch, sf, flat, torch.float32, dict(target=(1000, 1000, 1000), seed=3, step=1))
    assert list(st0.iterations) == [1, 1, 1]
    data = ensemble((70001, 5003, 123457), 11)
    cfg = dict(photon_energy_min=2.0, target=(20000, 6000, 40000), seed=7, step=3)
    main, st = run(torch, sf, data, torch.float32, cfg)   # two passes queued: the host finishes the solve
    assert st.iterations[0] > 2 and st.iterations[2] > 2
    for s in range(3):
        check_species(sf, main[s], data[s], s, st, cfg, np.float32)
    main2, st2 = run(torch, sf, data, torch.float32, cfg)  # now enough passes are queued
    assert list(st2.iterations) == list(st.iterations) and list(st2.w_threshold) == list(st.w_threshold)
    for s in range(3):
        a, b = main[s].host(), main2[s].host()
        assert all(np.array_equal(a[k], b[k]) for k in a)
