"""qed_step_merged against qed_step followed by qed_merge.

The merged call compacts the input photons after their round and writes each
appended photon that survives the step straight into the main photon arrays
(offsets from a single-pass look-back), instead of the merge reading it back
from its record.  Nothing in the arithmetic changes, so the merged ensemble
must equal the two-call result exactly: every array, the order and the
counts, for FP32 and FP64, with and without positions, over several
generation rounds."""
import numpy as np
import pytest

import synth

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def build(sf, torch, wl, dtype, x=None, main_extra=(400_000, 400_000, 5_000_000), app_cap=(400_000, 400_000, 5_000_000)):
    main, fields, app = [], [], []
    for s, sp in enumerate(wl.species):
        f = sp.fields if sp.fields.shape[0] else np.zeros((1, 6))
        main.append(sf.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, dtype=dtype, photon=s == 2,
                                         capacity=sp.n + main_extra[s], x=None if x is None else x[s]))
        fields.append(sf.Fields.from_array(f, dtype))
        app.append(sf.AppendBuffer(app_cap[s], dtype, positions=x is not None))
    return main, fields, app


def arrays(store):
    h = store.host()
    return {k: v for k, v in h.items() if k != "nev"}


def compare(sf, torch, wl, dtype, cfg, x=None, steps=1):
    tabs = sf.Tables()
    ma, fa, aa = build(sf, torch, wl, dtype, x)
    mb, fb, ab = build(sf, torch, wl, dtype, x)
    for k in range(steps):
        rc, st_a = sf.step(tabs, ma, fa, aa, wl.dt, 5, k, cfg)
        sf.merge(ma, fa, aa)
        rc_b, st_b = sf.step_merged(tabs, mb, fb, ab, wl.dt, 5, k, cfg)
        torch.cuda.synchronize()
        assert rc == 0 and rc_b == 0
        assert st_a.n_emit == st_b.n_emit and st_a.n_pair == st_b.n_pair and st_a.n_rounds == st_b.n_rounds
        for s in range(3):
            assert ma[s].count == mb[s].count, (k, s, ma[s].count, mb[s].count)
            A, B = arrays(ma[s]), arrays(mb[s])
            for name in A:
                assert np.array_equal(A[name], B[name]), (k, s, name)
        for s in range(2):
            assert aa[s].count == ab[s].count
            assert np.array_equal(aa[s].records(), ab[s].records())
    return st_a, [m.count for m in ma]


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_crossed_field_sample(dtype_name):
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 200), np.arange(0, 4_000_000, 200),
                                                  np.arange(0, 2_000_000, 200)])
    st, counts = compare(sf, torch, wl, getattr(torch, dtype_name), sf.step_cfg(push=False, gamma_min=2.0))
    print(f"{dtype_name}: {st.n_emit} photons, {st.n_pair} pairs, {st.n_rounds} rounds; merged counts {counts}")
    assert st.n_pair > 1000 and st.n_rounds >= 5


def test_positions_and_cascade_steps():
    """Positions on, push on, three consecutive steps of the rotating-field
    cascade (the merged ensemble feeds the next step)."""
    torch, sf = need_gpu()
    wl = synth.rotating_e(1_000_000, indices=np.arange(0, 1_000_000, 500))
    rng = np.random.default_rng(8)
    x = [rng.normal(0.0, 1e3, (sp.n, 3)) for sp in wl.species]
    st, counts = compare(sf, torch, wl, torch.float32, sf.step_cfg(push=True), x=x, steps=3)
    print(f"3 steps: merged counts {counts}")
    assert counts[2] > 0 and counts[0] > wl.species[0].n


def test_photon_capacity():
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 2000), np.arange(0, 4_000_000, 2000),
                                                  np.arange(0, 2_000_000, 2000)])
    main, fields, app = build(sf, torch, wl, torch.float32, main_extra=(100_000, 100_000, 10))
    rc, st = sf.step_merged(sf.Tables(), main, fields, app, wl.dt, 0, 0, sf.step_cfg(push=False, gamma_min=2.0),
                            check=False)
    torch.cuda.synchronize()
    assert rc == 2
    assert main[2].count <= main[2].capacity


def test_append_capacity():
    """The merged step sizes each round's appended-photon range on the device,
    clamped to the append capacity: with a photon append buffer far too small
    it reports the overflow with the capacity it would have needed and writes
    nothing past any capacity."""
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 2000), np.arange(0, 4_000_000, 2000),
                                                  np.arange(0, 2_000_000, 2000)])
    main, fields, app = build(sf, torch, wl, torch.float32, app_cap=(400_000, 400_000, 10_000))
    app[2].cap = 5_000  # the library sees 5,000 records; the 5,000 behind them must stay untouched
    rc, st = sf.step_merged(sf.Tables(), main, fields, app, wl.dt, 0, 0, sf.step_cfg(push=False, gamma_min=2.0),
                            check=False)
    torch.cuda.synchronize()
    assert rc == 2
    assert st.required_capacity[2] > 5_000
    assert app[2].count <= 5_000 and main[2].count <= main[2].capacity
    rec = app[2].rec_dtype.itemsize
    assert not app[2].data[5_000 * rec:].any()


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_rounds_that_append_no_photons(dtype_name):
    """A round whose leptons emit nothing leaves the merged step an empty
    appended-photon range, sized on the device.  Its photon pass must list
    no events, whatever the previous launch (here the input photons' pass)
    left in the event list.  A step with emission first fills the photon
    append buffers; a step without emission (pairs on) then starts from
    fresh copies of the input ensemble, its per-particle fields covering
    every particle, on the same append buffers, which still hold those
    photon records.  It must equal qed_step followed by qed_merge."""
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 400), np.arange(0, 4_000_000, 400),
                                                  np.arange(0, 2_000_000, 100)])
    tabs = sf.Tables()
    dtype = getattr(torch, dtype_name)
    ma, fa, aa = build(sf, torch, wl, dtype)
    mb, fb, ab = build(sf, torch, wl, dtype)
    cfg = sf.step_cfg(push=False, gamma_min=2.0)
    rc, st_a = sf.step(tabs, ma, fa, aa, wl.dt, 5, 0, cfg)
    rc_b, st_b = sf.step_merged(tabs, mb, fb, ab, wl.dt, 5, 0, cfg)
    torch.cuda.synchronize()
    assert rc == 0 and rc_b == 0 and st_a.n_emit == st_b.n_emit > 100_000
    # fresh input ensembles and fields (as many entries as particles); the append buffers are kept
    ma, fa, _ = build(sf, torch, wl, dtype)
    mb, fb, _ = build(sf, torch, wl, dtype)
    cfg = sf.step_cfg(push=False, gamma_min=2.0, emission=False)
    rc, st_a = sf.step(tabs, ma, fa, aa, wl.dt, 5, 1, cfg)
    sf.merge(ma, fa, aa)
    rc_b, st_b = sf.step_merged(tabs, mb, fb, ab, wl.dt, 5, 1, cfg)
    torch.cuda.synchronize()
    assert rc == 0 and rc_b == 0
    print(f"without emission: {st_a.n_emit} photons, {st_a.n_pair} pairs, {st_a.n_rounds} rounds")
    assert st_a.n_emit == st_b.n_emit == 0 and st_a.n_pair == st_b.n_pair > 0
    assert st_a.n_rounds == st_b.n_rounds
    for s in range(3):
        assert ma[s].count == mb[s].count, (s, ma[s].count, mb[s].count)
        A, B = arrays(ma[s]), arrays(mb[s])
        for name in A:
            assert np.array_equal(A[name], B[name]), (s, name)
    for s in range(2):
        assert aa[s].count == ab[s].count
        assert np.array_equal(aa[s].records(), ab[s].records())


def test_staged_records_equal_direct_stores(monkeypatch):
    """The FP32 lepton write kernel stages child records in LDS and writes them
    in half lines; with SFQED_WRITE_STAGING=0 it stores each record directly
    (512-thread blocks).  Staging changes how the records reach memory, not
    what they hold: every appended record, every main array and every count
    must be identical, on the same tables, over several generation rounds."""
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 400), np.arange(0, 4_000_000, 400),
                                                  np.arange(0, 2_000_000, 400)])
    tabs = sf.Tables()
    cfg = sf.step_cfg(push=False, gamma_min=2.0)
    runs = []
    monkeypatch.setenv("SFQED_WRITE_REPLAY", "0")  # the direct write kernel, staged or not
    for flag in ("1", "0"):
        monkeypatch.setenv("SFQED_WRITE_STAGING", flag)
        main, fields, app = build(sf, torch, wl, torch.float32)
        rc, st = sf.step(tabs, main, fields, app, wl.dt, 11, 0, cfg)
        torch.cuda.synchronize()
        assert rc == 0
        runs.append((st, [arrays(m) for m in main], [a.records() for a in app], [a.count for a in app]))
    (sa, ma, ra, ca), (sb, mb, rb, cb) = runs
    assert sa.n_emit == sb.n_emit and sa.n_pair == sb.n_pair and sa.n_rounds == sb.n_rounds and ca == cb
    print(f"{sa.n_emit} photons, {sa.n_pair} pairs, {sa.n_rounds} rounds: identical with and without staging")
    assert sa.n_emit > 100_000 and sa.n_rounds >= 5
    for s in range(3):
        assert np.array_equal(ra[s], rb[s]), s
        for name in ma[s]:
            assert np.array_equal(ma[s][name], mb[s][name]), (s, name)


def _replay_vs_direct(monkeypatch, sf, torch, wl, dtype, cfg, x=None, steps=1, merged=False):
    """Runs the same steps with the write pass replayed from the count pass's
    event log and with the direct write kernel; returns both results."""
    tabs = sf.Tables()
    runs = []
    for flag in ("0", "1", "1"):  # the first logged run may size the log pool; the second must replay
        monkeypatch.setenv("SFQED_WRITE_REPLAY", flag)
        main, fields, app = build(sf, torch, wl, dtype, x)
        sts = []
        for k in range(steps):
            fn = sf.step_merged if merged else sf.step
            rc, st = fn(tabs, main, fields, app, wl.dt, 3, k, cfg)
            assert rc == 0
            if not merged:
                sf.merge(main, fields, app)
            sts.append(st)
        torch.cuda.synchronize()
        runs.append((sts, [arrays(m) for m in main], [a.records() for a in app], [m.count for m in main]))
    direct, replay = runs[0], runs[2]
    assert all(st.log_replays == 0 for st in direct[0])
    assert all(st.log_replays > 0 and st.log_reruns == 0 for st in replay[0]), \
        [(st.log_replays, st.log_reruns) for st in replay[0]]
    for a, b in zip(direct[0], replay[0]):
        assert (a.n_emit, a.n_pair, a.n_rounds) == (b.n_emit, b.n_pair, b.n_rounds)
    assert direct[3] == replay[3]
    for s in range(3):
        assert np.array_equal(direct[2][s], replay[2][s]), s
        for name in direct[1][s]:
            assert np.array_equal(direct[1][s][name], replay[1][s][name]), (s, name)
    return replay[0][-1], replay[3]


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_replayed_writes_equal_direct_writes(monkeypatch, dtype_name):
    """The lepton write pass replayed from the count pass's event log (z, h and
    the child optical depth of every event, the final optical depth of every
    particle) writes what the direct write kernel writes by re-running each
    event from the tables: every record, array and count identical, over a
    multi-round step with both processes."""
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 400), np.arange(0, 4_000_000, 400),
                                                  np.arange(0, 2_000_000, 400)])
    st, counts = _replay_vs_direct(monkeypatch, sf, torch, wl, getattr(torch, dtype_name),
                                   sf.step_cfg(push=False, gamma_min=2.0))
    print(f"{dtype_name}: {st.n_emit} photons, {st.n_pair} pairs, {st.n_rounds} rounds, "
          f"{st.log_replays} launches replayed: identical to the direct writes")
    assert st.n_pair > 1000 and st.n_rounds >= 5


def test_replayed_writes_with_push_and_positions(monkeypatch):
    """The same with the Boris push and positions (the replay re-applies the
    push over each logged sub-interval), three merged steps of the rotating
    field cascade."""
    torch, sf = need_gpu()
    wl = synth.rotating_e(1_000_000, indices=np.arange(0, 1_000_000, 500))
    rng = np.random.default_rng(9)
    x = [rng.normal(0.0, 1e3, (sp.n, 3)) for sp in wl.species]
    st, counts = _replay_vs_direct(monkeypatch, sf, torch, wl, torch.float32, sf.step_cfg(push=True), x=x,
                                   steps=3, merged=True)
    print(f"3 merged steps with push and positions: counts {counts}, identical to the direct writes")
    assert counts[0] > wl.species[0].n


def test_short_fields_are_refused_before_any_change():
    """Per-particle fields with fewer entries than particles: both steps
    return QED_ERR_ARG before any device work, and the ensemble and the
    append buffers are left as they were."""
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 4000), np.arange(0, 4_000_000, 4000),
                                                  np.arange(0, 2_000_000, 4000)])
    main, fields, app = build(sf, torch, wl, torch.float32)
    short = sf.Fields(*[getattr(fields[2], c)[:-1] for c in ("ex", "ey", "ez", "bx", "by", "bz")], stride=1)
    before = [arrays(m) for m in main]
    counts = [m.count for m in main]
    for fn in (sf.step, sf.step_merged):
        rc, _ = fn(sf.Tables(), main, [fields[0], fields[1], short], app, wl.dt, 0, 0,
                   sf.step_cfg(push=False), check=False)
        assert rc == 1
        assert b"fields of species 2" in sf.lib().qed_last_error()
    torch.cuda.synchronize()
    assert [m.count for m in main] == counts and [a.count for a in app] == [0, 0, 0]
    for s in range(3):
        A = arrays(main[s])
        for name in A:
            assert np.array_equal(A[name], before[s][name]), (s, name)
