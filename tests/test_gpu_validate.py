"""The debug validation pass (qed_validate and qed_step_cfg.validate)
against its plain definition: a live particle is counted when any of its
momentum components, weight, optical depth, or its six field components (its
own, or the shared value) is NaN or infinite.  The step with validation on
refuses such an ensemble with QED_ERR_ARG and changes nothing; on a clean
ensemble it gives the same results as the step without it."""
import numpy as np
import pytest

import synth

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def _build(sf, wl, dtype, shared_photon_field=None):
    main, fields, app = [], [], []
    for s, sp in enumerate(wl.species):
        f = sp.fields if sp.fields.shape[0] else np.zeros((1, 6))
        if s == 2 and shared_photon_field is not None:
            f = np.asarray(shared_photon_field, dtype=np.float64).reshape(1, 6)
        main.append(sf.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, dtype=dtype, photon=s == 2,
                                         capacity=sp.n + (400_000 if s < 2 else 4_000_000)))
        fields.append(sf.Fields.from_array(f, dtype))
        app.append(sf.AppendBuffer(400_000 if s < 2 else 4_000_000, dtype))
    return main, fields, app


def _definition(main, fields):
    """The count the pass must return, from host copies."""
    out = []
    for m, f in zip(main, fields):
        n = m.count
        h = [t[:n].double().cpu().numpy() for t in (m.px, m.py, m.pz, m.w, m.tau)]
        ok = np.all(np.isfinite(np.stack(h, axis=1)), axis=1) if n else np.zeros(0, bool)
        fv = np.stack([t.double().cpu().numpy() for t in (f.ex, f.ey, f.ez, f.bx, f.by, f.bz)], axis=1)
        fok = np.all(np.isfinite(fv), axis=1)
        ok &= fok[:n] if f.stride == 1 else np.full(n, fok[0])
        out.append(int((~ok).sum()))
    return out


def _snapshot(main):
    return [{k: v.copy() for k, v in m.host().items()} for m in main]


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_counts_and_refusal(dtype_name):
    torch, sf = need_gpu()
    dtype = getattr(torch, dtype_name)
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 400), np.arange(0, 4_000_000, 400),
                                                  np.arange(0, 2_000_000, 400)])
    main, fields, app = _build(sf, wl, dtype)
    rc, bad = sf.validate(main, fields)
    assert rc == 0 and bad == [0, 0, 0]
    # plant non-finite values: two in one electron, one per other species, one in a field
    main[0].px[3] = float("nan")
    main[0].w[3] = float("inf")
    main[0].tau[8] = -float("inf")
    main[1].pz[5] = float("-inf")
    fields[2].bz[7] = float("nan")
    main[2].w[main[2].count - 1] = float("nan")
    main[2].px[main[2].count] = float("nan")  # beyond the count: not a live particle
    want = _definition(main, fields)
    assert want == [2, 1, 2]
    rc, bad = sf.validate(main, fields)
    assert rc == 1 and bad == want, (rc, bad, want)
    before = _snapshot(main)
    rc, _ = sf.step(sf.Tables(), main, fields, app, wl.dt, 0, 0, sf.step_cfg(push=False, validate=True), check=False)
    torch.cuda.synchronize()
    assert rc == 1
    after = _snapshot(main)
    for b, a in zip(before, after):
        for k in b:
            assert np.array_equal(b[k], a[k], equal_nan=k not in ("id", "alive", "nev")), k
    assert [x.count for x in app] == [0, 0, 0]


def test_shared_field_counts_every_particle():
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 4000), np.arange(0, 4_000_000, 4000),
                                                  np.arange(0, 2_000_000, 400)])
    main, fields, _ = _build(sf, wl, torch.float32, shared_photon_field=[0, 0, 1e-3, float("inf"), 0, 0])
    rc, bad = sf.validate(main, fields)
    assert rc == 1 and bad == [0, 0, main[2].count]


@pytest.mark.parametrize("merged", [False, True])
def test_clean_step_unchanged_by_validation(merged):
    torch, sf = need_gpu()
    wl = synth.crossed_field(10_000_000, indices=[np.arange(0, 4_000_000, 400), np.arange(0, 4_000_000, 400),
                                                  np.arange(0, 2_000_000, 400)])
    tabs = sf.Tables()
    res = []
    for validate in (False, True):
        main, fields, app = _build(sf, wl, torch.float32)
        fn = sf.step_merged if merged else sf.step
        rc, st = fn(tabs, main, fields, app, wl.dt, 3, 0, sf.step_cfg(push=False, gamma_min=2.0, validate=validate))
        torch.cuda.synchronize()
        assert rc == 0
        res.append((st.n_emit, st.n_pair, _snapshot(main), [a.records().tobytes() for a in app[:2]]))
    (e0, p0, m0, r0), (e1, p1, m1, r1) = res
    assert (e0, p0) == (e1, p1) and e0 > 0
    assert r0 == r1
    for b, a in zip(m0, m1):
        for k in b:
            assert np.array_equal(b[k], a[k]), k
