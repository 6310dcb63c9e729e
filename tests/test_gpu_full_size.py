"""The crossed-field step at full size (1e7 particles), in the configuration the
benchmark times (restore, then qed_step_merged; FP32, push off, gamma_min 2,
seed 0, step 0), checked against the oracle where it can follow single
particles and by properties that hold at any size.

* Sampled particles: 40 electrons, 40 positrons and 40 photons spread over the
  ensemble are stepped by the FP64 oracle together with every descendant
  (Algorithms 1 and 2 from the same random stream).  Leptons keep their index
  through the merge, so their final momenta compare directly; descendants are
  found in the merged GPU ensemble by id.  FP32 arithmetic and tables flip a
  decision now and then (a flipped particle's history differs from there on),
  so the bar is on the fraction that agrees and on the median error.
* Momentum conservation: with push off, recoil (p -> (1 - delta) p plus the
  photon delta p) and pair creation (k -> xi k + (1 - xi) k) conserve the total
  momentum exactly, so the weighted sum over all species before and after the
  step differs only by FP32 rounding.
* Counts: the merged counts follow from the step's statistics."""
import gc

import numpy as np
import pytest

import synth

from gpu_util import cast_inputs, need_gpu, run_oracle

pytestmark = pytest.mark.gpu


def total_momentum(torch, main):
    tot = torch.zeros(3, dtype=torch.float64, device="cuda")
    absum = torch.zeros((), dtype=torch.float64, device="cuda")
    for m in main:
        n = m.count
        if n == 0:
            continue
        w = m.w[:n].double()
        for c, t in enumerate((m.px, m.py, m.pz)):
            v = t[:n].double()
            tot[c] += (w * v).sum()
            absum += (w * v.abs()).sum()
    return tot.cpu().numpy(), float(absum)


def test_crossed_field_full_size():
    torch, sf = need_gpu()
    import bench
    torch.cuda.empty_cache()
    n_all = 10_000_000
    wl = synth.crossed_field(n_all)
    caps = [int(n_all * 12), int(n_all * 12), int(min(1e9, (1 << 30) - 1024))]
    dw = bench.DeviceWorkload(sf, torch, wl, caps, torch.float32)
    tables = sf.Tables()
    cfg = sf.step_cfg(push=False, gamma_min=2.0, nev=False)
    dw.restore()
    p_before, _ = total_momentum(torch, dw.main)
    rc, st = dw.step(tables, 0, cfg)
    torch.cuda.synchronize()
    assert rc == 0
    main = dw.main
    # counts
    n_in = dw.n
    assert main[0].count == n_in[0] + st.n_new[0] and main[1].count == n_in[1] + st.n_new[1]
    assert main[2].count == n_in[2] + st.n_new[2] - st.n_pair
    # momentum conservation over 6.6e8 particles
    p_after, absum = total_momentum(torch, main)
    dp = np.linalg.norm(p_after - p_before) / absum
    print(f"full size: {st.n_emit} photons, {st.n_pair} pairs, {st.n_rounds} rounds; counts "
          f"{[m.count for m in main]}; |delta P| / sum |p| = {dp:.2e}")
    assert dp < 1e-5

    # sampled particles through the oracle
    counts = [int(round(n_all * 0.4)), int(round(n_all * 0.4))]
    counts.append(n_all - sum(counts))
    idx = [np.arange(counts[0] // 80, counts[0], counts[0] // 40)[:40],
           np.arange(counts[1] // 80, counts[1], counts[1] // 40)[:40],
           np.arange(counts[2] // 80, counts[2], counts[2] // 40)[:40]]
    ws = synth.crossed_field(n_all, indices=idx)
    inp = cast_inputs(ws, np.float32)
    cap_o = [200_000, 200_000, 2_000_000]
    rco, sto, mo, ao = run_oracle(ws, inp, cap_o, seed=0, step_index=0, emission=1, pair=1, push=0, gamma_min=2.0)
    assert rco == 0
    # parents: leptons keep their index through the merge
    for s in range(2):
        i = torch.as_tensor(idx[s].astype(np.int64), device="cuda")
        pg = torch.stack([t[i] for t in (main[s].px, main[s].py, main[s].pz)], 1).double().cpu().numpy()
        po = mo[s].p[:mo[s].count]
        err = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1)
        print(f"species {s}: final momenta of 40 sampled parents, median rel. error {np.median(err):.1e}, "
              f"{(err < 1e-3).mean():.0%} within 1e-3")
        assert np.median(err) < 1e-4 and (err < 1e-3).mean() >= 0.9
    # descendants (and surviving sampled photons) found by id in the merged GPU ensemble
    for s in range(3):
        o = ao[s]
        keep = o.alive[:o.count] != 0
        ids_o = o.id[:o.count][keep]
        p_o = o.p[:o.count][keep]
        if s == 2:  # sampled input photons that made no pair are in the merged ensemble too
            alive_in = mo[2].alive[:mo[2].count] != 0
            ids_o = np.concatenate([mo[2].id[:mo[2].count][alive_in], ids_o])
            p_o = np.concatenate([mo[2].p[:mo[2].count][alive_in], p_o])
        ids_t = torch.as_tensor(ids_o.view(np.int64), device="cuda")
        gid = main[s].id[:main[s].count]
        hit = torch.isin(gid, ids_t)
        pos = torch.nonzero(hit).flatten()
        found_ids = gid[pos].cpu().numpy().view(np.uint64)
        pg = torch.stack([t[pos] for t in (main[s].px, main[s].py, main[s].pz)], 1).double().cpu().numpy()
        order_o = {int(v): k for k, v in enumerate(ids_o)}
        po = np.array([p_o[order_o[int(v)]] for v in found_ids]).reshape(-1, 3)
        frac = found_ids.size / max(ids_o.size, 1)
        err = np.linalg.norm(pg - po, axis=1) / np.maximum(np.linalg.norm(po, axis=1), 1e-30)
        print(f"species {s}: {ids_o.size} oracle particles, {frac:.2%} found on the GPU, median rel. error "
              f"{np.median(err) if err.size else 0:.1e}")
        assert ids_o.size > 0 and frac > 0.98
        assert np.median(err) < 1e-4 and (err < 1e-3).mean() > 0.95
    del dw, main
    gc.collect()
    torch.cuda.empty_cache()
