"""Checkpoint and resume on the GPU: the rotating-field cascade (push on,
qed_step_merged every step) run for 5 steps, saved to a file on the host,
restored into fresh device memory and run for 5 more steps ends bit for bit
where the same cascade run for 10 steps without a stop ends: every array of
every species, in order, and the counts after every step.  The same for the
standing-wave test problem on its grid (positions, gathered fields, photon
filter).  Both dtypes."""
import numpy as np
import pytest

import synth

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
SEEDS = 500


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_five_plus_five_equals_ten(tmp_path, dtype_name):
    torch, sf = need_gpu()
    from paper_2409_17299_amd import cascade, checkpoint
    dtype = getattr(torch, dtype_name)
    wl = synth.rotating_e(1_000_000, indices=np.arange(SEEDS))
    e0, wdt = wl.flags["e0"], wl.flags["omega_dt"]
    field = lambda k: synth.rotating_field(e0, wdt, k)  # noqa: E731
    sp = [(s.p, s.w, s.tau, s.id) for s in wl.species]
    cap, app_cap = [SEEDS * 100, SEEDS * 100, SEEDS * 400], [SEEDS * 40, SEEDS * 40, SEEDS * 160]
    tabs = sf.Tables()
    print(f"{dtype_name}: 10 steps straight", flush=True)
    counts_a, _, _, main_a, _ = cascade.run(tabs, sp, wl.dt, 10, field, cap, app_cap, dtype=dtype, seed=4)
    print(f"{dtype_name}: 5 steps, save, load, 5 steps", flush=True)
    counts_b1, _, _, main_b, _ = cascade.run(tabs, sp, wl.dt, 5, field, cap, app_cap, dtype=dtype, seed=4)
    path = checkpoint.save(tmp_path / "ck.npz", main_b, next_step=5, seed=4)
    del main_b
    torch.cuda.empty_cache()
    restored, meta = checkpoint.load(path)
    counts_b2, _, _, main_c, _ = cascade.run(tabs, None, wl.dt, 5, field, None, app_cap, seed=meta["seed"],
                                             start=meta["next_step"], main=restored)
    print(f"counts after 10 steps {counts_a[-1].tolist()}, resumed {counts_b2[-1].tolist()}")
    assert counts_a[-1].sum() > 5 * SEEDS  # the cascade has grown
    assert np.array_equal(counts_a[:6], counts_b1)
    assert np.array_equal(counts_a[5:], counts_b2)
    for s in range(3):
        a, c = main_a[s], main_c[s]
        assert a.count == c.count
        for name in ("px", "py", "pz", "w", "tau", "id", "alive"):
            ta = getattr(a, name)
            if ta is None:
                continue
            tc = getattr(c, name)
            assert ta[: a.count].cpu().numpy().tobytes() == tc[: c.count].cpu().numpy().tobytes(), (s, name)


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_standing_wave_resume(tmp_path, dtype_name):
    """The standing-wave test problem on its grid (positions wrapped and
    fields gathered every step, photon filter after every merge), stopped
    after 60 steps, saved with its positions, restored and run 60 more:
    bit for bit the 120-step run."""
    torch, sf = need_gpu()
    from paper_2409_17299_amd import cascade, checkpoint
    dtype = getattr(torch, dtype_name)
    seeds = 1000
    wl = synth.standing_wave(250_000, indices=np.arange(0, 250_000, 250_000 // seeds))
    sp = [(s.p, s.w, s.tau, s.id, s.x) for s in wl.species]
    cap, app_cap = [seeds * 100, seeds * 100, seeds * 400], [seeds * 20, seeds * 20, seeds * 200]
    tabs = sf.Tables()
    rs = dict(photon_energy_min=2.0)

    def run(steps, start=0, main=None, species=None):
        grid = cascade.standing_wave_grid(wl.flags, wl.dt, dtype)
        return cascade.run(tabs, species, wl.dt, steps, None, None if main is not None else cap, app_cap,
                           dtype=dtype, seed=6, grid=grid, resample=rs, start=start, main=main)

    counts_a, _, _, main_a, _ = run(120, species=sp)
    counts_b1, _, _, main_b, _ = run(60, species=sp)
    path = checkpoint.save(tmp_path / "sw.npz", main_b, next_step=60, seed=6)
    del main_b
    torch.cuda.empty_cache()
    restored, meta = checkpoint.load(path)
    assert restored[0].x is not None
    counts_b2, _, _, main_c, _ = run(60, start=meta["next_step"], main=restored)
    print(f"{dtype_name}: counts after 120 steps {counts_a[-1].tolist()}, resumed {counts_b2[-1].tolist()}")
    assert counts_a[-1, 2] > 0  # photons above the filter's energy have appeared
    assert np.array_equal(counts_a[:61], counts_b1)
    assert np.array_equal(counts_a[60:], counts_b2)
    for s in range(3):
        a, c = main_a[s], main_c[s]
        assert a.count == c.count
        for name in ("px", "py", "pz", "x", "y", "z", "w", "tau", "id", "alive"):
            ta = getattr(a, name)
            if ta is None:
                continue
            tc = getattr(c, name)
            assert ta[: a.count].cpu().numpy().tobytes() == tc[: c.count].cpu().numpy().tobytes(), (s, name)
