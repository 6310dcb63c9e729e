"""Multi-step cascade on the device: qed_step and qed_merge repeated over
global steps in a field that is constant within each step (Algorithm 2 per
step, the new particles merged into the ensemble after it).  The driver only
moves pointers and counts; every particle operation runs in libsfqed.

The field of step k comes from a caller's function (for the rotating-field
cascade: the electric field at the antinode of a rotating standing wave,
Sec. 5.1) or from a grid interpolated at the particles' positions (the
standing-wave test problem itself, `standing_wave_grid`), and the growth rate of N(t) ~ e^{Gamma t} is the figure of merit
(Sec. 5.2).  With resampling (global leveling after every merge, as the paper
runs its cascade) the number of macroparticles stays bounded and the growth
shows in the total weight instead.
"""
from __future__ import annotations

import time

import numpy as np

from . import (AppendBuffer, Fields, Store, field_buffers, gather_fields, merge, resample as resample_ensemble,
               resample_cfg, step, step_cfg, step_merged)


def run(tables, species, dt: float, steps: int, field_of_step, capacity, app_capacity, dtype=None, seed: int = 0,
        cfg=None, on_step=None, stream=None, resample=None, grid=None, merged=True, start: int = 0, main=None):
    """species: [(p [n, 3], w [n], tau [n], id [n])] or, with positions,
    [(p, w, tau, id, x [n, 3])] for e-, e+, photons;
    field_of_step(k): the [1, 6] field (ex ey ez bx by bz) shared by all
    particles during step k; or grid = (Grid1d, box, fill) for fields on a
    grid: fill(k, grid) sets the nodes of step k, then every position is
    wrapped into the box and the grid is interpolated at it (gather_fields);
    resample: None, or the keyword arguments of resample_cfg
    (photon_energy_min, target) applied after every merge, with the cascade's
    seed and the step index; merged: one qed_step_merged call per step (else
    qed_step then qed_merge; the results are identical); start: index of the
    first global step (a run restored from a checkpoint saved after step
    start - 1 continues with start); main: device stores to continue from
    (checkpoint.load gives them; species, capacity and dtype are then taken
    from them).  Returns (counts
    [steps + 1, 3], per-step stats, seconds per step, the final device stores,
    total weight [steps + 1, 3])."""
    import torch
    dtype = main[0].dtype if main is not None else (dtype or torch.float32)
    positions = main[0].x is not None if main is not None else len(species[0]) > 4
    if grid is not None and not positions:
        raise ValueError("fields on a grid need particle positions")
    cfg = cfg if cfg is not None else step_cfg(push=True, nev=False)
    if main is None:
        main = [Store.from_arrays(sp[0], sp[1], sp[2], sp[3], dtype=dtype, photon=s == 2, capacity=capacity[s],
                                  x=sp[4] if positions else None)
                for s, sp in enumerate(species)]
        for m in main:
            m.nev = None
    capacity = [m.capacity for m in main]
    app = [AppendBuffer(app_capacity[s], dtype, positions=positions) for s in range(3)]
    fbuf = [field_buffers(capacity[s], dtype) for s in range(3)] if grid is not None else None
    def weight():
        return [float(m.w[:m.count].double().sum()) if m.count else 0.0 for m in main]

    counts = [[m.count for m in main]]
    weights = [weight()]
    stats, secs = [], []
    for k in range(start, start + steps):
        t0 = time.perf_counter()
        if grid is not None:
            g, box, fill = grid
            fill(k, g)
            gather_fields(main, g, box, fbuf, stream=stream)
            fields = fbuf
        else:
            f = Fields.from_array(np.asarray(field_of_step(k), dtype=np.float64).reshape(1, 6), dtype)
            fields = [f, f, f]
            t0 = time.perf_counter()
        if merged:
            rc, st = step_merged(tables, main, fields, app, dt, seed, k, cfg, stream=stream, check=False)
        else:
            rc, st = step(tables, main, fields, app, dt, seed, k, cfg, stream=stream, check=False)
        if rc != 0:
            raise RuntimeError(f"cascade step {k}: status {rc}, required capacity {list(st.required_capacity)}")
        if not merged:
            merge(main, fields, app, stream=stream)
        if resample is not None:
            resample_ensemble(main, fields, resample_cfg(seed=seed, step=k, **resample), stream=stream)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        counts.append([m.count for m in main])
        weights.append(weight())
        stats.append(st)
        if on_step:
            on_step(k, counts[-1], st, secs[-1])
    return np.array(counts, dtype=np.int64), stats, secs, main, np.array(weights)


def growth_rate(counts: np.ndarray, dt: float, first: int = 0) -> float:
    """Least-squares slope of ln N_total against time over steps >= first."""
    n = counts.sum(axis=1).astype(np.float64)
    t = np.arange(n.size) * dt
    return float(np.polyfit(t[first:], np.log(n[first:]), 1)[0])


def standing_wave_grid(flags: dict, dt: float, dtype=None, stream=None):
    """(Grid1d, box, fill) for run(): the standing circularly polarised wave of
    the test problem (flags as synth.standing_wave_params gives them) filled
    on the device at t = k dt for step k, in a periodic cube of one
    wavelength."""
    from . import Grid1d, box, standing_wave
    L, x0 = flags["length"], flags["x0"]
    g = Grid1d(flags["nx"], x0, L, dtype)

    def fill(k, grid):
        standing_wave(grid, flags["e0"], flags["k"], flags["omega"], flags["xc"], k * dt, stream=stream)
    return g, box((x0, x0, x0), (L, L, L)), fill
