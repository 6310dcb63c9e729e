"""Cascades driven by the oracle's step and merge -- TEST INFRASTRUCTURE.

``run``: the rotating-field cascade.  ``run_grid``: the standing-wave test
problem with its fields on a grid (oracle.grid) and optional resampling
(oracle.resample).

Each global step holds the field of synth.rotating_field fixed (the electric
field at the antinode of a rotating standing wave, Sec. 5.1), runs one step of
every particle and its descendants (Algorithms 1 and 2) and merges the new
particles into the ensemble.  The growth rate of the cascade, N(t) ~ e^{Gamma t}
(Sec. 5.2), is the least-squares slope of ln N against time.
"""
from __future__ import annotations

import numpy as np

import oracle
import synth

from . import grid
from . import resample as ors


def _grow(store: oracle.Store, capacity: int) -> oracle.Store:
    if capacity <= store.capacity:
        return store
    s = oracle.Store(capacity)
    n = store.count
    s.state[:n] = store.state[:n]
    s.id[:n] = store.id[:n]
    s.root[:n] = store.root[:n]
    s.alive[:n] = store.alive[:n]
    s.nev[:n] = store.nev[:n]
    s.count = n
    return s


def _step_merge(main: list, fields: list, dt: float, seed: int, k: int, push: bool, positions: bool) -> list:
    """One step of every particle and its descendants, then the merge of the
    new particles into the ensemble (append stores grown until they suffice)."""
    n = sum(m.count for m in main)
    cap = max(1024, 8 * n)
    while True:
        app = [oracle.Store(cap) for _ in range(3)]
        snap = [(m.state[:m.count].copy(), m.alive[:m.count].copy(), m.nev[:m.count].copy()) for m in main]
        rc, st = oracle.step(main, fields, app, dt, seed, k, emission=1, pair=1, push=push, positions=positions)
        if rc == 0:
            break
        if rc != 2:
            raise RuntimeError(f"oracle step failed ({rc})")
        for m, (s, a, v) in zip(main, snap):  # undo and retry with larger append stores
            m.state[:m.count], m.alive[:m.count], m.nev[:m.count] = s, a, v
        cap *= 4
    main = [_grow(m, m.count + a.count) for m, a in zip(main, app)]
    if oracle.merge(main, app) != 0:
        raise RuntimeError("oracle merge failed")
    return main


def run(wl: synth.Workload, steps: int, seed: int = 0, dt: float | None = None, push: bool = True,
        on_step=None) -> np.ndarray:
    """Counts [steps + 1, 3] of e-, e+, photons after each merged step."""
    dt = wl.dt if dt is None else dt
    e0, wdt = wl.flags["e0"], wl.flags["omega_dt"]
    main = [oracle.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, capacity=max(sp.n, 1)) for sp in wl.species]
    counts = [[m.count for m in main]]
    for k in range(steps):
        f = synth.rotating_field(e0, wdt, k)
        main = _step_merge(main, [f, f, f], dt, seed, k, push, False)
        counts.append([m.count for m in main])
        if on_step:
            on_step(k, counts[-1])
    return np.array(counts, dtype=np.int64)


def _resample(main: list, seed: int, k: int, target, e_min: float) -> None:
    """Photon filter and global leveling of every species (oracle.resample),
    compacting the stores in place; weights are kept in FP32, as the
    ensemble stores them."""
    for s, m in enumerate(main):
        n = m.count
        keep, wn, _, _ = ors.resample(m.p, m.w, m.id[:n], seed, k, n_target=int(target[s]), e_min=e_min,
                                      photon=s == 2)
        idx = np.nonzero(keep)[0]
        m.state[:idx.size] = m.state[idx]
        m.state[:idx.size, 6] = wn[idx].astype(np.float32)
        m.id[:idx.size] = m.id[idx]
        m.root[:idx.size] = m.root[idx]
        m.alive[:idx.size] = m.alive[idx]
        m.nev[:idx.size] = m.nev[idx]
        m.count = int(idx.size)


def run_grid(wl: synth.Workload, steps: int, seed: int = 0, nodes_of_step=None, resample=None, on_step=None):
    """A cascade with given grid fields (the standing-wave test problem of
    Sec. 5.1): in step k the grid holds the field at t = k dt
    (nodes_of_step(k), by default the standing wave of wl.flags), every
    position is wrapped into the periodic box and sees the grid's field there
    (oracle.grid), then every particle and its descendants take the step with
    push and positions on, the new particles are merged, and, if `resample`
    holds (target, photon_energy_min), the ensemble is resampled with the
    cascade's seed and the step index.  Returns (counts [steps + 1, 3], the
    final stores)."""
    prm = wl.flags
    L, x0 = prm["length"], prm["x0"]
    lo, ln = (x0, x0, x0), (L, L, L)
    if nodes_of_step is None:
        def nodes_of_step(k):
            return grid.standing_wave_nodes(prm["nx"], x0, L, prm["e0"], prm["k"], prm["omega"], prm["xc"], k * wl.dt)
    main = [oracle.Store.from_arrays(sp.p, np.asarray(sp.w, np.float32), sp.tau, sp.id, x=sp.x,
                                     capacity=max(sp.n, 1)) for sp in wl.species]
    counts = [[m.count for m in main]]
    for k in range(steps):
        nodes = nodes_of_step(k)
        fields = []
        for m in main:
            xs, f = grid.gather(m.x, nodes, x0, L, lo, ln)
            m.state[:m.count, 3:6] = xs
            fields.append(f)
        main = _step_merge(main, fields, wl.dt, seed, k, True, True)
        if resample is not None:
            _resample(main, seed, k, resample[0], resample[1])
        counts.append([m.count for m in main])
        if on_step:
            on_step(k, counts[-1])
    return np.array(counts, dtype=np.int64), main


def growth_rate(counts: np.ndarray, dt: float, first: int = 0) -> float:
    """Gamma of N(t) ~ e^{Gamma t}: least-squares slope of ln N_total over steps >= first."""
    n = counts.sum(axis=1).astype(np.float64)
    t = np.arange(n.size) * dt
    return float(np.polyfit(t[first:], np.log(n[first:]), 1)[0])


def calibrate_rotating_dt(n_seeds: int = 2000, steps: int = 20, target: float = 200.0) -> float:
    """dt for which the cascade of n_seeds electrons grows by `target` in `steps` steps (bisection in ln dt)."""
    lo, hi = 2e3, 2e5
    for _ in range(12):
        dt = float(np.sqrt(lo * hi))
        wl = synth.rotating_e(1_000_000, indices=np.arange(n_seeds), dt=dt)
        c = run(wl, steps, dt=dt)
        g = c[-1].sum() / c[0].sum()
        print(f"  dt {dt:.4g}: N({steps})/N(0) = {g:.1f}", flush=True)
        if abs(np.log(g / target)) < 0.05:
            break
        if g > target:
            hi = dt
        else:
            lo = dt
    return dt
