"""Rotating-field cascade driven by the oracle's step and merge -- TEST
INFRASTRUCTURE.

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


def run(wl: synth.Workload, steps: int, seed: int = 0, dt: float | None = None, push: bool = True,
        on_step=None) -> np.ndarray:
    """Counts [steps + 1, 3] of e-, e+, photons after each merged step."""
    dt = wl.dt if dt is None else dt
    e0, wdt = wl.flags["e0"], wl.flags["omega_dt"]
    main = [oracle.Store.from_arrays(sp.p, sp.w, sp.tau, sp.id, capacity=max(sp.n, 1)) for sp in wl.species]
    counts = [[m.count for m in main]]
    for k in range(steps):
        f = synth.rotating_field(e0, wdt, k)
        n = sum(m.count for m in main)
        cap = max(1024, 8 * n)
        while True:
            app = [oracle.Store(cap) for _ in range(3)]
            snap = [(m.state[:m.count].copy(), m.alive[:m.count].copy(), m.nev[:m.count].copy()) for m in main]
            rc, st = oracle.step(main, [f, f, f], app, dt, seed, k, emission=1, pair=1, push=push)
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
        counts.append([m.count for m in main])
        if on_step:
            on_step(k, counts[-1])
    return np.array(counts, dtype=np.int64)


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
