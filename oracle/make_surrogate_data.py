"""Draws of the emission inverse CDF from the FP64 oracle, written as files for
training and evaluating the surrogate network -- TEST INFRASTRUCTURE (data
generation; nothing of the HIP library is used).

Each group shares one chi (log-uniform in the range, float32) and holds
`per_chi` raw uniforms k with r = (k + 1/2) / 2^32.  delta and 1 - delta come
from exact inversion of the FP64 cumulative spectrum (orc_sample_rad_grid).
Files in --out:
  x.npy  float32 [n, 2]  network inputs ln(chi)/ln(100), logit(r)/10
  t.npy  float32 [n]     target (logit(delta) - ln chi)/10
  chi.npy float32 [n], k.npy uint32 [n], ld.npy float64 [n] = ln delta,
  l1md.npy float64 [n] = ln(1 - delta)      (with --eval)
The input and output transforms are those of the library's default surrogate
configuration (qed_mlp_cfg_default).
"""
from __future__ import annotations

import argparse
import sys
import time
from pathlib import Path

import numpy as np
from numpy.lib.format import open_memmap

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
import synth  # noqa: E402

F1_SCALE = 1.0 / np.log(100.0)
F2_SCALE = 0.1
OUT_SCALE = 10.0


def draw_groups(g0: int, g1: int, per: int, seed: int, chi_range):
    chi, k = synth.surrogate_draws(np.arange(g0, g1), per, seed, chi_range)
    kk = k.astype(np.float64)
    r = (kk + 0.5) * 2.0**-32
    rc = ((2.0**32 - 1.0 - kk) + 0.5) * 2.0**-32
    d, omd = oracle.sample_rad_grid(chi.astype(np.float64), r, rc)
    return chi, k, r, rc, d, omd


def write(out: Path, n: int, per: int, seed: int, chi_range, evaluation: bool, chunk_groups: int):
    groups = n // per
    n = groups * per
    out.mkdir(parents=True, exist_ok=True)
    x = open_memmap(out / "x.npy", mode="w+", dtype=np.float32, shape=(n, 2))
    t = open_memmap(out / "t.npy", mode="w+", dtype=np.float32, shape=(n,))
    if evaluation:
        ev = {name: open_memmap(out / f"{name}.npy", mode="w+", dtype=dt, shape=(n,))
              for name, dt in (("chi", np.float32), ("k", np.uint32), ("ld", np.float64), ("l1md", np.float64))}
    t0 = time.time()
    for g0 in range(0, groups, chunk_groups):
        g1 = min(groups, g0 + chunk_groups)
        chi, k, r, rc, d, omd = draw_groups(g0, g1, per, seed, chi_range)
        a, b = g0 * per, g1 * per
        lc = np.log(chi.astype(np.float64))[:, None]
        ld, l1md = np.log(d), np.log(omd)
        x[a:b, 0] = np.broadcast_to(lc * F1_SCALE, r.shape).ravel()
        x[a:b, 1] = ((np.log(r) - np.log(rc)) * F2_SCALE).ravel()
        t[a:b] = ((ld - l1md - lc) / OUT_SCALE).ravel()
        if evaluation:
            ev["chi"][a:b] = np.repeat(chi, per)
            ev["k"][a:b] = k.ravel()
            ev["ld"][a:b] = ld.ravel()
            ev["l1md"][a:b] = l1md.ravel()
        print(f"  {b}/{n} draws, {time.time() - t0:.0f} s", flush=True)
    for arr in [x, t] + (list(ev.values()) if evaluation else []):
        arr.flush()
    return n


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=float, default=1e8)
    ap.add_argument("--per-chi", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--chi-min", type=float, default=1e-2)
    ap.add_argument("--chi-max", type=float, default=1e2)
    ap.add_argument("--eval", action="store_true", help="also write chi, k and the exact delta")
    ap.add_argument("--chunk-groups", type=int, default=4000)
    a = ap.parse_args(argv)
    oracle.lib()
    n = write(Path(a.out), int(a.n), a.per_chi, a.seed, (a.chi_min, a.chi_max), a.eval, a.chunk_groups)
    print(f"wrote {n} draws to {a.out}", flush=True)


if __name__ == "__main__":
    main()
