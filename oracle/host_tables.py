"""Node values of the host-CPU baseline's tables from the oracle -- TEST
INFRASTRUCTURE (used by the tests and by the benchmark's CPU leg only).

The baseline (host_simd) reads the reduced rates W * energy / alpha on a
uniform grid in ln chi, and the inverse spectra on grids in (ln chi, logit r):
for emission q = logit(delta) - ln chi, for pairs q = logit(xi) (delta and xi
the fractions the oracle's inversion returns at r).  This module only
evaluates the oracle at those nodes.
"""
from __future__ import annotations

import ctypes as C
from concurrent.futures import ThreadPoolExecutor
from functools import lru_cache

import numpy as np

import oracle

RATE_CHI = (1e-4, 1e4)
RATE_NODES = 2048
RAD_CHI, RAD_ROWS = (1e-4, 1e4), 256
PAIR_CHI, PAIR_ROWS = (1e-2, 1e4), 128
LOGIT_R = (-23.0, 23.0)   # every r = (k + 1/2) 2^-32 has |logit r| < 22.2
RAD_COLS, PAIR_COLS = 512, 512


def _grid(lo, hi, n):
    h = (hi - lo) / (n - 1)
    return lo + h * np.arange(n), h


def _sigmoid_pair(x):
    r = 1.0 / (1.0 + np.exp(-x))
    rc = 1.0 / (1.0 + np.exp(x))
    return r, rc


@lru_cache(maxsize=1)
def nodes(threads: int = 8) -> dict:
    s, hs = _grid(np.log(RATE_CHI[0]), np.log(RATE_CHI[1]), RATE_NODES)
    chi = np.exp(s)
    lnr = np.stack([np.log(np.maximum(oracle.rate_rad_reduced_many(chi), 1e-300)),
                    np.log(np.maximum(oracle.rate_pair_reduced_many(chi), 1e-300))])
    out = {"nr": RATE_NODES, "s0": float(s[0]), "hs": float(hs), "lnr": lnr,
           "qs0": [0.0, 0.0], "qhs": [0.0, 0.0], "qx0": [0.0, 0.0], "qhx": [0.0, 0.0], "q": [None, None]}
    # emission: q = logit(delta) - ln chi on the (ln chi, logit r) nodes
    sr, hsr = _grid(np.log(RAD_CHI[0]), np.log(RAD_CHI[1]), RAD_ROWS)
    xr, hxr = _grid(LOGIT_R[0], LOGIT_R[1], RAD_COLS)
    r, rc = _sigmoid_pair(xr)
    chi_r = np.exp(sr)
    d, od = oracle.sample_rad_grid(chi_r, np.tile(r, (RAD_ROWS, 1)), np.tile(rc, (RAD_ROWS, 1)))
    out["q"][0] = np.log(d) - np.log(od) - sr[:, None]
    out["qs0"][0], out["qhs"][0], out["qx0"][0], out["qhx"][0] = float(sr[0]), float(hsr), float(xr[0]), float(hxr)
    # pairs: q = logit(xi)
    sp, hsp = _grid(np.log(PAIR_CHI[0]), np.log(PAIR_CHI[1]), PAIR_ROWS)
    xp, hxp = _grid(LOGIT_R[0], LOGIT_R[1], PAIR_COLS)
    r, rc = _sigmoid_pair(xp)
    chi_p = np.exp(sp)

    def row(i):
        q = np.empty(PAIR_COLS)
        d, o = C.c_double(), C.c_double()
        for j in range(PAIR_COLS):
            oracle.lib().orc_sample_pair_r(chi_p[i], r[j], rc[j], 0, C.byref(d), C.byref(o))  # xi and 1 - xi
            q[j] = np.log(d.value) - np.log(o.value)
        return q

    with ThreadPoolExecutor(threads) as ex:
        out["q"][1] = np.stack(list(ex.map(row, range(PAIR_ROWS))))
    out["qs0"][1], out["qhs"][1], out["qx0"][1], out["qhx"][1] = float(sp[0]), float(hsp), float(xp[0]), float(hxp)
    return out

