"""Given fields on a grid -- TEST INFRASTRUCTURE (part of the oracle; only
tests may use it).

The paper's test problem (Sec. 5.1) is a plane standing circularly polarised
wave in a periodic box; the fields are homogeneous across the wave axis x, so
one periodic line of nodes along x holds them, and the QED step sees each
particle's field interpolated at its position.  The paper names neither the
interpolation nor the time at which the given field is taken.  The reading
implemented here:

* nodes x_i = x0 + i dx, dx = length / nx, periodic with period `length`, all
  six components at every node;
* a particle's field is the linear interpolation between the two nodes around
  its x (periodic), in FP64, rounded once to the dtype of the ensemble;
* before that, every coordinate is wrapped into the periodic box and stored
  (rounded to the dtype); the field is taken at the stored coordinate;
* the field of global step k is the one at t = k dt, held over the step
  (fields are constant within the step, as in the step itself).

Arithmetic follows the order below exactly (no fused operations), so that an
implementation doing the same FP64 operations agrees bit for bit.
"""
from __future__ import annotations

import numpy as np


def standing_wave_nodes(nx: int, x0: float, length: float, e0: float, k: float, omega: float, xc: float,
                        t: float) -> np.ndarray:
    """[nx, 6] (ex ey ez bx by bz) of the standing circularly polarised wave
    (Sec. 5.1) at time t: the sum of two circularly polarised waves of
    amplitude e0 / 2 running along +x and -x, electric field rotating in the
    y-z plane, antinode at xc:
        E = e0 cos(k (x - xc)) (0, cos wt, sin wt),
        B = e0 sin(k (x - xc)) (0, cos wt, sin wt)."""
    x = x0 + np.arange(nx, dtype=np.float64) * (length / nx)
    phi = k * (x - xc)
    ce, sb = e0 * np.cos(phi), e0 * np.sin(phi)
    ct, st = np.cos(omega * t), np.sin(omega * t)
    out = np.zeros((nx, 6))
    out[:, 1], out[:, 2] = ce * ct, ce * st
    out[:, 4], out[:, 5] = sb * ct, sb * st
    return out


def wrap(x, lo: float, length: float) -> np.ndarray:
    """x' = x - floor((x - lo) / length) length in [lo, lo + length) (FP64;
    the reciprocal 1 / length is rounded once; a result pushed onto the wrong
    side of an edge by rounding is moved back by one period)."""
    x = np.asarray(x, dtype=np.float64)
    if not length > 0.0:
        return x.copy()
    r = 1.0 / length
    hi = lo + length
    s = np.floor((x - lo) * r)
    w = x - s * length
    return np.where(w < lo, w + length, np.where(w >= hi, w - length, w))


def interpolate(nodes, x0: float, length: float, x) -> np.ndarray:
    """[n, 6] FP64 linear interpolation of the periodic node values at x."""
    g = np.asarray(nodes, dtype=np.float64)
    nx = g.shape[0]
    nxd = float(nx)
    u = (np.asarray(x, dtype=np.float64) - x0) * (nxd / length)
    q = np.floor(u)
    f = u - q
    i = q - nxd * np.floor(q / nxd)
    i = np.clip(i, 0.0, nxd - 1.0).astype(np.int64)
    j = np.where(i + 1 == nx, 0, i + 1)
    return (1.0 - f)[:, None] * g[i] + f[:, None] * g[j]


def gather(x, nodes, x0: float, length: float, box_lo, box_len, dtype=np.float64):
    """Positions [n, 3] (values of `dtype`) -> (wrapped positions [n, 3] and
    fields [n, 6], both rounded to dtype, as float64 arrays)."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    xs = np.empty_like(x)
    for a in range(3):
        w = wrap(x[:, a], box_lo[a], box_len[a]) if box_len[a] > 0.0 else x[:, a]
        xs[:, a] = np.asarray(w, dtype=dtype).astype(np.float64)
    g = np.asarray(nodes, dtype=dtype).astype(np.float64)
    f = interpolate(g, x0, length, xs[:, 0])
    return xs, f.astype(dtype).astype(np.float64)
