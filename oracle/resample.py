"""Ensemble resampling after the merge -- TEST INFRASTRUCTURE (part of the
oracle; only tests may use it).

Sec. 4.2 notes that the new particles can be filtered before they join the
ensemble (photons too soft ever to produce a pair) or thinned, and Sec. 5.1
keeps the number of macroparticles of its cascade in check with "global
leveling" resampling (citing Muraviev et al., Comput. Phys. Commun. 2021).
The paper gives no formulas; the reading implemented here:

* energy filter: a photon with |k| below e_min (in m_e c) is dropped; with
  e_min = 2 these are the photons below the pair threshold.  The comparison
  is kx^2 + ky^2 + kz^2 >= e_min^2 in FP64, summed left to right;
* global leveling of one species to a target count n_t: one threshold weight
  w_th for the whole species.  A particle with w >= w_th stays as it is; one
  with w < w_th stays with probability w / w_th and then carries the weight
  w_th, so that every particle's expected weight is unchanged.  w_th is the
  weight at which the expected number of particles, sum_i min(1, w_i / w_th),
  equals n_t;
* the draw of particle i is u = (x + 1/2) 2^-32 with x the first word of
  Philox4x32-10 keyed by the seed, counter (id_lo, id_hi, step, 0xFFFFFFFD);
  it stays when u < w_i / w_th (FP64);
* survivors keep their order.
"""
from __future__ import annotations

import numpy as np

from . import philox_stream

RESAMPLE_J = 0xFFFFFFFD  # reserved Philox counter word of the thinning draw


def leveling_threshold(w, n_target: int) -> float | None:
    """w_th with sum_i min(1, w_i / w_th) = n_target, or None when the species
    has no more than n_target particles.  Taken from the definition on the
    sorted weights: for w_th in [w_(k), w_(k+1)) the expected count is
    S_k / w_th + (N - k), S_k the sum of the k smallest weights, so the
    segment whose root S_k / (n_target - N + k) falls inside it gives w_th."""
    w = np.sort(np.asarray(w, dtype=np.float64))
    n = w.size
    if n_target <= 0 or n <= n_target:
        return None
    s = np.concatenate([[0.0], np.cumsum(w)])      # s[k] = sum of the k smallest
    k = np.arange(1, n + 1)
    denom = n_target - n + k
    ok = denom > 0
    wth = np.where(ok, s[k] / np.where(ok, denom, 1), np.inf)
    upper = np.concatenate([w[1:], [np.inf]])       # w_(k+1)
    inside = ok & (w[k - 1] <= wth) & (wth < upper)
    if not inside.any():                            # ties: the root sits on a weight value
        inside = ok & (np.abs(wth - w[k - 1]) <= 1e-15 * wth)
    return float(wth[np.argmax(inside)])


def keep_draws(seed: int, ids, step: int) -> np.ndarray:
    """u = (x + 1/2) 2^-32 of each particle's thinning draw."""
    x = philox_stream(seed, ids, step, RESAMPLE_J)[:, 0].astype(np.float64)
    return (x + 0.5) * 2.0 ** -32


def resample(p, w, ids, seed: int, step: int, n_target: int = 0, e_min: float = 0.0, photon: bool = False,
             w_th: float | None = None):
    """Survivors of one species: returns (keep mask, new weights, w_th, n_filtered).
    w_th may be given (to decide with another implementation's threshold);
    otherwise it is solved from the particles that pass the energy filter."""
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    keep = np.ones(w.size, dtype=bool)
    if photon and e_min > 0.0:
        keep = (p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1]) + p[:, 2] * p[:, 2] >= e_min * e_min
    n_filtered = int((~keep).sum())
    if w_th is None:
        w_th = leveling_threshold(w[keep], n_target)
    w_new = w.copy()
    if w_th is not None:
        u = keep_draws(seed, ids, step)
        low = w < w_th
        keep &= ~low | (u < w / w_th)
        w_new = np.where(low, w_th, w)
    return keep, w_new, w_th, n_filtered
