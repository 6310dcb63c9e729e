"""Writes synth/calibration.json: the global time steps of the synthetic
workloads, computed once with the FP64 oracle and then frozen.

* emission_static_b_dt: the mean time to the next emission of an electron with
  chi = 1 and gamma = 1e3 (the geometric centre of the gamma range),
  dt = 1 / W_rad(chi=1, gamma=1e3).
* crossed_field_dt: ten mean emission times of the leptons at t = 0,
  dt = 10 / <W_rad>, averaged over the first 2e5 electrons and 2e5 positrons.
* rotating_e_dt: the step for which the rotating-field cascade of 2000 seed
  electrons grows by about 200x in 20 steps (oracle.cascade.calibrate_rotating_dt).

Run: python -m oracle.calibrate_workloads [--cascade]
"""
from __future__ import annotations

import json
import sys

import numpy as np

import oracle
import synth


def emission_static_b_dt() -> float:
    gamma_ref = 1e3
    return gamma_ref / (oracle.ALPHA * oracle.rate_rad_reduced(1.0, definition=True))


def lepton_chi_crossed(sp) -> tuple[np.ndarray, np.ndarray]:
    # the field recipe fixes chi = |E| (gamma - n.p) exactly; recompute it from
    # the stored fields with the oracle's own chi for each particle
    g = np.sqrt(1.0 + np.einsum("ij,ij->i", sp.p, sp.p))
    chi = np.array([oracle.chi(sp.p[i], g[i], sp.fields[i, :3], sp.fields[i, 3:]) for i in range(sp.n)])
    return chi, g


def crossed_field_dt(n_sample: int = 200_000) -> float:
    full = 10_000_000
    wl = synth.crossed_field(full, indices=[np.arange(n_sample), np.arange(n_sample), np.arange(0)])
    rates = []
    for s in (0, 1):
        chi, g = lepton_chi_crossed(wl.species[s])
        rates.append(oracle.ALPHA / g * oracle.rate_rad_reduced_many(chi))
    mean_w = float(np.mean(np.concatenate(rates)))
    return 10.0 / mean_w


def main(argv):
    cal = synth.calibration()
    cal["emission_static_b_dt"] = emission_static_b_dt()
    cal["crossed_field_dt"] = crossed_field_dt()
    if "--cascade" in argv:
        from oracle.cascade import calibrate_rotating_dt
        cal["rotating_e_dt"] = calibrate_rotating_dt()
    synth._CAL.write_text(json.dumps(cal, indent=2, sort_keys=True) + "\n")
    print(json.dumps(cal, indent=2))


if __name__ == "__main__":
    main(sys.argv[1:])
