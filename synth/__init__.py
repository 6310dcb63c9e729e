"""Seeded synthetic ensembles shaped like the paper's workloads.

Every value is a pure function of (workload seed, stream, particle index)
through a counter-based 64-bit mixer, so any subsample can be regenerated
without the rest.  This module holds no part of the generator's arithmetic
(no chi, rate, spectrum or push): it only places momenta and fields so that a
target quantum parameter is met, following the recipes below.

Units: momenta in m_e c, fields in E_S (B in E_S/c), time in hbar/(m_e c^2).

Workloads (the paper's own test problem, a cascade in a rotating field at the
antinode of a standing wave, Sec. 5.1, is a PIC run; these stand in for its
per-particle generator load):

* ``emission_static_b``   1e5 electrons, gamma log-uniform in [1e2, 1e4],
  random directions, static B perpendicular to p with |B| = chi*/|p| and chi*
  log-uniform in [0.1, 10], E = 0.
* ``crossed_field``       1e7 particles (40% e-, 40% e+, 20% photons), energy
  log-uniform in [1e2, 1e4], crossed E perpendicular to B with |E| = |B| and
  chi* log-uniform in [0.1, 100] (|E| = chi*/(energy - n.p), n = E x B / |E|^2;
  directions with (energy - n.p)/energy < 1e-2 are redrawn).
* ``rotating_e``          1e6 seed electrons with gamma = 1e3 in a uniform
  rotating electric field E0 (0, cos wt, sin wt), B = 0.
* ``sampler``             (chi, 32-bit uniform) pairs for the inverse-CDF and
  surrogate samplers, chi log-uniform in a given range.
* ``static_b_sweep``      electrons and photons with chi* log-uniform in
  [1e-3, 1e3] in a static B perpendicular to the momentum (as the first).
* ``standing_wave``       the test problem of Sec. 5.1 itself: 2.5e5 seeds
  (half e-, half e+) at rest, uniform in a periodic cube of one wavelength
  (800 nm), in a plane standing circularly polarised wave of 6.25e15 V/m
  whose electric field rotates in the y-z plane, antinode at the centre; the
  field lives on 128 nodes along x; dt = 0.005 T.  ``standing_wave_nodes``
  gives the node values at time t.

Lengths are in hbar / (m_e c) (the reduced Compton wavelength) wherever
positions appear.
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np

ELECTRON, POSITRON, PHOTON = 0, 1, 2
_CAL = Path(__file__).resolve().parent / "calibration.json"

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_G = np.uint64(0x9E3779B97F4A7C15)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014)."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1) as a function of (seed, stream, index)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        base = _mix(np.uint64(seed) * _G + np.uint64(stream + 1) * _M2)
        z = _mix(idx * _G + base)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def bits32(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        base = _mix(np.uint64(seed) * _G + np.uint64(stream + 1) * _M2)
        z = _mix(idx * _G + base)
    return (z >> np.uint64(32)).astype(np.uint32)


def log_uniform(u: np.ndarray, lo: float, hi: float) -> np.ndarray:
    return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))


def direction(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Uniform on the unit sphere: cos(theta) = 2u - 1, phi = 2 pi v."""
    c = 2.0 * u - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    ph = 2.0 * np.pi * v
    return np.stack([s * np.cos(ph), s * np.sin(ph), c], axis=-1)


def perpendicular(n: np.ndarray, u: np.ndarray) -> np.ndarray:
    """A unit vector perpendicular to each unit vector n, at random angle 2 pi u."""
    a = np.zeros_like(n)
    use_y = np.abs(n[:, 0]) > 0.9
    a[~use_y, 0] = 1.0
    a[use_y, 1] = 1.0
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(n, e1)
    ph = 2.0 * np.pi * u
    return np.cos(ph)[:, None] * e1 + np.sin(ph)[:, None] * e2


def calibration() -> dict:
    return json.loads(_CAL.read_text()) if _CAL.exists() else {}


@dataclass
class Species:
    p: np.ndarray          # [n, 3] float64
    tau: np.ndarray        # [n] float64, optical depth still to be used up
    w: np.ndarray          # [n] float64 weights
    id: np.ndarray         # [n] uint64, unique over the ensemble
    fields: np.ndarray     # [n, 6] float64 (ex ey ez bx by bz) or [1, 6] shared
    index: np.ndarray      # [n] uint64, index within the species in the full workload
    x: np.ndarray | None = None  # [n, 3] float64 positions (workloads on a grid), else None

    @property
    def n(self) -> int:
        return int(self.id.size)


@dataclass
class Workload:
    name: str
    species: list          # [electrons, positrons, photons]
    dt: float
    flags: dict = field(default_factory=dict)
    recipe: str = ""

    @property
    def counts(self):
        return [s.n for s in self.species]


def _empty(shared_fields: bool = False) -> Species:
    return Species(np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0, np.uint64),
                   np.zeros((1 if shared_fields else 0, 6)), np.zeros(0, np.uint64))


def _select(n: int, indices) -> np.ndarray:
    if indices is None:
        return np.arange(n, dtype=np.uint64)
    idx = np.asarray(indices, dtype=np.uint64)
    assert idx.size == 0 or int(idx.max()) < n
    return idx


def _tau(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    return -np.log(uniform(seed, stream, idx))


# ----------------------------------------------------------------------------- workloads
def emission_static_b(n: int = 100_000, seed: int = 0, indices=None, chi_range=(0.1, 10.0),
                      gamma_range=(1e2, 1e4), dt: float | None = None) -> Workload:
    idx = _select(n, indices)
    g = log_uniform(uniform(seed, 0, idx), *gamma_range)
    d = direction(uniform(seed, 1, idx), uniform(seed, 2, idx))
    pm = np.sqrt(g * g - 1.0)
    p = d * pm[:, None]
    chi_t = log_uniform(uniform(seed, 3, idx), *chi_range)
    bdir = perpendicular(d, uniform(seed, 4, idx))
    B = bdir * (chi_t / pm)[:, None]
    f = np.concatenate([np.zeros_like(B), B], axis=1)
    e = Species(p, _tau(seed, 5, idx), np.ones(idx.size), idx.copy(), f, idx)
    if dt is None:
        dt = calibration().get("emission_static_b_dt", 1.0e5)
    return Workload("emission_static_b", [e, _empty(), _empty()], dt,
                    dict(emission=1, pair=0, push=0), "1e5 e-, static B perpendicular to p, chi* LU[0.1,10]")


def crossed_field(n: int = 10_000_000, seed: int = 0, indices=None, fractions=(0.4, 0.4, 0.2),
                  chi_range=(0.1, 100.0), energy_range=(1e2, 1e4), dt: float | None = None) -> Workload:
    counts = [int(round(n * fractions[0])), int(round(n * fractions[1]))]
    counts.append(n - counts[0] - counts[1])
    base = [0, counts[0], counts[0] + counts[1]]
    sp = []
    for s in range(3):
        idx = _select(counts[s], None if indices is None else indices[s])
        gidx = idx + np.uint64(base[s])          # index over the whole ensemble
        en = log_uniform(uniform(seed, 10, gidx), *energy_range)
        Ed = direction(uniform(seed, 11, gidx), uniform(seed, 12, gidx))
        Bd = perpendicular(Ed, uniform(seed, 13, gidx))
        nvec = np.cross(Ed, Bd)
        pm = np.sqrt(en * en - 1.0) if s < 2 else en
        d = np.zeros((idx.size, 3))
        todo = np.arange(idx.size)
        for attempt in range(16):  # redraw directions with (energy - n.p)/energy < 1e-2
            g = gidx[todo]
            cand = direction(uniform(seed, 20 + 2 * attempt, g), uniform(seed, 21 + 2 * attempt, g))
            good = (en[todo] - pm[todo] * np.einsum("ij,ij->i", nvec[todo], cand)) / en[todo] >= 1e-2
            d[todo[good]] = cand[good]
            todo = todo[~good]
            if todo.size == 0:
                break
        assert todo.size == 0
        p = d * pm[:, None]
        chi_t = log_uniform(uniform(seed, 14, gidx), *chi_range)
        Em = chi_t / (en - np.einsum("ij,ij->i", nvec, p))
        f = np.concatenate([Ed * Em[:, None], Bd * Em[:, None]], axis=1)
        sp.append(Species(p, _tau(seed, 15, gidx), np.ones(idx.size), gidx.copy(), f, idx))
    if dt is None:
        dt = calibration().get("crossed_field_dt", 1.0e5)
    return Workload("crossed_field", sp, dt, dict(emission=1, pair=1, push=1),
                    "1e7: 40% e-, 40% e+, 20% photons; crossed E, B with |E|=|B|; chi* LU[0.1,100]")


def rotating_e(n: int = 1_000_000, seed: int = 0, indices=None, gamma: float = 1e3,
               e0: float = 0.05, dt: float | None = None) -> Workload:
    idx = _select(n, indices)
    d = direction(uniform(seed, 30, idx), uniform(seed, 31, idx))
    p = d * np.sqrt(gamma * gamma - 1.0)
    f = np.zeros((1, 6))
    f[0, 1] = e0
    if dt is None:
        dt = calibration().get("rotating_e_dt", 2.0e4)
    return Workload("rotating_e", [Species(p, _tau(seed, 32, idx), np.ones(idx.size), idx.copy(), f, idx),
                                   _empty(True), _empty(True)], dt,
                    dict(emission=1, pair=1, push=1, e0=e0, omega_dt=2 * np.pi * 0.005),
                    "1e6 e-, gamma=1e3, E0 (0, cos wt, sin wt), B = 0")


def rotating_field(e0: float, omega_dt: float, step: int) -> np.ndarray:
    """The rotating field at step n (held constant over the step)."""
    f = np.zeros((1, 6))
    f[0, 1] = e0 * np.cos(omega_dt * step)
    f[0, 2] = e0 * np.sin(omega_dt * step)
    return f


def sampler(n: int, seed: int = 0, chi_range=(1e-2, 1e2), indices=None):
    """(chi, raw 32-bit uniform) pairs; r = (k + 1/2) / 2^32."""
    idx = _select(n, indices)
    chi = log_uniform(uniform(seed, 40, idx), *chi_range)
    return chi, bits32(seed, 41, idx)


def surrogate_draws(groups, per_group: int, seed: int = 0, chi_range=(1e-2, 1e2)):
    """Inputs of the surrogate's training and evaluation draws: for each group
    index g, chi_g log-uniform in chi_range (rounded to float32, the precision
    the sampler receives) and per_group raw 32-bit uniforms k[g, j]."""
    g = np.asarray(groups, dtype=np.uint64)
    chi = log_uniform(uniform(seed, 42, g), *chi_range).astype(np.float32)
    j = (g[:, None] * np.uint64(per_group) + np.arange(per_group, dtype=np.uint64)[None, :]).ravel()
    return chi, bits32(seed, 43, j).reshape(g.size, per_group)


def static_b_sweep(n: int = 200_000_000, seed: int = 0, indices=None, chi_range=(1e-3, 1e3),
                   energy_range=(1e2, 1e4)) -> Workload:
    half = n // 2
    sp = []
    for s, base in ((ELECTRON, 0), (PHOTON, half)):
        idx = _select(half, None if indices is None else indices[s])
        gidx = idx + np.uint64(base)
        en = log_uniform(uniform(seed, 50, gidx), *energy_range)
        d = direction(uniform(seed, 51, gidx), uniform(seed, 52, gidx))
        pm = np.sqrt(en * en - 1.0) if s == ELECTRON else en
        chi_t = log_uniform(uniform(seed, 53, gidx), *chi_range)
        B = perpendicular(d, uniform(seed, 54, gidx)) * (chi_t / pm)[:, None]
        f = np.concatenate([np.zeros_like(B), B], axis=1)
        sp.append(Species(d * pm[:, None], _tau(seed, 55, gidx), np.ones(idx.size), gidx.copy(), f, idx))
    return Workload("static_b_sweep", [sp[0], _empty(), sp[1]], calibration().get("emission_static_b_dt", 1e5),
                    dict(emission=1, pair=1, push=0), "1e8 e- + 1e8 photons, chi* LU[1e-3,1e3], static B")


# ----------------------------------------------------------------------------- the standing-wave test problem
# CODATA 2018: reduced Compton wavelength of the electron (m) and the Schwinger
# field m_e^2 c^3 / (e hbar) (V/m)
COMPTON_BAR_M = 3.8615926796e-13
SCHWINGER_V_PER_M = 1.32328585e18


def standing_wave_params(wavelength_m: float = 800e-9, amplitude_v_per_m: float = 6.25e15, nx: int = 128,
                         dt_over_period: float = 0.005) -> dict:
    """Geometry and field of the Sec. 5.1 test problem in code units: the box
    is the cube [-L/2, L/2)^3 of one wavelength L, the electric antinode at the
    centre; omega = k = 2 pi / L and the period T = L (c = 1)."""
    length = wavelength_m / COMPTON_BAR_M
    k = 2.0 * np.pi / length
    return dict(length=length, x0=-0.5 * length, nx=int(nx), e0=amplitude_v_per_m / SCHWINGER_V_PER_M, k=k, omega=k,
                xc=0.0, period=length, dt=dt_over_period * length)


def standing_wave_nodes(nx: int, x0: float, length: float, e0: float, k: float, omega: float, xc: float,
                        t: float) -> np.ndarray:
    """[nx, 6] (ex ey ez bx by bz) at x_i = x0 + i length / nx and time t:
    E = e0 cos(k (x - xc)) (0, cos wt, sin wt), B = e0 sin(k (x - xc)) (0, cos wt, sin wt)."""
    x = x0 + np.arange(nx, dtype=np.float64) * (length / nx)
    phi = k * (x - xc)
    ce, sb = e0 * np.cos(phi), e0 * np.sin(phi)
    ct, st = np.cos(omega * t), np.sin(omega * t)
    out = np.zeros((nx, 6))
    out[:, 1], out[:, 2] = ce * ct, ce * st
    out[:, 4], out[:, 5] = sb * ct, sb * st
    return out


def standing_wave(n: int = 250_000, seed: int = 0, indices=None, gamma: float | None = None,
                  **params) -> Workload:
    """n seeds, the first half electrons and the rest positrons, uniform in the
    box; at rest, or (gamma given) with that gamma in random directions.
    indices: a subset of [0, n) (each index keeps its species and position)."""
    prm = standing_wave_params(**params)
    idx = _select(n, indices)
    half = n // 2
    length = prm["length"]
    x = np.stack([(uniform(seed, 50 + a, idx) - 0.5) * length for a in range(3)], axis=1)
    if gamma is None:
        p = np.zeros((idx.size, 3))
    else:
        p = direction(uniform(seed, 53, idx), uniform(seed, 54, idx)) * np.sqrt(gamma * gamma - 1.0)
    tau = _tau(seed, 55, idx)
    sp = []
    for s, sel in enumerate((idx < half, idx >= half)):
        sp.append(Species(p[sel], tau[sel], np.ones(int(sel.sum())), idx[sel].copy(), np.zeros((1, 6)),
                          idx[sel], x[sel]))
    ph = _empty(True)
    ph.x = np.zeros((0, 3))
    sp.append(ph)
    flags = dict(emission=1, pair=1, push=1, **prm)
    return Workload("standing_wave", sp, prm["dt"], flags,
                    f"{n} seeds (e-, e+) {'at rest' if gamma is None else f'gamma {gamma:g}'} in a periodic cube "
                    "of one wavelength; standing CP wave 6.25e15 V/m on 128 nodes; dt = 0.005 T")
