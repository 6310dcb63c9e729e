"""Pins of the oracle's field stage for the standing-wave test problem
(Sec. 5.1): the wave against Maxwell's equations and its closed-form special
points, the interpolation against numpy's periodic np.interp and exactness
at nodes and for linear data, the wrap against its defining properties."""
import numpy as np
import pytest

import synth
from oracle import grid


def test_standing_wave_special_points_and_invariants():
    prm = synth.standing_wave_params()
    L, e0 = prm["length"], prm["e0"]
    nx = 128
    for t in (0.0, 0.3 * L, L / 4):
        g = grid.standing_wave_nodes(nx, prm["x0"], L, e0, prm["k"], prm["omega"], 0.0, t)
        E, B = g[:, :3], g[:, 3:]
        # |E|^2 + |B|^2 = e0^2 at every node; E parallel to B; no x component
        assert np.allclose((E * E).sum(1) + (B * B).sum(1), e0 * e0, rtol=1e-14)
        assert np.allclose(np.cross(E, B), 0.0, atol=1e-15 * e0 * e0)
        assert np.all(E[:, 0] == 0.0) and np.all(B[:, 0] == 0.0)
        # node 64 is the centre (antinode of E, node of B); node 96 is a quarter wave away
        assert np.linalg.norm(E[64]) == pytest.approx(e0, rel=1e-15) and np.linalg.norm(B[64]) <= 1e-15 * e0
        assert np.linalg.norm(B[96]) == pytest.approx(e0, rel=1e-15) and np.linalg.norm(E[96]) <= 1e-15 * e0
    # the field rotates in the y-z plane: a quarter period turns E from +y to +z
    g0 = grid.standing_wave_nodes(nx, prm["x0"], L, e0, prm["k"], prm["omega"], 0.0, 0.0)
    g1 = grid.standing_wave_nodes(nx, prm["x0"], L, e0, prm["k"], prm["omega"], 0.0, prm["period"] / 4)
    assert g0[64, 1] == pytest.approx(e0) and g1[64, 2] == pytest.approx(e0) and abs(g1[64, 1]) < 1e-15


def test_standing_wave_solves_maxwell():
    # dB/dt = -curl E and dE/dt = curl B (c = 1) for fields of x and t alone:
    # dBy/dt = dEz/dx, dBz/dt = -dEy/dx, dEy/dt = -dBz/dx, dEz/dt = dBy/dx
    prm = synth.standing_wave_params()
    L, e0, k, w = prm["length"], prm["e0"], prm["k"], prm["omega"]
    x = np.linspace(-0.5 * L, 0.5 * L, 37)
    h = 1e-4 * L
    def f(xx, t):
        return np.array([grid.standing_wave_nodes(1, xi, L, e0, k, w, 0.0, t)[0] for xi in xx])
    for t in (0.0, 0.17 * L, 0.61 * L):
        dt_ = (f(x, t + h) - f(x, t - h)) / (2 * h)
        dx_ = (f(x + h, t) - f(x - h, t)) / (2 * h)
        scale = e0 * k
        assert np.allclose(dt_[:, 4], dx_[:, 2], atol=1e-6 * scale)
        assert np.allclose(dt_[:, 5], -dx_[:, 1], atol=1e-6 * scale)
        assert np.allclose(dt_[:, 1], -dx_[:, 5], atol=1e-6 * scale)
        assert np.allclose(dt_[:, 2], dx_[:, 4], atol=1e-6 * scale)
    # a standing wave: the two running components carry equal and opposite flux
    # (E x B averages to zero over a period at every x)
    ts = np.linspace(0, prm["period"], 64, endpoint=False)
    flux = np.mean([np.cross(f(x, t)[:, :3], f(x, t)[:, 3:])[:, 0] for t in ts], axis=0)
    assert np.allclose(flux, 0.0, atol=1e-15 * e0 * e0)


def test_synth_nodes_equal_oracle_nodes():
    prm = synth.standing_wave_params()
    for t in (0.0, 123.0 * prm["dt"]):
        a = synth.standing_wave_nodes(128, prm["x0"], prm["length"], prm["e0"], prm["k"], prm["omega"], 0.0, t)
        b = grid.standing_wave_nodes(128, prm["x0"], prm["length"], prm["e0"], prm["k"], prm["omega"], 0.0, t)
        assert np.array_equal(a, b)


def test_interpolation_against_np_interp():
    rng = np.random.default_rng(0)
    nx, x0, L = 128, -3.7, 11.3
    nodes = rng.normal(size=(nx, 6))
    xs = x0 + rng.uniform(-2.0, 3.0, 5000) * L           # several periods either side
    got = grid.interpolate(nodes, x0, L, xs)
    xp = x0 + np.arange(nx) * (L / nx)
    for c in range(6):
        ref = np.interp(xs, xp, nodes[:, c], period=L)
        assert np.allclose(got[:, c], ref, rtol=0, atol=1e-12)


def test_interpolation_exact_cases():
    # power-of-two geometry: node positions and shifts by whole periods are exact
    nx, x0, L = 16, -8.0, 16.0
    rng = np.random.default_rng(1)
    nodes = rng.normal(size=(nx, 6))
    xn = x0 + np.arange(nx) * 1.0
    assert np.array_equal(grid.interpolate(nodes, x0, L, xn), nodes)
    xs = np.round(rng.uniform(x0, x0 + L, 1000) * 2.0 ** 20) * 2.0 ** -20   # shifts by 16 m stay exact
    a = grid.interpolate(nodes, x0, L, xs)
    for m in (-3, 1, 5):
        assert np.array_equal(grid.interpolate(nodes, x0, L, xs + m * L), a)
    # linear data away from the wrap-around cell is reproduced
    lin = np.tile((2.0 + 0.5 * xn)[:, None], (1, 6))
    xi = rng.uniform(x0, x0 + L - 1.0, 1000)
    assert np.allclose(grid.interpolate(lin, x0, L, xi)[:, 3], 2.0 + 0.5 * xi, rtol=1e-15, atol=1e-14)
    # one node: a constant field (to the rounding of (1 - f) c + f c)
    assert np.allclose(grid.interpolate(np.ones((1, 6)) * 3.0, 0.0, 1.0, rng.normal(size=50)), 3.0,
                       rtol=5e-16, atol=0)


def test_wrap_properties():
    rng = np.random.default_rng(2)
    lo, L = -1035842.0299300797, 2071684.0598601594
    x = rng.uniform(lo - 2 * L, lo + 3 * L, 20000)
    x[:4] = [lo, lo + L, np.nextafter(lo, -np.inf), np.nextafter(lo + L, np.inf)]
    w = grid.wrap(x, lo, L)
    assert np.all(w >= lo) and np.all(w < lo + L)
    m = (x - w) / L
    assert np.allclose(m, np.round(m), atol=1e-9)
    inside = (x >= lo) & (x < lo + L)
    assert np.array_equal(w[inside], x[inside])          # identity inside the box
    assert np.array_equal(grid.wrap(w, lo, L), w)          # idempotent


def test_gather_rounds_positions_then_fields():
    prm = synth.standing_wave_params()
    nodes = grid.standing_wave_nodes(128, prm["x0"], prm["length"], prm["e0"], prm["k"], prm["omega"], 0.0, 0.0)
    rng = np.random.default_rng(3)
    L = prm["length"]
    x = rng.uniform(-1.5 * L, 1.5 * L, (1000, 3)).astype(np.float32).astype(np.float64)
    lo = (prm["x0"],) * 3
    xs, f = grid.gather(x, nodes, prm["x0"], L, lo, (L, L, L), dtype=np.float32)
    assert np.array_equal(xs, xs.astype(np.float32).astype(np.float64))
    assert np.array_equal(f, f.astype(np.float32).astype(np.float64))
    # the fields are those at the stored (rounded) coordinate, within float rounding of the wave
    exact = grid.standing_wave_nodes(1, 0.0, L, prm["e0"], prm["k"], prm["omega"], 0.0, 0.0)
    ce = prm["e0"] * np.cos(prm["k"] * xs[:, 0])
    assert np.allclose(f[:, 1], ce, atol=5e-4 * prm["e0"])   # linear interpolation error ~ (k dx)^2 / 8
    assert exact.shape == (1, 6)
    # an unwrapped axis keeps its coordinates
    xs2, _ = grid.gather(x, nodes, prm["x0"], L, lo, (L, 0.0, L), dtype=np.float32)
    assert np.array_equal(xs2[:, 1], x[:, 1])
