"""Pins of the oracle's special functions, rates, spectra and inverse CDFs.

The paper (Sec. 3) defers the rates to polynomial fits of the synchrotron
functions; the oracle computes the locally-constant-field spectra by
quadrature.  These tests tie it to things other than itself:
* scipy.special.kv and mpmath.besselk, and K_{1/2}(x) = sqrt(pi/2x) e^-x;
* closed forms of the limits chi -> 0 and chi -> oo, derived from the Mellin
  integrals int_0^oo y^(mu-1) K_nu(y) dy = 2^(mu-2) G((mu-nu)/2) G((mu+nu)/2);
* an mpmath evaluation of the rates in a different form (integrated by parts,
  so that only K_{2/3} and K_{1/3} appear, no integral of a Bessel function);
* the symmetry of the pair spectrum and the classical mean photon energy.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

G23 = math.gamma(2.0 / 3.0)


# ----------------------------------------------------------------------------- special functions
@pytest.mark.parametrize("nu", [1.0 / 3.0, 2.0 / 3.0, 5.0 / 3.0, 0.5])
def test_bessel_k_definition_vs_scipy(orc, nu):
    for x in np.geomspace(1e-6, 600, 37):
        ref = ss.kv(nu, x)
        assert abs(orc.bessel_k(nu, x, True) / ref - 1) < 5e-13, (nu, x)


def test_bessel_k_half_closed_form(orc):
    for x in np.geomspace(1e-8, 700, 41):
        ref = math.sqrt(math.pi / (2 * x)) * math.exp(-x)
        assert abs(orc.bessel_k(0.5, x, True) / ref - 1) < 2e-14


def test_bessel_mpmath_high_precision(orc):
    mp.mp.dps = 30
    for nu in (mp.mpf(1) / 3, mp.mpf(2) / 3):
        for x in ("1e-20", "1e-3", "0.7", "3", "40", "300"):
            ref = float(mp.besselk(nu, mp.mpf(x)))
            assert abs(orc.bessel_k(float(nu), float(x), True) / ref - 1) < 1e-14, (nu, x)
    # Ki_{1/3}(x) = int_x^oo K_{1/3}
    for x in ("1e-6", "0.3", "2", "25"):
        ref = float(mp.quad(lambda s: mp.besselk(mp.mpf(1) / 3, s), [mp.mpf(x), 1, 10, mp.inf]))
        assert abs(orc.bessel_ki(1.0 / 3.0, float(x), True) / ref - 1) < 1e-13, x


def test_ki_limits_and_recurrence(orc):
    # int_0^oo K_nu = pi / (2 cos(nu pi / 2)); Ki_{1/3}(0) = pi/sqrt3
    assert abs(orc.bessel_ki(1.0 / 3.0, 1e-40, True) / (math.pi / math.sqrt(3)) - 1) < 1e-14
    assert abs(orc.bessel_ki(0.5, 1e-40, True) / (math.pi / (2 * math.cos(math.pi / 4))) - 1) < 1e-12
    # Ki_{5/3} = 2 K_{2/3} - Ki_{1/3} (from K_{nu-1} + K_{nu+1} = -2 K_nu')
    for y in np.geomspace(1e-4, 200, 17):
        lhs = orc.bessel_ki(5.0 / 3.0, y, True)
        rhs = 2 * orc.bessel_k(2.0 / 3.0, y, True) - orc.bessel_ki(1.0 / 3.0, y, True)
        assert abs(lhs / rhs - 1) < 1e-12, y


def test_fast_tier_matches_definitions(orc):
    rng = np.random.default_rng(3)
    ys = np.exp(rng.uniform(np.log(1e-44), np.log(740), 400))
    for y in ys:
        assert abs(orc.bessel_k(2 / 3, y, False) / orc.bessel_k(2 / 3, y, True) - 1) < 5e-14, y
        assert abs(orc.bessel_ki(1 / 3, y, False) / orc.bessel_ki(1 / 3, y, True) - 1) < 5e-14, y


# ----------------------------------------------------------------------------- rates
def _mp_rate_rad(chi):
    """W_rad gamma/alpha by parts: int_0^1 [A K_{2/3}(y) - d y'(d) K_{1/3}(y)] dd / (sqrt3 pi),
    with d = u^3 to remove the d^{-2/3} end-point singularity."""
    chi = mp.mpf(chi)

    def f(u):
        d = u ** 3
        y = 2 * d / (3 * chi * (1 - d))
        a = 1 - d + 1 / (1 - d)
        yp = 2 / (3 * chi * (1 - d) ** 2)
        return (a * mp.besselk(mp.mpf(2) / 3, y) - d * yp * mp.besselk(mp.mpf(1) / 3, y)) * 3 * u * u

    dc = 3 * chi / (2 + 3 * chi)
    pts = sorted({mp.mpf(0), mp.cbrt(dc / 10), mp.cbrt(dc), mp.cbrt(1 - (1 - dc) / 10), mp.mpf(1)})
    return float(mp.quad(f, pts) / (mp.sqrt(3) * mp.pi))


def _mp_rate_pair(chi):
    """W_pair eps/alpha = 2 int_0^1/2 [A K_{2/3}(y) + Ki_{1/3}(y)] dxi / (sqrt3 pi), with
    int_0^1/2 Ki_{1/3}(y(xi)) dxi = Ki_{1/3}(8/3chi)/2 - int_0^1/2 xi K_{1/3}(y) |y'| dxi
    (y decreases on (0, 1/2))."""
    chi = mp.mpf(chi)
    third = mp.mpf(1) / 3

    def f(x):
        y = 2 / (3 * chi * x * (1 - x))
        a = x / (1 - x) + (1 - x) / x
        yp = 2 * (1 - 2 * x) / (3 * chi * (x * (1 - x)) ** 2)
        return a * mp.besselk(2 * third, y) - x * yp * mp.besselk(third, y)

    y0 = 8 / (3 * chi)
    ki0 = mp.quad(lambda s: mp.besselk(third, s), [y0, y0 + 1, y0 + 10, mp.inf])
    pts = [mp.mpf(0), 1 / (3 * chi) / 4, 1 / (3 * chi), mp.mpf("0.25"), mp.mpf("0.5")]
    pts = sorted(set(p for p in pts if p <= mp.mpf("0.5")))
    return float(2 * (mp.quad(f, pts) + ki0 / 2) / (mp.sqrt(3) * mp.pi))


@pytest.mark.parametrize("chi", [0.1, 1.0, 10.0])
def test_rate_rad_vs_mpmath_by_parts(orc, chi):
    mp.mp.dps = 20
    ref = _mp_rate_rad(chi)
    assert abs(orc.rate_rad_reduced(chi, True) / ref - 1) < 1e-12
    assert abs(orc.rate_rad_reduced(chi, False) / ref - 1) < 1e-12


@pytest.mark.parametrize("chi", [0.3, 2.0, 30.0])
def test_rate_pair_vs_mpmath_by_parts(orc, chi):
    mp.mp.dps = 20
    ref = _mp_rate_pair(chi)
    assert abs(orc.rate_pair_reduced(chi, True) / ref - 1) < 1e-12
    assert abs(orc.rate_pair_reduced(chi, False) / ref - 1) < 1e-12


def test_rate_rad_small_chi(orc):
    # chi -> 0: f = (3chi/2) int_0^oo (2K_{2/3} - Ki_{1/3}) dy / (sqrt3 pi) = 5 chi / (2 sqrt3),
    # with int K_{2/3} = pi and int Ki_{1/3} = int y K_{1/3} = pi/3; first correction -(8 sqrt3/15) chi
    lead = lambda c: 5 * c / (2 * math.sqrt(3))
    for c in (1e-5, 1e-4):
        r = orc.rate_rad_reduced(c, False) / lead(c)
        slope = (1 - r) / c
        assert abs(slope - 8 * math.sqrt(3) / 15) < 2e-3 * 8 * math.sqrt(3) / 15 + 10 * c


def test_rate_rad_large_chi(orc):
    # chi -> oo: f -> Gamma(2/3) 3^{2/3}/(2 sqrt3 pi) (B(1/3,8/3)+B(1/3,2/3)) chi^{2/3}
    #             = 14 Gamma(2/3) / 3^{7/3} chi^{2/3}
    c_inf = 14 * G23 / 3 ** (7 / 3)
    vals = {c: orc.rate_rad_reduced(c, False) / c ** (2 / 3) for c in (1e6, 1e8)}
    # the correction falls like chi^{-2/3}: extrapolate
    x1, x2 = 1e6 ** (-2 / 3), 1e8 ** (-2 / 3)
    a = (vals[1e8] * x1 - vals[1e6] * x2) / (x1 - x2)
    assert abs(a / c_inf - 1) < 1e-6
    assert abs(vals[1e8] / c_inf - 1) < 1e-4


def test_rate_pair_limits(orc):
    # chi -> 0 (Erber): f -> 3 sqrt3/(16 sqrt2) chi exp(-8/(3chi)), correction O(chi)
    erber = lambda c: 3 * math.sqrt(3) / (16 * math.sqrt(2)) * c * math.exp(-8 / (3 * c))
    for c in (0.005, 0.01, 0.02):
        r = orc.rate_pair_reduced(c, False) / erber(c)
        assert 0.1 < (1 - r) / c < 0.25, (c, r)
    # chi -> oo: f -> 15 3^{2/3} Gamma(2/3)^4 / (28 pi^2) chi^{2/3}
    c_inf = 15 * 3 ** (2 / 3) * G23 ** 4 / (28 * math.pi ** 2)
    vals = {c: orc.rate_pair_reduced(c, False) / c ** (2 / 3) for c in (1e6, 1e8)}
    x1, x2 = 1e6 ** (-2 / 3), 1e8 ** (-2 / 3)
    a = (vals[1e8] * x1 - vals[1e6] * x2) / (x1 - x2)
    assert abs(a / c_inf - 1) < 1e-5


def test_spectrum_identity_ki53(orc):
    # the emission spectrum equals (1/(sqrt3 pi)) [Ki_{5/3}(y) + d^2/(1-d) K_{2/3}(y)]
    for chi in (0.05, 1.0, 20.0):
        for d in (1e-4, 0.01, 0.3, 0.9):
            y = 2 * d / (3 * chi * (1 - d))
            alt = (orc.bessel_ki(5 / 3, y, True) + d * d / (1 - d) * orc.bessel_k(2 / 3, y, True)) / (
                math.sqrt(3) * math.pi)
            assert abs(orc.spec_rad(chi, d, True) / alt - 1) < 1e-12


# ----------------------------------------------------------------------------- CDF / inverse CDF
def test_pair_cdf_symmetric(orc):
    for chi in (0.05, 1.0, 100.0):
        assert abs(orc.cdf_pair(chi, 0.5) - 0.5) < 1e-13
        for r in (1e-5, 0.1, 0.37):
            x = orc.sample_pair_r(chi, r)
            x2 = orc.sample_pair_r(chi, 1 - r)
            assert abs(x + x2 - 1) < 1e-13


def test_inverse_cdf_roundtrip(orc):
    for chi in (1e-3, 0.1, 1.0, 30.0, 1e3):
        for r in (1e-7, 0.01, 0.3, 0.5, 0.8, 0.999):
            d = orc.sample_rad_r(chi, r)
            assert abs(orc.cdf_rad(chi, d, False) - r) < 1e-13 * max(1.0, 1 / min(r, 1 - r)) * min(r, 1 - r) + 1e-15
    for chi in (0.1, 3.0, 300.0):
        for r in (1e-6, 0.2, 0.45):
            x = orc.sample_pair_r(chi, r)
            assert abs(orc.cdf_pair(chi, x, False) - r) < 1e-13


def test_inverse_cdf_definitions_tier(orc):
    # fast tier sampler == definitions tier sampler
    for chi, r in ((0.2, 0.3), (5.0, 0.9), (50.0, 0.01)):
        a = orc.sample_rad_r(chi, r, False)
        b = orc.sample_rad_r(chi, r, True)
        assert abs(a / b - 1) < 1e-12


def test_classical_mean_photon_energy(orc):
    # chi -> 0: <delta> = (3chi/2) int y (2K_{2/3} - Ki_{1/3}) / int (2K_{2/3} - Ki_{1/3})
    #          = (3chi/2) (8/27 pi sqrt3 ... ) = 4 chi / (5 sqrt3); E[delta] = int_0^1 F^-1(r) dr
    chi = 1e-4
    m, _ = si.quad(lambda r: orc.sample_rad_r(chi, r), 0, 1, epsabs=0, epsrel=1e-9, limit=200,
                   points=[1e-3, 0.1, 0.5, 0.9, 0.999])
    ref = 4 * chi / (5 * math.sqrt(3))
    assert abs(m / ref - 1) < 5e-3  # O(chi) corrections: -(1.4...) chi
    # at finite chi the mean from the inverse CDF equals the first moment of the spectrum
    chi = 2.0
    m, _ = si.quad(lambda r: orc.sample_rad_r(chi, r), 0, 1, epsrel=1e-10, limit=200,
                   points=[1e-3, 0.1, 0.5, 0.9, 0.999])
    num, _ = si.quad(lambda d: d * orc.spec_rad(chi, d), 0, 1, epsrel=1e-11, limit=400,
                     points=[1e-6, 1e-3, 0.1, 0.5, 0.9, 0.99])
    assert abs(m / (num / orc.rate_rad_reduced(chi)) - 1) < 1e-7


def test_pair_mean_half(orc):
    m, _ = si.quad(lambda r: orc.sample_pair_r(3.0, r), 0, 1, epsrel=1e-10, limit=200, points=[0.01, 0.5, 0.99])
    assert abs(m - 0.5) < 1e-9


def test_cdf_vs_mpmath(orc):
    # F(delta) at one point from mpmath with the by-parts form of the numerator
    mp.mp.dps = 20
    chi, d0 = mp.mpf(1), mp.mpf("0.2")
    third = mp.mpf(1) / 3

    def num_f(u):
        d = u ** 3
        y = 2 * d / (3 * chi * (1 - d))
        a = 1 - d + 1 / (1 - d)
        yp = 2 / (3 * chi * (1 - d) ** 2)
        return (a * mp.besselk(2 * third, y) - d * yp * mp.besselk(third, y)) * 3 * u * u

    y0 = 2 * d0 / (3 * chi * (1 - d0))
    ki0 = mp.quad(lambda s: mp.besselk(third, s), [y0, y0 + 1, y0 + 10, mp.inf])
    # int_0^d0 Ki(y) dd = d0 Ki(y0) + int_0^d0 d K_{1/3}(y) y' dd
    u0 = mp.cbrt(d0)
    num = mp.quad(num_f, [0, u0 / 3, u0]) - d0 * ki0
    ref = float(num / (mp.sqrt(3) * mp.pi) / mp.mpf(_mp_rate_rad(1.0)))
    assert abs(orc.cdf_rad(1.0, 0.2) / ref - 1) < 1e-11
