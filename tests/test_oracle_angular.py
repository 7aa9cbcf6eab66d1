"""Pins of the oracle's angular factors: ilexp (Sec. "Angular expansion coefficients") and Y_lm."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

import oracle

Z_GRID = [1e-9, 1e-4, 0.01, 0.3, 1.0, 1.96, 3.0, 5.76, 8.0, 16.0, 36.0, 50.0, 100.0, 121.0]


@pytest.mark.parametrize("z", Z_GRID)
def test_ilexp_matches_library(z):
    # e_l(z) = exp(-z) i_l(z) with i_l the modified spherical Bessel function of the first kind
    e, de = oracle.ilexp(z, 12)
    with mp.workdps(40):
        for l in range(13):
            want = mp.exp(-z) * mp.sqrt(mp.pi / (2 * mp.mpf(z))) * mp.besseli(l + mp.mpf(1) / 2, z)
            assert abs(e[l] - float(want)) <= 1e-15 * abs(float(want)) + 1e-300
    if z > 1e-3:
        lib = special.spherical_in(np.arange(13), z) * math.exp(-z)
        ok = lib > 1e-290
        assert np.allclose(e[ok], lib[ok], rtol=1e-12, atol=0)


@pytest.mark.parametrize("z", [0.01, 0.5, 2.0, 5.76, 30.0, 121.0])
def test_ilexp_derivative_identity(z):
    # i_l' = i_{l+1} + (l/z) i_l, so d e_l/dz = e_{l+1} + (l/z - 1) e_l
    e, de = oracle.ilexp(z, 12)
    for l in range(12):
        want = e[l + 1] + (l / z - 1) * e[l]
        assert abs(de[l] - want) <= 1e-12 * (abs(e[l]) + abs(e[l + 1]) + abs(de[l]))


@pytest.mark.parametrize("z", [0.2, 1.0, 4.0, 20.0])
def test_ilexp_seeds_printed(z):
    # printed seeds: ilexp(x;0) = (1 - e^{-2x^2}) / (2x^2),
    # ilexp(x;1) = (x^2 - 1 + e^{-2x^2}(x^2 + 1)) / (2x^4), with z = x^2
    e, _ = oracle.ilexp(z, 2)
    e0 = -math.expm1(-2 * z) / (2 * z)
    e1 = (z - 1 + math.exp(-2 * z) * (z + 1)) / (2 * z * z)
    assert abs(e[0] - e0) < 1e-14 * e0
    assert abs(e[1] - e1) < 1e-9 * e1  # e1's printed form cancels at small z


@pytest.mark.parametrize("z", [50.0, 80.0, 121.0])
def test_ilexp_upward_recursion_where_stable(z):
    # the printed recursion ilexp(l) = ilexp(l-2) - (2l-1)/x^2 ilexp(l-1) is accurate for large z
    e, _ = oracle.ilexp(z, 12)
    v = [-math.expm1(-2 * z) / (2 * z), (z - 1 + math.exp(-2 * z) * (z + 1)) / (2 * z * z)]
    for l in range(2, 13):
        v.append(v[l - 2] - (2 * l - 1) / z * v[l - 1])
    assert np.allclose(e, v, rtol=1e-13, atol=0)


def test_ilexp_small_argument_limit():
    # Taylor limit printed for x -> 0: ilexp(x;l) -> x^{2l}/(2l+1)!!
    z = 1e-6
    e, _ = oracle.ilexp(z, 6)
    for l in range(7):
        dfact = np.prod(np.arange(1, 2 * l + 2, 2, dtype=float))
        assert abs(e[l] - z ** l / dfact) <= 2e-6 * z ** l / dfact


def _random_units(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_ylm_matches_scipy():
    for u in _random_units(20, 7):
        theta = math.acos(u[2])
        phi = math.atan2(u[1], u[0])
        for l in range(13):
            for m in range(l + 1):
                y, _ = oracle.ylm_conj(l, m, u)
                want = np.conj(special.sph_harm_y(l, m, theta, phi))
                assert abs(y - want) < 1e-13 * max(1.0, abs(want))


def test_legendre_seeds_printed():
    # printed seeds: P_00 = 1, P_10 = x, P_11 = -sqrt(1-x^2), P_20 = 3/2 x^2 - 1/2,
    # P_21 = -3x sqrt(1-x^2), P_22 = 3 - 3x^2.  With phi = 0, Y*_lm = N_lm P_lm(cos theta).
    seeds = {
        (0, 0): lambda x: 1.0,
        (1, 0): lambda x: x,
        (1, 1): lambda x: -math.sqrt(1 - x * x),
        (2, 0): lambda x: 1.5 * x * x - 0.5,
        (2, 1): lambda x: -3 * x * math.sqrt(1 - x * x),
        (2, 2): lambda x: 3 - 3 * x * x,
    }
    for x in (-0.9, -0.3, 0.2, 0.77):
        u = np.array([math.sqrt(1 - x * x), 0.0, x])
        for (l, m), P in seeds.items():
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            y, _ = oracle.ylm_conj(l, m, u)
            assert abs(y.imag) < 1e-15
            assert abs(y.real / N - P(x)) < 1e-14


def test_addition_theorem():
    # sum_{m=-l}^{l} Y*_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a . b), with Y_{l,-m} = (-1)^m Y*_lm
    us = _random_units(10, 11)
    for a, b in zip(us[:5], us[5:]):
        for l in range(13):
            s = 0j
            for m in range(l + 1):
                ya, _ = oracle.ylm_conj(l, m, a)
                yb, _ = oracle.ylm_conj(l, m, b)
                term = ya * np.conj(yb)
                s += term if m == 0 else 2 * term.real
            want = (2 * l + 1) / (4 * math.pi) * special.eval_legendre(l, float(a @ b))
            assert abs(s - want) < 1e-13


def test_pole_regular():
    # at the poles Y_lm, m > 0, vanishes and the oracle needs no special rule
    for z in (1.0, -1.0):
        u = np.array([0.0, 0.0, z])
        for l in range(13):
            for m in range(1, l + 1):
                y, _ = oracle.ylm_conj(l, m, u)
                assert y == 0
            y0, _ = oracle.ylm_conj(l, 0, u)
            assert abs(y0 - math.sqrt((2 * l + 1) / (4 * math.pi)) * z ** l) < 1e-13


def test_ylm_gradient_by_finite_differences():
    # gradient of Y*_lm(v / |v|) w.r.t. v, from the oracle's polynomial gradient projected on the sphere
    for u in _random_units(4, 3):
        for l in (1, 4, 9, 12):
            for m in (0, 1, l // 2, l):
                _, g = oracle.ylm_conj(l, m, u)
                gs = g - u * (u @ g)  # tangential part = gradient at |v| = 1
                h = 1e-5
                fd = np.zeros(3, dtype=complex)
                for x in range(3):
                    e = np.zeros(3)
                    e[x] = h
                    vp, vm = u + e, u - e
                    fd[x] = (oracle.ylm_conj(l, m, vp / np.linalg.norm(vp))[0]
                             - oracle.ylm_conj(l, m, vm / np.linalg.norm(vm))[0]) / (2 * h)
                assert np.abs(gs - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())
