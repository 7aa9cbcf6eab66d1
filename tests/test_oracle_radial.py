"""Pins of the oracle's radial expansion (Eqs. (01), (19), (02), (04) and the Gaussian-basis overlap)."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle


def _quad(f, pts):
    with mp.workdps(30):
        return mp.quad(f, pts)


@pytest.mark.parametrize("mu,s,rc", [(1.2, 0.5, 3.7), (2.9, 0.5, 5.0), (0.0, 0.5, 5.0), (4.8, 0.5, 5.0),
                                     (1.5, 0.12, 4.3), (3.0, 1.27, 5.5), (5.3, 0.5, 5.5)])
def test_overlap_recursion_matches_quadrature(mu, s, rc):
    # I_k = int_0^rc (1 - t/rc)^k exp(-(t-mu)^2/(2 s^2)) dt, k = 0..14
    I = oracle.overlap_integrals(0.0, rc, mu, s, rc, 14)
    for k in range(15):
        want = _quad(lambda t: (1 - t / rc) ** k * mp.exp(-(t - mu) ** 2 / (2 * s * s)),
                     [0, min(max(mu, 0), rc), rc])
        assert abs(I[k] - float(want)) <= 1e-13 * abs(float(want)) + 1e-300


def test_overlap_recursion_general_limits():
    # the same recursion with limits [r_soft, r_hard] (buffer zone)
    lo, hi, mu, s, rc = 4.0, 5.0, 3.7, 0.3, 5.0
    I = oracle.overlap_integrals(lo, hi, mu, s, rc, 10)
    for k in range(11):
        want = _quad(lambda t: (1 - t / rc) ** k * mp.exp(-(t - mu) ** 2 / (2 * s * s)), [lo, hi])
        assert abs(I[k] - float(want)) <= 1e-13 * abs(float(want))


@pytest.mark.parametrize("mu,s,s0", [(0.0, 0.5, 0.5), (1.2, 0.5, 0.5), (2.0, 0.3, 0.2), (0.7, 0.8, 0.12)])
def test_gaussian_basis_overlap_closed_form(mu, s, s0):
    B, dB_dmu, dB_ds = oracle.gauss_basis_overlap(mu, s, s0)

    def val(m, ss):
        cg = mp.sqrt(2) / (mp.sqrt(s0) * mp.pi ** mp.mpf("0.25"))
        return mp.quad(lambda t: cg * mp.exp(-t * t / (2 * s0 * s0)) * mp.exp(-(t - m) ** 2 / (2 * ss * ss)),
                       [0, m, mp.inf] if m > 0 else [0, mp.inf])

    with mp.workdps(30):
        assert abs(B - float(val(mp.mpf(mu), mp.mpf(s)))) < 1e-15 * max(1, abs(B))
        d1 = mp.diff(lambda m: val(m, mp.mpf(s)), mp.mpf(mu))
        d2 = mp.diff(lambda ss: val(mp.mpf(mu), ss), mp.mpf(s))
    assert abs(dB_dmu - float(d1)) < 1e-12 * max(1, abs(float(d1)))
    assert abs(dB_ds - float(d2)) < 1e-12 * max(1, abs(float(d2)))


def _bn_by_quadrature(p: oracle.Params, r):
    """b_n(r) = sum_a W_na (int over [0, r_c] of phi_a f G, polynomial a; int_0^inf phi_G G, Gaussian a)
    with f the density smoothing function as printed in Sec. "Density smoothing at the cutoff"."""
    S, W, *_ = oracle.basis_tables(p.n_max, p.r_cut, p.sigma0_r)
    rc = p.r_cut
    rs = rc if p.r_soft is None else p.r_soft
    s = p.sigma0_r + p.alpha_r * r
    with mp.workdps(30):
        def f(t):
            if t < rs:
                return 1
            return mp.exp(-p.n_f ** 2 / 2 * (t - rs) ** 2 / (rc - rs) ** 2)

        G = lambda t: mp.exp(-(t - r) ** 2 / (2 * s * s))
        ba = []
        for a in range(1, p.n_max):
            Na = mp.sqrt(mp.mpf(rc) / (2 * a + 5))
            pts = sorted(set([0, min(r, rc), rs, rc]))
            ba.append(mp.quad(lambda t: (1 - t / rc) ** (a + 2) / Na * f(t) * G(t), pts))
        s0 = mp.mpf(p.sigma0_r)
        cg = mp.sqrt(2) / (mp.sqrt(s0) * mp.pi ** mp.mpf("0.25"))
        ba.append(mp.quad(lambda t: cg * mp.exp(-t * t / (2 * s0 * s0)) * G(t), [0, r, mp.inf] if r > 0 else [0, mp.inf]))
        bn = W * mp.matrix(ba)
        return np.array([float(x) for x in bn])


@pytest.mark.parametrize("r", [0.0, 1.2, 2.3, 3.6])
def test_radial_coefficients_match_quadrature(r):
    p = oracle.Params(n_max=6, l_max=2, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5)
    b, _ = oracle.radial(p, r)
    want = _bn_by_quadrature(p, r)
    assert np.linalg.norm(b - want) < 1e-13 * np.linalg.norm(want)


@pytest.mark.parametrize("r", [1.0, 3.0, 4.1, 4.25])
def test_radial_coefficients_buffer_and_widths(r):
    # the paper's optimised hyper-parameters (Sec. "Hyperparameter optimization"), plus a buffer zone
    p = oracle.Params(n_max=8, l_max=2, r_cut=4.3, r_soft=3.8, sigma0_r=0.12, sigma0_perp=0.55,
                      alpha_r=0.14, alpha_perp=0.06, a=1.6)
    b, _ = oracle.radial(p, r)
    want = _bn_by_quadrature(p, r)
    assert np.linalg.norm(b - want) < 1e-12 * np.linalg.norm(want)


def test_smoothing_function_printed_value():
    # Sec. "Density smoothing at the cutoff": n_f = 4 brings f down to about 3.35e-4 at r_hard.
    golden = {}
    with open(__file__.replace("test_oracle_radial.py", "golden/smoothing_f_rhard.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                golden[k] = float(v)
    # the buffer-zone radial overlap integrates f G; f at r_hard follows from its definition
    f_rhard = math.exp(-golden["n_f"] ** 2 / 2)
    assert abs(f_rhard - golden["f_at_r_hard"]) < 0.005e-4
    # and the oracle's product-Gaussian split reproduces int f G on the buffer domain:
    p = oracle.Params(n_max=4, l_max=0, r_cut=5.0, r_soft=4.0, sigma0_r=0.5, sigma0_perp=0.5,
                      n_f=golden["n_f"])
    b, _ = oracle.radial(p, 4.6)
    assert np.linalg.norm(b - _bn_by_quadrature(p, 4.6)) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("params", [
    dict(n_max=8, l_max=2, r_cut=5.0, sigma0_r=0.5, sigma0_perp=0.5),
    dict(n_max=8, l_max=2, r_cut=4.5, sigma0_r=0.2, sigma0_perp=0.4, alpha_r=0.08, alpha_perp=0.08, a=1.0),
    dict(n_max=6, l_max=2, r_cut=4.3, r_soft=3.5, sigma0_r=0.12, sigma0_perp=0.55, alpha_r=0.14,
         alpha_perp=0.06, a=1.6),
])
def test_radial_derivative_by_richardson(params):
    p = oracle.Params(**params)
    for r in (1.3, 2.7, 3.9):
        _, db = oracle.radial(p, r)
        h = 1e-3
        d1 = (oracle.radial(p, r + h)[0] - oracle.radial(p, r - h)[0]) / (2 * h)
        d2 = (oracle.radial(p, r + h / 2)[0] - oracle.radial(p, r - h / 2)[0]) / h
        fd = (4 * d2 - d1) / 3
        assert np.linalg.norm(db - fd) < 1e-8 * max(1.0, np.linalg.norm(fd))


def test_amplitude_eq15():
    p = oracle.Params(n_max=4, l_max=0, r_cut=4.5, sigma0_r=0.2, sigma0_perp=0.4, alpha_r=0.08,
                      alpha_perp=0.08, a=1.0)
    r = 2.0
    A, dA = oracle.amplitude(p, r)
    x = r / 4.5
    want = (1 + 2 * x ** 3 - 3 * x ** 2) / ((0.2 + 0.08 * r) * (0.4 + 0.08 * r) ** 2)
    assert abs(A - want) < 1e-15 * want
    h = 1e-4
    fd = (oracle.amplitude(p, r + h)[0] - oracle.amplitude(p, r - h)[0]) / (2 * h)
    assert abs(dA - fd) < 1e-7 * abs(fd)
    # no-downscaling limit alpha_r = alpha_perp = a = 0
    p0 = oracle.Params(n_max=4, l_max=0, r_cut=4.5, sigma0_r=0.5, sigma0_perp=0.5)
    assert abs(oracle.amplitude(p0, 3.0)[0] - 1 / 0.125) < 1e-14
