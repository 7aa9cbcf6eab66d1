"""Pins of the oracle's radial basis tables (Sec. "Radial expansion coefficients").

Each check compares the oracle's S / W with something the paper or mathematics
fixes independently of how the oracle computed them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n_max,r_cut,s0", [(6, 3.7, 0.5), (8, 5.0, 0.5), (10, 5.5, 0.5), (8, 4.3, 0.12)])
def test_polynomial_block_closed_form(n_max, r_cut, s0):
    # N_alpha = sqrt(r_c/(2 alpha + 5)) makes int phi_a phi_b = sqrt((2a+5)(2b+5))/(a+b+5),
    # independent of r_c; the diagonal is 1 (normalisation stated with the basis).
    S, *_ = oracle.basis_tables(n_max, r_cut, s0)
    with mp.workdps(50):
        for a in range(1, n_max):
            for b in range(1, n_max):
                want = mp.sqrt((2 * a + 5) * (2 * b + 5)) / mp.mpf(a + b + 5)
                assert abs(S[a - 1, b - 1] - want) < mp.mpf("1e-40")
        assert abs(S[0, 0] - 1) < mp.mpf("1e-40")


@pytest.mark.parametrize("r_cut,s0", [(3.7, 0.5), (5.0, 0.2), (4.3, 0.12)])
def test_gaussian_basis_normalisation(r_cut, s0):
    # Eq. (06): phi_nmax is unit-normalised on [0, inf); over [0, r_c] its square integrates to erf(r_c/s0).
    S, *_ = oracle.basis_tables(6, r_cut, s0)
    with mp.workdps(50):
        assert abs(S[5, 5] - mp.erf(mp.mpf(r_cut) / mp.mpf(s0))) < mp.mpf("1e-40")


@pytest.mark.parametrize("n_max,r_cut,s0", [(6, 3.7, 0.5), (8, 5.0, 0.5), (10, 5.5, 0.5)])
def test_w_is_inverse_square_root(n_max, r_cut, s0):
    S, W, Whi, Wlo, eig = oracle.basis_tables(n_max, r_cut, s0)
    with mp.workdps(50):
        I = W * S * W
        for i in range(n_max):
            for j in range(n_max):
                assert abs(I[i, j] - (1 if i == j else 0)) < mp.mpf("1e-25")
        # symmetric
        for i in range(n_max):
            for j in range(n_max):
                assert abs(W[i, j] - W[j, i]) < mp.mpf("1e-35") * abs(W[i, j])
    assert min(eig) > 0


def _gauss_legendre_gram(n_max, r_cut, s0, Whi, Wlo):
    """Gram matrix of g_n = sum_a W_na phi_a by composite Gauss-Legendre in 40 digits,
    with the basis functions written out from the paper's definitions."""
    with mp.workdps(40):
        rc = mp.mpf(r_cut)
        s0 = mp.mpf(s0)
        W = mp.matrix(n_max, n_max)
        for i in range(n_max):
            for j in range(n_max):
                W[i, j] = mp.mpf(Whi[i, j]) + mp.mpf(Wlo[i, j])
        nodes, weights = [], []
        x, w = np.polynomial.legendre.leggauss(60)
        edges = [0, 0.25, 0.5, 1.0, 1.5, 2.0, 3.0, r_cut]
        edges = sorted(set(e for e in edges if e <= r_cut))
        # 60-point rule nodes in double are exact enough as sample points; weights scaled exactly
        for lo, hi in zip(edges[:-1], edges[1:]):
            for xi, wi in zip(x, w):
                nodes.append(mp.mpf(lo) + (mp.mpf(hi) - mp.mpf(lo)) * (mp.mpf(xi) + 1) / 2)
                weights.append(mp.mpf(wi) * (mp.mpf(hi) - mp.mpf(lo)) / 2)
        cg = mp.sqrt(2) / (mp.sqrt(s0) * mp.pi ** mp.mpf("0.25"))
        G = mp.matrix(n_max, n_max)
        for t, wt in zip(nodes, weights):
            phi = [(1 - t / rc) ** (a + 2) / mp.sqrt(rc / (2 * a + 5)) for a in range(1, n_max)]
            phi.append(cg * mp.exp(-t * t / (2 * s0 * s0)))
            g = [mp.fsum(W[n, a] * phi[a] for a in range(n_max)) for n in range(n_max)]
            for i in range(n_max):
                for j in range(n_max):
                    G[i, j] += wt * g[i] * g[j]
        return G


@pytest.mark.parametrize("n_max,r_cut,s0", [(6, 3.7, 0.5), (8, 5.0, 0.5)])
def test_orthonormal_basis_by_quadrature(n_max, r_cut, s0):
    # g_n = sum_a W_na phi_a must be orthonormal on [0, r_c]
    _, _, Whi, Wlo, _ = oracle.basis_tables(n_max, r_cut, s0)
    G = _gauss_legendre_gram(n_max, r_cut, s0, Whi, Wlo)
    err = max(abs(G[i, j] - (1 if i == j else 0)) for i in range(n_max) for j in range(n_max))
    assert err < 1e-12


def test_basis_degenerates_with_n_max():
    # The paper reports linear dependencies of the basis beyond n_max = 12: the
    # smallest eigenvalue of S falls by orders of magnitude with each added function.
    lmins = []
    for n in (4, 6, 8, 10, 12):
        *_, eig = oracle.basis_tables(n, 5.0, 0.5)
        lmins.append(float(min(eig)))
    assert all(b < a * 1e-1 for a, b in zip(lmins, lmins[1:]))
    assert lmins[-1] < 1e-16  # below double precision relative to |S| ~ 1 at n_max = 12
