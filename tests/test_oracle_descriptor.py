"""Pins of the oracle's c_nlm, power spectrum and normalised descriptor (Eqs. (08), (09))."""
import math

import numpy as np
import pytest
from scipy import special

import oracle
import synth


def _nl_from_vectors(vectors_per_centre):
    """A NeighbourList whose pairs are given directly as vectors d = r_j - r_i."""
    offs = [0]
    d = []
    for vs in vectors_per_centre:
        d.extend(vs)
        offs.append(len(d))
    n = len(d)
    return oracle.NeighbourList(np.arange(len(vectors_per_centre)), np.array(offs, dtype=np.int64),
                                np.zeros(n, dtype=np.int32), np.zeros((n, 3), dtype=np.int32),
                                np.array(d, dtype=np.float64).reshape(n, 3))


def _unpack(p: oracle.Params, v):
    """packed descriptor -> full p[a, b, l] (undo the sqrt(2) on a != b)"""
    nch = p.n_channels
    P = np.zeros((nch, nch, p.l_max + 1))
    k = 0
    for a in range(nch):
        for b in range(a, nch):
            for l in range(p.l_max + 1):
                P[a, b, l] = P[b, a, l] = v[k] / (1 if a == b else math.sqrt(2))
                k += 1
    return P


def _Rnl(p: oracle.Params, r):
    """4 pi A w_l b_n e_l for one neighbour at distance r, shape (n, l)."""
    b, _ = oracle.radial(p, r)
    A, _ = oracle.amplitude(p, r)
    sp = p.sigma0_perp + p.alpha_perp * r
    e, _ = oracle.ilexp(r * r / (sp * sp), p.l_max)
    w = np.ones(p.l_max + 1) if p.l_weight else 2 * np.arange(p.l_max + 1) + 1.0
    return 4 * math.pi * A * np.outer(b, w * e)


P_SETS = [
    dict(n_max=6, l_max=6, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5),
    dict(n_max=8, l_max=8, r_cut=4.5, sigma0_r=0.2, sigma0_perp=0.4, alpha_r=0.08, alpha_perp=0.08, a=1.0),
    dict(n_max=8, l_max=8, r_cut=4.3, sigma0_r=0.12, sigma0_perp=0.55, alpha_r=0.14, alpha_perp=0.06, a=1.6,
         r_soft=3.8),
]


@pytest.mark.parametrize("kw", P_SETS)
def test_single_neighbour_closed_form(kw):
    # one neighbour, no central atom: p_nn'l = 4 pi (2l+1) (A w_l e_l)^2 b_n b_n', any direction
    p = oracle.Params(central_weight=0.0, **kw)
    rng = np.random.default_rng(0)
    for r in (1.3, 2.4, 3.5):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        nl = _nl_from_vectors([[r * u]])
        q, pn, c = oracle.descriptor(p, nl, np.zeros(1, np.int32), want_c=True)
        full = _unpack(p, q[0] * pn[0])
        R = _Rnl(p, r)
        want = np.einsum("al,bl->abl", R, R) * (2 * np.arange(p.l_max + 1) + 1) / (4 * math.pi)
        assert np.abs(full - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("kw", P_SETS)
def test_addition_theorem_form_many_neighbours(kw):
    # With c_nlm = sum_j R_nl(j) Y*_lm(u_j) + delta_l0 C_n, the addition theorem gives
    # p_nn'l = sum_jk R_nl(j) R_n'l(k) (2l+1)/(4 pi) P_l(u_j . u_k) (+ central terms at l = 0),
    # which uses no spherical harmonics at all.
    p = oracle.Params(**kw)
    rng = np.random.default_rng(5)
    vs = []
    while len(vs) < 9:
        v = rng.uniform(-p.r_cut, p.r_cut, 3)
        if 0.9 < np.linalg.norm(v) < p.r_cut:
            vs.append(v)
    nl = _nl_from_vectors([vs])
    q, pn = oracle.descriptor(p, nl, np.zeros(1, np.int32))
    full = _unpack(p, q[0] * pn[0])
    rs = [np.linalg.norm(v) for v in vs]
    us = [v / r for v, r in zip(vs, rs)]
    Rs = [_Rnl(p, r) for r in rs]
    want = np.zeros_like(full)
    for j in range(len(vs)):
        for k in range(len(vs)):
            Pl = special.eval_legendre(np.arange(p.l_max + 1), float(us[j] @ us[k]))
            want += np.einsum("al,bl->abl", Rs[j], Rs[k]) * (2 * np.arange(p.l_max + 1) + 1) / (4 * math.pi) * Pl
    # central atom: r = 0, e_0 = 1, Y*_00 = 1/sqrt(4 pi); amplitude 1/(sigma_0r sigma_0perp^2)
    b0, _ = oracle.radial(p, 0.0)
    C = p.central_weight * 4 * math.pi / (p.sigma0_r * p.sigma0_perp ** 2) * b0 / math.sqrt(4 * math.pi)
    S0 = sum(R[:, 0] for R in Rs) / math.sqrt(4 * math.pi)  # neighbour part of c_n00
    want[:, :, 0] += np.outer(C, S0) + np.outer(S0, C) + np.outer(C, C)
    assert np.abs(full - want).max() < 1e-12 * np.abs(want).max()


def test_projection_by_sphere_quadrature():
    # The exact projection of one separable density (Eq. (05)) on g_n Y_lm (measure dr dOmega)
    # is A b_n e^{-z} int dOmega exp(z u.Omega) Y*_lm(Omega).  The oracle with w_l = 1 must match it;
    # Eq. (08) as printed (w_l = 2l+1) is that projection times 2l+1.
    p1 = oracle.Params(n_max=5, l_max=6, r_cut=4.0, sigma0_r=0.5, sigma0_perp=0.6, central_weight=0.0,
                       l_weight=1)
    p0 = oracle.Params(n_max=5, l_max=6, r_cut=4.0, sigma0_r=0.5, sigma0_perp=0.6, central_weight=0.0)
    r = 1.7
    u = np.array([0.3, -0.5, 0.8])
    u /= np.linalg.norm(u)
    nl = _nl_from_vectors([[r * u]])
    _, _, c1 = oracle.descriptor(p1, nl, np.zeros(1, np.int32), want_c=True)
    _, _, c0 = oracle.descriptor(p0, nl, np.zeros(1, np.int32), want_c=True)
    z = r * r / 0.6 ** 2
    x, w = np.polynomial.legendre.leggauss(96)
    th = np.arccos(x)
    ph = np.linspace(0, 2 * np.pi, 192, endpoint=False)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(len(ph), 2 * np.pi / len(ph)))
    Om = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    dens = np.exp(z * (Om @ u) - z)
    b, _ = oracle.radial(p1, r)
    A, _ = oracle.amplitude(p1, r)
    for l in range(7):
        for m in range(l + 1):
            ang = np.sum(W * dens * np.conj(special.sph_harm_y(l, m, TH, PH)))
            want = A * b * ang
            k = l * (l + 1) // 2 + m
            assert np.abs(c1[0, :, k] - want).max() < 1e-12 * np.abs(c1[0]).max()
            assert np.abs(c0[0, :, k] - (2 * l + 1) * want).max() < 1e-11 * np.abs(c0[0]).max()


def _box(n, L, seed):
    return synth.rsa_box(n, L, 1.2, seed)


def test_unit_norm_and_packed_norm():
    p = oracle.Params(n_max=6, l_max=6, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5)
    s = _box(20, 7.0, 3)
    nl = oracle.neighbors(s.positions, s.cell, s.pbc, p.r_cut)
    q, pn = oracle.descriptor(p, nl, np.zeros(20, np.int32))
    assert np.allclose(np.linalg.norm(q, axis=1), 1, atol=1e-14)
    # packed dot = full (n, n', l) sum
    full = _unpack(p, q[0] * pn[0])
    assert abs(np.sum(full ** 2) - pn[0] ** 2) < 1e-12 * pn[0] ** 2


def _rot(seed):
    A = np.random.default_rng(seed).standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q *= np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


@pytest.mark.parametrize("kw", P_SETS)
def test_rotation_permutation_translation_invariance(kw):
    p = oracle.Params(**kw)
    s = _box(24, 7.5, 9)
    spec = np.zeros(24, np.int32)
    nl = oracle.neighbors(s.positions, s.cell, s.pbc, p.r_cut)
    q, _ = oracle.descriptor(p, nl, spec)
    # rotation of the whole periodic structure (positions and cell)
    Rm = _rot(4)
    nlr = oracle.neighbors(s.positions @ Rm.T, s.cell @ Rm.T, s.pbc, p.r_cut)
    qr, _ = oracle.descriptor(p, nlr, spec)
    assert np.abs(q - qr).max() < 1e-12
    # permutation of atoms
    perm = np.random.default_rng(1).permutation(24)
    nlp = oracle.neighbors(s.positions[perm], s.cell, s.pbc, p.r_cut)
    qp, _ = oracle.descriptor(p, nlp, spec)
    assert np.abs(q[perm] - qp).max() < 1e-12
    # translation (with wrap into the cell)
    pos_t = (s.positions + np.array([1.3, -2.1, 0.4])) % 7.5
    nlt = oracle.neighbors(pos_t, s.cell, s.pbc, p.r_cut)
    qt, _ = oracle.descriptor(p, nlt, spec)
    assert np.abs(q - qt).max() < 1e-12


def test_species_channels():
    # neighbours of species s feed channel block s only; the central atom feeds its own species
    p = oracle.Params(n_max=4, l_max=3, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5, n_species=2)
    s = _box(16, 6.5, 21)
    spec = (np.arange(16) % 2).astype(np.int32)
    nl = oracle.neighbors(s.positions, s.cell, s.pbc, p.r_cut)
    _, _, c = oracle.descriptor(p, nl, spec, want_c=True)
    pc = oracle.Params(n_max=4, l_max=3, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5, n_species=1,
                       central_weight=0.0)
    for i in range(4):
        for sp in (0, 1):
            sel = np.nonzero(spec[nl.j[nl.offsets[i]:nl.offsets[i + 1]]] == sp)[0] + nl.offsets[i]
            sub = oracle.NeighbourList(np.array([0]), np.array([0, len(sel)]), nl.j[sel], nl.shift[sel], nl.d[sel])
            _, _, cs = oracle.descriptor(pc, sub, np.zeros(16, np.int32), want_c=True)
            got = c[i, sp * 4:(sp + 1) * 4].copy()
            if sp == spec[i]:
                b0, _ = oracle.radial(p, 0.0)
                got[:, 0] -= 4 * math.pi / (0.5 * 0.25) * b0 / math.sqrt(4 * math.pi)
            assert np.abs(got - cs[0]).max() < 1e-12 * np.abs(c[i]).max()


def test_zero_density():
    # isolated atom without its own Gaussian: p = 0 and q = 0
    p = oracle.Params(n_max=4, l_max=3, r_cut=3.0, sigma0_r=0.5, sigma0_perp=0.5, central_weight=0.0)
    nl = _nl_from_vectors([[]])
    q, pn = oracle.descriptor(p, nl, np.zeros(1, np.int32))
    assert pn[0] == 0 and np.all(q == 0)
