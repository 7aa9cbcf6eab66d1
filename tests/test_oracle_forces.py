"""Pins of the oracle's GAP energy (Sec. "Cohesive energy model") and of its analytic forces."""
import numpy as np
import pytest

import oracle
import synth


def test_gap_zeta_one_is_gemv():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((7, 30))
    qs = synth.sparse_set(11, 30, 1)
    al = rng.standard_normal(11)
    e, qbar, abar = oracle.gap(q, qs, al, 1)
    assert np.allclose(e, q @ (qs.T @ al), rtol=1e-13, atol=1e-14)
    assert np.allclose(qbar, np.tile(qs.T @ al, (7, 1)), rtol=1e-13, atol=1e-14)


def test_gap_self_similarity():
    # a sparse point equal to the descriptor has kernel value 1 for any zeta
    q = synth.sparse_set(3, 20, 5)
    for zeta in (1, 2, 3, 4):
        e, _, _ = oracle.gap(q[:1], q[:1], np.array([2.5]), zeta)
        assert abs(e[0] - 2.5) < 1e-14


@pytest.mark.parametrize("zeta", [2, 3, 4])
def test_gap_gradients_by_finite_differences(zeta):
    rng = np.random.default_rng(zeta)
    q = synth.sparse_set(4, 25, 7)
    qs = synth.sparse_set(9, 25, 8)
    al = rng.standard_normal(9)
    e, qbar, abar = oracle.gap(q, qs, al, zeta)
    h = 1e-6
    for i in range(4):
        for k in (0, 7, 24):
            qp = q.copy()
            qm = q.copy()
            qp[i, k] += h
            qm[i, k] -= h
            fd = (oracle.gap(qp, qs, al, zeta)[0][i] - oracle.gap(qm, qs, al, zeta)[0][i]) / (2 * h)
            assert abs(qbar[i, k] - fd) < 1e-8
    # E is linear in alpha: dE/dalpha_s is an exact difference
    for s in range(9):
        a2 = al.copy()
        a2[s] += 1.0
        assert abs(oracle.gap(q, qs, a2, zeta)[0].sum() - e.sum() - abar[s]) < 1e-12


def _energy(p, pos, cell, pbc, spec, qs, al, zeta):
    nl = oracle.neighbors(pos, cell, pbc, p.r_cut)
    q, _ = oracle.descriptor(p, nl, spec)
    return oracle.gap(q, qs, al, zeta, want_grad=False)[0].sum()


def _min_gap_to_cutoff(pos, cell, pbc, rc):
    nl = oracle.neighbors(pos, cell, pbc, rc + 0.05)
    r = np.linalg.norm(nl.d, axis=1)
    return np.min(np.abs(r - rc))


FORCE_SETS = [
    # a = 1: density amplitude and its derivative vanish at r_cut (Eq. (15))
    (dict(n_max=5, l_max=4, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5, a=1.0), 1, 3),
    # the paper's optimised new-SOAP parameters (Sec. "Cohesive energy model")
    (dict(n_max=6, l_max=5, r_cut=4.5, sigma0_r=0.2, sigma0_perp=0.4, alpha_r=0.08, alpha_perp=0.08, a=1.0), 1, 3),
    # buffer zone, r-dependent widths, two species
    (dict(n_max=4, l_max=4, r_cut=4.3, r_soft=3.6, sigma0_r=0.12, sigma0_perp=0.55, alpha_r=0.14,
          alpha_perp=0.06, a=1.6, n_species=2), 2, 3),
    # no downscaling (a = 0): FD steps kept away from r_cut
    (dict(n_max=6, l_max=6, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5), 1, 4),
]


@pytest.mark.parametrize("kw,nspec,zeta", FORCE_SETS)
def test_forces_match_finite_differences(kw, nspec, zeta):
    p = oracle.Params(**kw)
    s = synth.rsa_box(10, 6.0, 1.2, 31)  # L < 2 r_cut: several images of one atom are neighbours
    spec = (np.arange(10) % nspec).astype(np.int32)
    h = 1e-4
    assert _min_gap_to_cutoff(s.positions, s.cell, s.pbc, p.r_cut) > 4 * h
    qs = synth.sparse_set(12, p.dim, 77)
    al = synth.sparse_weights(12, 78)
    e, F, abar = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, zeta)
    fd = np.zeros_like(F)
    for i in range(10):
        for x in range(3):
            def E(dx):
                pos = s.positions.copy()
                pos[i, x] += dx
                return _energy(p, pos, s.cell, s.pbc, spec, qs, al, zeta)
            d1 = (E(h) - E(-h)) / (2 * h)
            d2 = (E(h / 2) - E(-h / 2)) / h
            fd[i, x] = -(4 * d2 - d1) / 3
    assert np.abs(F - fd).max() < 1e-7 * np.abs(F).max()
    # periodic structure: sum of forces vanishes
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max()


def test_isolated_cluster_zero_net_force_and_torque():
    p = oracle.Params(n_max=6, l_max=6, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5, a=1.0)
    s = synth.rsa_box(14, 6.0, 1.2, 44)
    pbc = np.zeros(3, np.int32)
    spec = np.zeros(14, np.int32)
    qs = synth.sparse_set(10, p.dim, 3)
    al = synth.sparse_weights(10, 4)
    _, F, _ = oracle.energy_forces(p, s.positions, s.cell, pbc, spec, qs, al, 4)
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-12 * scale
    tau = np.cross(s.positions - s.positions.mean(0), F).sum(0)
    assert np.abs(tau).max() < 1e-11 * scale * 6.0


def test_force_subset_matches_full():
    p = oracle.Params(n_max=5, l_max=4, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5)
    s = synth.rsa_box(60, 9.0, 1.2, 8)
    spec = np.zeros(60, np.int32)
    qs = synth.sparse_set(8, p.dim, 1)
    al = synth.sparse_weights(8, 2)
    e, F, _ = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, 2)
    atoms = np.array([3, 17, 41])
    es, Fs = oracle.energy_forces_subset(p, s.positions, s.cell, s.pbc, spec, qs, al, 2, atoms)
    assert np.allclose(Fs, F[atoms], rtol=0, atol=1e-13 * np.abs(F).max())
    assert np.allclose(es, e[atoms], rtol=1e-14, atol=0)
