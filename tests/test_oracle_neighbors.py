"""Pins of the oracle's brute-force neighbour list (the cutoff sphere of Sec. I)."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth


def test_matches_periodic_kdtree_large_box():
    # box wider than 2 r_cut: each neighbour is a single image, scipy's periodic KD-tree applies
    s = synth.rsa_box(300, 15.0, 1.2, 2)
    rc = 5.0
    nl = oracle.neighbors(s.positions, s.cell, s.pbc, rc)
    tree = cKDTree(s.positions, boxsize=15.0)
    pairs = tree.query_pairs(rc - 1e-12, output_type="ndarray")
    want = set()
    for i, j in pairs:
        want.add((i, j))
        want.add((j, i))
    got = set(zip(nl.centre_of_pair().tolist(), nl.j.tolist()))
    assert got == want
    assert nl.n_pairs == len(want)


def test_small_box_images_match_supercell():
    # box narrower than 2 r_cut: count neighbours of each atom in an explicit 5x5x5 supercell
    s = synth.rsa_box(6, 5.2, 1.2, 12)
    rc = 5.5
    nl = oracle.neighbors(s.positions, s.cell, s.pbc, rc)
    L = 5.2
    shifts = np.array([(a, b, c) for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3)], float) * L
    for i in range(6):
        d = (s.positions[None, :, :] + shifts[:, None, :] - s.positions[i]).reshape(-1, 3)
        r = np.linalg.norm(d, axis=1)
        want = np.sort(r[(r > 0) & (r < rc)])
        got = np.sort(np.linalg.norm(nl.d[nl.offsets[i]:nl.offsets[i + 1]], axis=1))
        assert np.allclose(got, want, rtol=0, atol=1e-12)
    # self-images appear (the box is smaller than the cutoff sphere)
    assert np.any(nl.j == nl.centre_of_pair())


def test_pairs_are_symmetric():
    s = synth.rsa_box(40, 7.0, 1.2, 3)
    nl = oracle.neighbors(s.positions, s.cell, s.pbc, 3.9)
    fwd = set(zip(nl.centre_of_pair().tolist(), nl.j.tolist(), map(tuple, nl.shift.tolist())))
    for i, j, t in fwd:
        assert (j, i, (-t[0], -t[1], -t[2])) in fwd


def test_triclinic_cell_images():
    # a sheared cell: compare with an explicit supercell count
    cell = np.array([[6.0, 0.0, 0.0], [2.5, 5.5, 0.0], [1.0, -1.5, 6.2]])
    rng = np.random.default_rng(4)
    frac = rng.random((8, 3))
    pos = frac @ cell
    rc = 4.0
    nl = oracle.neighbors(pos, cell, np.ones(3, np.int32), rc)
    rng_ = range(-3, 4)
    T = np.array([(a, b, c) for a in rng_ for b in rng_ for c in rng_], float) @ cell
    for i in range(8):
        d = (pos[None, :, :] + T[:, None, :] - pos[i]).reshape(-1, 3)
        r = np.linalg.norm(d, axis=1)
        want = np.sort(r[(r > 0) & (r < rc)])
        got = np.sort(np.linalg.norm(nl.d[nl.offsets[i]:nl.offsets[i + 1]], axis=1))
        assert len(got) == len(want) and np.allclose(got, want, atol=1e-12)
