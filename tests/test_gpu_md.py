"""Verlet-skin neighbour lists and the graph-replayed MD step.

- A list built to r_cut + skin gives the energies and forces of a list built
  to r_cut: the extra pairs weigh exactly zero, and only the order of the
  per-atom sums differs.
- GapMD runs NVE dynamics with a descriptor that is C^1 at r_cut: the list is
  rebuilt only when atoms have moved far enough, every step is one graph
  replay, the forces at the end equal those of a fresh list at the final
  positions, and the total energy stays constant to the integrator's accuracy.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# the amplitude exponent a = 2 takes the density and its slope to zero at r_cut
# (Eq. (15)), so the energy is C^1 where pairs enter and leave the cutoff
KW = dict(n_max=6, l_max=6, r_cut=4.5, r_soft=3.8, sigma0_r=0.3, sigma0_perp=0.5, a=2.0)


def _t(a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _model(soap, M=60, seed=31, scale=1.0):
    qs = synth.sparse_set(M, soap.dim, seed)
    al = synth.sparse_weights(M, seed + 1) * scale
    return _t(qs), _t(al)


def _oracle_check(positions, cell, pbc, qs, al, zeta, e, F, tol=1e-10):
    """Energies and forces at these positions against the oracle (an exact r_cut list)."""
    n = len(positions)
    eo, Fo, _ = oracle.energy_forces(oracle.Params(**KW), positions, cell, pbc, np.zeros(n, np.int32),
                                     qs.cpu().numpy(), al.cpu().numpy(), zeta)
    de = np.abs(e - eo).max() / np.abs(eo).max()
    dF = np.abs(F - Fo).max() / np.abs(Fo).max()
    print(f"vs oracle: rel e {de:.2e}, rel F {dF:.2e}")
    assert de <= tol and dF <= tol


def test_skin_list_gives_the_same_results():
    from paper_1905_02142_amd import Soap, SoapParams

    s = synth.rsa_box(300, 14.4, 1.2, 41)
    sp = _t(np.zeros(s.n_atoms, np.int32))
    ref = Soap(SoapParams(**KW))
    qs, al = _model(ref)
    nl0 = ref.neighbors(_t(s.positions), s.cell, s.pbc)
    e0, F0, ab0 = (t.cpu().numpy() for t in ref.energy_forces(nl0, sp, qs, al, 3))
    q0 = ref.descriptor(nl0, sp).cpu().numpy()
    sk = Soap(SoapParams(**KW))
    sk.set_neighbor_skin(1.0)
    nl1 = sk.neighbors(_t(s.positions), s.cell, s.pbc)
    assert nl1.n_pairs > 1.5 * nl0.n_pairs
    e1, F1, ab1 = (t.cpu().numpy() for t in sk.energy_forces(nl1, sp, qs, al, 3))
    q1 = sk.descriptor(nl1, sp).cpu().numpy()
    for a, b in ((q1, q0), (e1, e0), (F1, F0), (ab1, ab0)):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    _oracle_check(s.positions, s.cell, s.pbc, qs, al, 3, e1, F1)
    from paper_1905_02142_amd import _lib
    with pytest.raises(_lib.SoapError):
        sk.set_neighbor_skin(-0.1)


def test_pair_vector_refresh_matches_a_fresh_list():
    """After the atoms move by less than skin / 2, refreshing the pair vectors of
    the old skin list gives every pair of a fresh build the same vector bit for
    bit, and the same energies and forces to rounding."""
    from paper_1905_02142_amd import Soap, SoapParams

    s = synth.rsa_box(300, 14.4, 1.2, 44)
    sp = _t(np.zeros(s.n_atoms, np.int32))
    soap = Soap(SoapParams(**KW))
    qs, al = _model(soap)
    soap.set_neighbor_skin(0.6)
    nl = soap.neighbors(_t(s.positions), s.cell, s.pbc)
    moved = s.positions + np.random.default_rng(45).uniform(-0.1, 0.1, s.positions.shape)
    soap.update_pair_vectors(nl, _t(moved))
    fresh = Soap(SoapParams(**KW))
    fresh.set_neighbor_skin(0.6)
    nl2 = fresh.neighbors(_t(moved), s.cell, s.pbc)

    def table(n):
        P = n.n_pairs
        key = zip(n.center[:P].tolist(), n.j[:P].tolist(), n.img[:P].tolist())
        d = np.stack([n.dx[:P].cpu().numpy(), n.dy[:P].cpu().numpy(), n.dz[:P].cpu().numpy()], 1)
        return dict(zip(key, d))

    old, new = table(nl), table(nl2)
    for k, v in new.items():
        if np.linalg.norm(v) < KW["r_cut"]:  # every pair inside the cutoff is in the old list, same bits
            assert np.array_equal(old[k], v), k
    e1, F1, _ = (t.cpu().numpy() for t in soap.energy_forces(nl, sp, qs, al, 3))
    ref = Soap(SoapParams(**KW))
    nl0 = ref.neighbors(_t(moved), s.cell, s.pbc)
    e0, F0, _ = (t.cpu().numpy() for t in ref.energy_forces(nl0, sp, qs, al, 3))
    assert np.abs(e1 - e0).max() <= 1e-12 * np.abs(e0).max()
    assert np.abs(F1 - F0).max() <= 1e-12 * np.abs(F0).max()
    _oracle_check(moved, s.cell, s.pbc, qs, al, 3, e1, F1)


def test_md_rebuilds_replays_and_conserves_energy():
    from paper_1905_02142_amd import Soap, SoapParams
    from paper_1905_02142_amd.md import GapMD

    s = synth.rsa_box(200, 12.6, 1.5, 42)
    n = s.n_atoms
    soap = Soap(SoapParams(**KW))
    qs, al = _model(soap, scale=20.0)
    sp = _t(np.zeros(n, np.int32))
    rng = np.random.default_rng(43)
    masses = _t(np.full(n, 12.0))
    v = rng.standard_normal((n, 3)) * 0.01  # A/fs, roughly 1000 K for carbon
    v -= v.mean(axis=0)
    md = GapMD(soap, _t(s.positions), masses, s.cell, s.pbc, sp, qs, al, 3, dt=0.25, skin=0.3,
               velocities=_t(v))
    ep0, ek0 = md.energies()
    tot = []
    for _ in range(40):
        md.step(10)
        ep, ek = md.energies()
        tot.append(ep + ek)
    torch.cuda.synchronize()
    print("rebuilds", md.rebuilds, "repeated chunks", md.repeated_chunks, "host syncs", md.host_syncs,
          "E0", ep0 + ek0, "drift", max(abs(x - (ep0 + ek0)) for x in tot), "Ek0", ek0)
    assert md.steps == 400 and md.rebuilds >= 2
    # one host read-back per chunk of check_every steps, plus one per step of a repeated chunk
    assert md.host_syncs <= md.steps // md.check_every + md.check_every * md.repeated_chunks
    # energy: constant to well below the kinetic energy's scale
    assert max(abs(x - (ep0 + ek0)) for x in tot) <= 2e-3 * ek0
    # forces at the end equal those of a fresh exact-cutoff list at the final positions
    ref = Soap(SoapParams(**KW))
    nl = ref.neighbors(md.pos.clone(), s.cell, s.pbc)
    _, F, _ = ref.energy_forces(nl, sp, qs, al, 3)
    F, Fm = F.cpu().numpy(), md.F.cpu().numpy()
    assert np.abs(Fm - F).max() <= 1e-10 * np.abs(F).max()
    # and the oracle's at the same positions
    _oracle_check(md.pos.cpu().numpy(), s.cell, s.pbc, qs, al, 3, md.e.cpu().numpy(), Fm)
