"""Full-size workloads on the GPU, checked on sampled atoms against the oracle.

The oracle computes the energies and forces of a chosen set of atoms exactly
(every centre within r_cut of them is included), so each sampled atom is an
element-by-element check at the real problem size.  Whole-system properties are
checked as well: E = sum_s alpha_s dE/dalpha_s (E is linear in alpha) and zero
net force (the pair gradients enter the forces in +/- pairs).

  slab32768_3sp_n8l8   32768 atoms, half the cube at 0.1 and half at 0.02 A^-3,
                       three species (n_ch = 24, K = 2700), M = 2000, zeta = 4
  batch256_n8l6        256 independent cells of 16..2048 atoms, M = 1000, zeta = 2;
                       whole cells are compared with the oracle run on each alone
  box262144_n10l10     262144 atoms, n_max = l_max = 10, r_cut 5.5, M = 4000, zeta = 4
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _kw(w):
    return dict(n_max=w["n_max"], l_max=w["l_max"], r_cut=w["r_cut"], sigma0_r=w["sigma"], sigma0_perp=w["sigma"],
                n_species=w["n_species"])


def _run(w, precision="fp64"):
    from paper_1905_02142_amd import Soap, SoapParams

    ss = w["structures"]
    pos = np.concatenate([s.positions for s in ss])
    cells = np.stack([s.cell for s in ss])
    pbc = np.stack([s.pbc for s in ss])
    so = np.cumsum([0] + [s.n_atoms for s in ss]).astype(np.int32) if len(ss) > 1 else None
    soap = Soap(SoapParams(precision=precision, **_kw(w)))
    print(f"workload n_atoms={len(pos)} precision={precision}", flush=True)
    nl = soap.neighbors(_t(pos), cells, pbc, so)
    e, F, ab = soap.energy_forces(nl, _t(w["species"]), _t(w["q_sparse"]), _t(w["alpha"]), w["zeta"])
    torch.cuda.synchronize()
    return e.cpu().numpy(), F.cpu().numpy(), ab.cpu().numpy(), nl.n_pairs


def _whole_system_checks(w, e, F, ab):
    E = e.sum()
    assert abs((w["alpha"] * ab).sum() - E) <= 1e-11 * np.abs(w["alpha"] * ab).sum()
    assert np.abs(F.sum(0)).max() <= 1e-11 * np.abs(F).sum()


def _sampled(w, e, F, atoms, tol):
    s = w["structures"][0]
    p = oracle.Params(**_kw(w))
    eo, Fo = oracle.energy_forces_subset(p, s.positions, s.cell, s.pbc, w["species"], w["q_sparse"], w["alpha"],
                                         w["zeta"], atoms)
    de = np.abs(e[atoms] - eo).max() / np.abs(eo).max()
    dF = np.abs(F[atoms] - Fo).max() / np.abs(Fo).max()
    print(f"sampled {len(atoms)} atoms: rel e {de:.2e}, rel F {dF:.2e}")
    assert de <= tol and dF <= tol


def test_slab_three_species_sampled():
    w = synth.workload("slab32768_3sp_n8l8")
    e, F, ab, n_pairs = _run(w)
    _whole_system_checks(w, e, F, ab)
    z = w["structures"][0].positions[:, 2]
    L = w["structures"][0].cell[2, 2]
    rng = np.random.default_rng(77)
    dense = rng.choice(np.flatnonzero(z < 0.45 * L), 6, replace=False)
    sparse = rng.choice(np.flatnonzero((z > 0.55 * L) & (z < 0.95 * L)), 6, replace=False)
    edge = rng.choice(np.flatnonzero(np.abs(z - 0.5 * L) < 1.0), 4, replace=False)
    _sampled(w, e, F, np.concatenate([dense, sparse, edge]), 1e-10)


@pytest.mark.parametrize("name", ["box4096_n8l8", "slab32768_3sp_n8l8", "batch256_n8l6", "box262144_n10l10"])
def test_mixed_mode_force_rmse(name):
    # each workload's mixed-precision mode (the one its benchmark line times)
    # against the fp64 path: force RMSE at most 1e-4 eV/A, and the mode's
    # relative bound on energies and forces
    w = synth.workload(name)
    mode = w["mixed"]
    e, F, ab, _ = _run(w)
    eb, Fb, abb, _ = _run(w, mode)
    rmse = np.sqrt(np.mean((Fb - F) ** 2))
    print(f"{mode} vs fp64: force RMSE {rmse:.3e} eV/A, RMS force {np.sqrt(np.mean(F ** 2)):.3e}")
    bound = {"bf16": 5e-2, "bf16ps": 1e-1, "bf16x3": 1e-3, "f32": 1e-4}[mode]
    assert np.abs(eb - e).max() <= bound * np.abs(e).max()
    assert np.abs(Fb - F).max() <= bound * np.abs(F).max()
    assert rmse <= 1e-4


def test_batch256_whole_cells():
    w = synth.workload("batch256_n8l6")
    e, F, ab, _ = _run(w)
    _whole_system_checks(w, e, F, ab)
    ss = w["structures"]
    so = np.cumsum([0] + [s.n_atoms for s in ss])
    sizes = np.array([s.n_atoms for s in ss])
    p = oracle.Params(**_kw(w))
    for b in list(np.argsort(sizes)[:3]) + [int(np.argmax(sizes))]:
        s = ss[b]
        sl = slice(so[b], so[b + 1])
        eo, Fo, _ = oracle.energy_forces(p, s.positions, s.cell, s.pbc, w["species"][sl], w["q_sparse"], w["alpha"],
                                         w["zeta"])
        assert np.abs(e[sl] - eo).max() <= 1e-10 * np.abs(eo).max(), b
        assert np.abs(F[sl] - Fo).max() <= 1e-10 * np.abs(Fo).max(), b


def test_box262144_n10l10_sampled():
    w = synth.workload("box262144_n10l10")
    e, F, ab, n_pairs = _run(w)
    print(f"pairs {n_pairs}")
    _whole_system_checks(w, e, F, ab)
    atoms = np.random.default_rng(78).choice(len(e), 8, replace=False)
    # n_max = 10: W's entries reach ~5e6, which the double-double radial stage of
    # the fp64 mode absorbs
    _sampled(w, e, F, atoms, 1e-10)
