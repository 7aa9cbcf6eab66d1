"""torch.autograd bindings: gradients against the oracle and central finite differences.

The energy is E = sum_i sum_s alpha_s (q_i . q_s)^zeta; its position gradient is
-F and its alpha gradient sum_i (q_i . q_s)^zeta.  The finite-difference checks
keep every displacement small enough that no pair crosses r_cut (the pair count
is asserted unchanged), where the descriptor is smooth.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KW = dict(n_max=6, l_max=5, r_cut=4.2, sigma0_r=0.5, sigma0_perp=0.5, n_species=2)


def _setup(n_atoms=48, box=8.2, seed=31, M=40, zeta=3):
    from paper_1905_02142_amd import Soap, SoapParams

    s = synth.rsa_box(n_atoms, box, 1.2, seed)
    spec = synth.draw_species(n_atoms, (0.6, 0.4), seed + 1).astype(np.int32)
    p = oracle.Params(**KW)
    qs = synth.sparse_set(M, p.dim, seed + 2)
    al = synth.sparse_weights(M, seed + 3)
    soap = Soap(SoapParams(**KW))
    return soap, s, spec, qs, al, zeta, p


def _t(a, dtype=None, grad=False):
    t = torch.tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)
    return t.requires_grad_(grad)


def _pairs(soap, pos, s):
    return soap.neighbors(pos.detach(), s.cell, s.pbc).n_pairs


def test_gap_energy_gradients_match_oracle():
    from paper_1905_02142_amd.autograd import gap_energy

    soap, s, spec, qs, al, zeta, p = _setup()
    pos = _t(s.positions, grad=True)
    alpha = _t(al, grad=True)
    E = gap_energy(soap, pos, alpha, _t(spec, torch.int32), _t(qs), zeta, s.cell, s.pbc)
    E.backward()
    eo, Fo, abo = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, zeta)
    assert abs(E.item() - eo.sum()) <= 1e-10 * np.abs(eo).sum()
    gp = pos.grad.cpu().numpy()
    ga = alpha.grad.cpu().numpy()
    assert np.abs(gp + Fo).max() <= 1e-10 * np.abs(Fo).max()
    assert np.abs(ga - abo).max() <= 1e-10 * np.abs(abo).max()


def test_gap_energy_central_differences():
    from paper_1905_02142_amd.autograd import gap_energy

    soap, s, spec, qs, al, zeta, _ = _setup(seed=37)
    sp, qst = _t(spec, torch.int32), _t(qs)
    pos = _t(s.positions, grad=True)
    alpha = _t(al, grad=True)
    gap_energy(soap, pos, alpha, sp, qst, zeta, s.cell, s.pbc).backward()
    n0 = _pairs(soap, pos, s)

    def energy(x, a):
        with torch.no_grad():
            return gap_energy(soap, x, a, sp, qst, zeta, s.cell, s.pbc).item()

    rng = np.random.default_rng(5)
    h = 1e-4
    for atom, ax in zip(rng.integers(0, s.n_atoms, 6), rng.integers(0, 3, 6)):
        xp, xm = pos.detach().clone(), pos.detach().clone()
        xp[atom, ax] += h
        xm[atom, ax] -= h
        assert _pairs(soap, xp, s) == n0 and _pairs(soap, xm, s) == n0
        fd = (energy(xp, alpha.detach()) - energy(xm, alpha.detach())) / (2 * h)
        an = pos.grad[atom, ax].item()
        assert abs(fd - an) <= 1e-6 * pos.grad.abs().max().item() + 1e-9 * abs(an), (atom, ax, fd, an)
    # E is linear in alpha: central differences are exact up to rounding
    for k in rng.integers(0, len(al), 4):
        ap, am = alpha.detach().clone(), alpha.detach().clone()
        ap[k] += 0.5
        am[k] -= 0.5
        fd = energy(pos.detach(), ap) - energy(pos.detach(), am)
        assert abs(fd - alpha.grad[k].item()) <= 1e-10 * alpha.grad.abs().max().item()


def test_descriptor_vjp_directional_derivatives():
    from paper_1905_02142_amd.autograd import descriptor

    soap, s, spec, _, _, _, _ = _setup(n_atoms=40, seed=43)
    sp = _t(spec, torch.int32)
    pos = _t(s.positions, grad=True)
    q = descriptor(soap, pos, sp, s.cell, s.pbc)
    w = torch.tensor(np.random.default_rng(7).standard_normal(tuple(q.shape)), device=DEV)
    (q * w).sum().backward()
    n0 = _pairs(soap, pos, s)
    rng = np.random.default_rng(8)
    h = 1e-5
    for _ in range(3):
        d = torch.tensor(rng.standard_normal((s.n_atoms, 3)), device=DEV)
        xp, xm = pos.detach() + h * d, pos.detach() - h * d
        assert _pairs(soap, xp, s) == n0 and _pairs(soap, xm, s) == n0
        with torch.no_grad():
            lp = (descriptor(soap, xp, sp, s.cell, s.pbc) * w).sum().item()
            lm = (descriptor(soap, xm, sp, s.cell, s.pbc) * w).sum().item()
        fd = (lp - lm) / (2 * h)
        an = (pos.grad * d).sum().item()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_descriptor_gradcheck_tiny():
    from paper_1905_02142_amd import Soap, SoapParams
    from paper_1905_02142_amd.autograd import descriptor

    kw = dict(n_max=3, l_max=2, r_cut=3.0, sigma0_r=0.5, sigma0_perp=0.5)
    soap = Soap(SoapParams(**kw))
    # an isolated cluster in a large box: the pair set cannot change under small moves
    rng = np.random.default_rng(11)
    pos = np.array([[5.0, 5.0, 5.0], [6.3, 5.2, 5.1], [5.4, 6.4, 4.8], [4.9, 5.3, 6.35]]) + 0.05 * rng.standard_normal((4, 3))
    cell = np.eye(3) * 20.0
    pbc = np.ones(3, dtype=np.int32)
    sp = _t(np.zeros(4, np.int32))
    x = _t(pos, grad=True)
    f = lambda y: descriptor(soap, y, sp, cell, pbc)
    assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-7, rtol=1e-5)
