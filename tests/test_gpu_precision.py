"""Mixed-precision GAP contraction vs the FP64 oracle.

In the modes fp64, f32, bf16x3 and bf16 only the two GAP contractions (S = Q Q_s^T
and Qbar = G Q_s) change arithmetic; the descriptor, its adjoint and the radial
recursion stay FP64.  Bounds, relative to the largest |e_i|, |F| and
|dE/dalpha_s|, from the operand rounding u of each mode (S = q . q_s with unit
vectors of length K; k = S^zeta):
  FP32     u = 2^-24: S relative error ~ u sqrt(K), zeta-fold in k     -> 1e-4
  split    hi + lo BF16 keeps ~17 bits: u ~ 2^-17                       -> 1e-3
  BF16     u = 2^-8 per operand (8 significant bits): S off by ~2u,
           zeta-fold in k (3e-2 at zeta = 4)                           -> 5e-2
  bf16ps   the BF16 GAP contractions, and the power spectrum (Eq. (09)) and
           its adjoint from BF16 c: a product of two rounded entries is off by
           at most ~2u, so |dp_abl| <= 2u s_ab |C_al| |C_bl| (checked entry by
           entry below); the roundings of different entries are independent,
           so q moves by ~2u, zeta-fold in k (3e-2), on top of the BF16 GAP
           part                                                        -> 1e-1
The power spectrum of bf16ps is also checked entry by entry against that
rounding bound (test_matrix_core_power_spectrum_entries).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BOUNDS = {"fp64": 1e-10, "f32": 1e-4, "bf16x3": 1e-3, "bf16": 5e-2, "bf16ps": 1e-1}


@pytest.fixture(scope="module")
def case():
    kw = dict(n_max=8, l_max=8, r_cut=5.0, sigma0_r=0.5, sigma0_perp=0.5)
    s = synth.rsa_box(300, 14.4, 1.2, 1002)
    spec = np.zeros(300, np.int32)
    p = oracle.Params(**kw)
    qs = synth.sparse_set(130, p.dim, 77)
    al = synth.sparse_weights(130, 78)
    eo, Fo, abo = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, 4)
    return kw, s, spec, qs, al, eo, Fo, abo


@pytest.mark.parametrize("prec", ["fp64", "f32", "bf16x3", "bf16", "bf16ps"])
def test_mixed_precision_bounds(case, prec):
    from paper_1905_02142_amd import Soap, SoapParams

    kw, s, spec, qs, al, eo, Fo, abo = case
    soap = Soap(SoapParams(precision=prec, **kw))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=DEV)
    nl = soap.neighbors(t(s.positions), s.cell, s.pbc)
    e, F, ab = soap.energy_forces(nl, t(spec), t(qs), t(al), 4)
    torch.cuda.synchronize()
    e, F, ab = e.cpu().numpy(), F.cpu().numpy(), ab.cpu().numpy()
    de = np.abs(e - eo).max() / np.abs(eo).max()
    dF = np.abs(F - Fo).max() / np.abs(Fo).max()
    dab = np.abs(ab - abo).max() / np.abs(abo).max()
    print(f"{prec}: rel e {de:.2e}  rel F {dF:.2e}  rel dE/dalpha {dab:.2e}  "
          f"force RMSE {np.sqrt(np.mean((F - Fo) ** 2)):.2e} (RMS F {np.sqrt(np.mean(Fo ** 2)):.2e})")
    b = BOUNDS[prec]
    assert de < b and dF < b and dab < b
    # the lower precision must still give exactly conserved total force (gather symmetry)
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max()


def test_edge_tiles_and_ragged_sizes():
    # N, M and K that are not multiples of the 64-wide tiles, zeta = 1 and 3
    from paper_1905_02142_amd import Soap, SoapParams

    kw = dict(n_max=5, l_max=3, r_cut=3.7, sigma0_r=0.5, sigma0_perp=0.5)  # K = 60
    s = synth.rsa_box(71, 9.0, 1.2, 5)
    spec = np.zeros(71, np.int32)
    p = oracle.Params(**kw)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=DEV)
    for M, zeta in ((1, 1), (65, 3), (130, 2)):
        qs = synth.sparse_set(M, p.dim, M)
        al = synth.sparse_weights(M, M + 1)
        eo, Fo, abo = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, zeta)
        for prec in ("fp64", "bf16x3"):
            soap = Soap(SoapParams(precision=prec, **kw))
            nl = soap.neighbors(t(s.positions), s.cell, s.pbc)
            e, F, ab = soap.energy_forces(nl, t(spec), t(qs), t(al), zeta)
            torch.cuda.synchronize()
            b = BOUNDS[prec]
            assert np.abs(e.cpu().numpy() - eo).max() <= b * np.abs(eo).max()
            assert np.abs(F.cpu().numpy() - Fo).max() <= b * np.abs(Fo).max()
            assert np.abs(ab.cpu().numpy() - abo).max() <= b * np.abs(abo).max()


# (n_max, l_max, n_species, atoms, box edge, seed): one 16-channel tile and its
# ragged forms, two and three tiles (the 48-channel limit, at the smallest and
# the largest n_max bucket), l_max = 12 (2l + 1 = 25 columns, two 16-wide tiles)
# and each compiled basis bucket
PS_CASES = {
    "n8l8_1sp": (8, 8, 1, 200, 12.6, 21),
    "n5l3_3sp": (5, 3, 3, 90, 9.7, 22),     # 15 channels: one ragged tile
    "n6l5_3sp": (6, 5, 3, 90, 9.7, 23),     # 18: a second, nearly empty tile
    "n8l6_3sp": (8, 6, 3, 120, 10.7, 24),   # 24 channels
    "n6l3_8sp": (6, 3, 8, 120, 10.7, 25),   # 48: three full tiles
    "n12l3_4sp": (12, 3, 4, 60, 9.0, 26),   # 48 channels in the n_max = 12 bucket
    "n10l10_1sp": (10, 10, 1, 80, 9.0, 27),
    "n12l12_1sp": (12, 12, 1, 40, 8.4, 28),
}
U_BF16 = 2.0 ** -8  # unit roundoff of BF16 (8 significant bits)


def _ab_index(a, b, nch):
    return a * nch - a * (a - 1) // 2 + (b - a)


@pytest.mark.parametrize("name", list(PS_CASES))
def test_matrix_core_power_spectrum_entries(name):
    """Every entry of the bf16ps power spectrum p = q |p| within the rounding bound
    of its two BF16 factors: |p~_abl - p_abl| <= (2u + u^2) s_ab sqrt(p_aal p_bbl)
    (s_ab = sqrt(2) off the diagonal, |C_al|^2 = p_aal / s_aa by Eq. (09)) plus the
    FP32 accumulation over 2l + 1 terms; channels of a species absent from an
    environment give exact zeros."""
    from paper_1905_02142_amd import Soap, SoapParams

    n, l, ns, N, L, seed = PS_CASES[name]
    kw = dict(n_max=n, l_max=l, r_cut=4.5, sigma0_r=0.5, sigma0_perp=0.5, n_species=ns)
    s = synth.rsa_box(N, L, 1.2, seed)
    spec = synth.draw_species(N, [1.0] * ns, seed + 1) if ns > 1 else np.zeros(N, np.int32)
    soap = Soap(SoapParams(precision="bf16ps", **kw))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=DEV)
    nl = soap.neighbors(t(s.positions), s.cell, s.pbc)
    q, pn = soap.descriptor(nl, t(spec), with_norm=True)
    torch.cuda.synchronize()
    p_dev = q.cpu().numpy() * pn.cpu().numpy()[:, None]
    onl = oracle.neighbors(s.positions, s.cell, s.pbc, kw["r_cut"])
    qo, pno = oracle.descriptor(oracle.Params(**kw), onl, spec)
    p_ref = qo * pno[:, None]
    nch, L1 = n * ns, l + 1
    a_idx, b_idx = np.triu_indices(nch)
    ab = _ab_index(a_idx, b_idx, nch)
    diag = np.array([_ab_index(a, a, nch) for a in range(nch)])
    rows = (ab[:, None] * L1 + np.arange(L1)[None, :]).ravel()
    pa = p_ref[:, (diag[a_idx][:, None] * L1 + np.arange(L1)).ravel()]
    pb = p_ref[:, (diag[b_idx][:, None] * L1 + np.arange(L1)).ravel()]
    sab = np.repeat(np.where(a_idx != b_idx, np.sqrt(2.0), 1.0), L1)
    acc = (2 * l + 1) * 2.0 ** -24
    bound = ((2 * U_BF16 + U_BF16 ** 2) * 1.01 + acc) * sab * np.sqrt(np.maximum(pa * pb, 0.0)) + 1e-12 * pno[:, None]
    err = np.abs(p_dev[:, rows] - p_ref[:, rows])
    worst = (err / bound).max()
    print(f"{name}: K {soap.dim}, max |dp| / bound {worst:.3f}, max rel q error "
          f"{np.abs(q.cpu().numpy() - qo).max():.2e}")
    assert worst <= 1.0
    assert np.all(p_dev[:, rows][pa * pb == 0.0] == 0.0)
    # |p| follows from the entries, to the same relative accuracy
    assert np.allclose(pn.cpu().numpy(), pno, rtol=4 * U_BF16, atol=0)


@pytest.mark.parametrize("name", ["n8l6_3sp", "n6l3_8sp", "n12l3_4sp", "n12l12_1sp"])
def test_matrix_core_power_spectrum_forces(name):
    # the adjoint cbar = M C on the matrix cores: 24 and 48 channels of several
    # species (contraction over channels in one and in two 32-deep steps), and one
    # species at l_max = 12
    from paper_1905_02142_amd import Soap, SoapParams

    n, l, ns, N, L, seed = PS_CASES[name]
    kw = dict(n_max=n, l_max=l, r_cut=4.5, sigma0_r=0.5, sigma0_perp=0.5, n_species=ns)
    s = synth.rsa_box(N, L, 1.2, seed)
    spec = synth.draw_species(N, [1.0] * ns, seed + 1) if ns > 1 else np.zeros(N, np.int32)
    p = oracle.Params(**kw)
    qs = synth.sparse_set(60, p.dim, seed + 2)
    al = synth.sparse_weights(60, seed + 3)
    eo, Fo, abo = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, 2)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), device=DEV)
    for prec in ("bf16", "bf16ps"):
        soap = Soap(SoapParams(precision=prec, **kw))
        nl = soap.neighbors(t(s.positions), s.cell, s.pbc)
        e, F, ab = soap.energy_forces(nl, t(spec), t(qs), t(al), 2)
        torch.cuda.synchronize()
        e, F, ab = e.cpu().numpy(), F.cpu().numpy(), ab.cpu().numpy()
        de = np.abs(e - eo).max() / np.abs(eo).max()
        dF = np.abs(F - Fo).max() / np.abs(Fo).max()
        dab = np.abs(ab - abo).max() / np.abs(abo).max()
        print(f"{prec}: rel e {de:.2e}  rel F {dF:.2e}  rel dE/dalpha {dab:.2e}")
        b = BOUNDS[prec]
        assert de < b and dF < b and dab < b
        assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max()
