"""Launch-shape tuning: every setting meets the bounds of its precision against
the oracle; in FP64, settings that differ only in block size agree bit for bit
and the others (GAP order) to rounding; a repeated call with the same setting is
bitwise identical; and the autotuner installs the setting it returns."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KW = dict(n_max=8, l_max=6, r_cut=4.5, sigma0_r=0.5, sigma0_perp=0.5)
BOUNDS = {"fp64": 1e-10, "bf16": 5e-2}
SETTINGS = [dict(gap_fused=0, gap_slices=0, prep_block=256, cell_split=2, gap_tile=0),
            dict(gap_fused=0, gap_slices=0, prep_block=64, cell_split=2, gap_tile=0),
            dict(gap_fused=1, gap_slices=256, prep_block=128, cell_split=2, gap_tile=0),
            dict(gap_fused=1, gap_slices=2048, prep_block=256, cell_split=2, gap_tile=0),
            dict(gap_fused=0, gap_slices=0, prep_block=256, cell_split=2, gap_tile=1)]


@pytest.fixture(scope="module")
def case():
    s = synth.rsa_box(400, 16.0, 1.2, 1203)
    p = oracle.Params(**KW)
    qs = synth.sparse_set(150, p.dim, 91)
    al = synth.sparse_weights(150, 92)
    spec = np.zeros(s.n_atoms, np.int32)
    eo, Fo, abo = oracle.energy_forces(p, s.positions, s.cell, s.pbc, spec, qs, al, 3)
    return s, spec, qs, al, eo, Fo, abo


def _t(a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_every_setting_within_bounds(case, prec):
    from paper_1905_02142_amd import Soap, SoapParams

    s, spec, qs, al, eo, Fo, abo = case
    soap = Soap(SoapParams(precision=prec, **KW))
    nl = soap.neighbors(_t(s.positions), s.cell, s.pbc)
    outs = []
    for t in SETTINGS:
        soap.set_tuning(**t)
        assert soap.tuning == t
        e, F, ab = soap.energy_forces(nl, _t(spec), _t(qs), _t(al), 3)
        torch.cuda.synchronize()
        e, F, ab = e.cpu().numpy(), F.cpu().numpy(), ab.cpu().numpy()
        b = BOUNDS[prec]
        assert np.abs(e - eo).max() <= b * np.abs(eo).max(), t
        assert np.abs(F - Fo).max() <= b * np.abs(Fo).max(), t
        assert np.abs(ab - abo).max() <= b * np.abs(abo).max(), t
        outs.append((e, F, ab))
    if prec == "fp64":
        for t, o in zip(SETTINGS[1:], outs[1:]):
            same_order = t["gap_fused"] == SETTINGS[0]["gap_fused"]
            for x, y in zip(o, outs[0]):
                if same_order:
                    assert np.array_equal(x, y), t
                else:
                    assert np.abs(x - y).max() <= 1e-13 * np.abs(y).max(), t
        soap.set_tuning(**SETTINGS[1])
        again = [a.cpu().numpy() for a in soap.energy_forces(nl, _t(spec), _t(qs), _t(al), 3)]
        assert all(np.array_equal(x, y) for x, y in zip(again, outs[1]))


def test_invalid_setting_rejected():
    from paper_1905_02142_amd import Soap, SoapParams, _lib

    soap = Soap(SoapParams(**KW))
    with pytest.raises(_lib.SoapError):
        soap.set_tuning(prep_block=100)
    with pytest.raises(_lib.SoapError):
        soap.set_tuning(gap_fused=2)
    with pytest.raises(_lib.SoapError):
        soap.set_tuning(cell_split=4)
    with pytest.raises(_lib.SoapError):
        soap.set_tuning(gap_tile=2)


@pytest.mark.parametrize("prec", ["bf16", "bf16ps"])
def test_gap_tile_shapes_bitwise_equal(case, prec):
    # the two BF16 tile shapes take the same products in the same order
    from paper_1905_02142_amd import Soap, SoapParams

    s, spec, qs, al, eo, Fo, abo = case
    soap = Soap(SoapParams(precision=prec, **KW))
    nl = soap.neighbors(_t(s.positions), s.cell, s.pbc)
    outs = []
    for tile in (0, 1):
        soap.set_tuning(gap_tile=tile)
        outs.append([t.cpu().numpy() for t in soap.energy_forces(nl, _t(spec), _t(qs), _t(al), 3)])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_tuning_cache_reused(case, tmp_path):
    """The first autotune with a cache attached tunes and stores one entry; a
    second context with the same parameters and inputs takes it from the file
    without timing, and installs the same setting."""
    from paper_1905_02142_amd import Soap, SoapParams, _lib

    s, spec, qs, al, eo, Fo, abo = case
    path = str(tmp_path / "tuning.txt")
    first = Soap(SoapParams(precision="bf16", **KW))
    first.set_tuning_cache(path)
    nl = first.neighbors(_t(s.positions), s.cell, s.pbc)
    chosen = first.autotune(nl, _t(spec), _t(qs), _t(al), 3, repeats=1)
    assert first.tuning_cache_hits == 0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("soap-tuning %d " % _lib.SOAP_TUNING_CACHE_VERSION)
    key = first.tuning_key(s.n_atoms, len(al))
    stored, found = _lib.soap_tuning_cache_lookup(path, key)
    assert found and stored.as_dict() == chosen
    second = Soap(SoapParams(precision="bf16", **KW))
    second.set_tuning_cache(path)
    nl2 = second.neighbors(_t(s.positions), s.cell, s.pbc)
    again = second.autotune(nl2, _t(spec), _t(qs), _t(al), 3, repeats=1)
    assert second.tuning_cache_hits == 1 and again == chosen and second.tuning == chosen
    assert open(path).read().splitlines() == lines
    # another precision is another key: tuned and stored beside the first entry
    third = Soap(SoapParams(precision="fp64", **KW))
    third.set_tuning_cache(path)
    nl3 = third.neighbors(_t(s.positions), s.cell, s.pbc)
    third.autotune(nl3, _t(spec), _t(qs), _t(al), 3, repeats=1)
    assert third.tuning_cache_hits == 0 and len(open(path).read().splitlines()) == 2


def test_autotune_neighbors():
    # times cell_split 1..3, installs the fastest and leaves the list built with it:
    # the same pair set as a build with the default setting
    from paper_1905_02142_amd import Soap, SoapParams

    s = synth.rsa_box(3000, 40.0, 1.2, 1302)
    soap = Soap(SoapParams(**KW))
    pos = _t(s.positions)
    ref = soap.neighbors(pos, s.cell, s.pbc)
    n0 = ref.n_pairs
    key0 = np.lexsort((ref.img[:n0].cpu().numpy(), ref.j[:n0].cpu().numpy(), ref.center[:n0].cpu().numpy()))
    want = np.stack([ref.center[:n0].cpu().numpy()[key0], ref.j[:n0].cpu().numpy()[key0],
                     ref.img[:n0].cpu().numpy()[key0]])
    nl = soap.neighbors(pos, s.cell, s.pbc)
    chosen = soap.autotune_neighbors(pos, s.cell, s.pbc, nl, repeats=2)
    print("cell_split chosen", chosen["cell_split"])
    assert chosen["cell_split"] in (1, 2, 3) and soap.tuning == chosen
    n = nl.n_pairs
    assert n == n0
    c, j, img = (getattr(nl, k)[:n].cpu().numpy() for k in ("center", "j", "img"))
    order = np.lexsort((img, j, c))
    assert np.array_equal(np.stack([c[order], j[order], img[order]]), want)


def test_autotune_installs_its_choice(case):
    from paper_1905_02142_amd import Soap, SoapParams

    s, spec, qs, al, eo, Fo, abo = case
    soap = Soap(SoapParams(precision="bf16", **KW))
    nl = soap.neighbors(_t(s.positions), s.cell, s.pbc)
    chosen = soap.autotune(nl, _t(spec), _t(qs), _t(al), 3, repeats=2)
    print("autotune chose", chosen)
    assert soap.tuning == chosen
    assert chosen["prep_block"] in (64, 128, 256) and chosen["gap_fused"] in (0, 1)
    assert chosen["cell_split"] == 2  # not searched: the autotuner times the GAP call on a built list
    e, F, _ = soap.energy_forces(nl, _t(spec), _t(qs), _t(al), 3)
    torch.cuda.synchronize()
    assert np.abs(F.cpu().numpy() - Fo).max() <= 5e-2 * np.abs(Fo).max()


def test_cell_split_keeps_the_pair_set():
    """Bins of r_cut, r_cut/2 and r_cut/3: the same pairs with bitwise-equal
    vectors (only their order inside each atom's list changes), a consistent
    reverse index, and energies and forces equal to rounding.  On this box the
    coarse bins take the one-launch cell list and r_cut/3 bins (more than 8192)
    the multi-launch one, so the two agree as well."""
    from paper_1905_02142_amd import Soap, SoapParams

    s = synth.rsa_box(3000, 40.0, 1.2, 1301)
    spec = np.zeros(s.n_atoms, np.int32)
    p = oracle.Params(**KW)
    qs = synth.sparse_set(100, p.dim, 93)
    al = synth.sparse_weights(100, 94)
    soap = Soap(SoapParams(**KW))
    pos = _t(s.positions)
    ref = None
    for split in (1, 2, 3):
        soap.set_tuning(cell_split=split)
        nl = soap.neighbors(pos, s.cell, s.pbc)
        n = nl.n_pairs
        c, j, img, rev = (getattr(nl, k)[:n].cpu().numpy() for k in ("center", "j", "img", "rev"))
        d = np.stack([getattr(nl, k)[:n].cpu().numpy() for k in ("dx", "dy", "dz")], 1)
        off = nl.offsets.cpu().numpy()
        assert np.array_equal(c, np.repeat(np.arange(s.n_atoms), np.diff(off)))
        assert np.array_equal(rev[rev], np.arange(n)) and np.array_equal(c[rev], j)
        assert np.array_equal(d[rev], -d)
        order = np.lexsort((img, j, c))
        e, F, ab = (t.cpu().numpy() for t in soap.energy_forces(nl, _t(spec), _t(qs), _t(al), 3))
        cur = dict(off=off, j=j[order], img=img[order], d=d[order], e=e, F=F, ab=ab)
        if ref is None:
            ref = cur
            continue
        for k in ("off", "j", "img", "d"):
            assert np.array_equal(cur[k], ref[k]), (split, k)
        for k in ("e", "F", "ab"):
            assert np.abs(cur[k] - ref[k]).max() <= 1e-13 * np.abs(ref[k]).max(), (split, k)
