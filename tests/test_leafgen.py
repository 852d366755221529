"""Seeded synthetic inputs: determinism, anatomy fractions, vacuum rows where
the solver requires them, and material recipes."""
import numpy as np
import pytest

import leafgen as LG
from leafgen import geometry as G, materials as M


def test_dicot_deterministic_and_fractions():
    a = G.dicot(512, 1024, 200.0, 5)
    b = G.dicot(512, 1024, 200.0, 5)
    assert np.array_equal(a, b)
    assert a.max() <= 6            # healthy: no hyphae
    frac = np.bincount(a.ravel(), minlength=8) / a.size
    assert frac[G.D_CHL] > 0.05 and frac[G.D_CUT] > 0.005
    c = G.dicot(512, 1024, 200.0, 6)
    assert not np.array_equal(a, c)


def test_dicot_spongy_air_and_chloroplast_fill():
    L = G.DicotLayers()
    dx = 100.0
    lab = G.dicot(1024, 2048, dx, 11)
    ny = lab.shape[0]
    top = (ny * dx * 1e-3 + L.thickness) / 2
    spo_top = top - L.cuticle - L.upper_epidermis - L.palisade
    rows = slice(int((spo_top - L.spongy) / (dx * 1e-3)) + 5, int(spo_top / (dx * 1e-3)) - 5)
    air = (lab[rows] == 0).mean()
    assert 0.2 < air < 0.4                         # ~30 % air gaps
    mes = slice(rows.start, int((spo_top + L.palisade) / (dx * 1e-3)) - 5)
    chl = (lab[mes] == G.D_CHL).mean()
    assert 0.15 < chl < 0.25                       # ~20 % of the mesophyll


def test_diseased_adds_hyphae_only_near_top():
    h = G.dicot(512, 1024, 200.0, 5)
    d = G.dicot(512, 1024, 200.0, 5, diseased=True)
    diff = h != d
    assert diff.any()
    assert (d[diff] == G.D_HYP).all()
    rows = np.nonzero(diff.any(axis=1))[0]
    assert rows.min() > lab_mid(h)


def lab_mid(lab):
    return lab.shape[0] // 2


def test_monocot_labels():
    m = G.monocot(512, 1024, 40.0, 3)
    assert set(np.unique(m)) <= set(range(7))
    assert (m == G.M_VASC).any() and (m == G.M_CHL).any()


@pytest.mark.parametrize("make", [lambda: LG.configs.slab_config(),
                                  lambda: LG.configs.dicot_config(512, 1024, 200.0, 100),
                                  lambda: LG.configs.monocot_config(256, 512, 100),
                                  lambda: LG.configs.batched_config([400, 1000], 100, scale=0.25)])
def test_config_rows_are_vacuum(make):
    for inst in make():
        lab = inst.labels
        assert inst.j_trn < inst.j_src < inst.j_ref < inst.ny - inst.n_pml
        assert (lab[: inst.j_trn + 1] == 0).all() and (lab[inst.j_src:] == 0).all()
        assert lab.max() < inst.nk.shape[0]
        assert (inst.nk[0] == (1.0, 0.0)).all()


def test_batched_uneven_sizes():
    insts = LG.configs.batched_config([400, 700, 1000], 10, scale=0.25)
    sizes = {(i.nx, i.ny) for i in insts}
    assert len(sizes) == 6
    big = max(i.cells for i in insts)
    small = min(i.cells for i in insts)
    assert big / small > 5


def test_material_recipes():
    n, k = M.chloroplast(662e-9)
    assert n == 1.36 and k == pytest.approx(0.02 + 1e-5, rel=1e-3)
    assert M.chloroplast(900e-9)[1] == pytest.approx(1e-5, rel=1e-3)
    assert M.hypha(400e-9) == (1.7, pytest.approx(0.3))
    assert M.hypha(1000e-9)[1] == pytest.approx(0.05)
    assert M.cytoplasm(550e-9)[0] == pytest.approx(1.33)
    nk = M.dicot_nk(550e-9)
    assert nk.shape == (8, 2) and (nk[:, 0] ** 2 - nk[:, 1] ** 2 >= 1).all()
