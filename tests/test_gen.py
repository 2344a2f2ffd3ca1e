"""The seeded input generators (no method arithmetic): the recipes of the
workloads -- counts, boxes, masses, densities, pressures, in-box positions,
the clustered box's halo fraction, the ensemble's box sizes -- and that a
seed fixes the output."""
import math

import numpy as np
import pytest

import gen


def _in_box(d, box):
    for a, k in enumerate(("x", "y", "z")):
        assert np.all(d[k] >= 0.0) and np.all(d[k] < box[a]), k


def test_lattice_recipe():
    d = gen.lattice(16, jitter=0.1, seed=5)
    n = 16 ** 3
    assert d["x"].size == n and d["id"].tolist() == list(range(n))
    _in_box(d, (1.0, 1.0, 1.0))
    assert np.allclose(d["m"], 1.0 / n)
    dx = 1.0 / 16
    # jitter within +-0.1 dx of the lattice sites (periodic)
    off = (d["x"] / dx - 0.5) - np.round(d["x"] / dx - 0.5)
    assert np.max(np.abs(off)) <= 0.1 + 1e-12
    assert np.allclose(d["H"], gen.GAMMA_K * gen.ETA * dx)
    e = gen.lattice(16, jitter=0.0)
    assert np.allclose(np.sort(np.unique(np.round(e["x"] / dx - 0.5, 9))), np.arange(16))


def test_sod_recipe():
    d = gen.sod(20)
    nl, nr = 20 ** 3, 10 ** 3
    assert d["x"].size == nl + nr
    _in_box(d, (2.0, 1.0, 1.0))
    left = d["x"] < 1.0
    assert left.sum() == nl
    m = d["m"][0]
    assert np.allclose(d["m"], m)
    rho_l, rho_r = nl * m / 1.0, nr * m / 1.0
    assert rho_l == pytest.approx(1.0) and rho_r == pytest.approx(0.125)
    g1 = gen.GAMMA_GAS - 1.0
    assert np.allclose(g1 * rho_l * d["u"][left], 1.0)
    assert np.allclose(g1 * rho_r * d["u"][~left], 0.1)


def test_clustered_recipe_small():
    d = gen.clustered(24, seed=7, n_halos=5)
    n = 24 ** 3
    assert d["x"].size == n
    _in_box(d, (1.0, 1.0, 1.0))
    assert np.allclose(d["m"], 1.0 / n)
    assert np.all(d["H"] > 0) and np.all(d["H"] <= 0.2)
    # clustering: the cell-count distribution is far wider than Poisson
    cells = 8
    idx = (np.floor(d["x"] * cells) * cells * cells + np.floor(d["y"] * cells) * cells
           + np.floor(d["z"] * cells)).astype(int)
    c = np.bincount(idx, minlength=cells ** 3)
    assert c.var() > 5 * c.mean()
    # the initial H follow the local density: they span a wide range
    assert d["H"].max() / d["H"].min() > 5


def test_ensemble_recipe():
    d = gen.ensemble(4, (12, 16), seed=11)
    sizes = np.bincount(d["domain"], minlength=4)
    assert len(sizes) == 4 and d["boxes"].shape == (4, 3)
    for b in range(4):
        s = round(sizes[b] ** (1.0 / 3.0))
        assert s ** 3 == sizes[b] and 12 <= s <= 16
        sel = d["domain"] == b
        assert np.allclose(d["m"][sel], 1.0 / sizes[b])
        for k in ("x", "y", "z"):
            assert np.all(d[k][sel] >= 0.0) and np.all(d[k][sel] < 1.0)


@pytest.mark.parametrize("make", [lambda s: gen.lattice(8, vsigma=0.1, seed=s),
                                  lambda s: gen.clustered(12, seed=s, n_halos=2),
                                  lambda s: gen.ensemble(2, (8, 10), seed=s)])
def test_seed_fixes_output(make):
    a, b, c = make(3), make(3), make(4)
    for k in ("x", "y", "z", "H"):
        assert np.array_equal(a[k], b[k])
    assert not all(np.array_equal(a[k], c[k]) for k in ("x", "y", "z"))
