"""Pins of the oracle's DP-compress tabulation (the compression of the
embedding net cited in the Background section): each embedding net G(x) of
its scalar input x = R~[0] becomes piecewise quintics matching G, G' and G''
at both ends of every interval of a grid.

* at every grid node the table's value, slope and curvature equal the
  network's, evaluated independently in numpy (value) and by central finite
  differences of that numpy network (slope, curvature);
* adjacent intervals join with continuous value, slope and curvature;
* the interpolation error between nodes falls as h^6 (Hermite quintic):
  halving h cuts it by ~64;
* the tabulated model's forces are minus the gradient of its own energy
  (central differences), and its energy and forces approach the exact
  model's as h shrinks;
* inputs at or beyond the table's end are counted.
"""
import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I


def _G(desc, p, ti, tj, x):
    """Embedding net in numpy (the layer rule of the Background-section
    reading: tanh layers, [h, h] identity skips on doubled widths)."""
    off = desc.param_offsets()

    def blk(name):
        o, shp = off[name]
        return p[o:o + int(np.prod(shp))].reshape(shp)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    h = np.tanh(x[:, None] * blk(f"emb{ti}{tj}.W1")[0] + blk(f"emb{ti}{tj}.b1"))
    for l in (2, 3):
        z = h @ blk(f"emb{ti}{tj}.W{l}") + blk(f"emb{ti}{tj}.b{l}")
        h = np.concatenate([h, h], axis=1) + np.tanh(z)
    return h


def _grid(x1, x2, h):
    n1 = int(np.ceil(x1 / h))
    X1 = n1 * h
    H = 10 * h
    n2 = int(np.ceil((x2 - X1) / H)) if x2 > X1 else 0
    left = np.concatenate([np.arange(n1) * h, X1 + np.arange(n2) * H])
    width = np.concatenate([np.full(n1, h), np.full(n2, H)])
    return left, width


def _poly(c, t, der=0):
    q = np.polynomial.Polynomial(c)
    for _ in range(der):
        q = q.deriv()
    return q(t)


@pytest.fixture(scope="module")
def water():
    fr, desc, p, _ = I.workload("water192")
    return fr, desc, p


def test_grid_nodes_match_the_network(water):
    fr, desc, p = water
    x1, x2, h = 14.0, 42.0, 0.1
    tab = oracle.tabulate(desc, p, x1, x2, h)
    left, width = _grid(x1, x2, h)
    assert tab.shape == (4, len(left), 6, desc.m1)
    rng = np.random.default_rng(0)
    e = 1e-4
    for net in range(4):
        ti, tj = divmod(net, 2)
        ks = rng.choice(len(left), 12, replace=False)
        for k in ks:
            c = tab[net, k]                      # [6, m1]
            xl = left[k]
            g0 = _G(desc, p, ti, tj, xl)[0]
            gp = _G(desc, p, ti, tj, xl + e)[0]
            gm = _G(desc, p, ti, tj, xl - e)[0]
            assert np.allclose(c[0], g0, rtol=0, atol=1e-13)
            assert np.allclose(c[1], (gp - gm) / (2 * e), rtol=0, atol=1e-7)
            assert np.allclose(2 * c[2], (gp - 2 * g0 + gm) / (e * e), rtol=0, atol=2e-5)
            # the right end of the interval is the next node
            g1 = _G(desc, p, ti, tj, xl + width[k])[0]
            assert np.allclose([_poly(c[:, a], width[k]) for a in range(desc.m1)], g1, rtol=0, atol=1e-12)


def test_adjacent_intervals_join_smoothly(water):
    fr, desc, p = water
    x1, x2, h = 14.0, 42.0, 0.1
    tab = oracle.tabulate(desc, p, x1, x2, h)
    left, width = _grid(x1, x2, h)
    for k in (0, 57, len(left) // 2, int(np.ceil(x1 / h)) - 1, len(left) - 2):
        for d in range(3):
            a = np.array([_poly(tab[1, k, :, f], width[k], d) for f in range(desc.m1)])
            b = np.array([_poly(tab[1, k + 1, :, f], 0.0, d) for f in range(desc.m1)])
            assert np.allclose(a, b, rtol=1e-9, atol=1e-9 * 10 ** d), (k, d)


def test_interpolation_error_falls_as_h6(water):
    fr, desc, p = water
    x = np.random.default_rng(1).uniform(0.5, 13.0, 400)
    exact = _G(desc, p, 0, 1, x)
    errs = []
    for h in (0.4, 0.2):
        tab = oracle.tabulate(desc, p, 14.0, 14.0, h)
        k = np.floor(x / h).astype(int)
        t = x - k * h
        approx = np.stack([[_poly(tab[1, kk, :, a], tt) for a in range(desc.m1)] for kk, tt in zip(k, t)])
        errs.append(np.abs(approx - exact).max())
    ratio = errs[0] / errs[1]
    assert 30 < ratio < 130, (errs, ratio)


def test_compressed_model_forces_are_its_gradient(water):
    fr, desc, p = water
    tabspec = (oracle.tabulate(desc, p, 14.0, 42.0, 0.1), 14.0, 42.0, 0.1)
    r = oracle.compute(fr.coords, fr.types, fr.box, desc, p, table=tabspec)
    assert r["clipped"] == 0
    rng = np.random.default_rng(4)
    hfd = 1e-3
    for _ in range(10):
        i, a = int(rng.integers(fr.n)), int(rng.integers(3))
        E = []
        for k in (-2, -1, 1, 2):
            x = fr.coords.copy()
            x[i, a] += k * hfd
            E.append(oracle.compute(x, fr.types, fr.box, desc, p, table=tabspec, use_cells=False)["E"])
        dE = (E[0] - 8 * E[1] + 8 * E[2] - E[3]) / (12 * hfd)
        assert abs(-dE - r["F"][i, a]) < 1e-7, (i, a, -dE, r["F"][i, a])
    assert np.abs(r["F"].sum(0)).max() < 1e-12 * fr.n
    assert np.allclose(r["W"], r["W"].T, atol=1e-12)


def test_compressed_model_converges_to_exact(water):
    fr, desc, p = water
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    prev = None
    for h in (0.4, 0.2, 0.1):
        r = oracle.compute(fr.coords, fr.types, fr.box, desc, p, table=(oracle.tabulate(desc, p, 14.0, 42.0, h),
                                                                        14.0, 42.0, h))
        ferr = np.abs(r["F"] - o["F"]).max()
        if prev is not None:
            assert ferr < prev / 8
        prev = ferr
    assert prev < 1e-10
    assert abs(r["E"] - o["E"]) < 1e-11 * abs(o["E"])


def test_inputs_beyond_the_table_are_counted(water):
    fr, desc, p = water
    tab = oracle.tabulate(desc, p, 4.0, 8.0, 0.1)    # ends at x = 8, below the O-H bond inputs
    r = oracle.compute(fr.coords, fr.types, fr.box, desc, p, table=(tab, 4.0, 8.0, 0.1), debug=True)
    x = r["R"][:, :, 0][r["nlist"] >= 0]
    assert r["clipped"] == int((x >= 8.0).sum()) > 0
