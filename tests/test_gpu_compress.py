"""DP-compress on the GPU (DP_FP64_TAB) against the oracle's own tabulation.

* the device-built table against the oracle's: node values, slopes and
  curvatures (c0, c1, 2 c2) and the quintics evaluated inside the intervals;
* energies, forces and virial of the tabulated model against the oracle's
  tabulated model at the FP64 bars (water192, water12k, copper32k);
* the tabulated model against the exact one: the stated tolerance of the
  tabulation (forces within 1e-9 eV/A at h = 0.1);
* the table follows parameter updates; inputs past the table's end raise
  DP_FLAG_TABLE_RANGE and hold the end value, as in the oracle;
* no parameter gradient for the tabulated model.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRIDS = {"water": I.COMPRESS_GRID_WATER, "copper": I.COMPRESS_GRID_COPPER}


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_22867_amd import dpse
    dpse.lib()
    return torch.device("cuda:0")


def _grid_of(desc):
    return GRIDS["copper" if desc.ntypes == 1 else "water"]


def _run(dev, name, mode="fp64_tab", params=None, grid=None):
    from paper_2410_22867_amd import dpse
    fr, desc, p, _ = I.workload(name)
    p = p if params is None else params
    grid = grid or _grid_of(desc)
    model = dpse.Model(desc, p)
    model.compress(*grid)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, _ = ctx.build_nlist(x, t, fr.box)
    r = ctx.compute(x, t, fr.box, nl, mode=mode, want_atom_energy=True)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    out["status"] = ctx.status()
    return fr, desc, p, grid, model, ctx, out


@pytest.mark.parametrize("name", ["water192", "copper32k"])
def test_table_matches_oracle_table(dev, name):
    from paper_2410_22867_amd import dpse
    fr, desc, p, _ = I.workload(name)
    grid = _grid_of(desc)
    _say("table", name)
    model = dpse.Model(desc, p)
    model.compress(*grid)
    g = model.table().cpu().numpy()
    o = oracle.tabulate(desc, p, *grid)
    assert g.shape == o.shape
    assert np.abs(g[:, :, 0] - o[:, :, 0]).max() <= 1e-13
    assert np.abs(g[:, :, 1] - o[:, :, 1]).max() <= 1e-12
    assert np.abs(g[:, :, 2] - o[:, :, 2]).max() <= 1e-11
    # the quintics agree inside the intervals
    rng = np.random.default_rng(0)
    h = grid[2]
    for _ in range(200):
        net, k = int(rng.integers(g.shape[0])), int(rng.integers(g.shape[1]))
        tt = rng.uniform(0, h if k < int(np.ceil(grid[0] / h)) else 10 * h)
        pw = tt ** np.arange(6)
        assert np.abs(pw @ g[net, k] - pw @ o[net, k]).max() <= 1e-13


def _tab_oracle(fr, desc, p, grid, **kw):
    return oracle.compute(fr.coords, fr.types, fr.box, desc, p, table=(oracle.tabulate(desc, p, *grid), *grid), **kw)


@pytest.mark.parametrize("name", ["water192", "water12k", "copper32k"])
def test_tabulated_model_matches_oracle(dev, name):
    fr, desc, p, grid, model, ctx, r = _run(dev, name)
    _say("fp64_tab", name, fr.n)
    o = _tab_oracle(fr, desc, p, grid)
    assert o["clipped"] == 0 and r["status"] == 0
    assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["Ei"] - o["Ei"]).max() <= 1e-10 * np.abs(o["Ei"]).max()
    assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].reshape(3, 3) - o["W"]).max() <= 1e-9 * max(1.0, np.abs(o["W"]).max())
    # against the exact model: the tabulation's own error
    e = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    ferr = np.abs(r["F"] - e["F"]).max()
    _say(name, "tabulated vs exact: F max err", ferr, "E err/atom", abs(r["E"][0] - e["E"]) / fr.n)
    assert ferr <= 1e-9
    assert abs(r["E"][0] - e["E"]) <= 1e-10 * abs(e["E"])


def test_table_follows_parameter_updates_and_range_flag(dev):
    from paper_2410_22867_amd import dpse
    fr, desc, p, grid, model, ctx, r = _run(dev, "water192")
    q = p.copy()
    off, shp = desc.param_offsets()["emb01.W2"]
    q[off:off + 500] *= 1.3
    model.load_params(torch.tensor(q, device=dev))
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, _ = ctx.build_nlist(x, t, fr.box)
    r = ctx.compute(x, t, fr.box, nl, mode="fp64_tab")
    torch.cuda.synchronize()
    o = _tab_oracle(fr, desc, q, grid)
    assert abs(r["E"].item() - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"].cpu().numpy() - o["F"]).max() <= 1e-9
    assert ctx.status() == 0
    # a table that ends below the O-H inputs: values held at its end, flagged
    short = (4.0, 8.0, 0.1)
    fr, desc, p, grid, model, ctx, r = _run(dev, "water192", grid=short)
    o = _tab_oracle(fr, desc, p, short)
    assert o["clipped"] > 0
    assert r["status"] == dpse.FLAG_TABLE_RANGE
    assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    with pytest.raises(dpse.DPError) as e:
        ctx.backward_params(torch.ones(1, dtype=torch.float64, device=dev))
    assert e.value.code == -2
