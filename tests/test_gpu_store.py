"""Stored versus recomputed embedding activations (Computation Optimization
section: activations are kept when memory allows).  The context's workspace
budget decides per call whether the last embedding layer's output is kept
from the forward pass; both paths must match the FP64 oracle to the same bars
and each other to rounding."""
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BIG = 1 << 36


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


def _run(ctx, fr, dev, mode):
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    r = ctx.compute(x, t, fr.box, nl, mode=mode, want_atom_energy=True)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    assert int(ov.cpu().item()) == 0
    return out


def _bytes_per_atom(desc, esize):
    tiles = sum((s + 15) // 16 for s in desc.sel)
    return tiles * 16 * desc.m1 * esize


def _fp64_bars(r, o, n):
    assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].reshape(3, 3) - o["W"]).max() <= 1e-9 * max(1.0, np.abs(o["W"]).max())
    assert np.abs(r["Ei"] - o["Ei"]).max() <= 1e-10 * np.abs(o["Ei"]).max()


@pytest.mark.parametrize("name", ["water", "copper"])
def test_fp64_stored_matches_oracle_and_recompute(dev, name):
    from paper_2410_22867_amd import dpse
    if name == "water":
        fr, desc, p, _ = I.workload("water192")
    else:
        desc = I.COPPER
        p = I.init_params(desc, 11)
        fr = I.copper_fcc(5, 3.634, 0.1, seed=5)   # 500 atoms, 18.17 A box
    _say("store fp64", name, fr.n)
    model = dpse.Model(desc, p)
    cs = dpse.Context(model, fr.n, budget_bytes=BIG)
    cr = dpse.Context(model, fr.n, budget_bytes=0)
    cap = cs.store_info()[0]
    assert cap == fr.n * _bytes_per_atom(desc, 8)
    assert cr.store_info() == (0, False, False)
    rs = _run(cs, fr, dev, "fp64")
    assert cs.store_info()[1] is True
    rr = _run(cr, fr, dev, "fp64")
    assert cr.store_info()[1] is False
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    _fp64_bars(rs, o, fr.n)
    _fp64_bars(rr, o, fr.n)
    assert np.abs(rs["F"] - rr["F"]).max() <= 1e-12 * max(1.0, np.abs(rr["F"]).max())
    assert abs(rs["E"][0] - rr["E"][0]) <= 1e-13 * abs(rr["E"][0])


@pytest.mark.parametrize("mode", ["bf16", "fp16"])
def test_mixed_modes_recompute(dev, mode):
    """The mixed forms recompute whatever the budget (their half-precision
    layer is cheaper than the store's memory traffic)."""
    from paper_2410_22867_amd import dpse
    fr, desc, p, _ = I.workload("water192")
    _say("store", mode)
    model = dpse.Model(desc, p)
    cs = dpse.Context(model, fr.n, budget_bytes=BIG)
    r = _run(cs, fr, dev, mode)
    assert cs.store_info()[1] is False
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    assert np.sqrt(((r["F"] - o["F"]) ** 2).mean()) < 0.1 * np.sqrt((o["F"] ** 2).mean())
    _run(cs, fr, dev, "fp64")
    assert cs.store_info()[1] is True


def test_budget_decides_per_call(dev):
    """A budget that holds 192 atoms: the 192-atom frame stores, the 375-atom
    frame on the same context recomputes; both meet the FP64 bars."""
    from paper_2410_22867_amd import dpse
    small, desc, p, _ = I.workload("water192")
    large = I.water_box(125, 15.53, seed=3)
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, large.n, budget_bytes=small.n * _bytes_per_atom(desc, 8))
    _say("budget per call", small.n, large.n)
    r = _run(ctx, small, dev, "fp64")
    assert ctx.store_info()[1] is True
    _fp64_bars(r, oracle.compute(small.coords, small.types, small.box, desc, p), small.n)
    r = _run(ctx, large, dev, "fp64")
    assert ctx.store_info()[1] is False
    ol = oracle.compute(large.coords, large.types, large.box, desc, p)
    _fp64_bars(r, ol, large.n)
    r = _run(ctx, small, dev, "fp64")
    assert ctx.store_info()[1] is True
