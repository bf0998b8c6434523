"""Degenerate inputs through the C ABI, FP64 against the oracle.

* an empty frame (n = 0), alone and inside a batch;
* a single atom (no neighbours: D = 0, the fitting net's value at zero);
* a dilute frame whose atoms have 0-4 neighbours: isolated atoms of both
  types, a pair inside r_s (s = 1/r branch), a pair at r_s, a pair just
  inside and a pair just outside r_c, a group wrapped across the periodic
  corner, a short chain -- so every embedding tile is almost all padding;
* frames holding one type only (the other type's sections and nets empty).

Bars as for the full frames: energy 1e-10 relative (absolute 1e-12 eV where
the energy is near zero), forces 1e-9 eV/A, virial 1e-9 eV; neighbour lists
bit-exact.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


@pytest.fixture(scope="module")
def water():
    from paper_2410_22867_amd import dpse
    desc = I.WATER
    p = I.init_params(desc, I.MODEL_SEED_WATER)
    model = dpse.Model(desc, p)
    return desc, p, model


def dilute_frame() -> I.Frame:
    """Groups on a 10 A grid in a 40 A cube (groups farther than r_c = 6 A
    apart, periodic images included)."""
    L = 40.0
    rs, rc = I.WATER.rcut_smth, I.WATER.rcut
    atoms = [
        ((5.0, 5.0, 5.0), 0),                       # isolated O
        ((15.0, 5.0, 5.0), 1),                      # isolated H
        ((25.0, 5.0, 5.0), 0), ((25.3, 5.0, 5.0), 1),           # r = 0.3 < r_s
        ((35.0, 5.0, 5.0), 1), ((35.0, 5.0 + rc - 1e-3, 5.0), 1),  # just inside r_c
        ((5.0, 15.0, 5.0), 0), ((5.0, 15.0, 5.0 + rc + 1e-3), 0),  # just outside r_c
        ((15.0, 15.0, 5.0), 0), ((15.0 + rs, 15.0, 5.0), 1),     # r = r_s
        ((25.0, 25.0, 25.0), 0), ((26.1, 25.6, 25.2), 1), ((27.0, 26.5, 25.9), 1),
        ((28.2, 27.1, 26.0), 0), ((29.0, 28.3, 26.4), 1),        # chain
        ((0.2, 0.2, 0.2), 0), ((39.7, 0.3, 0.1), 1), ((0.1, 39.8, 39.9), 1),  # corner
        ((5.0, 35.0, 25.0), 1), ((5.9, 35.4, 25.3), 1), ((4.4, 35.7, 24.6), 0),
    ]
    x = np.array([a[0] for a in atoms], dtype=np.float64)
    t = np.array([a[1] for a in atoms], dtype=np.int32)
    return I.Frame(coords=np.mod(x, L), types=t, box=np.diag([L, L, L]))


def _run(dev, model, fr, mode="fp64", ctx=None):
    from paper_2410_22867_amd import dpse
    ctx = ctx or dpse.Context(model, max(fr.n, 1))
    x = torch.tensor(fr.coords.reshape(-1, 3), dtype=torch.float64, device=dev)
    t = torch.tensor(fr.types, dtype=torch.int32, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    r = ctx.compute(x, t, fr.box, nl, mode=mode, want_atom_energy=True)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    out["nl"] = nl.cpu().numpy()
    out["ov"] = int(ov.cpu().item())
    out["status"] = ctx.status()
    return out


def _check_fp64(r, o, n):
    e_tol = max(1e-10 * abs(o["E"]), 1e-12)
    assert abs(r["E"][0] - o["E"]) <= e_tol
    if n:
        assert np.abs(r["Ei"] - o["Ei"]).max() <= max(1e-10 * np.abs(o["Ei"]).max(), 1e-12)
        assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].reshape(3, 3) - o["W"]).max() <= 1e-9


@pytest.mark.parametrize("mode", ["fp64", "bf16", "fp16", "mix_fp32", "mix_fp16"])
def test_empty_frame(dev, water, mode):
    desc, p, model = water
    _say("empty frame", mode)
    fr = I.Frame(coords=np.zeros((0, 3)), types=np.zeros(0, np.int32), box=np.diag([20.0, 20.0, 20.0]))
    r = _run(dev, model, fr, mode)
    assert r["nl"].shape == (0, desc.nm)
    assert r["ov"] == 0
    assert r["E"][0] == 0.0
    assert np.all(r["W"] == 0.0)
    assert r["status"] == 0


@pytest.mark.parametrize("ty", [0, 1])
def test_single_atom(dev, water, ty):
    desc, p, model = water
    _say("single atom", ty)
    fr = I.Frame(coords=np.array([[3.0, 4.0, 5.0]]), types=np.array([ty], np.int32), box=np.diag([20.0, 20.0, 20.0]))
    r = _run(dev, model, fr)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    assert np.all(r["nl"] == -1)
    _check_fp64(r, o, fr.n)
    assert np.all(r["F"] == 0.0)
    assert r["status"] == 0


def test_dilute_frame_fp64(dev, water):
    desc, p, model = water
    fr = dilute_frame()
    _say("dilute frame", fr.n)
    r = _run(dev, model, fr)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    assert r["ov"] == 0
    assert np.array_equal(r["nl"], o["nlist"])
    cnt = (o["nlist"] >= 0).sum(1)
    assert cnt.min() == 0 and cnt.max() <= 4
    _check_fp64(r, o, fr.n)
    assert np.abs(r["F"].sum(0)).max() < 1e-9
    assert r["status"] == 0


@pytest.mark.parametrize("mode,tol", [("bf16", 0.05), ("fp16", 0.01), ("mix_fp32", 1e-5), ("mix_fp16", 0.01)])
def test_dilute_frame_mixed(dev, water, mode, tol):
    desc, p, model = water
    fr = dilute_frame()
    _say("dilute frame", mode)
    r = _run(dev, model, fr, mode)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    assert np.array_equal(r["nl"], o["nlist"])
    assert abs(r["E"][0] - o["E"]) <= tol * np.abs(o["Ei"]).sum()
    assert np.abs(r["F"] - o["F"]).max() <= tol * max(1.0, np.abs(o["F"]).max())
    assert np.isfinite(r["W"]).all()
    assert r["status"] == 0


@pytest.mark.parametrize("ty", [0, 1])
def test_one_type_only(dev, water, ty):
    desc, p, model = water
    fr0 = I.water_box(27, 14.0, seed=21)
    fr = I.Frame(coords=fr0.coords, types=np.full(fr0.n, ty, np.int32), box=fr0.box)
    _say("one type only", ty, fr.n)
    r = _run(dev, model, fr)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    assert np.array_equal(r["nl"], o["nlist"])
    _check_fp64(r, o, fr.n)
    assert r["status"] == 0


def test_batch_with_empty_frames(dev, water):
    """Frames: empty, dilute, single atom, empty, small water box, empty."""
    from paper_2410_22867_amd import dpse
    desc, p, model = water
    L0 = np.diag([20.0, 20.0, 20.0])
    frames = [I.Frame(np.zeros((0, 3)), np.zeros(0, np.int32), L0),
              dilute_frame(),
              I.Frame(np.array([[1.0, 2.0, 3.0]]), np.array([1], np.int32), L0),
              I.Frame(np.zeros((0, 3)), np.zeros(0, np.int32), L0),
              I.water_box(32, 10.5, seed=22),
              I.Frame(np.zeros((0, 3)), np.zeros(0, np.int32), L0)]
    off = np.cumsum([0] + [f.n for f in frames]).astype(np.int64)
    _say("batch with empty frames", [f.n for f in frames])
    ctx = dpse.Context(model, int(off[-1]), max_frames=len(frames))
    x = torch.tensor(np.concatenate([f.coords.reshape(-1, 3) for f in frames]), device=dev)
    t = torch.tensor(np.concatenate([f.types for f in frames]), device=dev)
    boxes = np.stack([f.box for f in frames])
    nl, ov = ctx.build_nlist_batch(x, t, boxes, off)
    r = ctx.compute_batch(x, t, boxes, off, nl, mode="fp64")
    torch.cuda.synchronize()
    assert int(ov.item()) == 0
    nl = nl.cpu().numpy()
    E = r["E"].cpu().numpy()
    F = r["F"].cpu().numpy()
    W = r["W"].cpu().numpy().reshape(-1, 3, 3)
    for f, fr in enumerate(frames):
        a0, a1 = off[f], off[f + 1]
        if fr.n == 0:
            assert E[f] == 0.0 and np.all(W[f] == 0.0)
            continue
        o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
        gl = nl[a0:a1].copy()
        m = gl >= 0
        gl[m] = (gl[m] // 27 - a0) * 27 + gl[m] % 27
        assert np.array_equal(gl, o["nlist"])
        assert abs(E[f] - o["E"]) <= max(1e-10 * abs(o["E"]), 1e-12)
        assert np.abs(F[a0:a1] - o["F"]).max() <= 1e-9
        assert np.abs(W[f] - o["W"]).max() <= 1e-9
    assert ctx.status() == 0


def test_types_changed_in_place_need_new_list(dev, water):
    """The column order by type is kept across computes on a list this
    context built; rebuilding the list into the same buffers after the
    types changed in place re-sorts, and a list from elsewhere always
    re-sorts."""
    from paper_2410_22867_amd import dpse
    desc, p, model = water
    fr = I.water_box(32, 10.5, seed=23)
    _say("types changed in place", fr.n)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    ctx.compute(x, t, fr.box, nl)
    ctx.compute(x, t, fr.box, nl)
    types2 = fr.types.copy()
    types2[::3] = 1 - types2[::3]
    t.copy_(torch.tensor(types2, device=dev))
    nl2, ov2 = ctx.build_nlist(x, t, fr.box, out=nl, overflow=ov)
    assert nl2.data_ptr() == nl.data_ptr()
    r = ctx.compute(x, t, fr.box, nl2, want_atom_energy=True)
    torch.cuda.synchronize()
    o = oracle.compute(fr.coords, types2, fr.box, desc, p)
    assert np.array_equal(nl2.cpu().numpy(), o["nlist"])
    rr = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    _check_fp64(rr, o, fr.n)
    # a list uploaded from the oracle (not built by this context)
    ext = torch.tensor(o["nlist"], device=dev)
    r = ctx.compute(x, t, fr.box, ext, want_atom_energy=True)
    torch.cuda.synchronize()
    rr = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    _check_fp64(rr, o, fr.n)
    assert ctx.status() == 0


def test_candidate_capacity_flag(dev, water):
    """More than 256 pairs within r_c per atom with sum(sel) = 138: the
    search and the Verlet format (which then keep 256 pairs in LDS) raise the
    capacity flag instead of writing past their buffers."""
    from paper_2410_22867_amd import dpse
    desc, p, model = water
    rng = np.random.default_rng(31)
    L = 12.5
    pts = []
    while len(pts) < 620:  # ~0.32 atoms per cubic angstrom, pairs at least 0.8 A apart
        q = rng.random(3) * L
        if all(np.linalg.norm((q - o + L / 2) % L - L / 2) > 0.8 for o in pts[-400:]):
            pts.append(q)
    fr = I.Frame(coords=np.array(pts), types=(np.arange(len(pts)) % 3 == 0).astype(np.int32) ^ 1,
                 box=np.diag([L, L, L]))
    _say("capacity flag", fr.n)
    for verlet in (False, True):
        ctx = dpse.Context(model, fr.n)
        x = torch.tensor(fr.coords, device=dev)
        t = torch.tensor(fr.types, device=dev)
        if verlet:
            ctx.skin_build(x, t, fr.box, 0.5)
            nl, ov = ctx.skin_format(x, t)
        else:
            nl, ov = ctx.build_nlist(x, t, fr.box)
        torch.cuda.synchronize()
        assert ctx.status() & dpse.FLAG_CAND_CAPACITY


def test_two_lists_one_context_and_list_rewritten_in_place(dev, water):
    """Two lists of the same size built on one context, then computes on each
    in turn (the reverse-entry index must follow the list in use), and a list
    buffer whose contents are replaced in place between computes: every
    compute matches the oracle of its own frame."""
    from paper_2410_22867_amd import dpse
    desc, p, model = water
    fa = I.water_box(64, 12.42, seed=41)
    fb = I.water_box(64, 12.42, seed=42)
    _say("two lists on one context", fa.n)
    ctx = dpse.Context(model, fa.n)
    xa = torch.tensor(fa.coords, device=dev)
    xb = torch.tensor(fb.coords, device=dev)
    t = torch.tensor(fa.types, device=dev)
    oa = oracle.compute(fa.coords, fa.types, fa.box, desc, p)
    ob = oracle.compute(fb.coords, fb.types, fb.box, desc, p)
    nla, _ = ctx.build_nlist(xa, t, fa.box)
    nlb, _ = ctx.build_nlist(xb, t, fb.box)
    for x, nl, o in ((xa, nla, oa), (xb, nlb, ob), (xa, nla, oa), (xb, nlb, ob)):
        r = ctx.compute(x, t, fa.box, nl, want_atom_energy=True)
        torch.cuda.synchronize()
        _check_fp64({k: v.cpu().numpy() for k, v in r.items() if v is not None}, o, fa.n)
    # same buffer, new contents written behind the context's back
    nl, _ = ctx.build_nlist(xa, t, fa.box)
    ctx.compute(xa, t, fa.box, nl)
    nl.copy_(torch.tensor(ob["nlist"], device=dev))
    r = ctx.compute(xb, t, fb.box, nl, want_atom_energy=True)
    torch.cuda.synchronize()
    _check_fp64({k: v.cpu().numpy() for k, v in r.items() if v is not None}, ob, fb.n)
    assert ctx.status() == 0
