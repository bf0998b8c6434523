"""Verlet (skin) neighbour list on the GPU (Evaluation section: lists rebuilt
every 50 steps with a 2 A skin) against the oracle's brute-force list.

The formatted list must equal, bit for bit, the plain all-pairs definition
on the current (possibly unwrapped) positions as long as no atom has moved
more than half the skin since the build; beyond that the device raises a
flag.  Forces computed with the formatted list (which also supplies the
reverse-entry index of the force gather) must meet the FP64 bars."""
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SKIN = 2.0


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


def _case(name):
    if name == "water192":
        fr, desc, p, _ = I.workload("water192")
    elif name == "water192_sel":  # sections too short: truncation counted on every format
        import dataclasses
        fr, _, _, _ = I.workload("water192")
        desc = dataclasses.replace(I.WATER, sel=(10, 20))
        p = I.init_params(desc, 1)
    elif name == "water375":
        desc = I.WATER
        p = I.init_params(desc, 7)
        fr = I.water_box(125, 15.53, seed=3)
    else:
        desc = I.COPPER
        p = I.init_params(desc, 11)
        fr = I.copper_fcc(5, 3.634, 0.1, seed=5)
    return fr, desc, p


def _displace(fr, max_disp, seed):
    """Seeded displacements of length < max_disp in random directions; some
    atoms leave [0, L) (positions are not wrapped between builds)."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(fr.n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d *= rng.uniform(0.0, max_disp, size=(fr.n, 1))
    return fr.coords + d


@pytest.mark.parametrize("name", ["water192", "water192_sel", "water375", "copper500"])
def test_format_equals_brute_force(dev, name):
    from paper_2410_22867_amd import dpse
    fr, desc, p = _case(name)
    _say("verlet", name, fr.n)
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    ctx.skin_build(x, t, fr.box, SKIN)
    nl, ov = ctx.skin_format(x, t)
    ref, rov = oracle.nlist(fr.coords, fr.types, fr.box, desc, use_cells=False)
    assert np.array_equal(nl.cpu().numpy(), ref)
    assert int(ov.cpu().item()) == rov
    assert (rov > 0) == (name == "water192_sel")
    cell, _ = ctx.build_nlist(x, t, fr.box)
    assert np.array_equal(cell.cpu().numpy(), ref)
    # drift by up to 0.95 * skin/2, across the box faces, no rebuild
    xd = _displace(fr, 0.95 * SKIN / 2, seed=17)
    assert ((xd < 0) | (xd >= np.diag(fr.box))).any()
    x.copy_(torch.tensor(xd))
    nl, ov = ctx.skin_format(x, t)
    ref, rov = oracle.nlist(xd, fr.types, fr.box, desc, use_cells=False)
    assert np.array_equal(nl.cpu().numpy(), ref)
    assert int(ov.cpu().item()) == rov
    r = ctx.compute(x, t, fr.box, nl, want_atom_energy=True)
    torch.cuda.synchronize()
    o = oracle.compute(xd, fr.types, fr.box, desc, p, use_cells=False)
    assert abs(r["E"].item() - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"].cpu().numpy() - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].cpu().numpy().reshape(3, 3) - o["W"]).max() <= 1e-9 * max(1.0, np.abs(o["W"]).max())
    assert ctx.status() & ~dpse.FLAG_SEL_OVERFLOW == 0


def test_exact_ties_perfect_lattice(dev):
    """A perfect FCC lattice: every coordination shell is a set of exactly
    equal r^2 (12, 6, 24, ... pairs), so the sections' order rests on the
    tie-break by packed index j*27 + image code.  The cell-list build, the
    Verlet build + format and the FP64 compute must all reproduce the
    oracle's brute-force list and results."""
    from paper_2410_22867_amd import dpse
    desc = I.COPPER
    p = I.init_params(desc, 13)
    fr = I.copper_fcc(6, 3.634, 0.0, seed=0)
    _say("ties", fr.n)
    ref, rov = oracle.nlist(fr.coords, fr.types, fr.box, desc, use_cells=False)
    assert rov == 0
    # the premise: row 0 holds many exactly equal distances
    L = np.diag(fr.box)
    j, sc = ref[0][ref[0] >= 0] // 27, ref[0][ref[0] >= 0] % 27
    s = np.stack([sc % 3 - 1, (sc // 3) % 3 - 1, sc // 9 - 1], axis=1)
    d = (fr.coords[j] - fr.coords[0]) + s * L
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    assert len(np.unique(r2)) < len(r2) // 4
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    cell, ov = ctx.build_nlist(x, t, fr.box)
    assert np.array_equal(cell.cpu().numpy(), ref)
    assert int(ov.cpu().item()) == 0
    ctx.skin_build(x, t, fr.box, SKIN)
    nl, ov = ctx.skin_format(x, t)
    assert np.array_equal(nl.cpu().numpy(), ref)
    assert int(ov.cpu().item()) == 0
    r = ctx.compute(x, t, fr.box, nl, want_atom_energy=True)
    torch.cuda.synchronize()
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p, use_cells=False)
    assert abs(r["E"].item() - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"].cpu().numpy() - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].cpu().numpy().reshape(3, 3) - o["W"]).max() <= 1e-9 * max(1.0, np.abs(o["W"]).max())
    assert ctx.status() == 0


def test_skin_exceeded_flag_and_rebuild(dev):
    from paper_2410_22867_amd import dpse
    fr, desc, p = _case("water192")
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    img = torch.zeros((fr.n, 3), dtype=torch.int32, device=dev)
    ctx.skin_build(x, t, fr.box, SKIN, images=img)
    xd = fr.coords.copy()
    xd[5, 0] += 0.6 * SKIN          # one atom beyond half the skin
    xd[7] += np.diag(fr.box) * np.array([1.0, -2.0, 0.0]) + 0.01
    x.copy_(torch.tensor(xd))
    ctx.skin_format(x, t)
    assert ctx.status() & dpse.FLAG_SKIN_EXCEEDED
    # a rebuild wraps in place (image counters record it) and clears the condition
    ctx.skin_build(x, t, fr.box, SKIN, images=img)
    nl, ov = ctx.skin_format(x, t)
    xw = x.cpu().numpy()
    L = np.diag(fr.box)
    assert ((xw >= 0) & (xw < L)).all()
    assert np.allclose(xw + img.cpu().numpy() * L, xd, rtol=0, atol=1e-12)
    assert np.array_equal(img.cpu().numpy(), np.floor(xd / L).astype(np.int32))
    assert img.cpu().numpy()[7].tolist()[1] == -2
    ref, _ = oracle.nlist(xw, fr.types, fr.box, desc, use_cells=False)
    assert np.array_equal(nl.cpu().numpy(), ref)
    assert ctx.status() & dpse.FLAG_SKIN_EXCEEDED == 0


def test_full_size_water12k_matches_cell_list(dev):
    from paper_2410_22867_amd import dpse
    fr, desc, p, _ = I.workload("water12k")
    _say("verlet water12k")
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    ctx.skin_build(x, t, fr.box, SKIN)
    nl, _ = ctx.skin_format(x, t)
    ref, _ = oracle.nlist(fr.coords, fr.types, fr.box, desc)
    assert np.array_equal(nl.cpu().numpy(), ref)
    xd = _displace(fr, 0.95 * SKIN / 2, seed=23)
    x.copy_(torch.tensor(xd))
    nl, _ = ctx.skin_format(x, t)
    rows = np.random.default_rng(4).choice(fr.n, 256, replace=False)
    ref, _ = oracle.nlist(xd, fr.types, fr.box, desc, rows=rows, use_cells=False)
    assert np.array_equal(nl.cpu().numpy()[rows], ref)
    assert ctx.status() & ~dpse.FLAG_SEL_OVERFLOW == 0


def test_format_requires_build(dev):
    from paper_2410_22867_amd import dpse
    fr, desc, p = _case("water192")
    ctx = dpse.Context(dpse.Model(desc, p), fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    with pytest.raises(dpse.DPError) as e:
        ctx.skin_format(x, t)
    assert e.value.code == -8
    ctx.skin_build(x, t, fr.box, SKIN)
    with pytest.raises(dpse.DPError):
        ctx.skin_format(x[:10], t[:10])
    with pytest.raises(dpse.DPError) as e:
        ctx.skin_build(x, t, fr.box, 7.0)   # r_c + skin = 13 A > 12.42 A edge
    assert e.value.code == -2
