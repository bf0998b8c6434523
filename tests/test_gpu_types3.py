"""Three atom types through the whole path: a water box of 2731 molecules
(8193 atoms) with every tenth oxygen given a third type (its own neighbour
section, nets and fitting net), so that nine embedding nets share the
launches (their work-groups apportioned among the nets by their work), the
first fitting layer sums three T sections, and every size threshold of the
full frames is crossed (one-row and per-net grids, the fused half-precision
first layer).  Checked through the C ABI against the FP64 oracle: FP64 at
the full-frame bars, the mixed forms at their force bars."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# force RMS error bars relative to the force RMS, as for the full frames
REL_F = {"bf16": 2e-2, "fp16": 4e-3, "mix_fp32": 2e-5, "mix_fp16": 4e-3}

_state = {}

DESC3 = dataclasses.replace(I.WATER, ntypes=3, sel=(46, 92, 24), masses=(I.MASS_O, I.MASS_H, 22.99))


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_22867_amd import dpse
    dpse.lib()
    dev = torch.device("cuda:0")
    nmol = 2731
    fr = I.water_box(nmol, I.water_density_box(nmol), seed=23)
    types = fr.types.copy()
    oxy = np.nonzero(types == 0)[0]
    types[oxy[::10]] = 2
    fr = I.Frame(fr.coords, types.astype(np.int32), fr.box)
    p = I.init_params(DESC3, 131, I.WATER_OUTPUT_SCALE)
    o = oracle.compute(fr.coords, fr.types, fr.box, DESC3, p)
    model = dpse.Model(DESC3, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    torch.cuda.synchronize()
    assert int(ov.item()) == 0
    return fr, o, ctx, x, t, nl


def _run(case, mode):
    fr, o, ctx, x, t, nl = case
    r = ctx.compute(x, t, fr.box, nl, mode=mode, want_atom_energy=True)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    return {k: v.cpu().numpy() for k, v in r.items()}


def test_three_types_fp64(case):
    fr, o = case[0], case[1]
    _say("three types fp64", fr.n, np.bincount(fr.types))
    r = _run(case, "fp64")
    assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].reshape(3, 3) - o["W"]).max() <= 1e-9 * max(1.0, np.abs(o["W"]).max())
    assert np.abs(r["Ei"] - o["Ei"]).max() <= 1e-10 * np.abs(o["Ei"]).max()


@pytest.mark.parametrize("mode", ["bf16", "fp16", "mix_fp32", "mix_fp16"])
def test_three_types_mixed(case, mode):
    fr, o = case[0], case[1]
    r = _run(case, mode)
    f_rms = np.sqrt(((r["F"] - o["F"]) ** 2).mean())
    f_scale = np.sqrt((o["F"] ** 2).mean())
    e_err = abs(r["E"][0] - o["E"]) / fr.n
    # the third type's atoms alone (their own nets and fitting net)
    t2 = fr.types == 2
    f_rms2 = np.sqrt(((r["F"][t2] - o["F"][t2]) ** 2).mean())
    _say("three types", mode, "F rms err", f_rms, "of", f_scale, "type-2 atoms", f_rms2, "E err/atom", e_err)
    assert f_rms <= REL_F[mode] * f_scale
    assert f_rms2 <= 2 * REL_F[mode] * f_scale
    assert e_err <= 5e-3


@pytest.mark.parametrize("mode", ["fp64", "bf16", "mix_fp32"])
def test_type_absent_from_large_frame(case, mode):
    """The oxygens of an 8200-molecule water box alone under the two-type
    water model: every column's hydrogen section is empty and the hydrogen
    centre type has no atoms, so two of the four nets have no columns and
    the other two one empty section each, on a frame large enough for the
    one-row grids and the fused first layer."""
    from paper_2410_22867_amd import dpse
    if "o_only" not in _state:
        dev = torch.device("cuda:0")
        nmol = 8200
        w = I.water_box(nmol, I.water_density_box(nmol), seed=29)
        keep = np.nonzero(w.types == 0)[0]
        fr = I.Frame(np.ascontiguousarray(w.coords[keep]), np.zeros(len(keep), np.int32), w.box)
        p = I.init_params(I.WATER, I.MODEL_SEED_WATER, I.WATER_OUTPUT_SCALE)
        o = oracle.compute(fr.coords, fr.types, fr.box, I.WATER, p)
        model = dpse.Model(I.WATER, p)
        ctx = dpse.Context(model, fr.n)
        x = torch.tensor(fr.coords, device=dev)
        t = torch.tensor(fr.types, device=dev)
        nl, ov = ctx.build_nlist(x, t, fr.box)
        torch.cuda.synchronize()
        assert int(ov.item()) == 0
        _state["o_only"] = (fr, o, ctx, x, t, nl)
    fr, o, ctx, x, t, nl = _state["o_only"]
    _say("type absent", mode, fr.n)
    r = _run(_state["o_only"], mode)
    if mode == "fp64":
        assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
        assert np.abs(r["F"] - o["F"]).max() <= 1e-9
        assert np.abs(r["Ei"] - o["Ei"]).max() <= 1e-10 * np.abs(o["Ei"]).max()
    else:
        f_rms = np.sqrt(((r["F"] - o["F"]) ** 2).mean())
        f_scale = np.sqrt((o["F"] ** 2).mean())
        _say("type absent", mode, "F rms err", f_rms, "of", f_scale)
        assert f_rms <= REL_F[mode] * f_scale
        assert abs(r["E"][0] - o["E"]) / fr.n <= 5e-3
