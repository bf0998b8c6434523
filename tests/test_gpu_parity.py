"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars (FP64): neighbour lists bit-exact; energy 1e-10 relative; forces
1e-9 eV/A max abs; virial 1e-9 eV; intermediate buffers (environment matrix,
T, D, dE/dD, dE/dR) to 1e-11 relative of their scale.  Mixed precision:
errors stated per result and bounded loosely here (the bench reports them).
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


_cache = {}


def _setup(name, dev, max_atoms=None):
    from paper_2410_22867_amd import dpse
    if name in _cache:
        return _cache[name]
    fr, desc, p, dt = I.workload(name)
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, max_atoms or fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    _cache[name] = (fr, desc, p, model, ctx, x, t)
    return _cache[name]


def _gpu_nlist(ctx, x, t, box):
    nl, ov = ctx.build_nlist(x, t, box)
    torch.cuda.synchronize()
    return nl.cpu().numpy(), int(ov.cpu().item())


@pytest.mark.parametrize("name", ["water192", "water12k", "copper32k", "water98k"])
def test_nlist_bit_exact(dev, name):
    fr, desc, p, model, ctx, x, t = _setup(name, dev)
    _say("nlist", name, fr.n)
    g, gov = _gpu_nlist(ctx, x, t, fr.box)
    if fr.n <= 40000:
        o, oov = oracle.nlist(fr.coords, fr.types, fr.box, desc)
        assert gov == oov == 0
        assert np.array_equal(g, o)
    else:
        rows = np.random.default_rng(0).choice(fr.n, 2000, replace=False)
        o, _ = oracle.nlist(fr.coords, fr.types, fr.box, desc, rows=rows)
        assert gov == 0
        assert np.array_equal(g[rows], o)
    assert ctx.status() == 0


def test_nlist_small_boxes_and_overflow(dev):
    """One and two cells per dimension (images of the same atom), and section
    overflow (truncation keeps the nearest, counted)."""
    import dataclasses
    from paper_2410_22867_amd import dpse
    for fr, desc in [(I.copper_fcc(3, 3.634, 0.1, seed=7), I.COPPER),
                     (I.water_box(64, 12.42, seed=11), I.WATER),
                     (I.water_box(64, 12.42, seed=12), dataclasses.replace(I.WATER, sel=(10, 20)))]:
        _say("nlist small", fr.n, desc.sel)
        model = dpse.Model(desc, I.init_params(desc, 1))
        ctx = dpse.Context(model, fr.n)
        x = torch.tensor(fr.coords, device=dev)
        t = torch.tensor(fr.types, device=dev)
        g, gov = _gpu_nlist(ctx, x, t, fr.box)
        o, oov = oracle.nlist(fr.coords, fr.types, fr.box, desc)
        assert gov == oov
        assert np.array_equal(g, o)
        flags = ctx.status()
        assert bool(flags & dpse.FLAG_SEL_OVERFLOW) == (oov > 0)


def _compute(ctx, x, t, box, mode):
    from paper_2410_22867_amd import dpse
    nl, ov = ctx.build_nlist(x, t, box)
    r = ctx.compute(x, t, box, nl, mode=mode, want_atom_energy=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items() if v is not None}


def test_fp64_water192_all_stages(dev):
    from paper_2410_22867_amd import dpse
    fr, desc, p, model, ctx, x, t = _setup("water192", dev)
    _say("fp64 water192")
    r = _compute(ctx, x, t, fr.box, "fp64")
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p, debug=True)
    nl = o["nlist"]
    real = nl >= 0
    env = ctx.copy_buffer(dpse.BUF_ENV).cpu().numpy().reshape(fr.n, desc.nm, 4)
    assert np.allclose(env, o["R"], rtol=1e-13, atol=1e-13)
    T = ctx.copy_buffer(dpse.BUF_T).cpu().numpy().reshape(fr.n, desc.m1, 4)
    assert np.abs(T - o["T"]).max() <= 1e-11 * np.abs(o["T"]).max()
    D = ctx.copy_buffer(dpse.BUF_D).cpu().numpy().reshape(fr.n, -1)
    assert np.abs(D - o["D"]).max() <= 1e-11 * np.abs(o["D"]).max()
    gD = ctx.copy_buffer(dpse.BUF_GD).cpu().numpy().reshape(fr.n, -1)
    assert np.abs(gD - o["gD"]).max() <= 1e-10 * np.abs(o["gD"]).max()
    nd = ctx.copy_buffer(dpse.BUF_NETD).cpu().numpy().reshape(fr.n, desc.nm, 4)
    assert np.abs(nd[real] - o["netd"][real]).max() <= 1e-10 * np.abs(o["netd"]).max()
    assert np.allclose(r["Ei"], o["Ei"], rtol=0, atol=1e-10 * np.abs(o["Ei"]).max())
    assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].reshape(3, 3) - o["W"]).max() <= 1e-9
    assert ctx.status() == 0


_ocache = {}


def _oracle_full(name, fr, desc, p):
    if name not in _ocache:
        _ocache[name] = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    return _ocache[name]


@pytest.mark.parametrize("name", ["water12k", "copper32k"])
def test_fp64_full_frames(dev, name):
    fr, desc, p, model, ctx, x, t = _setup(name, dev)
    _say("fp64 full", name)
    r = _compute(ctx, x, t, fr.box, "fp64")
    o = _oracle_full(name, fr, desc, p)
    assert abs(r["E"][0] - o["E"]) <= 1e-10 * abs(o["E"])
    assert np.abs(r["F"] - o["F"]).max() <= 1e-9
    assert np.abs(r["W"].reshape(3, 3) - o["W"]).max() <= 1e-9 * max(1.0, np.abs(o["W"]).max())
    assert np.abs(r["Ei"] - o["Ei"]).max() <= 1e-10 * np.abs(o["Ei"]).max()
    assert ctx.status() == 0


# force RMS error bars relative to the force RMS, per mixed form: BF16 keeps
# 8 mantissa bits, FP16 11, FP32 24 (the paper's MIX-fp32); the paper's
# MIX-fp16 is FP32 except the first fitting layer's FP16 products
REL_F = {"bf16": 2e-2, "fp16": 4e-3, "mix_fp32": 2e-5, "mix_fp16": 4e-3}


@pytest.mark.parametrize("name", ["water12k", "copper32k"])
@pytest.mark.parametrize("mode", ["bf16", "fp16", "mix_fp32", "mix_fp16"])
def test_mixed_full_frames(dev, name, mode):
    """Mixed precision at full size against the FP64 oracle: the mixed
    speedup is quoted at a force RMS error of at most 1 meV/A, asserted here
    on both systems, and at most REL_F of the force RMS (measured on water
    BF16 0.64%, FP16 0.09%; on copper 1.5% and 0.18%); energy within
    5 meV/atom."""
    fr, desc, p, model, ctx, x, t = _setup(name, dev)
    _say("mixed full", name, mode)
    r = _compute(ctx, x, t, fr.box, mode)
    o = _oracle_full(name, fr, desc, p)
    e_err = abs(r["E"][0] - o["E"]) / fr.n
    f_rms = np.sqrt(((r["F"] - o["F"]) ** 2).mean())
    f_scale = np.sqrt((o["F"] ** 2).mean())
    w_err = np.abs(r["W"].reshape(3, 3) - o["W"]).max() / fr.n
    _say(name, mode, "E err meV/atom", 1e3 * e_err, "F rms err meV/A", 1e3 * f_rms,
         "F rms meV/A", 1e3 * f_scale, "W err meV/atom", 1e3 * w_err)
    assert f_rms <= 1e-3
    # relative to the force scale (BF16 keeps 8 mantissa bits, FP16 11)
    assert f_rms <= REL_F[mode] * f_scale
    assert e_err <= 5e-3
    assert np.isfinite(r["W"]).all()
    assert ctx.status() == 0


def test_fp64_water98k_sampled(dev):
    """Full size of the mixed-precision workload: sampled atomic energies and
    forces (the oracle evaluates them one by one), global invariants."""
    fr, desc, p, model, ctx, x, t = _setup("water98k", dev)
    _say("fp64 water98k sampled")
    r = _compute(ctx, x, t, fr.box, "fp64")
    rows = np.random.default_rng(1).choice(fr.n, 64, replace=False)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p, rows=rows)
    assert np.abs(r["Ei"][rows] - o["Ei"]).max() <= 1e-10 * np.abs(o["Ei"]).max()
    for k in rows[:8]:
        f = oracle.force_on(fr.coords, fr.types, fr.box, desc, p, int(k))
        assert np.abs(r["F"][k] - f).max() <= 1e-9
    assert np.abs(r["F"].sum(0)).max() < 1e-9
    assert abs(r["E"][0] - r["Ei"].sum()) <= 1e-10 * abs(r["E"][0])
    W = r["W"].reshape(3, 3)
    assert np.abs(W - W.T).max() < 1e-8


@pytest.mark.parametrize("mode", ["bf16", "fp16", "mix_fp32", "mix_fp16"])
def test_mixed_water98k_sampled(dev, mode):
    """The mixed forms at the full size of their workload (98,304 atoms)
    against the FP64 oracle evaluated atom by atom: 64 sampled atomic
    energies and 8 sampled total forces, with the same relative bars as the
    full frames; the global invariants hold in the mixed forms too."""
    fr, desc, p, model, ctx, x, t = _setup("water98k", dev)
    _say("mixed water98k sampled", mode)
    r = _compute(ctx, x, t, fr.box, mode)
    rows = np.random.default_rng(2).choice(fr.n, 64, replace=False)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p, rows=rows)
    ei_err = np.abs(r["Ei"][rows] - o["Ei"])
    fo = np.array([oracle.force_on(fr.coords, fr.types, fr.box, desc, p, int(k)) for k in rows[:8]])
    f_err = np.sqrt(((r["F"][rows[:8]] - fo) ** 2).mean())
    f_scale = np.sqrt((r["F"] ** 2).mean())
    _say(mode, "E_i err max meV", 1e3 * ei_err.max(), "F rms err meV/A", 1e3 * f_err, "F rms meV/A", 1e3 * f_scale)
    assert ei_err.max() <= {"bf16": 5e-3, "fp16": 1e-3, "mix_fp32": 1e-5, "mix_fp16": 1e-3}[mode]
    assert f_err <= 1e-3
    assert f_err <= 2 * REL_F[mode] * f_scale   # 8 samples: twice the full-frame bar
    assert np.abs(r["F"].sum(0)).max() < 1e-9
    assert abs(r["E"][0] - r["Ei"].sum()) <= 1e-10 * abs(r["E"][0])
    W = r["W"].reshape(3, 3)
    assert np.abs(W - W.T).max() < 1e-6 * max(1.0, np.abs(W).max())
    assert ctx.status() == 0


@pytest.mark.parametrize("mode", ["bf16", "fp16", "mix_fp32", "mix_fp16"])
def test_mixed_water192_error_bounds(dev, mode):
    fr, desc, p, model, ctx, x, t = _setup("water192", dev)
    _say("mixed", mode)
    r = _compute(ctx, x, t, fr.box, mode)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p)
    e_err = abs(r["E"][0] - o["E"]) / fr.n
    f_rms = np.sqrt(((r["F"] - o["F"]) ** 2).mean())
    f_scale = np.sqrt((o["F"] ** 2).mean())
    _say(mode, "E err/atom", e_err, "F rms err", f_rms, "F rms", f_scale)
    assert e_err < 5e-3
    assert f_rms < 0.1 * f_scale
    assert np.isfinite(r["W"]).all()
