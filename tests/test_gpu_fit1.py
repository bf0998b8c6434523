"""The fused half-precision first fitting layer (BF16 / FP16 first layer on
frames of many atoms): the forward forms D = T T<^T inside the GEMM, the
backward folds the descriptor backward into the GEMM's epilogue.

Frames with type counts that are not multiples of the 16- and 32-column
tiles exercise the ragged column tails.  Checks, through the C ABI:
* energies and forces against the FP64 oracle at the mixed forms' bars, over
  all atoms and over the atoms of each type's last partial column tile;
* g_T = dE/dT against the same quantity formed from the compute's own T
  and dE/dD (dE/dD formed on request by the plain GEMM from the same dz1),
  to FP32 summation-order precision, and against the oracle's g_T;
* D written by the fused forward on a context that keeps the layer inputs
  for parameter gradients: T T<^T rounded to the operand type.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# force RMS error bars relative to the force RMS (as for the full frames)
REL_F = {"bf16": 2e-2, "fp16": 4e-3, "mix_fp16": 4e-3}
EI_MAX = {"bf16": 5e-3, "fp16": 1e-3, "mix_fp16": 1e-3}


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


_state = {}


def _frame():
    """2731 molecules (8193 atoms: 2731 O, 5462 H) at 1 g/cm^3."""
    if "fr" not in _state:
        nmol = 2731
        fr = I.water_box(nmol, I.water_density_box(nmol), seed=21)
        p = I.init_params(I.WATER, I.MODEL_SEED_WATER, I.WATER_OUTPUT_SCALE)
        o = oracle.compute(fr.coords, fr.types, fr.box, I.WATER, p, debug=True)
        _state["fr"] = (fr, p, o)
    return _state["fr"]


def _fused_expected(n):
    # the library takes the fused form when every compute unit gets a
    # 32-column work-group
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return (n + 31) // 32 >= cus


def _tail_atoms(types):
    """Atoms of each type's last partial 16-column tile (columns are a type's
    atoms in atom order)."""
    out = []
    for t in np.unique(types):
        idx = np.nonzero(types == t)[0]
        r = len(idx) % 16
        if r:
            out.extend(idx[-r:])
    return np.array(sorted(out))


@pytest.mark.parametrize("mode", ["bf16", "fp16", "mix_fp16"])
def test_fit1_fused_ragged(dev, mode):
    from paper_2410_22867_amd import dpse
    fr, p, o = _frame()
    if not _fused_expected(fr.n):
        pytest.skip("fewer columns than 32 per compute unit on this device")
    _say("fit1 fused", mode, fr.n)
    model = dpse.Model(I.WATER, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    r = ctx.compute(x, t, fr.box, nl, mode=mode, want_atom_energy=True)
    gT = ctx.copy_buffer(dpse.BUF_GT).cpu().numpy().reshape(fr.n, I.WATER.m1, 4)
    T = ctx.copy_buffer(dpse.BUF_T).cpu().numpy().reshape(fr.n, I.WATER.m1, 4)
    gD = ctx.copy_buffer(dpse.BUF_GD).cpu().numpy().reshape(fr.n, I.WATER.m1, 16)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    F = r["F"].cpu().numpy()
    Ei = r["Ei"].cpu().numpy()
    tail = _tail_atoms(fr.types)
    assert len(tail) > 0
    f_scale = np.sqrt((o["F"] ** 2).mean())
    f_rms = np.sqrt(((F - o["F"]) ** 2).mean())
    f_tail = np.sqrt(((F[tail] - o["F"][tail]) ** 2).mean())
    ei_err = np.abs(Ei - o["Ei"])
    _say(mode, "F rms err", f_rms, "tail", f_tail, "scale", f_scale, "Ei max err", ei_err.max(),
         "tail", ei_err[tail].max())
    assert f_rms <= REL_F[mode] * f_scale
    assert f_tail <= 2 * REL_F[mode] * f_scale
    assert ei_err.max() <= EI_MAX[mode]
    # g_T from the compute's own T and dE/dD: the first term over b < 16,
    # the second (rows a < 16) over a'
    ref = np.einsum("nab,nbk->nak", gD, T[:, :16, :])
    ref[:, :16, :] += np.einsum("nab,nak->nbk", gD, T)
    scale = np.abs(ref).max()
    err = np.abs(gT - ref)
    _say(mode, "gT vs T, dE/dD: max err", err.max(), "scale", scale, "tail", err[tail].max())
    assert err.max() <= 1e-5 * scale
    # and against the oracle's g_T, at the form's precision
    og = o["gT"]
    assert np.abs(gT - og).max() <= 0.05 * np.abs(og).max()


def test_fit1_fused_writes_d(dev):
    """On a context that keeps the layer inputs for parameter gradients, the
    fused forward writes D = T T<^T in the operand type."""
    from paper_2410_22867_amd import dpse
    fr, p, o = _frame()
    if not _fused_expected(fr.n):
        pytest.skip("fewer columns than 32 per compute unit on this device")
    _say("fit1 fused D", fr.n)
    model = dpse.Model(I.WATER, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    ctx.compute(x, t, fr.box, nl, mode="fp16", want_atom_energy=True)
    ctx.backward_params(torch.ones(1, dtype=torch.float64, device=dev))
    ctx.compute(x, t, fr.box, nl, mode="fp16", want_atom_energy=True)
    D = ctx.copy_buffer(dpse.BUF_D).cpu().numpy().reshape(fr.n, I.WATER.m1, 16)
    T = ctx.copy_buffer(dpse.BUF_T).cpu().numpy().reshape(fr.n, I.WATER.m1, 4).astype(np.float32)
    torch.cuda.synchronize()
    ref = np.einsum("nak,nbk->nab", T.astype(np.float64), T[:, :16, :].astype(np.float64))
    # the kernel rounds an FP32 sum to FP16: one unit in the last place of
    # FP16 (2^-10 relative) covers a different FP32 summation order
    tol = np.maximum(np.abs(ref) * 2.0 ** -10, 2.0 ** -24)
    err = np.abs(D - ref)
    _say("D max err / tol", (err / tol).max())
    assert (err <= tol * 1.01).all()
    assert ctx.status() == 0


@pytest.mark.parametrize("mode,tol", [("bf16", 0.05), ("fp16", 0.01), ("mix_fp16", 0.01)])
def test_fit1_fused_batch_param_grads(dev, mode, tol):
    """A batch large enough for the fused first layer (12 frames, ~9,500
    atoms): per-frame energies and forces against the oracle, and the
    parameter gradient of the energy MSE loss against the oracle's, with
    the mixed forms' bars (tol of the largest gradient entry)."""
    from paper_2410_22867_amd import dpse
    frames, targets = I.water_batch(12, seed=31, lo=230, hi=300)
    sizes = [f.n for f in frames]
    off = dpse.frame_offsets(sizes)
    if not _fused_expected(int(off[-1])):
        pytest.skip("fewer columns than 32 per compute unit on this device")
    _say("fit1 fused batch grads", mode, int(off[-1]))
    p = I.init_params(I.WATER, I.MODEL_SEED_WATER, I.WATER_OUTPUT_SCALE)
    x = torch.tensor(np.concatenate([f.coords for f in frames]), device=dev)
    t = torch.tensor(np.concatenate([f.types for f in frames]), device=dev)
    boxes = np.stack([f.box for f in frames])
    model = dpse.Model(I.WATER, p)
    ctx = dpse.Context(model, int(off[-1]), max_frames=len(frames))
    nl, ov = ctx.build_nlist_batch(x, t, boxes, off)
    params = torch.tensor(p, device=dev, requires_grad=True)
    E = dpse.dp_energy(params, x, t, boxes, off, ctx, nl, mode)
    tgt = torch.tensor(targets, device=dev)
    L = ((E - tgt) ** 2).mean()
    L.backward()
    r = ctx.compute_batch(x, t, boxes, off, nl, mode=mode)
    torch.cuda.synchronize()
    assert int(ov.item()) == 0
    g = params.grad.cpu().numpy()
    Em = E.detach().cpu().numpy()
    F = r["F"].cpu().numpy()
    B = len(frames)
    want = np.zeros_like(g)
    f_err, f_scale = [], []
    for f, fr in enumerate(frames):
        o = oracle.compute(fr.coords, fr.types, fr.box, I.WATER, p, grad_scale=2.0 * (Em[f] - targets[f]) / B)
        want += o["grad"]
        assert abs(Em[f] - o["E"]) / fr.n <= 5e-3
        a0, a1 = off[f], off[f + 1]
        f_err.append(((F[a0:a1] - o["F"]) ** 2).sum())
        f_scale.append((o["F"] ** 2).sum())
    f_rms = np.sqrt(sum(f_err) / (3 * off[-1]))
    f_ref = np.sqrt(sum(f_scale) / (3 * off[-1]))
    rel = np.abs(g - want).max() / np.abs(want).max()
    _say(mode, "F rms err", f_rms, "of", f_ref, "param grad max error / max |grad|", rel)
    assert f_rms <= REL_F[mode] * f_ref
    assert np.isfinite(g).all()
    assert rel <= tol
    assert ctx.status() == 0
