"""GPU parity of the batched path and of the parameter gradients of the
energy loss L = (1/B) sum_f (E_f - Ehat_f)^2 (FP64), against the oracle's
per-frame results and against central finite differences of the GPU
energies."""
import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_22867_amd import dpse
    frames, targets = I.water_batch(5, seed=9, lo=64, hi=180)
    desc = I.WATER
    p = I.init_params(desc, I.MODEL_SEED_WATER)
    sizes = [f.n for f in frames]
    off = dpse.frame_offsets(sizes)
    dev = torch.device("cuda:0")
    x = torch.tensor(np.concatenate([f.coords for f in frames]), device=dev)
    t = torch.tensor(np.concatenate([f.types for f in frames]), device=dev)
    boxes = np.stack([f.box for f in frames])
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, int(off[-1]), max_frames=len(frames))
    nl, ov = ctx.build_nlist_batch(x, t, boxes, off)
    return dict(frames=frames, targets=targets, desc=desc, p=p, off=off, x=x, t=t, boxes=boxes, model=model,
                ctx=ctx, nl=nl, ov=ov, dev=dev)


def test_batch_matches_per_frame_oracle(batch):
    b = batch
    _say("batch nlist+compute", [f.n for f in b["frames"]])
    r = b["ctx"].compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode="fp64")
    torch.cuda.synchronize()
    assert int(b["ov"].item()) == 0
    nl = b["nl"].cpu().numpy()
    E = r["E"].cpu().numpy()
    F = r["F"].cpu().numpy()
    W = r["W"].cpu().numpy().reshape(-1, 3, 3)
    for f, fr in enumerate(b["frames"]):
        a0, a1 = b["off"][f], b["off"][f + 1]
        o = oracle.compute(fr.coords, fr.types, fr.box, b["desc"], b["p"])
        gl = nl[a0:a1].copy()
        m = gl >= 0
        gl[m] = (gl[m] // 27 - a0) * 27 + gl[m] % 27
        assert np.array_equal(gl, o["nlist"])
        assert abs(E[f] - o["E"]) <= 1e-10 * abs(o["E"])
        assert np.abs(F[a0:a1] - o["F"]).max() <= 1e-9
        assert np.abs(W[f] - o["W"]).max() <= 1e-9


def _loss_and_grad(b):
    from paper_2410_22867_amd import dpse
    params = torch.tensor(b["p"], device=b["dev"], requires_grad=True)
    coords = b["x"].clone().requires_grad_(True)
    E = dpse.dp_energy(params, coords, b["t"], b["boxes"], b["off"], b["ctx"], b["nl"])
    tgt = torch.tensor(b["targets"], device=b["dev"])
    L = ((E - tgt) ** 2).mean()
    L.backward()
    torch.cuda.synchronize()
    return L.item(), E.detach().cpu().numpy(), params.grad.cpu().numpy(), coords.grad.cpu().numpy()


def test_param_grads_match_oracle(batch):
    b = batch
    _say("param grads vs oracle")
    L, E, g, gx = _loss_and_grad(b)
    B = len(b["frames"])
    want = np.zeros_like(g)
    for f, fr in enumerate(b["frames"]):
        dLdE = 2.0 * (E[f] - b["targets"][f]) / B
        o = oracle.compute(fr.coords, fr.types, fr.box, b["desc"], b["p"], grad_scale=dLdE)
        want += o["grad"]
    scale = np.abs(want).max()
    err = np.abs(g - want)
    assert err.max() <= 1e-9 * scale, (err.max(), scale, int(err.argmax()))
    # coordinate gradient: dL/dx = -F * dL/dE_f
    r = b["ctx"].compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode="fp64")
    F = r["F"].cpu().numpy()
    for f in range(B):
        a0, a1 = b["off"][f], b["off"][f + 1]
        assert np.allclose(gx[a0:a1], -F[a0:a1] * 2.0 * (E[f] - b["targets"][f]) / B, atol=1e-12)


def test_param_grads_with_stored_activations(batch):
    """A context whose workspace holds the last embedding layer's activations
    (FP64 forward stores them; the gradient pass then reads them instead of
    recomputing that layer) gives the same parameter gradient as the
    recomputing context, and the oracle's."""
    b = batch
    _say("param grads with stored activations")
    from paper_2410_22867_amd import dpse
    ctx2 = dpse.Context(b["model"], int(b["off"][-1]), max_frames=len(b["frames"]), budget_bytes=1 << 30)
    nl2, _ = ctx2.build_nlist_batch(b["x"], b["t"], b["boxes"], b["off"])
    b2 = dict(b, ctx=ctx2, nl=nl2)
    L2, E2, g2, _ = _loss_and_grad(b2)
    assert ctx2.store_info()[1] is True
    L1, E1, g1, _ = _loss_and_grad(b)
    assert b["ctx"].store_info()[1] is False
    scale = np.abs(g1).max()
    assert np.abs(g2 - g1).max() <= 1e-12 * scale
    B = len(b["frames"])
    want = np.zeros_like(g2)
    for f, fr in enumerate(b["frames"]):
        dLdE = 2.0 * (E2[f] - b["targets"][f]) / B
        want += oracle.compute(fr.coords, fr.types, fr.box, b["desc"], b["p"], grad_scale=dLdE)["grad"]
    assert np.abs(g2 - want).max() <= 1e-9 * np.abs(want).max()
    ctx2.close()


def test_param_grads_finite_differences(batch):
    b = batch
    _say("param grads vs FD")
    from paper_2410_22867_amd import dpse
    L0, E0, g, _ = _loss_and_grad(b)
    desc = b["desc"]
    off = desc.param_offsets()
    rng = np.random.default_rng(3)
    picks = []
    for name, (o, shp) in off.items():
        picks.append(o + int(rng.integers(int(np.prod(shp)))))
    h = 1e-5
    tgt = torch.tensor(b["targets"], device=b["dev"])

    def loss(pv):
        b["model"].set_params(pv)
        r = b["ctx"].compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode="fp64")
        return float(((r["E"] - tgt) ** 2).mean().item())

    for k in picks:
        q = b["p"].copy()
        q[k] += h
        lp = loss(q)
        q[k] -= 2 * h
        lm = loss(q)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])
    b["model"].set_params(b["p"])


@pytest.mark.parametrize("mode", ["bf16", "mix_fp32"])
def test_mixed_param_grads_with_store(batch, mode):
    """After a mixed-precision compute, a context whose workspace holds the
    FP64 activations fills it in the gradient pass (FP64 embedding forward
    of the same frame) and reads the last layer back: the parameter
    gradient matches that of the recomputing context, and a second gradient
    pass over the same compute gives the same result (up to the order of
    the FP64 atomic sums)."""
    b = batch
    _say("mixed param grads with store", mode)
    from paper_2410_22867_amd import dpse
    ctx2 = dpse.Context(b["model"], int(b["off"][-1]), max_frames=len(b["frames"]), budget_bytes=1 << 30)
    nl2, _ = ctx2.build_nlist_batch(b["x"], b["t"], b["boxes"], b["off"])
    B = len(b["frames"])
    dLdE = torch.linspace(-0.3, 0.5, B, dtype=torch.float64, device=b["dev"])
    grads = []
    for ctx, nl in ((b["ctx"], b["nl"]), (ctx2, nl2)):
        ctx.compute_batch(b["x"], b["t"], b["boxes"], b["off"], nl, mode=mode)
        g = [ctx.backward_params(dLdE).cpu().numpy() for _ in range(2)]
        torch.cuda.synchronize()
        grads.append(g)
    assert b["ctx"].store_info()[1:] == (False, False)
    assert ctx2.store_info()[1:] == (False, True)
    (g1, g1b), (g2, g2b) = grads
    scale = np.abs(g1).max()
    # the weight-gradient sums use FP64 atomics: equal up to summation order
    assert np.abs(g1b - g1).max() <= 1e-13 * scale
    assert np.abs(g2b - g2).max() <= 1e-13 * scale
    assert np.abs(g2 - g1).max() <= 1e-12 * scale
    # a following FP64 compute on the same context uses the store itself
    ctx2.compute_batch(b["x"], b["t"], b["boxes"], b["off"], nl2, mode="fp64")
    torch.cuda.synchronize()
    assert ctx2.store_info()[1:] == (True, False)
    ctx2.close()


@pytest.mark.parametrize("mode,tol", [("bf16", 0.05), ("fp16", 0.01), ("mix_fp32", 1e-4), ("mix_fp16", 0.01)])
def test_mixed_param_grads_close_to_oracle(batch, mode, tol):
    """Mixed-precision form of the training step: energies, forces and
    parameter gradients of the mixed model, compared with the FP64 oracle
    (error stated; bounded by tol of the largest gradient entry)."""
    b = batch
    from paper_2410_22867_amd import dpse
    params = torch.tensor(b["p"], device=b["dev"], requires_grad=True)
    coords = b["x"].clone().requires_grad_(True)
    E = dpse.dp_energy(params, coords, b["t"], b["boxes"], b["off"], b["ctx"], b["nl"], mode)
    tgt = torch.tensor(b["targets"], device=b["dev"])
    L = ((E - tgt) ** 2).mean()
    L.backward()
    torch.cuda.synchronize()
    g = params.grad.cpu().numpy()
    Em = E.detach().cpu().numpy()
    B = len(b["frames"])
    want = np.zeros_like(g)
    for f, fr in enumerate(b["frames"]):
        o = oracle.compute(fr.coords, fr.types, fr.box, b["desc"], b["p"], grad_scale=2.0 * (Em[f] - b["targets"][f]) / B)
        want += o["grad"]
    scale = np.abs(want).max()
    rel = np.abs(g - want).max() / scale
    _say(mode, "param grad max error / max |grad|", rel)
    assert np.isfinite(g).all()
    assert rel <= tol
    # the coordinate gradient is -F of the mixed model times dL/dE_f
    r = b["ctx"].compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode=mode)
    F = r["F"].cpu().numpy()
    gx = coords.grad.cpu().numpy()
    for f in range(B):
        a0, a1 = b["off"][f], b["off"][f + 1]
        assert np.allclose(gx[a0:a1], -F[a0:a1] * 2.0 * (Em[f] - b["targets"][f]) / B, atol=1e-12)


def test_parameter_updates_are_always_seen(batch):
    """DPEnergy loads the parameters on the device at every call: a change
    made in place through .data (which leaves the tensor's version counter
    alone) and a new tensor that may reuse the freed block both give the
    oracle's energies and gradients for the new parameters; the device
    update of the model matches the host one bit for bit."""
    b = batch
    from paper_2410_22867_amd import dpse
    _say("parameter updates")
    dev = b["dev"]
    tgt = torch.tensor(b["targets"], device=dev)
    B = len(b["frames"])

    def check(params, pnp):
        E = dpse.dp_energy(params, b["x"], b["t"], b["boxes"], b["off"], b["ctx"], b["nl"], "fp64")
        L = ((E - tgt) ** 2).mean()
        L.backward()
        torch.cuda.synchronize()
        Em = E.detach().cpu().numpy()
        g = params.grad.cpu().numpy()
        want = np.zeros_like(g)
        for f, fr in enumerate(b["frames"]):
            o = oracle.compute(fr.coords, fr.types, fr.box, b["desc"], pnp,
                               grad_scale=2.0 * (Em[f] - b["targets"][f]) / B)
            assert abs(Em[f] - o["E"]) <= 1e-10 * abs(o["E"])
            want += o["grad"]
        assert np.abs(g - want).max() <= 1e-9 * np.abs(want).max()

    p0 = b["p"].copy()
    params = torch.tensor(p0, device=dev, requires_grad=True)
    check(params, p0)
    # in place through .data: the version counter does not move
    off, shp = b["desc"].param_offsets()["fit1.W1"]
    p1 = p0.copy()
    p1[off:off + 1000] *= 1.5
    v = params._version
    params.data[off:off + 1000] *= 1.5
    assert params._version == v
    params.grad = None
    check(params, p1)
    # a new tensor after the old one is freed (the caching allocator may hand
    # back the same block)
    del params
    p2 = p1.copy()
    p2[5:200] += 0.01
    params = torch.tensor(p2, device=dev, requires_grad=True)
    check(params, p2)
    # the device update equals the host update
    m1 = dpse.Model(b["desc"], p0)
    m1.set_params(p2)
    m2 = dpse.Model(b["desc"], p0)
    m2.load_params(torch.tensor(p2, device=dev))
    c1 = dpse.Context(m1, int(b["off"][-1]), max_frames=B)
    c2 = dpse.Context(m2, int(b["off"][-1]), max_frames=B)
    for mode in ("fp64", "bf16", "fp16"):
        r1 = c1.compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode=mode)
        r2 = c2.compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(r1["E"], r2["E"]) and torch.equal(r1["F"], r2["F"])
    b["model"].set_params(b["p"])
