"""The training workload at full size: 64 water frames of uneven size
(116,808 atoms) in one launch.  Eight sampled frames against the per-frame
oracle (E, F, W at the FP64 bars), and the parameter gradient of the energy
MSE loss over the whole batch against the oracle's (1e-9 of its largest
entry), through the torch.autograd.Function."""
import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def full_batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_22867_amd import dpse
    (frames, targets), desc, p, _ = I.workload("waterbatch64")
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


def test_batch64_sampled_frames(full_batch):
    b = full_batch
    print("[gpu-test] batch64 frames", len(b["frames"]), int(b["off"][-1]), flush=True)
    r = b["ctx"].compute_batch(b["x"], b["t"], b["boxes"], b["off"], b["nl"], mode="fp64")
    torch.cuda.synchronize()
    assert int(b["ov"].item()) == 0
    E = r["E"].cpu().numpy()
    F = r["F"].cpu().numpy()
    W = r["W"].cpu().numpy().reshape(-1, 3, 3)
    nl = b["nl"].cpu().numpy()
    sizes = np.diff(b["off"])
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))} |
                   set(np.random.default_rng(5).choice(len(b["frames"]), 6, replace=False).tolist()))
    for f in picks:
        fr = b["frames"][f]
        a0, a1 = b["off"][f], b["off"][f + 1]
        o = oracle.compute(fr.coords, fr.types, fr.box, b["desc"], b["p"])
        gl = nl[a0:a1].copy()
        m = gl >= 0
        gl[m] = (gl[m] // 27 - a0) * 27 + gl[m] % 27
        assert np.array_equal(gl, o["nlist"])
        assert abs(E[f] - o["E"]) <= 1e-10 * abs(o["E"])
        assert np.abs(F[a0:a1] - o["F"]).max() <= 1e-9
        assert np.abs(W[f] - o["W"]).max() <= 1e-9
    assert b["ctx"].status() == 0


def test_batch64_param_grads_match_oracle(full_batch):
    b = full_batch
    from paper_2410_22867_amd import dpse
    print("[gpu-test] batch64 param grads", flush=True)
    params = torch.tensor(b["p"], device=b["dev"], requires_grad=True)
    E = dpse.dp_energy(params, b["x"], b["t"], b["boxes"], b["off"], b["ctx"], b["nl"], "fp64")
    tgt = torch.tensor(b["targets"], device=b["dev"])
    L = ((E - tgt) ** 2).mean()
    L.backward()
    torch.cuda.synchronize()
    g = params.grad.cpu().numpy()
    Em = E.detach().cpu().numpy()
    B = len(b["frames"])
    want = np.zeros_like(g)
    for f, fr in enumerate(b["frames"]):
        want += oracle.compute(fr.coords, fr.types, fr.box, b["desc"], b["p"],
                               grad_scale=2.0 * (Em[f] - b["targets"][f]) / B)["grad"]
    scale = np.abs(want).max()
    err = np.abs(g - want).max()
    print("[gpu-test] batch64 grad max err / max |grad|", err / scale, flush=True)
    assert err <= 1e-9 * scale
    assert b["ctx"].status() == 0
