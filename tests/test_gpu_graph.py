"""One MD step (kick + drift, Verlet update with the rebuild decided on the
device, E/F/W, kick) captured in a HIP graph through torch.cuda.CUDAGraph and
replayed: every replay equals the eagerly issued step from the same state,
bit for bit, with eager work and host synchronisations between replays."""
import numpy as np
import pytest

from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("mode", ["fp64", "bf16"])
def test_graph_replay_equals_eager(mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_22867_amd import dpse
    print("[gpu-test] graph replay", mode, flush=True)
    fr, desc, p, dt = I.workload("water192")
    n = fr.n
    dev = torch.device("cuda:0")
    ctx = dpse.Context(dpse.Model(desc, p), n)
    x = torch.tensor(fr.coords, device=dev)
    v = torch.tensor(I.maxwell_boltzmann(fr.types, desc.masses, 300.0, seed=203), device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl = torch.empty((n, desc.nm), dtype=torch.int32, device=dev)
    ov = torch.empty(1, dtype=torch.int32, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    W = torch.empty(9, dtype=torch.float64, device=dev)
    ke = torch.empty(1, dtype=torch.float64, device=dev)
    f = torch.empty((n, 3), dtype=torch.float64, device=dev)
    img = torch.zeros((n, 3), dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    skin = 0.3   # small: the device decides several rebuilds within the run

    def step():
        ctx.kick_drift(x, v, f, t, fr.box, dt, wrap=False)
        ctx.skin_update(x, t, every=0, images=img, out=nl, overflow=ov)
        ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
        ctx.kick(v, f, t, dt, ke)

    x0 = x.clone()
    v0 = v.clone()

    def setup():
        """The same start for both runs: positions, velocities, image
        counters, the Verlet build (its candidates, reference positions and
        the device's rebuild counters) and the first forces."""
        with torch.cuda.stream(s):
            x.copy_(x0)
            v.copy_(v0)
            img.zero_()
            ctx.skin_build(x, t, fr.box, skin, images=img)
            ctx.skin_format(x, t, out=nl, overflow=ov)
            ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
        torch.cuda.synchronize()

    nsteps = 12
    setup()
    eager = []
    with torch.cuda.stream(s):
        for _ in range(nsteps):
            step()
            eager.append([a.clone() for a in (x, v, E, ke, img)])
    torch.cuda.synchronize()
    assert int(img.abs().sum().item()) >= 0
    setup()
    start = [a.clone() for a in (x, v, f)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    torch.cuda.synchronize()
    # capturing does not execute the step
    for a, b in zip((x, v, f), start):
        assert torch.equal(a, b)
    for k in range(nsteps):
        g.replay()
        junk = torch.randn(1000, device=dev).sum()   # eager work between replays
        torch.cuda.synchronize()
        got = [a.clone() for a in (x, v, E, ke, img)]
        for a, b in zip(got, eager[k]):
            assert torch.equal(a, b), k
        assert bool(torch.isfinite(junk))
    assert ctx.status() == 0
