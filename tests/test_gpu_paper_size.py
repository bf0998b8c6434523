"""The Evaluation section's strong-scaling systems on one GPU (water557k:
557,568 atoms; copper535k: 535,680 atoms), FP64 and BF16, checked at full
size against the FP64 oracle evaluated atom by atom: sampled atomic energies
and total forces, with the global invariants (zero net force, E = sum of
E_i, symmetric virial) over the whole frame."""
import sys

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# BF16 bars: atomic energies within 5 meV on water (as for the water98k
# samples) and 15 meV on copper, whose 500-neighbour sums carry 2.5x water's
# relative BF16 error (copper32k force error 1.5% of the force RMS against
# water's 0.6%); the sampled force RMS error within twice the full frames'
# relative bar
BF16_EI = {"water557k": 5e-3, "copper535k": 1.5e-2}
BF16_REL_F = 2 * 2e-2


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["water557k", "copper535k"])
def system(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_22867_amd import dpse
    dpse.lib()
    dev = torch.device("cuda:0")
    fr, desc, p, dt = I.workload(request.param)
    _say("paper size", request.param, fr.n)
    model = dpse.Model(desc, p)
    ctx = dpse.Context(model, fr.n)
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl, ov = ctx.build_nlist(x, t, fr.box)
    torch.cuda.synchronize()
    assert int(ov.item()) == 0
    yield request.param, fr, desc, p, ctx, x, t, nl
    ctx.close()
    model.close()


@pytest.mark.parametrize("mode", ["fp64", "bf16"])
def test_paper_size_sampled(system, mode):
    name, fr, desc, p, ctx, x, t, nl = system
    r = ctx.compute(x, t, fr.box, nl, mode=mode, want_atom_energy=True)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    r = {k: v.cpu().numpy() for k, v in r.items()}
    rows = np.random.default_rng(7).choice(fr.n, 32, replace=False)
    o = oracle.compute(fr.coords, fr.types, fr.box, desc, p, rows=rows)
    fo = np.array([oracle.force_on(fr.coords, fr.types, fr.box, desc, p, int(k)) for k in rows[:4]])
    ei_err = np.abs(r["Ei"][rows] - o["Ei"]).max()
    f_err = np.abs(r["F"][rows[:4]] - fo).max()
    f_rms_err = np.sqrt(((r["F"][rows[:4]] - fo) ** 2).mean())
    f_scale = np.sqrt((r["F"] ** 2).mean())
    _say(name, mode, "E_i max err", ei_err, "F max err", f_err, "F rms err", f_rms_err, "F rms", f_scale)
    if mode == "fp64":
        assert ei_err <= 1e-10 * np.abs(o["Ei"]).max()
        assert f_err <= 1e-9
    else:
        assert ei_err <= BF16_EI[name]
        assert f_rms_err <= BF16_REL_F * f_scale
    assert np.abs(r["F"].sum(0)).max() < 1e-8
    assert abs(r["E"][0] - r["Ei"].sum()) <= 1e-10 * abs(r["E"][0])
    W = r["W"].reshape(3, 3)
    assert np.abs(W - W.T).max() < 1e-6 * max(1.0, np.abs(W).max())
