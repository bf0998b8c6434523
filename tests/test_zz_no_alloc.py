"""dp_build_nlist_noalloc (the entry point for callers that cannot allocate)
against dp_build_nlist on the same inputs, through the C ABI: the lists,
overflow counts and status bits are identical, on calls in a row whose second
input is smaller (the shared scratch keeps the first call's contents), with
section overflow and with the size limits rejected before any launch."""
import dataclasses
import sys

import numpy as np
import pytest

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


def _both(dpse, model, fr, dev):
    x = torch.tensor(fr.coords, device=dev)
    t = torch.tensor(fr.types, device=dev)
    ctx = dpse.Context(model, fr.n)
    ref, ref_ov = ctx.build_nlist(x, t, fr.box)
    out = torch.full((fr.n, model.desc.nm), -7, dtype=torch.int32, device=dev)
    ov = torch.full((1,), -7, dtype=torch.int32, device=dev)
    fl = torch.full((1,), -7, dtype=torch.int32, device=dev)
    dpse.build_nlist_noalloc(model, x, t, fr.box, out, ov, fl)
    torch.cuda.synchronize()
    ref_flags = ctx.status()
    return (ref.cpu().numpy(), int(ref_ov.item()), ref_flags), (out.cpu().numpy(), int(ov.item()), int(fl.item()))


def test_noalloc_matches_build_nlist_twice_smaller_second(dev):
    from paper_2410_22867_amd import dpse
    fr1, desc, p, _ = I.workload("water12k")
    fr2, _, _, _ = I.workload("water192")
    model = dpse.Model(desc, p)
    for fr in (fr1, fr2):
        _say("noalloc nlist", fr.n)
        (a, aov, afl), (b, bov, bfl) = _both(dpse, model, fr, dev)
        assert np.array_equal(a, b)
        assert aov == bov == 0
        assert afl == bfl == 0


def test_noalloc_overflow_and_flags(dev):
    from paper_2410_22867_amd import dpse
    desc = dataclasses.replace(I.WATER, sel=(10, 20))
    model = dpse.Model(desc, I.init_params(desc, 1))
    for fr in (I.water_box(216, 18.6, seed=12), I.water_box(64, 12.42, seed=13)):
        _say("noalloc overflow", fr.n)
        (a, aov, afl), (b, bov, bfl) = _both(dpse, model, fr, dev)
        assert np.array_equal(a, b)
        assert aov == bov > 0
        assert afl == bfl == dpse.FLAG_SEL_OVERFLOW


def test_noalloc_limits(dev):
    from paper_2410_22867_amd import dpse
    fr, desc, p, _ = I.workload("water192")
    model = dpse.Model(desc, p)
    n = 65537
    x = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    t = torch.zeros(n, dtype=torch.int32, device=dev)
    out = torch.empty((n, desc.nm), dtype=torch.int32, device=dev)
    ov = torch.empty(1, dtype=torch.int32, device=dev)
    with pytest.raises(dpse.DPError) as e:
        dpse.build_nlist_noalloc(model, x, t, np.diag([200.0, 200.0, 200.0]), out, ov)
    assert e.value.code == -3
    # a dilute box: 80^3 cells of 6 A exceed the cell limit
    with pytest.raises(dpse.DPError) as e:
        dpse.build_nlist_noalloc(model, x[:10], t[:10], np.diag([480.0, 480.0, 480.0]), out, ov)
    assert e.value.code == -3
