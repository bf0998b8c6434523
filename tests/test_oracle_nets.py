"""Pins of the oracle's two networks with non-zero weights in every layer.

Background section (DeePMD-kit subsection): the smoothed first column of R_i
passes through a three-layer "embedding net" whose output, contracted with
R_i, gives the descriptor D_i; a three-layer "fitting net" maps D_i to the
atomic energy E_i.  The layer details (tanh activations, identity skips on
equal and doubled widths, a linear output layer) are the DeePMD-kit readings
of the DP papers the section cites.

The descriptor D and the environment matrix R~ that feed these tests are
pinned elsewhere (single-neighbour closed forms, the constant-embedding
descriptor, rotation invariance).  Here the networks are evaluated a second
time, layer by layer in numpy from the flat parameter vector, and compared
with the oracle's per-atom energies and its T = G^T R~ / N_m.  Each test
also evaluates the plausible misreadings of the layer structure (no identity
skip, a tanh on the output layer, tanh(z) instead of h fed forward, the
doubled skip as [h, 0] or interleaved) and checks that every one of them is
far from the oracle, so a mistake of that kind in the oracle cannot pass.
"""
import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I


def _blk(desc, p, name):
    o, shp = desc.param_offsets()[name]
    return p[o:o + int(np.prod(shp))].reshape(shp)


def _fit_variants(desc, p, t, D):
    """E_i of centre type t from descriptor rows D [n, nd] under the reading
    and under each misreading (dict name -> [n])."""
    W = [_blk(desc, p, f"fit{t}.W{l}") for l in (1, 2, 3)]
    b = [_blk(desc, p, f"fit{t}.b{l}") for l in (1, 2, 3)]
    wo = _blk(desc, p, f"fit{t}.wo")
    bo = _blk(desc, p, f"fit{t}.bo")[0]
    eb = _blk(desc, p, "e_bias")[t]
    out = {}
    # reading: h1 = tanh(D W1 + b1); h_l = h_{l-1} + tanh(h_{l-1} W_l + b_l)
    # (equal widths); E = h3 . wo + bo + e_bias
    h = np.tanh(D @ W[0] + b[0])
    for l in (1, 2):
        h = h + np.tanh(h @ W[l] + b[l])
    out["reading"] = h @ wo + bo + eb
    # no identity skip on the equal-width layers
    h = np.tanh(D @ W[0] + b[0])
    for l in (1, 2):
        h = np.tanh(h @ W[l] + b[l])
    out["no_skip"] = h @ wo + bo + eb
    # tanh on the output layer
    h = np.tanh(D @ W[0] + b[0])
    for l in (1, 2):
        h = h + np.tanh(h @ W[l] + b[l])
    out["tanh_output"] = np.tanh(h @ wo + bo) + eb
    # tanh(z) (not h) fed to the next layer, skip kept in the final h
    t1 = np.tanh(D @ W[0] + b[0])
    t2 = np.tanh(t1 @ W[1] + b[1])
    h2 = t1 + t2
    t3 = np.tanh(t2 @ W[2] + b[2])
    out["tanh_fed"] = (h2 + t3) @ wo + bo + eb
    return out


def _emb_variants(desc, p, ti, tj, s):
    """G (last embedding layer, [m1]) of a neighbour with radial input s for
    net (ti, tj) under the reading and the misreadings."""
    W = [_blk(desc, p, f"emb{ti}{tj}.W{l}") for l in (1, 2, 3)]
    b = [_blk(desc, p, f"emb{ti}{tj}.b{l}") for l in (1, 2, 3)]
    out = {}
    h1 = np.tanh(s * W[0][0] + b[0])                       # 1 -> w: no skip (w != 1, 2)
    h2 = np.concatenate([h1, h1]) + np.tanh(h1 @ W[1] + b[1])   # w -> 2w: [h, h] skip
    h3 = np.concatenate([h2, h2]) + np.tanh(h2 @ W[2] + b[2])   # 2w -> 4w
    out["reading"] = h3
    h2 = np.tanh(h1 @ W[1] + b[1])
    out["no_skip"] = np.tanh(h2 @ W[2] + b[2])
    z = np.zeros_like(h1)
    h2 = np.concatenate([h1, z]) + np.tanh(h1 @ W[1] + b[1])
    h3 = np.concatenate([h2, np.zeros_like(h2)]) + np.tanh(h2 @ W[2] + b[2])
    out["skip_h_0"] = h3
    h2 = np.repeat(h1, 2) + np.tanh(h1 @ W[1] + b[1])
    h3 = np.repeat(h2, 2) + np.tanh(h2 @ W[2] + b[2])
    out["skip_interleaved"] = h3
    t2 = np.tanh(h1 @ W[1] + b[1])
    h2 = np.concatenate([h1, h1]) + t2
    out["tanh_fed"] = np.concatenate([h2, h2]) + np.tanh(t2 @ W[2] + b[2])
    return out


@pytest.fixture(scope="module")
def w192():
    fr, desc, p, _ = I.workload("water192")
    # non-zero output and e_bias so that every term of E_i is exercised
    p = p.copy()
    for t in range(desc.ntypes):
        o, _ = desc.param_offsets()[f"fit{t}.bo"]
        p[o] = 1.5 - 2.5 * t       # |h3 . wo + bo| ~ 1: tanh is far from linear there
    o, _ = desc.param_offsets()["e_bias"]
    p[o:o + 2] = [-1.25, 0.5]
    r = oracle.compute(fr.coords, fr.types, fr.box, desc, p, debug=True)
    return fr, desc, p, r


def test_fitting_net_layer_by_layer(w192):
    """E_i of every atom of both types from the oracle's D, evaluated again
    in numpy; every misreading is off by far more than rounding."""
    fr, desc, p, r = w192
    for t in range(desc.ntypes):
        idx = np.nonzero(fr.types == t)[0]
        var = _fit_variants(desc, p, t, r["D"][idx])
        assert np.allclose(var["reading"], r["Ei"][idx], rtol=0, atol=1e-12)
        for name in ("no_skip", "tanh_output", "tanh_fed"):
            assert np.abs(var[name] - r["Ei"][idx]).max() > 1e-2, name


def test_fitting_zero_hidden_weights_reduce_to_first_layer(w192):
    """W2 = W3 = 0 and b2 = b3 = 0: tanh(0) = 0, so the identity skips give
    h3 = h1 and E_i = tanh(D W1 + b1) . wo + bo + e_bias."""
    fr, desc, p, _ = w192
    q = p.copy()
    off = desc.param_offsets()
    for t in range(desc.ntypes):
        for nm in (f"fit{t}.W2", f"fit{t}.b2", f"fit{t}.W3", f"fit{t}.b3"):
            o, shp = off[nm]
            q[o:o + int(np.prod(shp))] = 0.0
    r = oracle.compute(fr.coords, fr.types, fr.box, desc, q, debug=True)
    for t in range(desc.ntypes):
        idx = np.nonzero(fr.types == t)[0]
        h1 = np.tanh(r["D"][idx] @ _blk(desc, q, f"fit{t}.W1") + _blk(desc, q, f"fit{t}.b1"))
        want = h1 @ _blk(desc, q, f"fit{t}.wo") + _blk(desc, q, f"fit{t}.bo")[0] + _blk(desc, q, "e_bias")[t]
        assert np.allclose(r["Ei"][idx], want, rtol=0, atol=1e-12)


def test_output_layer_is_linear(w192):
    """E_i - bo - e_bias scales linearly with w_out (no output activation)."""
    fr, desc, p, r0 = w192
    off = desc.param_offsets()
    q = p.copy()
    for t in range(desc.ntypes):
        o, shp = off[f"fit{t}.wo"]
        q[o:o + shp[0]] *= -2.5
    r1 = oracle.compute(fr.coords, fr.types, fr.box, desc, q)
    const = np.array([_blk(desc, p, f"fit{t}.bo")[0] + _blk(desc, p, "e_bias")[t] for t in fr.types])
    assert np.allclose(r1["Ei"] - const, -2.5 * (r0["Ei"] - const), rtol=1e-12, atol=1e-12)
    # forces scale the same way (the constants carry no gradient)
    assert np.allclose(r1["F"], -2.5 * r0["F"], rtol=1e-11, atol=1e-12)


def _one_neighbour(dvec, types):
    L = 20.0
    x = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0]]) + np.array([[0, 0, 0], dvec])
    return x, np.array(types, dtype=np.int32), np.diag([L, L, L])


@pytest.mark.parametrize("types", [(0, 1), (1, 0), (1, 1), (0, 0)])
def test_embedding_net_single_neighbour(types):
    """One neighbour: T = G(s) R~^T / N_m.  G is evaluated again in numpy
    from the flat parameters with non-zero weights and biases in all three
    layers (integer-ish weights of moderate size so that no layer saturates),
    for every (centre, neighbour) type pair."""
    desc = I.WATER
    rng = np.random.default_rng(17 + 2 * types[0] + types[1])
    p = I.init_params(desc, 5)
    off = desc.param_offsets()
    ti, tj = types
    for l, scale in ((1, 0.25), (2, 0.125), (3, 0.0625)):
        o, shp = off[f"emb{ti}{tj}.W{l}"]
        p[o:o + int(np.prod(shp))] = scale * rng.integers(-3, 4, size=int(np.prod(shp)))
        o, shp = off[f"emb{ti}{tj}.b{l}"]
        p[o:o + int(np.prod(shp))] = 0.25 * rng.integers(-2, 3, size=int(np.prod(shp)))
    dv = np.array([1.3, -0.7, 0.4])
    x, t, box = _one_neighbour(dv, types)
    r = oracle.compute(x, t, box, desc, p, debug=True)
    slot = desc.sel[0] if tj == 1 else 0          # first slot of the neighbour's section
    R = r["R"][0, slot]
    var = _emb_variants(desc, p, ti, tj, R[0])
    G = var["reading"]
    assert np.allclose(r["T"][0], np.outer(G, R) / desc.nm, rtol=1e-13, atol=1e-16)
    for name in ("no_skip", "skip_h_0", "skip_interleaved", "tanh_fed"):
        Gm = var[name]
        assert np.abs(np.outer(Gm, R) / desc.nm - r["T"][0]).max() > 1e-3 * np.abs(r["T"][0]).max(), name


def test_embedding_net_many_neighbours_descriptor():
    """Every neighbour of a water192 atom: T = sum_j G(s_j) R~_j^T / N_m with
    G from numpy and R~ from the oracle, then D = T T<^T; compared with the
    oracle's T and D for one atom of each type."""
    fr, desc, p, _ = I.workload("water192")
    r = oracle.compute(fr.coords, fr.types, fr.box, desc, p, debug=True, rows=[0, 1])
    for q, i in enumerate((0, 1)):
        ti = int(fr.types[i])
        T = np.zeros((desc.m1, 4))
        for tj in range(desc.ntypes):
            lo = sum(desc.sel[:tj])
            for slot in range(lo, lo + desc.sel[tj]):
                if r["nlist"][q, slot] < 0:
                    continue
                R = r["R"][q, slot]
                T += np.outer(_emb_variants(desc, p, ti, tj, R[0])["reading"], R)
        T /= desc.nm
        assert np.allclose(r["T"][q], T, rtol=1e-12, atol=1e-15)
        D = T @ T[:desc.m2].T
        assert np.allclose(r["D"][q], D.reshape(-1), rtol=1e-12, atol=1e-16)
