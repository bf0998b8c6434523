"""Pins of the oracle's neighbour list (Background section, Fig. 1(a): the
neighbour list of atom i within the cut-off radius; Evaluation section: the
cut-offs and per-type neighbour counts).

* cell-list enumeration == brute-force enumeration, bit for bit;
* an independent numpy enumeration of all 27 images gives the same sets;
* a perfect FCC lattice reproduces the textbook coordination shells
  (tests/golden/fcc_shells.json);
* symmetry (j, s) in nl(i)  <=>  (i, -s) in nl(j);
* sorted order and the -1 padding / overflow count.
"""
import dataclasses
import json
import os

import numpy as np
import pytest

import oracle
from paper_2410_22867_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _decode(e):
    j = e // 27
    sc = e % 27
    return j, np.stack([sc % 3 - 1, (sc // 3) % 3 - 1, sc // 9 - 1], axis=-1)


def test_cell_equals_brute_water192():
    fr, desc, _, _ = I.workload("water192")
    a, ova = oracle.nlist(fr.coords, fr.types, fr.box, desc, use_cells=False)
    b, ovb = oracle.nlist(fr.coords, fr.types, fr.box, desc, use_cells=True)
    assert ova == ovb == 0
    assert np.array_equal(a, b)


def test_cell_equals_brute_small_copper_and_tiny_boxes():
    # 3x3x3 FCC cells: L = 10.9 A, one cell per dimension (L < 2 rc).
    fr = I.copper_fcc(3, 3.634, 0.1, seed=7)
    a, _ = oracle.nlist(fr.coords, fr.types, fr.box, I.COPPER, use_cells=False)
    b, _ = oracle.nlist(fr.coords, fr.types, fr.box, I.COPPER, use_cells=True)
    assert np.array_equal(a, b)
    # water at two cells per dimension (12.42 / 6 = 2.07)
    fr = I.water_box(64, 12.42, seed=11)
    a, _ = oracle.nlist(fr.coords, fr.types, fr.box, I.WATER, use_cells=False)
    b, _ = oracle.nlist(fr.coords, fr.types, fr.box, I.WATER, use_cells=True)
    assert np.array_equal(a, b)


def test_sets_match_numpy_enumeration():
    """Independent enumeration: all (j, s) with |x_j + s L - x_i| < rc."""
    fr = I.water_box(27, 9.3, seed=5)
    desc = I.WATER
    nl, _ = oracle.nlist(fr.coords, fr.types, fr.box, desc, use_cells=False)
    L = np.diag(fr.box)
    shifts = np.array([(sx, sy, sz) for sz in (-1, 0, 1) for sy in (-1, 0, 1) for sx in (-1, 0, 1)])
    for i in range(fr.n):
        d = fr.coords[None, :, :] + (shifts * L)[:, None, :] - fr.coords[i]
        r = np.sqrt((d * d).sum(-1))
        sidx, j = np.nonzero(r < desc.rcut)
        keep = ~((j == i) & np.all(shifts[sidx] == 0, axis=1))
        want = set()
        for jj, ss in zip(j[keep], sidx[keep]):
            sc = (shifts[ss][0] + 1) + 3 * (shifts[ss][1] + 1) + 9 * (shifts[ss][2] + 1)
            want.add(27 * int(jj) + int(sc))
        got = set(int(e) for e in nl[i] if e >= 0)
        assert got == want, i


def test_fcc_shells_golden():
    g = json.load(open(os.path.join(GOLD, "fcc_shells.json")))
    fr = I.copper_fcc(6, g["a"], 0.0, seed=0)   # perfect lattice, L = 21.8 A
    desc = I.COPPER
    nl, ov = oracle.nlist(fr.coords, fr.types, fr.box, desc)
    assert ov == 0
    counts = (nl >= 0).sum(1)
    assert np.all(counts == g["total_within_rcut"])
    # shell structure of atom 0: sorted r^2 follows the golden multiplicities
    j, s = _decode(nl[0][nl[0] >= 0])
    d = fr.coords[j] + s * np.diag(fr.box) - fr.coords[0]
    r2 = (d * d).sum(1) / g["a"] ** 2
    assert np.all(np.diff(r2) >= -1e-12)
    shells = np.round(r2 * 2) / 2
    vals, mult = np.unique(shells, return_counts=True)
    assert np.allclose(vals, g["r2_over_a2"])
    assert list(mult) == g["multiplicity"]


def test_symmetry_sorting_and_padding():
    fr, desc, _, _ = I.workload("water192")
    nl, ov = oracle.nlist(fr.coords, fr.types, fr.box, desc)
    assert ov == 0
    L = np.diag(fr.box)
    pairs = set()
    for i in range(fr.n):
        sec_off = 0
        for t, sel in enumerate(desc.sel):
            row = nl[i, sec_off:sec_off + sel]
            real = row[row >= 0]
            # padding only at the end of a section
            assert np.all(row[len(real):] == -1)
            j, s = _decode(real)
            assert np.all(fr.types[j] == t)
            d = (fr.coords[j] - fr.coords[i]) + s * L
            r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            key = list(zip(r2, real))
            assert key == sorted(key)
            for jj, ss in zip(j, s):
                pairs.add((i, int(jj), tuple(ss)))
            sec_off += sel
    for i, j, s in pairs:
        assert (j, i, tuple(-np.array(s))) in pairs


def test_density_counts_water12k():
    """~30 O and ~60 H neighbours within 6 A at 1 g/cm^3 (0.0334 molecules/A^3
    times the cut-off sphere volume 904.8 A^3); no section overflow."""
    fr, desc, _, _ = I.workload("water12k")
    rows = np.arange(0, fr.n, 97)
    nl, ov = oracle.nlist(fr.coords, fr.types, fr.box, desc, rows=rows)
    assert ov == 0
    nO = (nl[:, :46] >= 0).sum(1).mean()
    nH = (nl[:, 46:] >= 0).sum(1).mean()
    assert 26 < nO < 33 and 54 < nH < 64


def test_overflow_is_counted():
    fr, desc, _, _ = I.workload("water192")
    small = dataclasses.replace(desc, sel=(10, 20))
    nl, ov = oracle.nlist(fr.coords, fr.types, fr.box, small)
    full, _ = oracle.nlist(fr.coords, fr.types, fr.box, desc)
    nO = (full[:, :46] >= 0).sum(1)
    nH = (full[:, 46:] >= 0).sum(1)
    assert ov == int(np.maximum(nO - 10, 0).sum() + np.maximum(nH - 20, 0).sum())
    # truncation keeps the nearest: prefix of the untruncated sections
    assert np.array_equal(nl[:, :10], full[:, :10])
    assert np.array_equal(nl[:, 10:30], full[:, 46:66])
