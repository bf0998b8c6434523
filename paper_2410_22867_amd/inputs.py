"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds geometry generators, the model hyper-parameters of the two
workloads named in the Evaluation section (water: cut-off 6 A, copper: 8 A,
fitting net (240, 240, 240), time steps 0.5 / 1.0 fs) and a seeded parameter
initialiser.  It contains none of the Deep Potential arithmetic (no switching
function, no network evaluation): both the CPU oracle and the GPU path read
the arrays produced here and interpret them on their own.

Units are "metal": Angstrom, eV, amu, fs.  Boxes are given as a 3x3 matrix of
row vectors (orthorhombic boxes are diagonal).  Coordinates are wrapped into
[0, L) along every axis.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

# O-H bond length and H-O-H angle of the water molecules (rigid geometry used
# only to place atoms; the potential itself is a random-weight Deep Potential).
OH_BOND = 0.9572
HOH_ANGLE_DEG = 104.52
WATER_VOLUME_PER_MOL = 29.915  # A^3 per molecule at 1 g/cm^3
MIN_OO = 2.5

MASS_O = 15.9994
MASS_H = 1.00794
MASS_CU = 63.546


@dataclasses.dataclass(frozen=True)
class ModelDesc:
    """Hyper-parameters of a DP se_a model (Evaluation section).

    ``sel[t]`` is the number of neighbour slots reserved for neighbours of type
    ``t``; the slots of all types concatenated give the padded neighbour count
    ``nm = sum(sel)``.  ``emb`` are the embedding-net widths (input width 1),
    ``m2`` the number of axis neurons, ``fit`` the fitting-net hidden widths.
    """

    ntypes: int
    rcut: float
    rcut_smth: float
    sel: Tuple[int, ...]
    emb: Tuple[int, ...]
    m2: int
    fit: Tuple[int, ...]
    masses: Tuple[float, ...]
    std_s: float = 1.0
    std_v: float = 1.0

    @property
    def nm(self) -> int:
        return int(sum(self.sel))

    @property
    def m1(self) -> int:
        return int(self.emb[-1])

    @property
    def ndesc(self) -> int:
        return self.m1 * self.m2

    def layer_shapes(self) -> List[Tuple[str, Tuple[int, ...]]]:
        """Names and shapes of every parameter block in flat-vector order.

        Order: embedding nets for (centre type, neighbour type) in row-major
        order, each as W_1, b_1, ..., W_L, b_L with W_l of shape
        [w_{l-1}, w_l] (row-major); then one fitting net per centre type as
        W_1, b_1, ..., W_L, b_L, w_out [w_L], b_out [1]; then e_bias[ntypes].
        """
        out = []
        for ti in range(self.ntypes):
            for tj in range(self.ntypes):
                prev = 1
                for l, w in enumerate(self.emb):
                    out.append((f"emb{ti}{tj}.W{l + 1}", (prev, w)))
                    out.append((f"emb{ti}{tj}.b{l + 1}", (w,)))
                    prev = w
        for t in range(self.ntypes):
            prev = self.ndesc
            for l, w in enumerate(self.fit):
                out.append((f"fit{t}.W{l + 1}", (prev, w)))
                out.append((f"fit{t}.b{l + 1}", (w,)))
                prev = w
            out.append((f"fit{t}.wo", (prev,)))
            out.append((f"fit{t}.bo", (1,)))
        out.append(("e_bias", (self.ntypes,)))
        return out

    @property
    def n_params(self) -> int:
        return int(sum(int(np.prod(s)) for _, s in self.layer_shapes()))

    def param_offsets(self) -> dict:
        off, d = 0, {}
        for name, shape in self.layer_shapes():
            n = int(np.prod(shape))
            d[name] = (off, shape)
            off += n
        return d


# Environment statistics: the trained models of the paper carry per-column
# normalisation of the environment matrix learned from data; with no data the
# mean is fixed at 0 (padded rows stay exactly 0) and sigma at about half the
# column spread measured on these synthetic systems, which gives the random
# model force magnitudes of order 0.1 eV/A on water.
WATER = ModelDesc(ntypes=2, rcut=6.0, rcut_smth=0.5, sel=(46, 92),
                  emb=(25, 50, 100), m2=16, fit=(240, 240, 240),
                  masses=(MASS_O, MASS_H), std_s=0.08, std_v=0.05)
COPPER = ModelDesc(ntypes=1, rcut=8.0, rcut_smth=2.0, sel=(500,),
                   emb=(32, 64, 128), m2=16, fit=(240, 240, 240),
                   masses=(MASS_CU,), std_s=0.05, std_v=0.035)

# DP-compress grids (x_fine, x_max, h) of the embedding input x = s(r)/std_s:
# the fine stride covers r >= 0.5 A for water (r_s, where s = 2/A) and
# r >= 1.5 A for copper; a coarse stride of 10 h continues to r = 0.01 A and
# 0.05 A (the random models let atoms approach far closer than real ones; at
# such inputs the first layer's tanh is saturated and G nearly constant).
COMPRESS_GRID_WATER = (25.0, 1250.0, 0.1)
COMPRESS_GRID_COPPER = (14.0, 400.0, 0.1)

DT_WATER_FS = 0.5
DT_COPPER_FS = 1.0
MODEL_SEED_WATER = 100
MODEL_SEED_COPPER = 101


# Output-layer scale of the water workloads' model.  A random-weight model
# has no repulsive core and no bonds: with the plain Xavier output layer its
# forces (RMS 0.15 eV/A on water12k) heat the 300 K liquid by thousands of
# kelvin within a few hundred femtoseconds and drive local densities past the
# sel = (46, 92) neighbour slots after ~70 steps.  One fixed factor on w_out
# (negative: the sign that, for this seed, pushes crowded neighbourhoods
# apart) keeps the 12,288-atom liquid within sel for 1000 velocity-Verlet
# steps at 0.5 fs with forces of RMS 15 meV/A.  Negation is exact in floating
# point and the scale only multiplies E_i - b_out - e_bias and every force,
# so relative errors are those of the unscaled model's output rescaled.
WATER_OUTPUT_SCALE = -0.1


def init_params(desc: ModelDesc, seed: int, out_scale: float = 1.0) -> np.ndarray:
    """Flat float64 parameter vector: Xavier-normal weights
    (std = sqrt(2 / (fan_in + fan_out))), hidden biases N(0, 1), output bias 0,
    e_bias 0; the output weights w_out are multiplied by out_scale."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in desc.layer_shapes():
        if name == "e_bias" or name.endswith(".bo"):
            parts.append(np.zeros(shape))
        elif name.endswith(".wo"):
            fan_in = shape[0]
            parts.append(out_scale * rng.normal(0.0, math.sqrt(2.0 / (fan_in + 1)), size=shape))
        elif ".W" in name:
            fan_in, fan_out = shape
            parts.append(rng.normal(0.0, math.sqrt(2.0 / (fan_in + fan_out)), size=shape))
        else:
            parts.append(rng.normal(0.0, 1.0, size=shape))
    return np.ascontiguousarray(np.concatenate([p.reshape(-1) for p in parts]), dtype=np.float64)


@dataclasses.dataclass
class Frame:
    coords: np.ndarray   # [n, 3] float64, wrapped into [0, L)
    types: np.ndarray    # [n] int32
    box: np.ndarray      # [3, 3] float64 row vectors

    @property
    def n(self) -> int:
        return int(self.types.shape[0])


def _random_rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _wrap(x, L):
    y = np.mod(x, L)
    # np.mod can return L itself for tiny negative inputs; fold it back.
    y = np.where(y >= L, y - L, y)
    return y


def water_box(n_mol: int, L: float, seed: int) -> Frame:
    """n_mol rigid water molecules (O, H, H) in a cubic PBC box of edge L.

    Oxygens sit on the first n_mol sites (seeded permutation) of an m^3 lattice
    (m = ceil(n_mol^(1/3)), spacing L/m), jittered uniformly by +-0.1 spacing
    per axis; molecules get uniformly random orientations.  A molecule is
    re-jittered while any periodic O-O distance is below 2.5 A.
    """
    rng = np.random.default_rng(seed)
    m = int(math.ceil(round(n_mol ** (1.0 / 3.0), 9)))
    while m ** 3 < n_mol:
        m += 1
    a = L / m
    sites = rng.permutation(m ** 3)[:n_mol]
    ijk = np.stack([sites % m, (sites // m) % m, sites // (m * m)], axis=1)
    base = (ijk + 0.5) * a
    jit = rng.uniform(-0.1 * a, 0.1 * a, size=(n_mol, 3))
    # Occupancy grid for the O-O distance check (only lattice neighbours can
    # violate the bound since a >= 2.5 A / 0.8 in every supported box).
    grid = -np.ones((m, m, m), dtype=np.int64)
    grid[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = np.arange(n_mol)
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if (dx, dy, dz) > (0, 0, 0)]
    for _ in range(10000):
        o = base + jit
        bad = np.zeros(n_mol, dtype=bool)
        for dx, dy, dz in offs:
            nb = grid[(ijk[:, 0] + dx) % m, (ijk[:, 1] + dy) % m, (ijk[:, 2] + dz) % m]
            ok = nb >= 0
            ii = np.nonzero(ok)[0]
            jj = nb[ok]
            d = o[jj] - o[ii]
            d -= L * np.round(d / L)
            close = np.einsum("ij,ij->i", d, d) < MIN_OO * MIN_OO
            bad[ii[close]] = True
            bad[jj[close]] = True
        if not bad.any():
            break
        nb_ = int(bad.sum())
        jit[bad] = rng.uniform(-0.1 * a, 0.1 * a, size=(nb_, 3))
    else:
        raise RuntimeError("water_box: could not satisfy the O-O distance bound")
    o = base + jit
    half = math.radians(HOH_ANGLE_DEG) / 2.0
    h1 = np.array([OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)])
    h2 = np.array([-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)])
    R = _random_rotations(rng, n_mol)
    x = np.empty((n_mol, 3, 3))
    x[:, 0] = o
    x[:, 1] = o + R @ h1
    x[:, 2] = o + R @ h2
    coords = _wrap(x.reshape(-1, 3), L)
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), n_mol)
    return Frame(np.ascontiguousarray(coords), types, np.diag([L, L, L]).astype(np.float64))


def copper_fcc(ncell, a: float, sigma: float, seed: int) -> Frame:
    """FCC copper, ncell^3 (or nx x ny x nz for a triple) conventional cells
    of edge a, Gaussian displacements."""
    rng = np.random.default_rng(seed)
    nc = (ncell, ncell, ncell) if np.isscalar(ncell) else tuple(ncell)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(np.arange(nc[0]), np.arange(nc[1]), np.arange(nc[2]),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    x = ((g[:, None, :] + basis[None, :, :]) * a).reshape(-1, 3)
    x = x + rng.normal(0.0, sigma, size=x.shape)
    L = np.array(nc, dtype=np.float64) * a
    coords = _wrap(x, L)
    types = np.zeros(coords.shape[0], dtype=np.int32)
    return Frame(np.ascontiguousarray(coords), types, np.diag(L).astype(np.float64))


def water_density_box(n_mol: int) -> float:
    return (n_mol * WATER_VOLUME_PER_MOL) ** (1.0 / 3.0)


def water_batch(nframes: int, seed: int, lo: int = 64, hi: int = 1024):
    """Frames of uneven size (n_mol uniform in [lo, hi]) at 1 g/cm^3 and the
    seeded random target energies E_hat_f = N_f * z_f, z_f ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    nmols = rng.integers(lo, hi + 1, size=nframes)
    frames = [water_box(int(nm), water_density_box(int(nm)), seed * 1000 + f)
              for f, nm in enumerate(nmols)]
    z = rng.normal(size=nframes)
    targets = np.array([fr.n * z[f] for f, fr in enumerate(frames)], dtype=np.float64)
    return frames, targets


def maxwell_boltzmann(types: np.ndarray, masses, T: float, seed: int) -> np.ndarray:
    """Velocities [n, 3] in A/fs at temperature T (K): Gaussian, zero total
    momentum, rescaled to exactly T with 3n - 3 degrees of freedom."""
    KB = 8.617333262e-5           # eV/K
    MVV2E = 1.0 / 9.64853321e-3   # amu A^2/fs^2 -> eV
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)[types]
    sd = np.sqrt(KB * T / (m * MVV2E))
    v = rng.normal(size=(types.shape[0], 3)) * sd[:, None]
    p = (m[:, None] * v).sum(axis=0)
    v -= p / m.sum()
    ke = 0.5 * MVV2E * (m[:, None] * v * v).sum()
    dof = 3 * types.shape[0] - 3
    t_now = 2.0 * ke / (dof * KB)
    v *= math.sqrt(T / t_now)
    return np.ascontiguousarray(v)


# ---------------------------------------------------------------------------
# The five workloads.  Seeds: geometry = workload index, model = 100 (water) /
# 101 (copper), velocities = 200 + workload index.

def workload(name: str):
    """Returns (frame or (frames, targets), desc, params, dt_fs)."""
    if name == "water192":
        fr = water_box(64, 12.42, seed=0)
        return fr, WATER, init_params(WATER, MODEL_SEED_WATER, WATER_OUTPUT_SCALE), DT_WATER_FS
    if name == "water12k":
        fr = water_box(4096, 49.7, seed=1)
        return fr, WATER, init_params(WATER, MODEL_SEED_WATER, WATER_OUTPUT_SCALE), DT_WATER_FS
    if name == "copper32k":
        fr = copper_fcc(20, 3.634, 0.1, seed=2)
        return fr, COPPER, init_params(COPPER, MODEL_SEED_COPPER), DT_COPPER_FS
    if name == "water98k":
        fr = water_box(32768, 99.4, seed=3)
        return fr, WATER, init_params(WATER, MODEL_SEED_WATER, WATER_OUTPUT_SCALE), DT_WATER_FS
    # the strong-scaling systems of the Evaluation section, on one GPU:
    # 0.56 M atoms of water (185,856 molecules at 1 g/cm^3) and 0.54 M atoms
    # of copper (62 x 60 x 36 FCC cells)
    if name == "water557k":
        nmol = 185856
        fr = water_box(nmol, water_density_box(nmol), seed=5)
        return fr, WATER, init_params(WATER, MODEL_SEED_WATER, WATER_OUTPUT_SCALE), DT_WATER_FS
    if name == "copper535k":
        fr = copper_fcc((62, 60, 36), 3.634, 0.1, seed=6)
        return fr, COPPER, init_params(COPPER, MODEL_SEED_COPPER), DT_COPPER_FS
    if name == "waterbatch64":
        return water_batch(64, seed=4), WATER, init_params(WATER, MODEL_SEED_WATER, WATER_OUTPUT_SCALE), DT_WATER_FS
    raise KeyError(name)


WORKLOADS = ("water192", "water12k", "copper32k", "water98k", "waterbatch64", "water557k", "copper535k")
