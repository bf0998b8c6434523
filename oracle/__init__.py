"""FP64 CPU oracle for Deep Potential se_a energy, forces, virial, parameter
gradients and velocity-Verlet NVE.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2410_22867_amd``) and never imports it.

The arithmetic lives in ``dp_oracle.c`` (plain C, OpenMP over independent
atoms, ``-O2 -ffp-contract=off``); this module only marshals arrays.  Every
function is pinned by ``tests/test_oracle_*.py`` against closed forms, brute
force, invariances and finite differences (see the module docstrings there).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

KCAL = None
MVV2E = 1.0 / 9.64853321e-3   # amu A^2 / fs^2 -> eV
FTM2V = 9.64853321e-3         # eV / (A amu) -> A / fs^2
KB = 8.617333262e-5           # eV / K


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.or_nparams.argtypes = [P, P]
        L.or_nparams.restype = i64
        L.or_nlist.argtypes = [i64, P, P, P, P, P, P, i64, ctypes.c_int, P, P]
        L.or_nlist.restype = ctypes.c_int
        L.or_compute.argtypes = [i64, P, P, P, P, P, P, P, i64, P, P, P, P, P, P, ctypes.c_double,
                                 P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.or_tab_nint.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_tab_nint.restype = ctypes.c_int
        L.or_tab_build.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.or_tab_build.restype = ctypes.c_int
        L.or_compute.restype = ctypes.c_int
        L.or_switch_fn.argtypes = [i64, P, ctypes.c_double, ctypes.c_double, P, P]
        L.or_switch_fn.restype = None
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def desc_arrays(desc):
    idesc = [desc.ntypes] + list(desc.sel) + [len(desc.emb)] + list(desc.emb) + [desc.m2, len(desc.fit)] + list(desc.fit)
    return (np.ascontiguousarray(idesc, dtype=np.int32),
            np.ascontiguousarray([desc.rcut, desc.rcut_smth, desc.std_s, desc.std_v], dtype=np.float64))


def n_params(desc) -> int:
    i, d = desc_arrays(desc)
    return int(lib().or_nparams(_ptr(i), _ptr(d)))


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def num_threads() -> int:
    return int(lib().or_num_threads())


def switch(r: np.ndarray, rs: float, rc: float):
    """s(r) and ds/dr of the quintic switch (FP64)."""
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
    s = np.empty_like(r)
    ds = np.empty_like(r)
    lib().or_switch_fn(r.size, _ptr(r), float(rs), float(rc), _ptr(s), _ptr(ds))
    return s, ds


def nlist(coords, types, box, desc, rows: Optional[Sequence[int]] = None, use_cells: bool = True):
    """Formatted neighbour rows [nrows, nm] (int32 packed 27*j + scode, -1 pad)
    and the overflow count.  use_cells requires an orthorhombic box."""
    x = np.ascontiguousarray(coords, dtype=np.float64)
    t = np.ascontiguousarray(types, dtype=np.int32)
    h = np.ascontiguousarray(box, dtype=np.float64).reshape(9)
    i, d = desc_arrays(desc)
    n = t.shape[0]
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nrows = n if r is None else r.shape[0]
    out = np.empty((nrows, desc.nm), dtype=np.int32)
    ov = np.zeros(1, dtype=np.int64)
    rc = lib().or_nlist(n, _ptr(x), _ptr(t), _ptr(h), _ptr(i), _ptr(d), _ptr(r), nrows, int(bool(use_cells)),
                        _ptr(out), _ptr(ov))
    if rc != 0:
        raise ValueError("or_nlist failed (bad types, non-orthorhombic box with cells, or capacity)")
    return out, int(ov[0])


def tabulate(desc, params, x1: float, x2: float, h: float) -> np.ndarray:
    """DP-compress table of every embedding net: [ntypes^2, nint, 6, m1]
    quintic coefficients on the grid (fine stride h on [0, x1), 10 h up to
    x2; see dp_oracle.c)."""
    i, d = desc_arrays(desc)
    nint = int(lib().or_tab_nint(float(x1), float(x2), float(h)))
    if nint <= 0:
        raise ValueError("bad table grid")
    p = np.ascontiguousarray(params, dtype=np.float64)
    out = np.empty((desc.ntypes ** 2, nint, 6, desc.m1), dtype=np.float64)
    if lib().or_tab_build(_ptr(i), _ptr(d), _ptr(p), float(x1), float(x2), float(h), _ptr(out)) != 0:
        raise ValueError("or_tab_build failed")
    return out


def compute(coords, types, box, desc, params, rows=None, nl=None, grad_scale: Optional[float] = None,
            debug: bool = False, use_cells: bool = True, table=None):
    """Energy, per-atom energies, forces [n,3], virial [3,3] of one frame.

    rows: centre atoms to evaluate (None: all).  With a subset, E and Ei cover
    only those atoms and F/W only their contributions.  grad_scale: if given,
    also returns grad = grad_scale * dE/dtheta (flat parameter layout).
    table: (coefficients from tabulate(), x1, x2, h) to evaluate the
    embedding nets from the DP-compress table instead; the result then also
    holds "clipped", the count of inputs at or beyond the table's end."""
    x = np.ascontiguousarray(coords, dtype=np.float64)
    t = np.ascontiguousarray(types, dtype=np.int32)
    h = np.ascontiguousarray(box, dtype=np.float64).reshape(9)
    p = np.ascontiguousarray(params, dtype=np.float64)
    i, d = desc_arrays(desc)
    n = t.shape[0]
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nrows = n if r is None else r.shape[0]
    if nl is None:
        nl, ov = nlist(x, t, h.reshape(3, 3), desc, rows=r, use_cells=use_cells)
    nl = np.ascontiguousarray(nl, dtype=np.int32)
    assert nl.shape == (nrows, desc.nm)
    E = np.zeros(1)
    Ei = np.zeros(nrows)
    F = np.zeros((n, 3))
    W = np.zeros(9)
    grad = np.zeros(n_params(desc)) if grad_scale is not None else None
    dbg = {}
    if debug:
        dbg = dict(R=np.zeros((nrows, desc.nm, 4)), T=np.zeros((nrows, desc.m1, 4)),
                   D=np.zeros((nrows, desc.ndesc)), gD=np.zeros((nrows, desc.ndesc)),
                   gT=np.zeros((nrows, desc.m1, 4)), netd=np.zeros((nrows, desc.nm, 4)))
    tab, tx1, tx2, th = (None, 0.0, 0.0, 0.0) if table is None else table
    if tab is not None:
        tab = np.ascontiguousarray(tab, dtype=np.float64)
    nclip = np.zeros(1, dtype=np.int64)
    rc = lib().or_compute(n, _ptr(x), _ptr(t), _ptr(h), _ptr(i), _ptr(d), _ptr(p), _ptr(r), nrows, _ptr(nl),
                          _ptr(E), _ptr(Ei), _ptr(F), _ptr(W), _ptr(grad),
                          float(grad_scale) if grad_scale is not None else 0.0,
                          _ptr(dbg.get("R")), _ptr(dbg.get("T")), _ptr(dbg.get("D")), _ptr(dbg.get("gD")),
                          _ptr(dbg.get("gT")), _ptr(dbg.get("netd")), _ptr(tab), float(tx1), float(tx2), float(th),
                          _ptr(nclip))
    if rc != 0:
        raise ValueError("or_compute failed")
    out = dict(E=float(E[0]), Ei=Ei, F=F, W=W.reshape(3, 3), nlist=nl)
    if table is not None:
        out["clipped"] = int(nclip[0])
    if grad is not None:
        out["grad"] = grad
    out.update(dbg)
    return out


def atoms_touching(nl_rows: np.ndarray, k: int) -> np.ndarray:
    """Atom indices j appearing in atom k's neighbour row (plus k itself)."""
    e = nl_rows[nl_rows >= 0]
    return np.unique(np.concatenate([[k], e // 27]))


def force_on(coords, types, box, desc, params, k: int, use_cells: bool = True) -> np.ndarray:
    """Total force on atom k, computed from the atoms whose neighbour lists can
    contain k.  With no section overflow the lists are symmetric, so these are
    k itself and the atoms in k's own list."""
    row, _ = nlist(coords, types, box, desc, rows=[k], use_cells=use_cells)
    cen = atoms_touching(row, k)
    res = compute(coords, types, box, desc, params, rows=cen, use_cells=use_cells)
    return res["F"][k]


# ---------------------------------------------------------------------------
# Velocity-Verlet NVE (metal units): a = F/m * FTM2V,
#   v(t+dt/2) = v(t) + dt/2 a(t);  x(t+dt) = x(t) + dt v(t+dt/2);
#   v(t+dt)   = v(t+dt/2) + dt/2 a(t+dt).

def kinetic_energy(v: np.ndarray, m: np.ndarray) -> float:
    return float(0.5 * MVV2E * np.sum(m[:, None] * v * v))


def nve(x0, v0, m, force_fn, dt: float, nsteps: int, wrap_box: Optional[np.ndarray] = None):
    """Integrates nsteps velocity-Verlet steps.  force_fn(x) -> (E, F).
    Returns (x, v, list of (E_pot, E_kin) at every step including step 0).
    wrap_box: orthorhombic edge lengths to wrap positions into [0, L)."""
    x = np.array(x0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    E, F = force_fn(x)
    hist = [(E, kinetic_energy(v, m))]
    for _ in range(nsteps):
        v = v + 0.5 * dt * FTM2V * F / m[:, None]
        x = x + dt * v
        if wrap_box is not None:
            L = np.asarray(wrap_box, dtype=np.float64)
            x = x - np.floor(x / L) * L
            x = np.where(x >= L, x - L, x)
        E, F = force_fn(x)
        v = v + 0.5 * dt * FTM2V * F / m[:, None]
        hist.append((E, kinetic_energy(v, m)))
    return x, v, hist
