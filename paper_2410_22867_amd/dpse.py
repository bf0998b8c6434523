"""Python binding of libdpse (include/dp.h): argument marshalling only.

Every step of the hot path runs in the HIP kernels of ``libdpse.so``; PyTorch
is used for device memory and the current stream.  Importing works without a
GPU; any call that needs the library raises if it is not built, and calls
that need a device fail with the library's own error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpse.so")

DP_FP64, DP_MIX_BF16, DP_MIX_FP16, DP_MIX_FP32, DP_MIX_FP16_FIT1 = 0, 1, 2, 3, 4
# "mix_fp32" and "mix_fp16" are the paper's MIX-fp32 (both nets in FP32) and
# MIX-fp16 (MIX-fp32 with the first fitting layer's products in FP16)
DP_FP64_TAB = 5
MODES = {"fp64": DP_FP64, "bf16": DP_MIX_BF16, "fp16": DP_MIX_FP16, "mix_fp32": DP_MIX_FP32,
         "mix_fp16": DP_MIX_FP16_FIT1, "fp64_tab": DP_FP64_TAB}

FLAG_NOT_WRAPPED, FLAG_OVERLAP, FLAG_NONFINITE, FLAG_CAND_CAPACITY, FLAG_SEL_OVERFLOW = 1, 2, 4, 8, 16
FLAG_BAD_INPUT, FLAG_SKIN_EXCEEDED, FLAG_TABLE_RANGE = 32, 64, 128

BUF_ENV, BUF_T, BUF_D, BUF_GD, BUF_NETD, BUF_GT = 0, 1, 2, 3, 4, 5

# Symbols declared in include/dp.h (checked by the CPU tests).
EXPORTS = ("dp_model_n_params", "dp_model_create", "dp_model_set_params", "dp_model_set_params_device",
           "dp_model_destroy", "dp_ctx_create",
           "dp_ctx_destroy", "dp_build_nlist", "dp_build_nlist_batch", "dp_nlist_skin_build", "dp_nlist_skin_format",
           "dp_nlist_skin_update", "dp_build_nlist_noalloc", "dp_model_compress", "dp_model_copy_table",
           "dp_compute", "dp_compute_batch",
           "dp_backward_params", "dp_md_kick_drift", "dp_md_kick", "dp_ctx_status", "dp_ctx_store_info",
           "dp_ctx_copy_buffer", "dp_ctx_profile", "dp_ctx_stage_times", "dp_last_error")

STAGES = ("nlist", "typesort", "env", "embed_fwd", "descriptor", "fit_fwd", "fit_bwd", "desc_bwd", "embed_bwd",
          "force", "reduce", "md")


class DPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdpse error {code}: {msg}")
        self.code = code


class ModelDesc(ctypes.Structure):
    _fields_ = [("ntypes", ctypes.c_int32), ("sel", ctypes.c_int32 * 4), ("n_emb", ctypes.c_int32),
                ("emb", ctypes.c_int32 * 4), ("m2", ctypes.c_int32), ("n_fit", ctypes.c_int32),
                ("fit", ctypes.c_int32 * 4), ("rcut", ctypes.c_double), ("rcut_smth", ctypes.c_double),
                ("std_s", ctypes.c_double), ("std_v", ctypes.c_double), ("masses", ctypes.c_double * 4)]


def make_desc(d) -> ModelDesc:
    """ctypes descriptor from any object with the ModelDesc fields of
    ``inputs.ModelDesc``."""
    c = ModelDesc()
    c.ntypes = d.ntypes
    for t, v in enumerate(d.sel):
        c.sel[t] = v
    c.n_emb = len(d.emb)
    for l, v in enumerate(d.emb):
        c.emb[l] = v
    c.m2 = d.m2
    c.n_fit = len(d.fit)
    for l, v in enumerate(d.fit):
        c.fit[l] = v
    c.rcut, c.rcut_smth, c.std_s, c.std_v = d.rcut, d.rcut_smth, d.std_s, d.std_v
    for t, v in enumerate(d.masses):
        c.masses[t] = v
    return c


_lib = None


def lib():
    """Loads libdpse.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libdpse.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "dp_model_n_params": (i64, [P]),
            "dp_model_create": (ctypes.c_int, [P, P, i64, PP]),
            "dp_model_set_params": (ctypes.c_int, [P, P, i64]),
            "dp_model_set_params_device": (ctypes.c_int, [P, P, i64, P]),
            "dp_model_destroy": (ctypes.c_int, [P]),
            "dp_ctx_create": (ctypes.c_int, [P, i64, i32, i64, PP]),
            "dp_ctx_destroy": (ctypes.c_int, [P]),
            "dp_build_nlist": (ctypes.c_int, [P, P, P, P, i64, P, P, P]),
            "dp_build_nlist_batch": (ctypes.c_int, [P, P, P, P, P, i32, P, P, P]),
            "dp_compute": (ctypes.c_int, [P, P, P, P, i64, P, i32, P, P, P, P, P]),
            "dp_compute_batch": (ctypes.c_int, [P, P, P, P, P, i32, P, i32, P, P, P, P]),
            "dp_backward_params": (ctypes.c_int, [P, P, P, P]),
            "dp_md_kick_drift": (ctypes.c_int, [P, P, P, P, P, P, i64, dbl, i32, P, P]),
            "dp_nlist_skin_build": (ctypes.c_int, [P, P, P, P, i64, dbl, P, P]),
            "dp_nlist_skin_format": (ctypes.c_int, [P, P, P, i64, P, P, P]),
            "dp_nlist_skin_update": (ctypes.c_int, [P, P, P, i64, i32, P, P, P, P, P]),
            "dp_build_nlist_noalloc": (ctypes.c_int, [P, P, P, P, i64, P, P, P, P]),
            "dp_model_compress": (ctypes.c_int, [P, dbl, dbl, dbl]),
            "dp_model_copy_table": (ctypes.c_int, [P, P, ctypes.POINTER(i64)]),
            "dp_md_kick": (ctypes.c_int, [P, P, P, P, i64, dbl, P, P]),
            "dp_ctx_status": (ctypes.c_int, [P, ctypes.POINTER(i32)]),
            "dp_ctx_store_info": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
            "dp_ctx_copy_buffer": (ctypes.c_int, [P, i32, P, ctypes.POINTER(i64), P]),
            "dp_ctx_profile": (ctypes.c_int, [P, i32]),
            "dp_ctx_stage_times": (ctypes.c_int, [P, P, P]),
            "dp_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise DPError(rc, lib().dp_last_error().decode())


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _box9(box) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(9))


class Model:
    """Device copy of a DP se_a model (dp_model_create)."""

    def __init__(self, desc, params: np.ndarray):
        self.desc = desc
        self._cdesc = make_desc(desc)
        p = np.ascontiguousarray(params, dtype=np.float64)
        self.n_params = int(p.size)
        h = ctypes.c_void_p()
        _check(lib().dp_model_create(ctypes.byref(self._cdesc), p.ctypes.data, p.size, ctypes.byref(h)))
        self.handle = h

    def set_params(self, params: np.ndarray) -> None:
        p = np.ascontiguousarray(params, dtype=np.float64)
        _check(lib().dp_model_set_params(self.handle, p.ctypes.data, p.size))

    def compress(self, x_fine: float, x_max: float, h: float) -> None:
        """DP-compress tables of the embedding nets (dp_model_compress)."""
        self.tab_grid = (float(x_fine), float(x_max), float(h))
        _check(lib().dp_model_compress(self.handle, *self.tab_grid))

    def table(self):
        """The device table as a float64 tensor [ntypes^2, nint, 6, m1]."""
        import torch
        nv = ctypes.c_int64(0)
        _check(lib().dp_model_copy_table(self.handle, None, ctypes.byref(nv)))
        out = torch.empty(int(nv.value), dtype=torch.float64, device="cuda")
        _check(lib().dp_model_copy_table(self.handle, _ptr(out), ctypes.byref(nv)))
        nt = self.desc.ntypes
        return out.reshape(nt * nt, -1, 6, self.desc.m1)

    def load_params(self, params) -> None:
        """Parameters from a device float64 tensor [n_params], on the current
        stream (no host round trip, no wait)."""
        if params.dtype != __import__("torch").float64 or not params.is_cuda or params.numel() != self.n_params:
            raise ValueError("load_params needs a float64 device tensor of n_params values")
        p = params.contiguous()
        _check(lib().dp_model_set_params_device(self.handle, _ptr(p), self.n_params, _stream()))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().dp_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_nlist_noalloc(model: Model, coords, types, box, out, overflow, flags=None) -> None:
    """dp_build_nlist_noalloc: the neighbour list into caller buffers, with
    no context and no device allocation by the library."""
    n = int(types.shape[0])
    _check(lib().dp_build_nlist_noalloc(model.handle, _ptr(coords), _ptr(types), _box9(box).ctypes.data, n,
                                        _ptr(out), _ptr(overflow), _ptr(flags), _stream()))


def n_params(desc) -> int:
    c = make_desc(desc)
    return int(lib().dp_model_n_params(ctypes.byref(c)))


class Context:
    """Work buffers for up to max_atoms atoms in max_frames frames (dp_ctx_create)."""

    def __init__(self, model: Model, max_atoms: int, max_frames: int = 1, budget_bytes: int = 0):
        self.model = model
        self.max_atoms = int(max_atoms)
        h = ctypes.c_void_p()
        _check(lib().dp_ctx_create(model.handle, int(max_atoms), int(max_frames), int(budget_bytes),
                                   ctypes.byref(h)))
        self.handle = h

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().dp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ nlist
    def build_nlist(self, coords, types, box, out=None, overflow=None):
        import torch
        n = int(types.shape[0])
        nm = int(sum(self.model.desc.sel))
        if out is None:
            out = torch.empty((n, nm), dtype=torch.int32, device=coords.device)
        if overflow is None:
            overflow = torch.empty(1, dtype=torch.int32, device=coords.device)
        b = _box9(box)
        _check(lib().dp_build_nlist(self.handle, _ptr(coords), _ptr(types), b.ctypes.data, n, _ptr(out),
                                    _ptr(overflow), _stream()))
        return out, overflow

    def skin_build(self, coords, types, box, skin, images=None):
        """Verlet build: wraps coords in place (images updated when given) and
        keeps every pair image within r_c + skin."""
        _check(lib().dp_nlist_skin_build(self.handle, _ptr(coords), _ptr(types), _box9(box).ctypes.data,
                                         int(types.shape[0]), float(skin), _ptr(images), _stream()))

    def skin_format(self, coords, types, out=None, overflow=None):
        """Sorted, truncated list on the current positions from the last Verlet build."""
        import torch
        n = int(types.shape[0])
        nm = int(sum(self.model.desc.sel))
        if out is None:
            out = torch.empty((n, nm), dtype=torch.int32, device=coords.device)
        if overflow is None:
            overflow = torch.empty(1, dtype=torch.int32, device=coords.device)
        _check(lib().dp_nlist_skin_format(self.handle, _ptr(coords), _ptr(types), n, _ptr(out), _ptr(overflow),
                                          _stream()))
        return out, overflow

    def skin_update(self, coords, types, every=0, images=None, out=None, overflow=None, rebuilds=None):
        """Verlet list of one MD step: rebuilt on the device when an atom moved
        beyond skin/2 (or every `every` updates), then formatted."""
        import torch
        n = int(types.shape[0])
        nm = int(sum(self.model.desc.sel))
        if out is None:
            out = torch.empty((n, nm), dtype=torch.int32, device=coords.device)
        if overflow is None:
            overflow = torch.empty(1, dtype=torch.int32, device=coords.device)
        _check(lib().dp_nlist_skin_update(self.handle, _ptr(coords), _ptr(types), n, int(every), _ptr(images),
                                          _ptr(out), _ptr(overflow), _ptr(rebuilds), _stream()))
        return out, overflow

    def build_nlist_batch(self, coords, types, boxes, frame_off, out=None, overflow=None):
        import torch
        n = int(types.shape[0])
        nm = int(sum(self.model.desc.sel))
        if out is None:
            out = torch.empty((n, nm), dtype=torch.int32, device=coords.device)
        if overflow is None:
            overflow = torch.empty(1, dtype=torch.int32, device=coords.device)
        bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 9))
        off = np.ascontiguousarray(frame_off, dtype=np.int64)
        _check(lib().dp_build_nlist_batch(self.handle, _ptr(coords), _ptr(types), bx.ctypes.data, off.ctypes.data,
                                          bx.shape[0], _ptr(out), _ptr(overflow), _stream()))
        return out, overflow

    # ------------------------------------------------------------ compute
    def compute(self, coords, types, box, nlist, mode="fp64", energy=None, atom_energy=None, forces=None,
                virial=None, want_atom_energy=False):
        import torch
        n = int(types.shape[0])
        dev = coords.device
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=dev)
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=dev)
        if virial is None:
            virial = torch.empty(9, dtype=torch.float64, device=dev)
        if atom_energy is None and want_atom_energy:
            atom_energy = torch.empty(n, dtype=torch.float64, device=dev)
        b = _box9(box)
        _check(lib().dp_compute(self.handle, _ptr(coords), _ptr(types), b.ctypes.data, n, _ptr(nlist),
                                MODES[mode] if isinstance(mode, str) else int(mode), _ptr(energy),
                                _ptr(atom_energy), _ptr(forces), _ptr(virial), _stream()))
        return dict(E=energy, Ei=atom_energy, F=forces, W=virial)

    def compute_batch(self, coords, types, boxes, frame_off, nlist, mode="fp64", energies=None, forces=None,
                      virials=None):
        import torch
        n = int(types.shape[0])
        dev = coords.device
        bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 9))
        off = np.ascontiguousarray(frame_off, dtype=np.int64)
        B = bx.shape[0]
        if energies is None:
            energies = torch.empty(B, dtype=torch.float64, device=dev)
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=dev)
        if virials is None:
            virials = torch.empty((B, 9), dtype=torch.float64, device=dev)
        _check(lib().dp_compute_batch(self.handle, _ptr(coords), _ptr(types), bx.ctypes.data, off.ctypes.data, B,
                                      _ptr(nlist), MODES[mode] if isinstance(mode, str) else int(mode),
                                      _ptr(energies), _ptr(forces), _ptr(virials), _stream()))
        return dict(E=energies, F=forces, W=virials)

    def backward_params(self, dL_dE, grad=None):
        import torch
        if grad is None:
            grad = torch.empty(self.model.n_params, dtype=torch.float64, device=dL_dE.device)
        _check(lib().dp_backward_params(self.handle, _ptr(dL_dE), _ptr(grad), _stream()))
        return grad

    # ------------------------------------------------------------ md
    def kick_drift(self, coords, vel, forces, types, box, dt, images=None, wrap=True):
        b = _box9(box) if wrap else None
        _check(lib().dp_md_kick_drift(self.handle, _ptr(coords), _ptr(vel), _ptr(forces), _ptr(types),
                                      None if b is None else b.ctypes.data, int(types.shape[0]), float(dt),
                                      int(bool(wrap)), _ptr(images), _stream()))

    def kick(self, vel, forces, types, dt, ke):
        _check(lib().dp_md_kick(self.handle, _ptr(vel), _ptr(forces), _ptr(types), int(types.shape[0]), float(dt),
                                _ptr(ke), _stream()))

    # ------------------------------------------------------------ inspection
    def status(self) -> int:
        f = ctypes.c_int32(0)
        _check(lib().dp_ctx_status(self.handle, ctypes.byref(f)))
        return int(f.value)

    def store_info(self) -> tuple:
        """(capacity in bytes, whether the last compute used the activation
        store, whether a parameter-gradient pass after a mixed-precision
        compute filled it)."""
        cap, used = ctypes.c_int64(0), ctypes.c_int32(0)
        _check(lib().dp_ctx_store_info(self.handle, ctypes.byref(cap), ctypes.byref(used)))
        return int(cap.value), used.value == 1, used.value == 2

    def profile(self, enable, stages=None) -> None:
        """Per-stage event timing: enable=False releases it; stages (names from
        STAGES) restricts it to those stages."""
        mask = 0
        if enable:
            mask = -1 if stages is None else sum(1 << STAGES.index(n) for n in stages)
        _check(lib().dp_ctx_profile(self.handle, int(mask)))

    def stage_times(self) -> dict:
        ms = np.zeros(len(STAGES), dtype=np.float64)
        cnt = np.zeros(len(STAGES), dtype=np.int64)
        _check(lib().dp_ctx_stage_times(self.handle, ms.ctypes.data, cnt.ctypes.data))
        return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(STAGES)}

    def copy_buffer(self, which: int):
        import torch
        nb = ctypes.c_int64(0)
        _check(lib().dp_ctx_copy_buffer(self.handle, int(which), None, ctypes.byref(nb), None))
        out = torch.empty(int(nb.value) // 8, dtype=torch.float64, device="cuda")
        _check(lib().dp_ctx_copy_buffer(self.handle, int(which), _ptr(out), ctypes.byref(nb), _stream()))
        return out


def frame_offsets(sizes: Sequence[int]) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))]).astype(np.int64)


def _autograd():
    import torch

    class DPEnergy(torch.autograd.Function):
        """Frame energies E_f of a batch as a differentiable function of the
        flat parameter vector and the coordinates.

        forward(params, coords, types, boxes, frame_off, ctx, nlist, mode) -> E [B]
        backward(gE) -> (dL/dparams via dp_backward_params, dL/dcoords = -F gE_f)

        mode is "fp64", "bf16" or "fp16" (the mixed forms give the mixed
        model's energies, forces and parameter gradients).

        The model of ``ctx`` is loaded from ``params`` (a device float64
        tensor) on every call, on the device and asynchronously, so in-place
        updates and new tensors are always seen.  Backward must run before
        another compute on ``ctx``.
        """

        @staticmethod
        def forward(fctx, params, coords, types, boxes, frame_off, dctx, nlist, mode="fp64"):
            dctx.model.load_params(params.detach())
            r = dctx.compute_batch(coords.detach(), types, boxes, frame_off, nlist, mode=mode)
            fctx.dctx = dctx
            fctx.frame_off = np.asarray(frame_off, dtype=np.int64)
            fctx.save_for_backward(r["F"])
            return r["E"]

        @staticmethod
        def backward(fctx, gE):
            (F,) = fctx.saved_tensors
            gE = gE.contiguous().to(torch.float64)
            gparams = fctx.dctx.backward_params(gE)
            sizes = torch.as_tensor(np.diff(fctx.frame_off), device=gE.device)
            gatom = torch.repeat_interleave(gE, sizes)
            gcoords = -F * gatom[:, None]
            return gparams, gcoords, None, None, None, None, None, None

    return DPEnergy


_DPEnergy = None


def dp_energy(params, coords, types, boxes, frame_off, ctx: Context, nlist, mode: str = "fp64"):
    """Differentiable batch energies (see DPEnergy)."""
    global _DPEnergy
    if _DPEnergy is None:
        _DPEnergy = _autograd()
    return _DPEnergy.apply(params, coords, types, boxes, frame_off, ctx, nlist, mode)
