#!/usr/bin/env python3
"""DP se_a energy+force MD-step throughput on one MI355X.

A step is one pass of the whole hot path over the frame: velocity-Verlet
kick + drift (+ wrap), neighbour-list build, energy/forces/virial
(environment matrix, embedding nets, descriptor, fitting net, backward,
force/virial scatter), second kick.  Inputs are synthetic (seeded generators,
random-weight model of the paper's water architecture) and resident in HBM
before timing starts.

Prints ONE JSON line.  `value` is the FP64 path's atom-steps/s; the mixed
precision forms (BF16 / FP16 matrix-core GEMMs) are reported beside it with
their speedup and their error against the FP64 oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TF = 78.6
PEAK_BF16_TF = 2500.0
PEAK_FP32_TF = 157.3
PEAK_HBM_GBS = 8000.0
# element kinds of (embedding, first fitting layer, fitting layers 2-3) per
# mode and the dense matrix peak of each kind (TFLOP/s)
MODE_KINDS = {"fp64": (0, 0, 0), "bf16": (1, 1, 1), "fp16": (2, 2, 2), "mix_fp32": (3, 3, 3), "mix_fp16": (3, 2, 3),
              "fp64_tab": (0, 0, 0)}
KIND_PEAK = {0: PEAK_FP64_TF, 1: PEAK_BF16_TF, 2: PEAK_BF16_TF, 3: PEAK_FP32_TF}
TABLE2_NAMES = {"fp64": "Double", "mix_fp32": "MIX-fp32", "mix_fp16": "MIX-fp16", "bf16": "BF16 GEMMs",
                "fp16": "FP16 GEMMs", "fp64_tab": "Double, tabulated embedding (DP-compress)"}


def stage_peaks(desc, mode):
    """Matrix peak (TFLOP/s) each matrix stage is bound by in a mode; the
    fitting stages mix the first layer's kind (nd x fw products) with the
    pair's (two fw x fw products), weighted by their flops."""
    ke, k1, k23 = MODE_KINDS[mode]
    f1 = desc.ndesc * desc.fit[0]
    f23 = 2 * desc.fit[0] * desc.fit[0]
    fit_peak = (f1 + f23) / (f1 / KIND_PEAK[k1] + f23 / KIND_PEAK[k23])
    return {"embed_fwd": KIND_PEAK[ke], "embed_bwd": KIND_PEAK[ke], "fit_fwd": fit_peak, "fit_bwd": fit_peak,
            "descriptor": PEAK_FP64_TF if ke == 0 else PEAK_FP32_TF,
            "desc_bwd": PEAK_FP64_TF if ke == 0 else PEAK_FP32_TF}


def algorithmic_flops(desc, real_rows, natoms, stored=False, tab=False):
    """Flops per launch of the matrix stages (real neighbour rows only).  The
    embedding backward recomputes layers 1-2 (and layer 3 unless its output
    was stored by the forward), then back-propagates through all three.
    Tabulated embedding (DP-compress): per row and feature a quintic (10) and
    the contraction (8) forward; value and slope quintics (20), dE/dG (8),
    the direct term (8) and the slope product (2) backward."""
    w1, fw, nd, m1 = desc.emb[0], desc.fit[0], desc.ndesc, desc.m1
    l12 = 2 * (w1 + desc.emb[0] * desc.emb[1])
    l3 = 2 * desc.emb[1] * desc.emb[2]
    gemm_row = l12 + l3
    contr = 2 * m1 * 4
    fit_fwd = 2 * (nd * fw + 2 * fw * fw) + 2 * fw
    fit_bwd = 2 * (2 * fw * fw + fw * nd)
    return {
        "embed_fwd": real_rows * (m1 * 18 if tab else gemm_row + contr),
        "embed_bwd": real_rows * (m1 * 38 if tab else (l12 if stored else gemm_row) + gemm_row + 2 * contr),
        "fit_fwd": natoms * fit_fwd,
        "fit_bwd": natoms * fit_bwd,
        "descriptor": natoms * 2 * m1 * desc.m2 * 4,
        "desc_bwd": natoms * 4 * m1 * desc.m2 * 4,
    }


# Vector-ALU model of the FP32 elementwise work of the embedding nets (the
# bound of the mixed forms' embedding kernels, whose products run on the
# matrix cores): 1024 SIMDs x 32 lanes x 2.4 GHz = 78.6 T lane-operations/s
# for FP32 add/mul/fma (a wave64 instruction issues in 2 cycles: the FP32
# vector peak of 157.3 TFLOP/s counts an fma as 2 flops; a throughput loop
# of independent fmas measures 2.75 cycles per instruction with its loop
# overhead), a quarter of that for the transcendental exp2 and reciprocal
# (measured 8.4 cycles per wave64 instruction).  A tanh costs 2 transcendentals + 3 operations (argument scale,
# 1 + e, the final fma); every unit of a width-keeping or width-doubling
# layer adds its skip (1), layer 1 its input fma (1); the backward adds per
# unit the derivative (1 - t^2) dh (2) and the skip's accumulation or, in
# layer 1, the dot product with W1 (1), and recomputes the forward.
ALU_OPS_PER_S = 1024 * 32 * 2.4e9
ALU_TRANS_PER_S = ALU_OPS_PER_S / 4


def embed_alu_seconds(desc, real_rows, stage):
    units = sum(desc.emb)
    fwd_t = units * 2 / ALU_TRANS_PER_S
    fwd_o = (units * 3 + units) / ALU_OPS_PER_S
    if stage == "embed_fwd":
        return real_rows * (fwd_t + fwd_o)
    return real_rows * (fwd_t + fwd_o + units * 3 / ALU_OPS_PER_S)


def measured_traffic(stage, workload):
    """HBM bytes per launch of an embedding kernel from the committed rocprofv3
    counter summary, only while the kernel source is the one it was taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_embed.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["sources_sha256"] or rec["workload"] != workload:
        return None
    key = "k_" + stage + "_f64"
    for name, v in rec["kernels"].items():
        if key in name:
            return int((v["read_MiB"] + v["write_MiB"]) * 1024 * 1024)
    return None


def stage_bytes(desc, real_rows, natoms, skin):
    """Algorithmic HBM bytes per launch of the memory-bound stages (FP64
    step; real neighbour rows only for gathers, the padded [n, nm] arrays as
    written).  nlist: the Verlet format reads each candidate (4 B index, 24 B
    position, 4 B type) for about real_rows * ((r_c + skin) / r_c)^3
    candidates and writes the list and its bookkeeping (3 x 4 B per slot),
    then the reverse map reads 3 and writes 1 word per slot.  env: list in,
    24 B per real row gathered, R~ out (32 B per slot).  force: list and
    reverse index in, two net_deriv rows (64 B), one position (24 B) and the
    8 B reverse check per real row, forces and per-atom virial rows out."""
    nm = desc.nm
    cand = real_rows * ((desc.rcut + skin) / desc.rcut) ** 3
    slots = natoms * nm
    return {
        "nlist": int(cand * 32 + slots * 4 * 3 + slots * 4 * 4),
        "env": int(slots * (4 + 32) + real_rows * 24 + natoms * (24 + 16 + 24)),
        "force": int(slots * 8 + real_rows * (64 + 24 + 8) + natoms * (24 + 72 + 24)),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="water12k",
                    choices=["water192", "water12k", "copper32k", "water98k", "waterbatch64"])
    ap.add_argument("--modes", default="fp64,bf16,fp16,mix_fp32,mix_fp16,fp64_tab")
    ap.add_argument("--nve-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--nlist", default="verlet", choices=["verlet", "rebuild"],
                    help="verlet: Verlet list formatted every step and rebuilt on the device when an atom has "
                         "moved beyond skin/2 or --rebuild-every steps have passed; rebuild: cell-list build "
                         "from scratch every step")
    ap.add_argument("--skin", type=float, default=2.0)
    ap.add_argument("--rebuild-every", type=int, default=50)
    ap.add_argument("--workspace-gib", type=float, default=64.0,
                    help="embedding-activation store budget; 0 recomputes the activations in the backward pass")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (known bytes) to scale HBM counters")
    ap.add_argument("--no-paper-size", action="store_true",
                    help="skip the 0.56 M-atom water and 0.54 M-atom copper steps")
    ap.add_argument("--no-latency", action="store_true", help="skip the 192-atom eager vs graph-replay step")
    ap.add_argument("--no-nve98k", action="store_true",
                    help="skip the 98,304-atom water NVE runs (FP64, BF16, FP16)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (one box of atoms per GPU; the "
              "spatial decomposition over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_22867_amd import dpse, inputs as I

    dev = torch.device("cuda:0")
    if args.workload == "waterbatch64":
        bench_batch(args, torch, dpse, I, dev)
        return
    modes = args.modes.split(",")
    fr, desc, params, dt = I.workload(args.workload)
    wl_index = {"water192": 0, "water12k": 1, "copper32k": 2, "water98k": 3}[args.workload]
    n = fr.n
    model = dpse.Model(desc, params)
    grid = I.COMPRESS_GRID_COPPER if desc.ntypes == 1 else I.COMPRESS_GRID_WATER
    if "fp64_tab" in modes:
        model.compress(*grid)
    ctx = dpse.Context(model, n, budget_bytes=int(args.workspace_gib * 2 ** 30))
    activations = {}
    x0 = torch.tensor(fr.coords, device=dev)
    v0 = torch.tensor(I.maxwell_boltzmann(fr.types, desc.masses, 300.0, seed=200 + wl_index), device=dev)
    t = torch.tensor(fr.types, device=dev)
    box = fr.box
    nm = desc.nm
    nl = torch.empty((n, nm), dtype=torch.int32, device=dev)
    ov = torch.empty(1, dtype=torch.int32, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    W = torch.empty(9, dtype=torch.float64, device=dev)
    ke = torch.empty(1, dtype=torch.float64, device=dev)
    f = torch.empty((n, 3), dtype=torch.float64, device=dev)
    nreb = torch.zeros(1, dtype=torch.int32, device=dev)
    verlet = args.nlist == "verlet"

    def step(x, v, mode, h=dt):
        """One MD step; every launch is asynchronous (no host wait)."""
        ctx.kick_drift(x, v, f, t, box, h, wrap=not verlet)
        if verlet:
            ctx.skin_update(x, t, every=args.rebuild_every, out=nl, overflow=ov, rebuilds=nreb)
        else:
            ctx.build_nlist(x, t, box, out=nl, overflow=ov)
        ctx.compute(x, t, box, nl, mode=mode, energy=E, forces=f, virial=W)
        ctx.kick(v, f, t, h, ke)

    def init_state(mode):
        x = x0.clone()
        v = v0.clone()
        if verlet:
            ctx.skin_build(x, t, box, args.skin)
            ctx.skin_format(x, t, out=nl, overflow=ov)
        else:
            ctx.build_nlist(x, t, box, out=nl, overflow=ov)
        ctx.compute(x, t, box, nl, mode=mode, energy=E, forces=f, virial=W)
        activations[mode] = "stored" if ctx.store_info()[1] else "recomputed"
        return x, v

    if args.calib_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # single-frame results on the initial configuration (accuracy)
    first = {}
    for mode in modes:
        x, v = init_state(mode)
        torch.cuda.synchronize()
        first[mode] = dict(E=float(E.item()), F=f.cpu().numpy().copy(), W=W.cpu().numpy().copy())
    real_rows = int((nl >= 0).sum().item())
    fl = ctx.status()
    if fl:
        raise RuntimeError(f"device status flags {fl} on the initial frame")

    # per-stage event timing (separate pass over all stages)
    stages = {}
    for mode in modes:
        x, v = init_state(mode)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(args.profile_steps):
            step(x, v, mode)
        torch.cuda.synchronize()
        st = ctx.stage_times()
        ctx.profile(False)
        stages[mode] = {k: (ms / c if c else 0.0, c) for k, (ms, c) in st.items()}
    st64 = stages.get("fp64", {})
    dom = max(st64, key=lambda k: st64[k][0]) if st64 else None

    # timed region; in FP64 the dominant stage is also timed with HIP events
    # recorded on its own stream inside the same region (roofline below)
    results = {}
    dom_live = None
    timed_flags = 0
    for mode in modes:
        x, v = init_state(mode)
        for _ in range(args.warmup):
            step(x, v, mode)
        live = mode == "fp64" and dom is not None
        if live:
            ctx.profile(True, stages=[dom])
        ctx.status()                     # clears the status word before the timed steps
        torch.cuda.synchronize()
        r0 = int(nreb.item())
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(x, v, mode)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rebuilds = int(nreb.item()) - r0
        if live:
            ms_dom, cnt = ctx.stage_times()[dom]
            ctx.profile(False)
            dom_live = (ms_dom / cnt, cnt) if cnt else None
        fl = ctx.status()
        timed_flags |= fl
        ms = el / args.steps * 1e3
        results[mode] = dict(ms_per_step=ms, atom_steps_per_s=n * args.steps / el,
                             ns_per_day=(args.steps / el) * dt * 0.0864, verlet_rebuilds=rebuilds,
                             status_flags=fl)
        print(f"# {mode}: {ms:.3f} ms/step, {n * args.steps / el:.4g} atom-steps/s, {rebuilds} rebuilds, "
              f"flags {fl}", file=sys.stderr, flush=True)
    if timed_flags & ~(dpse.FLAG_SEL_OVERFLOW | dpse.FLAG_SKIN_EXCEEDED | dpse.FLAG_TABLE_RANGE):
        raise RuntimeError(f"device status flags {timed_flags}")

    # NVE energy drift (velocity Verlet, metal units) over every step: the
    # same step as the timed one (rebuilds decided on the device, so every
    # list is exact while no section overflows); the energies and the
    # truncation counts are kept on the device and read once at the end.
    def nve(mode, nsteps, h):
        x, v = init_state(mode)
        hist = torch.empty((nsteps + 1, 3), dtype=torch.float64, device=dev)
        ctx.kick(v, torch.zeros_like(f), t, 0.0, ke)
        hist[0, 0] = E[0]
        hist[0, 1] = ke[0]
        hist[0, 2] = 0.0
        ctx.status()
        torch.cuda.synchronize()
        r0 = int(nreb.item())
        for k in range(nsteps):
            step(x, v, mode, h)
            hist[k + 1, 0] = E[0]
            hist[k + 1, 1] = ke[0]
            hist[k + 1, 2] = ov[0]
        hh = hist.cpu().numpy()
        bad = np.nonzero(hh[:, 2] > 0)[0]
        etot = hh[:, 0] + hh[:, 1]
        tps = np.arange(len(etot)) * h * 1e-3
        dev_meV = (etot - etot[0]) / n * 1e3
        T = hh[:, 1] * 2.0 / (3 * n * 8.617333262e-5)
        return dict(steps=nsteps, dt_fs=h,
                    steps_before_sel_overflow=int(bad[0]) - 1 if len(bad) else nsteps,
                    steps_with_sel_overflow=int(len(bad)),
                    verlet_rebuilds=int(nreb.item()) - r0,
                    max_dev_meV_per_atom=float(np.abs(dev_meV).max()),
                    final_dev_meV_per_atom=float(dev_meV[-1]),
                    slope_meV_per_atom_per_ps=float(np.polyfit(tps, dev_meV, 1)[0]),
                    T_start_K=round(float(T[0]), 2), T_end_K=round(float(T[-1]), 2),
                    flags=ctx.status())

    drift = {}
    if args.nve_steps > 0:
        for mode in modes:
            drift[mode] = nve(mode, args.nve_steps, dt)
            print(f"# nve {mode}: {drift[mode]}", file=sys.stderr, flush=True)
        if "fp64" in modes:
            # same simulated time at half the step: velocity Verlet's energy
            # error is second order in dt
            drift["fp64_half_dt"] = nve("fp64", 2 * args.nve_steps, 0.5 * dt)

    # roofline of the dominant FP64 kernel, timed inside the timed region
    flops = algorithmic_flops(desc, real_rows, n, stored=activations.get("fp64") == "stored")
    roof = None
    if dom in flops and dom_live is not None:
        avg_s = dom_live[0] * 1e-3
        ach = flops[dom] / avg_s / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP64_TF,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TF, 4), "traffic": measured_traffic(dom, args.workload),
                "avg_launch_ms": round(dom_live[0], 4), "launches_timed": dom_live[1],
                "flops_per_launch": flops[dom]}
    # the mixed forms' dominant matrix stage against the BF16/FP16 peak, the
    # memory-bound stages against HBM, and the whole step against the sum of
    # its stages' bounds (T_roof = sum_k max(F_k / P_k, B_k / BW))
    hbm = stage_bytes(desc, real_rows, n, args.skin)
    extra = {}
    for mode in modes:
        st = stages[mode]
        fl_m = algorithmic_flops(desc, real_rows, n, stored=activations.get(mode) == "stored", tab=mode == "fp64_tab")
        peaks = stage_peaks(desc, mode)
        mat = {k: fl_m[k] / (st[k][0] * 1e-3) / 1e12 for k in fl_m if st.get(k, (0, 0))[0] > 0}
        mem = {k: hbm[k] / (st[k][0] * 1e-3) / 1e9 for k in hbm if st.get(k, (0, 0))[0] > 0}
        # FP32 forms (all but fp64 and the table): the embedding stages' ALU bound
        alu = ({k: embed_alu_seconds(desc, real_rows, k) for k in ("embed_fwd", "embed_bwd")}
               if MODE_KINDS[mode][0] != 0 else {})
        t_roof = sum(max(fl_m.get(k, 0) / (peaks.get(k, PEAK_FP64_TF) * 1e12), hbm.get(k, 0) / (PEAK_HBM_GBS * 1e9),
                         alu.get(k, 0.0))
                     for k in st)
        dmat = max(mat, key=lambda k: st[k][0]) if mat else None
        peak = peaks[dmat] if dmat else None
        extra[mode] = {
            "dominant_matrix_stage": dmat,
            "dominant_achieved_TFLOPs": round(mat[dmat], 2) if dmat else None,
            "dominant_frac_of_peak": round(mat[dmat] / peak, 4) if dmat else None,
            "peak_TFLOPs": round(peak, 1) if peak else None,
            "matrix_stage_TFLOPs": {k: round(vv, 2) for k, vv in mat.items()},
            "hbm_stage_GBs": {k: round(vv, 1) for k, vv in mem.items()},
            "table_read_GBs": ({k: round(real_rows * 6 * desc.m1 * 8 / (st[k][0] * 1e-3) / 1e9, 1)
                                for k in ("embed_fwd", "embed_bwd") if st.get(k, (0, 0))[0] > 0}
                               if mode == "fp64_tab" else None),
            "embed_alu": ({k: {"bound": "alu", "T_alu_ms": round(alu[k] * 1e3, 4),
                               "T_meas_ms": round(st[k][0], 4), "frac": round(alu[k] * 1e3 / st[k][0], 4)}
                           for k in alu if st.get(k, (0, 0))[0] > 0} or None),
            "step_T_roof_ms": round(t_roof * 1e3, 4),
            "step_T_meas_ms": round(results[mode]["ms_per_step"], 4),
            "step_roof_frac": round(t_roof * 1e3 / results[mode]["ms_per_step"], 4),
        }

    # oracle on the host cores: a bounded sample of the same workload
    cpu = None
    o = None
    if not args.no_cpu_baseline:
        import oracle
        nthr = oracle.num_threads()

        def timed_frame(rows=None):
            tc = time.perf_counter()
            onl, _ = oracle.nlist(fr.coords, fr.types, fr.box, desc, rows=rows)
            r = oracle.compute(fr.coords, fr.types, fr.box, desc, params, nl=onl, rows=rows)
            return time.perf_counter() - tc, r

        _, o = timed_frame()                                  # warm-up (also the accuracy reference)
        times = [timed_frame()[0] for _ in range(3)]
        tf = float(np.median(times))
        rows1 = np.arange(0, n, max(1, n // 1024))[:1024]
        oracle.set_threads(1)
        timed_frame(rows1)
        t1 = float(np.median([timed_frame(rows1)[0] for _ in range(3)]))
        oracle.set_threads(nthr)
        cpu = {"value": round(n / tf, 2), "unit": "atom-steps/s", "cores": nthr, "kind": "oracle",
               "sample": f"one {args.workload} frame ({n} atoms: neighbour list + E, F, W), median of 3 runs "
                         f"after 1 warm-up, {tf:.3f} s each",
               "one_core": {"value": round(len(rows1) / t1, 2), "unit": "atom-steps/s", "cores": 1,
                            "sample": f"{len(rows1)} evenly spaced centre atoms of the same frame, median of 3 "
                                      f"after 1 warm-up, {t1:.3f} s each"}}
    acc = {}
    if o is not None:
        frms = float(np.sqrt((o["F"] ** 2).mean()))
        for mode, r in first.items():
            ferr = float(np.sqrt(((r["F"] - o["F"]) ** 2).mean()))
            acc[mode] = dict(E_meV_per_atom=abs(r["E"] - o["E"]) / n * 1e3,
                             F_rms_meV_per_A=ferr * 1e3,
                             F_rms_rel=ferr / frms,
                             F_max_meV_per_A=float(np.abs(r["F"] - o["F"]).max() * 1e3),
                             W_max_meV_per_atom=float(np.abs(r["W"].reshape(3, 3) - o["W"]).max() * 1e3 / n))
        # the structure of the paper's accuracy table (energy eV/atom, force
        # eV/A per precision), here as the error against the FP64 oracle on
        # the same synthetic frame (the paper's is against AIMD labels)
        acc["table2"] = [{"precision": TABLE2_NAMES.get(m, m), "mode": m,
                          "energy_eV_per_atom": acc[m]["E_meV_per_atom"] * 1e-3,
                          "force_rms_eV_per_A": acc[m]["F_rms_meV_per_A"] * 1e-3,
                          "force_rms_rel": acc[m]["F_rms_rel"]} for m in first]
        acc["force_rms_meV_per_A"] = frms * 1e3
        acc["energy_spread_meV_per_atom"] = float(np.std(o["Ei"]) * 1e3)
        acc["virial_max_meV_per_atom"] = float(np.abs(o["W"]).max() * 1e3 / n)

    base = results.get("fp64") or next(iter(results.values()))
    line = {
        "metric": "DP energy+force atom-steps/s & ns/day, 12k-atom water, FP64 vs mixed",
        "value": round(base["atom_steps_per_s"], 1),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(base["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "natoms": n, "dt_fs": dt,
                   "step": ("kick+drift, Verlet list (formatted every step; rebuilt on the device when an atom "
                            f"moved beyond skin/2 or every {args.rebuild_every} steps, skin {args.skin} A), "
                            "E/F/W, kick" if verlet else
                            "kick+drift, cell-list neighbour build, E/F/W, kick"),
                   "real_neighbour_rows": real_rows,
                   "embedding_activations": activations},
        "ns_per_day": round(base["ns_per_day"], 3),
        "modes": {m: {k: round(vv, 4) for k, vv in r.items()} for m, r in results.items()},
        "mixed_speedup": {m: round(results["fp64"]["ms_per_step"] / r["ms_per_step"], 3)
                          for m, r in results.items() if m != "fp64" and "fp64" in results},
        "accuracy_vs_oracle": acc,
        "nve_drift": drift,
        "stage_ms": {m: {k: round(vv[0], 4) for k, vv in s.items() if vv[1]} for m, s in stages.items()},
        "status_flags": timed_flags,
        "roofline": roof,
        "roofline_modes": extra,
        "cpu_baseline": cpu,
    }
    del ctx, model
    torch.cuda.synchronize()
    if not args.no_latency:
        line["latency_small"] = bench_latency(args, torch, dpse, I, dev)
    if args.nve_steps > 0 and not args.no_nve98k and args.workload == "water12k":
        line["nve_water98k"] = bench_nve_water98k(args, torch, dpse, I, dev)
    if not args.no_paper_size:
        line["paper_size"] = bench_paper_size(args, torch, dpse, I, dev)
    print(json.dumps(line), flush=True)


def bench_nve_water98k(args, torch, dpse, I, dev):
    """The 98,304-atom water system: 1000 velocity-Verlet steps at 0.5 fs in
    FP64, BF16 and FP16 (Verlet list rebuilt on the device; energies kept on
    the device and read at the end), and the mixed forms' difference from
    the FP64 GPU form on the identical initial frame."""
    fr, desc, params, dt = I.workload("water98k")
    n = fr.n
    model = dpse.Model(desc, params)
    ctx = dpse.Context(model, n, budget_bytes=int(args.workspace_gib * 2 ** 30))
    x0 = torch.tensor(fr.coords, device=dev)
    v0 = torch.tensor(I.maxwell_boltzmann(fr.types, desc.masses, 300.0, seed=203), device=dev)
    t = torch.tensor(fr.types, device=dev)
    nl = torch.empty((n, desc.nm), dtype=torch.int32, device=dev)
    ov = torch.empty(1, dtype=torch.int32, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    W = torch.empty(9, dtype=torch.float64, device=dev)
    ke = torch.empty(1, dtype=torch.float64, device=dev)
    f = torch.empty((n, 3), dtype=torch.float64, device=dev)
    nreb = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {"natoms": n, "dt_fs": dt}
    first = {}
    for mode in ("fp64", "bf16", "fp16"):
        x = x0.clone()
        v = v0.clone()
        ctx.skin_build(x, t, fr.box, args.skin)
        ctx.skin_format(x, t, out=nl, overflow=ov)
        ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
        torch.cuda.synchronize()
        first[mode] = (float(E.item()), f.cpu().numpy().copy())
        hist = torch.empty((args.nve_steps + 1, 3), dtype=torch.float64, device=dev)
        ctx.kick(v, torch.zeros_like(f), t, 0.0, ke)
        hist[0, 0] = E[0]
        hist[0, 1] = ke[0]
        hist[0, 2] = 0.0
        ctx.status()
        torch.cuda.synchronize()
        r0 = int(nreb.item())
        t0 = time.perf_counter()
        for k in range(args.nve_steps):
            ctx.kick_drift(x, v, f, t, fr.box, dt, wrap=False)
            ctx.skin_update(x, t, every=args.rebuild_every, out=nl, overflow=ov, rebuilds=nreb)
            ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
            ctx.kick(v, f, t, dt, ke)
            hist[k + 1, 0] = E[0]
            hist[k + 1, 1] = ke[0]
            hist[k + 1, 2] = ov[0]
        hh = hist.cpu().numpy()
        el = time.perf_counter() - t0
        bad = np.nonzero(hh[:, 2] > 0)[0]
        etot = hh[:, 0] + hh[:, 1]
        tps = np.arange(len(etot)) * dt * 1e-3
        dev_meV = (etot - etot[0]) / n * 1e3
        T = hh[:, 1] * 2.0 / (3 * n * 8.617333262e-5)
        out[mode] = dict(steps=args.nve_steps, ms_per_step=round(el / max(1, args.nve_steps) * 1e3, 3),
                         steps_before_sel_overflow=int(bad[0]) - 1 if len(bad) else args.nve_steps,
                         steps_with_sel_overflow=int(len(bad)), verlet_rebuilds=int(nreb.item()) - r0,
                         max_dev_meV_per_atom=float(np.abs(dev_meV).max()),
                         final_dev_meV_per_atom=float(dev_meV[-1]),
                         slope_meV_per_atom_per_ps=float(np.polyfit(tps, dev_meV, 1)[0]),
                         T_start_K=round(float(T[0]), 2), T_end_K=round(float(T[-1]), 2), flags=ctx.status())
        print(f"# water98k nve {mode}: {out[mode]}", file=sys.stderr, flush=True)
    e64, f64 = first["fp64"]
    out["initial_frame_vs_fp64_gpu"] = {
        m: {"E_meV_per_atom": abs(first[m][0] - e64) / n * 1e3,
            "F_rms_meV_per_A": float(np.sqrt(((first[m][1] - f64) ** 2).mean())) * 1e3,
            "F_rms_rel": float(np.sqrt(((first[m][1] - f64) ** 2).mean() / (f64 ** 2).mean()))}
        for m in ("bf16", "fp16")}
    del ctx, model
    torch.cuda.synchronize()
    return out


def bench_paper_size(args, torch, dpse, I, dev):
    """The Evaluation section's strong-scaling systems (0.56 M-atom water,
    0.54 M-atom copper) on one GPU: MD steps as in the main bench (Verlet
    list rebuilt on the device), FP64 and BF16, with the device memory the
    model and context take and the activation-store choice."""
    out = {}
    for wl in ("water557k", "copper535k"):
        fr, desc, params, dt = I.workload(wl)
        n = fr.n
        free0 = torch.cuda.mem_get_info()[0]
        model = dpse.Model(desc, params)
        # the activation store is allocated only when it holds every atom
        tiles = sum((s_ + 15) // 16 for s_ in desc.sel)
        store = n * tiles * desc.m1 * 16 * 8
        budget = store if store <= args.workspace_gib * 2 ** 30 else 0
        ctx = dpse.Context(model, n, budget_bytes=int(budget))
        x0 = torch.tensor(fr.coords, device=dev)
        v0 = torch.tensor(I.maxwell_boltzmann(fr.types, desc.masses, 300.0, seed=205), device=dev)
        t = torch.tensor(fr.types, device=dev)
        nl = torch.empty((n, desc.nm), dtype=torch.int32, device=dev)
        ov = torch.empty(1, dtype=torch.int32, device=dev)
        E = torch.empty(1, dtype=torch.float64, device=dev)
        W = torch.empty(9, dtype=torch.float64, device=dev)
        ke = torch.empty(1, dtype=torch.float64, device=dev)
        f = torch.empty((n, 3), dtype=torch.float64, device=dev)
        nreb = torch.zeros(1, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        used = (free0 - torch.cuda.mem_get_info()[0]) / 2 ** 30
        rec = {"natoms": n, "box_A": [round(float(v), 3) for v in np.diag(fr.box)], "dt_fs": dt,
               "device_memory_GiB": round(used, 2)}
        for mode in ("fp64", "bf16"):
            x = x0.clone()
            v = v0.clone()
            ctx.skin_build(x, t, fr.box, args.skin)
            ctx.skin_format(x, t, out=nl, overflow=ov)
            ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
            stored = ctx.store_info()[1]

            def step():
                ctx.kick_drift(x, v, f, t, fr.box, dt, wrap=False)
                ctx.skin_update(x, t, every=args.rebuild_every, out=nl, overflow=ov, rebuilds=nreb)
                ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
                ctx.kick(v, f, t, dt, ke)

            for _ in range(2):
                step()
            ctx.status()
            torch.cuda.synchronize()
            steps = 5
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            rec[mode] = {"ms_per_step": round(el / steps * 1e3, 3), "atom_steps_per_s": round(n * steps / el, 1),
                         "ns_per_day": round(steps / el * dt * 0.0864, 3), "steps": steps,
                         "embedding_activations": "stored" if stored else "recomputed",
                         "status_flags": ctx.status()}
            print(f"# {wl} {mode}: {rec[mode]}", file=sys.stderr, flush=True)
        out[wl] = rec
        del ctx, model
        torch.cuda.synchronize()
    out["paper_context"] = ("Evaluation section, 12,000 Fugaku nodes: 149 ns/day (copper, 0.54 M atoms) and "
                            "68.5 ns/day (water, 0.56 M atoms); context only, not a target")
    return out


def bench_latency(args, torch, dpse, I, dev):
    """The 192-atom water step (launch-bound: ~20 small kernels) issued
    eagerly and replayed from a HIP graph captured once (torch.cuda.CUDAGraph
    records the library's launches on the capture stream)."""
    fr, desc, params, dt = I.workload("water192")
    n = fr.n
    model = dpse.Model(desc, params)
    ctx = dpse.Context(model, n)
    out = {"workload": "water192", "natoms": n}
    for mode in ("fp64", "bf16"):
        x = torch.tensor(fr.coords, device=dev)
        v = torch.tensor(I.maxwell_boltzmann(fr.types, desc.masses, 300.0, seed=200), device=dev)
        t = torch.tensor(fr.types, device=dev)
        nl = torch.empty((n, desc.nm), dtype=torch.int32, device=dev)
        ov = torch.empty(1, dtype=torch.int32, device=dev)
        E = torch.empty(1, dtype=torch.float64, device=dev)
        W = torch.empty(9, dtype=torch.float64, device=dev)
        ke = torch.empty(1, dtype=torch.float64, device=dev)
        f = torch.empty((n, 3), dtype=torch.float64, device=dev)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ctx.skin_build(x, t, fr.box, args.skin)
            ctx.skin_format(x, t, out=nl, overflow=ov)
            ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)

            def step():
                ctx.kick_drift(x, v, f, t, fr.box, dt, wrap=False)
                ctx.skin_update(x, t, every=args.rebuild_every, out=nl, overflow=ov)
                ctx.compute(x, t, fr.box, nl, mode=mode, energy=E, forces=f, virial=W)
                ctx.kick(v, f, t, dt, ke)

            for _ in range(5):
                step()
        torch.cuda.synchronize()
        steps = 200
        with torch.cuda.stream(s):
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            s.synchronize()
            eager = (time.perf_counter() - t0) / steps
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step()
        torch.cuda.synchronize()
        for _ in range(5):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        graph = (time.perf_counter() - t0) / steps
        out[mode] = {"eager_ms_per_step": round(eager * 1e3, 4), "graph_ms_per_step": round(graph * 1e3, 4),
                     "graph_atom_steps_per_s": round(n / graph, 1), "graph_ns_per_day": round(dt * 0.0864 / graph, 2),
                     "status_flags": ctx.status()}
        print(f"# latency {mode}: {out[mode]}", file=sys.stderr, flush=True)
        del g
    return out


def bench_batch(args, torch, dpse, I, dev):
    """Training step on a batch of 64 water frames of uneven size: energies,
    forces and the parameter gradient of L = (1/B) sum_f (E_f - Ehat_f)^2,
    per mode.  The neighbour lists are built once (static frames)."""
    (frames, targets), desc, params, _ = I.workload("waterbatch64")
    sizes = [f.n for f in frames]
    off = dpse.frame_offsets(sizes)
    n = int(off[-1])
    B = len(frames)
    x = torch.tensor(np.concatenate([f.coords for f in frames]), device=dev)
    t = torch.tensor(np.concatenate([f.types for f in frames]), device=dev)
    boxes = np.stack([f.box for f in frames])
    tgt = torch.tensor(targets, device=dev)
    model = dpse.Model(desc, params)
    ctx = dpse.Context(model, n, max_frames=B, budget_bytes=int(args.workspace_gib * 2 ** 30))
    nl, ov = ctx.build_nlist_batch(x, t, boxes, off)
    grad = torch.empty(model.n_params, dtype=torch.float64, device=dev)
    p0 = torch.tensor(params, device=dev)
    pdev = p0.clone()
    lr = 1e-10   # small enough to keep the random model finite over the run; the update's cost is what is timed

    def step(mode, gE=None, update=True):
        """One training step: the model is loaded from the device parameter
        vector (no host round trip), E/F/W of every frame, the parameter
        gradient of the loss, and a plain gradient-descent update."""
        model.load_params(pdev)
        r = ctx.compute_batch(x, t, boxes, off, nl, mode=mode)
        g = gE if gE is not None else 2.0 * (r["E"] - tgt) / B
        ctx.backward_params(g, grad)
        if update:
            pdev.add_(grad, alpha=-lr)
        return r

    results, grads, ener = {}, {}, {}
    gE_ref = None
    # the tabulated embedding has no parameter gradient: not a training mode
    for mode in [m for m in args.modes.split(",") if m != "fp64_tab"]:
        for _ in range(args.warmup):
            step(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(mode)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        results[mode] = dict(ms_per_step=el / args.steps * 1e3, atom_steps_per_s=n * args.steps / el,
                             frames_per_s=B * args.steps / el, status_flags=ctx.status())
        print(f"# {mode}: {el / args.steps * 1e3:.3f} ms/step, {n * args.steps / el:.4g} atom-steps/s",
              file=sys.stderr, flush=True)
        pdev.copy_(p0)
        r = step(mode, update=False)
        if gE_ref is None:
            gE_ref = (2.0 * (r["E"] - tgt) / B).clone()
        r = step(mode, gE_ref, update=False)  # the same parameters and dL/dE for every mode
        torch.cuda.synchronize()
        grads[mode] = grad.cpu().numpy().copy()
        ener[mode] = (r["E"].cpu().numpy().copy(), r["F"].cpu().numpy().copy())
    acc = {}
    if "fp64" in grads:
        gref = grads["fp64"]
        E64, F64 = ener["fp64"]
        for mode in grads:
            if mode == "fp64":
                continue
            Em, Fm = ener[mode]
            acc[mode] = dict(grad_max_err_rel=float(np.abs(grads[mode] - gref).max() / np.abs(gref).max()),
                             E_meV_per_atom=float((np.abs(Em - E64) / np.asarray(sizes)).max() * 1e3),
                             F_rms_meV_per_A=float(np.sqrt(((Fm - F64) ** 2).mean()) * 1e3))
    line = {
        "metric": "DP training step (E, F, dL/dtheta) atom-steps/s, 64-frame water batch",
        "value": round(results[next(iter(results))]["atom_steps_per_s"], 1),
        "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(results[next(iter(results))]["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "waterbatch64", "frames": B, "natoms": n, "min_atoms": min(sizes),
                   "max_atoms": max(sizes), "step": "model loaded from the device parameter vector, batched E/F/W, parameter gradient of "
                           "the energy MSE loss, gradient-descent update"},
        "modes": {m: {k: round(v, 4) for k, v in r.items()} for m, r in results.items()},
        "mixed_vs_fp64": acc,
        "status_flags": ctx.status(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
