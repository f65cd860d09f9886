"""Benchmark: cell-updates/s of the viscous KT + RK2 step on one MI355X.

Headline workload: viscous hydro, eta/s = 0.08, 201 x 201 x 105 cells
(dx = dy = 0.16 fm, deta = 0.3), tau0 = 0.6 fm, h = 0.01 fm, 200 seeded Gaussian
hotspots, 1555-row synthetic EoS, FP64, the full 200-step run.  A step is one
full RK2 step (all three stencil passes, both root solves, the diagnostics
reduction) over the grid.  The timed region is `--steps` steps of ktmi_step from
the initial state (set before the region, inputs resident on the GPU), without
instrumentation, repeated `--reps` times; `value` is the median.  `--warmup`
steps run once, untimed, before the first repetition.

Prints one JSON line.  `roofline` comes from a separate run of the same steps
with the library's HIP events around every launch (on the library's stream):
the dominant kernel's algorithmic bytes per launch over its average duration,
against 8 TB/s; its VALU-issue ceiling uses the wave-VALU instruction count
recorded by rocprofv3 (profiles/traffic.json) while the kernel sources match.
`paths` times the other configurations the same way: the ideal Gubser grid
33x33x17 (50 steps), the benchmark grid in mixed precision, with quiet tiles
skipped, with the lambda_1 term, with bulk pressure and baryon density, the
mini-jet initial state with and without the learned root-solve guess, a batch of
64 uneven events in four forms (FP64 or mixed, with or without the network)
under HIP-graph replay with autotuned tiles, the 385x385x129 event in FP64 and
mixed precision, the freeze-out surface finder and the Cooper-Frye spectra.
`cpu_baseline` times the CPU oracle on a bounded sample of the headline workload
at one thread and at all host threads.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
VALU_WAVE_INSTS_PER_S = 256 * 2.4e9  # one wave64 VALU instruction per CU per clock (4 SIMDs x 16 lanes)

# Algorithmic HBM bytes per cell for each kernel of the FP64 viscous step: every
# field a kernel reads or writes, counted once per cell (stencil reuse assumed
# perfect).  stage1: reads e, u~(3), u~prev(3), pi~(10), T(4); writes e', u~'(3),
# pi~'(10), T'(4).  stage2_pi: reads e', u~'(3), pi~'(10), e, u~(3), u~prev(3),
# pi~(10); writes pi~(10).  stage2_T: reads e', u~'(3), pi~(10), T(4), T'(4);
# writes T(4), e(1), u~(3).
BYTES_PER_CELL = {"stage1": (21 + 18) * 8, "stage2_pi": (31 + 10) * 8, "stage2_T": (22 + 8) * 8,
                  "first_estimate": (4 + 3) * 8, "init": 0, "reduce": 0}
BYTES_PER_CELL_IDEAL = {"stage1": (8 + 5) * 8, "stage2_T": (8 + 4) * 8}
# With bulk pressure Pi and baryon density n the transported set has 12 fields:
# stage1 and stage2_pi read and write Pi and n with pi~ (+2 per pi~ block),
# stage2_T reads Pi^{n+1} (+1).
BYTES_PER_CELL_BULK = {"stage1": (23 + 20) * 8, "stage2_pi": (35 + 12) * 8,
                       "stage2_T": (23 + 8) * 8}
# Mixed precision stores pi~ (and its stage-1 value) in FP32: 4 bytes for each of
# their 10 values a cell reads or writes (stage1 10 + 10, stage2_pi 20 + 10,
# stage2_T 10).
BYTES_PER_CELL_MIXED = {"stage1": 11 * 8 + 10 * 4 + 8 * 8 + 10 * 4,
                        "stage2_pi": 11 * 8 + 20 * 4 + 10 * 4,
                        "stage2_T": 12 * 8 + 10 * 4 + 8 * 8}
# The step's minimum: the state read once and written once, and the stage-1
# prediction written once and read once (21 + 18 + 18 + 18 values, u~prev rotated
# by pointer): 600 B per cell-update in FP64.
STEP_BYTES_PER_CELL = 600


def source_sha256() -> str:
    """Hash of everything the step's stencil kernels are compiled from (their
    sources, the headers they include and the build flags): counter-derived
    figures recorded under profiles/ are used only while they match the code
    being timed."""
    import hashlib
    pkg = os.path.join(ROOT, "paper_1802_04449_amd")
    csrc = os.path.join(pkg, "csrc")
    files = [os.path.join(csrc, f) for f in ("ktmi_stencil.hip", "ktmi_kernels.hpp",
                                             "ktmi_device.hpp", "ktmi_mlp.hpp")]
    files += [os.path.join(ROOT, "include", "ktmi.h"), os.path.join(pkg, "build.py")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded(workload: str, kernel: str):
    """rocprofv3 record of `kernel` on `workload` for the current kernel sources:
    HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated against a plain
    copy) and wave-VALU instructions per launch, or None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_sha256():
        return None
    return rec.get("per_launch", {}).get(workload, {}).get(kernel)


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Timing helpers
# ---------------------------------------------------------------------------

def make_hydro(wl, stream=None, **over):
    import paper_1802_04449_amd as K
    d = dict(wl.params)
    d.update(over)
    g = K.Hydro(stream=stream, **d)
    g.set_eos(wl.eos)
    return g


def reset(g, wl):
    if wl.T4 is not None:
        g.set_initial_conserved(wl.T4)
    else:
        g.set_initial(wl.ic)


def timed_runs(g, wl, steps, reps, warmup=0, step_fn=None, reset_fn=None):
    """`reps` runs of `steps` steps from the initial state (reset before each,
    outside the timed region), uninstrumented; `warmup` steps run once before.
    Returns the wall times in seconds."""
    import torch
    step_fn = step_fn or g.step
    reset_fn = reset_fn or (lambda: reset(g, wl))
    if warmup:
        reset_fn()
        step_fn(warmup)
        torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        reset_fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step_fn(steps)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return ts


def kernel_times(g, wl, steps):
    """One instrumented run of `steps` steps from the initial state: per kernel
    total, launches and average duration (HIP events on the library's stream)."""
    import torch

    import paper_1802_04449_amd as K
    reset(g, wl)
    K.ktmi_set_timing(g.h, True)
    torch.cuda.synchronize()
    g.step(steps)
    torch.cuda.synchronize()
    out = {}
    for k, n in enumerate(K.ktmi_kernel_names()):
        tot, cnt = K.ktmi_timing(g.h, k)
        if cnt:
            out[n] = dict(total_ms=tot, launches=cnt, avg_ms=tot / cnt)
    K.ktmi_set_timing(g.h, False)
    return out


def rate(ncell, steps, ts):
    med = statistics.median(ts)
    return {"value": ncell * steps / med, "unit": "cell-updates/s", "steps": steps,
            "ms_per_step": med / steps * 1e3, "reps_s": [round(t, 5) for t in ts]}


def roofline_of(wl, per_kernel, bpc):
    """HBM roofline of the dominant kernel, the whole step's algorithmic rate, and
    the VALU-issue ceiling (wave-VALU instructions / (256 CUs x clock)) where the
    instruction count is on record for the current sources."""
    ncell = wl.ncell
    dom = max((n for n in per_kernel if n in bpc and bpc[n]),
              key=lambda n: per_kernel[n]["total_ms"])
    avg = per_kernel[dom]["avg_ms"]
    bytes_launch = bpc[dom] * ncell
    achieved = bytes_launch / (avg * 1e-3) / 1e9
    rec = recorded(wl.name, dom)
    out = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": None if rec is None else rec["fetch_bytes"] + rec["write_bytes"],
           "algorithmic_bytes": bytes_launch, "bytes_per_cell": bpc[dom], "avg_launch_ms": avg}
    if rec is not None and rec.get("valu_insts"):
        t_issue = rec["valu_insts"] / VALU_WAVE_INSTS_PER_S
        out["valu_issue"] = {"wave_insts": rec["valu_insts"], "ceiling_ms": t_issue * 1e3,
                             "frac": t_issue / (avg * 1e-3)}
    steps = max(v["launches"] for n, v in per_kernel.items() if n in bpc)
    step_ms = sum(v["total_ms"] for v in per_kernel.values()) / steps
    out["step"] = {"ms": step_ms,
                   "frac_600B": STEP_BYTES_PER_CELL * ncell / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "frac_kernels": sum(bpc.get(n, 0) * ncell * v["launches"]
                                       for n, v in per_kernel.items()) / steps /
                                   (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def kernels_summary(per_kernel, wl, bpc):
    out = {}
    for n, v in per_kernel.items():
        r = {"avg_ms": round(v["avg_ms"], 4), "launches": v["launches"]}
        if bpc.get(n):
            gbs = bpc[n] * wl.ncell / (v["avg_ms"] * 1e-3) / 1e9
            r["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        out[n] = r
    return out


# ---------------------------------------------------------------------------
# Paths
# ---------------------------------------------------------------------------

def single_path(wl, steps, reps, warmup=2, bpc=None, quiet=False, graph=False, stream=None,
                **over):
    """`wl` stepped alone: median of `reps` uninstrumented runs of `steps` steps
    from the initial state; per-kernel times from one instrumented run when bpc
    is given."""
    import torch
    st = stream if stream is not None else (torch.cuda.Stream() if graph else None)
    g = make_hydro(wl, stream=st, **over)
    if quiet:
        g.set_quiet_skip(True)
    if graph:
        g.set_graph(True)
    ts = timed_runs(g, wl, steps, reps, warmup)
    out = rate(wl.ncell, steps, ts)
    d = g.diag()
    out["newton_mean"] = d["newton_mean"]
    if quiet:
        import paper_1802_04449_amd as K
        out["quiet_tiles"], out["tiles"] = K.ktmi_quiet_tiles(g.h)
    if bpc:
        pk = kernel_times(g, wl, steps)
        out["kernels"] = kernels_summary(pk, wl, bpc)
    del g
    torch.cuda.synchronize()
    return out


def harvest_samples(wls, at_steps, cap=None, seed=1):
    """(E, M, e) of every non-vacuum cell of FP64 runs of `wls` at the given steps
    (ktmi_harvest), shuffled; at most `cap` samples."""
    from paper_1802_04449_amd import mlp
    states = []
    for wl in wls:
        g = make_hydro(wl)
        reset(g, wl)
        done = 0
        for t in at_steps:
            g.step(t - done)
            done = t
            states.append(g.harvest())
        del g
    E, M, e = mlp.samples_from_states(states, emin=1e-7, seed=seed)
    if cap is not None and E.size > cap:
        E, M, e = E[:cap], M[:cap], e[:cap]
    return E, M, e


def train_guess(E, M, e, train_steps=3000, batch=8192):
    """The learned root-solve guess trained on the GPU (library kernels)."""
    from paper_1802_04449_amd import mlp
    tr = mlp.Trainer(E, M, e, seed=3)
    loss0 = tr.loss()
    t0 = time.perf_counter()
    tr.train(train_steps, batch=batch)
    dt = time.perf_counter() - t0
    return tr.params, {"samples": int(E.size), "adam_steps": train_steps, "batch": batch,
                       "loss_initial": loss0, "loss_final": tr.loss(), "train_s": dt}


def minijet_path(params, train, steps, reps):
    """The mini-jet initial state on the benchmark grid, FP64, with the previous-
    stage start and with the learned start (BF16 matrix-core forward): the same
    run both ways; the fields agree to the FP64 bar (tested), the iteration
    counts and times differ."""
    import torch

    import paper_1802_04449_amd as K
    from hydro_inputs import workloads as W
    wl = W.hotspots_minijets(steps=steps)
    out = {"workload": wl.name, "training": train}
    for tag, guess in (("prev_guess", K.KTMI_GUESS_PREV), ("learned_guess", K.KTMI_GUESS_MLP)):
        g = make_hydro(wl, guess=guess)
        if guess == K.KTMI_GUESS_MLP:
            g.set_mlp(params, K.KTMI_MLP_BF16)
        ts = timed_runs(g, wl, steps, reps, warmup=2)
        r = rate(wl.ncell, steps, ts)
        r["newton_mean"] = g.diag()["newton_mean"]
        out[tag] = r
        del g
        torch.cuda.synchronize()
    out["learned_minus_prev_ms_per_step"] = (out["learned_guess"]["ms_per_step"] -
                                             out["prev_guess"]["ms_per_step"])
    return out


def batch_path(params, steps, reps, nev=64):
    """64 uneven events (grids 101^2..301^2 x {1, 33, 65, 105}, eta/s in {0, 0.08,
    0.16}) stepped together (one launch per class and stage) under HIP-graph replay,
    each event on the tile shape the autotuner found fastest for it (tuned once
    per precision, on a throwaway run); four forms: FP64 or mixed precision, with
    the previous-stage or the learned root-solve start."""
    import torch

    import paper_1802_04449_amd as K
    from paper_1802_04449_amd import autotune
    from hydro_inputs import workloads as W
    evs = W.event_batch(nev=nev, steps=steps)
    cells = sum(wl.ncell for wl in evs)
    st = torch.cuda.Stream()
    out = {"events": nev, "cells": cells, "steps": steps,
           "grids": sorted({(w.params["nx"], w.params["ne"]) for w in evs})[:3] + ["..."]}
    tiles = {}
    for precision in (0, 1):
        t0 = time.perf_counter()
        sel = []
        for wl in evs:
            h = make_hydro(wl, stream=st, precision=precision)
            reset(h, wl)
            t, _ = autotune.tune(h, steps=2, repeats=1, use_cache=False)
            sel.append(t)
            del h
        tiles[precision] = sel
        say(f"batch: tiles tuned for precision {precision} in {time.perf_counter() - t0:.1f} s")
    base = None
    for precision, learned in ((0, False), (0, True), (1, False), (1, True)):
        tag = ("fp64" if precision == 0 else "mixed") + ("_learned" if learned else "_prev")
        hs = []
        for wl, t in zip(evs, tiles[precision]):
            h = make_hydro(wl, stream=st, precision=precision, tile=t,
                           guess=K.KTMI_GUESS_MLP if learned else K.KTMI_GUESS_PREV)
            if learned:
                h.set_mlp(params, K.KTMI_MLP_BF16)
            reset(h, wl)
            hs.append(h)
        grp = K.Group(hs)
        grp.set_graph(True)

        def reset_all():
            for h, wl in zip(hs, evs):
                reset(h, wl)

        ts = timed_runs(None, None, steps, reps, warmup=2, step_fn=grp.step, reset_fn=reset_all)
        r = rate(cells, steps, ts)
        diags = [h.diag() for h in hs]
        solves = sum(d["solves"] for d in diags)
        r["newton_mean"] = sum(d["newton_mean"] * d["solves"] for d in diags) / max(solves, 1)
        r["classes"] = grp.classes
        if base is None:
            base = r["value"]
        r["speedup_vs_fp64_prev"] = r["value"] / base
        out[tag] = r
        say(f"batch {tag}: {r['ms_per_step']:.2f} ms per step")
        del grp, hs
        torch.cuda.synchronize()
    shapes = {}
    for t in tiles[0]:
        s = "x".join(map(str, K.ktmi_tile_shape(t)))
        shapes[s] = shapes.get(s, 0) + 1
    out["tiles_fp64"] = shapes
    return out


SURF_BYTES_PER_CELL = 16      # e of both slices
SURF_BYTES_PER_ELEMENT = 400  # its 192-byte record + 13 other fields x 2 slices of one corner cell


def surface_path(wl, warm_steps=10, reps=20, eps_f=0.3):
    """The freeze-out surface finder on two slices (with pi~) of the workload one
    step apart, after warm_steps steps; reps timed launches (HIP events on the
    library's stream).  Algorithmic bytes per launch: 16 B per cell (e of both
    slices) plus 400 B per element (its record and the other 13 fields of one
    corner cell in both slices)."""
    import torch

    import paper_1802_04449_amd as K
    g = make_hydro(wl)
    reset(g, wl)
    g.step(warm_steps)
    tA = g.diag()["tau"]
    A = g.snapshot(True)
    g.step(1)
    tB = g.diag()["tau"]
    B = g.snapshot(True)
    el = g.surface(A, tA, B, tB, eps_f)
    n_el = int(el.shape[0])
    cap = max(n_el, 1)
    out = torch.empty((cap, K.KTMI_SURF_REC), dtype=torch.float64, device=g.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=g.device)
    names = K.ktmi_kernel_names()
    ks = names.index("surface")
    torch.cuda.synchronize()
    K.ktmi_set_timing(g.h, True)
    for _ in range(reps):
        K.ktmi_surface(g.h, A.data_ptr(), tA, B.data_ptr(), tB, True, eps_f, out.data_ptr(), cap,
                       cnt.data_ptr())
    torch.cuda.synchronize()
    tot, launches = K.ktmi_timing(g.h, ks)
    K.ktmi_set_timing(g.h, False)
    avg_ms = tot / launches
    cubes = (wl.params["nx"] - 1) * (wl.params["ny"] - 1) * (wl.params["ne"] - 1)
    alg = SURF_BYTES_PER_CELL * wl.ncell + SURF_BYTES_PER_ELEMENT * n_el
    ach = alg / (avg_ms * 1e-3) / 1e9
    return {"value": cubes / (avg_ms * 1e-3), "unit": "hypercubes/s", "avg_launch_ms": avg_ms,
            "launches": launches, "elements": n_el, "eps_f": eps_f,
            "slices": f"steps {warm_steps} and {warm_steps + 1}, e, u~ and pi~",
            "roofline": {"bound": "hbm", "kernel": "surface", "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                         "algorithmic_bytes": alg}}


SPECTRA_FLOPS = 52  # FP64 operations per (element, bin) with delta f; exp and 1/x count as one


def spectra_path(wl, reps=3, eps_f=0.3, T=0.137):
    """Smooth Cooper-Frye spectra of the freeze-out surface between steps 10 and 11 on
    the paper's 41 x 15 x 48 (Y, pT, phi) bins for 8 species (light mesons and
    baryons), delta f on; reps timed calls (torch events on the call's stream)."""
    import numpy as np
    import torch

    import paper_1802_04449_amd as K
    g = make_hydro(wl)
    reset(g, wl)
    g.step(10)
    tA = g.diag()["tau"]
    A = g.snapshot(True)
    g.step(1)
    tB = g.diag()["tau"]
    B = g.snapshot(True)
    el = g.surface(A, tA, B, tB, eps_f)
    species = ([0.13957, 0.13498, 0.49368, 0.49761, 0.93827, 0.93957, 1.11568, 1.18937],
               [1.0, 1.0, 1.0, 1.0, 2.0, 2.0, 2.0, 2.0], [-1, -1, -1, -1, 1, 1, 1, 1], [0.0] * 8)
    Y = np.linspace(-4.0, 4.0, 41)
    x, _ = np.polynomial.laguerre.laggauss(15)
    pt = 0.35 * x
    u, _ = np.polynomial.legendre.leggauss(48)
    phi = np.pi * (u + 1.0)
    wP = eps_f + 0.1  # e + P at the freeze-out density (GeV/fm^3)
    K.spectra(el, T, wP, species, Y, pt, phi)  # warm-up
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        K.spectra(el, T, wP, species, Y, pt, phi)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    evals = int(el.shape[0]) * 8 * 41 * 15 * 48
    tfl = evals * SPECTRA_FLOPS / (ms * 1e-3) / 1e12
    return {"value": evals / (ms * 1e-3), "unit": "element-bin evaluations/s", "ms_per_call": ms,
            "elements": int(el.shape[0]), "species": 8, "bins": [41, 15, 48],
            "roofline": {"bound": "alu", "achieved": tfl, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": tfl / 78.6, "flops_per_evaluation": SPECTRA_FLOPS}}


def copy_calibration():
    """A plain device-to-device copy of 2^30 bytes, five times: rocprofv3's FETCH_SIZE and
    WRITE_SIZE per dispatch for it calibrate the counters against known traffic."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 8, "repeats": 5}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, steps_all=5, steps_one=1):
    """The CPU oracle as it stands, on the headline grid and initial state: after
    one untimed step (which includes the first-step estimate), `steps_one` steps at
    one thread and `steps_all` steps at all host threads (at most 16)."""
    import oracle as O
    from tests import gpu_common as G

    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    res = {}
    for tag, threads, steps in (("one_thread", 1, steps_one),
                                ("all_threads", min(16, nproc or 1), steps_all)):
        O.set_threads(threads)
        used = O.max_threads()
        o = O.Oracle(G.oracle_params(wl.params), eos=wl.eos)
        o.set_initial(wl.ic)
        o.step(1)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        res[tag] = {"value": wl.ncell * steps / dt, "cores": used, "seconds": dt, "steps": steps}
        say(f"cpu oracle {tag}: {res[tag]['value']:.3e} cell-updates/s")
        del o
    a = res["all_threads"]
    return {"value": a["value"], "unit": "cell-updates/s", "cores": a["cores"], "kind": "oracle",
            "sample": f"the full {wl.params['nx']}x{wl.params['ny']}x{wl.params['ne']} grid from "
                      f"the same initial state: steps 2..{1 + a['steps']} at {a['cores']} threads "
                      f"({a['seconds']:.1f} s); one thread: step 2 "
                      f"({res['one_thread']['seconds']:.1f} s)",
            "one_thread": res["one_thread"]["value"], "nproc": nproc, "cpu_model": cpu_model()}


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps per run (200: the whole headline run)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before the first run")
    ap.add_argument("--reps", type=int, default=5, help="timed runs; value is the median")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="hotspots",
                    choices=["hotspots", "gubser_dense", "large", "batch64", "bulk", "minijets"],
                    help="hotspots: the headline configuration; gubser_dense: the same grid and "
                         "physics with a smooth Gubser profile that leaves no vacuum cells; large: "
                         "385x385x129 single event; batch64: 64 uneven events in grouped launches; "
                         "bulk: the headline configuration with bulk pressure and baryon density; "
                         "minijets: the headline grid with the mini-jet initial state")
    ap.add_argument("--graph", action="store_true", help="replay each step as a HIP graph")
    ap.add_argument("--tile", type=int, default=-1, help="tile shape index (-1: library default)")
    ap.add_argument("--precision", type=int, default=0,
                    help="0: plain FP64; 1: mixed (FP32 flux/relaxation, FP64 root solve and sources)")
    ap.add_argument("--quiet-skip", action="store_true",
                    help="skip tiles whose neighbourhood stayed vacuum (bitwise identical results)")
    ap.add_argument("--no-paths", action="store_true", help="only the headline line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (counter calibration)")
    ap.add_argument("--only-surface", action="store_true",
                    help="only measure the freeze-out surface finder on the workload (profiling)")
    ap.add_argument("--only-spectra", action="store_true",
                    help="only measure the Cooper-Frye spectra on the workload's surface (profiling)")
    ap.add_argument("--only-batch", action="store_true",
                    help="only the 64-event batch (FP64 and mixed, with and without the network)")
    ap.add_argument("--batch-steps", type=int, default=20)
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1802_04449_amd as K
    from hydro_inputs import workloads as W

    wl = {"hotspots": W.hotspots_viscous, "gubser_dense": W.gubser_dense_viscous,
          "large": W.large_event, "bulk": W.hotspots_bulk, "batch64": W.hotspots_viscous,
          "minijets": W.hotspots_minijets}[args.workload](steps=args.steps)
    if args.only_surface:
        print(json.dumps({"workload": wl.name, "freezeout_surface": surface_path(wl)}), flush=True)
        return
    if args.only_spectra:
        print(json.dumps({"workload": wl.name, "cooper_frye_spectra": spectra_path(wl)}), flush=True)
        return
    if args.only_batch or args.workload == "batch64":
        E, M, e = harvest_samples([W.hotspots_viscous()], at_steps=range(0, 201, 20), cap=10 ** 7)
        params, train = train_guess(E, M, e)
        b = batch_path(params, args.batch_steps, 3)
        b["training"] = train
        print(json.dumps({"workload": "batch of 64 uneven events", "batch64": b}), flush=True)
        return

    p = wl.params
    bpc = BYTES_PER_CELL if p["viscous"] else BYTES_PER_CELL_IDEAL
    if p.get("zetas", 0) > 0 or p.get("baryon", 0):
        bpc = dict(BYTES_PER_CELL, **BYTES_PER_CELL_BULK)
    if args.precision == 1 and p["viscous"] and bpc is BYTES_PER_CELL:
        bpc = dict(BYTES_PER_CELL, **BYTES_PER_CELL_MIXED)
    stream = torch.cuda.Stream() if args.graph else None
    g = make_hydro(wl, stream=stream, tile=args.tile, precision=args.precision)
    if args.quiet_skip:
        g.set_quiet_skip(True)
    if args.graph:
        g.set_graph(True)
    say(f"headline: {wl.name}, {args.reps} runs of {args.steps} steps")
    ts = timed_runs(g, wl, args.steps, args.reps, args.warmup)
    head = rate(wl.ncell, args.steps, ts)
    diag = g.diag()
    # per-kernel durations: a separate instrumented run (graph replay off)
    if args.graph:
        g.set_graph(False)
    per_kernel = kernel_times(g, wl, args.steps)
    say(f"headline: {head['ms_per_step']:.3f} ms per step")
    out = {
        "metric": "cell-updates/s of viscous KT+RK2 step, plain FP64 vs batched/learned/FP32 @1e-6",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": p["nx"], "ny": p["ny"], "ne": p["ne"],
                   "dx": p["dx"], "deta": p["de"], "tau0": p["tau0"], "h": p["h"],
                   "eta_over_s": p["etas"], "ic": wl.note or "200 Gaussian hotspots, seed 1",
                   "eos": "1555-row synthetic crossover table",
                   "path": ("plain FP64" if args.precision == 0 else "mixed FP32/FP64") +
                           (", quiet tiles skipped" if args.quiet_skip else "") +
                           (", HIP graph" if args.graph else ""),
                   "timing": f"median of {args.reps} runs of {args.steps} steps from the "
                             f"initial state, uninstrumented"},
        "roofline": roofline_of(wl, per_kernel, bpc),
        "kernels": kernels_summary(per_kernel, wl, bpc),
        "reps_s": head["reps_s"],
        "tile": list(K.ktmi_tile_shape(K.ktmi_get_tile(g.h))),
        "graph": bool(args.graph),
        "diag": {k: diag[k] for k in ("tau", "eps_max", "newton_mean", "newton_max", "clamps",
                                      "nonconv", "nans", "vacuum", "errors")},
        "context": {"paper_table_II_viscous_gpu_cell_updates_per_s": 1.69e7,
                    "paper_hardware": "AMD FirePro S9150, 385x385x115 cells"},
    }
    del g
    torch.cuda.synchronize()
    headline_default = (args.workload == "hotspots" and args.precision == 0 and
                        not args.quiet_skip and args.tile < 0)
    if headline_default and not args.no_paths:
        paths = {}
        say("path: C0 ideal Gubser 33x33x17")
        w0 = W.gubser_ideal_33()
        paths["C0_gubser_ideal_33x33x17_fp64"] = single_path(w0, 50, 5)
        say("path: mixed precision")
        paths["C1_mixed_fp32_fp64"] = single_path(wl, args.steps, 3,
                                                  bpc=dict(BYTES_PER_CELL, **BYTES_PER_CELL_MIXED),
                                                  precision=1)
        say("path: quiet tiles")
        paths["C1_fp64_quiet_skip"] = single_path(wl, args.steps, 3, quiet=True)
        say("path: HIP graph")
        paths["C1_fp64_graph"] = single_path(wl, args.steps, 3, graph=True)
        say("path: lambda_1")
        paths["C1_fp64_lambda1"] = single_path(wl, args.steps, 3, bpc=BYTES_PER_CELL,
                                               lambda1_hat=-10.0)
        paths["C1_fp64_lambda1"]["note"] = "second-order lambda_1 term, lambda1_hat = -10"
        say("path: bulk and baryon")
        wb = W.hotspots_bulk(steps=args.steps)
        paths["C1_fp64_bulk_baryon"] = single_path(wb, args.steps, 3,
                                                   bpc=dict(BYTES_PER_CELL, **BYTES_PER_CELL_BULK))
        paths["C1_fp64_bulk_baryon"]["note"] = ("bulk pressure (zeta/s = 0.04) and net-baryon "
                                                "density transported")
        say("path: harvesting and training the root-solve guess")
        E, M, e = harvest_samples([wl], at_steps=range(0, 201, 20), cap=10 ** 7)
        params, train = train_guess(E, M, e)
        train["harvested_from"] = f"{wl.name} at steps 0, 20, ..., 200 (non-vacuum cells)"
        say(f"trained on {train['samples']} samples in {train['train_s']:.1f} s")
        say("path: C2 mini-jets")
        paths["C2_minijets_fp64"] = minijet_path(params, train, args.steps, 3)
        say("path: C3 batch of 64 events")
        paths["C3_batch64"] = batch_path(params, args.batch_steps, 3)
        say("path: C4 large event")
        w4 = W.large_event()
        paths["C4_large_385x385x129_fp64"] = single_path(w4, 20, 3, bpc=BYTES_PER_CELL)
        paths["C4_large_385x385x129_mixed"] = single_path(
            w4, 20, 3, bpc=dict(BYTES_PER_CELL, **BYTES_PER_CELL_MIXED), precision=1)
        for k in ("C4_large_385x385x129_fp64", "C4_large_385x385x129_mixed"):
            paths[k]["note"] = "first 20 of the 1000 steps (the rate is per step)"
        say("path: freeze-out surface and spectra")
        paths["freezeout_surface"] = surface_path(wl)
        paths["cooper_frye_spectra"] = spectra_path(wl)
        out["paths"] = paths
    if not args.no_cpu_baseline and headline_default:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
