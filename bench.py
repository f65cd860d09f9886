"""Benchmark: cell-updates/s of the viscous KT + RK2 step on one MI355X.

Workload (default): viscous hydro, eta/s = 0.08, 201 x 201 x 105 cells
(dx = dy = 0.16 fm, deta = 0.3), tau0 = 0.6 fm, h = 0.01 fm, 200 seeded Gaussian
hotspots, 1555-row synthetic EoS, FP64.  A step is one full RK2 step (all three
stencil passes, both root solves, the diagnostics reduction) over the grid.

Prints one JSON line.  `roofline` is measured live for the dominant kernel with
HIP events recorded on the library's stream around every launch in the timed
region; `cpu_baseline` times the CPU oracle on a bounded sample of the same
workload (rank 0, N = 1 only).  `paths` times the other paths on the same grid:
mixed precision, quiet-tile skipping, the freeze-out surface finder, the
Cooper-Frye spectra, the lambda_1 term, bulk pressure with baryon density, and a
grouped batch of 64 events with the learned root-solve guess.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s

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


def source_sha256() -> str:
    """Hash of everything the step's stencil kernels are compiled from (their
    sources, the headers they include and the build flags): counter-derived
    traffic recorded under profiles/ is used only while it matches the code
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


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from rocprofv3 FETCH_SIZE and
    WRITE_SIZE (calibrated against a plain copy), or None when no record exists
    for the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_sha256():
        return None
    r = rec.get("bytes_per_launch", {}).get(workload, {}).get(kernel)
    return None if r is None else r["fetch_bytes"] + r["write_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--workload", default="hotspots",
                    choices=["hotspots", "gubser_dense", "large", "batch64", "bulk"],
                    help="hotspots: the benchmark configuration; gubser_dense: the same grid and "
                         "physics with a smooth Gubser profile that leaves no vacuum cells; large: "
                         "385x385x129 single event; batch64: 64 uneven events in grouped launches; "
                         "bulk: the benchmark configuration with bulk pressure and baryon density")
    ap.add_argument("--graph", action="store_true", help="replay each step as a HIP graph")
    ap.add_argument("--autotune", action="store_true",
                    help="time every tile shape first (on a discarded run) and use the fastest")
    ap.add_argument("--tile", type=int, default=-1, help="tile shape index (-1: library default)")
    ap.add_argument("--precision", type=int, default=0,
                    help="0: plain FP64; 1: mixed (FP32 flux/relaxation, FP64 root solve and sources)")
    ap.add_argument("--quiet-skip", action="store_true",
                    help="skip tiles whose neighbourhood stayed vacuum (bitwise identical results)")
    ap.add_argument("--guess", default="prev", choices=["prev", "mlp"],
                    help="root-solve start: previous stage, or a network trained first on states "
                         "harvested from the same workload (GPU training kernels)")
    ap.add_argument("--no-paths", action="store_true",
                    help="skip the extra measurements: the same workload in mixed precision, and "
                         "the 64-event batch with mixed precision and the learned guess")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (counter calibration)")
    ap.add_argument("--only-surface", action="store_true",
                    help="only measure the freeze-out surface finder on the workload (profiling)")
    ap.add_argument("--only-spectra", action="store_true",
                    help="only measure the Cooper-Frye spectra on the workload's surface (profiling)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_04449_amd as K
    from hydro_inputs import workloads as W

    if args.workload == "batch64":
        print(json.dumps(bench_batch(args, learned=args.guess == "mlp")), flush=True)
        return
    wl = {"hotspots": W.hotspots_viscous, "gubser_dense": W.gubser_dense_viscous,
          "large": W.large_event, "bulk": W.hotspots_bulk}[args.workload](steps=args.steps)
    if args.only_surface:
        print(json.dumps({"workload": wl.name, "freezeout_surface": surface_path(wl)}), flush=True)
        return
    if args.only_spectra:
        print(json.dumps({"workload": wl.name, "cooper_frye_spectra": spectra_path(wl)}), flush=True)
        return
    p = wl.params
    stream = torch.cuda.Stream() if args.graph else None
    train = None
    if args.guess == "mlp":
        params, train = train_guess([wl])
    g = K.Hydro(tile=args.tile, precision=args.precision, stream=stream,
                guess=K.KTMI_GUESS_MLP if args.guess == "mlp" else K.KTMI_GUESS_PREV, **p)
    g.set_eos(wl.eos)
    if args.guess == "mlp":
        g.set_mlp(params, K.KTMI_MLP_BF16)
    if args.quiet_skip:
        g.set_quiet_skip(True)

    def initial():
        if wl.T4 is not None:
            g.set_initial_conserved(wl.T4)
        else:
            g.set_initial(wl.ic)

    tile_times = None
    if args.autotune:
        # tune on a throwaway copy of the state, then start the measured run afresh
        from paper_1802_04449_amd import autotune
        initial()
        tile, tile_times = autotune.tune(g, steps=3, use_cache=False)
    initial()
    if args.graph:
        g.set_graph(True)
    g.step(args.warmup)
    torch.cuda.synchronize()

    K.ktmi_set_timing(g.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    names = K.ktmi_kernel_names()
    per_kernel = {}
    for k, n in enumerate(names):
        tot, cnt = K.ktmi_timing(g.h, k)
        if cnt:
            per_kernel[n] = dict(total_ms=tot, launches=cnt, avg_ms=tot / cnt)
    K.ktmi_set_timing(g.h, False)
    diag = g.diag()

    dt = t1 - t0
    ncell = wl.ncell
    value = ncell * args.steps / dt
    dom = max(per_kernel, key=lambda n: per_kernel[n]["total_ms"])
    bpc = BYTES_PER_CELL if p["viscous"] else BYTES_PER_CELL_IDEAL
    if p.get("zetas", 0) > 0 or p.get("baryon", 0):
        bpc = dict(BYTES_PER_CELL, **BYTES_PER_CELL_BULK)
    bytes_launch = bpc[dom] * ncell
    achieved = bytes_launch / (per_kernel[dom]["avg_ms"] * 1e-3) / 1e9
    step_bytes = sum(bpc.get(n, 0) * ncell * per_kernel[n]["launches"] for n in per_kernel)
    out = {
        "metric": "cell-updates/s of viscous KT+RK2 step, plain FP64 vs batched/learned/FP32 @1e-6",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
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
                           (", learned guess (BF16 forward)" if args.guess == "mlp" else "")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(wl.name, dom) if args.precision == 0 else None),
                     "algorithmic_bytes": bytes_launch, "bytes_per_cell": bpc[dom],
                     "avg_launch_ms": per_kernel[dom]["avg_ms"]},
        "kernels": {n: round(v["avg_ms"], 4) for n, v in per_kernel.items()},
        "tile": list(K.ktmi_tile_shape(K.ktmi_get_tile(g.h))),
        "tile_ms_per_step": ({str(K.ktmi_tile_shape(t)): round(v, 3) for t, v in tile_times.items()}
                             if tile_times else None),
        "step_hbm_GBs_algorithmic": step_bytes / dt / 1e9,
        "diag": {k: diag[k] for k in ("tau", "eps_max", "newton_mean", "newton_max", "clamps",
                                      "nonconv", "nans", "vacuum")},
        "context": {"paper_table_II_viscous_gpu_cell_updates_per_s": 1.69e7,
                    "paper_hardware": "AMD FirePro S9150, 385x385x115 cells"},
    }
    out["graph"] = bool(args.graph)
    if train:
        out["training"] = train
    if args.precision == 0 and not args.no_paths and args.guess == "prev" and not args.quiet_skip:
        del g
        torch.cuda.synchronize()
        out["paths"] = {"mixed_fp32_fp64": mixed_path(wl, args)}
        out["paths"]["fp64_quiet_skip"] = mixed_path(wl, args, precision=0, quiet=True)
        out["paths"]["freezeout_surface"] = surface_path(wl)
        out["paths"]["cooper_frye_spectra"] = spectra_path(wl)
        out["paths"]["fp64_lambda1"] = mixed_path(wl, args, precision=0, lambda1_hat=-10.0)
        out["paths"]["fp64_lambda1"]["note"] = ("second-order lambda_1 term on, lambda1_hat = -10, "
                                                "tau_pi = 5 eta/(sT)")
        if wl.name.startswith("hotspots_viscous"):
            pw = wl.params
            wb = W.hotspots_bulk(nx=pw["nx"], ny=pw["ny"], ne=pw["ne"], dx=pw["dx"], dy=pw["dy"],
                                 de=pw["de"])
            out["paths"]["fp64_bulk_baryon"] = mixed_path(wb, args, precision=0,
                                                          bytes_per_cell=BYTES_PER_CELL_BULK)
            out["paths"]["fp64_bulk_baryon"]["note"] = (
                "bulk pressure (zeta/s = 0.04, tau_Pi = 5 (zeta/s) hbarc/T) and net-baryon "
                "density transported (16 components per face)")
        b = bench_batch(args, precision=1, learned=True, steps=10, warmup=2)
        out["paths"]["batch64_mixed_learned"] = {
            k: b[k] for k in ("value", "unit", "ms_per_step", "steps", "newton_mean", "training")}
        out["paths"]["batch64_mixed_learned"]["cells"] = b["config"]["cells"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)


def mixed_path(wl, args, precision=1, quiet=False, bytes_per_cell=None, **extra):
    """The same workload with FP32 reconstruction, fluxes and relaxation source
    (FP64 root solve, geometric source and state; errors against the FP64
    oracle are bounded by the GPU tests, <= 1e-6 in e and u~), or (precision 0,
    quiet) in FP64 with quiet tiles skipped (fields and diagnostics identical to
    the full computation bit for bit, tested).  `extra` overrides descriptor
    fields (the second-order path sets lambda1_hat).  With bytes_per_cell the
    timed steps also record each pass's average duration (HIP events on the
    library's stream) and its algorithmic HBM rate."""
    import torch

    import paper_1802_04449_amd as K
    d = dict(wl.params)
    d.update(extra)
    g = K.Hydro(precision=precision, **d)
    g.set_eos(wl.eos)
    if quiet:
        g.set_quiet_skip(True)
    if wl.T4 is not None:
        g.set_initial_conserved(wl.T4)
    else:
        g.set_initial(wl.ic)
    g.step(args.warmup)
    torch.cuda.synchronize()
    if bytes_per_cell:
        K.ktmi_set_timing(g.h, True)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"value": wl.ncell * args.steps / dt, "unit": "cell-updates/s",
           "ms_per_step": dt / args.steps * 1e3, "steps": args.steps}
    if bytes_per_cell:
        kern = {}
        for k, n in enumerate(K.ktmi_kernel_names()):
            tot, cnt = K.ktmi_timing(g.h, k)
            if cnt and n in bytes_per_cell:
                ms = tot / cnt
                gbs = bytes_per_cell[n] * wl.ncell / (ms * 1e-3) / 1e9
                kern[n] = {"avg_launch_ms": round(ms, 4), "achieved_GBs": round(gbs, 1),
                           "frac": round(gbs / HBM_PEAK_GBS, 4),
                           "bytes_per_cell": bytes_per_cell[n]}
        K.ktmi_set_timing(g.h, False)
        out["kernels"] = kern
    if quiet:
        out["quiet_tiles"], out["tiles"] = K.ktmi_quiet_tiles(g.h)
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
    g = K.Hydro(**wl.params)
    g.set_eos(wl.eos)
    if wl.T4 is not None:
        g.set_initial_conserved(wl.T4)
    else:
        g.set_initial(wl.ic)
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
    g = K.Hydro(**wl.params)
    g.set_eos(wl.eos)
    if wl.T4 is not None:
        g.set_initial_conserved(wl.T4)
    else:
        g.set_initial(wl.ic)
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


def train_guess(wls, steps_at=(0, 5, 10), train_steps=1500):
    """Learned root-solve guess for a set of events: harvest (E, M, e) from FP64
    runs of the given events at a few times, train on the GPU (library kernels)."""
    import paper_1802_04449_amd as K
    from paper_1802_04449_amd import mlp
    states = []
    for wl in wls:
        g = K.Hydro(**wl.params)
        g.set_eos(wl.eos)
        g.set_initial(wl.ic)
        done = 0
        for t in steps_at:
            g.step(t - done)
            done = t
            states.append(g.harvest())
        del g
    E, M, e = mlp.samples_from_states(states, emin=1e-7, seed=1)
    tr = mlp.Trainer(E, M, e, seed=3)
    loss0 = tr.loss()
    t0 = time.perf_counter()
    tr.train(train_steps, batch=4096)
    dt = time.perf_counter() - t0
    return tr.params, {"samples": int(E.size), "adam_steps": train_steps, "loss_initial": loss0,
                       "loss_final": tr.loss(), "train_s": dt,
                       "harvested_from": [f"{w.name} at steps {list(steps_at)}" for w in wls]}


def bench_batch(args, precision=None, learned=False, steps=None, warmup=None):
    """64 uneven events (grids 101^2..301^2 x {1, 33, 65, 105}, eta/s in {0, 0.08, 0.16})
    stepped together: per stage one launch per (mode, tile, precision, guess) class.
    learned: root solves start from a network trained first on harvested states
    of two of the events."""
    import torch

    import paper_1802_04449_amd as K
    from hydro_inputs import workloads as W

    precision = args.precision if precision is None else precision
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    evs = W.event_batch(nev=64, steps=steps)
    params, train = (None, None)
    if learned:
        params, train = train_guess([evs[0], evs[1]])
    st = torch.cuda.Stream()
    hs = []
    for wl in evs:
        guess = K.KTMI_GUESS_MLP if learned else K.KTMI_GUESS_PREV
        h = K.Hydro(stream=st, precision=precision, guess=guess, **wl.params)
        h.set_eos(wl.eos)
        if learned:
            h.set_mlp(params, K.KTMI_MLP_BF16)
        h.set_initial(wl.ic)
        hs.append(h)
    grp = K.Group(hs)
    if args.graph:
        grp.set_graph(True)
    grp.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grp.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = sum(wl.ncell for wl in evs)
    diags = [h.diag() for h in hs]
    solves = sum(d["solves"] for d in diags)
    iters = sum(d["newton_mean"] * d["solves"] for d in diags)
    path = ("FP64" if precision == 0 else "mixed FP32/FP64") + (", learned guess" if learned else "")
    out = {"metric": "cell-updates/s of viscous KT+RK2 step, plain FP64 vs batched/learned/FP32 @1e-6",
           "value": cells * steps / dt, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": dt / steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if precision == 0 else "f32+f64", "data": "synthetic",
           "config": {"workload": "batch of 64 uneven events", "cells": cells, "path": path,
                      "classes": grp.classes, "graph": bool(args.graph)},
           "newton_mean": iters / max(solves, 1)}
    if train:
        out["training"] = train
    del grp, hs
    return out


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


def cpu_baseline(wl, steps):
    """The CPU oracle as it stands, on the same grid and initial state, all host
    threads, `steps` steps (the set-up and first-step estimate are not timed)."""
    import oracle as O
    from tests import gpu_common as G

    threads = min(16, os.cpu_count() or 1)
    O.set_threads(threads)
    o = O.Oracle(G.oracle_params(wl.params), eos=wl.eos)
    o.set_initial(wl.ic)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": wl.ncell * steps / dt, "unit": "cell-updates/s", "cores": O.max_threads(),
            "kind": "oracle",
            "sample": f"full {wl.params['nx']}x{wl.params['ny']}x{wl.params['ne']} grid, first "
                      f"{steps} steps from the same initial state ({dt:.1f} s)"}


if __name__ == "__main__":
    main()
