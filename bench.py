#!/usr/bin/env python3
"""Throughput of the HELIOS radiative-equilibrium hot path on one MI355X.

A step is one radiative-equilibrium iteration of the whole hot path over the
batch: opacity mixing (helios_mix_opacity), the flux solve (helios_flux:
Planck sources, boundary fluxes, sublayer coefficients, 1 + 4 scattering
passes, Gauss and bin sums) and the FP64 temperature update with the
interface re-interpolation (helios_radeq), all in the library's HIP kernels,
with inputs resident in HBM.

Default workload (the largest one that fits one GPU): one production chunk
of 256 parameter-described atmospheres x 200 layers (401 points) x 3000
bins x 20 Gauss points, four float32 k-tables on a 20 T x 20 log P grid
(384 MB), mixed precision (FP32 sweeps, FP64 sums and update), started from
the warm-start network, seeded synthetic inputs
(paper_1606_05474_amd.workloads).  The single-atmosphere spectral workload
(100 layers x 3000 bins x 20 g, FP64 and mixed) and the uneven 512-atmosphere
batch are reported alongside, and the FP64 oracle's rate on one of the
chunk's atmospheres on the host cores.

Metric: layer*bin*g flux updates per second (one unit = one layer, both
sublayers, one bin, one g point, through one complete flux call).

Usage:  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
        python bench.py --workload {spectral,batch,chunk,production,exact,layers,modes}
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")
# Algorithmic bytes one layer*bin*g unit must move through one flux call
# (opacities at the sublayer's two points read; upward and downward per-g
# state at two points read and written; Planck values, w0 and g0 amortised
# over the 20 g-points): 16 + 64 + 0.8 + 0.8 in FP64, 8 + 32 + 0.4 + 0.4 in
# FP32.  The roofline fraction is quoted against these, whatever the kernel
# itself moves (it keeps no downward state between calls).
UNIT_BYTES = {"fp64": 81.6, "mixed": 40.8}


def sweep_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_1606_05474_amd", "csrc", "k_sweep.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def sweep_algorithmic_bytes(n: int, nb: int, ng: int, rbytes: int) -> int:
    """Bytes one flux-sweep launch must move for one atmosphere: opacities at
    the points, the upward-flux warm start in (the TOA point is never read)
    and out, the Planck values per (bin, point) (float64 in both precisions),
    w0 and g0 per (bin, layer), the two boundary fluxes and the Gauss
    weights, and the two Gauss-summed partials per (bin, point) (in the
    sweep's precision)."""
    npt = 2 * n + 1
    per_bin = (ng * npt * rbytes            # kappa
               + ng * (npt - 1) * rbytes    # F_up warm start in
               + ng * npt * rbytes          # F_up out
               + npt * 8                    # B
               + 2 * n * 8                  # w0, g0
               + 2 * 8                      # F_top, F_int
               + 2 * npt * rbytes)          # Gauss partials, up and down
    return nb * per_bin + ng * 8


def iso_algorithmic_bytes(n: int, nb: int, ng: int, rbytes: int) -> int:
    """As sweep_algorithmic_bytes for n isothermal layers: one opacity per
    layer, the warm start at the n + 1 interfaces (the top one is never
    read), one Planck value per layer, w0 and g0, the boundary fluxes and the
    Gauss-summed partials at the interfaces."""
    per_bin = (ng * n * rbytes + ng * n * rbytes + ng * (n + 1) * rbytes + n * 8 + 2 * n * 8 + 2 * 8
               + 2 * (n + 1) * rbytes)
    return nb * per_bin + ng * 8


def timed_steps(s, steps: int, warmup: int):
    """W untimed steps, then exactly K timed ones: wall clock between two
    device synchronisations, and HIP events recorded by the library around
    the flux sweep launches of every timed step, on the stream the sweep runs
    on.  Returns (wall seconds, sweep milliseconds per step)."""
    import torch

    from paper_1606_05474_amd import helios as H

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        s.step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:  # torch creates the events on their first record
        e0.record(stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        H.set_sweep_events(e0, e1)
        s.step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    H.set_sweep_events(None, None)
    return wall, sum(e0.elapsed_time(e1) for e0, e1 in ev) / steps


def require_running(s, what: str):
    """Every atmosphere of the batch must still be running: a converged or
    failed one would be skipped by the kernels and its work not done."""
    import numpy as np

    from paper_1606_05474_amd import helios as H

    st = s.status.cpu().numpy()
    if np.any(st != H.ATM_RUNNING):
        codes = {int(c): int((st == c).sum()) for c in np.unique(st)}
        print(f"{what}: not every atmosphere is running through the timed steps (status counts {codes})",
              file=sys.stderr, flush=True)
        sys.exit(3)
    return int(st.size)


def c5_chunk(args):
    """One production chunk: args.n_atm atmospheres (seed 5) of 200 layers x
    3000 bins x 20 g, mixed precision, dead band, network warm start.  The
    convergence test runs at tolerance 0 during the measurement, so no
    atmosphere (and no layer of the dead band) can freeze and every step does
    the whole chunk's work; require_running checks that."""
    import numpy as np
    import torch

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import warmstart as WS
    from paper_1606_05474_amd import workloads as W

    n, nb, ng = 200, 3000, 20
    atms, kt = W.learned_workload(5, args.n_atm, 0, n=n, nb=nb)
    b = H.Batch(atms)
    s = H.Solver(b, H.KTable(kt), prec=H.MIXED, opts=H.REOptions(deadband=1, tol=0.0), bin_fluxes=False)
    x = np.stack([a["params"] for a in atms])
    s.reset(np.concatenate([a["T0"] for a in atms]))
    t_tune = time.perf_counter()
    s.autotune()
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    net = WS.load(args.weights)
    fb = s.warm_reset(net, x, net.logP, m0=0.3)
    wall, sweep_ms = timed_steps(s, args.steps, args.warmup)
    running = require_running(s, "production chunk")
    units = len(atms) * n * nb * ng
    alg = UNIT_BYTES["mixed"] * units
    gbs = alg / (sweep_ms * 1e-3) / 1e9
    out = {
        "value": units * args.steps / wall, "ms_per_step": wall / args.steps * 1e3, "units_per_step": units,
        "sweep_ms": sweep_ms, "running": running, "network_fallbacks": int((fb != 0).sum()),
        "autotune_s": t_tune, "shapes": {str(k): list(v) for k, v in H.sweep_shapes(s.b, H.MIXED).items()},
        "roofline": {"bound": "hbm", "kernel": "sweep_kernel (flux sweep, one launch per step)",
                     "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": traffic_entry("c5chunk") if len(atms) == 256 else None,
                     "bytes_per_unit": UNIT_BYTES["mixed"], "units_per_launch": units,
                     "algorithmic_bytes_per_launch": alg, "avg_launch_ms": sweep_ms,
                     "kernel_own_bytes_per_launch": len(atms) * sweep_algorithmic_bytes(n, nb, ng, 4)},
    }
    cpu_atm = atms[0]
    del s, b
    torch.cuda.empty_cache()
    return out, cpu_atm, kt


def c3_batch(steps: int, warmup: int):
    """RE-iteration throughput of the uneven 512-atmosphere batch (n ~
    U{50..200}, 400-3000 strided bins), mixed precision, isothermal start,
    tolerance 0 during the measurement (every atmosphere running)."""
    import numpy as np
    import torch

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    atms, kt = W.batch_workload(n_atm=512)
    atms.sort(key=lambda a: int(a["n"]))  # contiguous size classes
    b = H.Batch(atms)
    s = H.Solver(b, H.KTable(kt), prec=H.MIXED, opts=H.REOptions(tol=0.0), bin_fluxes=False)
    T0 = np.concatenate([a["T0"] for a in atms])
    s.reset(T0)
    s.autotune()
    s.reset(T0)
    wall, sweep_ms = timed_steps(s, steps, warmup)
    running = require_running(s, "uneven batch")
    units = int(sum(int(a["n"]) * len(a["lambda_c"]) * int(a["ng"]) for a in atms))
    alg = UNIT_BYTES["mixed"] * units
    out = {"value": units * steps / wall, "unit": "layer*bin*g/s", "ms_per_step": wall / steps * 1e3,
           "units_per_step": units, "steps": steps, "running": running,
           "sweep_ms_per_step": sweep_ms, "sweep_frac_of_hbm_peak": alg / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "shapes": {str(k): list(v) for k, v in H.sweep_shapes(s.b, H.MIXED).items()}}
    del s, b
    torch.cuda.empty_cache()
    return out


def cpu_baseline_c5(atm: dict, kt: dict, budget_s: float):
    """The FP64 oracle as it stands on the host: whole RE iterations (profile,
    opacity, flux with 1 + 4 passes, RE step) of one 200-layer x 3000-bin x
    20-g atmosphere of the chunk, from its isothermal start: one iteration on
    one core, then iterations on all the cores it may use (OpenMP over
    columns; at most 16, the host share of one GPU) until budget_s passed."""
    import numpy as np

    import oracle as ref

    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    threads = max(1, min(16, avail))
    n, nb, ng = int(atm["n"]), len(atm["lambda_c"]), int(atm["ng"])
    P = ref.grid(atm["P_c"])
    T_c = np.array(atm["T0"], np.float64)
    m = np.ones(n)
    hist = np.zeros(n, np.int32)
    F_up = np.zeros((nb, ng, 2 * n + 1))

    def iteration(th):
        T = ref.profile(P, T_c)
        kap = ref.mix_opacity(kt, T, P, atm["vmr"], atm["bin_index"], ng)
        res = ref.flux(atm, kap, T, P, F_up, n_scat=4, n_threads=th, want_dn=False)
        ref.radeq(atm, P, res["F_bol"], T_c, m, hist)

    t0 = time.perf_counter()
    iteration(1)
    one = time.perf_counter() - t0
    iters = 0
    t0 = time.perf_counter()
    while True:
        iteration(threads)
        iters += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    wall = time.perf_counter() - t0
    units = n * nb * ng
    return {"value": units * iters / wall, "unit": "layer*bin*g/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} full RE iterations (profile, opacity, 1 + 4 pass flux, RE step) of one "
                      f"{n}-layer x {nb}-bin x {ng}-g atmosphere of the chunk on {threads} threads "
                      f"({wall:.1f} s wall), after one iteration on one core ({one:.1f} s)",
            "single_core": {"value": units / one, "seconds_per_iteration": one},
            "nproc": nproc, "cpus_available": avail}


def run_gpu(prec: int, steps: int, warmup: int, atm: dict, kt: dict, **solver_kw):
    import torch

    from paper_1606_05474_amd import helios as H

    b = H.Batch([atm])
    ktd = H.KTable(kt)
    # tolerance 0: the atmosphere cannot converge (and freeze) while it is timed
    solver_kw.setdefault("opts", H.REOptions(tol=0.0))
    s = H.Solver(b, ktd, prec=prec, **solver_kw)
    s.reset(atm["T0"])
    s.autotune()  # the library's sweep-shape autotuner (kept for the process)
    shape = H.sweep_shapes(s.b, prec)
    s.reset(atm["T0"])
    wall, sweep_ms = timed_steps(s, steps, warmup)
    require_running(s, "single atmosphere")
    n, nb, ng = int(atm["n"]), len(atm["lambda_c"]), int(atm["ng"])
    units = n * nb * ng
    rbytes = 4 if prec == H.MIXED else 8
    alg = sweep_algorithmic_bytes(n, nb, ng, rbytes)
    return {
        "value": units * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "sweep_ms": sweep_ms,
        "sweep_bytes": alg,
        "sweep_gbs": alg / (sweep_ms * 1e-3) / 1e9,
        "shape": {str(k): list(v) for k, v in shape.items()},
        "status": int(s.status[0].item()),
        "updates": int(s.iters[0].item()),
    }


def run_batch(prec: int, steps: int, warmup: int, atms: list, kt: dict, max_iter: int):
    """The uneven batch: throughput of RE iterations over every atmosphere
    (all running), then a full graph-replayed solve to convergence."""
    import numpy as np
    import torch

    from paper_1606_05474_amd import helios as H

    b = H.Batch(atms)
    # mixed precision takes the dead band (thin layers within the tolerance keep
    # their temperature; without it their FP32 drift can run away)
    s = H.Solver(b, H.KTable(kt), prec=prec, opts=H.REOptions(deadband=1 if prec == H.MIXED else 0))
    T0 = np.concatenate([a["T0"] for a in atms])
    s.reset(T0)
    t_tune = time.perf_counter()
    s.autotune()
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    shapes = H.sweep_shapes(s.b, prec)
    s.reset(T0)
    for _ in range(warmup):
        s.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()  # torch creates the underlying events on their first record
    e1.record()
    torch.cuda.synchronize()
    sweep_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        H.set_sweep_events(e0, e1)
        s.step()
        e1.synchronize()
        sweep_ms += e0.elapsed_time(e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    H.set_sweep_events(None, None)
    running = int((s.status == H.ATM_RUNNING).sum().item())
    # the per-step event sync serialises the host; re-time without it
    s.reset(T0)
    for _ in range(warmup):
        s.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    torch.cuda.synchronize()
    wall_free = time.perf_counter() - t0
    units = int(sum(int(a["n"]) * len(a["lambda_c"]) * int(a["ng"]) for a in atms))
    rbytes = 4 if prec == H.MIXED else 8
    alg = sum(sweep_algorithmic_bytes(int(a["n"]), len(a["lambda_c"]), int(a["ng"]), rbytes) for a in atms)
    t_solve = time.perf_counter()
    conv, iters = s.solve(T0, max_iter=max_iter, check_every=10, graph=True)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t_solve
    out = {
        "units_per_s": units * steps / wall_free,
        "ms_per_step": wall_free / steps * 1e3,
        "sweep_ms": sweep_ms / steps,
        "sweep_gbs": alg / (sweep_ms / steps * 1e-3) / 1e9,
        "running_during_timing": running,
        "solve_s": t_solve,
        "converged": int(conv.sum()),
        "converged_atm_per_s": float(conv.sum()) / t_solve,
        "median_updates": float(np.median(iters)),
        "max_updates": int(iters.max()),
        "autotune_s": t_tune,
        "shapes": {str(k): list(v) for k, v in shapes.items()},
    }
    del s, b
    torch.cuda.empty_cache()
    return out


def batch_main(args):
    """Uneven 512-atmosphere batch (n ~ U{50..200}, 400-3000 strided bins)."""
    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    H.lib()
    atms, kt = W.batch_workload(n_atm=args.n_atm)
    atms.sort(key=lambda a: int(a["n"]))  # contiguous size classes
    res = {}
    for name, prec in (("mixed", H.MIXED), ("fp64", H.FP64)):
        if args.prec in ("both", name):
            res[name] = run_batch(prec, args.steps, args.warmup, atms, kt, args.max_iter)
            print(f"# {name}: {json.dumps(res[name])}", file=sys.stderr, flush=True)
    head = res.get("fp64") or res.get("mixed")
    line = {
        "metric": "layer*bin*g flux updates/s",
        "value": head["units_per_s"],
        "unit": "layer*bin*g/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if "fp64" in res else "f32", "data": "synthetic",
        "config": {"workload": f"uneven batch of {len(atms)} atmospheres: n ~ U{{50..200}} layers, "
                               "400-3000 strided bins of 0.3-30 um, 20 g, four float32 k-tables, 1+4 passes",
                   "n_atm": len(atms), "units_per_step": int(sum(int(a["n"]) * len(a["lambda_c"]) * 20
                                                                 for a in atms))},
        "results": res,
    }
    print(json.dumps(line))
    return 0


def chunk_main(args):
    """RE-iteration throughput on one production chunk: N parameter-described
    atmospheres of 200 layers x 3000 bins x 20 g, mixed precision with the
    dead band, started from the network (timed steps only, no solve)."""
    import numpy as np
    import torch

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import warmstart as WS
    from paper_1606_05474_amd import workloads as W

    atms, kt = W.learned_workload(5, args.n_atm, 0, n=200, nb=3000)
    b = H.Batch(atms)
    s = H.Solver(b, H.KTable(kt), prec=H.MIXED, opts=H.REOptions(deadband=1), bin_fluxes=False)
    x = np.stack([a["params"] for a in atms])
    s.reset(np.concatenate([a["T0"] for a in atms]))
    s.autotune()
    net = WS.load(args.weights)
    s.warm_reset(net, x, net.logP, m0=0.3)
    for _ in range(args.warmup):
        s.step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    e1.record()
    torch.cuda.synchronize()
    sweep_ms = 0.0
    for _ in range(args.steps):
        H.set_sweep_events(e0, e1)
        s.step()
        e1.synchronize()
        sweep_ms += e0.elapsed_time(e1)
    H.set_sweep_events(None, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    units = len(atms) * 200 * 3000 * 20
    alg = len(atms) * sweep_algorithmic_bytes(200, 3000, 20, 4)
    sweep_ms /= args.steps
    line = {"metric": "layer*bin*g flux updates/s", "value": units * args.steps / wall, "unit": "layer*bin*g/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
            "data": "synthetic",
            "config": {"workload": f"production chunk: {len(atms)} parameter-described atmospheres x 200 layers x "
                                   "3000 bins x 20 g, mixed precision, dead band, network start",
                       "shapes": {str(k): list(v) for k, v in H.sweep_shapes(s.b, H.MIXED).items()}},
            "roofline": {"bound": "hbm", "kernel": "sweep_kernel (flux sweep)",
                         "achieved": alg / (sweep_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": traffic_entry("chunk") if len(atms) == 128 else None,
                         "algorithmic_bytes_per_launch": alg, "avg_launch_ms": sweep_ms}}
    print(json.dumps(line))
    return 0


def layers_main(args):
    """The layer-resolution study of Sec. 3.3 on a synthetic stand-in: one
    physical atmosphere solved to radiative equilibrium on sublayered grids
    of 21, 51, 101 and 501 layers and on isothermal-layer grids of 51, 101,
    201 and 1001 layers (FP64, all 3000 bins, tolerance 1e-3 sigma T_int^4),
    then post-processed (80 scattering passes) to TOA emission spectra.
    Reported: each profile against the 501-layer sublayered one (linear in
    log P at the model's layer centres), each spectrum's deviation from that
    model's spectrum, the updates to converge and the time per update.  The
    step control counts any sign change within the 6-step window as an
    oscillation: with the strict-alternation reading a 400-layer model
    oscillates with period 4 and its step multipliers never shrink.

    The 1001-layer isothermal model does not converge: under the step control
    its deep layers run away from the isothermal start (the oracle does the
    same on a 30-bin stand-in, with either oscillation reading), as the paper
    reports no convergence with 1001 isothermal layers.  --layers-budget
    bounds its wall time, --layers-save writes its state when the budget ends
    first (layer temperatures, step multipliers, sign histories, updates), and
    --layers-resume continues from such a file (its scattering iteration
    restarts from zero fluxes; the temperature iteration continues)."""
    import time

    import numpy as np
    import torch

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    kt = W.table_ktab(2)
    KT = H.KTable(kt)
    lc, dl = W.bins(3000)
    groups = {"noniso": ("noniso", (21, 51, 101, 501)), "iso": ("iso", (51, 101, 201)),
              "iso_deep": ("iso", (1001,))}
    if args.layers_models:
        groups = {k: v for k, v in groups.items() if k in args.layers_models.split(",")}
    res = {}
    log = lambda *v: print("#", *v, file=sys.stderr, flush=True)  # noqa: E731
    for name, (layers, ns) in groups.items():
        atms = [W.resolution_atmosphere(6, n, lc, dl) for n in ns]
        b = H.Batch(atms)
        s = H.Solver(b, KT, prec=H.FP64, layers=layers, bin_fluxes=False, opts=H.REOptions(osc_any=1))
        s.reset(b.cat_layer([a["T0"] for a in atms]))
        resumed = 0
        if name == "iso_deep" and args.layers_resume and os.path.exists(args.layers_resume):
            with np.load(args.layers_resume) as d:
                s.T_c.copy_(torch.as_tensor(d["T_c"], device=s.T_c.device))
                s._reset_state()  # interface temperatures and the zero-flux start from the saved profile
                s.m.copy_(torch.as_tensor(d["m"], device=s.m.device))
                s.hist.copy_(torch.as_tensor(d["hist"], device=s.hist.device))
                s.iters.copy_(torch.as_tensor(d["iters"], device=s.iters.device))
                resumed = int(d["iters"].max())
            log(f"{name}: resumed at {resumed} updates")
        budget = args.layers_budget if name == "iso_deep" else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, block = resumed, 2000
        stopped = False
        conv, iters = np.zeros(len(ns), bool), s.iters.cpu().numpy()
        while done < args.max_iter:
            conv, iters, _ = s.run(block - 1, check_every=100, graph=True)
            done += block
            tmax = [round(float(t.max()), 1) for t in b.split_layer(s.T_c)]
            log(f"{name}: {done} updates, converged {conv.tolist()}, updates {iters.tolist()}, max T {tmax}, "
                f"{time.perf_counter() - t0:.1f} s")
            if conv.all():
                break
            if budget is not None and time.perf_counter() - t0 > budget:
                stopped = True
                break
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        if stopped and args.layers_save:
            np.savez(args.layers_save, T_c=s.T_c.cpu().numpy(), m=s.m.cpu().numpy(), hist=s.hist.cpu().numpy(),
                     iters=s.iters.cpu().numpy())
            log(f"{name}: state after {int(iters.max())} updates saved to {args.layers_save}")
        T = [t.cpu().numpy() for t in b.split_layer(s.T_c)]
        toa, _ = H.emission_spectrum(b, KT, s.T_c, n_scat=80, layers=layers)
        # one RE update's time on this batch with every member running
        # tolerance 0: no member can freeze while the update is timed
        s2 = H.Solver(b, KT, prec=H.FP64, layers=layers, bin_fluxes=False, opts=H.REOptions(osc_any=1, tol=0.0))
        s2.reset(s.T_c)
        for _ in range(3):
            s2.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            s2.step()
        e1.record()
        torch.cuda.synchronize()
        for k, n in enumerate(ns):
            res[f"{layers}{n}"] = {"P_c": atms[k]["P_c"], "T": T[k], "spec": toa[k].cpu().numpy(),
                                   "converged": bool(conv[k]), "updates": int(iters[k])}
        res[name] = {"seconds": sec, "resumed_at": resumed, "ms_per_update_all_running": e0.elapsed_time(e1) / 10}
    if "noniso501" not in res:
        print(json.dumps({"metric": "layer resolution study", "partial": True,
                          "models": {k: {"converged": v["converged"], "updates": v["updates"]}
                                     for k, v in res.items() if "T" in v},
                          "time": {k: v for k, v in res.items() if "T" not in v}}))
        return 0
    ref_m = res["noniso501"]
    lp_ref = np.log(ref_m["P_c"])[::-1]
    out = {}
    for key, m in res.items():
        if "T" not in m:
            continue
        T_ref = np.interp(np.log(m["P_c"]), lp_ref, ref_m["T"][::-1])
        dT = np.abs(m["T"] - T_ref)
        dev = np.abs(m["spec"] / ref_m["spec"] - 1.0)
        bright = ref_m["spec"] >= 1e-3 * ref_m["spec"].max()  # bins that carry the emitted flux
        k_max = int(np.argmax(dT))
        out[key] = {"converged": m["converged"], "updates": m["updates"], "T_range_K": [float(m["T"].min()),
                                                                                     float(m["T"].max())],
                    "max_abs_dT_vs_noniso501_K": float(dT.max()),
                    "max_abs_dT_at_bar": float(m["P_c"][k_max] / 1e6),
                    "median_abs_dT_vs_noniso501_K": float(np.median(dT)),
                    "max_abs_dT_between_1e-4_and_10_bar_K": float(dT[(m["P_c"] >= 1e2) & (m["P_c"] <= 1e7)].max()),
                    "spectrum_median_rel_dev": float(np.median(dev)),
                    "spectrum_max_rel_dev": float(dev.max()),
                    "spectrum_bins_above_1pct": float(np.mean(dev > 0.01)),
                    "spectrum_max_rel_dev_bright_bins": float(dev[bright].max()),
                    "spectrum_bright_bins_above_1pct": float(np.mean(dev[bright] > 0.01))}
    line = {"metric": "layer resolution study", "value": None, "unit": None, "n_gpus": 1, "dtype": "f64",
            "data": "synthetic", "higher_is_better": None,
            "config": {"workload": "one atmosphere (stellar 3026 K, irradiation 780 K, T_int 200 K, g 893 cm s^-2, "
                                   "synthetic 4-species tables, w0 and g0 per bin), 3000 bins x 20 g, P centres "
                                   "1e-6 .. 1e3 bar; RE to 1e-3 sigma T_int^4 in FP64 from 1000 K (any sign change in the "
                                   "6-step window shrinks the step), spectra with 80 "
                                   "scattering passes on each model's own grid; reference: 501 sublayered layers"},
            "models": out,
            "time": {k: res[k] for k in groups}}
    print(json.dumps(line))
    return 0


def modes_main(args):
    """The solver flavours on the single-atmosphere spectral workload (100
    layers x 3000 bins x 20 g): the sublayered two-stream solve, the same on
    isothermal layers (helios_flux_iso) and with H2 Rayleigh scattering
    (helios_flux_rayleigh), each in FP64 and mixed precision; per mode the
    RE-iteration rate and the sweep's time and rate of algorithmic bytes."""
    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    atm, kt = W.spectral_workload()
    n, nb, ng = int(atm["n"]), len(atm["lambda_c"]), int(atm["ng"])
    modes = {"two-stream": {}, "isothermal layers": {"layers": "iso"},
             "Rayleigh H2": {"rayleigh_mbar": 2.4 * 1.67262192369e-24}}
    out = {}
    for prec, pname in ((H.FP64, "fp64"), (H.MIXED, "mixed")):
        rb = 8 if prec == H.FP64 else 4
        for mode, kw in modes.items():
            r = run_gpu(prec, args.steps, args.warmup, atm, kt, **kw)
            if mode == "isothermal layers":
                alg = iso_algorithmic_bytes(n, nb, ng, rb)
            elif mode == "Rayleigh H2":
                alg = sweep_algorithmic_bytes(n, nb, ng, rb) - nb * 2 * n * 8  # no w0, g0
            else:
                alg = r["sweep_bytes"]
            gbs = alg / (r["sweep_ms"] * 1e-3) / 1e9
            out[f"{mode} {pname}"] = {"layer*bin*g/s": r["value"], "ms_per_iteration": r["ms_per_step"],
                                      "sweep_ms": r["sweep_ms"], "sweep_alg_GBs": gbs,
                                      "sweep_frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "running": r["status"] == H.ATM_RUNNING}
            print("#", mode, pname, json.dumps(out[f"{mode} {pname}"]), file=sys.stderr, flush=True)
    # post-processing (Sec. 2.6, Sec. 3.3): 1 + 80 passes, the paper's 101 isothermal layers and the
    # sublayered grid, FP64; a step is one such flux call plus its opacity mixing and RE update
    spectra = {}
    for layers, n_sp in (("iso", 101), ("noniso", 100)):
        atm_s, _ = W.spectral_workload(n=n_sp, ktab=kt)
        r = run_gpu(H.FP64, max(10, args.steps // 10), 3, atm_s, kt, n_scat=80, layers=layers)
        alg = (iso_algorithmic_bytes if layers == "iso" else sweep_algorithmic_bytes)(n_sp, nb, ng, 8)
        spectra[f"{n_sp} {'isothermal' if layers == 'iso' else 'sublayered'} layers, 81 passes, fp64"] = {
            "ms_per_spectrum_flux_call": r["sweep_ms"], "ms_per_step": r["ms_per_step"],
            "sweep_alg_GBs": alg / (r["sweep_ms"] * 1e-3) / 1e9}
        print("# spectrum", layers, json.dumps(spectra), file=sys.stderr, flush=True)
    line = {"metric": "layer*bin*g flux updates/s per solver mode", "value": None, "unit": "layer*bin*g/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": "one atmosphere, 100 layers x 3000 bins x 20 g, table opacities, 1 + 4 "
                                   "scattering passes; a step: opacity mixing, flux call, RE update"},
            "modes": out, "post_processing_spectrum": spectra}
    print(json.dumps(line))
    return 0


def exact_main(args):
    """The exact pure-absorption mode (Sec. 2.1.2) on the single-atmosphere
    spectral workload with w0 = 0: throughput of helios_flux_exact, and the
    two-stream solve (one pass, exact for w0 = 0) for D in {1.66, 1.8, 1.9, 2}
    against it (the diffusivity study of Sec. 2.1.1)."""
    import numpy as np
    import torch

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    kt = W.table_ktab(2)
    atm, _ = W.spectral_workload(ktab=kt)
    atm = dict(atm)
    atm["w0"] = np.zeros_like(atm["w0"])
    atm["g0"] = np.zeros_like(atm["g0"])
    b = H.Batch([atm])
    s = H.Solver(b, H.KTable(kt), prec=H.FP64)
    s.reset(atm["T0"])
    H.mix_opacity(b, s.kt, s.T_pt, s.kappa, H.FP64)
    F_dn = torch.zeros_like(s.F_up_g)
    bol_x = torch.zeros_like(s.F_bol)
    ub = torch.zeros_like(s.F_up_bin)
    db = torch.zeros_like(s.F_dn_bin)
    for _ in range(args.warmup):
        H.flux_exact(b, s.kappa, s.T_pt, s.F_up_g, F_dn, ub, db, bol_x, s.ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        H.flux_exact(b, s.kappa, s.T_pt, s.F_up_g, F_dn, ub, db, bol_x, s.ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    n, nb, ng = int(atm["n"]), len(atm["lambda_c"]), int(atm["ng"])
    npt = 2 * n + 1
    ex = bol_x.cpu().numpy().reshape(-1, 3)
    study = {}
    for D in (1.66, 1.8, 1.9, 2.0):
        up = torch.zeros_like(s.F_up_g)
        bol = torch.zeros_like(s.F_bol)
        H.flux(b, s.kappa, s.T_pt, up, ub, db, bol, s.ws, n_scat=0, D=D, prec=H.FP64)
        torch.cuda.synchronize()
        ts = bol.cpu().numpy().reshape(-1, 3)
        study[str(D)] = {"toa_up_rel": float(abs(ts[-1, 0] - ex[-1, 0]) / ex[-1, 0]),
                         "max_up_rel": float(np.max(np.abs(ts[:, 0] - ex[:, 0]) / ex[:, 0])),
                         "max_net_rel_gross": float(np.max(np.abs(ts[:, 2] - ex[:, 2]) / (ex[:, 0] + ex[:, 1])))}
    # bytes the exact kernel must move: opacities in, both per-g streams out,
    # Planck values, the Gauss partials
    alg = nb * (ng * npt * 8 + 2 * ng * npt * 8 + npt * 8 + 2 * npt * 8)
    line = {"metric": "layer*bin*g flux updates/s", "value": n * nb * ng / (ms * 1e-3), "unit": "layer*bin*g/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "exact pure-absorption mode: one atmosphere, 100 layers x 3000 bins x 20 g, "
                                   "w0 = 0, one sweep each way (a step: one helios_flux_exact call)"},
            "roofline": {"bound": "hbm", "kernel": "exact_kernel and the sums (whole call)",
                         "achieved": alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "algorithmic_bytes_per_launch": alg},
            "diffusivity_study_vs_exact": study}
    print(json.dumps(line))
    return 0


def production_main(args):
    """Converged atmospheres per second: the production form (a refilled
    device batch, network warm start with isothermal fallback, mixed
    precision) against the
    plain form (FP64, one atmosphere at a time, isothermal start) on the same
    parameter set (seed 5: 200 layers x 3000 bins x 20 g), same tolerance."""
    import numpy as np

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import warmstart as WS

    H.lib()
    if not os.path.exists(args.weights):
        print(f"no trained warm-start network at {args.weights}", file=sys.stderr)
        return 2
    net = WS.load(args.weights)
    log = lambda *v: print("#", *v, file=sys.stderr, flush=True)  # noqa: E731
    prod = WS.production(net, seed=5, count=args.n_atm, pool=args.chunk, max_iter=args.max_iter,
                         restart_after=args.restart_after or None, keep_T=args.plain_count, tol=args.prod_tol,
                         verify=not args.no_fp64_stage, log=log)
    base = WS.plain(seed=5, count=args.plain_count, max_iter=args.max_iter, keep_T=args.plain_count, log=log)
    base_g = WS.plain(seed=5, count=args.plain_count, max_iter=args.max_iter, graph=True, log=log)
    if args.save_profiles:  # the production form's converged profiles, for checks outside this run
        keep = [k for k in range(len(prod["T"])) if prod["conv_flags"][k]]
        np.savez(args.save_profiles, index=np.array(keep), T=np.stack([prod["T"][k] for k in keep]),
                 plain_T=np.stack([base["T"][k] for k in keep]), plain_converged=base["conv_flags"][keep])
    both = [k for k in range(args.plain_count) if base["conv_flags"][k] and prod["conv_flags"][k]]
    dT = [float(np.abs(prod["T"][k] - base["T"][k]).max()) for k in both]
    # the precision check (outside the timed regions): the production profiles
    # under the FP64 convergence test, and against the same schedule in FP64
    resid = WS.fp64_residual(prod["T"], seed=5)
    ok = [k for k in range(len(prod["T"])) if prod["conv_flags"][k]]
    c64, T64 = WS.same_start_fp64(net, seed=5, count=len(prod["T"]), max_iter=args.max_iter, tol=args.prod_tol)
    both64 = [k for k in ok if c64[k]]
    dT64 = [float(np.abs(prod["T"][k] - T64[k]).max()) for k in both64]
    log(f"FP64 test of the production profiles: max resid {max(resid[ok]):.3g} (tol 1e-3); "
        f"same-schedule FP64 max |dT| median {np.median(dT64):.3g} K")
    units = 200 * 3000 * 20
    line = {
        "metric": "converged atmospheres/s",
        "value": prod["converged_per_s"],
        "unit": "atmospheres/s",
        "n_gpus": 1, "steps": prod["converged"], "warmup": 0,  # a step here: one converged atmosphere
        "ms_per_step": prod["seconds"] / max(1, prod["converged"]) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.n_atm} parameter-described atmospheres (seed 5), 200 layers x 3000 bins x "
                               f"20 g, one device batch of {args.chunk} refilled as atmospheres finish, mixed "
                               f"precision with dead band to tolerance {args.prod_tol:g}, network warm start with "
                               f"isothermal fallback, isothermal restart after {args.restart_after} updates "
                               "(0: none), first step multipliers "
                               f"0.3, {args.max_iter} updates at most"
                               + ("" if args.no_fp64_stage else
                                  "; an atmosphere counts as converged once it passes the plain form's FP64 test "
                                  "at 1e-3 (it continues in FP64 until it does)")
                               + "; plain form: FP64, one atmosphere at a time, isothermal start, every layer "
                               "stepped, tolerance 1e-3 sigma T_int^4; the production profiles are also checked "
                               "with the scattering iteration settled (fp64_convergence_test_of_production_profiles)",
                   "n_atm": args.n_atm, "pool": args.chunk},
        "production": {"converged": prod["converged"], "count": prod["count"], "seconds": prod["seconds"],
                       "median_updates": float(np.median(prod["updates"])), "fallbacks": prod["fallbacks"],
                       "restarts": prod["restarts"], "fp64_polished": prod["polished"],
                       "fp64_stage": prod["fp64_stage"],
                       "input_generation_s_not_timed": prod["input_generation_s"],
                       "layer_bin_g_per_s": float(prod["updates"].sum()) * units / prod["seconds"]},
        "plain_fp64_one_at_a_time": {"converged": base["converged"], "count": base["count"],
                                     "seconds": base["seconds"], "converged_per_s": base["converged_per_s"],
                                     "median_updates": float(np.median(base["updates"]))},
        "speedup_converged_per_s": prod["converged_per_s"] / base["converged_per_s"]
        if base["converged_per_s"] > 0 else None,
        "plain_fp64_graph_replayed": {"converged": base_g["converged"], "count": base_g["count"],
                                      "seconds": base_g["seconds"], "converged_per_s": base_g["converged_per_s"],
                                      "median_updates": float(np.median(base_g["updates"])),
                                      "note": "the plain form with captured blocks of 10 updates replayed (host-"
                                              "launch cost removed; graph replay belongs to the batching extension)"},
        "speedup_vs_graph_replayed_plain": prod["converged_per_s"] / base_g["converged_per_s"]
        if base_g["converged_per_s"] > 0 else None,
        "fp64_convergence_test_of_production_profiles": {
            "atmospheres": len(ok), "max_resid": float(max(resid[ok])) if ok else None, "tol": 1e-3,
            "pass": int(sum(resid[k] < 1e-3 for k in ok))},
        "max_abs_dT_vs_fp64_same_schedule_K": {"atmospheres": len(both64),
                                               "max": max(dT64) if dT64 else None,
                                               "median": float(np.median(dT64)) if dT64 else None},
        "max_abs_dT_vs_plain_fp64_isothermal_start_K": {
            "atmospheres": len(both), "max": max(dT) if dT else None,
            "median": float(np.median(dT)) if dT else None,
            "note": "different starts reach different profiles where a layer's divergence hardly depends "
                    "on its temperature; both meet the same tolerance"},
    }
    print(json.dumps(line))
    return 0


def cpu_baseline(atm: dict, kt: dict, budget_s: float = 10.0):
    """The FP64 oracle as it stands, timed on the host: whole RE iterations
    (profile, opacity, flux with 1 + 4 passes, RE step) of the same
    atmosphere, repeated until about budget_s of wall time has passed."""
    import numpy as np

    import oracle as ref

    threads = max(1, min(16, os.cpu_count() or 1))
    n, nb, ng = int(atm["n"]), len(atm["lambda_c"]), int(atm["ng"])
    P = ref.grid(atm["P_c"])
    T_c = np.array(atm["T0"], np.float64)
    m = np.ones(n)
    hist = np.zeros(n, np.int32)
    F_up = np.zeros((nb, ng, 2 * n + 1))
    iters = 0
    t0 = time.perf_counter()
    while True:
        T = ref.profile(P, T_c)
        kap = ref.mix_opacity(kt, T, P, atm["vmr"], atm["bin_index"], ng)
        res = ref.flux(atm, kap, T, P, F_up, n_scat=4, n_threads=threads, want_dn=False)
        ref.radeq(atm, P, res["F_bol"], T_c, m, hist)
        iters += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    wall = time.perf_counter() - t0
    return {"value": n * nb * ng * iters / wall, "unit": "layer*bin*g/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} full RE iterations of the same 100-layer x 3000-bin x 20-g atmosphere "
                      f"({wall:.1f} s wall, OpenMP over columns)"}


def traffic_entry(prec_name: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current sweep source."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(prec_name)
    if not e or e.get("source_sha") != sweep_source_hash():
        return None
    return e.get("bytes_per_launch")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--extra-steps", type=int, default=50,
                    help="timed steps of each extra workload of the default line")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="default line: only the production chunk (and the CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="seconds of all-core oracle iterations in the CPU baseline")
    ap.add_argument("--prec", choices=["both", "fp64", "mixed"], default="both",
                    help="precisions to run (profiling runs pick one)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--workload", choices=["c5", "spectral", "batch", "chunk", "production", "exact", "layers",
                                           "modes"],
                    default="c5",
                    help="c5: one production chunk (the headline line, with the spectral atmosphere and the "
                         "uneven batch alongside); "
                         "spectral: one 100-layer x 3000-bin atmosphere in FP64 and mixed precision; "
                         "batch: the uneven 512-atmosphere batch, throughput and solve to convergence; "
                         "chunk: RE-iteration throughput of one production chunk; "
                         "production: converged atmospheres/s, batched + network + mixed against plain FP64; "
                         "exact: the exact pure-absorption mode and the diffusivity study; "
                         "layers: the layer-resolution study (sublayered against isothermal layers); "
                         "modes: the two-stream, isothermal-layer and Rayleigh solves side by side")
    ap.add_argument("--chunk", type=int, default=256, help="atmospheres per device batch (production pool)")
    ap.add_argument("--plain-count", type=int, default=64, help="atmospheres solved by the plain form")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1606_05474_amd", "data", "warmstart_mlp.npz"),
                    help="trained warm-start network (production)")
    ap.add_argument("--n-atm", type=int, default=None,
                    help="atmospheres (batch: 512 by default, production: 4096)")
    ap.add_argument("--save-profiles", default=None,
                    help="production: write the converged profiles of the first --plain-count atmospheres "
                         "(production and plain form) to this .npz")
    ap.add_argument("--restart-after", type=int, default=1000,
                    help="production: updates after which a network-started atmosphere restarts isothermally "
                         "(0: never)")
    ap.add_argument("--prod-tol", type=float, default=1e-3,
                    help="convergence tolerance of the production form's mixed-precision stage (the plain "
                         "form uses 1e-3 in FP64)")
    ap.add_argument("--no-fp64-stage", action="store_true",
                    help="production: count an atmosphere as converged on the mixed-precision test alone")
    ap.add_argument("--subset-atm", type=int, default=512,
                    help="default line: atmospheres of the production-form subset (0: skip it)")
    ap.add_argument("--subset-plain", type=int, default=16,
                    help="default line: atmospheres of the plain-form subset")
    ap.add_argument("--layers-models", default=None,
                    help="layers: comma-separated groups to run (noniso, iso, iso_deep; default all)")
    ap.add_argument("--layers-budget", type=float, default=None,
                    help="layers: seconds of updates for the 1001-layer isothermal model in this run")
    ap.add_argument("--layers-save", default=None,
                    help="layers: where to write the 1001-layer model's state when its budget ends first")
    ap.add_argument("--layers-resume", default=None,
                    help="layers: continue the 1001-layer model from a state written by --layers-save")
    ap.add_argument("--max-iter", type=int, default=None,
                    help="update cap (batch: 300; production: 1500 for both forms; layers: 1000000)")
    args = ap.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); the "
              "path shards by atmosphere (each GPU runs this library on its own atmospheres, with no "
              "communication until the profiles are gathered), so one GPU's rate is the figure",
              file=sys.stderr)
        return 2

    import torch

    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.copy_calibration:
        # a copy kernel of known size: 1 GiB read + 1 GiB written per launch,
        # each launch from its own source so no launch finds its input in a cache
        xs = [torch.full((1 << 28,), float(i), dtype=torch.float32, device="cuda") for i in range(5)]
        y = torch.empty_like(xs[0])
        for x in xs:
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * xs[0].numel() * 4, "launches": len(xs)}))
        return 0
    H.lib()  # fails loudly if the native library is missing
    if args.n_atm is None:
        args.n_atm = {"production": 4096, "chunk": 128, "c5": 256}.get(args.workload, 512)
    if args.max_iter is None:
        args.max_iter = {"production": 1500, "layers": 1000000}.get(args.workload, 300)
    if args.workload == "batch":
        return batch_main(args)
    if args.workload == "production":
        return production_main(args)
    if args.workload == "chunk":
        return chunk_main(args)
    if args.workload == "layers":
        return layers_main(args)
    if args.workload == "modes":
        return modes_main(args)
    if args.workload == "exact":
        return exact_main(args)
    if args.workload == "spectral":
        return spectral_main(args)
    return c5_main(args)


def c5_main(args):
    """The default line: the production chunk, with the spectral single
    atmosphere (FP64 and mixed) and the uneven batch as extra keys, and the
    oracle's rate on one of the chunk's atmospheres."""
    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    log = lambda *v: print("#", *v, file=sys.stderr, flush=True)  # noqa: E731
    if not os.path.exists(args.weights):
        print(f"no trained warm-start network at {args.weights}", file=sys.stderr)
        return 2
    chunk, cpu_atm, kt = c5_chunk(args)
    log("production chunk", json.dumps(chunk))
    extra = {}
    if args.extras:
        atm2, _ = W.spectral_workload(ktab=kt)
        for name, prec in (("fp64", H.FP64), ("mixed", H.MIXED)):
            r = run_gpu(prec, args.extra_steps, args.warmup, atm2, kt)
            units2 = int(atm2["n"]) * len(atm2["lambda_c"]) * int(atm2["ng"])
            extra[f"spectral_100x3000x20_{name}"] = {
                "value": r["value"], "unit": "layer*bin*g/s", "ms_per_step": r["ms_per_step"],
                "steps": args.extra_steps, "sweep_ms": r["sweep_ms"],
                "sweep_frac_of_hbm_peak": UNIT_BYTES[name] * units2 / (r["sweep_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "traffic": traffic_entry(name), "shape": r["shape"]}
            log("spectral", name, json.dumps(extra[f"spectral_100x3000x20_{name}"]))
        extra["uneven_batch_512_mixed"] = c3_batch(args.extra_steps, args.warmup)
        log("uneven batch", json.dumps(extra["uneven_batch_512_mixed"]))
    if args.extras and args.subset_atm > 0:
        key = f"converged_atmospheres_per_s_first_{args.subset_atm}"
        extra[key] = production_subset(args, log)
        log("production subset", json.dumps(extra[key]))
    line = {
        "metric": "layer*bin*g flux updates/s",
        "value": chunk["value"],
        "unit": "layer*bin*g/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chunk["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"production chunk: {args.n_atm} parameter-described atmospheres (seed 5) x 200 "
                               "layers x 3000 bins (0.3-30 um) x 20 g, four float32 k-tables 20 T x 20 log P, "
                               "mixed precision (FP32 sweeps, FP64 sums and update), 1+4 scattering passes, "
                               "network warm start, dead band; convergence test at tolerance 0 while timed",
                   "n_atm": args.n_atm, "n_layer": 200, "n_bin": 3000, "n_g": 20, "n_scat": 4,
                   "step": "mix_opacity + flux + radeq", "units_per_step": chunk["units_per_step"],
                   "shapes": chunk["shapes"]},
        "roofline": chunk["roofline"],
        "running_through_timed_steps": chunk["running"],
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_c5(cpu_atm, kt, args.cpu_budget)
    print(json.dumps(line))
    return 0


def production_subset(args, log):
    """Converged atmospheres per second on the first atmospheres of the
    production parameter set (seed 5, 200 layers x 3000 bins x 20 g): the
    production form (refilled device batch, network start, mixed precision,
    FP64 acceptance test) on args.subset_atm of them against the plain form
    (FP64, one at a time, isothermal start) on the first args.subset_plain,
    both to 1e-3 sigma T_int^4 and at most 1500 updates.  A short batch
    spends a larger share of its time in its slowest atmospheres than the
    4096-atmosphere run does, so this rate is below that run's."""
    import numpy as np

    from paper_1606_05474_amd import warmstart as WS

    net = WS.load(args.weights)
    prod = WS.production(net, seed=5, count=args.subset_atm, pool=args.chunk, max_iter=1500, restart_after=1000,
                         tol=1e-3, verify=True, log=log)
    base = WS.plain(seed=5, count=args.subset_plain, max_iter=1500, log=log)
    return {"production": {"count": prod["count"], "converged": prod["converged"], "seconds": prod["seconds"],
                           "converged_per_s": prod["converged_per_s"],
                           "median_updates": float(np.median(prod["updates"])), "fp64_stage": prod["fp64_stage"]},
            "plain_fp64_one_at_a_time": {"count": base["count"], "converged": base["converged"],
                                         "seconds": base["seconds"], "converged_per_s": base["converged_per_s"],
                                         "median_updates": float(np.median(base["updates"]))},
            "ratio": prod["converged_per_s"] / base["converged_per_s"] if base["converged_per_s"] > 0 else None}


def spectral_main(args):
    """The single-atmosphere spectral workload (100 layers x 3000 bins x 20 g)
    in FP64 and mixed precision."""
    from paper_1606_05474_amd import helios as H
    from paper_1606_05474_amd import workloads as W

    kt = W.table_ktab(2)
    atm, _ = W.spectral_workload(ktab=kt)
    fp64 = run_gpu(H.FP64, args.steps, args.warmup, atm, kt) if args.prec in ("both", "fp64") else None
    mixed = run_gpu(H.MIXED, args.steps, args.warmup, atm, kt) if args.prec in ("both", "mixed") else None
    if fp64 is None or mixed is None:
        print(json.dumps({"fp64": fp64, "mixed": mixed}))
        return 0
    n, nb, ng = int(atm["n"]), len(atm["lambda_c"]), int(atm["ng"])
    units = n * nb * ng
    gbs = UNIT_BYTES["fp64"] * units / (fp64["sweep_ms"] * 1e-3) / 1e9
    line = {
        "metric": "layer*bin*g flux updates/s",
        "value": fp64["value"],
        "unit": "layer*bin*g/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single atmosphere at full spectral size: 100 layers, 3000 bins 0.3-30 um, "
                               "20 g, four float32 k-tables 20 T x 20 log P, FP64, 1+4 scattering passes",
                   "n_layer": n, "n_bin": nb, "n_g": ng, "n_scat": 4, "step": "mix_opacity + flux + radeq"},
        "roofline": {"bound": "hbm", "kernel": "sweep_kernel (flux sweep)", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": traffic_entry("fp64"), "bytes_per_unit": UNIT_BYTES["fp64"],
                     "algorithmic_bytes_per_launch": UNIT_BYTES["fp64"] * units,
                     "avg_launch_ms": fp64["sweep_ms"], "kernel_own_bytes_per_launch": fp64["sweep_bytes"],
                     "sweep_shape": fp64["shape"]},
        "mixed_precision": {"value": mixed["value"], "ms_per_step": mixed["ms_per_step"],
                            "sweep_ms": mixed["sweep_ms"],
                            "frac": UNIT_BYTES["mixed"] * units / (mixed["sweep_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "traffic": traffic_entry("mixed"), "sweep_shape": mixed["shape"]},
    }
    # the FP64 solver keeps the paper's fluxes between iterations (its sweep
    # converts them as it reads and stores); the same steps with the per-g
    # state kept as deviations show what that conversion costs
    dev = run_gpu(H.FP64, args.steps, args.warmup, atm, kt, state="deviation")
    line["fp64_deviation_state"] = {"value": dev["value"], "ms_per_step": dev["ms_per_step"],
                                    "sweep_ms": dev["sweep_ms"], "sweep_shape": dev["shape"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(atm, kt, args.cpu_budget)
    print(json.dumps(line))
    return 0

if __name__ == "__main__":
    sys.exit(main())
