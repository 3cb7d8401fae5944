"""The learned warm start: training data from the solver, training of the
network on the device, and its evaluation against the isothermal start.

    python -m paper_1606_05474_amd.warmstart generate --seed 4 --count 20000 --out data.npz
    python -m paper_1606_05474_amd.warmstart train --data data.npz --test test.npz --out mlp.npz
    python -m paper_1606_05474_amd.warmstart evaluate --weights mlp.npz --seed 40 --count 256

* generate: atmospheres described by six parameters (workloads.learned_workload:
  100 layers, 1000 strided bins, 20 g) are solved to radiative equilibrium
  from the isothermal 1000 K start by the batched solver, in chunks; the
  converged layer temperatures are the targets.
* train: the network (6 -> 256 x 3 -> 100, GELU) is fitted by the library's
  BF16 forward/backward kernels and its Adam step, mean squared error in
  normalised units; normalisation constants come from the training set.
* evaluate: the same atmospheres solved from the isothermal start and from
  the network's start (helios_warm_start, isothermal fallback, restart after
  a cap); reports updates to converge and wall time for both.

Everything that computes runs in libhelios; this module only moves arrays.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import helios as H
from . import workloads as W

DIMS = (6, 256, 256, 256, 100)
ATM_STOPPED = 2  # a status the production form gives atmospheres it stops (any but RUNNING is skipped)


def generate(seed: int, count: int, start: int = 0, chunk: int = 1024, prec: int = H.MIXED, max_iter: int = 400,
             n: int = 100, nb: int = 1000, log=print):
    """Converged profiles of atmospheres start..start+count-1 of a parameter
    set.  Returns dict(params [N][6] f32, T [N][n] f64, converged [N], updates
    [N], logP [n] log10 dyn cm^-2 of the layer centres, seconds)."""
    kt = W.table_ktab(2, nbt=3000)
    ktd = H.KTable(kt)
    P, T, conv, its = [], [], [], []
    t0 = time.perf_counter()
    logP = None
    for c0 in range(start, start + count, chunk):
        c = min(chunk, start + count - c0)
        atms, _ = W.learned_workload(seed, c, c0, n=n, nb=nb, ktab=kt)
        b = H.Batch(atms)
        s = H.Solver(b, ktd, prec=prec)
        T0 = np.concatenate([a["T0"] for a in atms])
        cv, it = s.solve(T0, max_iter=max_iter, check_every=10, graph=True)
        P.append(np.stack([a["params"] for a in atms]))
        T.append(s.T_c.cpu().numpy().reshape(c, n))
        conv.append(cv)
        its.append(it)
        logP = np.log10(atms[0]["P_c"])
        log(f"chunk {c0}..{c0 + c - 1}: {int(cv.sum())}/{c} converged, median updates {np.median(it):.0f}, "
            f"{time.perf_counter() - t0:.0f} s")
        del s, b
        torch.cuda.empty_cache()
    return {"params": np.concatenate(P), "T": np.concatenate(T), "converged": np.concatenate(conv),
            "updates": np.concatenate(its), "logP": logP, "seconds": time.perf_counter() - t0}


def train(data: dict, test: dict | None = None, epochs: int = 400, batch: int = 512, lr: float = 1e-3,
          seed: int = 0, log=print):
    """Fit the network to the converged profiles of `data` on the device.
    Returns (net, history)."""
    ok = data["converged"].astype(bool)
    x = data["params"][ok].astype(np.float32)
    T = data["T"][ok].astype(np.float32)
    net = H.MLP(DIMS)
    net.init(seed)
    net.set_norm(x.mean(0), 1.0 / (x.std(0) + 1e-6), T.mean(0), T.std(0) + 1e-3)
    net.logP = np.asarray(data["logP"], np.float64)
    xd = torch.as_tensor(x, device="cuda")
    Td = torch.as_tensor(T, device="cuda")
    N = x.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    steps_per_epoch = max(1, N // batch)
    total = epochs * steps_per_epoch
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(N, device="cuda", generator=g)
        for j in range(steps_per_epoch):
            idx = perm[j * batch:(j + 1) * batch]
            # cosine decay of the step size over the run
            rate = lr * 0.5 * (1.0 + np.cos(np.pi * k / total))
            net.train_step(xd[idx].contiguous(), Td[idx].contiguous(), lr=float(max(rate, lr * 0.01)))
            k += 1
        if ep % 50 == 0 or ep == epochs - 1:
            rec = {"epoch": ep, "train_rms_K": rms_error(net, x, T)}
            if test is not None:
                tok = test["converged"].astype(bool)
                rec["test_rms_K"] = rms_error(net, test["params"][tok], test["T"][tok])
            rec["seconds"] = time.perf_counter() - t0
            hist.append(rec)
            log(json.dumps(rec))
    return net, hist


def rms_error(net: H.MLP, x, T) -> float:
    """Root-mean-square temperature error of the network's profiles (K)."""
    pred = net.forward(np.asarray(x, np.float32)).cpu().numpy().astype(np.float64)
    return float(np.sqrt(np.mean((pred - np.asarray(T, np.float64)) ** 2)))


def save(net: H.MLP, path: str, meta: dict | None = None):
    np.savez(path, dims=np.array(net.dims), params=net.params.cpu().numpy(), logP=net.logP,
             meta=np.frombuffer(json.dumps(meta or {}).encode(), np.uint8),
             **{k: v.astype(np.float32) for k, v in net.norm().items()})


def load(path: str) -> H.MLP:
    d = np.load(path)  # plain arrays only
    net = H.MLP(tuple(int(v) for v in d["dims"]), training=False)
    net.set_norm(d["in_shift"], d["in_scale"], d["out_shift"], d["out_scale"])
    net.set_params(d["params"])
    net.logP = d["logP"].astype(np.float64)
    return net


def evaluate(net: H.MLP, seed: int = 40, count: int = 256, start: int = 0, prec: int = H.FP64, max_iter: int = 600,
             restart_after: int = 400, n: int = 100, nb: int = 1000, deadband: int = 0, m0: float = 1.0,
             log=print):
    """Updates to converge and wall time from the isothermal start and from
    the network's start, same atmospheres, same tolerance."""
    kt = W.table_ktab(2, nbt=3000)
    atms, _ = W.learned_workload(seed, count, start, n=n, nb=nb, ktab=kt)
    b = H.Batch(atms)
    s = H.Solver(b, H.KTable(kt), prec=prec, opts=H.REOptions(deadband=deadband))
    x = np.stack([a["params"] for a in atms])
    T0 = np.concatenate([a["T0"] for a in atms])
    out = {}
    for mode in ("isothermal", "network"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "isothermal":
            s.reset(T0)
            conv, it, rs = s.run(max_iter, 10, graph=True)
            fb = np.zeros(count, np.int32)
        else:
            fb = s.warm_reset(net, x, net.logP, m0=m0)
            conv, it, rs = s.run(max_iter, 10, graph=True, restart_after=restart_after)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[mode] = {"converged": int(conv.sum()), "count": count, "median_updates": float(np.median(it)),
                     "mean_updates": float(np.mean(it)), "median_updates_converged":
                         float(np.median(it[conv])) if conv.any() else None,
                     "fallbacks": int(fb.sum()), "restarts": int(rs.sum()), "seconds": wall,
                     "converged_per_s": float(conv.sum()) / wall}
        log(mode, json.dumps(out[mode]))
    return out


def production(net: H.MLP | None, seed: int = 5, count: int = 4096, start: int = 0, pool: int = 256,
               n: int = 200, nb: int = 3000, max_iter: int = 1500, restart_after: int = 1000,
               check_every: int = 10, deadband: int = 1, polish_iter: int = 0, m0: float = 0.3, keep_T: int = 0,
               tol: float = 1e-3, refill_min: int = 32, verify: bool = True, verify_tol: float = 1e-3,
               verify_iter: int = 300, log=print):
    """The production form: atmospheres start..start+count-1 of a parameter
    set solved by one device batch of up to `pool` atmospheres that is
    refilled as atmospheres finish (size-class sweeps, graph replay of blocks
    of `check_every` updates, finished atmospheres skipped):

    1. each atmosphere starts from the network (isothermal where its profile
       is unusable) or, with net=None, isothermally;
    2. it iterates in mixed precision (FP32 sweeps, FP64 sums and update),
       with the dead band on by default; a network-started atmosphere still
       running after `restart_after` updates restarts isothermally; one still
       running after `max_iter` updates leaves the batch unconverged (or, with
       polish_iter > 0, continues in FP64 from its full state for up to that
       many updates, all such atmospheres as one batch at the end);
    3. whenever `refill_min` atmospheres of the batch have finished, new
       atmospheres take their slots in place (Solver.refill: same sizes, so
       the batch's buffers and the captured graph stay valid), and the device
       keeps working on a full batch; once no new atmospheres are left and at
       most half of the batch runs, the running ones move into a smaller
       batch (Solver.subset carries their state);
    4. with `verify`, an atmosphere that passed the test in mixed precision
       continues in FP64 (temperatures, step control and warm start carried
       over) until it passes the plain form's FP64 test at `verify_tol` (at
       most `verify_iter` more updates, usually none): only then does it
       count as converged, so both forms meet the same test in FP64.

    The mixed stage's test is the plain form's with tolerance `tol`.  The
    timed region starts after the one-time shape tuning
    and excludes the host-side generation of the inputs; it includes the
    device batches' construction, the network inference and every update.
    Returns totals and the converged profiles of the first `keep_T`
    atmospheres."""
    kt = W.table_ktab(2, nbt=3000)
    ktd = H.KTable(kt)
    opts = H.REOptions(deadband=deadband, tol=tol)
    conv = np.zeros(count, bool)
    its = np.zeros(count, np.int64)
    restarted = np.zeros(count, bool)
    T_out = [None] * count
    gen = [0.0]
    fallbacks = [0]
    refills = [0]

    def make(k0, k):
        tg = time.perf_counter()
        atms, _ = W.learned_workload(seed, k, start + k0, n=n, nb=nb, ktab=kt)
        gen[0] += time.perf_counter() - tg
        sv = H.Solver(H.Batch(atms), ktd, prec=H.MIXED, opts=opts, bin_fluxes=False)
        if net is not None:
            fb = sv.warm_reset(net, np.stack([a["params"] for a in atms]), net.logP, m0=m0)
        else:
            sv.reset(np.concatenate([a["T0"] for a in atms]))
            fb = np.zeros(k, np.int32)
        fallbacks[0] += int(fb.sum())
        return sv

    vstats = {"checked": 0, "passed_at_once": 0, "updates": 0, "failed": 0}

    def fp64_verify(sv, ids, idx):
        """The FP64 stage: atmospheres idx of sv continue in FP64 until the
        plain form's test passes there."""
        idx = np.asarray(idx, np.int64)
        if idx.size == 0:
            return
        s64 = sv.subset(idx, prec=H.FP64)
        s64.opts = H.REOptions(deadband=deadband, tol=verify_tol)
        it0 = s64.iters.cpu().numpy().copy()
        c, it, _, T, _, _ = _run_compacting(s64, verify_iter, 2, None)
        for k, a in enumerate(ids[idx]):
            a = int(a)
            conv[a], its[a], T_out[a] = bool(c[k]), int(it[k]), T[k]
        extra = it - it0
        vstats["checked"] += int(idx.size)
        vstats["passed_at_once"] += int(np.sum(c & (extra == 0)))
        vstats["updates"] += int(extra.sum())
        vstats["failed"] += int(np.sum(~c))
        del s64

    def harvest(sv, ids, which, over):
        st = sv.status.cpu().numpy()
        it = sv.iters.cpu().numpy()
        Tc = sv.T_c.cpu().numpy()
        ok = [k for k in which if st[k] == H.ATM_CONVERGED and not over[k]]
        for k in which:
            a = int(ids[k])
            conv[a] = k in ok and not verify
            its[a] = it[k]
            T_out[a] = Tc[int(sv.b.lay_off[k]):int(sv.b.lay_off[k + 1])].copy()
        if verify:
            fp64_verify(sv, ids, ok)

    first = min(pool, count)
    s = make(0, first)
    s.autotune()  # one-time shape tuning for this process, outside the timed region
    del s
    log(f"production: sweep shapes tuned, solving {count} atmospheres")
    gen[0] = 0.0
    fallbacks[0] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = make(0, first)
    ids = np.arange(first)  # atmosphere held by each slot, -1 once a slot is empty for good
    nxt = first
    rs_cur = np.zeros(first, bool)
    over_parts = []  # (solver, indices, original ids) of atmospheres that reached max_iter
    s.capture(check_every)
    while True:
        s.replay()
        st = s.status.cpu().numpy()
        it = s.iters.cpu().numpy()
        if restart_after is not None and s._warm is not None:
            late = np.where(s._warm & ~rs_cur & (st == H.ATM_RUNNING) & (it >= restart_after) & (ids >= 0))[0]
            if late.size:
                s.restart(late, s._T_iso)
                rs_cur[late] = True
                restarted[ids[late]] = True
                st = s.status.cpu().numpy()
        over = (st == H.ATM_RUNNING) & (it >= max_iter) & (ids >= 0)
        if over.any():  # stop them now (any status but RUNNING is skipped); harvested as unconverged
            s.status[torch.as_tensor(np.where(over)[0], device=s.b.device)] = ATM_STOPPED
        running = (st == H.ATM_RUNNING) & ~over & (ids >= 0)
        done = (ids >= 0) & ~running
        nrun, ndone = int(running.sum()), int(done.sum())
        left = count - nxt
        if nrun == 0 and left == 0:
            fs = np.where(done)[0]
            harvest(s, ids, fs, over)
            if over.any() and polish_iter > 0:
                over_parts.append((s, np.where(over)[0], ids[over]))
            break
        if left > 0 and ndone >= min(refill_min, left):
            # finished atmospheres leave their slots; new ones take them in place,
            # so the batch, its buffers and the captured graph stay as they are
            fs = np.where(done)[0]
            harvest(s, ids, fs, over)
            if over.any() and polish_iter > 0:
                over_parts.append((s.subset(np.where(over)[0], prec=H.FP64), None, ids[over]))
            k_new = min(fs.size, left)
            slots = fs[:k_new]
            tg = time.perf_counter()
            atms, _ = W.learned_workload(seed, k_new, start + nxt, n=n, nb=nb, ktab=kt)
            gen[0] += time.perf_counter() - tg
            if net is not None:
                fb = s.refill(slots, atms, net=net, x=np.stack([a["params"] for a in atms]), m0=m0)
                fallbacks[0] += int(fb.sum())
            else:
                s.refill(slots, atms)
            ids[slots] = np.arange(nxt, nxt + k_new)
            rs_cur[slots] = False
            empty = fs[k_new:]
            if empty.size:
                s.status[torch.as_tensor(empty, device=s.b.device)] = ATM_STOPPED
                ids[empty] = -1
            nxt += k_new
            refills[0] += 1
            if refills[0] % 16 == 0:  # progress: finished so far, elapsed
                log(f"production: {nxt - nrun - k_new} of {count} finished or stopped, "
                    f"{time.perf_counter() - t0 - gen[0]:.0f} s")
        elif left == 0 and nrun <= int((ids >= 0).sum()) // 2 and s.b.n_atm > 8:
            # the last atmospheres: harvest the finished ones and move the running
            # ones into a smaller batch, so later launches cover live atmospheres only
            fs = np.where(done)[0]
            harvest(s, ids, fs, over)
            if over.any() and polish_iter > 0:
                over_parts.append((s.subset(np.where(over)[0], prec=H.FP64), None, ids[over]))
            keep = np.where(running)[0]
            s2 = s.subset(keep)
            ids, rs_cur = ids[keep], rs_cur[keep]
            del s
            s = s2
            s.capture(check_every)
    polished = 0
    if over_parts:
        srcs = [(sv if idx is None else sv.subset(idx, prec=H.FP64)) for sv, idx, _ in over_parts]
        oid = np.concatenate([o for _, _, o in over_parts])
        s3 = H.Solver.concat([(sv, np.arange(sv.b.n_atm)) for sv in srcs], prec=H.FP64)
        del srcs, over_parts
        c3, it3, _, T3, _, _ = _run_compacting(s3, polish_iter, check_every, None)
        for k, a in enumerate(oid):
            conv[a], its[a], T_out[a] = c3[k], it3[k], T3[k]
        polished = int(oid.size)
        del s3
    del s
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0 - gen[0]
    torch.cuda.empty_cache()
    out = {"count": count, "converged": int(conv.sum()), "seconds": seconds, "updates": its,
           "fallbacks": fallbacks[0], "restarts": int(restarted.sum()), "polished": polished,
           "fp64_stage": dict(vstats) if verify else None,
           "T": T_out[:keep_T], "conv_flags": conv, "converged_per_s": float(conv.sum()) / seconds,
           "input_generation_s": gen[0], "refills": refills[0]}
    log(f"production: {out['converged']}/{count} converged in {seconds:.1f} s (inputs generated in "
        f"{gen[0]:.1f} s, not timed), median updates {np.median(its):.0f}, fallbacks {fallbacks[0]}, "
        f"restarts {out['restarts']}, FP64 polish {polished}, batch refills {refills[0]}, FP64 stage {vstats}")
    return out


def _run_compacting(s: H.Solver, max_iter: int, check_every: int, restart_after: int | None,
                    min_live: int = 8):
    """Iterate a batch in captured blocks of `check_every` updates; whenever
    at most half of the atmospheres of the current batch are still running
    (and more than `min_live`), move the running ones into a smaller batch
    (Solver.subset) so that later launches cover live atmospheres only.
    Returns (converged, updates, restarted, final layer temperatures, the
    last solver and the original index of each of its atmospheres)."""
    n0 = s.b.n_atm
    conv = np.zeros(n0, bool)
    its = np.zeros(n0, np.int64)
    restarted = np.zeros(n0, bool)
    T_out = [None] * n0
    live = np.arange(n0)  # original index of each atmosphere of the current batch
    rs_cur = np.zeros(n0, bool)

    def harvest(sv, which):
        st = sv.status.cpu().numpy()
        it = sv.iters.cpu().numpy()
        Tc = sv.T_c.cpu().numpy()
        for k in which:
            a = int(live[k])
            conv[a] = st[k] == H.ATM_CONVERGED
            its[a] = it[k]
            T_out[a] = Tc[int(sv.b.lay_off[k]):int(sv.b.lay_off[k + 1])].copy()

    done = 0
    s.capture(check_every)
    while done < max_iter:
        s.replay()
        done += check_every
        st = s.status.cpu().numpy()
        if restart_after is not None and s._warm is not None:
            it = s.iters.cpu().numpy()
            late = np.where(s._warm & ~rs_cur & (st == H.ATM_RUNNING) & (it >= restart_after))[0]
            if late.size:
                s.restart(late, s._T_iso)
                rs_cur[late] = True
                restarted[live[late]] = True
                st = s.status.cpu().numpy()
        running = st == H.ATM_RUNNING
        if not running.any():
            break
        if running.sum() <= len(live) // 2 and len(live) > min_live:
            harvest(s, np.where(~running)[0])
            keep = np.where(running)[0]
            s = s.subset(keep)
            live = live[keep]
            rs_cur = rs_cur[keep]
            s.capture(check_every)
    harvest(s, range(len(live)))
    return conv, its, restarted, T_out, s, live


def plain(seed: int = 5, count: int = 64, start: int = 0, n: int = 200, nb: int = 3000, max_iter: int = 400,
          keep_T: int = 0, graph: bool = False, log=print):
    """The plain form: the same atmospheres one at a time, FP64, isothermal
    start, an eager iteration loop (timed per atmosphere with its inputs
    resident on the device).  graph=True replays captured blocks of 10
    updates instead (no host launch cost per kernel; a sensitivity check,
    since graph replay belongs to the batching extension)."""
    kt = W.table_ktab(2, nbt=3000)
    ktd = H.KTable(kt)
    atms, _ = W.learned_workload(seed, count, start, n=n, nb=nb, ktab=kt)
    out = {"count": count, "converged": 0, "seconds": 0.0, "updates": [], "T": [], "conv_flags": []}
    for k, atm in enumerate(atms):
        b = H.Batch([atm])
        s = H.Solver(b, ktd, prec=H.FP64)
        if k == 0:
            s.reset(atm["T0"])
            s.autotune()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.reset(atm["T0"])
        conv, it, _ = s.run(max_iter, 10, graph=graph)
        torch.cuda.synchronize()
        out["seconds"] += time.perf_counter() - t0
        out["converged"] += int(conv[0])
        out["updates"].append(int(it[0]))
        out["conv_flags"].append(bool(conv[0]))
        if k < keep_T:
            out["T"].append(s.T_c.cpu().numpy())
        del s, b
    out["updates"] = np.array(out["updates"])
    out["conv_flags"] = np.array(out["conv_flags"])
    out["converged_per_s"] = out["converged"] / out["seconds"]
    log(f"plain{' (graph replay)' if graph else ''}: {out['converged']}/{count} converged in {out['seconds']:.1f} s, "
        f"median updates {np.median(out['updates']):.0f}")
    return out


def fp64_residual(T_list, seed: int = 5, start: int = 0, n: int = 200, nb: int = 3000, n_flux: int = 40,
                  tol: float = 1e-3):
    """Convergence measure of given layer temperatures under the FP64 path:
    the opacities are mixed once, the flux solve is repeated n_flux times on
    the fixed profile (its scattering passes start from the previous call's
    upward fluxes, so they converge), then the RE step's test is evaluated.
    Returns max_i |dF_i| / sigma T_int^4 per atmosphere (numpy)."""
    kt = W.table_ktab(2, nbt=3000)
    ktd = H.KTable(kt)
    atms, _ = W.learned_workload(seed, len(T_list), start, n=n, nb=nb, ktab=kt)
    b = H.Batch(atms)
    s = H.Solver(b, ktd, prec=H.FP64, opts=H.REOptions(tol=tol))
    s.reset(np.concatenate([np.asarray(T, np.float64) for T in T_list]))
    H.mix_opacity(b, ktd, s.T_pt, s.kappa, H.FP64)
    for _ in range(n_flux):
        H.flux(b, s.kappa, s.T_pt, s.F_up_g, s.F_up_bin, s.F_dn_bin, s.F_bol, s.ws, n_scat=s.n_scat, D=s.D,
               prec=H.FP64)
    H.radeq(b, s.F_bol, s.T_c, s.T_pt, s.m, s.hist, s.status, s.resid, s.opts, iters=s.iters)
    return s.resid.cpu().numpy().copy()


def same_start_fp64(net: H.MLP, seed: int = 5, count: int = 64, start: int = 0, n: int = 200, nb: int = 3000,
                    max_iter: int = 1500, restart_after: int = 1000, deadband: int = 1, m0: float = 0.3,
                    tol: float = 7e-4):
    """The production schedule (network start, dead band, compaction,
    isothermal restart of stragglers) entirely in FP64: the reference that
    isolates the effect of the reduced precision.  Returns (converged flags,
    layer temperatures per atmosphere)."""
    kt = W.table_ktab(2, nbt=3000)
    ktd = H.KTable(kt)
    atms, _ = W.learned_workload(seed, count, start, n=n, nb=nb, ktab=kt)
    b = H.Batch(atms)
    s = H.Solver(b, ktd, prec=H.FP64, opts=H.REOptions(deadband=deadband, tol=tol))
    x = np.stack([a["params"] for a in atms])
    s.warm_reset(net, x, net.logP, m0=m0)
    conv, _, _, T_list, _, _ = _run_compacting(s, max_iter, 10, restart_after)
    return conv, T_list


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--seed", type=int, default=4)
    g.add_argument("--count", type=int, default=20000)
    g.add_argument("--start", type=int, default=0)
    g.add_argument("--chunk", type=int, default=1024)
    g.add_argument("--prec", choices=["fp64", "mixed"], default="mixed")
    g.add_argument("--max-iter", type=int, default=400)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, nargs="+")
    t.add_argument("--test")
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--batch", type=int, default=512)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True)
    e.add_argument("--seed", type=int, default=40)
    e.add_argument("--count", type=int, default=256)
    e.add_argument("--prec", choices=["fp64", "mixed"], default="fp64")
    e.add_argument("--restart-after", type=int, default=400)
    e.add_argument("--max-iter", type=int, default=600)
    e.add_argument("--deadband", type=int, default=0)
    e.add_argument("--m0", type=float, default=0.3)
    e.add_argument("--n", type=int, default=100)
    e.add_argument("--nb", type=int, default=1000)
    a = ap.parse_args(argv)
    H.lib()
    log = lambda *v: print(*v, flush=True)  # noqa: E731
    if a.cmd == "generate":
        d = generate(a.seed, a.count, a.start, a.chunk, H.MIXED if a.prec == "mixed" else H.FP64, a.max_iter, log=log)
        np.savez(a.out, **d)
    elif a.cmd == "train":
        parts = [dict(np.load(p)) for p in a.data]
        data = {k: np.concatenate([p[k] for p in parts]) for k in ("params", "T", "converged", "updates")}
        data["logP"] = parts[0]["logP"]
        test = dict(np.load(a.test)) if a.test else None
        net, hist = train(data, test, a.epochs, a.batch, a.lr, log=log)
        save(net, a.out, {"history": hist, "n_train": int(data["converged"].sum())})
    else:
        net = load(a.weights)
        evaluate(net, a.seed, a.count, prec=H.MIXED if a.prec == "mixed" else H.FP64, max_iter=a.max_iter,
                 restart_after=a.restart_after, deadband=a.deadband, m0=a.m0, n=a.n, nb=a.nb, log=log)
    return 0


if __name__ == "__main__":
    sys.exit(main())
