"""FP64 oracle reference for the production workload (test infrastructure).

Only this oracle and the seeded input generators are used; nothing here runs
on the GPU or reads a GPU result as an input.

    python -m oracle.c5_reference solve --count 8 --out REF.npz [--threads 6]
        Solves atmospheres 0..count-1 of the production parameter set (seed 5:
        200 layers x 3000 bins x 20 g) to radiative equilibrium with the
        paper's method as the oracle implements it (isothermal 1000 K start,
        zero-flux start of the scattering iteration and the previous fluxes as
        its warm start, 1 + 4 passes, the step control of Sec. 2.2.4,
        tolerance 1e-3 sigma T_int^4, at most 1500 updates).  Results are
        written after every atmosphere, so an interrupted run keeps what it
        finished; a rerun continues from the file.

    python -m oracle.c5_reference compare --ref REF.npz --prod PROD.npz
        Checks layer temperatures produced elsewhere (an npz with T [k][200]
        and the atmosphere index of each row) against the reference: the
        oracle's FP64 convergence measure at each given profile (opacities at
        that profile, the flux solve repeated from the isothermal flux until
        the scattering iteration has settled, then max_i |dF_i| / sigma
        T_int^4), and the largest temperature difference to the oracle's own
        converged profile, over all layers, between 1e-4 and 10 bar, and over
        the layers whose own temperature controls their flux divergence
        (finite differences of the oracle at its profile; the convergence test
        leaves the others weakly determined).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as ref  # noqa: E402
from paper_1606_05474_amd import workloads as W  # noqa: E402  (seeded inputs only)

SEED, N, NB = 5, 200, 3000
PAPER_OPTS = {"tol": 1e-3}


def atmospheres(count: int, start: int = 0):
    kt = W.table_ktab(2, nbt=NB)
    atms, _ = W.learned_workload(SEED, count, start, n=N, nb=NB, ktab=kt)
    return atms, kt


def solve_main(args):
    done = {}
    if os.path.exists(args.out):
        with np.load(args.out) as d:
            done = {int(k): (d["T"][i], bool(d["converged"][i]), int(d["iterations"][i]), float(d["resid"][i]),
                             float(d["seconds"][i])) for i, k in enumerate(d["index"])}
    atms, kt = atmospheres(args.count, 0)
    for k, atm in enumerate(atms):
        if k in done:
            continue
        t0 = time.perf_counter()
        sol = ref.solve(atm, kt, max_iter=args.max_iter, opts=PAPER_OPTS, n_threads=args.threads)
        sec = time.perf_counter() - t0
        done[k] = (sol["T_c"], bool(sol["converged"]), int(sol["iterations"]), float(sol["resid"][-1]), sec)
        idx = sorted(done)
        tmp = args.out + ".tmp.npz"
        np.savez(tmp, index=np.array(idx), T=np.stack([done[i][0] for i in idx]),
                 converged=np.array([done[i][1] for i in idx]), iterations=np.array([done[i][2] for i in idx]),
                 resid=np.array([done[i][3] for i in idx]), seconds=np.array([done[i][4] for i in idx]))
        os.replace(tmp, args.out)
        print(json.dumps({"atmosphere": k, "converged": bool(sol["converged"]), "iterations": int(sol["iterations"]),
                          "resid": float(sol["resid"][-1]), "seconds": round(sec, 1)}), flush=True)
    return 0


def fp64_measure(atm, kt, T_c, threads: int, calls: int):
    """max_i |dF_i| / sigma T_int^4 of the given layer temperatures with the
    scattering iteration settled (repeated flux calls at the fixed profile,
    starting from the isothermal flux)."""
    P = ref.grid(atm["P_c"])
    T_c = np.array(T_c, np.float64)
    T = ref.profile(P, T_c)
    kap = ref.mix_opacity(kt, T, P, atm["vmr"], atm["bin_index"], atm["ng"])
    F_up = ref.isothermal_start(atm, T)
    for _ in range(calls):
        r = ref.flux(atm, kap, T, P, F_up, n_threads=threads, want_dn=False)
    net = r["F_bol"][:, 2]
    dF = net[2::2] - net[:-1:2]
    return float(np.max(np.abs(dF)) / (ref.sigma_sb() * atm["T_int"] ** 4))


def well_conditioned(atm, kt, T_c, threads: int, calls: int, stride: int = 4, dT: float = 1.0):
    """Layers whose own temperature moves their net-flux divergence by at
    least 1% of d(sigma T^4)/dT, by finite differences of the oracle at the
    given profile: the scattering iteration is settled first, then layers
    i = j, j + stride, ... are raised by dT together (one flux call each from
    the settled state), so that the neighbours of a raised layer are not."""
    P = ref.grid(atm["P_c"])
    T_c = np.array(T_c, np.float64)
    n = T_c.size

    def divergence(Tc, F_up):
        T = ref.profile(P, Tc)
        kap = ref.mix_opacity(kt, T, P, atm["vmr"], atm["bin_index"], atm["ng"])
        net = ref.flux(atm, kap, T, P, F_up, n_threads=threads, want_dn=False)["F_bol"][:, 2]
        return net[2::2] - net[:-1:2]

    T = ref.profile(P, T_c)
    kap = ref.mix_opacity(kt, T, P, atm["vmr"], atm["bin_index"], atm["ng"])
    F_up = ref.isothermal_start(atm, T)
    for _ in range(calls):
        ref.flux(atm, kap, T, P, F_up, n_threads=threads, want_dn=False)
    base = divergence(T_c, F_up.copy())
    ok = np.zeros(n, bool)
    for j in range(stride):
        Tp = T_c.copy()
        Tp[j::stride] += dT
        d = np.abs(divergence(Tp, F_up.copy()) - base) / dT
        ok[j::stride] = d[j::stride] >= 0.01 * 4.0 * ref.sigma_sb() * T_c[j::stride] ** 3
    return ok


def compare_main(args):
    with np.load(args.ref) as d:
        ref_T = {int(k): d["T"][i] for i, k in enumerate(d["index"]) if bool(d["converged"][i])}
    with np.load(args.prod) as d:
        prod_idx = [int(k) for k in d["index"]]
        prod_T = d["T"]
    count = max(prod_idx) + 1
    atms, kt = atmospheres(count, 0)
    logp = np.log10(atms[0]["P_c"] / 1e6)
    band = (logp >= -4.0) & (logp <= 1.0)
    rows = []
    for i, k in enumerate(prod_idx):
        if args.with_ref_only and k not in ref_T:
            continue
        row = {"atmosphere": k, "fp64_resid": fp64_measure(atms[k], kt, prod_T[i], args.threads, args.calls)}
        if k in ref_T:
            dT = np.abs(prod_T[i] - ref_T[k])
            row["max_abs_dT_K"] = float(dT.max())
            row["max_abs_dT_1e-4_to_10_bar_K"] = float(dT[band].max())
            wc = well_conditioned(atms[k], kt, ref_T[k], args.threads, args.calls)
            row["well_conditioned_layers"] = int(wc.sum())
            row["max_abs_dT_well_conditioned_K"] = float(dT[wc].max()) if wc.any() else None
        rows.append(row)
        print(json.dumps(row), flush=True)
    res = np.array([r["fp64_resid"] for r in rows])
    with_ref = [r for r in rows if "max_abs_dT_K" in r]
    summary = {"profiles": len(rows), "fp64_resid_max": float(res.max()), "fp64_resid_median": float(np.median(res)),
               "pass_1e-3": int((res < 1e-3).sum()), "with_oracle_profile": len(with_ref)}
    if with_ref:
        a = np.array([r["max_abs_dT_K"] for r in with_ref])
        bnd = np.array([r["max_abs_dT_1e-4_to_10_bar_K"] for r in with_ref])
        wcm = np.array([r["max_abs_dT_well_conditioned_K"] for r in with_ref
                        if r["max_abs_dT_well_conditioned_K"] is not None])
        summary.update({"max_abs_dT_K_median": float(np.median(a)), "max_abs_dT_K_max": float(a.max()),
                        "band_max_abs_dT_K_median": float(np.median(bnd)), "band_max_abs_dT_K_max": float(bnd.max()),
                        "well_conditioned_max_abs_dT_K_median": float(np.median(wcm)) if wcm.size else None,
                        "well_conditioned_max_abs_dT_K_max": float(wcm.max()) if wcm.size else None})
    print(json.dumps({"summary": summary}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"rows": rows, "summary": summary}, f, indent=1)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("solve")
    s.add_argument("--count", type=int, default=64)
    s.add_argument("--out", required=True)
    s.add_argument("--threads", type=int, default=0)
    s.add_argument("--max-iter", type=int, default=1500)
    c = sub.add_parser("compare")
    c.add_argument("--ref", required=True)
    c.add_argument("--prod", required=True)
    c.add_argument("--threads", type=int, default=0)
    c.add_argument("--calls", type=int, default=20, help="flux calls (5 passes each) at each fixed profile")
    c.add_argument("--out", default=None)
    c.add_argument("--with-ref-only", action="store_true",
                   help="check only the profiles whose atmosphere has an oracle profile in --ref")
    args = ap.parse_args(argv)
    return solve_main(args) if args.cmd == "solve" else compare_main(args)


if __name__ == "__main__":
    sys.exit(main())
