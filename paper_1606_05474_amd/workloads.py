"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *draws inputs*; it holds none of the method's arithmetic (no
grid interfaces, no Planck function, no quadrature, no opacity mixing).  Both
the GPU path and the CPU oracle consume the arrays it returns.

Every generator uses numpy's PCG64 (``default_rng``) with a documented seed
and draw order, so a given call always returns the same arrays.

Units are cgs: pressure in dyn cm^-2 (1 bar = 1e6), wavelength in cm,
gravity in cm s^-2, opacities in cm^2 g^-1, masses in proton masses.

Workloads (sizes from the paper's default set-up: 1 microbar - 1 kbar, 20
Gauss points, 0.3-30 micron bins log-spaced, blackbody star):
  plain     n=50 layers, 30 bins, power-law k(g), w0 ~ U(0,0.5), g0 = 0
  spectral  n=100 layers, 3000 bins, four species k-tables on a
            20 T x 20 log P grid, w0 ~ U(0,0.9), g0 ~ U(0,0.5)
  batch     uneven atmospheres (n in 50..200, bins 400..3000 as strided
            subsets of the 3000-bin tables), per-atmosphere irradiation,
            internal temperature and gravity
  learned   atmospheres described by six parameters (irradiation and
            internal temperature, gravity, metallicity, C/O, opacity scale)
            with a smooth stand-in chemistry, for the warm-start network
            (100 layers x 1000 bins) and the production sweep (200 layers x
            3000 bins)
"""
from __future__ import annotations

import numpy as np

BAR = 1.0e6
MICRON = 1.0e-4
SPECIES = ("CO", "CO2", "H2O", "CH4")
SPECIES_MASS = np.array([28.0, 44.0, 18.0, 16.0])  # proton masses
MMW = 2.4  # mean molecular mass of the H2-dominated gas, proton masses
N_G = 20


# --------------------------------------------------------------- axes
def pressure_centres(n: int, top_bar: float = 1e-6, bottom_bar: float = 1e3) -> np.ndarray:
    """Layer-centre pressures, bottom -> top, log-uniform (dyn cm^-2)."""
    lg = np.linspace(np.log10(bottom_bar), np.log10(top_bar), n)
    return (10.0 ** lg) * BAR


def point_log10p_bar(n: int, top_bar: float = 1e-6, bottom_bar: float = 1e3) -> np.ndarray:
    """2n+1 log-uniform sample positions (log10 bar) used to draw per-point
    inputs (mixing ratios): the n centres plus positions halfway between them
    and half a step beyond the two ends.  Input construction only."""
    a, b = np.log10(bottom_bar), np.log10(top_bar)
    step = (b - a) / (n - 1)
    return a - 0.5 * step + 0.5 * step * np.arange(2 * n + 1)


def bins(nb: int, lo_um: float = 0.3, hi_um: float = 30.0):
    """nb bins log-spaced between lo and hi: centres (geometric) and widths, cm."""
    e = lo_um * (hi_um / lo_um) ** (np.arange(nb + 1) / nb) * MICRON
    return np.sqrt(e[:-1] * e[1:]), np.diff(e)


def subset_bins(lambda_c_full: np.ndarray, nb: int):
    """Strided subset of a finer bin set: indices round(linspace(0, N-1, nb)),
    the subset's centres, and widths recomputed from log-midpoints."""
    N = lambda_c_full.size
    idx = np.round(np.linspace(0, N - 1, nb)).astype(np.int32)
    c = lambda_c_full[idx]
    if nb == 1:
        return idx, c, np.array([lambda_c_full[-1] - lambda_c_full[0]])
    inner = np.sqrt(c[:-1] * c[1:])
    lo = c[0] * np.sqrt(c[0] / c[1])
    hi = c[-1] * np.sqrt(c[-1] / c[-2])
    edges = np.concatenate([[lo], inner, [hi]])
    return idx, c, np.diff(edges)


# ---------------------------------------------------------- k coefficients
def sorted_log_k(rng: np.random.Generator, nb: int, ng: int = N_G,
                 mu: float = -2.0, sd: float = 1.5) -> np.ndarray:
    """log10 k per (bin, g): N(mu, sd) draws sorted ascending along g, so
    k(g) is monotone in g as a k-distribution is."""
    return np.sort(rng.normal(mu, sd, size=(nb, ng)), axis=1)


def powerlaw_ktab(seed: int = 1, nb: int = 30, ng: int = N_G) -> dict:
    """Single-absorber power law k = 10^s (P/1 bar)^0.5 (T/1000 K), s sorted
    N(-2, 1.5) per bin.  Mixing ratio 1 at mass MMW, so kappa = k."""
    rng = np.random.default_rng([seed, 100])
    s = sorted_log_k(rng, nb, ng)
    return {"mode": "powerlaw", "k0": (10.0 ** s)[None].copy(), "p_exp": 0.5, "t_exp": 1.0,
            "P_ref": 1.0 * BAR, "T_ref": 1000.0, "mass": np.array([MMW]), "mmw": MMW}


def table_ktab(seed: int = 2, nbt: int = 3000, ng: int = N_G, nT: int = 20, nP: int = 20,
               T_lo: float = 100.0, T_hi: float = 3000.0, lP_lo_bar: float = -6.0,
               lP_hi_bar: float = 3.0) -> dict:
    """Four float32 k-tables [species][T][log P][bin][g] on a uniform
    T x log10 P grid.  Species j draws s_j = sorted N(-2, 1.5) from the
    sub-seed (seed, j) and is tabulated as 10^s_j (P/1 bar)^0.5 (T/1000 K).
    The log10 P axis is stored in cgs units (log10 dyn cm^-2)."""
    T_ax = np.linspace(T_lo, T_hi, nT)
    lP_ax = np.linspace(lP_lo_bar, lP_hi_bar, nP)
    k = np.empty((len(SPECIES), nT, nP, nbt, ng), dtype=np.float32)
    for j in range(len(SPECIES)):
        rng = np.random.default_rng([seed, j])
        base = (10.0 ** sorted_log_k(rng, nbt, ng)).astype(np.float64)
        fac = np.outer(T_ax / 1000.0, (10.0 ** lP_ax) ** 0.5)  # [T][P]
        k[j] = (fac[:, :, None, None] * base[None, None]).astype(np.float32)
    return {"mode": "table", "k": k, "T_min": float(T_ax[0]), "T_step": float(T_ax[1] - T_ax[0]),
            "logP_min": float(lP_ax[0] + 6.0), "logP_step": float(lP_ax[1] - lP_ax[0]),
            "mass": SPECIES_MASS.copy(), "mmw": MMW}


def smooth_vmr(rng: np.random.Generator, lp_bar: np.ndarray, nsp: int = 4) -> np.ndarray:
    """Equilibrium-like volume mixing ratios per species at the given log10 P
    (bar): X = clip(10^(a + b tanh((logP - c)/w)), 1e-8, 1e-3) with a, b, c, w
    drawn in that order per species."""
    out = np.empty((nsp, lp_bar.size))
    for j in range(nsp):
        a = rng.uniform(-5.5, -3.5)
        b = rng.uniform(-1.5, 1.5)
        c = rng.uniform(-3.0, 1.0)
        w = rng.uniform(0.5, 2.0)
        out[j] = np.clip(10.0 ** (a + b * np.tanh((lp_bar - c) / w)), 1e-8, 1e-3)
    return out


# ------------------------------------------------------------- workloads
def plain_workload(seed: int = 1, n: int = 50, nb: int = 30, ng: int = N_G):
    """The plain FP64 single-atmosphere case.  Returns (atm, ktab)."""
    rng = np.random.default_rng([seed, 0])
    lc, dl = bins(nb)
    atm = {
        "n": n, "ng": ng, "P_c": pressure_centres(n), "grav": 1000.0,
        "T_star": 5000.0, "T_irr": 1500.0, "T_int": 200.0, "mmw": MMW,
        "lambda_c": lc, "dlambda": dl, "bin_index": np.arange(nb, dtype=np.int32),
        "w0": rng.uniform(0.0, 0.5, size=(nb, n)), "g0": np.zeros((nb, n)),
        "vmr": np.ones((1, 2 * n + 1)), "T0": np.full(n, 1000.0),
    }
    return atm, powerlaw_ktab(seed, nb, ng)


def spectral_atmosphere(rng: np.random.Generator, n: int, lambda_c_full: np.ndarray,
                        dlambda_full: np.ndarray, nb: int, ng: int = N_G, T_irr: float = 1500.0,
                        T_int: float = 200.0, grav: float = 1000.0, vmr_scale: float = 1.0,
                        w0_max: float = 0.9, g0_max: float = 0.5) -> dict:
    """One table-opacity atmosphere drawn from rng (draw order: bins are
    deterministic; then mixing-ratio parameters, then w0, then g0)."""
    if nb == lambda_c_full.size:
        idx, lc, dl = np.arange(nb, dtype=np.int32), lambda_c_full.copy(), dlambda_full.copy()
    else:
        idx, lc, dl = subset_bins(lambda_c_full, nb)
    vmr = smooth_vmr(rng, point_log10p_bar(n)) * vmr_scale
    w0 = rng.uniform(0.0, w0_max, size=(nb, n))
    g0 = rng.uniform(0.0, g0_max, size=(nb, n))
    return {
        "n": n, "ng": ng, "P_c": pressure_centres(n), "grav": grav,
        "T_star": 5000.0, "T_irr": T_irr, "T_int": T_int, "mmw": MMW,
        "lambda_c": lc, "dlambda": dl, "bin_index": idx,
        "w0": w0, "g0": g0, "vmr": vmr, "T0": np.full(n, 1000.0),
    }


def spectral_workload(seed: int = 2, n: int = 100, nb: int = 3000, ng: int = N_G,
                      ktab: dict | None = None):
    """The full-spectral single-atmosphere case.  Returns (atm, ktab)."""
    if ktab is None:
        ktab = table_ktab(seed, nbt=3000, ng=ng)
    lc_full, dl_full = bins(ktab["k"].shape[3])
    rng = np.random.default_rng([seed, 0])
    atm = spectral_atmosphere(rng, n, lc_full, dl_full, nb, ng)
    return atm, ktab


def resolution_atmosphere(seed: int, n: int, lambda_c_full: np.ndarray, dlambda_full: np.ndarray,
                          ng: int = N_G, T_star: float = 3026.0, T_irr: float = 780.0, T_int: float = 200.0,
                          grav: float = 893.0) -> dict:
    """One physical atmosphere sampled on n layers, the same for every n: the
    mixing-ratio parameters come from rng [seed, 1] and are evaluated at this
    grid's points; w0 ~ U(0, 0.9) and g0 ~ U(0, 0.5) are drawn per bin from
    rng [seed, 2] and constant with height.  Scalars of a cool sub-Neptune
    around an M dwarf (stellar 3026 K, irradiation 780 K, g = 893 cm s^-2),
    all bins of the table."""
    nb = lambda_c_full.size
    vmr = smooth_vmr(np.random.default_rng([seed, 1]), point_log10p_bar(n))
    rng = np.random.default_rng([seed, 2])
    w0 = np.repeat(rng.uniform(0.0, 0.9, size=(nb, 1)), n, axis=1)
    g0 = np.repeat(rng.uniform(0.0, 0.5, size=(nb, 1)), n, axis=1)
    return {
        "n": n, "ng": ng, "P_c": pressure_centres(n), "grav": grav,
        "T_star": T_star, "T_irr": T_irr, "T_int": T_int, "mmw": MMW,
        "lambda_c": lambda_c_full.copy(), "dlambda": dlambda_full.copy(),
        "bin_index": np.arange(nb, dtype=np.int32), "w0": w0, "g0": g0, "vmr": vmr,
        "T0": np.full(n, 1000.0),
    }


def batch_workload(seed: int = 3, n_atm: int = 512, n_range=(50, 200), nb_range=(400, 3000),
                   ng: int = N_G, ktab: dict | None = None):
    """Uneven batch: per atmosphere n ~ U{n_range}, bins ~ U{nb_range} (strided
    subset of the table bins), T_irr ~ U(800, 2800), T_int ~ U(100, 600),
    log10 g[m s^-2] ~ U(0.7, 1.7).  Draw order per atmosphere: n, nb, T_irr,
    T_int, log g, then the atmosphere's own inputs.  Returns (atms, ktab)."""
    if ktab is None:
        ktab = table_ktab(2, nbt=3000, ng=ng)
    lc_full, dl_full = bins(ktab["k"].shape[3])
    rng = np.random.default_rng([seed, 0])
    atms = []
    for _ in range(n_atm):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        nb = int(rng.integers(nb_range[0], nb_range[1] + 1))
        T_irr = float(rng.uniform(800.0, 2800.0))
        T_int = float(rng.uniform(100.0, 600.0))
        grav = float(10.0 ** rng.uniform(0.7, 1.7)) * 100.0
        atms.append(spectral_atmosphere(rng, n, lc_full, dl_full, nb, ng, T_irr, T_int, grav))
    return atms, ktab


# ------------------------------------------------------ learned warm start
PARAM_NAMES = ("T_irr", "T_int", "log10_g", "metallicity", "C_to_O", "log10_opacity_scale")
SOLAR_C, SOLAR_O = 2.5e-4, 5.0e-4  # number ratios to H2 (stand-in solar values)


def draw_params(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Six parameters per atmosphere [count][6], float32, drawn per index i
    from default_rng([seed, 1, i]) in this order: T_irr ~ U(800, 2800) K,
    T_int ~ U(100, 600) K, log10 g[m s^-2] ~ U(0.7, 1.7), [M/H] ~ U(-1, 2),
    C/O ~ U(0.3, 1.5), log10 opacity scale ~ U(-1, 1)."""
    out = np.empty((count, 6), np.float64)
    for k in range(count):
        rng = np.random.default_rng([seed, 1, start + k])
        out[k] = [rng.uniform(800.0, 2800.0), rng.uniform(100.0, 600.0), rng.uniform(0.7, 1.7),
                  rng.uniform(-1.0, 2.0), rng.uniform(0.3, 1.5), rng.uniform(-1.0, 1.0)]
    return out.astype(np.float32)


def standin_vmr(lp_bar: np.ndarray, metallicity: float, c_to_o: float) -> np.ndarray:
    """Volume mixing ratios of CO, CO2, H2O, CH4 at log10 P (bar) for a
    metallicity and C/O: oxygen n_O = 5e-4 10^[M/H], carbon n_C = C/O n_O;
    the carbon sits in CH4 at depth and in CO (90 %) and CO2 (10 %) aloft,
    switching smoothly around 1 bar (logistic in log P, width 0.75 dex);
    water takes the oxygen left over.  Each ratio is clipped to
    [1e-8, 1e-3].  A smooth stand-in for an equilibrium-chemistry table,
    input construction only."""
    n_O = SOLAR_O * 10.0 ** metallicity
    n_C = c_to_o * n_O
    f_deep = 1.0 / (1.0 + np.exp(-lp_bar / 0.75))
    ch4 = n_C * f_deep
    co = 0.9 * n_C * (1.0 - f_deep)
    co2 = 0.1 * n_C * (1.0 - f_deep)
    h2o = np.maximum(n_O - co - 2.0 * co2, 0.0)
    return np.clip(np.stack([co, co2, h2o, ch4]), 1e-8, 1e-3)


def param_atmosphere(params, index_seed, n: int, lambda_c_full: np.ndarray, dlambda_full: np.ndarray, nb: int,
                     ng: int = N_G) -> dict:
    """The atmosphere of one parameter row: stand-in chemistry times the
    opacity scale, w0 ~ U(0, 0.9) and g0 ~ U(0, 0.5) per (bin, layer) from
    default_rng(index_seed), T_star = 5000 K, isothermal 1000 K start."""
    T_irr, T_int, lg, mh, co, lsc = (float(v) for v in params)
    rng = np.random.default_rng(index_seed)
    if nb == lambda_c_full.size:
        idx, lc, dl = np.arange(nb, dtype=np.int32), lambda_c_full.copy(), dlambda_full.copy()
    else:
        idx, lc, dl = subset_bins(lambda_c_full, nb)
    vmr = standin_vmr(point_log10p_bar(n), mh, co) * 10.0 ** lsc
    return {
        "n": n, "ng": ng, "P_c": pressure_centres(n), "grav": 10.0 ** lg * 100.0,
        "T_star": 5000.0, "T_irr": T_irr, "T_int": T_int, "mmw": MMW,
        "lambda_c": lc, "dlambda": dl, "bin_index": idx,
        "w0": rng.uniform(0.0, 0.9, size=(nb, n)), "g0": rng.uniform(0.0, 0.5, size=(nb, n)),
        "vmr": vmr, "T0": np.full(n, 1000.0), "params": np.asarray(params, np.float32),
    }


def learned_workload(seed: int, count: int, start: int = 0, n: int = 100, nb: int = 1000, ng: int = N_G,
                     ktab: dict | None = None):
    """Atmospheres start..start+count-1 of a parameter set: seed 4 is the
    training set and 40 the held-out set of the warm-start network (100
    layers, 1000 strided bins); seed 5 with n = 200, nb = 3000 is the
    production sweep.  Returns (atms, ktab)."""
    if ktab is None:
        ktab = table_ktab(2, nbt=3000, ng=ng)
    lc_full, dl_full = bins(ktab["k"].shape[3])
    P = draw_params(seed, count, start)
    atms = [param_atmosphere(P[k], [seed, 2, start + k], n, lc_full, dl_full, nb, ng) for k in range(count)]
    return atms, ktab
