"""FP64 CPU oracle of the HELIOS radiative-equilibrium hot path.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the smoke check of the
entry module and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the GPU library: the C source
next to this file (``helios_ref.c``) is compiled on its own with gcc, and the
only thing the two sides share is the seeded input arrays.

Each wrapper follows one passage of Malik et al. (2017); the citation is on
the C function it calls.  Everything is float64, cgs units, one atmosphere per
call; the wrappers only marshal numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "helios_ref.c")
_LIB = os.path.join(_HERE, "libhelios_ref.so")

M_PROTON = 1.67262192369e-24  # g (CODATA 2018)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c99", "-Wall", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d, i = ctypes.c_double, ctypes.c_int
        P = ctypes.c_void_p
        lib.ref_sigma_sb.restype = d
        lib.ref_gauss_legendre.argtypes = [i, P, P]
        lib.ref_grid.argtypes = [i, P, P]
        lib.ref_profile.argtypes = [i, P, P, P]
        lib.ref_planck.argtypes = [d, d]
        lib.ref_planck.restype = d
        lib.ref_planck_table.argtypes = [i, i, P, P, P]
        lib.ref_boundary.argtypes = [i, P, P, d, d, d, P, P]
        lib.ref_mix_table.argtypes = [i, P, P, i, P, P, d, i, i, d, d, d, d, i, i, P, i, P, P]
        lib.ref_mix_powerlaw.argtypes = [i, P, P, i, P, P, d, i, i, P, d, d, d, d, i, P, P]
        lib.ref_branch.argtypes = [d, d]
        lib.ref_branch.restype = i
        for f in (lib.ref_sub_up, lib.ref_sub_down):
            f.argtypes = [d, d, d, d, d, d, d, d]
            f.restype = d
        lib.ref_sub_trans.argtypes = [d, d, d, d]
        lib.ref_sub_trans.restype = d
        lib.ref_flux.argtypes = [i, i, i, P, d, P, P, P, P, d, d, d, P, P, P, i, d,
                                 P, P, P, P, P, i]
        lib.ref_flux.restype = i
        lib.ref_flux_iso.argtypes = [i, i, i, P, d, P, P, P, P, d, d, d, P, P, P, i, d,
                                     P, P, P, P, P, i]
        lib.ref_flux_rayleigh.argtypes = [i, i, i, P, d, P, P, P, P, d, d, d, P, d, i, d,
                                          P, P, P, P, P, i]
        lib.ref_flux_rayleigh.restype = i
        lib.ref_rayleigh_h2.argtypes = [d]
        lib.ref_rayleigh_h2.restype = d
        lib.ref_flux_iso.restype = i
        lib.ref_flux_exact.argtypes = [i, i, i, P, d, P, P, P, P, d, d, d, P, P, P, P, P, P, i]
        lib.ref_flux_exact.restype = i
        lib.ref_radeq.argtypes = [i, P, P, d, d, d, P, P, P, d, i, d, i, i, d, d, d, d, i, P]
        lib.ref_radeq.restype = i
        for name in ("ref_E1", "ref_exact_trans", "ref_exact_diffusivity"):
            getattr(lib, name).argtypes = [d]
            getattr(lib, name).restype = d
        for name in ("ref_exact_up", "ref_exact_down"):
            getattr(lib, name).argtypes = [d, d, d, d, i]
            getattr(lib, name).restype = d
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------- scalars
def sigma_sb() -> float:
    return _load().ref_sigma_sb()


def planck(lam: float, T: float) -> float:
    return _load().ref_planck(float(lam), float(T))


def planck_table(lambda_c, T_pt) -> np.ndarray:
    """B(lambda_l, T_p) as [bin][point]."""
    lc, T = _f64(lambda_c), _f64(T_pt)
    out = np.zeros((lc.size, T.size))
    _load().ref_planck_table(lc.size, T.size, _p(lc), _p(T), _p(out))
    return out


def isothermal_flux(atm: dict, T_pt, D: float = 2.0) -> np.ndarray:
    """(2 pi / D) B(lambda_l, T_p) [bin][point]: the flux of both streams in
    an isothermal column (each sublayer relation maps it to itself)."""
    return (2.0 * np.pi / D) * planck_table(atm["lambda_c"], T_pt)


def isothermal_start(atm: dict, T_pt, D: float = 2.0) -> np.ndarray:
    """Warm start [bin][g][point] equal to the isothermal flux in every g."""
    iso = isothermal_flux(atm, T_pt, D)
    return np.ascontiguousarray(np.broadcast_to(iso[:, None, :], (iso.shape[0], int(atm["ng"]), iso.shape[1])))


def gauss_legendre(n: int):
    """Nodes on [0,1] (ascending) and halved weights (sum 1)."""
    y = np.zeros(n)
    w = np.zeros(n)
    if _load().ref_gauss_legendre(int(n), _p(y), _p(w)) != 0:
        raise ValueError("bad n")
    return y, w


def grid(P_c) -> np.ndarray:
    P_c = _f64(P_c)
    n = P_c.size
    out = np.zeros(2 * n + 1)
    _load().ref_grid(n, _p(P_c), _p(out))
    return out


def profile(P_pt, T_c) -> np.ndarray:
    P_pt, T_c = _f64(P_pt), _f64(T_c)
    n = T_c.size
    out = np.zeros(2 * n + 1)
    _load().ref_profile(n, _p(P_pt), _p(T_c), _p(out))
    return out


def boundary(lambda_c, dlambda, T_star, T_irr, T_int):
    lc, dl = _f64(lambda_c), _f64(dlambda)
    top = np.zeros(lc.size)
    bot = np.zeros(lc.size)
    _load().ref_boundary(lc.size, _p(lc), _p(dl), float(T_star), float(T_irr), float(T_int),
                         _p(top), _p(bot))
    return top, bot


# ----------------------------------------------------------------- opacity
def mix_opacity(ktab: dict, T_pt, P_pt, vmr, bin_index, ng: int) -> np.ndarray:
    """kappa[bin][g][pt] at the points (eq:kappa_gauss, eq:mixing)."""
    T_pt, P_pt = _f64(T_pt), _f64(P_pt)
    vmr = _f64(vmr)
    bi = np.ascontiguousarray(bin_index, dtype=np.int32)
    mass = _f64(ktab["mass"])
    nsp, npt = vmr.shape
    nb = bi.size
    out = np.zeros((nb, ng, npt))
    lib = _load()
    if ktab["mode"] == "table":
        k = np.ascontiguousarray(ktab["k"], dtype=np.float32)
        _, nT, nP, nbt, ngt = k.shape
        assert ngt == ng
        lib.ref_mix_table(npt, _p(T_pt), _p(P_pt), nsp, _p(vmr), _p(mass), float(ktab["mmw"]),
                          nT, nP, float(ktab["T_min"]), float(ktab["T_step"]),
                          float(ktab["logP_min"]), float(ktab["logP_step"]), nbt, ng, _p(k),
                          nb, _p(bi), _p(out))
    else:
        k0 = _f64(ktab["k0"])
        _, nbt, ngt = k0.shape
        assert ngt == ng
        lib.ref_mix_powerlaw(npt, _p(T_pt), _p(P_pt), nsp, _p(vmr), _p(mass), float(ktab["mmw"]),
                             nbt, ng, _p(k0), float(ktab["p_exp"]), float(ktab["t_exp"]),
                             float(ktab["P_ref"]), float(ktab["T_ref"]), nb, _p(bi), _p(out))
    return out


# --------------------------------------------------------------- two-stream
def branch(dtau, w0) -> int:
    return _load().ref_branch(float(dtau), float(w0))


def sub_up(dtau, w0, g0, D, B_u, B_d, F_up_d, F_dn_u) -> float:
    return _load().ref_sub_up(*(float(v) for v in (dtau, w0, g0, D, B_u, B_d, F_up_d, F_dn_u)))


def sub_down(dtau, w0, g0, D, B_u, B_d, F_up_d, F_dn_u) -> float:
    return _load().ref_sub_down(*(float(v) for v in (dtau, w0, g0, D, B_u, B_d, F_up_d, F_dn_u)))


def sub_trans(dtau, w0, g0, D=2.0) -> float:
    return _load().ref_sub_trans(float(dtau), float(w0), float(g0), float(D))


def flux(atm: dict, kappa, T_pt, P_pt, F_up, n_scat: int = 4, D: float = 2.0,
         n_threads: int = 0, want_dn: bool = True):
    """One two-stream flux solve of one atmosphere.

    ``F_up`` [bin][g][pt] is the warm start and is updated in place.  Returns a
    dict with F_dn (if wanted), F_up_bin, F_dn_bin [bin][pt] and F_bol [pt][3].
    """
    n = int(atm["n"])
    npt = 2 * n + 1
    lc, dl = _f64(atm["lambda_c"]), _f64(atm["dlambda"])
    nb = lc.size
    ng = int(atm["ng"])
    _, gw = gauss_legendre(ng)
    kappa = _f64(kappa)
    assert kappa.shape == (nb, ng, npt)
    T_pt, P_pt = _f64(T_pt), _f64(P_pt)
    w0, g0 = _f64(atm["w0"]), _f64(atm["g0"])
    assert w0.shape == (nb, n) and g0.shape == (nb, n)
    assert F_up.dtype == np.float64 and F_up.flags.c_contiguous and F_up.shape == (nb, ng, npt)
    F_dn = np.zeros((nb, ng, npt)) if want_dn else None
    up_bin = np.zeros((nb, npt))
    dn_bin = np.zeros((nb, npt))
    bol = np.zeros((npt, 3))
    rc = _load().ref_flux(n, nb, ng, _p(P_pt), float(atm["grav"]), _p(T_pt), _p(lc), _p(dl), _p(gw),
                          float(atm["T_star"]), float(atm["T_irr"]), float(atm["T_int"]),
                          _p(kappa), _p(w0), _p(g0), int(n_scat), float(D),
                          _p(F_up), _p(F_dn) if want_dn else None,
                          _p(up_bin), _p(dn_bin), _p(bol), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle flux failed")
    return {"F_dn": F_dn, "F_up_bin": up_bin, "F_dn_bin": dn_bin, "F_bol": bol}


def rayleigh_h2(lam: float) -> float:
    """H2 Rayleigh cross-section per molecule (cm^2) at wavelength lam (cm)."""
    return _load().ref_rayleigh_h2(float(lam))


def flux_rayleigh(atm: dict, kappa, T_pt, P_pt, F_up, n_scat: int = 4, D: float = 2.0,
                  n_threads: int = 0, want_dn: bool = True):
    """``flux`` with H2 Rayleigh scattering added to the absorption
    opacities ``kappa`` (Sec. 2.1.4): per sublayer and g-point the albedo is
    the scattering share of the extinction and g0 = 0; atm["w0"], atm["g0"]
    are not used."""
    n = int(atm["n"])
    npt = 2 * n + 1
    lc, dl = _f64(atm["lambda_c"]), _f64(atm["dlambda"])
    nb = lc.size
    ng = int(atm["ng"])
    _, gw = gauss_legendre(ng)
    kappa = _f64(kappa)
    assert kappa.shape == (nb, ng, npt)
    T_pt, P_pt = _f64(T_pt), _f64(P_pt)
    assert F_up.dtype == np.float64 and F_up.flags.c_contiguous and F_up.shape == (nb, ng, npt)
    F_dn = np.zeros((nb, ng, npt)) if want_dn else None
    up_bin = np.zeros((nb, npt))
    dn_bin = np.zeros((nb, npt))
    bol = np.zeros((npt, 3))
    mbar = float(atm.get("mmw", 2.4)) * M_PROTON
    rc = _load().ref_flux_rayleigh(n, nb, ng, _p(P_pt), float(atm["grav"]), _p(T_pt), _p(lc), _p(dl), _p(gw),
                                   float(atm["T_star"]), float(atm["T_irr"]), float(atm["T_int"]),
                                   _p(kappa), mbar, int(n_scat), float(D),
                                   _p(F_up), _p(F_dn) if want_dn else None,
                                   _p(up_bin), _p(dn_bin), _p(bol), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle Rayleigh flux failed")
    return {"F_dn": F_dn, "F_up_bin": up_bin, "F_dn_bin": dn_bin, "F_bol": bol}


def flux_iso(atm: dict, kappa_lay, T_lay, P_int, F_up, n_scat: int = 4, D: float = 2.0,
             n_threads: int = 0, want_dn: bool = True):
    """One flux solve on the isothermal-layer grid (Sec. 2.2.1): n layers
    with temperatures T_lay [n] and opacities kappa_lay [bin][g][n] between
    the n + 1 interfaces P_int.  ``F_up`` [bin][g][n+1] is the warm start and
    is updated in place.  Returns F_dn (if wanted), F_up_bin, F_dn_bin
    [bin][n+1] and F_bol [n+1][3] on the interfaces."""
    n = int(atm["n"])
    nif = n + 1
    lc, dl = _f64(atm["lambda_c"]), _f64(atm["dlambda"])
    nb = lc.size
    ng = int(atm["ng"])
    _, gw = gauss_legendre(ng)
    kappa = _f64(kappa_lay)
    assert kappa.shape == (nb, ng, n)
    T_lay, P_int = _f64(T_lay), _f64(P_int)
    assert T_lay.shape == (n,) and P_int.shape == (nif,)
    w0, g0 = _f64(atm["w0"]), _f64(atm["g0"])
    assert w0.shape == (nb, n) and g0.shape == (nb, n)
    assert F_up.dtype == np.float64 and F_up.flags.c_contiguous and F_up.shape == (nb, ng, nif)
    F_dn = np.zeros((nb, ng, nif)) if want_dn else None
    up_bin = np.zeros((nb, nif))
    dn_bin = np.zeros((nb, nif))
    bol = np.zeros((nif, 3))
    rc = _load().ref_flux_iso(n, nb, ng, _p(P_int), float(atm["grav"]), _p(T_lay), _p(lc), _p(dl), _p(gw),
                              float(atm["T_star"]), float(atm["T_irr"]), float(atm["T_int"]),
                              _p(kappa), _p(w0), _p(g0), int(n_scat), float(D),
                              _p(F_up), _p(F_dn) if want_dn else None,
                              _p(up_bin), _p(dn_bin), _p(bol), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle isothermal-grid flux failed")
    return {"F_dn": F_dn, "F_up_bin": up_bin, "F_dn_bin": dn_bin, "F_bol": bol}


# ------------------------------------------------------------------ RE step
RE_DEFAULTS = dict(tol=1e-3, norm_sigma_tint=1, T_floor=10.0, window=6, osc_any=0, shrink=0.67,
                   grow=1.1, fpre_c=1e5, fpre_p=0.9, deadband=0)


def radeq(atm: dict, P_pt, F_bol, T_c, m, hist, opts: dict | None = None):
    """One RE step (updates T_c, m, hist in place).  Returns (code, resid):
    code 1 converged (nothing moves), 0 stepped, -5 non-finite input, -2 a
    point grid whose pressures do not decrease upward (nothing moves)."""
    o = dict(RE_DEFAULTS)
    if opts:
        o.update(opts)
    n = T_c.size
    P_pt, F_bol = _f64(P_pt), _f64(F_bol)
    assert T_c.dtype == np.float64 and m.dtype == np.float64 and hist.dtype == np.int32
    resid = np.zeros(1)
    code = _load().ref_radeq(n, _p(P_pt), _p(F_bol), float(atm["grav"]),
                             float(atm.get("mmw", 2.4)) * M_PROTON, float(atm["T_int"]),
                             _p(T_c), _p(m), _p(hist), float(o["tol"]), int(o["norm_sigma_tint"]),
                             float(o["T_floor"]), int(o["window"]), int(o["osc_any"]), float(o["shrink"]),
                             float(o["grow"]), float(o["fpre_c"]), float(o["fpre_p"]), int(o["deadband"]),
                             _p(resid))
    return code, float(resid[0])


def solve(atm: dict, ktab: dict, max_iter: int = 200, n_scat: int = 4, D: float = 2.0,
          opts: dict | None = None, T_init=None, n_threads: int = 0, callback=None, warm: str = "flux",
          layers: str = "noniso", rayleigh: bool = False):
    """Full RE iteration of one atmosphere (Sec. 2.2.3): profile -> opacity ->
    flux -> RE step, until converged or max_iter steps were taken.

    warm = "flux": the scattering warm start is the previous iteration's
    upward flux, zeros at the first (the paper's description).
    warm = "deviation": the warm start keeps each column's deviation from the
    isothermal flux (2 pi / D) B across iterations and starts from that flux;
    the choice of a warm start changes the trajectory, not the fixed point.

    layers = "iso" solves on the isothermal-layer grid (Sec. 2.2.1): the
    layers keep their centre temperatures and opacities, fluxes live on the
    interfaces, and the RE step takes the same interface net fluxes.  There
    the deviation warm start refers interface i to the layer above it (the
    top interface to the top layer).

    rayleigh = True adds H2 Rayleigh scattering (``flux_rayleigh``; the
    sublayered grid only).

    Returns a dict with T_c, iterations, converged flag, resid history and the
    last flux result.
    """
    if rayleigh and layers != "noniso":
        raise ValueError("Rayleigh scattering is solved on the sublayered grid")
    if layers not in ("noniso", "iso"):
        raise ValueError(layers)
    n = int(atm["n"])
    ng = int(atm["ng"])
    nb = len(atm["lambda_c"])
    P_pt = grid(atm["P_c"])
    T_c = _f64(atm["T0"] if T_init is None else T_init).copy()
    m = np.ones(n)
    hist = np.zeros(n, dtype=np.int32)
    F_up = np.zeros((nb, ng, (n + 1) if layers == "iso" else (2 * n + 1)))
    vmr_c = _f64(atm["vmr"])[:, 1::2]
    resids = []
    converged = False
    it = 0
    res = None
    iso_prev = None
    while True:
        if layers == "iso":
            if warm == "deviation":
                iso = isothermal_flux(atm, T_c[np.minimum(np.arange(n + 1), n - 1)], D)
                F_up += (iso if iso_prev is None else iso - iso_prev)[:, None, :]
                iso_prev = iso
            kap = mix_opacity(ktab, T_c, P_pt[1::2], vmr_c, atm["bin_index"], ng)
            res = flux_iso(atm, kap, T_c, P_pt[0::2], F_up, n_scat=n_scat, D=D, n_threads=n_threads,
                           want_dn=False)
            bol = np.zeros((2 * n + 1, 3))  # interfaces at the even points; the step reads no other
            bol[0::2] = res["F_bol"]
        else:
            T_pt = profile(P_pt, T_c)
            if warm == "deviation":
                iso = isothermal_flux(atm, T_pt, D)
                F_up += (iso if iso_prev is None else iso - iso_prev)[:, None, :]
                iso_prev = iso
            kap = mix_opacity(ktab, T_pt, P_pt, atm["vmr"], atm["bin_index"], ng)
            fn = flux_rayleigh if rayleigh else flux
            res = fn(atm, kap, T_pt, P_pt, F_up, n_scat=n_scat, D=D, n_threads=n_threads, want_dn=False)
            bol = res["F_bol"]
        code, r = radeq(atm, P_pt, bol, T_c, m, hist, opts)
        resids.append(r)
        if callback is not None:
            callback(it, T_c, r)
        if code == 1:
            converged = True
            break
        if code < 0:
            break
        it += 1
        if it >= max_iter:
            break
    return {"T_c": T_c, "iterations": it, "converged": converged, "resid": np.array(resids),
            "flux": res, "P_pt": P_pt, "F_up": F_up, "m": m, "hist": hist}


# ------------------------------------------------------ exact pure absorption
def E1(x) -> float:
    return _load().ref_E1(float(x))


def exact_trans(dtau) -> float:
    return _load().ref_exact_trans(float(dtau))


def exact_diffusivity(dtau) -> float:
    return _load().ref_exact_diffusivity(float(dtau))


def exact_up(dtau, B1, B2, F1_up, iso=False) -> float:
    return _load().ref_exact_up(float(dtau), float(B1), float(B2), float(F1_up), int(bool(iso)))


def exact_down(dtau, B1, B2, F2_dn, iso=False) -> float:
    return _load().ref_exact_down(float(dtau), float(B1), float(B2), float(F2_dn), int(bool(iso)))


def flux_exact(atm: dict, kappa, T_pt, P_pt, n_threads: int = 0):
    """Pure-absorption solve of one atmosphere with the exact layer relations
    (Sec. 2.1.2; w0, g0 and D do not enter; one sweep each way).  Returns a
    dict with F_up, F_dn [bin][g][pt], F_up_bin, F_dn_bin [bin][pt] and F_bol
    [pt][3]."""
    n = int(atm["n"])
    npt = 2 * n + 1
    lc, dl = _f64(atm["lambda_c"]), _f64(atm["dlambda"])
    nb = lc.size
    ng = int(atm["ng"])
    _, gw = gauss_legendre(ng)
    kappa = _f64(kappa)
    assert kappa.shape == (nb, ng, npt)
    T_pt, P_pt = _f64(T_pt), _f64(P_pt)
    F_up = np.zeros((nb, ng, npt))
    F_dn = np.zeros((nb, ng, npt))
    up_bin = np.zeros((nb, npt))
    dn_bin = np.zeros((nb, npt))
    bol = np.zeros((npt, 3))
    rc = _load().ref_flux_exact(n, nb, ng, _p(P_pt), float(atm["grav"]), _p(T_pt), _p(lc), _p(dl), _p(gw),
                                float(atm["T_star"]), float(atm["T_irr"]), float(atm["T_int"]), _p(kappa),
                                _p(F_up), _p(F_dn), _p(up_bin), _p(dn_bin), _p(bol), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle exact flux failed")
    return {"F_up": F_up, "F_dn": F_dn, "F_up_bin": up_bin, "F_dn_bin": dn_bin, "F_bol": bol}


# ------------------------------------------------- direct column solution
def column_direct(atm: dict, kappa_col, B_col, w0_col, g0_col, F_top: float, F_int: float,
                  P_pt, D: float = 2.0) -> tuple[np.ndarray, np.ndarray]:
    """Solve one column's discrete two-stream system exactly (the limit of
    infinitely many scattering passes).  Each sublayer relation is affine in
    its two incoming fluxes; its coefficients are read off the oracle's own
    sublayer functions, the 2(2n+1) equations plus both boundary conditions
    are assembled densely and solved with LAPACK."""
    n = int(atm["n"])
    npt = 2 * n + 1
    g = float(atm["grav"])
    N = 2 * npt  # unknowns: up[0..2n], dn[0..2n]
    A = np.zeros((N, N))
    b = np.zeros(N)
    U = lambda p: p          # noqa: E731
    Dn = lambda p: npt + p   # noqa: E731
    row = 0
    A[row, Dn(2 * n)] = 1.0
    b[row] = F_top
    row += 1
    A[row, U(0)] = 1.0
    A[row, Dn(0)] = -1.0
    b[row] = F_int
    row += 1
    for s in range(2 * n):
        dtau = 0.5 * (kappa_col[s] + kappa_col[s + 1]) * (P_pt[s] - P_pt[s + 1]) / g
        w0, g0 = w0_col[s // 2], g0_col[s // 2]
        Bu, Bd = B_col[s + 1], B_col[s]
        for fn, out in ((sub_up, U(s + 1)), (sub_down, Dn(s))):
            # the flux coefficients are read with the sources switched off, so
            # that no difference of large numbers enters
            c0 = fn(dtau, w0, g0, D, Bu, Bd, 0.0, 0.0)
            cu = fn(dtau, w0, g0, D, 0.0, 0.0, 1.0, 0.0)
            cd = fn(dtau, w0, g0, D, 0.0, 0.0, 0.0, 1.0)
            A[row, out] = 1.0
            A[row, U(s)] -= cu
            A[row, Dn(s + 1)] -= cd
            b[row] = c0
            row += 1
    assert row == N
    x = np.linalg.solve(A, b)
    return x[:npt], x[npt:]
