"""Python binding of libhelios (include/helios.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  torch provides device memory and streams.  The library must be
built (``python -m paper_1606_05474_amd.build``); importing this module on a
machine without it raises.

Names follow the C ABI: ``grid``, ``profile``, ``mix_opacity``,
``transmission``, ``workspace_bytes``, ``flux``, ``radeq`` wrap
``helios_grid`` ... ``helios_radeq``.
"""
from __future__ import annotations

import copy
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelios.so")

HELIOS_OK = 0
HELIOS_NOT_CONVERGED = 1
FP64, MIXED = 0, 1
KTAB_TABLE, KTAB_POWERLAW = 0, 1
NORM_SIGMA_T4, NORM_SIGMA_TINT4 = 0, 1
ATM_RUNNING, ATM_CONVERGED, ATM_BADGRID, ATM_NUMERIC = 0, 1, -2, -5
STATE_DEVIATION, STATE_FLUX = 0x000, 0x100  # per-g convention, OR'ed into prec
GRID_ISOTHERMAL = 0x200  # OR'ed into prec of autotune / sweep_shapes: helios_flux_iso's shapes
CONVERT_TO_DEVIATION, CONVERT_TO_FLUX, CONVERT_ZERO_FLUX = 0, 1, 2
LAYERS_SUBLAYERED, LAYERS_ISOTHERMAL = 0, 1
MAX_SPECIES = 8
CELL_ALIGN = 32  # column stride of the cell arrays: 2n+1 rounded up to this
NOALLOC_WS_BYTES = 64 << 20  # static workspace of helios_flux_noalloc (HELIOS_NOALLOC_WS_BYTES)

_P = ctypes.c_void_p


class HeliosAtm(ctypes.Structure):
    _fields_ = [("n_atm", ctypes.c_int32), ("n_g", ctypes.c_int32),
                ("n_layer_h", _P), ("n_bin_h", _P), ("n_layer", _P), ("n_bin", _P),
                ("lay_off", _P), ("pt_off", _P), ("bin_off", _P), ("lb_off", _P), ("pb_off", _P),
                ("cell_off", _P), ("bin_index", _P), ("bin_index_h", _P), ("lambda_c", _P), ("dlambda", _P), ("P_c", _P),
                ("P_pt", _P), ("grav", _P), ("T_star", _P), ("T_irr", _P), ("T_int", _P), ("status", _P)]


class HeliosKtab(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n_species", ctypes.c_int32), ("n_T", ctypes.c_int32),
                ("n_P", ctypes.c_int32), ("n_bin_table", ctypes.c_int32), ("n_g", ctypes.c_int32),
                ("T_min", ctypes.c_double), ("T_step", ctypes.c_double), ("logP_min", ctypes.c_double),
                ("logP_step", ctypes.c_double), ("k", _P), ("k0", _P), ("p_exp", ctypes.c_double),
                ("t_exp", ctypes.c_double), ("P_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
                ("species_mass", _P), ("mmw", ctypes.c_double)]


class HeliosReOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("norm", ctypes.c_int32), ("window", ctypes.c_int32),
                ("osc_any", ctypes.c_int32), ("deadband", ctypes.c_int32), ("T_floor", ctypes.c_double),
                ("shrink", ctypes.c_double), ("grow", ctypes.c_double), ("fpre_c", ctypes.c_double),
                ("fpre_p", ctypes.c_double)]


class HeliosReState(ctypes.Structure):
    _fields_ = [("m", _P), ("hist", _P), ("iter", _P)]


class HeliosMlp(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_hidden_layers", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("params", _P), ("params_bf16", _P), ("adam_m", _P), ("adam_v", _P),
                ("in_shift", _P), ("in_scale", _P), ("out_shift", _P), ("out_scale", _P)]


_lib = None


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhelios.so not found at {LIB_PATH}; build it with "
                               "`python -m paper_1606_05474_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        A = ctypes.POINTER(HeliosAtm)
        i32, dbl, sz = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        L.helios_grid.argtypes = [A, _P]
        L.helios_profile.argtypes = [A, _P, _P, _P]
        L.helios_mix_opacity.argtypes = [A, ctypes.POINTER(HeliosKtab), _P, _P, _P, ctypes.c_int, _P]
        L.helios_transmission.argtypes = [A, _P, _P, _P, _P, dbl, _P, ctypes.c_int, _P]
        L.helios_workspace_bytes.argtypes = [A, ctypes.c_int]
        L.helios_workspace_bytes.restype = sz
        L.helios_flux.argtypes = [A, _P, _P, _P, _P, i32, dbl, _P, _P, _P, _P, _P, _P, sz, ctypes.c_int, _P]
        L.helios_flux_iso.argtypes = L.helios_flux.argtypes
        L.helios_flux_noalloc.argtypes = [A, _P, _P, _P, _P, i32, dbl, _P, _P, _P, _P, _P, ctypes.c_int, _P]
        L.helios_flux_rayleigh.argtypes = [A, _P, _P, dbl, i32, dbl, _P, _P, _P, _P, _P, _P, sz, ctypes.c_int, _P]
        L.helios_flux_exact.argtypes = [A, _P, _P, _P, _P, _P, _P, _P, _P, sz, i32, _P]
        L.helios_state_convert.argtypes = [A, _P, dbl, _P, i32, i32, ctypes.c_int, _P]
        L.helios_autotune_reset.argtypes = []
        L.helios_radeq.argtypes = [A, _P, _P, _P, ctypes.POINTER(HeliosReState), ctypes.POINTER(HeliosReOpts),
                                   _P, _P, _P]
        L.helios_autotune.argtypes = [A, _P, _P, _P, _P, i32, dbl, _P, _P, sz, ctypes.c_int, _P]
        L.helios_sweep_shapes.argtypes = [A, ctypes.c_int, _P, i32]
        N = ctypes.POINTER(HeliosMlp)
        L.helios_mlp_param_count.argtypes = [N]
        L.helios_mlp_param_count.restype = sz
        L.helios_mlp_workspace_bytes.argtypes = [N, i32]
        L.helios_mlp_workspace_bytes.restype = sz
        L.helios_mlp_sync.argtypes = [N, _P]
        L.helios_mlp_forward.argtypes = [N, _P, i32, _P, _P, sz, _P]
        L.helios_mlp_backward.argtypes = [N, _P, _P, i32, _P, _P, _P, sz, _P]
        L.helios_mlp_adam.argtypes = [N, _P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]
        L.helios_warm_start.argtypes = [A, N, _P, _P, dbl, dbl, dbl, _P, _P, _P, sz, _P]
        L.helios_set_sweep_events.argtypes = [_P, _P]
        L.helios_set_sweep_events.restype = ctypes.c_int
        L.helios_last_error.restype = ctypes.c_char_p
        L.helios_version.restype = i32
        for f in ("helios_grid", "helios_profile", "helios_mix_opacity", "helios_transmission",
                  "helios_flux", "helios_flux_iso", "helios_flux_rayleigh", "helios_flux_exact",
                  "helios_flux_noalloc",
                  "helios_state_convert", "helios_autotune_reset",
                  "helios_radeq", "helios_autotune", "helios_sweep_shapes", "helios_mlp_sync",
                  "helios_mlp_forward", "helios_mlp_backward", "helios_mlp_adam", "helios_warm_start"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


class HeliosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"helios error {code}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise HeliosError(rc, lib().helios_last_error().decode())
    return rc


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ------------------------------------------------------------ batch layout
class Batch:
    """A batch of atmospheres resident on the device, with its descriptor.

    ``atms`` is a list of dicts with keys n, ng, P_c, grav, T_star, T_irr,
    T_int, lambda_c, dlambda, bin_index, w0 [nb][n], g0 [nb][n], vmr
    [nsp][2n+1] (the workload generator's format).  Arrays are concatenated
    in the order of the list.
    """

    def __init__(self, atms: list, device="cuda"):
        if not atms:
            raise ValueError("empty batch")
        dev = torch.device(device)
        self.atms = atms
        self.n_atm = len(atms)
        self.ng = int(atms[0]["ng"])
        if any(int(a["ng"]) != self.ng for a in atms):
            raise ValueError("all atmospheres of a batch share n_g")
        n = np.array([int(a["n"]) for a in atms], np.int64)
        nb = np.array([len(a["lambda_c"]) for a in atms], np.int64)
        npt = 2 * n + 1
        cs = (npt + CELL_ALIGN - 1) // CELL_ALIGN * CELL_ALIGN
        self.n, self.nb, self.npt, self.cs = n, nb, npt, cs

        def off(x):
            return np.concatenate([[0], np.cumsum(x)]).astype(np.int64)

        self.lay_off, self.pt_off, self.bin_off = off(n), off(npt), off(nb)
        self.lb_off, self.pb_off, self.cell_off = off(nb * n), off(nb * npt), off(nb * self.ng * cs)
        self.total_n, self.total_pt = int(self.lay_off[-1]), int(self.pt_off[-1])
        self.total_bin, self.total_cell = int(self.bin_off[-1]), int(self.cell_off[-1])
        self.total_lb, self.total_pb = int(self.lb_off[-1]), int(self.pb_off[-1])
        self.nsp = int(np.asarray(atms[0]["vmr"]).shape[0])

        f64 = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)  # noqa: E731
        i32 = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.int32), device=dev)    # noqa: E731
        i64 = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.int64), device=dev)    # noqa: E731
        cat = lambda key: np.concatenate([np.ravel(np.asarray(a[key], np.float64)) for a in atms])  # noqa: E731
        self.h_n_layer = np.ascontiguousarray(n, np.int32)
        self.h_n_bin = np.ascontiguousarray(nb, np.int32)
        self.h_bin_index = np.ascontiguousarray(np.concatenate([np.asarray(a["bin_index"], np.int32) for a in atms]))
        self.d = {
            "n_layer": i32(n), "n_bin": i32(nb), "lay_off": i64(self.lay_off), "pt_off": i64(self.pt_off),
            "bin_off": i64(self.bin_off), "lb_off": i64(self.lb_off), "pb_off": i64(self.pb_off),
            "cell_off": i64(self.cell_off),
            "bin_index": i32(self.h_bin_index),
            "lambda_c": f64(cat("lambda_c")), "dlambda": f64(cat("dlambda")), "P_c": f64(cat("P_c")),
            "P_pt": torch.zeros(self.total_pt, dtype=torch.float64, device=dev),
            "grav": f64([a["grav"] for a in atms]), "T_star": f64([a["T_star"] for a in atms]),
            "T_irr": f64([a["T_irr"] for a in atms]), "T_int": f64([a["T_int"] for a in atms]),
        }
        self.w0 = f64(cat("w0"))
        self.g0 = f64(cat("g0"))
        vmr = np.concatenate([np.asarray(a["vmr"], np.float64) for a in atms], axis=1)
        self.vmr = f64(vmr)  # [nsp][total_pt]
        d = self.d
        self.desc = HeliosAtm(
            self.n_atm, self.ng, self.h_n_layer.ctypes.data, self.h_n_bin.ctypes.data,
            *[_ptr(d[k]) for k in ("n_layer", "n_bin", "lay_off", "pt_off", "bin_off", "lb_off", "pb_off",
                                   "cell_off", "bin_index")],
            self.h_bin_index.ctypes.data,
            *[_ptr(d[k]) for k in ("lambda_c", "dlambda", "P_c", "P_pt", "grav", "T_star", "T_irr", "T_int")],
            None)
        self.device = dev

    def replace(self, slots, atms):
        """Put new atmospheres into the given slots of the batch, in place:
        each must have the slot's layer and bin counts, n_g and table bins,
        so every offset and buffer stays where it is (a captured graph that
        reads them stays valid).  The point pressures are recomputed
        (helios_grid) for the whole batch."""
        for a, atm in zip(slots, atms):
            a = int(a)
            n, nb = int(atm["n"]), len(atm["lambda_c"])
            if n != int(self.n[a]) or nb != int(self.nb[a]) or int(atm["ng"]) != self.ng:
                raise ValueError(f"slot {a}: the new atmosphere's sizes differ from the slot's")
            if not np.array_equal(np.asarray(atm["bin_index"], np.int32),
                                  self.h_bin_index[self.bin_off[a]:self.bin_off[a + 1]]):
                raise ValueError(f"slot {a}: the new atmosphere uses other table bins")
            dev = self.device
            f64 = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)  # noqa: E731
            d = self.d
            d["P_c"][self.lay_off[a]:self.lay_off[a + 1]] = f64(atm["P_c"])
            d["lambda_c"][self.bin_off[a]:self.bin_off[a + 1]] = f64(atm["lambda_c"])
            d["dlambda"][self.bin_off[a]:self.bin_off[a + 1]] = f64(atm["dlambda"])
            for key in ("grav", "T_star", "T_irr", "T_int"):
                d[key][a] = float(atm[key])
            self.w0[self.lb_off[a]:self.lb_off[a + 1]] = f64(np.ravel(atm["w0"]))
            self.g0[self.lb_off[a]:self.lb_off[a + 1]] = f64(np.ravel(atm["g0"]))
            self.vmr[:, self.pt_off[a]:self.pt_off[a + 1]] = f64(atm["vmr"])
            self.atms[a] = atm
        grid(self)

    def with_status(self, status):
        """A view of this batch whose descriptor carries a device status
        array: atmospheres that are not ATM_RUNNING are skipped by
        mix_opacity and flux.  Shares every buffer with this batch."""
        v = copy.copy(self)
        v.desc = HeliosAtm.from_buffer_copy(self.desc)
        v.desc.status = _ptr(status)
        v._status = status  # keep the array alive with the view
        return v

    @property
    def P_pt(self):
        return self.d["P_pt"]

    # ---- helpers to cut concatenated arrays back into atmospheres
    def split_pt(self, x):
        return [x[self.pt_off[a]:self.pt_off[a + 1]] for a in range(self.n_atm)]

    def split_layer(self, x):
        return [x[self.lay_off[a]:self.lay_off[a + 1]] for a in range(self.n_atm)]

    def split_cell(self, x):
        """Per-atmosphere [bin][g][point] views of a cell array (padding dropped)."""
        return [x[self.cell_off[a]:self.cell_off[a + 1]].reshape(int(self.nb[a]), self.ng, int(self.cs[a]))
                [:, :, :int(self.npt[a])] for a in range(self.n_atm)]

    def pack_cell(self, per_atm, dtype=torch.float64):
        """A device cell array from per-atmosphere [bin][g][point] arrays."""
        out = np.zeros(self.total_cell, np.float64)
        for a, arr in enumerate(per_atm):
            v = out[self.cell_off[a]:self.cell_off[a + 1]].reshape(int(self.nb[a]), self.ng, int(self.cs[a]))
            v[:, :, :int(self.npt[a])] = np.asarray(arr, np.float64)
        return torch.as_tensor(out, device=self.device).to(dtype)

    def split_pb(self, x):
        return [x[self.pb_off[a]:self.pb_off[a + 1]].reshape(int(self.nb[a]), int(self.npt[a]))
                for a in range(self.n_atm)]

    def cat_layer(self, per_atm):
        return torch.as_tensor(np.concatenate([np.asarray(v, np.float64) for v in per_atm]),
                               device=self.device)


class KTable:
    """An opacity source resident on the device (helios_ktab)."""

    def __init__(self, kt: dict, device="cuda"):
        dev = torch.device(device)
        self.mass = np.ascontiguousarray(kt["mass"], np.float64)
        self.nsp = self.mass.size
        if kt["mode"] == "table":
            k = np.ascontiguousarray(kt["k"], np.float32)
            self.k = torch.as_tensor(k, device=dev)
            _, nT, nP, nbt, ng = k.shape
            self.desc = HeliosKtab(KTAB_TABLE, self.nsp, nT, nP, nbt, ng, kt["T_min"], kt["T_step"],
                                   kt["logP_min"], kt["logP_step"], self.k.data_ptr(), None, 0.0, 0.0,
                                   1.0, 1.0, self.mass.ctypes.data, kt["mmw"])
        else:
            k0 = np.ascontiguousarray(kt["k0"], np.float64)
            self.k0 = torch.as_tensor(k0, device=dev)
            _, nbt, ng = k0.shape
            self.desc = HeliosKtab(KTAB_POWERLAW, self.nsp, 0, 0, nbt, ng, 0.0, 0.0, 0.0, 0.0, None,
                                   self.k0.data_ptr(), kt["p_exp"], kt["t_exp"], kt["P_ref"], kt["T_ref"],
                                   self.mass.ctypes.data, kt["mmw"])


def rdtype(prec: int):
    return torch.float32 if (prec & 0xff) == MIXED else torch.float64


# --------------------------------------------------------------- the calls
def grid(b: Batch, stream=None):
    _check(lib().helios_grid(ctypes.byref(b.desc), _stream(stream)))
    return b.P_pt


def profile(b: Batch, T_c, T_pt, stream=None):
    _check(lib().helios_profile(ctypes.byref(b.desc), _ptr(T_c), _ptr(T_pt), _stream(stream)))
    return T_pt


def mix_opacity(b: Batch, kt: KTable, T_pt, kappa, prec=FP64, vmr=None, stream=None):
    v = b.vmr if vmr is None else vmr
    _check(lib().helios_mix_opacity(ctypes.byref(b.desc), ctypes.byref(kt.desc), _ptr(T_pt), _ptr(v),
                                    _ptr(kappa), prec, _stream(stream)))
    return kappa


def transmission(b: Batch, kappa, T_pt, out, D=2.0, prec=FP64, stream=None):
    _check(lib().helios_transmission(ctypes.byref(b.desc), _ptr(kappa), _ptr(T_pt), _ptr(b.w0), _ptr(b.g0),
                                     float(D), _ptr(out), prec, _stream(stream)))
    return out


def set_sweep_events(before=None, after=None):
    """Record torch.cuda.Event pairs around the flux sweep kernel of this
    thread's next helios_flux calls (None, None turns it off)."""
    hb = None if before is None else before.cuda_event
    ha = None if after is None else after.cuda_event
    _check(lib().helios_set_sweep_events(hb, ha))


def autotune_reset():
    """Forget the shapes the autotuner chose in this process."""
    _check(lib().helios_autotune_reset())


def state_convert(b: Batch, T_pt, F_g, mode, D=2.0, prec=FP64, layers="noniso", stream=None):
    """helios_state_convert: a per-g cell array between fluxes and deviations
    from (2 pi / D) B (mode CONVERT_TO_DEVIATION / CONVERT_TO_FLUX), or the
    zero-flux start in deviation form (CONVERT_ZERO_FLUX)."""
    if layers not in LAYERS:
        raise ValueError(f"layers must be one of {LAYERS}")
    lay = LAYERS_SUBLAYERED if layers == "noniso" else LAYERS_ISOTHERMAL
    _check(lib().helios_state_convert(ctypes.byref(b.desc), _ptr(T_pt), float(D), _ptr(F_g), int(mode), lay,
                                      int(prec), _stream(stream)))
    return F_g


def autotune(b: Batch, kappa, T_pt, F_up_g, ws, n_scat=4, D=2.0, prec=FP64, stream=None, layers="noniso"):
    """Time the compiled sweep shapes per size class of the batch and keep
    the fastest for later flux calls on that grid (synchronous; F_up_g is
    restored)."""
    if layers not in LAYERS:
        raise ValueError(f"layers must be one of {LAYERS}")
    flag = GRID_ISOTHERMAL if layers == "iso" else 0
    _check(lib().helios_autotune(ctypes.byref(b.desc), _ptr(kappa), _ptr(T_pt), _ptr(b.w0), _ptr(b.g0),
                                 int(n_scat), float(D), _ptr(F_up_g), _ptr(ws), ws.numel() * ws.element_size(),
                                 prec | flag, _stream(stream)))


def sweep_shapes(b: Batch, prec=FP64, layers="noniso"):
    """{class upper layer bound: (K, L)} for the classes present in the batch
    (the sweep of helios_flux, or of helios_flux_iso with layers="iso")."""
    if layers not in LAYERS:
        raise ValueError(f"layers must be one of {LAYERS}")
    out = np.zeros(3 * 8, np.int32)
    flag = GRID_ISOTHERMAL if layers == "iso" else 0
    k = _check(lib().helios_sweep_shapes(ctypes.byref(b.desc), prec | flag, out.ctypes.data, 8))
    o = out[:3 * k].reshape(k, 3)
    return {int(r[0]): (int(r[1]), int(r[2])) for r in o if r[1] > 0}


def workspace_bytes(b: Batch, prec=FP64) -> int:
    return int(lib().helios_workspace_bytes(ctypes.byref(b.desc), prec))


def flux_exact(b: Batch, kappa, T_pt, F_up_g, F_dn_g, F_up_bin, F_dn_bin, F_bol, ws, state=STATE_DEVIATION,
               stream=None):
    """helios_flux_exact: pure absorption with the exact layer relations
    (FP64; the per-g outputs are deviations from pi B, or the fluxes with
    state=STATE_FLUX)."""
    _check(lib().helios_flux_exact(ctypes.byref(b.desc), _ptr(kappa), _ptr(T_pt), _ptr(F_up_g), _ptr(F_dn_g),
                                   _ptr(F_up_bin), _ptr(F_dn_bin), _ptr(F_bol), _ptr(ws),
                                   ws.numel() * ws.element_size(), int(state), _stream(stream)))


LAYERS = ("noniso", "iso")


def flux(b: Batch, kappa, T_pt, F_up_g, F_up_bin, F_dn_bin, F_bol, ws, n_scat=4, D=2.0, F_dn_g=None,
         prec=FP64, stream=None, layers="noniso"):
    """helios_flux (layers="noniso", the sublayered grid) or helios_flux_iso
    (layers="iso", the isothermal-layer grid)."""
    if layers not in LAYERS:
        raise ValueError(f"layers must be one of {LAYERS}")
    fn = lib().helios_flux if layers == "noniso" else lib().helios_flux_iso
    _check(fn(ctypes.byref(b.desc), _ptr(kappa), _ptr(T_pt), _ptr(b.w0), _ptr(b.g0),
              int(n_scat), float(D), _ptr(F_up_g), _ptr(F_dn_g), _ptr(F_up_bin),
              _ptr(F_dn_bin), _ptr(F_bol), _ptr(ws), ws.numel() * ws.element_size(),
              prec, _stream(stream)))


def flux_noalloc(b: Batch, kappa, T_pt, F_up_g, F_up_bin, F_dn_bin, F_bol, n_scat=4, D=2.0, F_dn_g=None,
                 prec=FP64, stream=None):
    """helios_flux_noalloc: helios_flux on the library's static device
    workspace (batches needing at most NOALLOC_WS_BYTES of it)."""
    _check(lib().helios_flux_noalloc(ctypes.byref(b.desc), _ptr(kappa), _ptr(T_pt), _ptr(b.w0), _ptr(b.g0),
                                     int(n_scat), float(D), _ptr(F_up_g), _ptr(F_dn_g), _ptr(F_up_bin),
                                     _ptr(F_dn_bin), _ptr(F_bol), prec, _stream(stream)))


def flux_rayleigh(b: Batch, kappa, T_pt, F_up_g, F_up_bin, F_dn_bin, F_bol, ws, mbar, n_scat=4, D=2.0,
                  F_dn_g=None, prec=FP64, stream=None):
    """helios_flux_rayleigh: ``kappa`` holds absorption opacities; H2
    Rayleigh scattering (mean molecular mass ``mbar`` in g) sets the
    per-sublayer, per-g albedo; the batch's w0, g0 are not used."""
    _check(lib().helios_flux_rayleigh(ctypes.byref(b.desc), _ptr(kappa), _ptr(T_pt), float(mbar), int(n_scat),
                                      float(D), _ptr(F_up_g), _ptr(F_dn_g), _ptr(F_up_bin), _ptr(F_dn_bin),
                                      _ptr(F_bol), _ptr(ws), ws.numel() * ws.element_size(), prec,
                                      _stream(stream)))


def emission_spectrum(b: Batch, kt: KTable, T_c, n_scat=80, D=2.0, prec=FP64, stream=None, layers="noniso",
                      start="zero"):
    """Post-processing of converged profiles (Sec. 2.6, Sec. 3): one flux
    call with many scattering passes, from zero fluxes (start="zero", the
    paper's start of the scattering iteration) or from the isothermal flux
    (start="isothermal"); returns the upward flux at the top of each
    atmosphere per bin (a list of [n_bin] device arrays) and the per-bin
    upward fluxes at every point.  The paper post-processes on isothermal
    layers (layers="iso", Sec. 3.3)."""
    if start not in ("zero", "isothermal"):
        raise ValueError("start must be 'zero' or 'isothermal'")
    dev = b.device
    rd = rdtype(prec)
    T_c = torch.as_tensor(T_c, dtype=torch.float64, device=dev)
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device=dev)
    grid(b, stream=stream)
    profile(b, T_c, T_pt, stream=stream)
    kap = torch.zeros(b.total_cell, dtype=rd, device=dev)
    mix_opacity(b, kt, T_pt, kap, prec, stream=stream)
    F_up = torch.zeros(b.total_cell, dtype=rd, device=dev)
    if start == "zero":  # zero fluxes in deviation form
        state_convert(b, T_pt, F_up, CONVERT_ZERO_FLUX, D=D, prec=prec, layers=layers, stream=stream)
    ub = torch.zeros(b.total_pb, dtype=torch.float64, device=dev)
    db = torch.zeros(b.total_pb, dtype=torch.float64, device=dev)
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device=dev)
    ws = torch.zeros(workspace_bytes(b, prec), dtype=torch.uint8, device=dev)
    flux(b, kap, T_pt, F_up, ub, db, bol, ws, n_scat=n_scat, D=D, prec=prec, stream=stream, layers=layers)
    per_bin = b.split_pb(ub)
    return [pb_a[:, -1] for pb_a in per_bin], per_bin


@dataclass
class REOptions:
    tol: float = 1e-3
    norm: int = NORM_SIGMA_TINT4
    window: int = 6
    osc_any: int = 0
    T_floor: float = 10.0
    shrink: float = 0.67
    grow: float = 1.1
    fpre_c: float = 1e5
    fpre_p: float = 0.9
    deadband: int = 0

    def c(self) -> HeliosReOpts:
        return HeliosReOpts(self.tol, self.norm, self.window, self.osc_any, self.deadband, self.T_floor,
                            self.shrink, self.grow, self.fpre_c, self.fpre_p)


def radeq(b: Batch, F_bol, T_c, T_pt, m, hist, status, resid=None, opts: REOptions | None = None,
          iters=None, stream=None):
    st = HeliosReState(_ptr(m), _ptr(hist), _ptr(iters))
    o = (opts or REOptions()).c()
    _check(lib().helios_radeq(ctypes.byref(b.desc), _ptr(F_bol), _ptr(T_c), _ptr(T_pt), ctypes.byref(st),
                              ctypes.byref(o), _ptr(status), _ptr(resid), _stream(stream)))


# ------------------------------------------------------- warm-start network
class MLP:
    """The warm-start network's device state (helios_mlp): FP32 master
    parameters, their BF16 copy, Adam moments and the normalisation of inputs
    and outputs.  dims = (n_in, n_hidden, ..., n_hidden, n_out)."""

    def __init__(self, dims=(6, 256, 256, 256, 100), device="cuda", training=True):
        dims = tuple(int(d) for d in dims)
        if len(dims) < 3 or len(set(dims[1:-1])) != 1:
            raise ValueError("dims must be (n_in, H, ..., H, n_out)")
        dev = torch.device(device)
        self.dims, self.device = dims, dev
        self.count = sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))
        f32 = dict(dtype=torch.float32, device=dev)
        self.params = torch.zeros(self.count, **f32)
        self.params_bf16 = torch.zeros(self.count, dtype=torch.int16, device=dev)
        self.adam_m = torch.zeros(self.count, **f32) if training else None
        self.adam_v = torch.zeros(self.count, **f32) if training else None
        self.in_shift = torch.zeros(dims[0], **f32)
        self.in_scale = torch.ones(dims[0], **f32)
        self.out_shift = torch.zeros(dims[-1], **f32)
        self.out_scale = torch.ones(dims[-1], **f32)
        self.desc = HeliosMlp(dims[0], dims[1], len(dims) - 2, dims[-1], _ptr(self.params), _ptr(self.params_bf16),
                              _ptr(self.adam_m), _ptr(self.adam_v), _ptr(self.in_shift), _ptr(self.in_scale),
                              _ptr(self.out_shift), _ptr(self.out_scale))
        n = int(lib().helios_mlp_param_count(ctypes.byref(self.desc)))
        if n != self.count:
            raise HeliosError(-1, f"parameter count {n} != {self.count}")
        self._ws = {}
        self.grad = torch.zeros(self.count, **f32)
        self.loss = torch.zeros(1, **f32)
        self.step_count = 0

    def layers(self, flat=None):
        """[(W, b)] views of a flat parameter vector (default: the master parameters)."""
        flat = self.params if flat is None else flat
        out, off = [], 0
        for i in range(len(self.dims) - 1):
            o, n = self.dims[i + 1], self.dims[i]
            out.append((flat[off:off + o * n].view(o, n), flat[off + o * n:off + o * n + o]))
            off += o * n + o
        return out

    def init(self, seed=0):
        """He-normal hidden weights, scaled-down output layer, zero biases."""
        rng = np.random.default_rng(seed)
        parts = []
        for i in range(len(self.dims) - 1):
            o, n = self.dims[i + 1], self.dims[i]
            sd = np.sqrt(2.0 / n) if i < len(self.dims) - 2 else np.sqrt(1.0 / n) * 0.1
            parts += [rng.normal(0.0, sd, o * n), np.zeros(o)]
        self.set_params(np.concatenate(parts))
        self.adam_m is not None and self.adam_m.zero_()
        self.adam_v is not None and self.adam_v.zero_()
        self.step_count = 0

    def set_params(self, flat):
        self.params.copy_(torch.as_tensor(np.asarray(flat, np.float32), device=self.device))
        _check(lib().helios_mlp_sync(ctypes.byref(self.desc), _stream(None)))

    def set_norm(self, in_shift, in_scale, out_shift, out_scale):
        for t, v in ((self.in_shift, in_shift), (self.in_scale, in_scale), (self.out_shift, out_shift),
                     (self.out_scale, out_scale)):
            t.copy_(torch.as_tensor(np.asarray(v, np.float32), device=self.device))

    def norm(self):
        return {k: getattr(self, k).cpu().numpy().astype(np.float64)
                for k in ("in_shift", "in_scale", "out_shift", "out_scale")}

    def workspace(self, batch):
        ws = self._ws.get(batch)
        if ws is None:
            nbytes = int(lib().helios_mlp_workspace_bytes(ctypes.byref(self.desc), int(batch)))
            if nbytes == 0:
                raise HeliosError(-1, f"bad batch {batch}")
            ws = self._ws[batch] = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return ws

    def _rows(self, x, width, name):
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        if x.dim() != 2 or x.shape[1] != width:
            raise ValueError(f"{name} must be [batch][{width}], got {tuple(x.shape)}")
        return x

    def forward(self, x, out=None, stream=None):
        x = self._rows(x, self.dims[0], "x")
        B = x.shape[0]
        out = torch.empty(B, self.dims[-1], dtype=torch.float32, device=self.device) if out is None else out
        if out.dtype != torch.float32 or out.numel() != B * self.dims[-1] or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 [batch][n_out] tensor")
        ws = self.workspace(B)
        _check(lib().helios_mlp_forward(ctypes.byref(self.desc), _ptr(x), B, _ptr(out), _ptr(ws), ws.numel(),
                                        _stream(stream)))
        return out

    def backward(self, x, T, stream=None):
        """Loss (device scalar) and gradient (flat, device) on a batch."""
        x = self._rows(x, self.dims[0], "x")
        T = self._rows(T, self.dims[-1], "T")
        B = x.shape[0]
        if T.shape[0] != B:
            raise ValueError("x and T need the same number of rows")
        ws = self.workspace(B)
        _check(lib().helios_mlp_backward(ctypes.byref(self.desc), _ptr(x), _ptr(T), B, _ptr(self.loss),
                                         _ptr(self.grad), _ptr(ws), ws.numel(), _stream(stream)))
        return self.loss, self.grad

    def adam(self, grad=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        g = self.grad if grad is None else grad
        if g.dtype != torch.float32 or g.numel() != self.count or not g.is_contiguous():
            raise ValueError("grad must be a contiguous float32 vector of param_count entries")
        _check(lib().helios_mlp_adam(ctypes.byref(self.desc), _ptr(g), self.step_count, lr, beta1, beta2, eps,
                                     _stream(stream)))

    def train_step(self, x, T, lr=1e-3, stream=None):
        loss, _ = self.backward(x, T, stream=stream)
        self.adam(lr=lr, stream=stream)
        return loss

    def save(self, path):
        np.savez(path, dims=np.array(self.dims), params=self.params.cpu().numpy(),
                 **{k: v.astype(np.float32) for k, v in self.norm().items()})

    @classmethod
    def load(cls, path, device="cuda", training=False):
        d = np.load(path)  # plain arrays only, no pickled objects
        net = cls(tuple(int(v) for v in d["dims"]), device=device, training=training)
        net.set_norm(d["in_shift"], d["in_scale"], d["out_shift"], d["out_scale"])
        net.set_params(d["params"])
        return net


def warm_start(b: Batch, net: MLP, x, logP_net, T_c, fallback, T_iso=1000.0, T_lo=10.0, T_hi=1.0e4, stream=None):
    """Initial layer temperatures of every atmosphere of the batch from the
    network (helios_warm_start); fallback[a] = 1 where the isothermal start
    was taken instead."""
    x = net._rows(x, net.dims[0], "x")
    lp = torch.as_tensor(logP_net, dtype=torch.float64, device=b.device).contiguous()
    if x.shape[0] != b.n_atm or lp.numel() != net.dims[-1]:
        raise ValueError("x needs one row per atmosphere and logP_net one value per network output")
    if T_c.numel() != b.total_n or fallback.numel() != b.n_atm or fallback.dtype != torch.int32:
        raise ValueError("T_c needs one value per layer, fallback one int32 per atmosphere")
    ws = net.workspace(b.n_atm)
    _check(lib().helios_warm_start(ctypes.byref(b.desc), ctypes.byref(net.desc), _ptr(x), _ptr(lp), float(T_iso),
                                   float(T_lo), float(T_hi), _ptr(T_c), _ptr(fallback), _ptr(ws), ws.numel(),
                                   _stream(stream)))
    return T_c, fallback


# ------------------------------------------------------------ RE buffers
class Solver:
    """Device buffers of one batch's radiative-equilibrium iteration, and the
    iteration itself: opacity -> flux -> RE step per iteration, all enqueued
    on one stream; the host reads the per-atmosphere status every
    ``check_every`` iterations.

    The batch descriptor the solver passes carries its status array, so an
    atmosphere that converged (or failed) is skipped by every later kernel
    while the rest of the batch iterates on.  ``graph=True`` in ``solve``
    captures ``check_every`` iterations into one HIP graph (torch.cuda.CUDAGraph)
    and replays it, so a block of iterations costs one launch from the host.

    ``state`` is the convention of the per-g warm start kept between
    iterations: "flux" (the fluxes themselves, the paper's reading of
    Sec. 2.2.3; the FP64 default) or "deviation" (deviations from the
    isothermal flux, which keep FP32 sweeps accurate at depth; the mixed
    default).  ``start`` is the scattering iteration's state at the first
    iteration: "zero" (zero fluxes, the paper's start) or "isothermal"
    (F = (2 pi / D) B).
    """

    def __init__(self, b: Batch, kt: KTable, prec=FP64, n_scat=4, D=2.0, opts: REOptions | None = None,
                 bin_fluxes: bool = True, layers: str = "noniso", rayleigh_mbar: float | None = None,
                 state: str | None = None, start: str = "zero"):
        dev = b.device
        rd = rdtype(prec)
        if layers not in LAYERS:
            raise ValueError(f"layers must be one of {LAYERS}")
        if rayleigh_mbar is not None and layers != "noniso":
            raise ValueError("Rayleigh scattering is solved on the sublayered grid")
        if prec not in (FP64, MIXED):
            raise ValueError("prec must be FP64 or MIXED (the state convention is its own argument)")
        state = state or ("flux" if prec == FP64 else "deviation")
        if state not in ("flux", "deviation") or start not in ("zero", "isothermal"):
            raise ValueError("state must be 'flux' or 'deviation', start 'zero' or 'isothermal'")
        self.state, self.start = state, start
        self.pflags = prec | (STATE_FLUX if state == "flux" else STATE_DEVIATION)
        self.kt, self.prec, self.n_scat, self.D = kt, prec, n_scat, D
        self.layers = layers  # "iso": the isothermal-layer grid (helios_flux_iso)
        self.rayleigh_mbar = rayleigh_mbar  # H2 Rayleigh scattering with this mean molecular mass (g)
        self.bin_fluxes = bin_fluxes  # keep the per-bin fluxes of every step (the iteration needs only F_bol)
        self.opts = opts or REOptions()
        self.T_c = torch.zeros(b.total_n, dtype=torch.float64, device=dev)
        self.T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device=dev)
        self.kappa = torch.zeros(b.total_cell, dtype=rd, device=dev)
        self.F_up_g = torch.zeros(b.total_cell, dtype=rd, device=dev)
        self.F_up_bin = torch.zeros(b.total_pb, dtype=torch.float64, device=dev) if bin_fluxes else None
        self.F_dn_bin = torch.zeros(b.total_pb, dtype=torch.float64, device=dev) if bin_fluxes else None
        self.F_bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device=dev)
        self.ws = torch.zeros(workspace_bytes(b, prec), dtype=torch.uint8, device=dev)
        self.m = torch.ones(b.total_n, dtype=torch.float64, device=dev)
        self.hist = torch.zeros(b.total_n, dtype=torch.int32, device=dev)
        self.status = torch.zeros(b.n_atm, dtype=torch.int32, device=dev)
        self.resid = torch.zeros(b.n_atm, dtype=torch.float64, device=dev)
        self.iters = torch.zeros(b.n_atm, dtype=torch.int32, device=dev)
        self.b = b.with_status(self.status)
        self._graph = None
        self._warm = None
        self._x = None  # network inputs per atmosphere (network starts only)
        self._T_iso = 1000.0
        grid(b)

    def _start_fluxes(self, b=None):
        """Write the first iteration's per-g state of the running atmospheres
        of ``b`` (default: the solver's batch view) in the solver's
        convention: zero fluxes or the isothermal flux."""
        b = self.b if b is None else b
        lay = "iso" if self.layers == "iso" else "noniso"
        if self.start == "zero" and self.state == "deviation":
            state_convert(b, self.T_pt, self.F_up_g, CONVERT_ZERO_FLUX, D=self.D, prec=self.prec, layers=lay)
        elif self.start == "isothermal" and self.state == "flux":
            state_convert(b, self.T_pt, self.F_up_g, CONVERT_TO_FLUX, D=self.D, prec=self.prec, layers=lay)

    def _only(self, which):
        """A view of the batch in which only the listed atmospheres run."""
        st = torch.full((self.b.n_atm,), ATM_CONVERGED, dtype=torch.int32, device=self.b.device)
        st[torch.as_tensor(np.asarray(which, np.int64), device=self.b.device)] = ATM_RUNNING
        return self.b.with_status(st)

    def _reset_state(self):
        self.F_up_g.zero_()
        self.m.fill_(1.0)
        self.hist.zero_()
        self.status.zero_()
        self.iters.zero_()
        profile(self.b, self.T_c, self.T_pt)
        self._start_fluxes()

    def reset(self, T_init):
        """Start every atmosphere from the given layer temperatures."""
        self.T_c.copy_(torch.as_tensor(T_init, dtype=torch.float64, device=self.b.device))
        self._warm = None
        self._reset_state()

    def warm_reset(self, net: MLP, x, logP_net, T_iso=1000.0, T_lo=10.0, T_hi=1.0e4, m0=1.0):
        """Start from the network's profiles (helios_warm_start); atmospheres
        whose network profile is unusable start isothermal at T_iso.  The
        step multipliers of network-started atmospheres start at m0 (a start
        close to equilibrium needs smaller first steps).  Returns the
        per-atmosphere fallback flags (numpy)."""
        fb = torch.zeros(self.b.n_atm, dtype=torch.int32, device=self.b.device)
        warm_start(self.b, net, x, logP_net, self.T_c, fb, T_iso=T_iso, T_lo=T_lo, T_hi=T_hi)
        self._x = np.asarray(x, np.float32).copy()
        self._reset_state()
        fb = fb.cpu().numpy()
        if m0 != 1.0:
            self.m.fill_(m0)
            for a in np.where(fb != 0)[0]:
                self.m[int(self.b.lay_off[a]):int(self.b.lay_off[a + 1])] = 1.0
        self._warm = fb == 0
        self._T_iso = float(T_iso)
        return fb

    def refill(self, slots, atms, net: MLP | None = None, x=None, m0=1.0):
        """Replace the atmospheres in the given slots by new ones of the same
        sizes (Batch.replace) and start them, in place: from the network's
        profiles (isothermal where unusable; step multipliers m0) when a
        network and the new rows of parameters x are given, else
        isothermally at the solver's isothermal temperature.  The other
        atmospheres continue untouched, and every buffer keeps its place, so
        a captured graph stays valid.  Returns the fallback flags of the new
        atmospheres."""
        slots = np.asarray(slots, np.int64)
        b = self.b
        b.replace(slots, atms)
        fb = np.zeros(slots.size, np.int32)
        if net is not None:
            if self._x is None:
                self._x = np.zeros((b.n_atm, net.dims[0]), np.float32)
            self._x[slots] = np.asarray(x, np.float32)
            T_tmp = torch.empty_like(self.T_c)
            fb_all = torch.zeros(b.n_atm, dtype=torch.int32, device=b.device)
            warm_start(b, net, self._x, net.logP, T_tmp, fb_all, T_iso=self._T_iso)
            fb = fb_all.cpu().numpy()[slots]
        for k, a in enumerate(slots):
            a = int(a)
            lo, hi = int(b.lay_off[a]), int(b.lay_off[a + 1])
            if net is not None:
                self.T_c[lo:hi] = T_tmp[lo:hi]
            else:
                self.T_c[lo:hi] = self._T_iso
            self.m[lo:hi] = m0 if (net is not None and fb[k] == 0) else 1.0
            self.hist[lo:hi] = 0
            self.F_up_g[int(b.cell_off[a]):int(b.cell_off[a + 1])] = 0
        idx = torch.as_tensor(slots, device=b.device)
        self.iters[idx] = 0
        self.resid[idx] = 0.0
        self.status[idx] = ATM_RUNNING
        if self._warm is None:
            self._warm = np.zeros(b.n_atm, bool)
        self._warm[slots] = (fb == 0) if net is not None else False
        profile(self.b, self.T_c, self.T_pt)
        self._start_fluxes(self._only(slots))
        return fb

    def restart(self, which, T_iso=1000.0):
        """Restart the listed atmospheres from the isothermal profile (their
        update counters keep counting); the others are untouched."""
        b = self.b
        for a in which:
            a = int(a)
            self.T_c[int(b.lay_off[a]):int(b.lay_off[a + 1])] = T_iso
            self.m[int(b.lay_off[a]):int(b.lay_off[a + 1])] = 1.0
            self.hist[int(b.lay_off[a]):int(b.lay_off[a + 1])] = 0
            self.F_up_g[int(b.cell_off[a]):int(b.cell_off[a + 1])] = 0
            self.status[a] = ATM_RUNNING
        profile(self.b, self.T_c, self.T_pt)
        if len(which):
            self._start_fluxes(self._only(which))

    def subset(self, keep, prec=None):
        """A solver over the atmospheres `keep` (indices into this batch) that
        continues their iteration: temperatures, step multipliers, sign
        histories, update counts and per-g warm starts are carried over, every
        carried atmosphere is running.  Used to compact a batch whose active
        set has shrunk, so later launches cover only live atmospheres, and to
        continue atmospheres in another precision (the per-g warm start is
        converted where the two solvers keep different conventions)."""
        return Solver.concat([(self, keep)], prec=prec)

    @staticmethod
    def concat(parts, prec=None):
        """One solver over the listed atmospheres of several solvers (parts =
        [(solver, indices), ...], in order), each continuing its iteration as
        in `subset`.  The first part's tables and options are used; prec
        defaults to the first part's."""
        s0 = parts[0][0]
        keeps = [np.asarray(k, np.int64) for _, k in parts]
        dev = s0.b.device
        nb = Batch([src.b.atms[int(a)] for (src, _), keep in zip(parts, keeps) for a in keep], device=dev)
        p_new = s0.prec if prec is None else prec
        s = Solver(nb, s0.kt, prec=p_new, n_scat=s0.n_scat, D=s0.D, opts=s0.opts, bin_fluxes=s0.bin_fluxes,
                   layers=s0.layers, rayleigh_mbar=s0.rayleigh_mbar,
                   state=s0.state if p_new == s0.prec else None, start=s0.start)
        k = 0
        warm = []
        to_flux, to_dev = [], []  # carried atmospheres whose convention changes
        for (src, _), keep in zip(parts, keeps):
            b0 = src.b
            for a in keep:
                a = int(a)
                ls, le = int(b0.lay_off[a]), int(b0.lay_off[a + 1])
                ns = int(nb.lay_off[k])
                s.T_c[ns:ns + le - ls] = src.T_c[ls:le]
                s.m[ns:ns + le - ls] = src.m[ls:le]
                s.hist[ns:ns + le - ls] = src.hist[ls:le]
                cs, ce = int(b0.cell_off[a]), int(b0.cell_off[a + 1])
                nc = int(nb.cell_off[k])
                s.F_up_g[nc:nc + ce - cs] = src.F_up_g[cs:ce].to(s.F_up_g.dtype)
                if src.state != s.state:
                    (to_flux if s.state == "flux" else to_dev).append(k)
                k += 1
            if keep.size:
                idx = torch.as_tensor(keep, device=dev)
                lo = k - keep.size
                s.iters[lo:k] = src.iters[idx]
                s.resid[lo:k] = src.resid[idx]
            warm.append(src._warm[keep] if src._warm is not None else np.zeros(keep.size, bool))
        s._warm = np.concatenate(warm) if any(src._warm is not None for src, _ in parts) else None
        s._T_iso = s0._T_iso
        profile(s.b, s.T_c, s.T_pt)
        lay = "iso" if s.layers == "iso" else "noniso"
        for idx, mode in ((to_flux, CONVERT_TO_FLUX), (to_dev, CONVERT_TO_DEVIATION)):
            if idx:
                state_convert(s._only(idx), s.T_pt, s.F_up_g, mode, D=s.D, prec=s.prec, layers=lay)
        return s

    def step(self, stream=None):
        """One RE iteration for every running atmosphere of the batch (enqueue only)."""
        b = self.b
        mix_opacity(b, self.kt, self.T_pt, self.kappa, self.prec, stream=stream)
        if self.rayleigh_mbar is not None:
            flux_rayleigh(b, self.kappa, self.T_pt, self.F_up_g, self.F_up_bin, self.F_dn_bin, self.F_bol,
                          self.ws, self.rayleigh_mbar, n_scat=self.n_scat, D=self.D, prec=self.pflags,
                          stream=stream)
        else:
            flux(b, self.kappa, self.T_pt, self.F_up_g, self.F_up_bin, self.F_dn_bin, self.F_bol, self.ws,
                 n_scat=self.n_scat, D=self.D, prec=self.pflags, stream=stream, layers=self.layers)
        radeq(b, self.F_bol, self.T_c, self.T_pt, self.m, self.hist, self.status, self.resid, self.opts,
              iters=self.iters, stream=stream)

    def autotune(self):
        """Pick the sweep shape per size class on the current state (the
        opacities are mixed first); the solver's buffers are left as they were
        apart from kappa."""
        mix_opacity(self.b, self.kt, self.T_pt, self.kappa, self.prec)
        autotune(self.b, self.kappa, self.T_pt, self.F_up_g, self.ws, n_scat=self.n_scat, D=self.D,
                 prec=self.pflags, layers=self.layers)

    def capture(self, n_steps):
        """Capture n_steps iterations into a HIP graph (replayed by
        ``replay``).  The captured kernels read the solver's buffers in place,
        so a later ``reset`` needs no new capture."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                for _ in range(n_steps):
                    self.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self._graph = (g, n_steps)
        return g

    def replay(self):
        self._graph[0].replay()

    def run(self, max_iter=200, check_every=10, graph=False, restart_after=None):
        """Iterate from the current state until every atmosphere converged or
        about max_iter steps were taken (see solve).  With restart_after, a
        warm-started atmosphere still running after that many updates is
        restarted once from the isothermal profile.  Returns (converged
        flags, updates taken, restarted flags) as numpy arrays."""
        if graph and (self._graph is None or self._graph[1] != check_every):
            # capturing enqueues nothing that runs; the state is untouched
            self.capture(check_every)
        restarted = np.zeros(self.b.n_atm, bool)
        done = 0
        while done <= max_iter:
            if graph:
                self.replay()
                done += check_every
            else:
                k = min(check_every, max_iter + 1 - done)
                for _ in range(k):
                    self.step()
                done += k
            st = self.status.cpu().numpy()
            if restart_after is not None and self._warm is not None:
                it = self.iters.cpu().numpy()
                late = np.where(self._warm & ~restarted & (st != ATM_CONVERGED) & (it >= restart_after))[0]
                if late.size:
                    self.restart(late, self._T_iso)
                    restarted[late] = True
                    st = self.status.cpu().numpy()
            if np.all(st != ATM_RUNNING):
                break
        st = self.status.cpu().numpy()
        return st == ATM_CONVERGED, self.iters.cpu().numpy(), restarted

    def solve(self, T_init, max_iter=200, check_every=10, graph=False):
        """Iterate until every atmosphere converged or max_iter temperature
        updates were taken.  Returns (converged flags, updates taken) per
        atmosphere as numpy arrays; the counts come from the device, so
        checking only every ``check_every`` steps loses nothing (converged
        atmospheres are frozen).  With graph=True the blocks of check_every
        iterations are replayed from one captured graph (the last block may
        run a few iterations past max_iter + 1 calls; frozen atmospheres make
        that harmless apart from the time)."""
        self.reset(T_init)
        conv, iters, _ = self.run(max_iter, check_every, graph)
        return conv, iters
