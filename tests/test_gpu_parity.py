"""GPU (HIP, gfx950) path versus the FP64 CPU oracle, element by element, on
the same seeded inputs.  Tolerances:
  * FP64: net flux per point within 1e-10 of the oracle's gross flux
    (|net_gpu - net_ref| / (up_ref + down_ref)), per-g and per-bin fluxes
    within 1e-11 of their column's largest value, temperatures of a single
    update within 1e-9 K;
  * MIXED (FP32 sweeps, compensated sums, FP64 update): net flux within 1e-4
    of the gross flux.
All calls go through the C ABI (libhelios.so) via the ctypes binding.
"""
import os

import numpy as np
import pytest
import torch

import oracle as ref
from gpu_helpers import (MIXED_SIGMA_TOL, col_rel_error, net_flux_error, net_flux_error_sigma, oracle_state,
                         smooth_profile, to_flux, well_conditioned_layers)
from paper_1606_05474_amd import workloads as W

pytestmark = pytest.mark.gpu

H = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global H
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1606_05474_amd import helios

    H = helios
    H.lib()
    yield


def _t(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    return x.detach().cpu().numpy()


def test_native_library_is_the_in_tree_build():
    import paper_1606_05474_amd

    pkg = os.path.dirname(os.path.abspath(paper_1606_05474_amd.__file__))
    assert os.path.dirname(H.LIB_PATH) == pkg
    with open("/proc/self/maps") as f:
        maps = f.read()
    assert H.LIB_PATH in maps


# ------------------------------------------------------------- grid / profile
def test_grid_and_profile_match_oracle():
    atms = [W.plain_workload(n=n, nb=3)[0] for n in (2, 7, 50)]
    b = H.Batch(atms)
    H.grid(b)
    torch.cuda.synchronize()
    T_c = [smooth_profile(a) for a in atms]
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(T_c), T_pt)
    P_all, T_all = _np(b.P_pt), _np(T_pt)
    for a, atm in enumerate(atms):
        P = ref.grid(atm["P_c"])
        np.testing.assert_allclose(b.split_pt(P_all)[a], P, rtol=4e-16, atol=0)
        np.testing.assert_allclose(b.split_pt(T_all)[a], ref.profile(P, T_c[a]), rtol=1e-14, atol=0)


# ------------------------------------------------------------------ opacity
@pytest.mark.parametrize("prec", [0, 1])
def test_mix_opacity_powerlaw(prec):
    atm, kt = W.plain_workload()
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap_ref = oracle_state(atm, kt, T_c)
    T_pt = _t(T)
    kap = torch.zeros(b.total_cell, dtype=H.rdtype(prec), device="cuda")
    H.mix_opacity(b, H.KTable(kt), T_pt, kap, prec)
    got = b.split_cell(_np(kap).astype(np.float64))[0]
    np.testing.assert_allclose(got, kap_ref, rtol=1e-13 if prec == 0 else 2e-6, atol=0)


@pytest.fixture(scope="module")
def small_table():
    return W.table_ktab(2, nbt=300)


@pytest.mark.parametrize("prec", [0, 1])
def test_mix_opacity_table_with_clamping(prec, small_table):
    kt = small_table
    lc, dl = W.bins(300)
    rng = np.random.default_rng(7)
    atm = W.spectral_atmosphere(rng, 40, lc, dl, 77)
    b = H.Batch([atm])
    H.grid(b)
    # span the table and beyond it on both axes (T 50..3400 K; P beyond 1e3 bar at the bottom)
    T_c = np.linspace(3400.0, 50.0, atm["n"])
    P, T, kap_ref = oracle_state(atm, kt, T_c)
    kap = torch.zeros(b.total_cell, dtype=H.rdtype(prec), device="cuda")
    H.mix_opacity(b, H.KTable(kt), _t(T), kap, prec)
    got = b.split_cell(_np(kap).astype(np.float64))[0]
    np.testing.assert_allclose(got, kap_ref, rtol=1e-13 if prec == 0 else 3e-6, atol=0)


# ------------------------------------------------------- sublayer coefficients
def test_transmission_coefficients_match_oracle(small_table):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(8)
    atm = W.spectral_atmosphere(rng, 30, lc, dl, 12, ng=20)
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap_ref = oracle_state(atm, small_table, T_c)
    out = torch.zeros(2 * b.ng * b.total_lb, 5, dtype=torch.float64, device="cuda")
    H.transmission(b, b.pack_cell([kap_ref]), _t(T), out)
    got = _np(out).reshape(12, 20, 60, 5)
    n = atm["n"]
    worst = 0.0
    branches = set()
    for l in range(12):
        B = np.array([ref.planck(atm["lambda_c"][l], t) for t in T])
        for g in range(0, 20, 3):
            for s in range(2 * n):
                dtau = 0.5 * (kap_ref[l, g, s] + kap_ref[l, g, s + 1]) * (P[s] - P[s + 1]) / atm["grav"]
                w0, g0 = atm["w0"][l, s // 2], atm["g0"][l, s // 2]
                branches.add(ref.branch(dtau, w0))
                Bu, Bd = B[s + 1], B[s]
                a_ref = ref.sub_up(dtau, w0, g0, 2.0, 0, 0, 1.0, 0.0)
                c_ref = ref.sub_up(dtau, w0, g0, 2.0, 0, 0, 0.0, 1.0)
                su_ref = ref.sub_up(dtau, w0, g0, 2.0, Bu, Bd, 0.0, 0.0)
                sd_ref = ref.sub_down(dtau, w0, g0, 2.0, Bu, Bd, 0.0, 0.0)
                T_ref = ref.sub_trans(dtau, w0, g0)
                v = got[l, g, s]
                scale_s = max(abs(su_ref), abs(sd_ref), np.pi * max(Bu, Bd)) + 1e-300
                errs = [abs(v[0] - T_ref), abs(v[1] - a_ref), abs(v[2] - c_ref),
                        abs(v[3] - su_ref) / scale_s, abs(v[4] - sd_ref) / scale_s]
                worst = max(worst, max(errs))
    assert branches >= {1, 2}, branches
    assert worst < 1e-11, worst


# ------------------------------------------------------------------- flux
def _gpu_flux(b, kap, T, prec, n_scat=4, F_up0=None, want_dn=True):
    rd = H.rdtype(prec)
    F_up = torch.zeros(b.total_cell, dtype=rd, device="cuda") if F_up0 is None else F_up0
    F_dn = torch.zeros(b.total_cell, dtype=rd, device="cuda") if want_dn else None
    ub = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    db = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    ws = torch.zeros(H.workspace_bytes(b, prec), dtype=torch.uint8, device="cuda")
    H.flux(b, kap.to(rd), T, F_up, ub, db, bol, ws, n_scat=n_scat, F_dn_g=F_dn, prec=prec)
    torch.cuda.synchronize()
    return F_up, F_dn, ub, db, bol


def _check_flux_fp64(b, a, T, res_ref, F_up_ref, F_up, F_dn, ub, db, bol, tol=1e-10):
    """FP64 flux call of atmosphere a (point temperatures T) against the
    oracle's result; the per-g GPU arrays hold deviations from the
    isothermal flux, which the oracle's own Planck values turn into fluxes."""
    bol_a = b.split_pt(_np(bol).reshape(-1, 3))[a]
    err_net = net_flux_error(bol_a, res_ref["F_bol"])
    assert err_net.max() < tol, err_net.max()
    err_sig = net_flux_error_sigma(bol_a, res_ref["F_bol"], b.atms[a]["T_int"])
    assert err_sig.max() < tol, err_sig.max()
    iso = ref.isothermal_flux(b.atms[a], T)
    gu = to_flux(b.split_cell(_np(F_up))[a], iso)
    assert col_rel_error(gu, F_up_ref).max() < 1e-11
    if F_dn is not None:
        gd = to_flux(b.split_cell(_np(F_dn))[a], iso)
        assert col_rel_error(gd, res_ref["F_dn"]).max() < 1e-11
    assert col_rel_error(b.split_pb(_np(ub))[a], res_ref["F_up_bin"]).max() < 1e-11
    assert col_rel_error(b.split_pb(_np(db))[a], res_ref["F_dn_bin"]).max() < 1e-11
    bol_a = b.split_pt(_np(bol).reshape(-1, 3))[a]
    np.testing.assert_allclose(bol_a[:, :2], res_ref["F_bol"][:, :2], rtol=1e-12)


def test_flux_fp64_plain_two_calls_warm_start():
    atm, kt = W.plain_workload()
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap = oracle_state(atm, kt, T_c)
    up_ref = ref.isothermal_start(atm, T)
    r1 = ref.flux(atm, kap, T, P, up_ref)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, b.pack_cell([kap]), _t(T), 0)
    _check_flux_fp64(b, 0, T, r1, up_ref, F_up, F_dn, ub, db, bol)
    # second call warm-started from the first call's upward fluxes, new temperatures
    T2 = T * 1.01
    # the warm start keeps each column's deviation from the isothermal flux
    up_ref += (ref.isothermal_flux(atm, T2) - ref.isothermal_flux(atm, T))[:, None, :]
    r2 = ref.flux(atm, kap, T2, P, up_ref)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, b.pack_cell([kap]), _t(T2), 0, F_up0=F_up)
    _check_flux_fp64(b, 0, T2, r2, up_ref, F_up, F_dn, ub, db, bol)


@pytest.mark.parametrize("n,nb,n_scat", [(100, 40, 4), (37, 9, 0), (61, 5, 11), (200, 6, 4)])
def test_flux_fp64_table_scattering(n, nb, n_scat, small_table):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(n)
    atm = W.spectral_atmosphere(rng, n, lc, dl, nb)
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap = oracle_state(atm, small_table, T_c)
    up_ref = ref.isothermal_start(atm, T)
    r = ref.flux(atm, kap, T, P, up_ref, n_scat=n_scat)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, b.pack_cell([kap]), _t(T), 0, n_scat=n_scat)
    _check_flux_fp64(b, 0, T, r, up_ref, F_up, F_dn, ub, db, bol)


def test_flux_without_downward_output_is_identical():
    atm, kt = W.plain_workload()
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, kt, smooth_profile(atm))
    a = _gpu_flux(b, b.pack_cell([kap]), _t(T), 0, want_dn=True)
    c = _gpu_flux(b, b.pack_cell([kap]), _t(T), 0, want_dn=False)
    assert torch.equal(a[0], c[0]) and torch.equal(a[4], c[4])


@pytest.mark.parametrize("prec", [0, 1])
def test_flux_without_per_bin_outputs_is_identical(prec):
    """NULL per-bin outputs skip only their stores: the bolometric fluxes and
    the warm start are bitwise those of a call that writes them."""
    atm, kt = W.plain_workload()
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, kt, smooth_profile(atm))
    a = _gpu_flux(b, b.pack_cell([kap]), _t(T), prec)
    rd = H.rdtype(prec)
    F_up = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    ws = torch.zeros(H.workspace_bytes(b, prec), dtype=torch.uint8, device="cuda")
    H.flux(b, b.pack_cell([kap]).to(rd), _t(T), F_up, None, None, bol, ws, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(a[0], F_up) and torch.equal(a[4], bol)


def test_flux_mixed_precision_within_tolerance(small_table):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(3)
    atm = W.spectral_atmosphere(rng, 100, lc, dl, 60)
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, small_table, smooth_profile(atm))
    up_ref = ref.isothermal_start(atm, T)
    r = ref.flux(atm, kap, T, P, up_ref)
    # the mixed path computes its own float32 opacities from the same table
    kap_m = torch.zeros(b.total_cell, dtype=torch.float32, device="cuda")
    H.mix_opacity(b, H.KTable(small_table), _t(T), kap_m, 1)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, kap_m, _t(T), 1)
    err = net_flux_error(_np(bol).reshape(-1, 3), r["F_bol"])
    assert err.max() < 1e-4, err.max()
    err_sig = net_flux_error_sigma(_np(bol).reshape(-1, 3), r["F_bol"], atm["T_int"])
    assert err_sig.max() < MIXED_SIGMA_TOL, err_sig.max()
    assert col_rel_error(b.split_pb(_np(ub))[0], r["F_up_bin"]).max() < 1e-4


# ----------------------------------------------------------------- RE step
@pytest.mark.parametrize("deadband", [0, 1])
def test_radeq_matches_oracle_single_update(deadband):
    atms = [W.plain_workload(n=n, nb=8)[0] for n in (50, 23)]
    b = H.Batch(atms)
    H.grid(b)
    rng = np.random.default_rng(5)
    F_bols, T_cs, ms, hs = [], [], [], []
    for atm in atms:
        n = atm["n"]
        P = ref.grid(atm["P_c"])
        inc = rng.normal(0, 3e4, 2 * n + 1)
        if deadband:  # every third layer inside the tolerance band
            for i in range(0, n, 3):
                inc[2 * i + 1:2 * i + 3] = rng.normal(0, 1.0, 2)
        net = 9e4 + np.cumsum(inc)
        F = np.zeros((2 * n + 1, 3))
        F[:, 0] = 5e8 + net
        F[:, 1] = 5e8
        F[:, 2] = F[:, 0] - F[:, 1]
        F_bols.append(F)
        T_cs.append(smooth_profile(atm))
        ms.append(rng.uniform(0.1, 2.0, n))
        # random histories with full and partial windows
        hs.append(((rng.integers(0, 7, n) << 16) | rng.integers(0, 64, n)).astype(np.int32))
    F_d = _t(np.concatenate([f.ravel() for f in F_bols]))
    T_d = b.cat_layer(T_cs)
    m_d = b.cat_layer(ms)
    h_d = _t(np.concatenate(hs), torch.int32)
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    status = torch.zeros(b.n_atm, dtype=torch.int32, device="cuda")
    resid = torch.zeros(b.n_atm, dtype=torch.float64, device="cuda")
    iters = torch.zeros(b.n_atm, dtype=torch.int32, device="cuda")
    H.radeq(b, F_d, T_d, T_pt, m_d, h_d, status, resid, H.REOptions(deadband=deadband), iters=iters)
    torch.cuda.synchronize()
    for a, atm in enumerate(atms):
        T_ref, m_ref, h_ref = T_cs[a].copy(), ms[a].copy(), hs[a].copy()
        code, r = ref.radeq(atm, ref.grid(atm["P_c"]), F_bols[a], T_ref, m_ref, h_ref, {"deadband": deadband})
        if deadband:
            kept = T_ref == T_cs[a]
            assert kept[::3].all() and kept.sum() >= len(kept) // 3
        assert code == 0
        np.testing.assert_allclose(b.split_layer(_np(T_d))[a], T_ref, rtol=0, atol=1e-9)
        np.testing.assert_allclose(b.split_layer(_np(m_d))[a], m_ref, rtol=1e-15)
        np.testing.assert_array_equal(b.split_layer(_np(h_d))[a], h_ref)
        assert _np(resid)[a] == pytest.approx(r, rel=1e-13)
        P = ref.grid(atm["P_c"])
        np.testing.assert_allclose(b.split_pt(_np(T_pt))[a], ref.profile(P, T_ref), rtol=1e-14)
    assert np.all(_np(status) == H.ATM_RUNNING) and np.all(_np(iters) == 1)


def test_radeq_converged_and_numeric_status():
    atm = W.plain_workload(n=10, nb=4)[0]
    b = H.Batch([atm, atm, atm])
    H.grid(b)
    npt = 21
    F = np.zeros((3, npt, 3))
    F[:, :, 0] = 1e8
    F[:, :, 1] = 1e8 - 9.07e4
    F[:, :, 2] = F[:, :, 0] - F[:, :, 1]
    F[1, 6, 2] += 5e3  # an interface: not converged
    F[2, 8, 2] = np.nan
    T = b.cat_layer([np.full(10, 800.0)] * 3)
    T0 = _np(T).copy()
    m = torch.ones(30, dtype=torch.float64, device="cuda")
    h = torch.zeros(30, dtype=torch.int32, device="cuda")
    st = torch.zeros(3, dtype=torch.int32, device="cuda")
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.radeq(b, _t(F.ravel()), T, T_pt, m, h, st)
    torch.cuda.synchronize()
    assert list(_np(st)) == [H.ATM_CONVERGED, H.ATM_RUNNING, H.ATM_NUMERIC]
    Tn = _np(T)
    assert np.all(Tn[:10] == T0[:10]) and np.all(Tn[20:] == T0[20:]) and np.any(Tn[10:20] != T0[10:20])
    # a converged atmosphere stays frozen even if its fluxes change
    F[0, 3, 2] += 1e6
    H.radeq(b, _t(F.ravel()), T, T_pt, m, h, st)
    torch.cuda.synchronize()
    assert np.all(_np(T)[:10] == T0[:10]) and _np(st)[0] == H.ATM_CONVERGED


# ---------------------------------------------------------- end to end
def test_plain_re_solve_matches_oracle():
    """The plain FP64 workload from the paper's start (zero fluxes, then the
    previous step's fluxes) on both sides: same number of temperature updates
    to reach |dF|/sigma T_int^4 < 1e-3 and the same converged profile."""
    atm, kt = W.plain_workload()
    sol = ref.solve(atm, kt, max_iter=200)
    assert sol["converged"]
    b = H.Batch([atm])
    s = H.Solver(b, H.KTable(kt), prec=H.FP64)
    conv, iters = s.solve(atm["T0"], max_iter=200)
    assert conv[0]
    T_gpu = _np(s.T_c)
    dT = np.abs(T_gpu - sol["T_c"])
    assert dT.max() < 0.1, dT.max()
    assert abs(int(iters[0]) - sol["iterations"]) <= 10, (iters[0], sol["iterations"])


# ---------------------------------------------------------- ragged batches
def test_ragged_batch_equals_oracle_per_atmosphere(small_table):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(21)
    atms = [W.spectral_atmosphere(rng, n, lc, dl, nb, T_irr=ti, T_int=tint, grav=gr)
            for n, nb, ti, tint, gr in [(50, 30, 1200.0, 150.0, 900.0), (120, 7, 2500.0, 500.0, 3000.0),
                                        (9, 60, 900.0, 0.0, 500.0), (200, 3, 1800.0, 300.0, 2000.0)]]
    b = H.Batch(atms)
    H.grid(b)
    T_cs = [smooth_profile(a, 1500 + 100 * i, 700 + 50 * i) for i, a in enumerate(atms)]
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(T_cs), T_pt)
    kap = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    H.mix_opacity(b, H.KTable(small_table), T_pt, kap, 0)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, kap, T_pt, 0)
    for a, atm in enumerate(atms):
        P, T, kap_ref = oracle_state(atm, small_table, T_cs[a])
        np.testing.assert_allclose(b.split_cell(_np(kap))[a], kap_ref, rtol=1e-13)
        up_ref = ref.isothermal_start(atm, T)
        r = ref.flux(atm, kap_ref, T, P, up_ref)
        _check_flux_fp64(b, a, T, r, up_ref, F_up, F_dn, ub, db, bol)


# ------------------------------------------------------------- edge cases
def test_edge_minimal_atmosphere_one_bin_one_g():
    rng = np.random.default_rng(2)
    lc, dl = W.bins(1)
    atm = {"n": 2, "ng": 1, "P_c": W.pressure_centres(2), "grav": 1000.0, "T_star": 5000.0,
           "T_irr": 1500.0, "T_int": 0.0, "lambda_c": lc, "dlambda": dl,
           "bin_index": np.zeros(1, np.int32), "w0": rng.uniform(0, 0.5, (1, 2)),
           "g0": rng.uniform(-0.5, 0.5, (1, 2)), "vmr": np.ones((1, 5)), "T0": np.full(2, 1000.0)}
    kt = {"mode": "powerlaw", "k0": np.array([[[0.05]]]), "p_exp": 0.5, "t_exp": 1.0, "P_ref": 1e6,
          "T_ref": 1000.0, "mass": np.array([2.4]), "mmw": 2.4}
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, kt, [1300.0, 800.0])
    up_ref = ref.isothermal_start(atm, T)
    r = ref.flux(atm, kap, T, P, up_ref)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, b.pack_cell([kap]), _t(T), 0)
    _check_flux_fp64(b, 0, T, r, up_ref, F_up, F_dn, ub, db, bol)


def test_edge_pure_scattering_and_isothermal_layers():
    """w0 = 1 everywhere (pure-scattering branch) and optically thin layers
    (isothermal branch) in one column set."""
    lc, dl = W.bins(4)
    n = 12
    w0 = np.ones((4, n))
    w0[1] = 0.3
    atm = {"n": n, "ng": 3, "P_c": W.pressure_centres(n), "grav": 1000.0, "T_star": 5000.0,
           "T_irr": 1500.0, "T_int": 300.0, "lambda_c": lc, "dlambda": dl,
           "bin_index": np.arange(4, dtype=np.int32), "w0": w0, "g0": np.full((4, n), 0.2),
           "vmr": np.ones((1, 2 * n + 1)), "T0": np.full(n, 1000.0)}
    kt = {"mode": "powerlaw", "k0": np.array([[[1e-9, 1e-7, 1e-6]] * 4]), "p_exp": 0.5, "t_exp": 1.0,
          "P_ref": 1e6, "T_ref": 1000.0, "mass": np.array([2.4]), "mmw": 2.4}
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, kt, smooth_profile(atm))
    up_ref = ref.isothermal_start(atm, T)
    r = ref.flux(atm, kap, T, P, up_ref, n_scat=6)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, b.pack_cell([kap]), _t(T), 0, n_scat=6)
    _check_flux_fp64(b, 0, T, r, up_ref, F_up, F_dn, ub, db, bol)


def test_errors_are_reported_and_nothing_runs():
    atm, kt = W.plain_workload()
    b = H.Batch([atm])
    H.grid(b)
    z = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    small_ws = torch.zeros(16, dtype=torch.uint8, device="cuda")
    pb = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HeliosError) as e:
        H.flux(b, z, b.P_pt, z, pb, pb, bol, small_ws)
    assert e.value.code == -4
    with pytest.raises(H.HeliosError) as e:
        H.flux(b, z, b.P_pt, z, pb, pb, bol, small_ws, n_scat=-1)
    assert e.value.code == -1


SHAPES = [(K, L, prec) for K in (4, 8, 14, 26) for L in (16, 32) for prec in (0, 1) if K * L >= 100] + [
    (26, 64, 0), (26, 64, 1)]  # the long-column shape


@pytest.mark.parametrize("K,L,prec", SHAPES)
def test_flux_every_sweep_shape(K, L, prec, small_table, monkeypatch):
    """Every compiled (sublayers per lane, lanes per column) instantiation of
    the sweep gives the oracle's fluxes (FP64 1e-10, mixed 1e-4)."""
    monkeypatch.setenv("HELIOS_SWEEP_K", str(K))
    monkeypatch.setenv("HELIOS_SWEEP_L", str(L))
    lc, dl = W.bins(300)
    rng = np.random.default_rng(K * 100 + L)
    atm = W.spectral_atmosphere(rng, 50, lc, dl, 7)
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, small_table, smooth_profile(atm))
    up_ref = ref.isothermal_start(atm, T)
    r = ref.flux(atm, kap, T, P, up_ref, n_scat=3)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, b.pack_cell([kap]), _t(T), prec, n_scat=3)
    if prec == 0:
        _check_flux_fp64(b, 0, T, r, up_ref, F_up, F_dn, ub, db, bol)
    else:
        assert net_flux_error(_np(bol).reshape(-1, 3), r["F_bol"]).max() < 1e-4
        err_sig = net_flux_error_sigma(_np(bol).reshape(-1, 3), r["F_bol"], atm["T_int"])
        assert err_sig.max() < MIXED_SIGMA_TOL, err_sig.max()
        assert col_rel_error(to_flux(b.split_cell(_np(F_up))[0], ref.isothermal_flux(atm, T)), up_ref).max() < 1e-4


# ------------------------------------------------------- batching features
@pytest.mark.parametrize("prec", [0, 1])
def test_ragged_batch_spanning_every_size_class(prec, small_table):
    """One atmosphere per size class (and the class edges, up to the 832-layer
    maximum), interleaved so that each class launch skips other classes' bins."""
    lc, dl = W.bins(300)
    rng = np.random.default_rng(31 + prec)
    ns = [65, 2, 209, 32, 832, 113, 33, 401, 64, 400]
    atms = [W.spectral_atmosphere(rng, n, lc, dl, 3 + (i % 3)) for i, n in enumerate(ns)]
    b = H.Batch(atms)
    H.grid(b)
    shapes = H.sweep_shapes(b, prec)
    assert len(shapes) == 6
    for hi, (K, L) in shapes.items():
        assert K * L >= 2 * max(n for n in ns if n <= hi)
    T_cs = [smooth_profile(a) for a in atms]
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(T_cs), T_pt)
    kap = torch.zeros(b.total_cell, dtype=H.rdtype(prec), device="cuda")
    H.mix_opacity(b, H.KTable(small_table), T_pt, kap, prec)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, kap, T_pt, prec)
    for a, atm in enumerate(atms):
        P, T, kap_ref = oracle_state(atm, small_table, T_cs[a])
        up_ref = ref.isothermal_start(atm, T)
        r = ref.flux(atm, kap_ref, T, P, up_ref)
        if prec == 0:
            _check_flux_fp64(b, a, T, r, up_ref, F_up, F_dn, ub, db, bol)
        else:
            bol_a = b.split_pt(_np(bol).reshape(-1, 3))[a]
            err = net_flux_error(bol_a, r["F_bol"])
            assert err.max() < 1e-4, (a, err.max())
            err_sig = net_flux_error_sigma(bol_a, r["F_bol"], atm["T_int"])
            assert err_sig.max() < MIXED_SIGMA_TOL, (a, err_sig.max())


def test_status_skips_atmospheres_that_are_not_running(small_table):
    """Atmospheres marked converged or failed in the descriptor's status are
    left untouched by mix_opacity and flux; the others match the oracle."""
    lc, dl = W.bins(300)
    rng = np.random.default_rng(41)
    atms = [W.spectral_atmosphere(rng, n, lc, dl, nb) for n, nb in [(40, 9), (70, 5), (25, 12)]]
    b0 = H.Batch(atms)
    H.grid(b0)
    status = _t([H.ATM_RUNNING, H.ATM_CONVERGED, H.ATM_NUMERIC], torch.int32)
    b = b0.with_status(status)
    T_cs = [smooth_profile(a) for a in atms]
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(T_cs), T_pt)
    sentinel = 12345.0
    kap = torch.full((b.total_cell,), sentinel, dtype=torch.float64, device="cuda")
    H.mix_opacity(b, H.KTable(small_table), T_pt, kap, 0)
    F_up = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    F_dn = torch.full((b.total_cell,), sentinel, dtype=torch.float64, device="cuda")
    ub = torch.full((b.total_pb,), sentinel, dtype=torch.float64, device="cuda")
    db = torch.full((b.total_pb,), sentinel, dtype=torch.float64, device="cuda")
    bol = torch.full((b.total_pt * 3,), sentinel, dtype=torch.float64, device="cuda")
    ws = torch.zeros(H.workspace_bytes(b, 0), dtype=torch.uint8, device="cuda")
    H.flux(b, kap, T_pt, F_up, ub, db, bol, ws, F_dn_g=F_dn, prec=0)
    torch.cuda.synchronize()
    for a in (1, 2):
        assert np.all(b.split_cell(_np(kap))[a] == sentinel)
        assert np.all(b.split_cell(_np(F_up))[a] == 0.0)
        assert np.all(b.split_cell(_np(F_dn))[a] == sentinel)
        assert np.all(b.split_pb(_np(ub))[a] == sentinel) and np.all(b.split_pb(_np(db))[a] == sentinel)
        assert np.all(b.split_pt(_np(bol).reshape(-1, 3))[a] == sentinel)
    P, T, kap_ref = oracle_state(atms[0], small_table, T_cs[0])
    np.testing.assert_allclose(b.split_cell(_np(kap))[0], kap_ref, rtol=1e-13)
    up_ref = ref.isothermal_start(atms[0], T)
    r = ref.flux(atms[0], kap_ref, T, P, up_ref)
    _check_flux_fp64(b, 0, T, r, up_ref, F_up, F_dn, ub, db, bol)


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_restores_warm_start_and_keeps_parity(prec, small_table):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(51)
    atms = [W.spectral_atmosphere(rng, n, lc, dl, nb) for n, nb in [(30, 40), (100, 30), (60, 20)]]
    b = H.Batch(atms)
    H.grid(b)
    T_cs = [smooth_profile(a) for a in atms]
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(T_cs), T_pt)
    kap = torch.zeros(b.total_cell, dtype=H.rdtype(prec), device="cuda")
    H.mix_opacity(b, H.KTable(small_table), T_pt, kap, prec)
    F_up0 = torch.rand(b.total_cell, dtype=torch.float64, device="cuda", generator=torch.Generator(
        device="cuda").manual_seed(5)).to(H.rdtype(prec)) * 1e5
    F_up = F_up0.clone()
    ws = torch.zeros(H.workspace_bytes(b, prec), dtype=torch.uint8, device="cuda")
    H.autotune(b, kap, T_pt, F_up, ws, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(F_up, F_up0)
    shapes = H.sweep_shapes(b, prec)
    assert set(shapes) == {32, 64, 112}
    for hi, (K, L) in shapes.items():
        assert K * L >= 2 * max(a["n"] for a in atms if a["n"] <= hi)
        assert L in (16, 32) and K in (4, 8, 14, 26)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, kap, T_pt, prec)
    for a, atm in enumerate(atms):
        P, T, kap_ref = oracle_state(atm, small_table, T_cs[a])
        up_ref = ref.isothermal_start(atm, T)
        r = ref.flux(atm, kap_ref, T, P, up_ref)
        bol_a = b.split_pt(_np(bol).reshape(-1, 3))[a]
        err = net_flux_error(bol_a, r["F_bol"])
        assert err.max() < (1e-10 if prec == 0 else 1e-4), (a, err.max())
        err_sig = net_flux_error_sigma(bol_a, r["F_bol"], atm["T_int"])
        assert err_sig.max() < (1e-10 if prec == 0 else MIXED_SIGMA_TOL), (a, err_sig.max())


def test_graph_replayed_solve_equals_eager_solve():
    """Blocks of RE iterations captured into one HIP graph and replayed
    (host status reads between replays) reach bit-for-bit the eager loop's
    temperatures, update counts and fluxes; the kernels' sums run in a fixed
    order, so the two loops are the same arithmetic."""
    atms = [W.plain_workload(n=n, nb=16)[0] for n in (30, 50, 12)]
    kt = W.plain_workload(n=30, nb=16)[1]
    T0 = np.concatenate([a["T0"] for a in atms])
    b = H.Batch(atms)
    eager = H.Solver(b, H.KTable(kt), prec=H.FP64)
    ce, ie = eager.solve(T0, max_iter=300, check_every=7)
    graphed = H.Solver(b, H.KTable(kt), prec=H.FP64)
    cg, ig = graphed.solve(T0, max_iter=300, check_every=7, graph=True)
    assert ce.all() and cg.all()
    assert np.array_equal(ie, ig)
    assert torch.equal(eager.T_c, graphed.T_c)
    assert torch.equal(eager.F_bol, graphed.F_bol)
    # a second solve replays the same graph from a fresh state
    cg2, ig2 = graphed.solve(T0, max_iter=300, check_every=7, graph=True)
    assert np.array_equal(ig2, ie) and torch.equal(graphed.T_c, eager.T_c)


# ------------------------------------------------ full-size and converged cases
@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_production_atmosphere_against_oracle(prec):
    """One atmosphere at the production size (200 layers x 3000 bins x 20 g,
    stand-in chemistry, four float32 tables) in the launch configuration the
    benchmarks use: the whole flux call against the oracle on the same
    opacities (FP64 1e-10, mixed 1e-4 relative net flux)."""
    atms, kt = W.learned_workload(5, 1, 0, n=200, nb=3000)
    atm = atms[0]
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm, 2300.0, 900.0)
    P, T, kap_ref = oracle_state(atm, kt, T_c)
    up_ref = ref.isothermal_start(atm, T)
    r = ref.flux(atm, kap_ref, T, P, up_ref)
    T_pt = _t(T)
    kap = torch.zeros(b.total_cell, dtype=H.rdtype(prec), device="cuda")
    H.mix_opacity(b, H.KTable(kt), T_pt, kap, prec)
    F_up, F_dn, ub, db, bol = _gpu_flux(b, kap, T_pt, prec, want_dn=False)
    err = net_flux_error(_np(bol).reshape(-1, 3), r["F_bol"])
    assert err.max() < (1e-10 if prec == 0 else 1e-4), err.max()
    err_sig = net_flux_error_sigma(_np(bol).reshape(-1, 3), r["F_bol"], atm["T_int"])
    assert err_sig.max() < (1e-10 if prec == 0 else MIXED_SIGMA_TOL), err_sig.max()


def test_compacted_batch_continues_the_same_iteration():
    """Moving the running atmospheres of a batch into a smaller one
    (Solver.subset) carries their whole state: the continued iteration gives
    bit-for-bit the temperatures and update counts of the uncompacted run."""
    atms = [W.plain_workload(n=40, nb=12, seed=s)[0] for s in (1, 2, 3, 4, 5)]
    kt = W.plain_workload(n=40, nb=12)[1]
    T0 = np.concatenate([a["T0"] for a in atms])
    b = H.Batch(atms)
    full = H.Solver(b, H.KTable(kt), prec=H.FP64)
    full.reset(T0)
    for _ in range(120):
        full.step()
    part = H.Solver(b, H.KTable(kt), prec=H.FP64)
    part.reset(T0)
    for _ in range(50):
        part.step()
    keep = np.array([4, 1, 2])
    sub = part.subset(keep)
    for _ in range(70):
        sub.step()
    torch.cuda.synchronize()
    for k, a in enumerate(keep):
        np.testing.assert_array_equal(b.split_layer(_np(full.T_c))[a], sub.b.split_layer(_np(sub.T_c))[k])
        assert int(_np(full.iters)[a]) == int(_np(sub.iters)[k])


def test_post_processing_spectrum_with_80_passes():
    """The post-processing step (many scattering passes on a converged
    profile): TOA upward flux per bin against the oracle with the same 80
    passes from the same zero-flux start (Sec. 2.2.3), FP64."""
    lc, dl = W.bins(300)
    rng = np.random.default_rng(81)
    atm = W.spectral_atmosphere(rng, 100, lc, dl, 300)
    kt = W.table_ktab(2, nbt=300)
    T_c = smooth_profile(atm, 1900.0, 1100.0)
    b = H.Batch([atm])
    toa, per_bin = H.emission_spectrum(b, H.KTable(kt), T_c, n_scat=80)
    P, T, kap = oracle_state(atm, kt, T_c)
    r = ref.flux(atm, kap, T, P, np.zeros((300, atm["ng"], 2 * atm["n"] + 1)), n_scat=80, want_dn=False)
    got = _np(toa[0])
    want = r["F_up_bin"][:, -1]
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    assert col_rel_error(_np(per_bin[0]), r["F_up_bin"]).max() < 1e-11


# ----------------------------------------------------- exact pure absorption
def _exact_gpu(b, kap, T):
    F_up = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    F_dn = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    ub = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    db = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    ws = torch.zeros(H.workspace_bytes(b, 0), dtype=torch.uint8, device="cuda")
    H.flux_exact(b, kap, T, F_up, F_dn, ub, db, bol, ws)
    torch.cuda.synchronize()
    return F_up, F_dn, ub, db, bol


@pytest.mark.parametrize("case", ["plain", "table", "transparent"])
def test_flux_exact_matches_oracle(case, small_table):
    """Exact pure-absorption mode (Sec. 2.1.2) against the oracle: per-g
    fluxes, per-bin fluxes and the net flux (1e-10, as the FP64 two-stream
    path), over isothermal-form, non-isothermal and transparent sublayers."""
    if case == "plain":
        atm, kt = W.plain_workload()
    else:
        kt = small_table
        lc, dl = W.bins(300)
        atm = W.spectral_atmosphere(np.random.default_rng(19), 61, lc, dl, 23)
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap = oracle_state(atm, kt, T_c)
    if case == "transparent":  # some points without opacity: zero-depth sublayers
        kap[:, :, 10:20] = 0.0
        kap[:, :, -3:] = 0.0
    r = ref.flux_exact(atm, kap, T, P)
    F_up, F_dn, ub, db, bol = _exact_gpu(b, b.pack_cell([kap]), _t(T))
    err_net = net_flux_error(b.split_pt(_np(bol).reshape(-1, 3))[0], r["F_bol"])
    assert err_net.max() < 1e-10, err_net.max()
    err_sig = net_flux_error_sigma(b.split_pt(_np(bol).reshape(-1, 3))[0], r["F_bol"], atm["T_int"])
    assert err_sig.max() < 1e-10, err_sig.max()
    iso = ref.isothermal_flux(atm, T)  # pi B for D = 2
    assert col_rel_error(to_flux(b.split_cell(_np(F_up))[0], iso), r["F_up"]).max() < 1e-11
    assert col_rel_error(to_flux(b.split_cell(_np(F_dn))[0], iso), r["F_dn"]).max() < 1e-11
    assert col_rel_error(b.split_pb(_np(ub))[0], r["F_up_bin"]).max() < 1e-11
    assert col_rel_error(b.split_pb(_np(db))[0], r["F_dn_bin"]).max() < 1e-11


def test_flux_exact_ragged_batch_equals_single_atmospheres(small_table):
    """A batch of uneven atmospheres gives each one's single-atmosphere result."""
    lc, dl = W.bins(300)
    rng = np.random.default_rng(23)
    atms = [W.spectral_atmosphere(rng, n, lc, dl, nb) for n, nb in ((30, 7), (150, 3), (2, 5))]
    b = H.Batch(atms)
    H.grid(b)
    Ts, kaps = [], []
    for atm in atms:
        P, T, kap = oracle_state(atm, small_table, smooth_profile(atm))
        Ts.append(T)
        kaps.append(kap)
    out = _exact_gpu(b, b.pack_cell(kaps), _t(np.concatenate(Ts)))
    bol = b.split_pt(_np(out[4]).reshape(-1, 3))
    for a, atm in enumerate(atms):
        P = ref.grid(atm["P_c"])
        r = ref.flux_exact(atm, kaps[a], Ts[a], P)
        assert net_flux_error(bol[a], r["F_bol"]).max() < 1e-10
        assert net_flux_error_sigma(bol[a], r["F_bol"], atm["T_int"]).max() < 1e-10
