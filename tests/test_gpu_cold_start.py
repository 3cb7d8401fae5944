"""The paper's start and warm start of the scattering iteration (Sec. 2.2.3:
the coupled fluxes start at zero, and later temperature steps start from the
fluxes of the previous step), the conversion between the per-g conventions,
the temperature floor and the grid check of the RE step, and full-size
parity in the sweep shape the benchmarks run -- GPU against the FP64 oracle.

Tolerances as in test_gpu_parity: FP64 net flux within 1e-10 of the gross
flux per point (and of max(|net|, sigma T_int^4)), per-g and per-bin fluxes
within 1e-11 of their column's largest value; mixed precision 1e-4 of the
gross flux and MIXED_SIGMA_TOL of max(|net|, sigma T_int^4); converged
profiles within 0.1 K and +-10 updates.
"""
import numpy as np
import pytest
import torch

import oracle as ref
from gpu_helpers import (MIXED_SIGMA_TOL, col_rel_error, net_flux_error, net_flux_error_sigma, oracle_state,
                         smooth_profile, well_conditioned_layers)
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


@pytest.fixture(scope="module")
def small_table():
    return W.table_ktab(2, nbt=300)


def _t(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _np(x):
    return x.detach().cpu().numpy()


def _flux(b, kap, T, prec, F_up, n_scat=4, want_dn=True, layers="noniso"):
    rd = H.rdtype(prec)
    F_dn = torch.zeros(b.total_cell, dtype=rd, device="cuda") if want_dn else None
    ub = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    db = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    ws = torch.zeros(H.workspace_bytes(b, prec), dtype=torch.uint8, device="cuda")
    H.flux(b, kap, T, F_up, ub, db, bol, ws, n_scat=n_scat, F_dn_g=F_dn, prec=prec, layers=layers)
    torch.cuda.synchronize()
    return F_dn, ub, db, bol


def _table_atmosphere(seed, n, nb, small_table):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(seed)
    return W.spectral_atmosphere(rng, n, lc, dl, nb)


# --------------------------------------------------- the zero-flux start
@pytest.mark.parametrize("n,nb,n_scat", [(50, 30, 4), (37, 9, 0), (120, 12, 11)])
def test_zero_flux_start_with_the_flux_state(n, nb, n_scat, small_table):
    """FP64 flux call whose per-g arrays hold fluxes, started from zeros (the
    paper's first scattering pass), against the oracle started from zeros."""
    atm = _table_atmosphere(n, n, nb, small_table)
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap = oracle_state(atm, small_table, T_c)
    up_ref = np.zeros((nb, atm["ng"], 2 * n + 1))
    r = ref.flux(atm, kap, T, P, up_ref, n_scat=n_scat)
    F_up = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    F_dn, ub, db, bol = _flux(b, b.pack_cell([kap]), _t(T), H.FP64 | H.STATE_FLUX, F_up, n_scat=n_scat)
    bol = _np(bol).reshape(-1, 3)
    assert net_flux_error(bol, r["F_bol"]).max() < 1e-10
    assert net_flux_error_sigma(bol, r["F_bol"], atm["T_int"]).max() < 1e-10
    assert col_rel_error(b.split_cell(_np(F_up))[0], up_ref).max() < 1e-11
    assert col_rel_error(b.split_cell(_np(F_dn))[0], r["F_dn"]).max() < 1e-11
    assert col_rel_error(b.split_pb(_np(ub))[0], r["F_up_bin"]).max() < 1e-11
    assert col_rel_error(b.split_pb(_np(db))[0], r["F_dn_bin"]).max() < 1e-11


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_flux_start_in_deviation_form(prec, small_table):
    """The same start for the deviation convention: helios_state_convert
    writes -(2 pi / D) B, the flux call runs in deviations, and converting
    its output back gives the oracle's fluxes (FP64 1e-10 net / 1e-11
    per g; mixed 1e-4 of the gross flux)."""
    n, nb = 60, 20
    atm = _table_atmosphere(3, n, nb, small_table)
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm, 2100.0, 700.0)
    P, T, kap = oracle_state(atm, small_table, T_c)
    up_ref = np.zeros((nb, atm["ng"], 2 * n + 1))
    r = ref.flux(atm, kap, T, P, up_ref)
    T_pt = _t(T)
    rd = H.rdtype(prec)
    F_up = torch.full((b.total_cell,), 12345.0, dtype=rd, device="cuda")  # not read by the zero start
    H.state_convert(b, T_pt, F_up, H.CONVERT_ZERO_FLUX, prec=prec)
    F_dn, ub, db, bol = _flux(b, b.pack_cell([kap], rd), T_pt, prec, F_up)
    bol = _np(bol).reshape(-1, 3)
    H.state_convert(b, T_pt, F_up, H.CONVERT_TO_FLUX, prec=prec)
    H.state_convert(b, T_pt, F_dn, H.CONVERT_TO_FLUX, prec=prec)
    torch.cuda.synchronize()
    err_sig = net_flux_error_sigma(bol, r["F_bol"], atm["T_int"]).max()
    if prec == H.FP64:
        assert net_flux_error(bol, r["F_bol"]).max() < 1e-10
        assert err_sig < 1e-10, err_sig
        assert col_rel_error(b.split_cell(_np(F_up))[0], up_ref).max() < 1e-11
        assert col_rel_error(b.split_cell(_np(F_dn))[0], r["F_dn"]).max() < 1e-11
    else:
        assert net_flux_error(bol, r["F_bol"]).max() < 1e-4
        assert err_sig < MIXED_SIGMA_TOL, err_sig
        assert col_rel_error(b.split_cell(_np(F_up))[0], up_ref).max() < 1e-4


@pytest.mark.parametrize("layers", ["noniso", "iso"])
def test_state_convert_reference_and_round_trip(layers):
    """The conversion's reference is (2 pi / D) B at the bin centre and the
    point temperature (on the isothermal-layer grid: the layer's B at both
    of its points, the top layer's at the TOA point), as the oracle's
    isothermal flux; atmospheres that are not running are left alone."""
    atms = [W.plain_workload(n=n, nb=nb, seed=s)[0] for n, nb, s in ((30, 7, 1), (12, 5, 2))]
    b = H.Batch(atms)
    H.grid(b)
    T_cs = [smooth_profile(a, 1500.0, 600.0) for a in atms]
    T_pts = [ref.profile(ref.grid(a["P_c"]), Tc) for a, Tc in zip(atms, T_cs)]
    T_pt = _t(np.concatenate(T_pts))
    D = 1.8
    x0 = torch.as_tensor(np.random.default_rng(4).normal(0, 1e5, b.total_cell), device="cuda")
    x = x0.clone()
    H.state_convert(b, T_pt, x, H.CONVERT_TO_FLUX, D=D, layers=layers)
    torch.cuda.synchronize()
    for a, atm in enumerate(atms):
        Tp = T_pts[a]
        if layers == "iso":  # reference temperature of each point on the isothermal-layer grid
            n = atm["n"]
            Tp = np.array([Tp[2 * min(p // 2, n - 1) + 1] for p in range(2 * n + 1)])
        iso = ref.isothermal_flux(atm, Tp, D)
        got = b.split_cell(_np(x))[a] - b.split_cell(_np(x0))[a]
        assert np.abs(got - iso[:, None, :]).max() <= 1e-9 * iso.max()
    H.state_convert(b, T_pt, x, H.CONVERT_TO_DEVIATION, D=D, layers=layers)
    torch.cuda.synchronize()
    scale = max(float(ref.isothermal_flux(a, Tp, D).max()) for a, Tp in zip(atms, T_pts))
    assert (x - x0).abs().max().item() <= 1e-15 * scale * 4
    # a frozen atmosphere is skipped
    st = torch.tensor([H.ATM_RUNNING, H.ATM_CONVERGED], dtype=torch.int32, device="cuda")
    y = x0.clone()
    H.state_convert(b.with_status(st), T_pt, y, H.CONVERT_ZERO_FLUX, D=D, layers=layers)
    torch.cuda.synchronize()
    lo, hi = int(b.cell_off[1]), int(b.cell_off[2])
    assert torch.equal(y[lo:hi], x0[lo:hi])
    assert not torch.equal(y[:lo], x0[:lo])


def test_flux_state_warm_start_is_the_previous_fluxes(small_table):
    """Two temperature steps in the flux convention: the second call starts
    from the fluxes the first one left (the paper's warm start), per call
    against the oracle carrying its own fluxes (FP64 1e-10 / 1e-11)."""
    n, nb = 80, 15
    atm = _table_atmosphere(9, n, nb, small_table)
    b = H.Batch([atm])
    H.grid(b)
    T_c = smooth_profile(atm)
    P, T, kap = oracle_state(atm, small_table, T_c)
    up_ref = np.zeros((nb, atm["ng"], 2 * n + 1))
    ref.flux(atm, kap, T, P, up_ref)
    F_up = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    _flux(b, b.pack_cell([kap]), _t(T), H.FP64 | H.STATE_FLUX, F_up)
    T_c2 = T_c + 25.0 * np.cos(np.linspace(0, 5, n))
    P, T2, kap2 = oracle_state(atm, small_table, T_c2)
    r2 = ref.flux(atm, kap2, T2, P, up_ref)
    F_dn, ub, db, bol = _flux(b, b.pack_cell([kap2]), _t(T2), H.FP64 | H.STATE_FLUX, F_up)
    bol = _np(bol).reshape(-1, 3)
    assert net_flux_error(bol, r2["F_bol"]).max() < 1e-10
    assert net_flux_error_sigma(bol, r2["F_bol"], atm["T_int"]).max() < 1e-10
    assert col_rel_error(b.split_cell(_np(F_up))[0], up_ref).max() < 1e-11
    assert col_rel_error(b.split_cell(_np(F_dn))[0], r2["F_dn"]).max() < 1e-11


def test_exact_mode_flux_state_outputs_the_fluxes(small_table):
    """helios_flux_exact with the flux convention writes F = G + pi B: the
    same per-g arrays as the deviation output plus the oracle's pi B."""
    n, nb = 40, 10
    atm = dict(_table_atmosphere(5, n, nb, small_table))
    atm["w0"] = np.zeros_like(atm["w0"])
    b = H.Batch([atm])
    H.grid(b)
    P, T, kap = oracle_state(atm, small_table, smooth_profile(atm))
    outs = []
    for state in (H.STATE_DEVIATION, H.STATE_FLUX):
        F_up = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
        F_dn = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
        bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
        ws = torch.zeros(H.workspace_bytes(b, 0), dtype=torch.uint8, device="cuda")
        H.flux_exact(b, b.pack_cell([kap]), _t(T), F_up, F_dn, None, None, bol, ws, state=state)
        torch.cuda.synchronize()
        outs.append((b.split_cell(_np(F_up))[0], b.split_cell(_np(F_dn))[0], _np(bol)))
    piB = ref.isothermal_flux(atm, T, 2.0)[:, None, :]
    assert np.array_equal(outs[0][2], outs[1][2])
    assert col_rel_error(outs[1][0], outs[0][0] + piB).max() < 1e-15
    assert col_rel_error(outs[1][1], outs[0][1] + piB).max() < 1e-15
    r = ref.flux_exact(atm, kap, T, P)
    assert col_rel_error(outs[1][0], r["F_up"]).max() < 1e-11


# ------------------------------------------------ RE loops from the paper's start
def test_plain_re_solve_follows_the_oracle_iteration():
    """The plain FP64 workload with the paper's start and warm start on both
    sides: the first temperature steps agree per step, the converged profile
    within 0.1 K and the number of updates within 10."""
    atm, kt = W.plain_workload()
    steps = []
    sol = ref.solve(atm, kt, max_iter=200, callback=lambda it, T_c, r: steps.append(T_c.copy()))
    assert sol["converged"]
    b = H.Batch([atm])
    s = H.Solver(b, H.KTable(kt), prec=H.FP64)
    assert s.state == "flux" and s.start == "zero"
    s.reset(atm["T0"])
    for k in range(5):
        s.step()
        torch.cuda.synchronize()
        assert np.abs(_np(s.T_c) - steps[k]).max() < 1e-6, k
    conv, iters = s.solve(atm["T0"], max_iter=200)
    assert conv[0]
    assert np.abs(_np(s.T_c) - sol["T_c"]).max() < 0.1
    assert abs(int(iters[0]) - sol["iterations"]) <= 10, (iters[0], sol["iterations"])


def test_deviation_warm_start_reaches_the_paper_profile():
    """The deviation convention between temperature steps (from the same
    zero-flux start) changes the trajectory, not the fixed point: against
    the oracle's paper reading, 0.1 K and +-10 updates."""
    atm, kt = W.plain_workload()
    sol = ref.solve(atm, kt, max_iter=200)
    b = H.Batch([atm])
    s = H.Solver(b, H.KTable(kt), prec=H.FP64, state="deviation")
    conv, iters = s.solve(atm["T0"], max_iter=200)
    assert conv[0] and sol["converged"]
    assert np.abs(_np(s.T_c) - sol["T_c"]).max() < 0.1
    assert abs(int(iters[0]) - sol["iterations"]) <= 10, (iters[0], sol["iterations"])


def test_mixed_precision_reaches_the_paper_profile():
    """Mixed precision (deviation convention, zero-flux start) against the
    oracle's paper reading: within 0.1 K over the well-conditioned layers
    (27 of the 50 here).  The optically thick bottom layers and the thin
    upper ones, whose divergence hardly depends on their own temperature,
    are weakly determined by the convergence test and are not held to it
    (measured: up to 12 K at the top layer of this workload)."""
    atm, kt = W.plain_workload()
    sol = ref.solve(atm, kt, max_iter=300)
    assert sol["converged"]
    b = H.Batch([atm])
    s = H.Solver(b, H.KTable(kt), prec=H.MIXED)
    conv, iters = s.solve(atm["T0"], max_iter=300)
    assert conv[0]
    dT = np.abs(_np(s.T_c) - sol["T_c"])
    ok = well_conditioned_layers(atm, kt, sol)
    # the excluded layers and their differences (shown with pytest -s)
    print("excluded layers, |dT| K:", {int(i): round(float(dT[i]), 4) for i in np.where(~ok)[0]})
    assert ok.sum() >= atm["n"] // 2, ok.sum()
    assert dT[ok].max() < 0.1, (dT[ok].max(), dT.max(), np.argmax(dT))


# ------------------------------------------------------------- RE step edges
def test_radeq_floor_matches_the_oracle_bit_for_bit():
    """Layers whose step would take them below 10 K (Sec. 2.2.4 leaves the
    bound open; both sides floor at 10 K) end exactly at the floor, with the
    step multipliers and sign histories of the oracle bit for bit."""
    atm = W.plain_workload(n=30, nb=4)[0]
    n = atm["n"]
    b = H.Batch([atm])
    H.grid(b)
    P = ref.grid(atm["P_c"])
    rng = np.random.default_rng(17)
    T_c = smooth_profile(atm, 900.0, 300.0)
    cold = np.array([3, 11, 12, 25])
    T_c[cold] = [14.0, 11.0, 25.0, 10.5]
    net = 9e4 + np.cumsum(rng.normal(0, 2e4, 2 * n + 1))
    for i in cold:  # the net flux grows across these layers: they cool
        net[2 * i + 2:] += 5e4
    F = np.zeros((2 * n + 1, 3))
    F[:, 0] = 4e8 + net
    F[:, 1] = 4e8
    F[:, 2] = F[:, 0] - F[:, 1]
    m0 = rng.uniform(0.5, 2.0, n)
    h0 = ((rng.integers(0, 7, n) << 16) | rng.integers(0, 64, n)).astype(np.int32)
    T_d, m_d, h_d = _t(T_c), _t(m0), _t(h0, torch.int32)
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    H.radeq(b, _t(F.ravel()), T_d, T_pt, m_d, h_d, status)
    torch.cuda.synchronize()
    T_ref, m_ref, h_ref = T_c.copy(), m0.copy(), h0.copy()
    code, _ = ref.radeq(atm, P, F, T_ref, m_ref, h_ref)
    assert code == 0
    floored = T_ref == 10.0
    assert floored[cold].all(), T_ref[cold]
    T_got = _np(T_d)
    assert np.array_equal(T_got[floored], T_ref[floored])
    np.testing.assert_allclose(T_got[~floored], T_ref[~floored], rtol=0, atol=1e-9)
    np.testing.assert_allclose(_np(m_d), m_ref, rtol=1e-15)
    np.testing.assert_array_equal(_np(h_d), h_ref)
    np.testing.assert_allclose(_np(T_pt), ref.profile(P, T_ref), rtol=1e-14)


def test_radeq_flags_a_pressure_grid_that_does_not_decrease():
    """Layer-centre pressures that do not decrease from the bottom up (the
    grid of Sec. 2.2.1 is ordered BOA -> TOA) set the atmosphere's status
    to BADGRID; nothing of it moves, the rest of the batch steps as usual,
    and the oracle's step refuses the same grid."""
    good, kt = W.plain_workload(n=20, nb=6)
    bad = dict(good)
    bad["P_c"] = np.array(good["P_c"], np.float64)
    bad["P_c"][[7, 8]] = bad["P_c"][[8, 7]]
    b = H.Batch([good, bad])
    H.grid(b)
    s = H.Solver(b, H.KTable(kt), prec=H.FP64)
    s.reset(np.concatenate([good["T0"], bad["T0"]]))
    s.step()
    torch.cuda.synchronize()
    assert list(_np(s.status)) == [H.ATM_RUNNING, H.ATM_BADGRID]
    T_bad = b.split_layer(_np(s.T_c))[1].copy()
    assert np.all(T_bad == bad["T0"])
    bol1 = _np(s.F_bol).copy()
    s.step()
    torch.cuda.synchronize()
    assert list(_np(s.status)) == [H.ATM_RUNNING, H.ATM_BADGRID]
    assert np.all(b.split_layer(_np(s.T_c))[1] == T_bad)
    # the flux call skips the flagged atmosphere: its fluxes stay as they were
    lo, hi = 3 * int(b.pt_off[1]), 3 * int(b.pt_off[2])
    # (the first call ran on the bad grid before the step flagged it: NaN where dtau < 0)
    assert np.array_equal(_np(s.F_bol)[lo:hi], bol1[lo:hi], equal_nan=True)
    P_bad = ref.grid(bad["P_c"])
    F = np.zeros((2 * bad["n"] + 1, 3))
    code, _ = ref.radeq(bad, P_bad, F, np.array(bad["T0"], np.float64), np.ones(bad["n"]),
                        np.zeros(bad["n"], np.int32))
    assert code == -2


# ------------------------------------------ full size, in the benchmark's shape
@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_spectral_atmosphere_in_the_benchmark_shape(prec, monkeypatch):
    """The single-atmosphere spectral workload (100 layers x 3000 bins x 20 g,
    four 20 x 20 float32 tables) with the sweep forced to the shape the
    benchmark's autotuner picks for it (14 sublayers per lane, 16 lanes per
    column): the whole flux call against the oracle on the same opacities
    (FP64 1e-10, mixed 1e-4 relative net flux; FP64 per-g fluxes 1e-11)."""
    monkeypatch.setenv("HELIOS_SWEEP_K", "14")
    monkeypatch.setenv("HELIOS_SWEEP_L", "16")
    kt = W.table_ktab(2)
    atm, _ = W.spectral_workload(ktab=kt)
    b = H.Batch([atm])
    H.grid(b)
    assert H.sweep_shapes(b, prec) == {112: (14, 16)}
    T_c = smooth_profile(atm, 2000.0, 800.0)
    P, T, kap_ref = oracle_state(atm, kt, T_c)
    up_ref = np.zeros((len(atm["lambda_c"]), atm["ng"], 2 * atm["n"] + 1))
    r = ref.flux(atm, kap_ref, T, P, up_ref, want_dn=False)
    rd = H.rdtype(prec)
    kap = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    T_pt = _t(T)
    H.mix_opacity(b, H.KTable(kt), T_pt, kap, prec)
    F_up = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    H.state_convert(b, T_pt, F_up, H.CONVERT_ZERO_FLUX, prec=prec)
    _, ub, db, bol = _flux(b, kap, T_pt, prec, F_up, want_dn=False)
    bol = _np(bol).reshape(-1, 3)
    err = net_flux_error(bol, r["F_bol"])
    if prec == H.FP64:
        assert err.max() < 1e-10, err.max()
        assert net_flux_error_sigma(bol, r["F_bol"], atm["T_int"]).max() < 1e-10
        H.state_convert(b, T_pt, F_up, H.CONVERT_TO_FLUX, prec=prec)
        torch.cuda.synchronize()
        assert col_rel_error(b.split_cell(_np(F_up))[0], up_ref).max() < 1e-11
        assert col_rel_error(b.split_pb(_np(ub))[0], r["F_up_bin"]).max() < 1e-11
    else:
        assert err.max() < 1e-4, err.max()
        err_sig = net_flux_error_sigma(bol, r["F_bol"], atm["T_int"]).max()
        assert err_sig < MIXED_SIGMA_TOL, err_sig


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_production_atmospheres_in_the_chunk_shape(prec, monkeypatch):
    """Three production atmospheres (200 layers x 3000 bins x 20 g, seed 5)
    as one batch, with the sweep in the shape the production chunk runs (14
    sublayers per lane, 32 lanes per column: the DPP-row scans and their
    row join): two flux calls from the paper's zero-flux start at a fixed
    non-isothermal profile, each against the oracle on the same inputs
    (FP64 1e-10, mixed 1e-4 relative net flux, per atmosphere and point)."""
    monkeypatch.setenv("HELIOS_SWEEP_K", "14")
    monkeypatch.setenv("HELIOS_SWEEP_L", "32")
    kt = W.table_ktab(2)
    atms, _ = W.learned_workload(5, 3, 0, n=200, nb=3000, ktab=kt)
    b = H.Batch(atms)
    H.grid(b)
    assert H.sweep_shapes(b, prec) == {208: (14, 32)}
    T_c = [smooth_profile(a, 2200.0 - 200.0 * k, 600.0 + 100.0 * k) for k, a in enumerate(atms)]
    refs = []
    for a, atm in enumerate(atms):
        P, T, kap_ref = oracle_state(atm, kt, T_c[a])
        up = np.zeros((len(atm["lambda_c"]), atm["ng"], 2 * atm["n"] + 1))
        r1 = ref.flux(atm, kap_ref, T, P, up, want_dn=False)
        r2 = ref.flux(atm, kap_ref, T, P, up, want_dn=False)  # warm start: the first call's fluxes
        refs.append((r1["F_bol"], r2["F_bol"]))
    rd = H.rdtype(prec)
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(T_c), T_pt)
    kap = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    H.mix_opacity(b, H.KTable(kt), T_pt, kap, prec)
    F_up = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    H.state_convert(b, T_pt, F_up, H.CONVERT_ZERO_FLUX, prec=prec)
    tol = 1e-10 if prec == H.FP64 else 1e-4
    for call in range(2):
        _, _, _, bol = _flux(b, kap, T_pt, prec, F_up, want_dn=False)
        per_atm = b.split_pt(_np(bol).reshape(-1, 3))
        for a, atm in enumerate(atms):
            err = net_flux_error(per_atm[a], refs[a][call])
            assert err.max() < tol, (call, a, err.max())
            err_sig = net_flux_error_sigma(per_atm[a], refs[a][call], atm["T_int"]).max()
            assert err_sig < (1e-10 if prec == H.FP64 else MIXED_SIGMA_TOL), (call, a, err_sig)
