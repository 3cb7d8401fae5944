"""Production atmospheres at their radiative equilibrium: the GPU flux solve
against the FP64 oracle's at the oracle's own converged profiles.

tests/golden/c5_oracle_flux.npz holds, for the first atmospheres of the
production parameter set (seed 5: 200 layers x 3000 bins x 20 g), the
oracle's converged layer temperatures (Sec. 2.2.4 to 1e-3 sigma T_int^4 from
the isothermal 1000 K start) and its bolometric fluxes at those profiles with
the scattering iteration settled (20 flux solves of 1 + 4 passes from the
isothermal flux, each warm-started from the previous one); it is written by
`python -m oracle.c5_reference golden`, which runs the oracle only.  Here the
same atmospheres, as one batch in the production sweep shape, take the same 20
solves from the same start: FP64 to 1e-10 of the gross flux and of
max(|net|, sigma T_int^4) per point, mixed precision to 1e-4 of the gross flux
and, against max(|net|, sigma T_int^4), to MIXED_SIGMA_TOL or a few float32
roundings of the gross flux where that is larger (the atmospheres with T_int
near 100-150 K: mixed_sigma_bound).
"""
import os

import numpy as np
import pytest
import torch

from gpu_helpers import mixed_sigma_bound, net_flux_error, net_flux_error_sigma
from paper_1606_05474_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle_flux.npz")
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
def golden():
    with np.load(GOLDEN) as d:
        g = {k: d[k] for k in d.files}
    kt = W.table_ktab(2, nbt=int(g["n_bin"]))
    idx = [int(k) for k in g["index"]]
    atms, _ = W.learned_workload(int(g["seed"]), max(idx) + 1, 0, n=int(g["n_layer"]), nb=int(g["n_bin"]), ktab=kt)
    return g, kt, [atms[k] for k in idx]


@pytest.mark.parametrize("prec", [0, 1])
def test_settled_flux_at_the_oracle_equilibrium(prec, golden, monkeypatch):
    monkeypatch.setenv("HELIOS_SWEEP_K", "14")  # the production chunk's sweep shape
    monkeypatch.setenv("HELIOS_SWEEP_L", "32")
    g, kt, atms = golden
    b = H.Batch(atms)
    H.grid(b)
    assert H.sweep_shapes(b, prec) == {208: (14, 32)}
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, b.cat_layer(list(g["T_c"])), T_pt)
    rd = H.rdtype(prec)
    kap = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    H.mix_opacity(b, H.KTable(kt), T_pt, kap, prec)
    F_up = torch.zeros(b.total_cell, dtype=rd, device="cuda")  # deviation form: the isothermal flux
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    ws = torch.zeros(H.workspace_bytes(b, prec), dtype=torch.uint8, device="cuda")
    for _ in range(int(g["calls"])):
        H.flux(b, kap, T_pt, F_up, None, None, bol, ws, n_scat=4, prec=prec)
    torch.cuda.synchronize()
    per_atm = b.split_pt(bol.cpu().numpy().reshape(-1, 3))
    for a, atm in enumerate(atms):
        err = net_flux_error(per_atm[a], g["F_bol"][a]).max()
        sig = net_flux_error_sigma(per_atm[a], g["F_bol"][a], atm["T_int"]).max()
        if prec == 0:
            assert err < 1e-10 and sig < 1e-10, (a, err, sig)
        else:
            assert err < 1e-4 and sig < mixed_sigma_bound(g["F_bol"][a], atm["T_int"]), (a, err, sig)
