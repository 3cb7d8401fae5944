"""helios_flux_noalloc (the flux solve on the library's static device
workspace, for callers that cannot allocate) against helios_flux on a
caller-owned workspace, through the C ABI: identical inputs give identical
results, on two calls in a row whose second batch is smaller (the second
call finds the first one's contents in the shared array), in FP64 and in
mixed precision; a batch whose workspace exceeds the static size is refused
with nothing written."""
import numpy as np
import pytest
import torch

from gpu_helpers import smooth_profile
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


def _atmospheres(sizes, seed):
    lc, dl = W.bins(300)
    rng = np.random.default_rng(seed)
    return [W.spectral_atmosphere(rng, n, lc, dl, nb) for n, nb in sizes]


def _inputs(b, kt, prec):
    """Opacities, point temperatures and a non-trivial warm start of the batch."""
    H.grid(b)
    T_c = b.cat_layer([smooth_profile(a, 1500.0 + 30 * k, 700.0) for k, a in enumerate(b.atms)])
    T_pt = torch.zeros(b.total_pt, dtype=torch.float64, device="cuda")
    H.profile(b, T_c, T_pt)
    kap = torch.zeros(b.total_cell, dtype=H.rdtype(prec), device="cuda")
    H.mix_opacity(b, H.KTable(kt), T_pt, kap, prec)
    g = torch.Generator(device="cuda").manual_seed(5)
    F0 = (torch.rand(b.total_cell, generator=g, device="cuda", dtype=torch.float64) * 1e3).to(H.rdtype(prec))
    return kap, T_pt, F0


def _run(b, kap, T_pt, F0, prec, noalloc):
    rd = H.rdtype(prec)
    F_up = F0.clone()
    F_dn = torch.zeros(b.total_cell, dtype=rd, device="cuda")
    ub = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    db = torch.zeros(b.total_pb, dtype=torch.float64, device="cuda")
    bol = torch.zeros(b.total_pt * 3, dtype=torch.float64, device="cuda")
    if noalloc:
        H.flux_noalloc(b, kap, T_pt, F_up, ub, db, bol, n_scat=4, F_dn_g=F_dn, prec=prec)
    else:
        ws = torch.full((H.workspace_bytes(b, prec),), 0xA5, dtype=torch.uint8, device="cuda")
        H.flux(b, kap, T_pt, F_up, ub, db, bol, ws, n_scat=4, F_dn_g=F_dn, prec=prec)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (F_up, F_dn, ub, db, bol)]


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_flux_equals_flux_on_two_calls(prec):
    kt = W.table_ktab(2, nbt=300)
    big = H.Batch(_atmospheres([(60, 40), (37, 9), (120, 17)], seed=31))
    small = H.Batch(_atmospheres([(20, 6)], seed=32))
    assert H.workspace_bytes(small, prec) < H.workspace_bytes(big, prec) <= H.NOALLOC_WS_BYTES
    for b in (big, small):  # the second call is the smaller batch
        kap, T_pt, F0 = _inputs(b, kt, prec)
        got = _run(b, kap, T_pt, F0, prec, noalloc=True)
        want = _run(b, kap, T_pt, F0, prec, noalloc=False)
        for name, x, y in zip(("F_up_g", "F_dn_g", "F_up_bin", "F_dn_bin", "F_bol"), got, want):
            assert np.all(np.isfinite(y)), name
            assert np.array_equal(x, y), (name, float(np.max(np.abs(x.astype(np.float64) - y))))


def test_noalloc_flux_refuses_a_batch_beyond_the_static_workspace():
    lc, dl = W.bins(3000)
    rng = np.random.default_rng(33)
    atm = W.spectral_atmosphere(rng, 100, lc, dl, 3000)
    b = H.Batch([atm])
    assert H.workspace_bytes(b, H.FP64) > H.NOALLOC_WS_BYTES
    H.grid(b)
    kap = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    T_pt = torch.full((b.total_pt,), 1000.0, dtype=torch.float64, device="cuda")
    F_up = torch.zeros(b.total_cell, dtype=torch.float64, device="cuda")
    bol = torch.full((b.total_pt * 3,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HeliosError) as e:
        H.flux_noalloc(b, kap, T_pt, F_up, None, None, bol, prec=H.FP64)
    assert e.value.code == -4
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(bol == -7.0))
