"""In-place refill of a batch's slots (Solver.refill, Batch.replace): a new
atmosphere put into a finished atmosphere's slot follows the same iteration
as in a batch of its own, the other atmospheres continue as if nothing had
happened, and a graph captured before the refill stays valid."""
import numpy as np
import pytest
import torch

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


@pytest.mark.parametrize("prec", [0, 1])
def test_refilled_slot_follows_a_fresh_solve(prec):
    kt = W.table_ktab(2)
    KT = H.KTable(kt)
    atms, _ = W.learned_workload(5, 4, 0, n=20, nb=40, ktab=kt)
    T0 = lambda sel: np.concatenate([atms[k]["T0"] for k in sel])  # noqa: E731
    s = H.Solver(H.Batch(atms[:3]), KT, prec=prec)
    s.reset(T0([0, 1, 2]))
    for _ in range(5):
        s.step()
    s.capture(6)  # recorded before the refill, replayed after it
    s.refill([1], [atms[3]])
    s.replay()
    torch.cuda.synchronize()
    got = s.b.split_layer(s.T_c.cpu().numpy())
    # the untouched members against the same batch without the refill
    s2 = H.Solver(H.Batch(atms[:3]), KT, prec=prec)
    s2.reset(T0([0, 1, 2]))
    for _ in range(11):
        s2.step()
    torch.cuda.synchronize()
    want = s2.b.split_layer(s2.T_c.cpu().numpy())
    for a in (0, 2):
        np.testing.assert_allclose(got[a], want[a], rtol=1e-13, atol=0)
    # the new member against a batch of its own, six updates from its start
    s3 = H.Solver(H.Batch([atms[3]]), KT, prec=prec)
    s3.reset(atms[3]["T0"])
    for _ in range(6):
        s3.step()
    torch.cuda.synchronize()
    np.testing.assert_allclose(got[1], s3.T_c.cpu().numpy(), rtol=1e-13, atol=0)
    assert int(s.iters[1].item()) == int(s3.iters[0].item()) == 6
    assert s.b.atms[1] is atms[3]


def test_refill_refuses_other_sizes():
    kt = W.table_ktab(2)
    atms, _ = W.learned_workload(5, 2, 0, n=20, nb=40, ktab=kt)
    other, _ = W.learned_workload(5, 1, 2, n=24, nb=40, ktab=kt)
    s = H.Solver(H.Batch(atms), H.KTable(kt), prec=H.FP64)
    with pytest.raises(ValueError):
        s.refill([0], other)
