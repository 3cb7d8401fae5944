import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionstart(session):
    # The oracle is plain C; make sure the shared object matches its source.
    import oracle  # noqa: F401  (test infrastructure)

    oracle._load()


@pytest.fixture(scope="session")
def ref():
    import oracle

    return oracle


@pytest.fixture(autouse=True)
def _fresh_sweep_shapes(request):
    """Every GPU test starts from the default sweep shapes: shapes another
    test tuned (helios_autotune keeps them for the process) are forgotten."""
    if request.node.get_closest_marker("gpu") is not None:
        from paper_1606_05474_amd import helios

        helios.autotune_reset()
    yield
