import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    """The FP64 CPU oracle (built here if the shared object is missing)."""
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    O.lib()
    return O


@pytest.fixture(scope="session")
def ionogram_sweep():
    """The 112,400-ray oblique-ionogram sweep (grid, fan, limits)."""
    from paper_2506_18579_amd import synth
    return synth.ionogram_workload(0)


@pytest.fixture(scope="session")
def ionogram_sweep_oracle(orc, ionogram_sweep):
    """Oracle results for every ray of the sweep (traced once per session,
    OpenMP over all host cores) and the re-tracing function of the sweep."""
    from parity import oracle_tracer
    tr = oracle_tracer(orc, ionogram_sweep)
    return tr(*ionogram_sweep.fan.expand()), tr
