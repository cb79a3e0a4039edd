import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only checks")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


def pytest_runtest_logstart(nodeid, location):
    # name the case before any GPU work starts, so a hard failure still shows it
    if "gpu" in nodeid:
        print(f"\n[start] {nodeid}", flush=True)


@pytest.fixture(scope="session")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_14467_amd as P

    P.lib()
    return torch.device("cuda:0")
