import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.build(force=False)
    return O


@pytest.fixture(autouse=True)
def _announce(request):
    # names the running case on the real stderr before any GPU work starts, so that a
    # run that dies mid-test still shows which case it was
    if request.node.get_closest_marker("gpu") is not None:
        sys.__stderr__.write("\n[gpu-case] %s\n" % request.node.nodeid)
        sys.__stderr__.flush()
    yield


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01584_amd import gd
    gd.lib()  # fails loudly when libgd.so is missing
    return torch.device("cuda:0")
