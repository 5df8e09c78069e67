import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O
    if not os.path.exists(O._LIB_PATH):
        O.build()
    return O


@pytest.fixture(scope="session")
def sts_mod():
    """The HIP library's binding (skips without a GPU)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_04243_amd import sts
    sts.lib()
    return sts


@pytest.fixture(scope="session")
def oracle_run(oracle_lib):
    """Oracle of a named workload after its configured run from its seeded
    state, cached for the session (several GPU tests compare against it)."""
    from paper_1802_04243_amd import workloads as W
    cache = {}

    def get(name, scheme):
        key = (name, scheme)
        if key not in cache:
            p, run = W.workload(name)
            o = oracle_lib.Oracle(p)
            o.set_fields(*W.initial_fields(p, run["seed"]))
            for _ in range(run["steps"]):
                o.step(run["dt"], run["inner"], scheme)
            cache[key] = o
        return cache[key]
    return get
