import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def tiny_graph():
    from paper_2512_11606_amd import synth
    return synth.make_graph("tiny")


@pytest.fixture(scope="session")
def tiny_oracle(tiny_graph):
    import oracle
    return oracle.OracleGraph.from_graph(tiny_graph)


@pytest.fixture(scope="session")
def tiny_Pi(tiny_graph):
    import oracle
    return oracle.exact_dense(tiny_graph)
