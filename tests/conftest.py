import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def c1():
    from workloads import config_inputs
    return config_inputs("c1")


@pytest.fixture(scope="session")
def gctx():
    """A library context on cuda:0 (GPU tests only)."""
    import torch
    import paper_2307_14437_amd as gofd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = gofd.Context()
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def oracle_csc(tr):
    """Vertex-major structure of the oracle's I: offsets, ascending node numbers, weights."""
    import numpy as np
    d1 = tr.d + 1
    verts = tr.verts.reshape(-1)
    nodes = np.repeat(tr.inside, d1)
    w = tr.lam.reshape(-1)
    order = np.lexsort((nodes, verts))
    off = np.zeros(tr.nv + 1, dtype=np.int64)
    np.add.at(off, verts + 1, 1)
    return np.cumsum(off), nodes[order], w[order]
