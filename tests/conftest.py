import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle cases that take more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def kl_basis_small():
    """Oracle KL basis (64 modes of the workload kernel) on small grids, computed once per session."""
    from oracle import kl
    import workloads as W
    f = W.KS_FIELD
    lam, B = kl.basis(f["sigma2"], f["corr_len"], f["n_modes"], [4, 8, 16, 32, 64], ref_n=64)
    return lam, B
