import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def small_cfg():
    from paper_2401_15758_amd import inputs
    return dict(inputs.CFG_SMALL)


@pytest.fixture(scope="session")
def small_problem(small_cfg):
    from oracle.problem import burgers_problem
    from paper_2401_15758_amd import inputs
    return burgers_problem(small_cfg, inputs.draws(small_cfg, seed=0))


@pytest.fixture(scope="session")
def small_dense(small_problem):
    """Dense data-misfit Hessian H (n x n) of the 128-point problem at x_b."""
    import numpy as np
    p = small_problem
    traj = p.fwd(p.xb)
    Hd = p.misfit_hessian(traj, np.eye(p.n))
    return traj, 0.5 * (Hd + Hd.T), Hd
