import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def tiny_oracle():
    import numpy as np
    import workloads as W
    from oracle import discretise, greens
    arr = W.tiny()
    disc = discretise.Discretisation(arr)
    Z = greens.assemble_dense(disc)
    inc = W.normal_x()
    v = greens.plane_wave_rhs(disc, inc.theta_deg, inc.phi_deg, inc.pol)[:, 0]
    return dict(array=arr, disc=disc, Z=Z, v=v, x_lu=np.linalg.solve(Z, v),
                self_blocks=greens.self_blocks(disc))
