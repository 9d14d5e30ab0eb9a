import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds")


@pytest.fixture(scope="session")
def cube4():
    import workloads as w
    from oracle import fem

    p = w.unit_cube_problem(4, freq=1.0)
    return p, fem.Mesh(p.tets, p.coords, p.face_bc)
