import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def tiny():
    from workloads import get_workload
    from workloads.cameras import pack_cameras
    import oracle
    w = get_workload("tiny")
    scene = w.make_scene()
    cams = pack_cameras(w.cameras())
    V = oracle.view_map(w.display)
    return w, scene, cams, V
