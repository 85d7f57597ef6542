import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


_MESHES = {}


def get_mesh(level, trisections=0):
    """Session cache of generated meshes (input generator output)."""
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    key = (level, trisections)
    if key not in _MESHES:
        _MESHES[key] = icosahedral_mesh(level, trisections=trisections)
    return _MESHES[key]


@pytest.fixture(scope="session")
def mesh_cache():
    return get_mesh
