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


def get_mesh(level):
    """Session cache of generated meshes (input generator output)."""
    from paper_2404_08849_amd.inputs.meshgen import icosahedral_mesh
    if level not in _MESHES:
        _MESHES[level] = icosahedral_mesh(level)
    return _MESHES[level]


@pytest.fixture(scope="session")
def mesh_cache():
    return get_mesh
