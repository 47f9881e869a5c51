import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


COS25 = np.float32(np.cos(np.radians(25.0)))


@pytest.fixture(scope="session")
def scene256():
    import scenegen
    s = scenegen.make_scene(1, 8, 0)
    return s, scenegen.render_gbuffer(s, scenegen.orbit_view(0), 256, 256)
