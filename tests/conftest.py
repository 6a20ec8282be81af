import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def video_frames():
    """Frames 0 and 1 of the 1280x720 K=4 ring video (rendered once per session)."""
    import scenes

    c = scenes.config2()
    frames = [c["seq"].frame(t) for t in range(2)]
    return c, frames


@pytest.fixture(scope="session")
def streaming_frame():
    """Frame 0 of the 1920x1080 K=8 streaming workload (rendered once per session)."""
    import scenes

    c = scenes.config5()
    return c, c["seq"].frame(0)
