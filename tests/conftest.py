import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


import pytest  # noqa: E402


@pytest.fixture(scope="session")
def bt():
    """The HIP binding; (re)builds libbtoep.so when it is missing or older than a source."""
    import paper_2407_13066_amd as pkg
    from paper_2407_13066_amd import build
    if build.stale():
        build.build()
    pkg.load_library()
    return pkg
