import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long oracle runs")


def pytest_sessionstart(session):
    """Build the HIP library once if it is missing (hipcc cross-compiles for
    gfx950 without a GPU); the tests then load what is built."""
    lib = os.path.join(ROOT, "paper_2508_06678_amd", "libqg.so")
    if not os.path.exists(lib):
        from paper_2508_06678_amd import build
        build.build()
