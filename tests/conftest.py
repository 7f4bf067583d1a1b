import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_sessionstart(session):
    # load what is built; build only when nothing is
    lib = os.path.join(ROOT, "paper_2005_10494_amd", "libbmd.so")
    if not os.path.exists(lib):
        from paper_2005_10494_amd import build
        build.build()
