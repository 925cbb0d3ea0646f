import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


def _ensure_built():
    lib = os.path.join(ROOT, "paper_2511_23438_amd", "libmpsim.so")
    if not os.path.exists(lib):
        from paper_2511_23438_amd import build
        build.build()


_ensure_built()
