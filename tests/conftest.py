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
    """Build the library when it is missing or was built from other sources
    (the build records a hash of its sources next to the library)."""
    from paper_2511_23438_amd import build
    if not build.is_current():
        print("libmpsim.so missing or stale: rebuilding", file=sys.stderr, flush=True)
        build.build()


_ensure_built()
