import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def _ensure_host_libs():
    """Build the C oracle / generator libraries if they are missing (gcc, seconds)."""
    need = [os.path.join(ROOT, "oracle", "libaxo.so"), os.path.join(ROOT, "synth", "libaxsynth.so")]
    if all(os.path.exists(p) for p in need):
        return
    import __graft_entry__

    __graft_entry__.build_host()


_ensure_host_libs()
