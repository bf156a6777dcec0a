"""Shared pytest configuration: the ``gpu`` marker and the repository root on
``sys.path`` so ``oracle``, ``workloads`` and the library package import."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: oracle test that takes tens of seconds")
