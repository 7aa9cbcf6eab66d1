"""Every module of the package, the benchmark and the entry points import
without a GPU (catches syntax and import errors in code the CPU tests do not
otherwise run)."""
import importlib
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name", ["paper_1905_02142_amd", "paper_1905_02142_amd.soap", "paper_1905_02142_amd.md",
                                  "paper_1905_02142_amd.autograd", "paper_1905_02142_amd.speedtest",
                                  "paper_1905_02142_amd.build", "bench", "__graft_entry__", "synth"])
def test_module_imports(name):
    pytest.importorskip("torch")
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    importlib.import_module(name)
