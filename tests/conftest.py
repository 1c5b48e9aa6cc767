"""Shared pytest configuration.

Markers
  gpu   needs an MI355X (gfx950) GPU and the built HIP library; skipped when
        torch sees no GPU.  Everything else runs on the CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible to torch")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def read_golden(name):
    """Non-comment, non-blank lines of tests/golden/<name>."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.lstrip().startswith("#")]


def parse_scheme():
    """The one-level scheme fixture as a list of (A terms, B terms, C terms),
    each a list of (quadrant, sign)."""
    out = []
    for ln in read_golden("strassen_one_level.txt"):
        parts = [p.split() for p in ln.split("|")]
        name, groups = parts[0][0], parts[1:]
        terms = [[(int(t[1:]), 1 if t[0] == "+" else -1) for t in g] for g in groups]
        out.append((name, terms[0], terms[1], terms[2]))
    return out
