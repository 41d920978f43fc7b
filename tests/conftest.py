import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    """GPU tests are skipped, with the reason, where no GPU is visible; they
    still fail loudly on a GPU machine whose HIP library is missing."""
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover - torch is part of the image
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible in this process")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def pytest_terminal_summary(terminalreporter):
    """Largest strict elementwise gradient errors the parity checks saw."""
    parity = sys.modules.get("parity")
    rep = getattr(parity, "STRICT_REPORT", None)
    if rep:
        terminalreporter.write_line(
            "gradient parity: %d checks; strict elementwise relative error "
            "max %.3e on non-cancelling samples (%d samples), max %.3e on all samples"
            % (len(rep), max(r["strict_max"] for r in rep), sum(r["n_plain"] for r in rep),
               max(r["strict_all"] for r in rep)))
