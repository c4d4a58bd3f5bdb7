import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped, not failed, where no GPU is visible.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(params=[0, 1], ids=["f32-valu", "f32-mfma"])
def f32_decoder(request):
    """Runs a test with each FP32 decoder form (vector ALUs, matrix cores)."""
    from paper_2101_10994_amd import ngl
    old = ngl.get_option(ngl.OPT_F32_DECODER)
    ngl.set_option(ngl.OPT_F32_DECODER, request.param)
    yield request.param
    ngl.set_option(ngl.OPT_F32_DECODER, old)
