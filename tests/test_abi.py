"""The C-ABI library loads on the host and exports every entry point its header declares
(no compute calls: those need a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raybornhf.h")
LIB = os.path.join(ROOT, "paper_2211_00316_amd", "libraybornhf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w ]*?[\s\*]+)(rb_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2211_00316_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_five_stages():
    names = declared_functions()
    for n in ("rb_trace_rays", "rb_build_green", "rb_born_forward", "rb_born_adjoint",
              "rb_frequency_step", "rb_backproject", "rb_residual", "rb_create"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_symbol_list_matches_header():
    from paper_2211_00316_amd import _lib

    assert sorted(_lib.SYMBOLS) == declared_functions()


def test_mask_count_matches_oracle(lib):
    from oracle.medium import Grid
    from paper_2211_00316_amd import _lib

    for nx, dx, mr in ((128, 0.8e-3, 0.045), (97, 0.37e-3, 0.0171), (512, 0.45e-3, 0.099)):
        x0 = -(nx - 1) * dx / 2
        g = _lib.Grid(nx, nx, dx, x0, x0, mr)
        assert _lib.mask_count(g) == Grid(nx, nx, dx, x0, x0, mr).mask_index().size


def test_context_without_gpu_fails_loudly():
    import torch

    from paper_2211_00316_amd import _lib

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        _lib.Context()


def test_step_bytes_is_host_arithmetic(lib):
    # rb_step_bytes needs no GPU: positive for a valid geometry, growing with the tracer's
    # sample budget until one launch holds every transducer, 0 for an invalid geometry.
    from paper_2211_00316_amd import _lib

    g = _lib.Grid(128, 128, 0.8e-3, -50.8e-3, -50.8e-3, 0.045)
    r = _lib.Ring(64, 0.05, 0.0)
    tp = _lib.TraceParams(360, 628, 0.2e-3, 1500.0)
    small = _lib.step_bytes(g, r, tp, _lib.RB_BF16, 1 << 24)
    big = _lib.step_bytes(g, r, tp, _lib.RB_BF16, 1 << 34)
    huge = _lib.step_bytes(g, r, tp, _lib.RB_BF16, 1 << 40)
    assert 0 < small < big == huge
    assert _lib.step_bytes(g, r, tp, _lib.RB_F32, 1 << 34) > big   # FP32 operands are wider
    bad = _lib.Grid(0, 128, 0.8e-3, -50.8e-3, -50.8e-3, 0.045)
    assert _lib.step_bytes(bad, r, tp, _lib.RB_BF16, 1 << 30) == 0


def test_workspace_bytes_is_host_arithmetic(lib):
    # rb_workspace_bytes (what rb_reserve allocates) needs no GPU: it covers the step's own
    # buffers, grows with the sample budget until one tracer launch holds every transducer,
    # and is 0 for an invalid geometry or precision.
    from paper_2211_00316_amd import _lib

    g = _lib.Grid(128, 128, 0.8e-3, -50.8e-3, -50.8e-3, 0.045)
    r = _lib.Ring(64, 0.05, 0.0)
    tp = _lib.TraceParams(360, 628, 0.2e-3, 1500.0)
    for prec in (_lib.RB_F32, _lib.RB_BF16, _lib.RB_F16):
        small = _lib.workspace_bytes(g, r, tp, prec, 1 << 24)
        big = _lib.workspace_bytes(g, r, tp, prec, 1 << 34)
        assert 0 < small < big == _lib.workspace_bytes(g, r, tp, prec, 1 << 40)
        # the step buffers and every standalone entry point's workspace, beyond what a
        # context that only steps needs (minus the context's few fixed words)
        assert big >= _lib.step_bytes(g, r, tp, prec, 1 << 34) - 8192
    bad = _lib.Grid(0, 128, 0.8e-3, -50.8e-3, -50.8e-3, 0.045)
    assert _lib.workspace_bytes(bad, r, tp, _lib.RB_BF16, 1 << 30) == 0
    assert _lib.workspace_bytes(g, r, tp, 7, 1 << 30) == 0
