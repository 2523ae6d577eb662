"""The C-ABI library loads and exports every function include/mttkrp.h declares
(no compute call: runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mttkrp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mttkrp", "gram_solve", "als_sweep", "mtk_create", "mtk_destroy", "mtk_check",
              "mtk_quantize_fp8", "mtk_server_create", "mtk_server_submit", "mtk_server_poll"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2411_04785_amd import mttkrp as b
    if not os.path.exists(b.LIB_PATH):
        pytest.fail("libmttkrp.so not built (python -m paper_2411_04785_amd.build)")
    L = ctypes.CDLL(b.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(declared_functions()) == sorted(b.EXPORTED)


def test_invalid_arguments_rejected_without_gpu():
    from paper_2411_04785_amd import mttkrp as b
    L = b.lib()
    assert L.mtk_create(None, 0) == b.MTK_EINVAL
    assert L.mtk_destroy(None) == b.MTK_OK
    assert L.mtk_last_error(None) == b"NULL context"


def test_dimtree_choice_without_gpu():
    # Host-only query: the sweep forms Y = X x3 C for FP32 / bf16x3 when K >= 8 R.
    from paper_2411_04785_amd.mttkrp import Context
    assert Context.sweep_uses_dimtree((512, 512, 512), 32, "fp32")
    assert Context.sweep_uses_dimtree((1024, 1024, 1024), 64, "bf16x3")
    assert Context.sweep_uses_dimtree((40, 36, 32), 4, "fp32")
    assert not Context.sweep_uses_dimtree((40, 36, 31), 4, "fp32")
    assert not Context.sweep_uses_dimtree((768, 768, 768), 128, "fp8")
    assert not Context.sweep_uses_dimtree((512, 512, 512), 0, "fp32")
    assert not Context.sweep_uses_dimtree((512, 512, 512), 129, "fp32")
