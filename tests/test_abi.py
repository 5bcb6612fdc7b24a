"""Host-side checks of the C ABI: the library loads without a GPU and exports
every function include/mgx.h declares; the oracle and the product share no
code."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    from paper_2411_03040_amd import mgx
    names = mgx.header_functions()
    assert "mgx_formal_solve" in names and "mgx_iterate" in names and len(names) >= 18
    L = mgx.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2411_03040_amd import mgx
    src = open(os.path.join(ROOT, "paper_2411_03040_amd", "mgx.py")).read()
    for n in mgx.header_functions():
        assert f'"{n}"' in src, n


def test_product_does_not_touch_oracle():
    pkg = os.path.join(ROOT, "paper_2411_03040_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "liboracle" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2411_03040_amd" not in text or f == "__init__.py", f
            assert "mgx_internal" not in text and "mgx.h" not in text, f


def test_create_without_gpu_fails_cleanly():
    from paper_2411_03040_amd import mgx
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present: covered by the GPU tests")
    except ImportError:
        pass
    with pytest.raises(mgx.MgxError) as e:
        mgx.Context(device=0, use_torch_stream=False)
    assert e.value.status == mgx.MGX_EINVAL
