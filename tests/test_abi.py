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


def test_options_checked_before_the_device():
    """Invalid options fail with MGX_EINVAL before any HIP call, so this
    runs without a GPU: a branch threshold of 0 (every segment would take the
    semi-analytic form, including unshifted ones, dividing by a zero shift)
    and one below the stated minimum."""
    from paper_2411_03040_amd import mgx
    L = mgx.lib()
    for thr in (0.0, 0.05, float("nan")):
        o = mgx.Options()
        L.mgx_default_options(ctypes.byref(o))
        o.branch_threshold = thr
        h = ctypes.c_void_p()
        st = L.mgx_create(ctypes.byref(h), 0, None, ctypes.byref(o))
        assert st == mgx.MGX_EINVAL
        assert L.mgx_last_error(None) == b"invalid options"
        st = L.mgx_batch_create(ctypes.byref(h), 0, None, ctypes.byref(o))
        assert st == mgx.MGX_EINVAL
        assert L.mgx_batch_last_error(None) == b"invalid options"


def test_formal_solve_shape_fits_lds():
    """One bin per line and 2016 lines: the line chunk is capped so the LDS
    staging fits (the workgroup would otherwise stage 1024 lines per
    record); the usual workloads keep their shape (every line of the outflow
    and the clumpy cloud in one workgroup).  The record chunk is sized to
    share a CU's 160 KiB among the workgroups it holds."""
    from paper_2411_03040_amd import mgx
    for prec in (mgx.FP32, mgx.FP64):
        nlc, nth, lds = mgx.formal_solve_shape(prec, 2016, 1)
        assert lds <= 160 * 1024 - 1024 and nth % 64 == 0 and nth >= nlc and nlc >= 1
        for nl, nb in ((9, 31), (19, 39), (1, 1024), (1, 1), (300, 7)):
            nlc, nth, lds = mgx.formal_solve_shape(prec, nl, nb)
            assert lds <= 160 * 1024 - 1024 and nth <= 1024 and nth >= nlc * nb
    assert mgx.formal_solve_shape(mgx.FP32, 9, 31)[0] == 9
    assert mgx.formal_solve_shape(mgx.FP32, 19, 39)[0] == 19
    assert mgx.formal_solve_shape(mgx.FP64, 9, 31)[0] == 9
    with pytest.raises(mgx.MgxError):
        mgx.formal_solve_shape(mgx.FP32, 1, 1025)


def test_profile_code_hash_ignores_comments_only(tmp_path):
    """The committed kernel profiles are keyed to a hash of the kernel code
    with comments and whitespace stripped: comment edits keep a profile
    valid, any code edit invalidates it."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = ("// header\n__global__ void k(float *x) { /* block\n comment */\n"
           "    x[0] = 1.0f;  // trailing\n}\n")
    a = tmp_path / "a.hip"
    a.write_text(src)
    b = tmp_path / "b.hip"
    b.write_text(src.replace("// trailing", "// other words").replace("// header", "")
                 .replace("    x[0]", "  x[0]"))
    c = tmp_path / "c.hip"
    c.write_text(src.replace("1.0f", "2.0f"))
    assert bench.code_sha256(str(a)) == bench.code_sha256(str(b))
    assert bench.code_sha256(str(a)) != bench.code_sha256(str(c))
