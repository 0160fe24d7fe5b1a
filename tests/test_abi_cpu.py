"""CPU-only checks of the C ABI: the library loads, exports every function
include/pa.h declares, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def _lib():
    from paper_2602_14016_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_2602_14016_amd import build
        build.build(verbose=False)
    return native.load(), native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ["pa_init_field", "pa_forward", "pa_adjoint_gradient", "pa_precondition", "pa_assimilate",
                     "pa_create", "pa_destroy", "pa_workspace_bytes", "pa_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib, native = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in native.EXPORTS, name


def test_create_validates_before_device_calls():
    lib, nv = _lib()
    out = ctypes.c_void_p()
    good = nv.Physics(1e-3, 0.0, 5e-3, 0.0, 4, 0)
    cases = [
        (good, 7, 1),       # not a power of two
        (good, 2048, 1),    # too large
        (good, 4, 1),       # too small
        (good, 64, 0),      # no members
        (good, 8, 65536),   # more members than the launch grid's second dimension holds
        (nv.Physics(-1.0, 0.0, 5e-3, 0.0, 4, 0), 64, 1),
        (nv.Physics(1e-3, -0.1, 5e-3, 0.0, 4, 0), 64, 1),
        (nv.Physics(1e-3, 0.0, 0.0, 0.0, 4, 0), 64, 1),
        (nv.Physics(1e-3, 0.0, float("nan"), 0.0, 4, 0), 64, 1),
        (nv.Physics(1e-3, 0.0, 5e-3, 1.0, 40, 0), 64, 1),   # forcing wavenumber beyond N/2
        (nv.Physics(1e-3, 0.0, 5e-3, 0.0, 4, 1), 64, 1),    # reserved field set
    ]
    for phys, N, B in cases:
        rc = lib.pa_create(ctypes.byref(phys), N, B, None, ctypes.byref(out))
        assert rc == -1, (N, B, rc)
        assert out.value is None
        assert lib.pa_last_error()
    assert lib.pa_create(None, 64, 1, None, ctypes.byref(out)) == -1
    assert lib.pa_create(ctypes.byref(good), 64, 1, None, None) == -1


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib, nv = _lib()
    out = ctypes.c_void_p()
    good = nv.Physics(1e-3, 0.0, 5e-3, 0.0, 4, 0)
    assert lib.pa_create(ctypes.byref(good), 64, 1, None, ctypes.byref(out)) == -3
    assert out.value is None


def test_null_context_calls_are_rejected():
    lib, nv = _lib()
    b = ctypes.c_size_t()
    assert lib.pa_destroy(None) == 0
    assert lib.pa_workspace_bytes(None, 10, 5, 1, 0, ctypes.byref(b)) == -1
    assert lib.pa_checkpoint_bytes(None, 10, 5, ctypes.byref(b)) == -1
    assert lib.pa_forward(None, None, 1, None, None, None, None, 1, None, None, 0) == -1
    assert lib.pa_adjoint_gradient(None, None, 1, None, None, None, 1, None, 0) == -1
    assert lib.pa_precondition(None, None, 0.5, None, None, None, 0) == -1
    assert lib.pa_assimilate(None, None, 1, None, None, 0, 1, 1, 1, None, None, None, 0) == -1
    assert lib.pa_set_tiles(None, None) == -1
    assert lib.pa_get_tiles(None, None) == -1


def test_product_path_has_no_cpu_fallback():
    # the package never imports the oracle and fails loudly without the library
    import paper_2602_14016_amd
    pkg = os.path.dirname(paper_2602_14016_amd.__file__)
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f
    from paper_2602_14016_amd import native
    with pytest.raises(RuntimeError):
        native.load(os.path.join(pkg, "does_not_exist.so"))
