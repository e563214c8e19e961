"""C ABI checks that need no GPU: the library builds, loads and exports every entry
point that include/arc.h declares; without a device arc_create fails cleanly."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT, gpu_available

HEADER = os.path.join(ROOT, "include", "arc.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:arc_status|void|const char\*)\s+(arc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("arc_create", "arc_destroy", "arc_last_error", "arc_trace", "arc_chem_step", "arc_get_field",
                     "arc_healpix_dirs"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1807_07094_amd import arc

    lib = arc.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_create_without_device_fails_cleanly():
    from paper_1807_07094_amd import arc

    h = C.c_void_p()
    assert arc.lib().arc_create(0, C.byref(h)) == -4  # ARC_E_DEVICE
    assert h.value is None
    assert arc.lib().arc_last_error(None) == b"null context"
    arc.lib().arc_destroy(None)


def test_binding_rejects_missing_library(monkeypatch, tmp_path):
    import importlib

    from paper_1807_07094_amd import arc

    mod = importlib.reload(arc)
    monkeypatch.setattr(mod, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mod, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        mod.lib()
    importlib.reload(arc)
