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


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the C layout of include/arc.h: a small C
    program built with the host compiler prints sizeof and offsetof of each field."""
    import shutil
    import subprocess

    from paper_1807_07094_amd import arc

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"arc_grid": arc.Grid, "arc_sources": arc.Sources, "arc_freq_bins": arc.Bins,
               "arc_trace_params": arc.TraceParams, "arc_rates": arc.Rates, "arc_ledger": arc.Ledger,
               "arc_tune_result": arc.TuneResult, "arc_chem_params": arc.ChemParams,
               "arc_chem_stats": arc.ChemStats, "arc_train_params": arc.TrainParams,
               "arc_train_report": arc.TrainReport}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "arc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
