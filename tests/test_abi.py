"""The C ABI: libqrt.so loads without a GPU and exports every function that
include/qrt.h declares, with a binding for each (no compute call here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?(?:int|void|char|int64_t|size_t)\s*\**\s*(qrt_\w+)\s*\(", src, flags=re.M)
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("qrt_create", "qrt_destroy", "qrt_set_grid", "qrt_set_point_source", "qrt_set_sphere_source",
                 "qrt_set_dust", "qrt_set_observers", "qrt_set_sequence", "qrt_set_transport", "qrt_run",
                 "qrt_read_images", "qrt_reset_images", "qrt_get_counters", "qrt_generate_points", "qrt_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2406_15632_amd import qrt
    if not os.path.exists(qrt.LIB_PATH):
        pytest.fail("libqrt.so is not built (run __graft_entry__.build())")
    lib = qrt.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in qrt.SIGNATURES, f"no binding for {name}"


def test_binding_refuses_a_missing_library(tmp_path):
    from paper_2406_15632_amd import qrt
    saved = qrt._lib
    qrt._lib = None
    try:
        with pytest.raises(ImportError):
            qrt.load(str(tmp_path / "absent.so"))
    finally:
        qrt._lib = saved


def test_binding_structs_match_the_header(tmp_path):
    """Every struct of the binding has the size and field offsets of the C
    header (compiled with the host C compiler)."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_2406_15632_amd import qrt
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"qrt_counters": qrt.qrt_counters, "qrt_train_cfg": qrt.qrt_train_cfg,
               "qrt_train_report": qrt.qrt_train_report, "qrt_mask_report": qrt.qrt_mask_report,
               "qrt_batch_scene": qrt.qrt_batch_scene, "qrt_timing": qrt.qrt_timing}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qrt.h"', "int main(void) {"]
    for name, st in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                           check=True).stdout.split("\n") if l)
    for name, st in structs.items():
        assert int(got[name]) == C.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, f"{name}.{f}"
