"""The C ABI library loads and exports every entry point include/mcrt.h
declares; error paths that need no GPU work (no device here) behave."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcrt.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mcrt_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("mcrt_set_grid", "mcrt_set_dust", "mcrt_set_sources", "mcrt_run_packets",
              "mcrt_temperatures", "mcrt_raytrace_image", "mcrt_raytrace_adjoint",
              "mcrt_run_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1203_2941_amd import _lib
    L = _lib.lib()
    for n in declared():
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"


def test_binding_structs_match_header_layout(tmp_path):
    """Size and every field offset of the ctypes structures against the C
    compiler's layout of include/mcrt.h."""
    import subprocess
    from paper_1203_2941_amd import _lib
    structs = {"mcrt_packet_record": _lib.PacketRecord, "mcrt_run_opts": _lib.RunOpts,
               "mcrt_run_stats": _lib.RunStats}
    inc = os.path.join(ROOT, "include")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mcrt.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_create_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1203_2941_amd import _lib
    L = _lib.lib()
    h = C.c_void_p()
    st = L.mcrt_create(C.byref(h), 0, 0)
    assert st != 0 and not h.value
    assert len(L.mcrt_last_error(None)) > 0
    assert L.mcrt_create(C.byref(h), 0, 7) == _lib.EINVAL


def test_null_context_is_rejected():
    from paper_1203_2941_amd import _lib
    L = _lib.lib()
    assert L.mcrt_reset(None, None) == _lib.EINVAL
    assert L.mcrt_run_packets(None, 0, 1, 0, None, None, None) == _lib.EINVAL
    L.mcrt_destroy(None)
