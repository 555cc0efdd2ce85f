"""The C ABI library: builds, loads, exports every declared symbol, and its
struct layouts agree with the binding.  No GPU needed (no compute calls)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "edupic.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char \*)\s*\*?\s*(edp_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2103_09642_amd import edupic
    if not os.path.exists(edupic.LIB_PATH):
        from paper_2103_09642_amd import build
        build.build()
    return C.CDLL(edupic.LIB_PATH)


def test_every_declared_symbol_is_exported(lib):
    from paper_2103_09642_amd import edupic
    names = _declared()
    assert len(names) >= 20
    assert sorted(edupic.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2103_09642_amd", "libedupic.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (edp_\w+)$", out, re.M))
    assert set(names) <= exported
    for n in names:
        getattr(lib, n)


def test_struct_layouts_match_binding(tmp_path):
    """sizeof/offsetof of the header's structs equal the ctypes mirrors."""
    from paper_2103_09642_amd import edupic
    src = tmp_path / "lay.c"
    fields = {"edp_case_desc": edupic.CaseDesc, "edp_xsec": edupic.Xsec, "edp_counts": edupic.Counts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    for cname, py in fields.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_error_paths_without_a_device(lib):
    """Null arguments are rejected with EDP_EINVAL and a message, no crash."""
    from paper_2103_09642_amd import edupic
    L = edupic.load()
    assert L.edp_case_bytes(None, None) == edupic.EDP_EINVAL
    assert b"cross sections" in L.edp_last_error()
    assert L.edp_sync(None) == edupic.EDP_EINVAL
    assert L.edp_set_option(None, 1, 0) == edupic.EDP_EINVAL
    assert L.edp_create(None, 0, None) == edupic.EDP_EINVAL
