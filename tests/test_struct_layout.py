"""Every struct of the C ABI header has the same layout in the Python binding:
the header is compiled as plain C by the host compiler, which prints the size
of each struct and the offset of each member, and the ctypes structures must
list the same members in the same order at the same offsets (a renamed,
reordered or retyped member on either side fails here, without a GPU)."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrbms.h")

# header struct -> ctypes structure of the binding
BINDING = {
    "lrbms_problem": "Problem_C",
    "lrbms_model_info": "ModelInfo_C",
    "lrbms_offline_opts": "OfflineOpts_C",
    "lrbms_offline_report": "OfflineReport_C",
    "lrbms_tune_report": "TuneReport_C",
    "lrbms_kernel_stat": "KernelStat_C",
    "lrbms_server_info_t": "ServerInfo_C",
}


def header_structs():
    """Member names, in order, of every `typedef struct NAME { ... } NAME;`."""
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"typedef\s+struct\s+(\w+)\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        assert m.group(1) == m.group(3)
        names = []
        for decl in m.group(2).split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                nm = re.search(r"(\w+)\s*(\[\s*\d+\s*\])?\s*$", part.strip())
                assert nm, part
                names.append(nm.group(1))
        out[m.group(1)] = names
    return out


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = header_structs()
    d = tmp_path_factory.mktemp("layout")
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "lrbms.h"', "int main(void) {"]
    for s, names in structs.items():
        src.append(f'  printf("{s} %zu\\n", sizeof({s}));')
        for n in names:
            src.append(f'  printf("{s}.{n} %zu\\n", offsetof({s}, {n}));')
    src += ["  return 0;", "}"]
    (d / "layout.c").write_text("\n".join(src) + "\n")
    exe = str(d / "layout")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    str(d / "layout.c"), "-o", exe], check=True)
    lines = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    return structs, dict(ln.split() for ln in lines if ln)


def test_every_header_struct_has_a_binding(c_layout):
    structs, _ = c_layout
    assert set(structs) == set(BINDING)


@pytest.mark.parametrize("name", sorted(BINDING))
def test_binding_matches_c_layout(c_layout, name):
    from paper_1405_2810_amd import lrbms
    structs, lay = c_layout
    cls = getattr(lrbms, BINDING[name])
    assert [f for f, _ in cls._fields_] == structs[name]
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == int(lay[f"{name}.{f}"]), f
    assert C.sizeof(cls) == int(lay[name])
