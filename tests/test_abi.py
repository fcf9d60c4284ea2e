"""The C-ABI library loads and exports every symbol include/snect.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "snect.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(snect_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    import paper_1711_08095_amd as sn
    assert declared_symbols() == sorted(sn.EXPORTS)


def test_library_exports_every_declared_symbol():
    import paper_1711_08095_amd as sn
    if not os.path.exists(sn.LIB_PATH):
        pytest.skip("libsnect.so not built")
    lib = ctypes.CDLL(sn.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_null_arguments_are_rejected_without_a_device():
    import paper_1711_08095_amd as sn
    if not os.path.exists(sn.LIB_PATH):
        pytest.skip("libsnect.so not built")
    lib = sn.load()
    assert lib.snect_create(None, 0, None) == -1
    assert lib.snect_problem_destroy(None) == -1
    assert lib.snect_problem_info(None, None) == -1
    assert lib.snect_train(None, None, 0, 1, None, None) == -1
    assert lib.snect_last_error(None) == b"null context"


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct of the header has the size and field offsets the Python
    binding uses (checked with the host C compiler)."""
    import paper_1711_08095_amd as sn
    pairs = {"snect_tensor": sn.Tensor, "snect_graph": sn.Graph, "snect_params": sn.Params,
             "snect_factors": sn.Factors, "snect_info": sn.Info, "snect_exec": sn.Exec,
             "snect_server_config": sn.ServerConfig}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "snect.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
