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
