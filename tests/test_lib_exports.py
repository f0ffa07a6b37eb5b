"""The C-ABI library loads and exports every function include/luda.h declares
(no device work: only the host-side CRC table self-check is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "luda.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(luda_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["luda_ctx_create", "luda_compact", "luda_compact_dev", "luda_compact_batch",
                 "luda_build_tables_dev", "luda_result_free"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2004_03054_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.EXPORTS) <= set(declared_functions())


def test_crc_shift_tables_selfcheck():
    from paper_2004_03054_amd import binding
    assert binding.selftest_crc() == 0


def test_status_strings():
    from paper_2004_03054_amd import binding
    L = binding.lib()
    for code, name in binding.STATUS.items():
        assert L.luda_status_str(code).decode() == name
