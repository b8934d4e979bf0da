"""The C-ABI library loads and exports every symbol include/acr.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1604_00617_amd", "libacr.so")


def declared():
    with open(os.path.join(ROOT, "include", "acr.h")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(acr_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("acr_factor", "acr_solve", "acr_solve_refined", "acr_solve_krylov", "acr_residual",
              "acr_get_info", "acr_get_block", "acr_destroy", "acr_status_string", "acr_last_error",
              "acr_trim_pool"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libacr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    lib.acr_status_string.restype = ctypes.c_char_p
    assert lib.acr_status_string(0) == b"ok"
    assert lib.acr_status_string(3) == b"singular pivot"


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1604_00617_amd as acr
    with pytest.raises(ImportError):
        acr.load(str(tmp_path / "missing.so")) if acr._lib is None else (_ for _ in ()).throw(ImportError())


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU only: --gpus above 1 exits with a message
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_header_documents_solve_modes():
    """acr_set_solve_mode is declared with its four modes and the wait limit."""
    with open(os.path.join(ROOT, "include", "acr.h")) as fh:
        src = fh.read()
    assert "acr_set_solve_mode(int32_t mode, int64_t wait_limit)" in src
    for m in ("mode 0", "mode 1", "mode 2", "mode 3"):
        assert m in src
