"""The C-ABI library loads and exports every symbol declared in include/wcl.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wcl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wcl_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["wcl_create", "wcl_set_gauge", "wcl_set_params", "wcl_apply", "wcl_apply_op", "wcl_solve",
              "wcl_grad", "wcl_bench_hop", "wcl_last_error", "wcl_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1612_06556_amd import wcl
    if not os.path.exists(wcl.LIB_PATH):
        pytest.fail("libwcl.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(wcl.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    opts = wcl.wcl_default_opts()
    assert opts.tol == 1e-10 and opts.use_ras == 1 and opts.ras_iters == 4
    assert ctypes.sizeof(wcl.wcl_solve_info) == 32


def _struct_fields(name):
    src = open(os.path.join(ROOT, "include", "wcl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src).group(1)
    return [m.group(2) for m in re.finditer(r"\b(int|double|const double\s*\*)\s*([a-z_0-9]+)\s*(\[\d+\])?\s*;", body)]


@pytest.mark.parametrize("name", ["wcl_solve_opts", "wcl_solve_info", "wcl_kstat", "wcl_tuning"])
def test_binding_structs_match_the_header(name):
    """The ctypes structures list the header's fields in the header's order."""
    from paper_1612_06556_amd import wcl
    fields = [f for f, _ in getattr(wcl, name)._fields_]
    assert fields == _struct_fields(name)


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1612_06556_amd import wcl
    monkeypatch.setattr(wcl, "LIB_PATH", os.path.join(ROOT, "no_such_libwcl.so"))
    monkeypatch.setattr(wcl, "_lib", None)
    with pytest.raises(RuntimeError):
        wcl.load()


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_create_refuses_fields_beyond_32bit_offsets():
    """Fields are addressed with 32-bit byte offsets: a lattice whose FP64
    links would reach 4 GiB (576 bytes a site) is refused before anything is
    allocated."""
    from paper_1612_06556_amd import wcl
    lib = wcl.load()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(48, 48, 48, 96)   # 10,616,832 sites
    rc = lib.wcl_create(dims, -1, None, None, ctypes.byref(h))
    assert rc == wcl.WCL_EINVAL and not h.value
    assert b"too large" in lib.wcl_last_error()
