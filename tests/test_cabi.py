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


def test_every_call_refuses_a_null_context():
    """Each exported call validates its context before touching the device:
    a null context gives WCL_EINVAL and a message (wcl_destroy(NULL) is a
    no-op returning WCL_OK); runs without a GPU."""
    from paper_1612_06556_amd import wcl
    lib = wcl.load()
    n = None
    d = ctypes.c_double()
    i = ctypes.c_int()
    st = wcl.wcl_kstat()
    tu = wcl.wcl_tuning()
    opts = wcl.wcl_default_opts()
    info = (wcl.wcl_solve_info * 1)()
    calls = {
        "wcl_set_stream": lambda: lib.wcl_set_stream(n, n),
        "wcl_set_gauge": lambda: lib.wcl_set_gauge(n, n),
        "wcl_set_compression": lambda: lib.wcl_set_compression(n, 1),
        "wcl_set_params": lambda: lib.wcl_set_params(n, 0.12, 1.0),
        "wcl_set_ras": lambda: lib.wcl_set_ras(n, 1, 4, 0, 0),
        "wcl_set_ras_cores": lambda: lib.wcl_set_ras_cores(n, n),
        "wcl_apply": lambda: lib.wcl_apply(n, n, n, 1, 0, 32),
        "wcl_apply_op": lambda: lib.wcl_apply_op(n, 0, n, n, 1, 32),
        "wcl_apply_noalloc": lambda: lib.wcl_apply_noalloc(n, n, n, 1, 0, 32),
        "wcl_solve": lambda: lib.wcl_solve(n, n, n, 1, ctypes.byref(opts), info),
        "wcl_grad": lambda: lib.wcl_grad(n, n, n, n, ctypes.byref(d)),
        "wcl_bench_hop": lambda: lib.wcl_bench_hop(n, 32, 1, 1, 1, ctypes.byref(d)),
        "wcl_bench_clover": lambda: lib.wcl_bench_clover(n, 32, 1, 1, ctypes.byref(d)),
        "wcl_bench_stream": lambda: lib.wcl_bench_stream(n, ctypes.c_double(1.0), 1, ctypes.byref(d), ctypes.byref(d)),
        "wcl_profile": lambda: lib.wcl_profile(n, 1),
        "wcl_profile_mask": lambda: lib.wcl_profile_mask(n, 1),
        "wcl_profile_read": lambda: lib.wcl_profile_read(n, 0, ctypes.byref(st)),
        "wcl_set_tuning": lambda: lib.wcl_set_tuning(n, 128, 2, 1, 0),
        "wcl_set_hop_tiles": lambda: lib.wcl_set_hop_tiles(n, 1),
        "wcl_set_hop_staging": lambda: lib.wcl_set_hop_staging(n, 1),
        "wcl_set_batch_tuning": lambda: lib.wcl_set_batch_tuning(n, 1),
        "wcl_autotune": lambda: lib.wcl_autotune(n, 32, 1, n, n, 1, ctypes.byref(tu)),
        "wcl_autotune_hop": lambda: lib.wcl_autotune_hop(n, 32, 1, ctypes.byref(i)),
    }
    for name, call in calls.items():
        rc = call()
        assert rc == wcl.WCL_EINVAL, (name, rc)
        assert lib.wcl_last_error(), name
    assert lib.wcl_destroy(n) == wcl.WCL_OK
    # every context-taking call of the header is exercised above
    ctx_calls = [c for c in _declared() if c not in ("wcl_create", "wcl_destroy", "wcl_last_error",
                                                    "wcl_default_opts")]
    assert sorted(ctx_calls) == sorted(calls), sorted(set(ctx_calls) ^ set(calls))


def test_create_validates_before_allocating():
    """wcl_create's argument checks (documented in the header) run before any
    device call: odd or short extents, a bad boundary condition, tiles that
    are odd or do not divide the lattice, and null pointers are refused."""
    from paper_1612_06556_amd import wcl
    lib = wcl.load()

    def create(dims, tbc=-1, tile=None, out=True):
        h = ctypes.c_void_p()
        d = (ctypes.c_int * 4)(*dims) if dims is not None else None
        t = (ctypes.c_int * 4)(*tile) if tile is not None else None
        rc = lib.wcl_create(d, tbc, t, None, ctypes.byref(h) if out else None)
        assert not h.value
        return rc

    assert create((8, 8, 8, 7)) == wcl.WCL_EINVAL          # odd extent
    assert create((8, 8, 8, 2)) == wcl.WCL_EINVAL          # extent below 4
    assert create((8, 8, 8, 8), tbc=0) == wcl.WCL_EINVAL   # t_bc must be +1 or -1
    assert create((8, 8, 8, 8), tile=(3, 2, 2, 2)) == wcl.WCL_EINVAL
    assert create((8, 8, 8, 8), tile=(6, 2, 2, 2)) == wcl.WCL_EINVAL   # does not divide 8
    assert create(None) == wcl.WCL_EINVAL
    assert create((8, 8, 8, 8), out=False) == wcl.WCL_EINVAL
