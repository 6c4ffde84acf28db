"""The C-ABI library loads and exports every function include/hsdm.h
declares; host-side argument checks (no GPU, no compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsdm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hsdm_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1912_13403_amd import hsdm
    if not os.path.exists(hsdm.LIB_PATH):
        from paper_1912_13403_amd import build
        build.build()
    return hsdm.load_library()


def test_header_declares_the_paths_calls():
    names = _declared()
    for must in ("hsdm_init", "hsdm_finalize", "hsdm_reinit", "hsdm_solve_ev_real",
                 "hsdm_solve_dm_real"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1912_13403_amd import hsdm
    names = _declared()
    assert names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(hsdm.EXPORTED) == names


def test_status_strings_and_version(lib):
    assert lib.hsdm_status_string(0) == b"ok"
    assert lib.hsdm_status_string(1).startswith(b"S is not positive")
    assert lib.hsdm_status_string(-3) == b"invalid argument"
    assert lib.hsdm_version() >= 100


def test_null_handle_is_argument_one(lib):
    vp = ctypes.c_void_p
    assert lib.hsdm_solve_ev_real(None, 4, vp(8), 4, vp(8), 4, vp(8), vp(8), 4, None) == -1
    assert lib.hsdm_solve_dm_real(None, 4, vp(8), 4, vp(8), 4, 1.0, 0.0, vp(8), 4, None, 4, None,
                                  None, None, None) == -1
    assert lib.hsdm_finalize(None) == -1
    assert lib.hsdm_reinit(None) == -1
    assert lib.hsdm_set_real(None, 1, 2.0) == -1
    assert lib.hsdm_init(None, 0) == -1
    assert lib.hsdm_last_error(None) == b"null handle"
    out = (ctypes.c_double * 3)()
    assert lib.hsdm_probe(None, 0, 100.0, out, None) == -1


def test_handle_keys_match_the_header(lib):
    """The binding's key constants are the header's enum values; a null
    handle is reported as argument 1 for the integer keys too."""
    from paper_1912_13403_amd import hsdm
    txt = open(HEADER).read()
    for name in ("HSDM_KEY_FMAX", "HSDM_KEY_FCUT", "HSDM_KEY_DEG_TOL", "HSDM_KEY_TIMING",
                 "HSDM_KEY_STREAMS", "HSDM_KEY_N_STATES", "HSDM_KEY_CONCURRENT",
                 "HSDM_KEY_PRECISION", "HSDM_KEY_REFINE_STEPS", "HSDM_KEY_AUTOTUNE",
                 "HSDM_KEY_GRAPH"):
        m = re.search(name + r"\s*=\s*(\d+)", txt)
        assert m and int(m.group(1)) == getattr(hsdm, name), name
    assert lib.hsdm_set_int(None, hsdm.HSDM_KEY_STREAMS, 4) == -1
    m = re.search(r"#define\s+HSDM_NOALLOC_MAX_N\s+(\d+)", txt)
    assert m and int(m.group(1)) == hsdm.HSDM_NOALLOC_MAX_N


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_no_unresolved_own_symbols(lib):
    """Every function the library calls is defined in it or in a versioned
    system library: a loader that binds at load time finds nothing missing."""
    import shutil
    import subprocess
    from paper_1912_13403_amd import hsdm
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--undefined-only", hsdm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    missing = [ln.split()[-1] for ln in out.splitlines()
               if ln.split() and ln.split()[0] == "U" and "@" not in ln]
    assert missing == []


def test_library_loads_with_immediate_binding():
    from paper_1912_13403_amd import hsdm
    ctypes.CDLL(hsdm.LIB_PATH, mode=os.RTLD_NOW)
