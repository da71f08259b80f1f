"""The C-ABI library loads on the CPU and exports every symbol that
include/*.h declares; the Python binding declares the same set."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(bq_[a-z_]+)\s*\(",
                                text, flags=re.M))
    return names


def _lib_path():
    from paper_2307_02043_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2307_02043_amd import build_lib
        build_lib.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    d = _declared()
    for must in ("bq_create", "bq_destroy", "bq_forward", "bq_grad", "bq_wprox"):
        assert must in d


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2307_02043_amd import _lib
    assert set(_lib.EXPORTED) == _declared()


def test_create_rejects_bad_arguments_without_touching_the_gpu():
    from paper_2307_02043_amd import _lib as L
    lib = L.load()
    out = ctypes.c_void_p()
    g = L.Geom(10, 0.1, 0.4, 1.33, 0, 0, 1e-5, 10, 0)   # N = 10 is unsupported
    d = (L.Illum * 1)(L.Illum(0.0, 0.0, 1.0))
    assert lib.bq_create(ctypes.byref(g), d, 1, None, ctypes.byref(out)) == L.BQ_EUNSUPPORTED
    assert b"N" in lib.bq_last_error(None)
    g = L.Geom(16, -0.1, 0.4, 1.33, 0, 0, 1e-5, 10, 0)
    assert lib.bq_create(ctypes.byref(g), d, 1, None, ctypes.byref(out)) == L.BQ_EINVAL
    g = L.Geom(16, 0.1, 0.4, 1.33, 0, 0, 1e-5, 10, 0)
    bad = (L.Illum * 1)(L.Illum(0.0, 0.5, 0.5))
    assert lib.bq_create(ctypes.byref(g), bad, 1, None, ctypes.byref(out)) == L.BQ_EINVAL
    assert lib.bq_create(ctypes.byref(g), d, 0, None, ctypes.byref(out)) == L.BQ_EINVAL
    assert lib.bq_destroy(None) == L.BQ_OK
    # entry points that need a context reject a null one before any device work
    assert lib.bq_autotune(None, 4, None) == L.BQ_EINVAL
    assert lib.bq_set_plan(None, 0, 0) == L.BQ_EINVAL
    assert lib.bq_set_batch_limit(None, 0) == L.BQ_EINVAL
    assert lib.bq_timing(None, 0) == L.BQ_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: without the built library the binding raises."""
    import pytest
    from paper_2307_02043_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libbq.so"))
    with pytest.raises(ImportError, match="is missing"):
        _lib.load()


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus N > 1 exits with a message before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_raw_buffer_accesses_stay_in_range():
    """Every offset the padded-line passes of G can form through a raw
    buffer resource lies inside that resource, each resource is under 2^31
    bytes and inside its allocation, and the y pass maps its workgroups one
    to one onto (system, class, line block) for batches of 1..40 (host-side
    enumeration over the launch grids of every built grid and precision)."""
    from paper_2307_02043_amd import _lib as L
    lib = L.load()
    buf = ctypes.create_string_buffer(4096)
    n = ctypes.c_longlong()
    bad = lib.bq_audit_raw_ranges(buf, len(buf), ctypes.byref(n))
    assert bad == 0, buf.value.decode()
    assert n.value > 50_000_000  # every (thread, value) of every launch shape
