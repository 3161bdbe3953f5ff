"""Host-side checks of libwefq.so: exported symbols, host tables, error paths (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest
from scipy.special import roots_genlaguerre, roots_legendre

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib
from oracle import gaunt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "wefq.h")).read()
    return sorted(set(re.findall(r"\b(wefq_[A-Za-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = header_symbols()
    assert "wefq_apply_Q" in names and "wefq_build_core" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(_lib.exported_symbols())


@pytest.mark.parametrize("L", [4, 8, 12, 16])
def test_host_coo_matches_oracle_gaunt(L):
    """3j closed form (library) vs exact sphere quadrature (oracle): same rows, same order."""
    mine = wefq.host_coo(L)
    ref = gaunt.coo(L) if L <= 12 else None
    if ref is None:
        assert len(mine["g"]) == 601569
        # spot-check against the oracle's dense Gaunt tensor for a few q1 values
        g = gaunt.gaunt_dense(L)
        idx = np.arange(0, len(mine["g"]), 997)
        assert np.abs(g[mine["q1"][idx], mine["q2"][idx], mine["q3"][idx]] - mine["g"][idx]).max() < 1e-13
        return
    assert len(mine["g"]) == len(ref["g"])
    for k in ("q1", "q2", "q3", "c"):
        assert np.array_equal(mine[k], ref[k])
    # the oracle's quadrature Gaunt carries ~1e-14 rounding at L = 12; the closed
    # form in the library is exact to the last bit (checked against exact rationals)
    assert np.abs(mine["g"] - ref["g"]).max() < 5e-14


@pytest.mark.parametrize("n,alpha", [(7, 0.5), (37, 1.0), (37, 0.75), (28, 0.5)])
def test_host_gauss_laguerre_matches_scipy(n, alpha):
    x, w = wefq.host_gauss(1, n, alpha)
    xr, wr = roots_genlaguerre(n, alpha)
    assert np.abs(x - xr).max() < 1e-12 * x.max()
    assert np.abs(w / wr - 1).max() < 1e-10


@pytest.mark.parametrize("n", [1, 5, 19, 73])
def test_host_gauss_legendre_matches_scipy(n):
    x, w = wefq.host_gauss(0, n)
    xr, wr = roots_legendre(n)
    assert np.abs(x - xr).max() < 1e-14
    assert np.abs(w - wr).max() < 1e-14


def test_error_paths_without_device():
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.wefq_build_core(None, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    desc = _lib.CoreDesc(0, 0.0, 0.0, 17, 4, 0, 0)
    assert lib.wefq_build_core(ctypes.byref(desc), None, ctypes.byref(h)) == _lib.WEFQ_EUNSUPPORTED
    assert b"[0, 16]" in lib.wefq_last_error()
    desc = _lib.CoreDesc(9, 0.0, 0.0, 4, 4, 0, 0)
    assert lib.wefq_build_core(ctypes.byref(desc), None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    for pads in ((65, 0), (0, -1)):                      # quadrature padding outside [0, 64]
        desc = _lib.CoreDesc(1, 0.0, 0.0, 4, 4, 0, 0, 0, None, *pads)
        assert lib.wefq_build_core(ctypes.byref(desc), None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
        assert b"pad" in lib.wefq_last_error()
    # angular factor: too many coefficients, a null array, a non-finite coefficient
    coef = (ctypes.c_double * 40)(*([1.0] * 40))
    ptr = ctypes.cast(coef, ctypes.POINTER(ctypes.c_double))
    for n_beta, p in ((_lib.MAX_BETA + 1, ptr), (-1, ptr), (3, None)):
        desc = _lib.CoreDesc(0, 0.0, 0.0, 4, 4, 0, 0, n_beta, p)
        assert lib.wefq_build_core(ctypes.byref(desc), None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    coef[1] = float("nan")
    desc = _lib.CoreDesc(0, 0.0, 0.0, 4, 4, 0, 0, 3, ptr)
    assert lib.wefq_build_core(ctypes.byref(desc), None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    assert b"non-finite" in lib.wefq_last_error()
    assert lib.wefq_apply_Q(None, 1, None, None, 1, 1, 1, None) == _lib.WEFQ_EINVAL
    n = ctypes.c_int64()
    assert lib.wefq_mode_index(None, 0, 0, 0, ctypes.byref(n)) == _lib.WEFQ_EINVAL
    assert lib.wefq_destroy(None) == _lib.WEFQ_EINVAL
    n = ctypes.c_int64()
    assert lib.wefq_host_coo(17, ctypes.byref(n), None, None, None, None, None) == _lib.WEFQ_EUNSUPPORTED
    x = np.empty(3)
    assert lib.wefq_host_gauss(2, 3, 0.0, x.ctypes.data_as(ctypes.c_void_p),
                               x.ctypes.data_as(ctypes.c_void_p)) == _lib.WEFQ_EINVAL
    with pytest.raises(wefq.WefqError):
        wefq.host_gauss(1, 0)


def test_core_load_rejects_bad_files_before_device_work(tmp_path):
    """wefq_core_load checks header, size and checksum before any HIP call."""
    L_ = _lib.lib()
    h = ctypes.c_void_p()
    missing = str(tmp_path / "missing.wefq").encode()
    assert L_.wefq_core_load(missing, 0, 0, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    garbage = tmp_path / "garbage.wefq"
    garbage.write_bytes(b"not a core file" * 10)
    assert L_.wefq_core_load(str(garbage).encode(), 0, 0, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    assert b"not a valid core file" in L_.wefq_last_error()
    empty = tmp_path / "empty.wefq"
    empty.write_bytes(b"")
    assert L_.wefq_core_load(str(empty).encode(), 0, 0, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    assert L_.wefq_core_save(None, missing) == _lib.WEFQ_EINVAL
    assert not h.value


def test_header_compiles_as_plain_c(tmp_path):
    """include/wefq.h is a C header: it compiles with a C99 compiler, pedantic, no C++."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "wefq.h"\n'
                   "int main(void) {\n"
                   "  wefq_core_desc d = {0};\n"
                   "  wefq_core_info i;\n"
                   "  (void)i;\n"
                   "  return d.n_beta + WEFQ_MAX_BETA - 33;\n"
                   "}\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    res = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc, "-c", str(src),
                          "-o", str(tmp_path / "use.o")], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


def test_no_fallback_without_the_library(monkeypatch):
    """Without libwefq.so every entry raises ImportError: there is no CPU path to fall back on."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libwefq.so")
    with pytest.raises(ImportError):
        wefq.Core("hs", 2, 2, device=0)
    with pytest.raises(ImportError):
        wefq.host_coo(2)


def _fnv1a(data):
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _core_file(version, n_beta, beta0=1.0):
    """A core file for K = 1, L = 0 (one channel, NK = 2): header, angular record for
    version 2, then a zero payload with its FNV-1a checksum."""
    import struct
    payload = bytes(8 * 8)
    angular = struct.pack("<ii33d", n_beta, 0, *([beta0] + [0.0] * 32)) if version == 2 else b""
    header = struct.pack("<8sIIiiiiiiddqQQ", b"WEFQCORE", version, 80 + len(angular), 1, 1, 0, 1, 2, 0,
                         1.0, 0.0, 10, 8, _fnv1a(payload))
    return header + angular + payload


def test_core_load_checks_the_angular_record(tmp_path):
    """A version-2 (angular factor) file with n_beta outside [1, WEFQ_MAX_BETA] or a
    non-finite coefficient is refused; a well-formed one passes every file check (and then
    needs a device)."""
    L_ = _lib.lib()
    h = ctypes.c_void_p()
    for n_beta in (0, _lib.MAX_BETA + 1, -3):
        p = tmp_path / f"bad{n_beta}.wefq"
        p.write_bytes(_core_file(2, n_beta))
        assert L_.wefq_core_load(str(p).encode(), 0, 0, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    p = tmp_path / "nan.wefq"
    p.write_bytes(_core_file(2, 1, float("nan")))
    assert L_.wefq_core_load(str(p).encode(), 0, 0, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    assert b"non-finite" in L_.wefq_last_error()
    p = tmp_path / "wrongsize.wefq"
    p.write_bytes(_core_file(1, 0)[:80] + _core_file(2, 1)[80:])       # version 1 header, v2 body
    assert L_.wefq_core_load(str(p).encode(), 0, 0, None, ctypes.byref(h)) == _lib.WEFQ_EINVAL
    for version in (1, 2):
        p = tmp_path / f"good{version}.wefq"
        p.write_bytes(_core_file(version, 1))
        st = L_.wefq_core_load(str(p).encode(), 0, 0, None, ctypes.byref(h))
        assert st in (_lib.WEFQ_OK, _lib.WEFQ_EHIP), L_.wefq_last_error()
        if st == _lib.WEFQ_OK:
            L_.wefq_destroy(h)


def test_host_tables_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The host C++ (real-Gaunt table, channels, Gauss rules) built with g++ and
    AddressSanitizer + UndefinedBehaviorSanitizer, alone (no HIP source on the line), and run
    over L = 0..8: no report, and the test program's exact checks hold."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(os.path.dirname(here), "paper_2605_28475_amd", "csrc")
    exe = str(tmp_path / "host_tables_san")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-pthread"]
    res = subprocess.run([gxx] + flags + ["-I", csrc, os.path.join(here, "host_tables_driver.cpp"),
                                          os.path.join(csrc, "host_tables.cpp"), "-o", exe],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    # the process environment is kept as it is; ASan is told not to insist on being the first
    # library in the initial list
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "0 failures" in run.stdout
