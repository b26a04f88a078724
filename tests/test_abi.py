"""The C ABI library loads, exports every symbol include/sht.h declares, and
rejects invalid descriptors on the host (no GPU work is issued)."""
import ctypes
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sht.h")


@pytest.fixture(scope="module")
def L():
    from paper_1010_1260_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1010_1260_amd import build
        build.build()
    return _lib


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sht_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ["sht_plan", "sht_alm2map", "sht_alm2map_adjoint", "sht_plan_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(L.EXPORTED)
    out = os.popen(f"nm -D --defined-only {L.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", out), name


def test_status_strings_and_version(L):
    lib = L.load()
    assert lib.sht_version().decode().count(".") == 2
    for code in range(-6, 1):
        s = lib.sht_status_string(code).decode()
        assert s.startswith("SHT_")


def _desc(L, lmax=8, nrings=3, cth=None, sth=None, nphi=None, mval=None, start=None, nm=None,
          nmaps=1, precision=0, flags=0, npix=0):
    keep = []
    cth = np.array([0.5, 0.0, -0.5]) if cth is None else np.asarray(cth, float)
    sth = np.sqrt((1 - cth) * (1 + cth)) if sth is None else np.asarray(sth, float)
    nphi = np.full(len(cth), 8, np.int64) if nphi is None else np.asarray(nphi, np.int64)
    phi0 = np.zeros(len(cth))
    keep += [cth, sth, nphi, phi0]
    d = L.GeometryDesc()
    d.lmax = lmax
    d.nm = (lmax + 1 if mval is None else len(mval)) if nm is None else nm
    if mval is not None:
        mv = np.asarray(mval, np.int32)
        keep.append(mv)
        d.mval = mv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.nrings = nrings if nrings is not None else len(cth)
    d.cth = cth.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.sth = sth.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.phi0 = phi0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.nphi = nphi.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if start is not None:
        st = np.asarray(start, np.int64)
        keep.append(st)
        d.ringstart = st.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.nmaps = nmaps
    d.precision = precision
    d.flags = flags
    d.npix = npix
    return d, keep


@pytest.mark.parametrize("case,expect", [
    (dict(lmax=-1), "INVALID"),
    (dict(lmax=20000), "INVALID"),
    (dict(nm=0), "INVALID"),
    (dict(lmax=4, nm=6), "INVALID"),
    (dict(mval=[0, 2, 2]), "INVALID"),
    (dict(mval=[3, 1]), "INVALID"),
    (dict(mval=[0, 9]), "INVALID"),
    (dict(nrings=0), "INVALID"),
    (dict(cth=[1.5, 0.0, -0.5], sth=[0.0, 1.0, 0.8]), "INVALID"),
    (dict(cth=[0.5, 0.0, -0.5], sth=[0.5, 1.0, 0.5]), "INVALID"),   # cos^2 + sin^2 != 1
    (dict(nphi=[8, 0, 8]), "INVALID"),
    (dict(nphi=[8, 20000, 8]), "UNSUPPORTED"),
    (dict(start=[0, 4, 16]), "INVALID"),                           # overlapping rings
    (dict(start=[0, -8, 16]), "INVALID"),
    (dict(nmaps=0), "INVALID"),
    (dict(precision=7), "UNSUPPORTED"),
    (dict(flags=1 << 5), "INVALID"),
    (dict(npix=23), "INVALID"),                                   # shorter than the rings
    (dict(npix=-1), "INVALID"),
])
def test_plan_rejects_invalid_descriptors_on_host(L, case, expect):
    lib = L.load()
    d, keep = _desc(L, **case)
    h = ctypes.c_void_p(1234)
    rc = lib.sht_plan(ctypes.byref(h), ctypes.byref(d))
    want = {"INVALID": L.SHT_ERR_INVALID_ARG, "UNSUPPORTED": L.SHT_ERR_UNSUPPORTED}[expect]
    assert rc == want
    assert h.value is None


def test_null_arguments(L):
    lib = L.load()
    assert lib.sht_plan(None, None) == L.SHT_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.sht_plan(ctypes.byref(h), None) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_plan_destroy(None) == L.SHT_ERR_BAD_HANDLE
    n = ctypes.c_size_t()
    assert lib.sht_plan_workspace_size(None, ctypes.byref(n)) == L.SHT_ERR_BAD_HANDLE
    assert lib.sht_alm2map(None, None, None, None, 0, None) == L.SHT_ERR_BAD_HANDLE
    assert lib.sht_alm2map_adjoint(None, None, None, None, 0, None) == L.SHT_ERR_BAD_HANDLE
    c = ctypes.c_int32()
    assert lib.sht_plan_get_config(None, ctypes.byref(c)) == L.SHT_ERR_BAD_HANDLE
    assert lib.sht_plan_set_config(None, 2) == L.SHT_ERR_BAD_HANDLE
    assert lib.sht_plan_autotune(None, None, None, None, 0, None, None) == L.SHT_ERR_BAD_HANDLE


def test_package_import_fails_loudly_without_library(tmp_path):
    # a copy of the binding pointing at a missing library must raise, not fall back
    import importlib.util
    src = os.path.join(ROOT, "paper_1010_1260_amd", "_lib.py")
    spec = importlib.util.spec_from_file_location("_lib_copy", src)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with pytest.raises(ImportError):
        mod.load(str(tmp_path / "missing.so"))


def test_one_hip_runtime_whatever_the_import_order():
    """torch bundles a HIP runtime with the system's soname; importing the
    package before torch must still leave one runtime in the process, or
    torch's device memory and streams would be foreign to the library's."""
    import subprocess
    code = ("import sys; sys.path.insert(0, %r); import paper_1010_1260_amd; "
            "maps = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
