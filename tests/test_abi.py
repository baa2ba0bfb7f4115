"""CPU checks of the C ABI: the library loads, exports every declared symbol, and rejects
malformed arguments before touching the device.  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2205_08417_amd import snrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snrt.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(snrt_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(snrt.LIB_PATH):
        from paper_2205_08417_amd import build
        build.build()
    return snrt.lib()


def test_header_and_binding_agree():
    assert _declared() == sorted(snrt.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name
    out = os.popen(f"nm -D --defined-only {snrt.LIB_PATH}").read()
    exported = set(re.findall(r"\bT (snrt_[a-z0-9_]+)\b", out))
    assert set(_declared()) <= exported
    # the C ABI is all that is exported under the snrt_ prefix
    assert exported == set(_declared())


def test_abi_version(L):
    assert snrt.snrt_abi_version() == 2


def test_rejects_null_and_bad_sizes_before_device_use(L):
    h = ctypes.c_void_p()
    assert L.snrt_mesh_create(None, 1, 3, None, None, None, None, 0, 0) == snrt.SNRT_E_ARG
    assert "out is NULL" in snrt.snrt_last_error()
    assert L.snrt_mesh_create(ctypes.byref(h), 4, 5, None, None, None, None, 0, 0) == \
        snrt.SNRT_E_UNSUPPORTED
    assert L.snrt_mesh_create(ctypes.byref(h), -1, 3, None, None, None, None, 0, 0) == \
        snrt.SNRT_E_ARG
    assert L.snrt_mesh_create(ctypes.byref(h), 4, 3, None, None, None, None, 0, 0) == \
        snrt.SNRT_E_ARG
    assert L.snrt_mesh_create(ctypes.byref(h), 4, 3, None, None, None, None, 0, 7) == \
        snrt.SNRT_E_ARG
    assert L.snrt_quad_create(ctypes.byref(h), 0, None, None) == snrt.SNRT_E_UNSUPPORTED
    assert L.snrt_quad_create(ctypes.byref(h), 2048, None, None) == snrt.SNRT_E_UNSUPPORTED
    assert L.snrt_step(None, None, None, None, None, None, None, 0, None) == snrt.SNRT_E_ARG
    assert L.snrt_mass(None, None, None, None, None) == snrt.SNRT_E_ARG
    assert L.snrt_permute(None, 0, None, None, 4, None) == snrt.SNRT_E_ARG


def test_rejects_malformed_connectivity_before_device_use(L):
    from paper_2205_08417_amd import inputs as I
    m = I.four_triangle_mesh()
    bad = m.face_nbr.copy()
    bad[0, 0] = 2                  # cell 2 does not list cell 0 back
    with pytest.raises(snrt.SnrtError, match="not symmetric"):
        snrt.snrt_mesh_create(bad, m.face_normal, m.area, m.centroid, m.nbfaces)
    bad = m.face_nbr.copy()
    bad[0, 2] = -9                 # boundary id 8 >= nbfaces
    with pytest.raises(snrt.SnrtError, match="boundary face id"):
        snrt.snrt_mesh_create(bad, m.face_normal, m.area, m.centroid, m.nbfaces)
    area = m.area.copy()
    area[1] = 0.0
    with pytest.raises(snrt.SnrtError, match="area"):
        snrt.snrt_mesh_create(m.face_nbr, m.face_normal, area, m.centroid, m.nbfaces)
    with pytest.raises(snrt.SnrtError, match="centroids"):
        snrt.snrt_mesh_create(m.face_nbr, m.face_normal, m.area, None, m.nbfaces)
    w = np.array([1.0, -1.0])
    with pytest.raises(snrt.SnrtError, match="weight"):
        snrt.snrt_quad_create(np.array([[1.0, 0, 0], [0, 1.0, 0]]), w)


def test_package_does_not_import_oracle():
    """The product path never references the test oracle."""
    pkg = os.path.join(ROOT, "paper_2205_08417_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower() or f == "inputs.py", f
