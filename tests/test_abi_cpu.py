"""Host-side checks of the C-ABI library (no GPU needed): the library loads,
exports every entry point declared in include/lmfmm.h, and rejects invalid
arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2511_12450_amd import lmfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lmfmm.h")).read()
    return sorted(set(re.findall(r"\b(lm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = lmfmm.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(lmfmm.exported_symbols()) == set(names)


def test_version():
    assert b"gfx950" in lmfmm.lib().lm_version()


@pytest.mark.parametrize("d,k,eta,msg", [
    ([0.0, -1.0], [1.0, 2.0, 3.0], None, "increasing"),
    ([0.0], [1.0, -2.0], None, "positive"),
    ([np.nan], [1.0, 2.0], None, "non-finite"),
    ([0.0], [1.0, 2.0], [1.0, 0.0], "eta"),
])
def test_layers_rejects_invalid(d, k, eta, msg):
    with pytest.raises(lmfmm.LmError) as e:
        lmfmm.Layers(d, k, eta)
    assert e.value.status == -1 and msg in str(e.value)


def test_geometry_rejects_invalid_before_device_work():
    lay = lmfmm.Layers([0.0], [2.0, 3.0])
    tri = np.array([[0.0, 1.0], [1.0, 1.0], [0.5, 2.0]])
    bad = [
        (np.array([0, 2]), tri[:2], "fewer than 3"),
        (np.array([1, 4]), tri, "node_offsets[0]"),
        (np.array([0, 3]), np.array([[0.0, 1.0], [np.inf, 1.0], [0.5, 2.0]]), "non-finite"),
        (np.array([0, 3]), np.array([[0.0, 1.0], [0.0, 1.0], [0.5, 2.0]]), "degenerate"),
    ]
    for off, xy, msg in bad:
        off = np.ascontiguousarray(off, dtype=np.int64)
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        h = ctypes.c_void_p()
        st = lmfmm.lib().lm_create_geometry(lay.h, off.size - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                            xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None,
                                            ctypes.byref(h))
        assert st == -1, msg
        assert msg in lmfmm.lib().lm_last_error().decode()
        assert not h.value


def test_null_handles_rejected():
    L = lmfmm.lib()
    assert L.lm_matvec(None, 0, 1, None, None, None) == -1
    assert L.lm_geometry_info(None, None, None, None) == -1
    assert L.lm_rhs(None, 1, None, None, None) == -1
