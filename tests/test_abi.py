"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
entry point declared in include/helm.h, and rejects invalid geometry before touching
the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1208_3956_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "helm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "helm_setup" in names and "helm_solve" in names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def _setup(c, omega=2 * np.pi * 5, h=0.05, J=2, **kw):
    n_y, n_x = c.shape
    o = L.helm_default_opts(n_x, n_y)
    o.pml_outer, o.pml_iface = kw.pop("pml_outer", 4), kw.pop("pml_iface", 3)
    for k, v in kw.items():
        setattr(o, k, v)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return L.helm_setup(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), omega, h, o, J)


@pytest.mark.parametrize("case,msg", [
    (dict(J=0), "J must be"),
    (dict(omega=0.0), "omega"),
    (dict(h=-1.0), "h must"),
    (dict(dim=4), "dim"),
    (dict(dim=3), "every axis"),
    (dict(J=12), "at least two columns"),
    (dict(J=1, pml_outer=25), "64"),
    (dict(J=2, pml_iface=60), "64"),
])
def test_setup_rejects_bad_geometry(case, msg):
    c = np.ones((20, 20))
    with pytest.raises(L.HelmError) as e:
        _setup(c, **case)
    assert e.value.status == L.HELM_EINVAL
    assert msg in str(e.value)
    assert msg in L.helm_last_error(None)


@pytest.mark.parametrize("bad", [0.0, -1.0, np.nan, np.inf])
def test_setup_rejects_bad_medium(bad):
    c = np.ones((20, 20))
    c[4, 7] = bad
    with pytest.raises(L.HelmError) as e:
        _setup(c)
    assert e.value.status == L.HELM_EINVAL


def test_interface_inside_outer_pml_rejected():
    c = np.ones((20, 20))
    beta = (ctypes.c_int * 1)(3)          # column 3 lies in the outer PML of width 4
    with pytest.raises(L.HelmError) as e:
        _setup(c, beta=ctypes.cast(beta, ctypes.POINTER(ctypes.c_int)))
    assert "interior" in str(e.value)


def test_destroy_null_is_noop():
    L.lib().helm_destroy(None)


def test_grad_null_handle_is_einval():
    assert L.lib().helm_grad(None, 1, None, 1, None, None, 1e-6, None, None, None) == L.HELM_EINVAL


def test_setup_rejects_oversized_3d_slabs():
    """A 28-column slab with N_z = 308 has blocks of 8624 unknowns (> 8192)."""
    o = L.helm_default_opts(20, 20)
    o.dim, o.pml_outer, o.pml_iface = 3, 4, 3
    o.n[2] = 300
    c = np.ascontiguousarray(np.ones((300, 20, 20)))
    with pytest.raises(L.HelmError) as e:
        L.helm_setup(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2 * np.pi * 5, 0.05, o, 1)
    assert e.value.status == L.HELM_EINVAL and "8192" in str(e.value)
