"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
header declares, reports statuses, and rejects invalid arguments before
touching a device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdsw.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hdsw_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    from paper_2003_02585_amd import hdsw as H
    assert _declared() == sorted(H.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2003_02585_amd import hdsw as H
    lib = ctypes.CDLL(H.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults():
    from paper_2003_02585_amd import hdsw as H
    for s in range(7):
        assert H.hdsw_status_str(s).startswith("HDSW")
    o = H.hdsw_default_options()
    assert (o.precision, o.rounds, o.gmres_m, o.dedup, o.graphs) == (H.HDSW_MIXED, 1, 0, 1, 1)
    assert o.pml_R == 1e-16 and o.tol == 1e-10


@pytest.mark.parametrize("bad", [
    dict(N=30, P=4),            # N not divisible by P
    dict(W=0),                  # no layer
    dict(kmul=-1.0),            # nonpositive wavenumber
    dict(knan=True),            # non-finite wavenumber
    dict(rounds=0),
])
def test_setup_rejects_invalid_arguments(bad):
    # validation happens on the host before any device allocation
    from paper_2003_02585_amd import hdsw as H
    N = bad.get("N", 32)
    kap = np.full((N, N), 40.0) * bad.get("kmul", 1.0)
    if bad.get("knan"):
        kap[3, 4] = np.nan
    opt = H.hdsw_default_options(rounds=bad.get("rounds", 1))
    with pytest.raises(H.HdswError) as ei:
        H.hdsw_setup(kap, 1.0 / N, (bad.get("P", 2),) * 2, bad.get("W", 8), opt)
    assert ei.value.status == H.HDSW_EINVAL


@pytest.mark.parametrize("bad", [
    dict(N=(12, 12, 13), P=(2, 2, 2)),    # an axis not divisible by its subdomains
    dict(N=(12, 12, 12), P=(2, 2, 12)),   # one node per subdomain on an axis
    dict(W=0),
    dict(rounds=5),
])
def test_setup_rejects_invalid_3d_arguments(bad):
    from paper_2003_02585_amd import hdsw as H
    N = bad.get("N", (12, 12, 12))
    kap = np.full(tuple(reversed(N)), 40.0)
    opt = H.hdsw_default_options(rounds=bad.get("rounds", 1))
    with pytest.raises(H.HdswError) as ei:
        H.hdsw_setup(kap, 1.0 / N[0], bad.get("P", (2, 2, 2)), bad.get("W", 3), opt)
    assert ei.value.status == H.HDSW_EINVAL


def test_allocator_hooks_default_and_pairing():
    # no hooks by default; one hook without the other is refused on the host
    from paper_2003_02585_amd import hdsw as H
    o = H.hdsw_default_options()
    assert not o.dev_alloc and not o.dev_free and not o.alloc_ctx
    alloc = H.DEV_ALLOC_FN(lambda n, c: None)
    kap = np.full((32, 32), 40.0)
    with pytest.raises(H.HdswError) as ei:
        H.hdsw_setup(kap, 1.0 / 32, (2, 2), 8, H.hdsw_default_options(dev_alloc=alloc))
    assert ei.value.status == H.HDSW_EINVAL


def test_binding_refuses_unknown_contexts():
    import ctypes
    from paper_2003_02585_amd import hdsw as H
    with pytest.raises(ValueError):
        H._sizes(ctypes.c_void_p(12345))


def test_setup_rejects_four_dimensions():
    from paper_2003_02585_amd import hdsw as H
    kap = np.full((4, 4, 4, 4), 40.0)
    with pytest.raises(H.HdswError) as ei:
        H.hdsw_setup(kap, 0.25, (2, 2, 2), 1, H.hdsw_default_options())
    assert ei.value.status == H.HDSW_EINVAL
