"""CPU-side checks of the C-ABI library: it loads, exports every function of
include/rav.h, validates descriptors before touching a device, and its
host-side patch/owner maps (the index code the kernels use) equal the
oracle's bit for bit."""
import ctypes

import numpy as np
import pytest

import rav_inputs as ri
from oracle import patches as pt
from oracle.grid import Grid
from paper_2103_10127_amd import capi


def test_library_exports_every_header_symbol():
    lib = capi.lib()
    names = capi.header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
        assert name in capi.SIGNATURES, name


@pytest.mark.parametrize("field,value,status", [
    ("dim", 4, -1), ("n_levels", 1, -1), ("n_cells", 30, -1), ("omega", 0.0, -1),
    ("nu_pre", -1, -1), ("eta_out", -1.0, -1), ("bc_dirichlet_mask", 0x100, -1),
    ("n_incl", 70, -1), ("smoother", 7, -1), ("inv_precision", 5, -1),
    ("n_levels", 2, -1),   # with n_cells = 512 (set below): a 256x256 coarsest grid is too large
])
def test_invalid_descriptor_rejected_without_device(field, value, status):
    d = capi.make_desc(dim=2, n_cells=32, n_levels=3)
    setattr(d, field, value)
    if (field, value) == ("n_levels", 2):
        d.n_cells = 512
    h = ctypes.c_void_p()
    st = capi.lib().rav_create(ctypes.byref(d), None, ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert len(capi.lib().rav_last_error(None)) > 0


def test_unsupported_combinations():
    lib = capi.lib()
    h = ctypes.c_void_p()
    d = capi.make_desc(dim=3, n_cells=8, n_levels=2, dmask=ri.ALL_DIRICHLET_3D, kind="vertex", smoother="av")
    assert lib.rav_create(ctypes.byref(d), None, ctypes.byref(h)) == -6
    d = capi.make_desc(dim=3, n_cells=8, n_levels=2, dmask=ri.ALL_DIRICHLET_3D, kind="vertex", smoother="mv")
    assert lib.rav_create(ctypes.byref(d), None, ctypes.byref(h)) == -6
    d = capi.make_desc(smoother="av", precision="bf16")
    assert lib.rav_create(ctypes.byref(d), None, ctypes.byref(h)) == -6


@pytest.mark.parametrize("dim,N,nl,kind,dm", [
    (2, 16, 3, "vertex", ri.ALL_DIRICHLET_2D), (2, 12, 2, "vertex", ri.OUTFLOW_2D),
    (3, 4, 2, "element", ri.ALL_DIRICHLET_3D), (3, 6, 2, "element", ri.OUTFLOW_3D),
    (3, 4, 2, "vertex", ri.ALL_DIRICHLET_3D), (3, 4, 2, "vertex", ri.OUTFLOW_3D),
    (2, 10, 2, "element", ri.ALL_DIRICHLET_2D)])
def test_host_maps_match_oracle(dim, N, nl, kind, dm):
    d = capi.make_desc(dim=dim, n_cells=N, n_levels=nl, dmask=dm, kind=kind)
    okind = pt.VERTEX if kind == "vertex" else pt.ELEMENT
    for level in range(nl):
        Nl = N >> (nl - 1 - level)
        g = Grid(dim, Nl, dm)
        ps = pt.PatchSet(g, okind)
        own = capi.map_owner(d, level, g.n)
        np.testing.assert_array_equal(own, ps.owner)
        for i in range(ps.count):
            dofs, owned = capi.map_patch(d, level, i)
            np.testing.assert_array_equal(dofs, ps.dofs[i])
            np.testing.assert_array_equal(np.nonzero(owned)[0], ps.owned[i])


def test_host_owner_map_512_counts():
    """Owner map of the 512x512 level: every free DoF owned once, and owned
    counts per patch reproduce the bucket histogram."""
    d = capi.make_desc(dim=2, n_cells=512, n_levels=7)
    g = Grid(2, 512, ri.ALL_DIRICHLET_2D)
    own = capi.map_owner(d, 6, g.n)
    assert np.array_equal(own >= 0, g.free)
    counts = np.bincount(own[own >= 0], minlength=g.nP)
    hist = np.bincount(counts)
    assert hist[9] == 259081 + 2036 + 4 and hist[5] == 1018 + 4 and hist[3] == 1


@pytest.mark.parametrize("dim,N,nl", [(2, 8192, 10), (3, 256, 6)])
def test_levels_beyond_32bit_index_math_rejected(dim, N, nl):
    """A finest level of 2^28 or more entries would overflow the kernels'
    32-bit index math: rav_create refuses it before any device work."""
    dm = ri.ALL_DIRICHLET_2D if dim == 2 else ri.ALL_DIRICHLET_3D
    d = capi.make_desc(dim=dim, n_cells=N, n_levels=nl, dmask=dm, kind="vertex" if dim == 2 else "element")
    h = ctypes.c_void_p()
    assert capi.lib().rav_create(ctypes.byref(d), None, ctypes.byref(h)) == -6
    assert h.value is None
    assert b"2^28" in capi.lib().rav_last_error(None) or "2^28" in str(capi.lib().rav_last_error(None))


def test_largest_supported_2d_level_passes_the_index_check():
    """N = 4096 in 2D (151 M entries) is below the bound: a descriptor that is
    invalid only in omega fails on omega, i.e. after the size check."""
    d = capi.make_desc(dim=2, n_cells=4096, n_levels=10)
    d.omega = 0.0
    h = ctypes.c_void_p()
    assert capi.lib().rav_create(ctypes.byref(d), None, ctypes.byref(h)) == -1


@pytest.mark.parametrize("dim,N,nl,dm", [(2, 8, 2, ri.ALL_DIRICHLET_2D), (2, 12, 2, ri.OUTFLOW_2D),
                                         (3, 4, 2, ri.OUTFLOW_3D)])
def test_q1q1_host_maps_match_oracle(dim, N, nl, dm):
    """Stabilized Q1-Q1 vertex patches (Sec. 3): patch DoF lists in local order
    and the literal owned set (pressure + co-located velocity) against the oracle."""
    from oracle import q1q1 as q
    d = capi.make_desc(dim=dim, n_cells=N, n_levels=nl, dmask=dm, discretization="q1q1")
    for level in range(nl):
        g = q.GridQ1(dim, N >> (nl - 1 - level), dm)
        ps = q.PatchSetQ1(g)
        np.testing.assert_array_equal(capi.map_owner(d, level, g.n), ps.owner)
        for i in range(ps.count):
            dofs, owned = capi.map_patch(d, level, i)
            np.testing.assert_array_equal(dofs, ps.dofs[i])
            np.testing.assert_array_equal(np.nonzero(owned)[0], ps.owned[i])


@pytest.mark.parametrize("field,value,status", [
    ("beta", 0.0, -1), ("smoother", 7, -1), ("inv_precision", 2, -6), ("patch", 1, -6), ("discretization", 5, -1),
    ("n_levels", 2, -1),   # with n_cells = 256: 3 * 129^2 coarsest unknowns exceed the dense solve
])
def test_q1q1_invalid_descriptors_rejected_without_device(field, value, status):
    d = capi.make_desc(dim=2, n_cells=32, n_levels=3, discretization="q1q1")
    setattr(d, field, value)
    if (field, value) == ("n_levels", 2):
        d.n_cells = 256
    h = ctypes.c_void_p()
    assert capi.lib().rav_create(ctypes.byref(d), None, ctypes.byref(h)) == status
    assert h.value is None
