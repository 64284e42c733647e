"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function that include/igr.h declares, and argument
validation rejects bad input before any device call."""

import ctypes
import os
import re

import pytest

from paper_2505_07392_amd import igr

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "igr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(igr_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("igr_init", "igr_sigma_solve", "igr_rhs", "igr_step", "igr_finalize", "igr_compute_dt",
                     "igr_sums", "igr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = igr.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(igr._SIGNATURES)


def _grid(n=8):
    return igr.Grid(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n)


def _bc(kind=1):
    return igr.BC((ctypes.c_int32 * 6)(*([kind] * 6)), 0, None)


def _init(grid, gamma, alpha, bc, opts):
    h = ctypes.c_void_p()
    rc = igr.lib().igr_init(ctypes.byref(grid) if grid else None, gamma, alpha, ctypes.byref(bc) if bc else None,
                            ctypes.byref(opts) if opts else None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case,code", [
    ("null", igr.IGR_EINVAL), ("gamma", igr.IGR_EINVAL), ("alpha", igr.IGR_EINVAL), ("extent", igr.IGR_EINVAL),
    ("pair", igr.IGR_EINVAL), ("precision", igr.IGR_EINVAL), ("order", igr.IGR_EUNSUPPORTED),
    ("sweeps", igr.IGR_EINVAL), ("spacing", igr.IGR_EINVAL), ("sigma_block", igr.IGR_EINVAL),
    ("smoother", igr.IGR_EINVAL), ("rbgs_odd_periodic", igr.IGR_EUNSUPPORTED),
    ("plane_too_large", igr.IGR_EINVAL), ("split_march", igr.IGR_EUNSUPPORTED),
    ("negative_mu", igr.IGR_EINVAL), ("negative_zeta", igr.IGR_EINVAL),
])
def test_init_rejects_bad_arguments(case, code):
    grid, bc, opts, gamma, alpha = _grid(), _bc(), igr.Opts(0, 5, 5, 0), 1.4, 0.01
    if case == "null":
        grid = None
    elif case == "gamma":
        gamma = 1.0
    elif case == "alpha":
        alpha = -1.0
    elif case == "extent":
        grid = igr.Grid(0, 8, 8, 0.1, 0.1, 0.1)
    elif case == "pair":
        bc = igr.BC((ctypes.c_int32 * 6)(0, 1, 0, 0, 0, 0), 0, None)
    elif case == "precision":
        opts = igr.Opts(7, 5, 5, 0)
    elif case == "order":
        opts = igr.Opts(0, 4, 5, 0)
    elif case == "sweeps":
        opts = igr.Opts(0, 5, -1, 0)
    elif case == "spacing":
        grid = igr.Grid(8, 8, 8, 0.0, 0.1, 0.1)
    elif case == "sigma_block":
        opts = igr.Opts(0, 5, 5, 9)
    elif case == "smoother":
        opts = igr.Opts(0, 5, 5, 0, 2)
    elif case == "rbgs_odd_periodic":
        grid = igr.Grid(8, 7, 8, 0.1, 0.1, 0.1)
        bc = igr.BC((ctypes.c_int32 * 6)(1, 1, 0, 0, 1, 1), 0, None)
        opts = igr.Opts(0, 5, 5, 0, 1)
    elif case == "plane_too_large":
        grid = igr.Grid(50000, 50000, 1, 1e-4, 1e-4, 1e-4)   # padded x-y plane beyond 32-bit offsets
    elif case == "split_march":
        opts = igr.Opts(4, 5, 5, 3)   # the split form runs single or two-sweep passes only
    elif case == "negative_mu":
        opts = igr.Opts(0, 5, 5, 0, 0, -1e-3, 0.0)
    elif case == "negative_zeta":
        opts = igr.Opts(0, 5, 5, 0, 0, 1e-3, -1e-3)
    rc, h = _init(grid, gamma, alpha, bc, opts)
    assert rc == code
    assert h.value is None
    assert igr.lib().igr_last_error()


def test_inflow_needs_nonperiodic_x():
    patches = (igr.Patch * 1)(igr.Patch(0.5, 0.5, 0.1, 0.0, 1.0, 1.0, 0.0, 0.0, 1.0))
    bc = igr.BC((ctypes.c_int32 * 6)(*([0] * 6)), 1, patches)
    rc, _ = _init(_grid(), 1.4, 0.0, bc, igr.Opts(0, 5, 5, 0))
    assert rc == igr.IGR_EINVAL


def test_null_context_calls():
    L = igr.lib()
    assert L.igr_finalize(None) == igr.IGR_OK
    assert L.igr_rhs(None, None, None, None, None) == igr.IGR_EINVAL
    assert L.igr_step(None, None, None, 0.5, 0.0, None, None) == igr.IGR_EINVAL
    assert L.igr_check(None, None) == igr.IGR_EINVAL
    opts = igr.Opts()
    assert L.igr_get_opts(None, ctypes.byref(opts)) == igr.IGR_EINVAL
    assert L.igr_advance(None, None, None, 1, 0.5, 0.0, None, None) == igr.IGR_EINVAL


def test_kernel_names():
    names = igr.kernel_names()
    assert "flux_rk" in names and "jacobi" in names
    assert "stress" in names and "viscous" in names
