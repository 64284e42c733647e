"""The allocation-free CFL time step (igr_compute_dt_noalloc) against the
context-based igr_compute_dt, through the C ABI.

Both run the same reduction kernels on the same fixed grid, so the FP64
time steps agree bitwise.  Two calls in a row, the second on a smaller
grid, check that the shared device array carries nothing over; a state
with a negative density must report IGR_ENONFINITE, and the next valid
call must succeed (the flag is cleared per call)."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2505_07392_amd import igr, inputs
from gpu_common import banner

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _noalloc_dt(s, U, cfl):
    dt = ctypes.c_double(0.0)
    grid = igr.Grid(s.nx, s.ny, s.nz, s.dx, s.dy, s.dz)
    rc = igr.lib().igr_compute_dt_noalloc(ctypes.byref(grid), s.gamma, igr.PRECISION[s.precision][0],
                                          ctypes.c_void_p(U.data_ptr()), cfl, ctypes.byref(dt),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, dt.value


@pytest.mark.parametrize("precision", ["f64", "f32", "f16", "bf16"])
def test_noalloc_dt_matches_context_dt(precision):
    for n, seed in ((40, 1), (17, 2)):        # second call: a smaller grid
        banner(f"noalloc dt {precision} {n}^3 seed {seed}")
        w = inputs.periodic_box(n=n, seed=seed)
        s = igr.Solver.from_workload(w, precision=precision)
        U = s.state_from(w.U)
        want = s.compute_dt(U, 0.5)
        rc, got = _noalloc_dt(s, U, 0.5)
        assert rc == igr.IGR_OK, igr.lib().igr_last_error().decode()
        assert got == want, (got, want)
        s.close()


def test_noalloc_dt_nonfinite_then_recovers():
    banner("noalloc dt non-finite flag")
    w = inputs.periodic_box(n=20, seed=4)
    s = igr.Solver.from_workload(w, precision="f64")
    bad = w.U.copy()
    bad[0, 3, 4, 5] = -1.0                    # rho < 0 in one cell
    Ub = s.state_from(bad)
    rc, _ = _noalloc_dt(s, Ub, 0.5)
    assert rc == igr.IGR_ENONFINITE
    U = s.state_from(w.U)
    rc, got = _noalloc_dt(s, U, 0.5)
    assert rc == igr.IGR_OK
    assert got == s.compute_dt(U, 0.5)
    s.close()


def test_noalloc_dt_rejects_bad_arguments():
    s = igr.Solver(8, 8, 8, 0.125, 0.125, 0.125)
    U = s.new_state()
    dt = ctypes.c_double(0.0)
    L = igr.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = igr.Grid(8, 8, 8, 0.125, 0.125, 0.125)
    assert L.igr_compute_dt_noalloc(None, 1.4, 0, ctypes.c_void_p(U.data_ptr()), 0.5, ctypes.byref(dt), st) \
        == igr.IGR_EINVAL
    assert L.igr_compute_dt_noalloc(ctypes.byref(g), 1.0, 0, ctypes.c_void_p(U.data_ptr()), 0.5,
                                    ctypes.byref(dt), st) == igr.IGR_EINVAL
    assert L.igr_compute_dt_noalloc(ctypes.byref(g), 1.4, 9, ctypes.c_void_p(U.data_ptr()), 0.5,
                                    ctypes.byref(dt), st) == igr.IGR_EINVAL
    big = igr.Grid(50000, 50000, 1, 1.0, 1.0, 1.0)
    assert L.igr_compute_dt_noalloc(ctypes.byref(big), 1.4, 0, ctypes.c_void_p(U.data_ptr()), 0.5,
                                    ctypes.byref(dt), st) == igr.IGR_EINVAL
    s.close()
