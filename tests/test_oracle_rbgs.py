"""Pins of the oracle's red-black Gauss-Seidel smoother (the paper's
alternative to Jacobi sweeps, "Discretization"), CPU only.

Against the brute-force assembly A = D - O of the 7-point operator (the one
the Jacobi pins use): a red-black sweep equals the Gauss-Seidel iteration
written out cell by cell in red-then-black order; after a sweep every black
cell satisfies its equation exactly (its neighbours are all red and final);
sweeps converge to the dense solve, faster than Jacobi; and for uniform
density with alpha = h^2 on a periodic box the constant error mode becomes
6/7 on red and (6/7)^2 on black cells after one sweep.
"""

import itertools

import numpy as np
import torch

from oracle import igr_ref as ref
from test_oracle_sigma import _assemble, _fields


def _problem():
    # even periodic extent (y), extrapolation elsewhere, a jet disc on x-min
    jet = ref.Patch(yc=0.4, zc=0.45, r=0.2, rho=0.37, ux=2.0, uy=0.1, uz=-0.2, p=3.0)
    return ref.Problem(5, 6, 4, 0.21, 0.17, 0.23, alpha=0.05,
                       faces=(ref.EXTRAP, ref.EXTRAP, ref.PERIODIC, ref.PERIODIC, ref.EXTRAP, ref.EXTRAP),
                       patches=(jet,), smoother="rbgs")


def _brute_force_gs(prob, D, O, b, sig):
    """Gauss-Seidel in red-then-black order, one cell at a time, on the
    assembled rows (the iterate is updated in place)."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    x = sig.ravel().copy()
    bb = b.ravel()
    lin = lambda i, j, k: (k * ny + j) * nx + i
    for colour in (0, 1):
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            if (i + j + k) % 2 != colour:
                continue
            c = lin(i, j, k)
            x[c] = (bb[c] + O[c] @ x) / D[c]      # a zero-gradient ghost couples to the old x[c]
    return x


def test_rbgs_sweep_is_gauss_seidel_in_red_black_order():
    prob = _problem()
    rho, U, b, sig = _fields(prob, 7)
    D, O = _assemble(prob, rho)
    rho_pad = ref.pad_state(prob, U)[0]
    got = ref.rbgs_sweep(prob, torch.from_numpy(sig), torch.from_numpy(b), rho_pad).numpy().ravel()
    want = _brute_force_gs(prob, D, O, b, sig)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_black_cells_satisfy_their_equations_after_a_sweep():
    prob = _problem()
    rho, U, b, sig = _fields(prob, 8)
    D, O = _assemble(prob, rho)
    A = np.diag(D) - O
    rho_pad = ref.pad_state(prob, U)[0]
    out = ref.rbgs_sweep(prob, torch.from_numpy(sig), torch.from_numpy(b), rho_pad).numpy().ravel()
    r = b.ravel() - A @ out
    black = ~ref.red_cells(prob).numpy().ravel()
    inner = np.diag(O) == 0          # no zero-gradient face (whose ghost is the cell's previous value)
    assert (black & inner).sum() > 10
    assert np.abs(r[black & inner]).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(r[~black]).max() > 1e-3          # red cells are one half-sweep behind


def test_rbgs_converges_to_dense_solve_faster_than_jacobi():
    prob = _problem()
    rho, U, b, sig = _fields(prob, 9)
    D, O = _assemble(prob, rho)
    exact = np.linalg.solve(np.diag(D) - O, b.ravel())
    rho_pad = ref.pad_state(prob, U)[0]
    bt = torch.from_numpy(b)
    s_gs = torch.zeros(prob.shape, dtype=torch.float64)
    s_j = torch.zeros(prob.shape, dtype=torch.float64)
    for _ in range(10):
        s_gs = ref.rbgs_sweep(prob, s_gs, bt, rho_pad)
        s_j = ref.jacobi_sweep(prob, s_j, bt, rho_pad)
    e_gs = np.abs(s_gs.numpy().ravel() - exact).max()
    e_j = np.abs(s_j.numpy().ravel() - exact).max()
    assert e_gs < 0.5 * e_j
    for _ in range(300):
        s_gs = ref.rbgs_sweep(prob, s_gs, bt, rho_pad)
    assert np.abs(s_gs.numpy().ravel() - exact).max() <= 1e-12 * np.abs(exact).max()


def test_uniform_density_constant_mode():
    n, h = 8, 0.125
    prob = ref.Problem(n, n, n, h, h, h, alpha=h * h, faces=(ref.PERIODIC,) * 6, smoother="rbgs")
    U = torch.zeros((5, n, n, n), dtype=torch.float64)
    U[0] = 2.0
    U[4] = 2.5
    rho_pad = ref.pad_state(prob, U)[0]
    one = torch.ones(prob.shape, dtype=torch.float64)
    out = ref.rbgs_sweep(prob, one, torch.zeros_like(one), rho_pad)
    red = ref.red_cells(prob)
    assert torch.allclose(out[red], torch.full_like(out[red], 6.0 / 7.0), rtol=0, atol=1e-15)
    assert torch.allclose(out[~red], torch.full_like(out[~red], 36.0 / 49.0), rtol=0, atol=1e-15)


def test_sigma_solve_dispatches_on_the_smoother():
    prob = _problem()
    rho, U, b, sig = _fields(prob, 10)
    got, bb = ref.sigma_solve(prob, U, torch.from_numpy(sig), nsweeps=2)
    rho_pad = ref.pad_state(prob, U)[0]
    s = torch.from_numpy(sig)
    for _ in range(2):
        s = ref.rbgs_sweep(prob, s, bb, rho_pad)
    assert torch.equal(got, s)
