"""Pins of the oracle's entropic-pressure solve (eq. 9; "Discretization":
7-point stencil, a fixed number of warm-started Jacobi sweeps).

The discrete operator is assembled here by brute force, one cell at a time
from the textbook 7-point formula, independently of the oracle's
whole-array code; the oracle's sweep must equal D^-1 (b + O Sigma) of that
assembly, the operator must be symmetric, Jacobi run to convergence must
reproduce a dense solve, and the uniform-density contraction factor is the
closed form 6/7 when alpha = h^2.
"""

import itertools

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref


def _problem():
    # non-cubic, anisotropic, mixed boundaries, a jet disc on x-min
    nx, ny, nz = 6, 5, 4
    h = (0.21, 0.17, 0.23)
    jet = ref.Patch(yc=0.4, zc=0.45, r=0.2, rho=0.37, ux=2.0, uy=0.1, uz=-0.2, p=3.0)
    return ref.Problem(nx, ny, nz, *h, alpha=0.05,
                       faces=(ref.EXTRAP, ref.EXTRAP, ref.PERIODIC, ref.PERIODIC, ref.EXTRAP, ref.EXTRAP),
                       patches=(jet,))


def _rho_ghost(prob, rho, jet_rho, owner, cell, d, s):
    """Density seen across face (cell, d, s): neighbour or ghost per BC."""
    idx = list(cell)  # (i, j, k)
    idx[d] += s
    n = prob.n(d)
    if 0 <= idx[d] < n:
        return rho[idx[2], idx[1], idx[0]], tuple(idx), False
    if prob.axis_kind(d) == ref.PERIODIC:
        idx[d] %= n
        return rho[idx[2], idx[1], idx[0]], tuple(idx), False
    i, j, k = cell
    if d == 0 and s < 0 and owner[k, j] >= 0:
        return jet_rho, None, True
    return rho[k, j, i], None, True


def _assemble(prob, rho):
    """Brute-force D (diagonal of the sweep) and O (coupling incl. the
    zero-gradient ghost self-coupling) for the sweep ordering x fastest."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    N = nx * ny * nz
    lin = lambda i, j, k: (k * ny + j) * nx + i
    D = np.zeros(N)
    O = np.zeros((N, N))
    pa = prob.patches[0]      # one sharp disc: owner 0 inside, -1 outside
    owner = np.full((nz, ny), -1)
    chi = np.zeros((nz, ny))
    for k, j in itertools.product(range(nz), range(ny)):
        y, z = (j + 0.5) * prob.dy, (k + 0.5) * prob.dz
        if (y - pa.yc) ** 2 + (z - pa.zc) ** 2 <= pa.r ** 2:
            owner[k, j], chi[k, j] = 0, 1.0
    assert owner.max() == 0 and owner.min() == -1   # the disc covers some columns, not all
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        c = lin(i, j, k)
        D[c] += 1.0 / rho[k, j, i]
        for d in range(3):
            for s in (-1, 1):
                rnb, nb, ghost = _rho_ghost(prob, rho, 0.0, owner, (i, j, k), d, s)
                if ghost and d == 0 and s < 0 and owner[k, j] >= 0:
                    x = chi[k, j]
                    rnb = x * prob.patches[0].rho + (1 - x) * rho[k, j, i]
                beta = 0.5 * (1.0 / rho[k, j, i] + 1.0 / rnb)
                coef = prob.alpha * beta / prob.h(d) ** 2
                D[c] += coef
                target = c if nb is None else lin(*nb)
                O[c, target] += coef
    return D, O


def _fields(prob, seed):
    rng = np.random.default_rng(seed)
    shape = prob.shape
    rho = 0.5 + rng.random(shape)
    U = np.stack([rho, rho * rng.standard_normal(shape) * 0.1, rho * 0.0, rho * 0.0, 3.0 + rng.random(shape)])
    return rho, torch.from_numpy(U), rng.standard_normal(shape), rng.standard_normal(shape)


@pytest.mark.parametrize("seed", [0, 1])
def test_sweep_matches_brute_force_assembly(seed):
    prob = _problem()
    rho, U, b, sig = _fields(prob, seed)
    D, O = _assemble(prob, rho)
    got = ref.jacobi_sweep(prob, torch.from_numpy(sig), torch.from_numpy(b), ref.pad_state(prob, U)[0])
    expect = (b.ravel() + O @ sig.ravel()) / D
    assert np.abs(got.numpy().ravel() - expect).max() <= 1e-13 * np.abs(expect).max()


def test_operator_symmetric_and_matches_apply():
    prob = _problem()
    rho, U, b, sig = _fields(prob, 2)
    D, O = _assemble(prob, rho)
    A = np.diag(D) - O
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    got = ref.apply_sigma_operator(prob, U, torch.from_numpy(sig)).numpy().ravel()
    assert np.abs(got - A @ sig.ravel()).max() <= 1e-13 * np.abs(got).max()
    # positive definite: the Jacobi splitting of an SPD, diagonally dominant matrix converges
    assert np.linalg.eigvalsh(A).min() > 0


def test_jacobi_converges_to_dense_solve():
    prob = _problem()
    rho, U, b, sig = _fields(prob, 3)
    D, O = _assemble(prob, rho)
    exact = np.linalg.solve(np.diag(D) - O, b.ravel())
    s = torch.zeros(prob.shape, dtype=torch.float64)
    rho_pad = ref.pad_state(prob, U)[0]
    bt = torch.from_numpy(b)
    for _ in range(400):
        s = ref.jacobi_sweep(prob, s, bt, rho_pad)
    assert np.abs(s.numpy().ravel() - exact).max() <= 1e-12 * np.abs(exact).max()


def test_uniform_density_contraction_six_sevenths():
    """Uniform rho, periodic, alpha = h^2: D = 7/rho and O e = 6/rho e for
    the constant mode (factor 6/7) and -6/rho e for the checkerboard mode."""
    n = 8
    h = 0.125
    prob = ref.Problem(n, n, n, h, h, h, alpha=h * h, faces=(ref.PERIODIC,) * 6)
    rho = 2.0
    U = torch.zeros((5, n, n, n), dtype=torch.float64)
    U[0] = rho
    U[4] = 2.5
    rho_pad = ref.pad_state(prob, U)[0]
    zero = torch.zeros(prob.shape, dtype=torch.float64)
    one = torch.ones(prob.shape, dtype=torch.float64)
    out = ref.jacobi_sweep(prob, one, zero, rho_pad)
    assert torch.allclose(out, one * 6.0 / 7.0, rtol=0, atol=1e-15)
    k, j, i = np.meshgrid(range(n), range(n), range(n), indexing="ij")
    cb = torch.from_numpy((-1.0) ** (i + j + k))
    out = ref.jacobi_sweep(prob, cb, zero, rho_pad)
    assert torch.allclose(out, -cb * 6.0 / 7.0, rtol=0, atol=1e-15)
    # five sweeps: (6/7)^5 = 0.4627...
    s = one
    for _ in range(5):
        s = ref.jacobi_sweep(prob, s, zero, rho_pad)
    assert abs(float(s[0, 0, 0]) - (6.0 / 7.0) ** 5) < 1e-15


def test_sigma_solve_uses_source_and_warm_start():
    """sigma_solve = source followed by exactly nsweeps sweeps from sigma0."""
    prob = _problem()
    rho, U, b, sig = _fields(prob, 4)
    s0 = torch.from_numpy(sig)
    got, bb = ref.sigma_solve(prob, U, s0, nsweeps=3)
    Upad = ref.pad_state(prob, U)
    s = s0
    for _ in range(3):
        s = ref.jacobi_sweep(prob, s, bb, Upad[0])
    assert torch.equal(got, s)
    got0, _ = ref.sigma_solve(prob, U, s0, nsweeps=0)
    assert torch.equal(got0, s0)


def test_residual_decreases_with_sweeps():
    prob = _problem()
    prob.alpha = 0.01
    rho, U, b, sig = _fields(prob, 5)
    s = torch.zeros(prob.shape, dtype=torch.float64)
    r = []
    for k in (1, 5, 20):
        sk, _ = ref.sigma_solve(prob, U, s, nsweeps=k)
        r.append(ref.sigma_residual_l2(prob, U, sk))
    assert r[0] > r[1] > r[2]


def test_residual_is_the_norm_of_the_assembled_system():
    """sigma_residual_l2 = ||b - A Sigma||_2 with A from the brute-force
    assembly: with zero momentum in the domain the source is non-zero only
    in the cells beside the jet disc (whose ghost state moves), so the
    residual of a random Sigma is ||b - A Sigma|| with that sparse b; with
    momentum, the residual at the dense solution of A Sigma = b is zero to
    round-off."""
    prob = _problem()
    rho, U, b, sig = _fields(prob, 6)
    D, O = _assemble(prob, rho)
    A = np.diag(D) - O
    U0 = U.clone()
    U0[1:4] = 0.0
    b0 = ref.sigma_source(prob, ref.pad_state(prob, U0)).numpy()
    assert np.count_nonzero(b0[:, :, 1:]) == 0      # only the x = 0 layer sees the moving jet ghost
    got = ref.sigma_residual_l2(prob, U0, torch.from_numpy(sig))
    want = np.linalg.norm(b0.ravel() - A @ sig.ravel())
    assert abs(got - want) <= 1e-13 * want
    bsrc = ref.sigma_source(prob, ref.pad_state(prob, U)).numpy().ravel()
    assert np.abs(bsrc).max() > 0
    exact = np.linalg.solve(A, bsrc).reshape(prob.shape)
    assert ref.sigma_residual_l2(prob, U, torch.from_numpy(exact)) <= 1e-12 * np.linalg.norm(bsrc)
