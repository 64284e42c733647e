"""Pins of the oracle's reconstruction and Sigma source (CPU only).

Reconstruction ("Discretization"; Algorithm 1, stencil q = -2..3): a
fifth-order finite-volume interpolant is exact for cell averages of every
polynomial of degree <= 4 and not for degree 5; left and right states are
mirror images.  Source (eq. 9, left side): for a linear velocity u = A x the
central differences are exact, so b = alpha [tr(A^2) + tr(A)^2].
"""

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref


def _line_problem(n):
    return ref.Problem(n, 1, 1, 1.0, 1.0, 1.0, faces=(ref.PERIODIC,) * 6)


def _cell_averages(k, lo, n):
    """Exact averages of x^k over cells [i, i+1], i = lo .. lo+n-1."""
    i = np.arange(lo, lo + n, dtype=np.float64)
    return ((i + 1) ** (k + 1) - i ** (k + 1)) / (k + 1)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_reconstruction_exact_for_degree_le_4(k):
    n = 10
    prob = _line_problem(n)
    avg = _cell_averages(k, -3, n + 6)                     # padded cells -3..n+2
    q = torch.from_numpy(avg).reshape(1, 1, -1).expand(7, 7, -1).contiguous()
    left, right = ref.reconstruct(prob, q, 0)
    faces = np.arange(0, n + 1, dtype=np.float64)          # face f at x = f
    exact = faces ** k
    scale = max(1.0, np.abs(exact).max())
    assert np.abs(left[0, 0].numpy() - exact).max() <= 1e-12 * scale
    assert np.abs(right[0, 0].numpy() - exact).max() <= 1e-12 * scale


def test_reconstruction_not_exact_for_degree_5():
    n = 10
    prob = _line_problem(n)
    q = torch.from_numpy(_cell_averages(5, -3, n + 6)).reshape(1, 1, -1).expand(7, 7, -1).contiguous()
    left, _ = ref.reconstruct(prob, q, 0)
    err = np.abs(left[0, 0].numpy() - np.arange(0, n + 1) ** 5.0).max()
    assert err > 1e-3


def test_reconstruction_mirror_symmetry():
    n = 12
    prob = _line_problem(n)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(n + 6)
    q = torch.from_numpy(v).reshape(1, 1, -1).expand(7, 7, -1).contiguous()
    qm = torch.from_numpy(v[::-1].copy()).reshape(1, 1, -1).expand(7, 7, -1).contiguous()
    left, right = ref.reconstruct(prob, q, 0)
    left_m, right_m = ref.reconstruct(prob, qm, 0)
    # same weights, opposite summation order: equal to rounding
    assert torch.allclose(left[0, 0], right_m[0, 0].flip(0), rtol=0, atol=1e-14)
    assert torch.allclose(right[0, 0], left_m[0, 0].flip(0), rtol=0, atol=1e-14)


def test_reconstruction_weights_match_linear_weno5_combination():
    """The five-cell interpolant is 1/10, 6/10, 3/10 times the three
    third-order candidate stencils (standard optimal linear weights)."""
    c0 = np.array([2, -7, 11, 0, 0]) / 6.0   # cells i-2..i
    c1 = np.array([0, -1, 5, 2, 0]) / 6.0    # cells i-1..i+1
    c2 = np.array([0, 0, 2, 5, -1]) / 6.0    # cells i..i+2
    comb = 0.1 * c0 + 0.6 * c1 + 0.3 * c2
    assert np.allclose(comb, np.array(ref.RECON_LEFT) / ref.RECON_DENOM, atol=1e-15)
    assert np.allclose(comb[::-1], np.array(ref.RECON_RIGHT) / ref.RECON_DENOM, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_source_exact_for_linear_velocity(seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3))
    nx, ny, nz = 7, 6, 5
    h = (0.3, 0.2, 0.25)
    alpha = 0.7
    prob = ref.Problem(nx, ny, nz, *h, alpha=alpha)
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h[2], (np.arange(ny) + 0.5) * h[1],
                          (np.arange(nx) + 0.5) * h[0], indexing="ij")
    X = np.stack([x, y, z])
    u = np.einsum("ij,j...->i...", A, X)
    rho = 1.3
    U = torch.from_numpy(np.concatenate([np.full((1,) + x.shape, rho), rho * u,
                                         np.full((1,) + x.shape, 5.0)]))
    b = ref.sigma_source(prob, ref.pad_state(prob, U))
    expect = alpha * (np.trace(A @ A) + np.trace(A) ** 2)
    inner = b[1:-1, 1:-1, 1:-1].numpy()     # boundary cells see extrapolated ghosts
    assert np.abs(inner - expect).max() <= 1e-11 * max(1.0, abs(expect))


def test_source_rotation_is_negative():
    """Rigid rotation u = (-y, x, 0): tr(G^2) = -2, tr(G) = 0, b = -2 alpha."""
    n = 6
    prob = ref.Problem(n, n, n, 1.0, 1.0, 1.0, alpha=0.5)
    z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    U = torch.from_numpy(np.stack([np.ones_like(x), -y, x, np.zeros_like(x), np.full_like(x, 9.0)]))
    b = ref.sigma_source(prob, ref.pad_state(prob, U))
    assert np.allclose(b[1:-1, 1:-1, 1:-1].numpy(), -1.0, atol=1e-13)


def test_source_zero_for_uniform_flow():
    n = 5
    prob = ref.Problem(n, n, n, 0.1, 0.1, 0.1, alpha=1.0, faces=(ref.PERIODIC,) * 6)
    U = torch.tensor([1.1, 0.3, -0.2, 0.5, 4.0], dtype=torch.float64).reshape(5, 1, 1, 1).expand(5, n, n, n)
    b = ref.sigma_source(prob, ref.pad_state(prob, U.contiguous()))
    assert torch.count_nonzero(b) == 0
