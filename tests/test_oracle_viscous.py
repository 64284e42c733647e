"""Pins of the oracle's viscous terms (eqs. (1)-(3) with the stress of
eq. (5); "Discretization": second-order velocity gradients; Algorithm 1:
gradients reconstructed to the faces with the reconstruction weights).

* a linear velocity field u = A x + c: the central gradient is A exactly,
  the stress is mu (A + A^T) + (zeta - 2 mu / 3) tr(A) I (written out here
  with numpy), and the viscous momentum flux is uniform, so L_v of the
  momenta vanishes while the energy gains the heating -div(u . tau) =
  sum_k tau_kd A_kd, both exact away from the boundaries;
* a rigid rotation (antisymmetric A) has no stress and no viscous term;
* a shear wave u_y = eps sin(k x) on a periodic grid is an eigenvector of
  the discrete viscous operator: L_v(rho v) = -mu s(kh) / h^2 u_y with the
  symbol s = 2 r(kh) sin(kh) sin(kh/2) of central gradient, face
  interpolation by the mean of the two one-sided reconstructions (r: the
  six-point, or for third order the four-point, midpoint interpolant) and
  face difference -- derived here from the Fourier modes, independently of
  the oracle's code path;
* sum over a periodic box of L_v is zero to round-off (conservation).
"""

import math

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref

MU, ZETA = 0.013, 0.007


def _state(rho, u, p, gamma=1.4):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    return torch.cat([rho[None], rho[None] * u, E[None]])


def _grid(n, faces, mu=MU, zeta=ZETA, order=5):
    h = (0.1, 0.13, 0.09)
    return ref.Problem(*n, *h, alpha=0.0, faces=faces, nsweeps=0, mu=mu, zeta=zeta, order=order)


def _centres(prob):
    z, y, x = torch.meshgrid(*[(torch.arange(prob.n(d), dtype=torch.float64) + 0.5) * prob.h(d) for d in (2, 1, 0)],
                             indexing="ij")
    return torch.stack([x, y, z])


def _linear(prob, A, c, rho0=1.3, p0=2.0):
    X = _centres(prob)
    u = torch.einsum("ij,j...->i...", torch.from_numpy(A), X) + torch.from_numpy(c).reshape(3, 1, 1, 1)
    rho = torch.full(prob.shape, rho0, dtype=torch.float64)
    return _state(rho, u, torch.full(prob.shape, p0, dtype=torch.float64))


def _viscous(prob, U):
    Upad = ref.pad_state(prob, U)
    Gm = ref.velocity_gradient(prob, Upad)
    return Gm, ref.viscous_flux_divergence(prob, Upad, ref.pad_gradient(prob, Gm))


INNER = (slice(4, -4), slice(4, -4), slice(4, -4))   # cells whose stencils never reach a ghost


def test_linear_velocity_gradient_stress_and_heating():
    rng = np.random.default_rng(0)
    A = rng.uniform(-1.0, 1.0, (3, 3))
    c = rng.uniform(-0.5, 0.5, 3)
    prob = _grid((14, 13, 12), ("extrap",) * 6)
    U = _linear(prob, A, c)
    Gm, Lv = _viscous(prob, U)
    for i in range(3):
        for j in range(3):
            g = Gm[i][j][1:-1, 1:-1, 1:-1]
            assert torch.allclose(g, torch.full_like(g, A[i, j]), rtol=0, atol=1e-12)
    tau = ref.viscous_stress(prob, Gm)
    want = MU * (A + A.T) + (ZETA - 2.0 * MU / 3.0) * np.trace(A) * np.eye(3)
    for i in range(3):
        for j in range(3):
            t = tau[i][j][1:-1, 1:-1, 1:-1]
            assert torch.allclose(t, torch.full_like(t, want[i, j]), rtol=0, atol=1e-12)
    # uniform stress: no momentum change; energy: sum_d d/dx_d (u . tau e_d)
    # = sum_{k,d} tau_kd A_kd (rho uniform: the face velocities are exact)
    for f in range(4):
        assert Lv[f][INNER].abs().max() <= 1e-12
    heat = float((want * A).sum())
    assert torch.allclose(Lv[4][INNER], torch.full_like(Lv[4][INNER], heat), rtol=1e-12, atol=1e-13)
    assert abs(heat) > 1e-3


@pytest.mark.parametrize("which", ["shear", "compression"])
def test_heating_of_plain_flows(which):
    """u = (0, a x, 0): tau_yx = mu a, heating mu a^2; u = (a x, 0, 0):
    tau_xx = (4 mu / 3 + zeta) a, heating (4 mu / 3 + zeta) a^2."""
    a = 0.7
    A = np.zeros((3, 3))
    if which == "shear":
        A[1, 0] = a
        want = MU * a * a
    else:
        A[0, 0] = a
        want = (4.0 * MU / 3.0 + ZETA) * a * a
    prob = _grid((16, 10, 10), ("extrap",) * 6)
    _, Lv = _viscous(prob, _linear(prob, A, np.zeros(3)))
    assert torch.allclose(Lv[4][INNER], torch.full_like(Lv[4][INNER], want), rtol=1e-12, atol=0)


def test_rigid_rotation_has_no_viscous_term():
    w = np.array([0.3, -0.8, 0.5])
    A = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])   # u = w x X
    prob = _grid((12, 12, 12), ("extrap",) * 6)
    Gm, Lv = _viscous(prob, _linear(prob, A, np.array([0.1, 0.2, -0.3])))
    tau = ref.viscous_stress(prob, Gm)
    for i in range(3):
        for j in range(3):
            assert tau[i][j][1:-1, 1:-1, 1:-1].abs().max() <= 1e-14
    assert Lv[(slice(None),) + INNER].abs().max() <= 1e-13


def _symbol(theta, order):
    """s(kh) of the discrete viscous operator on a shear wave (see module
    docstring).  Midpoint interpolants: the mean of the left (2, -13, 47,
    27, -3)/60 and right (-3, 27, 47, -13, 2)/60 stencils is (1, -8, 37, 37,
    -8, 1)/60; for third order, of (-1, 5, 2)/6 and (2, 5, -1)/6 it is
    (-1, 7, 7, -1)/12."""
    if order == 5:
        r = (2 * 37 * math.cos(theta / 2) - 2 * 8 * math.cos(1.5 * theta) + 2 * math.cos(2.5 * theta)) / 60.0
    else:
        r = (2 * 7 * math.cos(theta / 2) - 2 * math.cos(1.5 * theta)) / 12.0
    return 2.0 * r * math.sin(theta) * math.sin(theta / 2)


@pytest.mark.parametrize("order", [5, 3])
@pytest.mark.parametrize("mode", [1, 3, 7])
def test_shear_wave_is_an_eigenvector(order, mode):
    n = 32
    prob = _grid((n, 4, 3), ("periodic",) * 6, order=order)
    h = prob.dx
    k = 2.0 * math.pi * mode / (n * h)
    X = _centres(prob)
    eps, rho0 = 1e-2, 1.7
    u = torch.zeros((3,) + prob.shape, dtype=torch.float64)
    u[1] = eps * torch.sin(k * X[0])
    U = _state(torch.full(prob.shape, rho0, dtype=torch.float64), u, torch.full(prob.shape, 1.0, dtype=torch.float64))
    _, Lv = _viscous(prob, U)
    want = -MU * _symbol(k * h, order) / h ** 2 * u[1]
    assert torch.allclose(Lv[2], want, rtol=0, atol=1e-12 * float(want.abs().max()))
    assert Lv[0].abs().max() == 0.0
    assert Lv[1].abs().max() <= 1e-15 and Lv[3].abs().max() <= 1e-15
    # the symbol tends to (kh)^2: second-order gradients, higher-order faces
    if mode == 1:
        assert abs(_symbol(k * h, order) / (k * h) ** 2 - 1.0) < 0.02


def test_viscous_terms_conserve_on_a_periodic_box():
    rng = np.random.default_rng(3)
    prob = _grid((10, 9, 8), ("periodic",) * 6)
    shape = prob.shape
    rho = torch.from_numpy(1.0 + 0.2 * rng.random(shape))
    u = torch.from_numpy(0.5 * (2.0 * rng.random((3,) + shape) - 1.0))
    U = _state(rho, u, torch.from_numpy(1.0 + 0.2 * rng.random(shape)))
    _, Lv = _viscous(prob, U)
    scale = Lv.abs().reshape(5, -1).sum(1)
    tot = Lv.reshape(5, -1).sum(1)
    assert tot[0] == 0.0
    assert (tot[1:].abs() <= 1e-13 * scale[1:]).all()
    assert (scale[1:] > 0).all()


def test_zero_viscosity_is_the_euler_rhs():
    rng = np.random.default_rng(4)
    prob = _grid((9, 8, 7), ("periodic",) * 6, mu=0.0, zeta=0.0)
    shape = prob.shape
    U = _state(torch.from_numpy(1.0 + 0.2 * rng.random(shape)), torch.from_numpy(0.3 * rng.random((3,) + shape)),
               torch.from_numpy(1.0 + 0.1 * rng.random(shape)))
    S0 = torch.zeros(shape, dtype=torch.float64)
    L, _ = ref.rhs(prob, U, S0)
    Upad = ref.pad_state(prob, U)
    L0 = ref.flux_divergence(prob, Upad, ref.pad_sigma(prob, ref.sigma_solve(prob, U, S0, Upad=Upad)[0], ref.G))
    assert torch.equal(L, L0)
