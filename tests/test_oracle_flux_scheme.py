"""Pins of the oracle's flux, divergence and time stepping.

* Flux consistency: the LLF flux of two equal states is the physical flux
  of eqs. (6)-(8) (tau = 0), written out here by hand.
* A uniform state has L(U) = 0 exactly (every face computes the same flux).
* Axis permutation and mirror symmetry of the whole right-hand side
  (Sigma solve included).
* alpha = 0: Sigma vanishes and the scheme equals an independent per-cell
  fifth-order LLF code (tests/plain_llf.py).
* SSP-RK3 applied to L(U) = -kappa U gives the stability polynomial
  1 + z + z^2/2 + z^3/6, z = -kappa dt.
* dt against a per-cell loop.
"""

import math

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref
from paper_2505_07392_amd import inputs
from helpers import problem_from
import plain_llf


def _hand_flux(U, S, d, gamma):
    rho, mx, my, mz, E = U
    m = (mx, my, mz)
    p = (gamma - 1) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho)
    un = m[d] / rho
    F = [m[d], mx * un, my * un, mz * un, (E + p + S) * un]
    F[1 + d] = F[1 + d] + p + S
    return F


@pytest.mark.parametrize("d", [0, 1, 2])
def test_flux_consistency(d):
    rng = np.random.default_rng(d)
    prob = ref.Problem(4, 4, 4, 1, 1, 1)
    U = torch.from_numpy(inputs.random_state(4, 4, 4, seed=d))
    S = torch.from_numpy(rng.standard_normal((4, 4, 4)))
    F = ref.llf_flux(prob, U, U, S, S, d)
    expect = torch.stack(_hand_flux(U, S, d, prob.gamma))
    assert torch.allclose(F, expect, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("faces", [(ref.PERIODIC,) * 6, (ref.EXTRAP,) * 6])
def test_uniform_state_is_stationary(faces):
    prob = ref.Problem(7, 6, 5, 0.1, 0.2, 0.3, alpha=0.01, faces=faces)
    U = torch.tensor([0.9, 0.3, -0.4, 0.2, 3.1], dtype=torch.float64).reshape(5, 1, 1, 1)
    U = U.expand(5, 5, 6, 7).contiguous()
    sig0 = torch.full(prob.shape, 0.37, dtype=torch.float64)
    L, sig = ref.rhs(prob, U, sig0)
    assert torch.count_nonzero(L) == 0


def _swap_xy(U):
    V = U.transpose(-1, -2)
    return torch.stack([V[0], V[2], V[1], V[3], V[4]]).contiguous()


def test_axis_permutation_symmetry():
    nx, ny, nz = 9, 7, 6
    w = inputs.Workload("t", nx, ny, nz, 0.11, 0.13, 0.17, inputs.random_state(nx, ny, nz, 7),
                        alpha=0.02, faces=(ref.EXTRAP, ref.EXTRAP, ref.PERIODIC, ref.PERIODIC,
                                           ref.EXTRAP, ref.EXTRAP), nsweeps=3)
    prob = problem_from(w)
    U = torch.from_numpy(w.U)
    sig0 = torch.from_numpy(np.random.default_rng(1).random(prob.shape))
    L, sig = ref.rhs(prob, U, sig0)
    prob_t = ref.Problem(ny, nx, nz, 0.13, 0.11, 0.17, alpha=0.02,
                         faces=(ref.PERIODIC, ref.PERIODIC, ref.EXTRAP, ref.EXTRAP, ref.EXTRAP, ref.EXTRAP),
                         nsweeps=3)
    L_t, sig_t = ref.rhs(prob_t, _swap_xy(U), sig0.transpose(-1, -2).contiguous())
    assert torch.allclose(sig_t, sig.transpose(-1, -2), rtol=0, atol=1e-12 * float(sig.abs().max()))
    scale = L.abs().amax(dim=(1, 2, 3), keepdim=True)
    assert ((_swap_xy(L) - L_t).abs() <= 1e-12 * scale).all()


def test_mirror_symmetry_x():
    nx, ny, nz = 10, 5, 4
    U = torch.from_numpy(inputs.random_state(nx, ny, nz, 11))
    prob = ref.Problem(nx, ny, nz, 0.1, 0.1, 0.1, alpha=0.01, nsweeps=4)
    sig0 = torch.from_numpy(np.random.default_rng(2).random(prob.shape))
    L, sig = ref.rhs(prob, U, sig0)
    flip = lambda V: torch.stack([V[0], -V[1], V[2], V[3], V[4]]).flip(-1)
    L_m, sig_m = ref.rhs(prob, flip(U), sig0.flip(-1))
    assert torch.allclose(sig_m, sig.flip(-1), rtol=0, atol=1e-13)
    scale = L.abs().amax(dim=(1, 2, 3), keepdim=True)
    assert ((flip(L) - L_m).abs() <= 1e-12 * scale).all()


def test_alpha_zero_matches_independent_plain_llf():
    n = 16
    w = inputs.entropy_wave(n, amp=0.2, u=(0.7, 0.3, -0.2))
    x = (np.arange(n) + 0.5) / n
    # add a pressure and velocity wave so every flux component is exercised
    rho = w.U[0, 0, 0]
    ux = 0.7 + 0.1 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.1 * np.sin(4 * np.pi * x)
    U = inputs.conserved(rho[None, None, :], ux[None, None, :], 0.3, -0.2, p[None, None, :])
    prob = ref.Problem(n, 1, 1, 1.0 / n, 1.0 / n, 1.0 / n, alpha=0.0, faces=(ref.PERIODIC,) * 6)
    Ut = torch.from_numpy(U)
    sig = torch.zeros(prob.shape, dtype=torch.float64)
    cells = [list(U[:, 0, 0, i]) for i in range(n)]
    dt = 0.2 / n
    for _ in range(3):
        Ut, sig = ref.rk3_step(prob, Ut, sig, dt)
        cells = plain_llf.rk3_1d(cells, 1.0 / n, dt, prob.gamma)
    assert torch.count_nonzero(sig) == 0
    ref_cells = torch.tensor(cells, dtype=torch.float64).T.reshape(5, 1, 1, n)
    assert torch.allclose(Ut, ref_cells, rtol=0, atol=1e-13)


def test_rk3_stability_polynomial():
    prob = ref.Problem(3, 3, 3, 1, 1, 1)
    kappa, dt = 1.7, 0.37
    U = torch.from_numpy(np.random.default_rng(0).random((5, 3, 3, 3)))
    sig = torch.zeros((3, 3, 3), dtype=torch.float64)
    lin = lambda prob, V, s: (-kappa * V, s)
    out, _ = ref.rk3_step(prob, U, sig, dt, rhs_fn=lin)
    z = -kappa * dt
    assert torch.allclose(out, U * (1 + z + z * z / 2 + z ** 3 / 6), rtol=1e-15, atol=0)


def test_dt_matches_cell_loop():
    nx, ny, nz = 5, 4, 3
    U = inputs.random_state(nx, ny, nz, 5)
    h = (0.1, 0.2, 0.3)
    prob = ref.Problem(nx, ny, nz, *h)
    smax = 0.0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                rho, mx, my, mz, E = U[:, k, j, i]
                p = 0.4 * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho)
                c = math.sqrt(1.4 * p / rho)
                s = sum((abs(m / rho) + c) / hd for m, hd in zip((mx, my, mz), h))
                smax = max(smax, s)
    assert abs(ref.compute_dt(prob, torch.from_numpy(U), 0.5) - 0.5 / smax) <= 1e-15 * 0.5 / smax
