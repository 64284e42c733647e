"""Pins of the oracle's third-order reconstruction (the paper's other order,
"Discretization"), CPU only.

A third-order finite-volume interpolant from three cell averages is exact
for cell averages of every polynomial of degree <= 2 and not for degree 3;
it is the 1/3, 2/3 combination of the two second-order candidate stencils
(the optimal linear weights of WENO3); left and right states are mirror
images; the whole scheme converges at third order on a smooth entropy wave.
"""

import math

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref
from paper_2505_07392_amd import inputs
from helpers import problem_from, state_of


def _line_problem(n):
    return ref.Problem(n, 1, 1, 1.0, 1.0, 1.0, faces=(ref.PERIODIC,) * 6, order=3)


def _cell_averages(k, lo, n):
    i = np.arange(lo, lo + n, dtype=np.float64)
    return ((i + 1) ** (k + 1) - i ** (k + 1)) / (k + 1)


def _line(v):
    return torch.from_numpy(v).reshape(1, 1, -1).expand(7, 7, -1).contiguous()


@pytest.mark.parametrize("k", [0, 1, 2])
def test_third_order_exact_for_degree_le_2(k):
    n = 10
    left, right = ref.reconstruct(_line_problem(n), _line(_cell_averages(k, -3, n + 6)), 0)
    exact = np.arange(0, n + 1, dtype=np.float64) ** k
    scale = max(1.0, np.abs(exact).max())
    assert np.abs(left[0, 0].numpy() - exact).max() <= 1e-12 * scale
    assert np.abs(right[0, 0].numpy() - exact).max() <= 1e-12 * scale


def test_third_order_not_exact_for_degree_3():
    n = 10
    left, right = ref.reconstruct(_line_problem(n), _line(_cell_averages(3, -3, n + 6)), 0)
    exact = np.arange(0, n + 1) ** 3.0
    assert np.abs(left[0, 0].numpy() - exact).max() > 1e-2
    assert np.abs(right[0, 0].numpy() - exact).max() > 1e-2


def test_third_order_weights_are_the_linear_weno3_combination():
    s0 = np.array([-1, 3, 0]) / 2.0    # cells i-1, i   (upwind second-order)
    s1 = np.array([0, 1, 1]) / 2.0     # cells i, i+1   (centred second-order)
    comb = s0 / 3.0 + 2.0 * s1 / 3.0
    assert np.allclose(comb, np.array(ref.RECON3_LEFT) / ref.RECON3_DENOM, atol=1e-15)
    assert np.allclose(comb[::-1], np.array(ref.RECON3_RIGHT) / ref.RECON3_DENOM, atol=1e-15)


def test_third_order_mirror_symmetry():
    n = 12
    v = np.random.default_rng(4).standard_normal(n + 6)
    left, right = ref.reconstruct(_line_problem(n), _line(v), 0)
    left_m, right_m = ref.reconstruct(_line_problem(n), _line(v[::-1].copy()), 0)
    assert torch.allclose(left[0, 0], right_m[0, 0].flip(0), rtol=0, atol=1e-14)
    assert torch.allclose(right[0, 0], left_m[0, 0].flip(0), rtol=0, atol=1e-14)


def test_entropy_wave_third_order():
    T = 0.05
    errs = []
    for n in (16, 32, 64):
        w = inputs.entropy_wave(n, amp=0.2)
        prob = problem_from(w)
        prob.order = 3
        U = state_of(w)
        sig = torch.zeros(prob.shape, dtype=torch.float64)
        nst = int(math.ceil(T / (0.25 / n)))
        for _ in range(nst):
            U, sig = ref.rk3_step(prob, U, sig, T / nst)
        xc = (np.arange(n) + 0.5) / n
        k, h = 2 * math.pi, 1.0 / n
        exact = 1 + 0.2 * np.sin(k * (xc - T)) * (math.sin(k * h / 2) / (k * h / 2))
        errs.append(np.abs(U[0, 0, 0].numpy() - exact).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 2.7, orders
    assert max(orders) < 3.5, orders
