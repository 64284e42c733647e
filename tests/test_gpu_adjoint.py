"""GPU checks of the hand-written adjoint (FP64).

* igr_rhs_adjoint and igr_step_adjoint against the oracle's discrete
  adjoint (torch.autograd through oracle/igr_ref.py) on the same inputs,
  with fifth- and third-order reconstruction, without and with the viscous
  terms: cotangents of U, of the warm-start Sigma and of the jet pressures.
* Transposition: <J v, w> computed by central differences of the GPU
  forward equals <v, J^T w> from the adjoint, without and with the viscous
  terms.
* The 128^3 gradient workload (2 x 2 Mach-2 jets, 40 fixed-dt steps,
  checkpoints every 10 steps, loss = time-integrated thermodynamic pressure
  force on the plane x = 0.75 L): dJ/dp_jet and a random-direction dJ/drho0
  against central finite differences (h = 1e-6), <= 1e-6 relative; the
  same at x = 4 dx with the viscous terms.
"""

import math

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref
from paper_2505_07392_amd import igr, inputs
from paper_2505_07392_amd.autograd import run_checkpointed
from helpers import problem_from
from gpu_common import banner, to_host

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

ADJ_TOL = 1e-10


def _case(nx=20, ny=9, nz=7, jets=True, faces=None, seed=0):
    U = inputs.random_state(nx, ny, nz, seed, amp=0.2, umax=0.3)
    dx = 1.0 / max(nx, ny, nz)
    js = []
    if jets:
        js = [inputs.Jet(yc=0.3 * ny * dx, zc=0.45 * nz * dx, r=2.5 * dx, rho=0.6, ux=2.0, uy=0.1, uz=-0.1,
                         p=2.0, width=1.2 * dx)]
    faces = faces or ("extrap", "extrap", "periodic", "periodic", "extrap", "extrap")
    return inputs.Workload("adj", nx, ny, nz, dx, 1.1 * dx, 0.9 * dx, U, alpha=0.7 * dx * dx, faces=faces,
                           jets=js, nsweeps=3)


def _rel(got, want):
    got, want = np.asarray(got), np.asarray(want)
    scale = np.abs(want).max()
    return float(np.abs(got - want).max() / scale) if scale > 0 else float(np.abs(got).max())


def _oracle_problem(w, p_tensor=None, order=5):
    prob = problem_from(w, order=order)
    if p_tensor is not None:
        for i, pa in enumerate(prob.patches):
            pa.p = p_tensor[i]
    return prob


CASES = {
    "mixed_jet": lambda: _case(),
    "periodic": lambda: _case(12, 10, 9, jets=False, faces=("periodic",) * 6, seed=1),
    "extrap_thin": lambda: _case(17, 1, 5, jets=False, faces=("extrap", "extrap", "periodic", "periodic",
                                                               "extrap", "extrap"), seed=2),
}


# shear and bulk viscosity of the viscous cases (eq. (5))
VISC = (2e-3, 1e-3)


def _with_viscosity(w, visc):
    if visc:
        w = w.with_state(w.U)
        w.mu, w.zeta = VISC
    return w


@pytest.mark.parametrize("visc", [False, True])
@pytest.mark.parametrize("order", [5, 3])
@pytest.mark.parametrize("name", sorted(CASES))
def test_rhs_adjoint_matches_oracle_autograd(name, order, visc):
    w = _with_viscosity(CASES[name](), visc)
    banner(f"rhs adjoint {name} order {order} viscous {visc}")
    rng = np.random.default_rng(5)
    sig0 = rng.random((w.nz, w.ny, w.nx)) * 0.1
    Lbar = rng.standard_normal((5, w.nz, w.ny, w.nx))
    Sbar = rng.standard_normal((w.nz, w.ny, w.nx))
    s = igr.Solver.from_workload(w, order=order)
    Ub, Sb, pb = s.rhs_adjoint(s.state_from(w.U), s.field_from(sig0), s.state_from(Lbar), s.field_from(Sbar))
    # oracle autograd
    U = torch.from_numpy(w.U.copy()).requires_grad_(True)
    S0 = torch.from_numpy(sig0).requires_grad_(True)
    p = torch.tensor([j.p for j in w.jets], dtype=torch.float64, requires_grad=True)
    prob = _oracle_problem(w, p if w.jets else None, order)
    L, Sn = ref.rhs(prob, U, S0)
    inputs_ = [U, S0] + ([p] if w.jets else [])
    grads = torch.autograd.grad((L, Sn), inputs_, (torch.from_numpy(Lbar), torch.from_numpy(Sbar)),
                                allow_unused=True)
    for f in range(5):
        assert _rel(to_host(s, Ub)[f], grads[0][f].numpy()) <= ADJ_TOL, f
    assert _rel(to_host(s, Sb), grads[1].numpy()) <= ADJ_TOL
    if w.jets:
        assert abs(pb[0, 4].item() - grads[2][0].item()) <= ADJ_TOL * abs(grads[2][0].item())
    if visc:
        # the viscous terms move the gradient far beyond the tolerance
        w0 = w.with_state(w.U)
        w0.mu, w0.zeta = 0.0, 0.0
        U0 = torch.from_numpy(w.U.copy()).requires_grad_(True)
        L0, S0n = ref.rhs(_oracle_problem(w0, None, order), U0, torch.from_numpy(sig0))
        g0 = torch.autograd.grad((L0, S0n), (U0,), (torch.from_numpy(Lbar), torch.from_numpy(Sbar)))[0]
        assert _rel(g0.numpy(), grads[0].numpy()) > 1e3 * ADJ_TOL


@pytest.mark.parametrize("visc", [False, True])
@pytest.mark.parametrize("order", [5, 3])
def test_step_adjoint_matches_oracle_autograd(order, visc):
    w = _with_viscosity(_case(16, 8, 6, seed=3), visc)
    banner(f"step adjoint vs oracle autograd, order {order}, viscous {visc}")
    rng = np.random.default_rng(6)
    sig0 = rng.random((w.nz, w.ny, w.nx)) * 0.1
    Ubar = rng.standard_normal((5, w.nz, w.ny, w.nx))
    Sbar = rng.standard_normal((w.nz, w.ny, w.nx))
    dt = 0.3 * ref.compute_dt(problem_from(w), torch.from_numpy(w.U), 0.5)
    s = igr.Solver.from_workload(w, order=order)
    Ub, Sb, pb = s.step_adjoint(s.state_from(w.U), s.field_from(sig0), dt, s.state_from(Ubar), s.field_from(Sbar))
    U = torch.from_numpy(w.U.copy()).requires_grad_(True)
    S0 = torch.from_numpy(sig0).requires_grad_(True)
    p = torch.tensor([j.p for j in w.jets], dtype=torch.float64, requires_grad=True)
    U1, S1 = ref.rk3_step(_oracle_problem(w, p, order), U, S0, dt)
    gU, gS, gp = torch.autograd.grad((U1, S1), (U, S0, p), (torch.from_numpy(Ubar), torch.from_numpy(Sbar)))
    for f in range(5):
        assert _rel(to_host(s, Ub)[f], gU[f].numpy()) <= ADJ_TOL, f
    assert _rel(to_host(s, Sb), gS.numpy()) <= ADJ_TOL
    assert abs(pb[0, 4].item() - gp[0].item()) <= ADJ_TOL * abs(gp[0].item())


@pytest.mark.parametrize("visc", [False, True])
def test_step_adjoint_transposition_fd(visc):
    """<(F(U + h v) - F(U - h v)) / 2h, w> = <v, J^T w> on the GPU alone."""
    w = _with_viscosity(_case(24, 10, 8, seed=4), visc)
    banner(f"step adjoint transposition (viscous {visc})")
    rng = np.random.default_rng(8)
    dt = 0.3 * ref.compute_dt(problem_from(w), torch.from_numpy(w.U), 0.5)
    v = rng.standard_normal(w.U.shape) * np.abs(w.U).max(axis=(1, 2, 3), keepdims=True) * 1e-2
    wU = rng.standard_normal(w.U.shape)
    wS = rng.standard_normal((w.nz, w.ny, w.nx))
    s = igr.Solver.from_workload(w)

    def F(U0):
        U = s.state_from(U0)
        S = s.new_field()
        s.step(U, S, dt_fixed=dt)
        return to_host(s, U), to_host(s, S)

    h = 1e-5
    Up, Sp = F(w.U + h * v)
    Um, Sm = F(w.U - h * v)
    lhs = (np.sum((Up - Um) * wU) + np.sum((Sp - Sm) * wS)) / (2 * h)
    Ub, _, _ = s.step_adjoint(s.state_from(w.U), s.new_field(), dt, s.state_from(wU), s.field_from(wS))
    rhs = float(np.sum(to_host(s, Ub) * v))
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs)


def _plane_loss(s, w, dt, i0):
    """Per-step loss term on the padded state: dt * sum_{j,k} (p_{i0-1} + p_{i0})/2 dy dz."""
    G = igr.G

    def loss(U):
        sl = U[:, G:-G, G:-G, G + i0 - 1:G + i0 + 1]
        rho, m, E = sl[0], sl[1:4], sl[4]
        p = (w.gamma - 1.0) * (E - 0.5 * (m * m).sum(0) / rho)
        return dt * (0.5 * (p[..., 0] + p[..., 1])).sum() * (w.dy * w.dz)

    return loss


# viscosity of the viscous gradient case: cell Reynolds number about 40 in
# the jets, viscous diffusion number about 5e-3 at the workload's fixed dt
GRAD_VISC = (1e-3, 5e-4)


def _gradient_run(w, plane):
    """Adjoint gradients (dJ/dp_jet, dJ/dU0) and J of the 128^3 workload."""
    s = igr.Solver.from_workload(w)
    dt = w.dt_fixed
    i0 = int(0.75 * w.nx) if plane == "x=0.75L" else 4
    loss_fn = _plane_loss(s, w, dt, i0)
    U0 = s.state_from(w.U).requires_grad_(True)
    S0 = s.new_field()
    p = torch.tensor([j.p for j in w.jets], dtype=torch.float64, requires_grad=True)
    J, _, _ = run_checkpointed(s, U0, S0, p, dt, w.nsteps, loss_fn, every=10)
    J.backward()
    return s, loss_fn, float(J), p.grad.clone(), U0.grad.detach().clone()


@pytest.mark.parametrize("plane", ["x=0.75L", "x=4dx", "x=4dx viscous"])
def test_gradient_workload_128_against_finite_differences(plane):
    """At x = 0.75 L (the specified plane) no signal from the inlet arrives
    within 40 steps (at most ~0.3 cells per step), and with u = 0 there a
    density perturbation leaves p unchanged, so dJ/dp_jet and dJ/drho0 are
    zero in exact arithmetic: the finite differences give exactly 0 and the
    adjoint gives round-off.  The plane at 4 cells lies in the jets' initial
    plug, where the derivatives are far above the h = 1e-6 noise floor
    (about 1e-16 J / h), and adjoint and central differences must agree to
    1e-6 relative.  The viscous case runs the same workload with the
    viscous terms of eq. (5), which must move dJ/dp_jet by far more than
    that tolerance."""
    w = inputs.gradient_jets(128)
    visc = plane.endswith("viscous")
    plane = plane.split()[0]
    if visc:
        w0 = w
        w = w.with_state(w.U)
        w.mu, w.zeta = GRAD_VISC
    banner(f"gradient workload 128^3: 40 steps, checkpoints every 10, FD h=1e-6, plane {plane}, viscous {visc}")
    s, loss_fn, Jv, gp, gU = _gradient_run(w, plane)
    dt = w.dt_fixed
    if visc:
        gp0 = _gradient_run(w0, plane)[3]
        moved = float((gp - gp0).abs().max() / gp.abs().max())
        print(f"[gpu-case] viscous terms move dJ/dp_jet by {moved:.3e} (relative)", flush=True)
        assert moved > 1e-4

    def J_of(pv, Uv):
        with torch.no_grad():
            for i, j in enumerate(w.jets):
                s.set_jet_state(i, j.rho, j.ux, j.uy, j.uz, float(pv[i]))
            U = s.state_from(Uv)
            S = s.new_field()
            total = 0.0
            for _ in range(w.nsteps):
                s.step(U, S, dt_fixed=dt, sync=False)
                total += float(loss_fn(U))
            s.check()
            return total

    h = 1e-6
    base = np.array([j.p for j in w.jets])
    for i in range(len(w.jets)):
        e = np.zeros_like(base)
        e[i] = h
        fd = (J_of(base + e, w.U) - J_of(base - e, w.U)) / (2 * h)
        print(f"[gpu-case] {plane} dJ/dp_{i}: adjoint {gp[i].item():.12e} fd {fd:.12e}", flush=True)
        if plane == "x=0.75L":
            assert fd == 0.0 and abs(gp[i].item()) <= 1e-30
        else:
            assert abs(gp[i].item() - fd) <= 1e-6 * abs(fd)
    # a direction in the initial density (m and E unchanged): a random
    # positive field on the first 8 planes, where the jets' plug moves, so
    # that the derivative is a coherent sum far above the FD noise floor
    rng = np.random.default_rng(9)
    v = np.zeros_like(w.U)
    v[0, :, :, :8] = rng.random(w.U.shape[1:3] + (8,))
    fd = (J_of(base, w.U + h * v) - J_of(base, w.U - h * v)) / (2 * h)
    ad = float((Solver_interior(gU) * torch.from_numpy(v).to(gU.device)).sum())
    print(f"[gpu-case] {plane} dJ/drho0 . v: adjoint {ad:.12e} fd {fd:.12e} (J = {Jv:.6e})", flush=True)
    if plane == "x=0.75L":
        assert fd == 0.0 and abs(ad) <= 1e-12 * Jv
    else:
        assert abs(ad - fd) <= 1e-6 * abs(fd)


def Solver_interior(a):
    return igr.Solver.interior(a)


def test_adjoint_rejects_red_black():
    w = _case(ny=10)
    s = igr.Solver.from_workload(w, smoother="rbgs")
    U = s.state_from(w.U)
    sig = s.new_field()
    with pytest.raises(igr.IGRError) as e:
        s.rhs_adjoint(U, sig, torch.zeros_like(U), torch.zeros_like(sig))
    assert e.value.code == igr.IGR_EUNSUPPORTED
