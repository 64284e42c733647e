"""The precision forms on the 512^3 multi-jet box over 200 steps, the
configuration the FP64-vs-FP32-vs-BF16-storage comparison is defined on
(4 x 4 Mach-3 discs, 10 sweeps, alpha = 4 dx^2, two-sweep Sigma passes).

Every form runs 200 igr_advance steps of one fixed dt (0.8 x the CFL step
of the initial state) from the same initial state; the FP64 run (parity-
tested against the oracle on full-size windows) is the reference.  Per
field (rho, m_x, m_y, m_z, E, Sigma and the derived pressure) the relative
L1 error sum|form - f64| / sum|f64| must meet the stated bounds: 1e-5 for
FP32 storage, 3e-3 for the split form (FP32 state, BF16 stage differences
and BF16 Sigma).  Whole-state FP16 and BF16 storage are reported, not
bounded (they miss 3e-3 here).  With the viscous terms the FP32 and
split forms are held to the same bounds against the viscous FP64 run."""

import pytest
import torch

from paper_2505_07392_amd import igr, inputs
from gpu_common import banner

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

N, STEPS = 512, 200
BOUND = {"f32": 1e-5, "bf16d": 3e-3}
FIELDS = ("rho", "mx", "my", "mz", "E", "Sigma", "p")


def _workload():
    w = inputs.multi_jet(n=N, jets_per_side=4, radius_cells=10.0, mach=3.0, seed=0, nsweeps=10,
                         build_state=False)
    w.alpha = 4.0 * w.dx * w.dx
    return w


def _fields(s, U, S, gamma):
    """rho, m, E, Sigma and p of the interior as FP64 device tensors."""
    u = s.interior(U).to(torch.float64)
    sg = s.interior(S).to(torch.float64)
    p = (gamma - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0])
    return [u[0], u[1], u[2], u[3], u[4], sg, p]


def _run(w, precision, dt, steps=STEPS):
    s = igr.Solver.from_workload(w, precision=precision, sigma_block=2)
    U = s.new_state()
    inputs.fill_multi_jet_state(w, s.interior(U))
    S = s.new_field()
    if dt is None:
        dt = 0.8 * s.compute_dt(U, w.cfl)
    banner(f"{precision} (mu {w.mu:g}): {steps} steps of dt = {dt:.6e} on the {N}^3 multi-jet box")
    s.advance(U, S, steps, dt_fixed=dt)
    return s, U, S, dt


@pytest.fixture(scope="module")
def reference():
    w = _workload()
    s, U, S, dt = _run(w, "f64", None)
    ref = _fields(s, U, S, w.gamma)
    del U, S
    s.close()
    return w, dt, ref


@pytest.mark.parametrize("precision", ["f32", "bf16d", "f16", "bf16"])
def test_forms_against_f64_after_200_steps(reference, precision):
    w, dt, ref = reference
    s, U, S, _ = _run(w, precision, dt)
    got = _fields(s, U, S, w.gamma)
    err = {}
    for name, g, r in zip(FIELDS, got, ref):
        err[name] = float((g - r).abs().sum() / r.abs().sum())
    del got, U, S
    s.close()
    torch.cuda.empty_cache()
    print(f"[gpu-case] {precision} rel L1 after {STEPS} steps: "
          + ", ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    if precision in BOUND:
        assert max(err.values()) <= BOUND[precision], err
    else:
        # reported only; the values must still be finite
        assert all(v == v for v in err.values()), err


# the viscous terms (eqs. (2)-(3), (5)): the FP32 and split forms against
# the FP64 run (parity-tested against the oracle with the viscous terms on
# 1024^3 windows) over 100 fixed-dt steps, at their bounds
VISC_MU, VISC_ZETA, VISC_STEPS = 1e-4, 5e-5, 100


@pytest.fixture(scope="module")
def viscous_reference():
    w = _workload()
    w.mu, w.zeta = VISC_MU, VISC_ZETA
    s, U, S, dt = _run(w, "f64", None, VISC_STEPS)
    ref = _fields(s, U, S, w.gamma)
    del U, S
    s.close()
    return w, dt, ref


@pytest.mark.parametrize("precision", ["f32", "bf16d"])
def test_viscous_forms_against_f64(viscous_reference, precision):
    w, dt, ref = viscous_reference
    s, U, S, _ = _run(w, precision, dt, VISC_STEPS)
    got = _fields(s, U, S, w.gamma)
    err = {name: float((g - r).abs().sum() / r.abs().sum()) for name, g, r in zip(FIELDS, got, ref)}
    del got, U, S
    s.close()
    torch.cuda.empty_cache()
    print(f"[gpu-case] viscous {precision} rel L1 after {VISC_STEPS} steps: "
          + ", ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    assert all(v <= BOUND[precision] for v in err.values()), err
