"""GPU parity of the viscous terms (eqs. (2)-(3) with the stress of
eq. (5)) against the FP64 oracle, through the C ABI: right-hand sides and
RK3 steps with shear and bulk viscosity on the mixed small cases (jet discs,
periodic and outflow faces, ragged tiles), third-order reconstruction, the
viscous contribution on its own (L(mu, zeta) - L(0, 0), at 1e-10 of its own
size), conservation on a periodic box, the FP32, 16-bit storage and split forms,
the 256^3 box on sampled windows, and the adjoint's FP64-only rule."""

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref
from paper_2505_07392_amd import igr, inputs
from helpers import problem_from
from gpu_common import TOL, banner, rel_linf, to_host, window
from test_gpu_parity import CASES

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

MU, ZETA = 4e-3, 2e-3


def _viscous(w, mu=MU, zeta=ZETA):
    w = w.with_state(w.U)
    w.mu, w.zeta = mu, zeta
    return w


@pytest.fixture(scope="module", params=sorted(CASES))
def vcase(request):
    return request.param, _viscous(CASES[request.param]())


def _sigma0(w, seed=7):
    return np.random.default_rng(seed).random((w.nz, w.ny, w.nx)) * 0.1


@pytest.mark.parametrize("order", [5, 3])
def test_viscous_rhs(vcase, order):
    name, w = vcase
    banner(f"viscous rhs {name} order {order}")
    s = igr.Solver.from_workload(w, order=order)
    U = s.state_from(w.U)
    sig = s.field_from(_sigma0(w))
    L = to_host(s, s.rhs(U, sig))
    prob = problem_from(w, order=order)
    Lo, so = ref.rhs(prob, torch.from_numpy(w.U), torch.from_numpy(_sigma0(w)))
    assert rel_linf(L, Lo.numpy()).max() <= TOL
    assert rel_linf(to_host(s, sig), so.numpy()).max() <= TOL
    # the viscous contribution alone, against its own size
    s0 = igr.Solver.from_workload(_viscous(w, 0.0, 0.0), order=order)
    L0 = to_host(s0, s0.rhs(s0.state_from(w.U), s0.field_from(_sigma0(w))))
    Lo0, _ = ref.rhs(problem_from(_viscous(w, 0.0, 0.0), order=order), torch.from_numpy(w.U),
                     torch.from_numpy(_sigma0(w)))
    dv, dvo = L - L0, (Lo - Lo0).numpy()
    assert np.abs(dvo[1:]).max() > 0
    err = np.abs(dv - dvo).max() / np.abs(dvo).max()
    print(f"[gpu-case] viscous part {name}: rel err {err:.2e}", flush=True)
    assert err <= 1e-10


# (smoother, sweeps, CFL time step): the case's odd count (the stress from
# its own kernel), an even count (the first two-level Sigma pass forms it;
# with a CFL step in FP64 that pass also forms the CFL maxima), red-black
# passes (the same with one pass per sweep)
STEP_MODES = {"jacobi_case": ("jacobi", None, False), "jacobi_4": ("jacobi", 4, False),
              "jacobi_4_cfl": ("jacobi", 4, True), "rbgs_3": ("rbgs", 3, False)}


@pytest.mark.parametrize("mode", sorted(STEP_MODES))
def test_viscous_steps(vcase, mode):
    name, w = vcase
    smoother, nsweeps, cfl = STEP_MODES[mode]
    ext = (w.nx, w.ny, w.nz)
    if smoother == "rbgs" and any(w.faces[2 * d] == "periodic" and ext[d] % 2 for d in range(3)):
        pytest.skip("red-black sweeps need even periodic extents")
    banner(f"viscous 3 steps {name} {mode}")
    s = igr.Solver.from_workload(w, nsweeps=nsweeps, smoother=smoother)
    U = s.state_from(w.U)
    sig = s.field_from(_sigma0(w))
    prob = problem_from(w, nsweeps=nsweeps)
    prob.smoother = smoother
    Uo, so = torch.from_numpy(w.U.copy()), torch.from_numpy(_sigma0(w))
    dt = 0.5 * ref.compute_dt(prob, Uo, 0.5)
    for _ in range(3):
        if cfl:
            dt = ref.compute_dt(prob, Uo, 0.25)
            dt_g = s.step(U, sig, cfl=0.25)
            assert abs(dt_g - dt) <= 1e-14 * dt
        else:
            s.step(U, sig, dt_fixed=dt)
        Uo, so = ref.rk3_step(prob, Uo, so, dt)
    assert rel_linf(to_host(s, U), Uo.numpy()).max() <= TOL
    assert rel_linf(to_host(s, sig), so.numpy()).max() <= TOL


# degenerate extents: single planes, rows and columns (z chunks of one
# plane, tiles narrower than a wave, halos reaching ghosts on both sides)
DEGENERATE = {
    "5x3x1_extrap": ((5, 3, 1), ("extrap",) * 6),
    "1x7x4_periodic": ((1, 7, 4), ("periodic",) * 6),
    "64x2x1_mixed": ((64, 2, 1), ("extrap", "extrap", "periodic", "periodic", "periodic", "periodic")),
    "3x1x1_periodic": ((3, 1, 1), ("periodic",) * 6),
}


@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_viscous_degenerate_extents(name):
    (nx, ny, nz), faces = DEGENERATE[name]
    U0 = inputs.random_state(nx, ny, nz, 11, amp=0.3, umax=0.4)
    dx = 1.0 / max(nx, ny, nz)
    w = _viscous(inputs.Workload("degenerate", nx, ny, nz, dx, 1.1 * dx, 0.9 * dx, U0, alpha=0.7 * dx * dx,
                                 faces=faces, jets=[], nsweeps=5))
    banner(f"viscous degenerate extents {name}")
    s = igr.Solver.from_workload(w)
    prob = problem_from(w)
    L = to_host(s, s.rhs(s.state_from(w.U), s.field_from(_sigma0(w))))
    Lo, _ = ref.rhs(prob, torch.from_numpy(w.U), torch.from_numpy(_sigma0(w)))
    assert rel_linf(L, Lo.numpy()).max() <= TOL
    # the viscous contribution alone, against its own size
    w0 = _viscous(w, 0.0, 0.0)
    s0 = igr.Solver.from_workload(w0)
    L0 = to_host(s0, s0.rhs(s0.state_from(w.U), s0.field_from(_sigma0(w))))
    Lo0, _ = ref.rhs(problem_from(w0), torch.from_numpy(w.U), torch.from_numpy(_sigma0(w)))
    dv, dvo = L - L0, (Lo - Lo0).numpy()
    assert np.abs(dvo[1:]).max() > 0
    assert np.abs(dv - dvo).max() <= 1e-10 * np.abs(dvo).max()
    # two steps
    U = s.state_from(w.U)
    sig = s.field_from(_sigma0(w))
    Uo, so = torch.from_numpy(w.U.copy()), torch.from_numpy(_sigma0(w))
    dt = 0.5 * ref.compute_dt(prob, Uo, 0.5)
    for _ in range(2):
        s.step(U, sig, dt_fixed=dt)
        Uo, so = ref.rk3_step(prob, Uo, so, dt)
    assert rel_linf(to_host(s, U), Uo.numpy()).max() <= TOL
    assert rel_linf(to_host(s, sig), so.numpy()).max() <= TOL


@pytest.mark.parametrize("nsweeps", [None, 4])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16d"])
def test_viscous_advance_with_cfl_matches_steps(prec, nsweeps):
    """With viscosity igr_advance takes each later time step from the CFL
    maxima that the last stage's viscous kernel forms as it completes the
    new state; igr_step forms them from the state it starts from (FP64: in
    its first Sigma pass, FP32: the standalone reduction).  Both evaluate the
    same FP64 expression on the stored values (one rounding of dt allowed,
    in case the compiler contracts it differently in the two kernels), so
    the states agree to a few units of the arithmetic."""
    w = _viscous(CASES["mixed_70x9x7"]())
    banner(f"viscous advance vs steps ({prec}, sweeps {nsweeps})")
    s = igr.Solver.from_workload(w, precision=prec, nsweeps=nsweeps)
    U1, U2 = s.state_from(w.U), s.state_from(w.U)
    S1, S2 = s.field_from(_sigma0(w)), s.field_from(_sigma0(w))
    dts = [s.step(U1, S1, cfl=0.4) for _ in range(3)]
    dt_last = s.advance(U2, S2, 3, cfl=0.4)
    assert abs(dt_last - dts[-1]) <= 1e-15 * dts[-1]
    a, b = to_host(s, U1).astype(np.float64), to_host(s, U2).astype(np.float64)
    d = rel_linf(b, a).max()
    print(f"[gpu-case] viscous advance vs steps {prec}: max rel diff {d:.3e}", flush=True)
    assert d <= {"f64": 1e-14, "f32": 1e-6, "bf16d": 1e-5}[prec]


def test_viscous_conservation_periodic_box():
    w = _viscous(inputs.periodic_box(n=48, seed=1), 2e-3, 1e-3)
    banner("viscous conservation 48^3")
    s = igr.Solver.from_workload(w)
    U = s.state_from(w.U)
    sig = s.new_field()
    t0 = np.array(s.sums(U))
    for _ in range(10):
        s.step(U, sig, cfl=0.4)
    t1 = np.array(s.sums(U))
    scale = np.abs(w.U).sum(axis=(1, 2, 3)) * w.dx ** 3
    assert (np.abs(t1 - t0) <= 1e-12 * scale).all(), (t1 - t0) / scale


# per-form bounds of the stored-precision forms (as without viscosity):
# whole-state BF16 storage is held at its known-miss level only
FORM_BOUND = {"f32": 1e-5, "f16": 3e-3, "bf16d": 3e-3, "bf16": 6e-2}


@pytest.mark.parametrize("prec", sorted(FORM_BOUND))
def test_viscous_precision_forms(prec):
    """The FP32 form, the 16-bit storage forms and the split form (FP32
    arithmetic; where the stage output is stored in 16 bits -- the whole
    stage state, or the split form's difference from U^n -- the viscous
    kernel reads back what the flux kernel rounded and rounds the sum
    again) against the FP64 oracle after 10 steps."""
    w = _viscous(inputs.periodic_box(n=32, seed=2))
    banner(f"viscous {prec} form 32^3, 10 steps")
    prob = problem_from(w)
    Uo = torch.from_numpy(w.U.copy())
    So = torch.zeros(prob.shape, dtype=torch.float64)
    dt = 0.8 * ref.compute_dt(prob, Uo, 0.5)
    for _ in range(10):
        Uo, So = ref.rk3_step(prob, Uo, So, dt)
    s = igr.Solver.from_workload(w, precision=prec)
    U = s.state_from(w.U)
    S = s.new_field()
    for _ in range(10):
        s.step(U, S, dt_fixed=dt, sync=False)
    s.check()
    g, o = to_host(s, U).astype(np.float64), Uo.numpy()
    err = np.abs(g - o).sum(axis=(1, 2, 3)) / np.abs(o).sum(axis=(1, 2, 3))
    print(f"[gpu-case] viscous {prec} rel L1 {err}", flush=True)
    assert (err <= FORM_BOUND[prec]).all()


def test_viscous_full_size_step_sampled():
    """The 256^3 periodic box with viscosity, one igr_advance step, against
    the oracle's step on periodic windows around sampled cells (the
    viscous stencil reaches 4 cells per stage, inside the 3 + S + 1 of the
    Sigma solve and flux)."""
    w = _viscous(inputs.periodic_box(n=256, seed=0), 1e-3, 5e-4)
    banner("viscous full-size step 256^3 sampled")
    s = igr.Solver.from_workload(w)
    U = s.state_from(w.U)
    S = s.new_field()
    dt = 0.8 * ref.compute_dt(problem_from(w), torch.from_numpy(w.U), 0.5)
    s.advance(U, S, 1, dt_fixed=dt)
    Ug, Sg = to_host(s, U), to_host(s, S)
    R = 29
    n = 2 * R + 1
    prob = ref.Problem(n, n, n, w.dx, w.dy, w.dz, alpha=w.alpha, faces=("periodic",) * 6, nsweeps=w.nsweeps,
                       mu=w.mu, zeta=w.zeta)
    scale = np.abs(Ug).reshape(5, -1).max(axis=1)
    # the samples of the inviscid full-size test: their periodic windows'
    # seams (far from the sample, but stepped by the oracle too) keep a
    # positive pressure for one step
    rng = np.random.default_rng(5)
    for p in [tuple(rng.integers(0, 256, 3)) for _ in range(2)]:
        Uw, Sw = ref.rk3_step(prob, torch.from_numpy(window(w.U, p, R)), torch.zeros((n, n, n), dtype=torch.float64),
                              dt)
        k, j, i = p
        err = np.abs(Ug[:, k, j, i] - Uw[:, R, R, R].numpy()) / scale
        print(f"[gpu-case] viscous sample {p}: {err}", flush=True)
        assert (err <= TOL).all()
        assert abs(Sg[k, j, i] - float(Sw[R, R, R])) <= TOL * np.abs(Sg).max()


def test_viscous_adjoint_runs_in_fp64_only():
    """The adjoint (checked against the oracle's autograd with viscosity in
    tests/test_gpu_adjoint.py) is an FP64 feature: an FP32 viscous context
    reports IGR_EUNSUPPORTED."""
    w = _viscous(CASES["mixed_70x9x7"]())
    banner("viscous adjoint: FP32 rejected")
    s = igr.Solver.from_workload(w, precision="f32")
    U = s.state_from(w.U)
    sig = s.new_field()
    with pytest.raises(igr.IGRError) as e:
        s.rhs_adjoint(U, sig, s.new_state(), s.new_field())
    assert e.value.code == igr.IGR_EUNSUPPORTED
