"""Precision forms (FP32 state and arithmetic; FP16 or BF16 storage with
FP32 arithmetic; the split form: FP32 state, BF16 stage differences and
BF16 Sigma; FP64 dt and sums in all) against the FP64 oracle.

Per-field relative L1 error, sum |g - o| / sum |o|, after a run with a
fixed time step (the same dt for every form).  Bounds: 1e-5 for FP32 and
3e-3 for 16-bit storage.  FP16 storage (11 significand bits, the paper's
storage format) and the split form (every stage state a BF16 difference
from the FP32 state, Sigma in BF16) meet 3e-3.  Storing whole stage states
in BF16 (8 significand bits) does not: rounding every stored RK stage value
to 2^-9 relative accumulates to 1-5 % in 20-30 steps on these workloads
(the same numbers come out of a CPU emulation that rounds the oracle's
stage values), so that form has a test of its own that guards the known
miss at its measured level (<= 6e-2), not the 3e-3 bound.  Identically-zero
oracle fields are skipped.
"""

import numpy as np
import pytest
import torch

from oracle import igr_ref as ref
from paper_2505_07392_amd import igr, inputs
from helpers import problem_from
from gpu_common import banner, to_host

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

BOUND = {"f32": 1e-5, "f16": 3e-3, "bf16d": 3e-3}
# whole-state BF16 storage misses 3e-3; this guards its measured level only
BF16_KNOWN_MISS = 6e-2


def rel_l1(got, want):
    out = []
    for g, o in zip(got, want):
        den = np.abs(o).sum()
        out.append(np.abs(g - o).sum() / den if den > 0 else 0.0)
    return np.array(out)


def _run_gpu(w, precision, dt, nsteps, sigma_block=0):
    s = igr.Solver.from_workload(w, precision=precision, sigma_block=sigma_block)
    U = s.state_from(w.U)
    S = s.new_field()
    for _ in range(nsteps):
        s.step(U, S, dt_fixed=dt, sync=False)
    s.check()
    return to_host(s, U), to_host(s, S)


def _run_oracle(w, dt, nsteps):
    prob = problem_from(w)
    U = torch.from_numpy(w.U.copy())
    S = torch.zeros(prob.shape, dtype=torch.float64)
    for _ in range(nsteps):
        U, S = ref.rk3_step(prob, U, S, dt)
    return U.numpy(), S.numpy()


@pytest.fixture(scope="module")
def box_reference():
    w = inputs.periodic_box(n=48, seed=2)
    dt = 0.8 * ref.compute_dt(problem_from(w), torch.from_numpy(w.U), 0.5)
    return w, dt, _run_oracle(w, dt, 20)


@pytest.mark.parametrize("sigma_block", [1, 2])
@pytest.mark.parametrize("precision", ["f32", "f16", "bf16d"])
def test_precision_periodic_box(box_reference, precision, sigma_block):
    w, dt, (Uo, So) = box_reference
    banner(f"precision {precision}: periodic box 48^3, 20 steps, sigma_block={sigma_block}")
    Ug, Sg = _run_gpu(w, precision, dt, 20, sigma_block)
    err = rel_l1(np.concatenate([Ug, Sg[None]]), np.concatenate([Uo, So[None]]))
    print(f"[gpu-case] {precision} rel L1 (rho, mx, my, mz, E, Sigma) = {err}", flush=True)
    assert (err <= BOUND[precision]).all(), err


@pytest.mark.parametrize("sigma_block", [1, 2])
def test_whole_state_bf16_known_miss_periodic_box(box_reference, sigma_block):
    """Whole-state BF16 storage misses the 3e-3 bound (see the module
    docstring); this only guards against it getting worse."""
    w, dt, (Uo, So) = box_reference
    banner(f"whole-state bf16 (known miss): periodic box 48^3, 20 steps, sigma_block={sigma_block}")
    Ug, Sg = _run_gpu(w, "bf16", dt, 20, sigma_block)
    err = rel_l1(np.concatenate([Ug, Sg[None]]), np.concatenate([Uo, So[None]]))
    print(f"[gpu-case] bf16 rel L1 (rho, mx, my, mz, E, Sigma) = {err}", flush=True)
    assert (err <= BF16_KNOWN_MISS).all(), err


@pytest.fixture(scope="module")
def jet_reference():
    w = inputs.multi_jet(n=40, jets_per_side=2, radius_cells=6.0, mach=3.0, nsweeps=10)
    w.alpha = 4.0 * w.dx * w.dx
    dt = 0.8 * ref.compute_dt(problem_from(w), torch.from_numpy(w.U), 0.5)
    return w, dt, _run_oracle(w, dt, 30)


@pytest.mark.parametrize("sigma_block", [1, 2])
@pytest.mark.parametrize("precision", ["f32", "f16", "bf16d"])
def test_precision_jets(jet_reference, precision, sigma_block):
    w, dt, (Uo, So) = jet_reference
    banner(f"precision {precision}: Mach-3 jets 40^3, 30 steps, sigma_block={sigma_block}")
    Ug, Sg = _run_gpu(w, precision, dt, 30, sigma_block)
    err = rel_l1(np.concatenate([Ug, Sg[None]]), np.concatenate([Uo, So[None]]))
    keep = [i for i in range(6) if np.abs(np.concatenate([Uo, So[None]])[i]).sum() > 0]
    print(f"[gpu-case] {precision} rel L1 (rho, mx, my, mz, E, Sigma) = {err}", flush=True)
    assert (err[keep] <= BOUND[precision]).all(), err


@pytest.mark.parametrize("sigma_block", [1, 2])
def test_whole_state_bf16_known_miss_jets(jet_reference, sigma_block):
    w, dt, (Uo, So) = jet_reference
    banner(f"whole-state bf16 (known miss): Mach-3 jets 40^3, 30 steps, sigma_block={sigma_block}")
    Ug, Sg = _run_gpu(w, "bf16", dt, 30, sigma_block)
    err = rel_l1(np.concatenate([Ug, Sg[None]]), np.concatenate([Uo, So[None]]))
    keep = [i for i in range(6) if np.abs(np.concatenate([Uo, So[None]])[i]).sum() > 0]
    print(f"[gpu-case] bf16 rel L1 (rho, mx, my, mz, E, Sigma) = {err}", flush=True)
    assert (err[keep] <= BF16_KNOWN_MISS).all(), err


def test_fp64_parity_of_reductions_in_all_forms():
    """dt and sums are FP64 reductions in every form: they equal the FP64
    oracle's values on the form's own (rounded) state."""
    w = inputs.periodic_box(n=32, seed=3)
    banner("FP64 reductions in f32/bf16 forms")
    for precision in ("f32", "f16", "bf16", "bf16d"):
        s = igr.Solver.from_workload(w, precision=precision)
        U = s.state_from(w.U)
        Ur = to_host(s, U)                        # the stored (rounded) state, widened exactly
        prob = problem_from(w)
        dt = s.compute_dt(U, 0.5)
        want = ref.compute_dt(prob, torch.from_numpy(Ur), 0.5)
        assert abs(dt - want) <= 1e-14 * want
        sums = np.array(s.sums(U))
        want_s = ref.conserved_sums(prob, torch.from_numpy(Ur)).numpy()
        scale = np.abs(Ur).sum(axis=(1, 2, 3)) * w.dx ** 3
        assert (np.abs(sums - want_s) <= 1e-13 * scale).all()


@pytest.mark.parametrize("precision,n,want", [
    ("f64", 16, 2), ("f64", 256, 2),
    ("f16", 256, 1), ("bf16", 256, 1), ("f16", 384, 2),
    ("f32", 248, 1), ("f32", 256, 2),
    ("bf16d", 275, 1), ("bf16d", 276, 2),
])
def test_default_pass_structure(precision, n, want):
    """sigma_block 0 resolves to two-sweep passes in FP64, and in the forms
    with FP32 arithmetic once one sweep's working set (padded elements x
    (2 x Sigma bytes + rho bytes + 4)) exceeds 256 MiB: 254^3 x 16 B =
    250 MiB stays single, 262^3 x 16 B = 274 MiB pairs; the split form reads
    the FP32 1/rho stored by the first sweep (12 B: 281^3 stays single,
    282^3 pairs).  An explicit choice is kept."""
    banner(f"default pass structure {precision} {n}^3")
    s = igr.Solver(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n, precision=precision)
    assert s.sigma_block == want
    s.close()
    s = igr.Solver(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n, precision=precision, sigma_block=3 - want)
    assert s.sigma_block == 3 - want
    s.close()


# one-step bound per form at full size, relative to each field's maximum:
# the three stage values are rounded to storage once each (FP32: 2^-24,
# FP16: 2^-11, BF16: 2^-8 relative), everything else is FP32 arithmetic
STEP_BOUND = {"f32": 1e-5, "f16": 3e-3, "bf16": 2e-2, "bf16d": 3e-3}


@pytest.mark.parametrize("precision", ["f32", "f16", "bf16", "bf16d"])
def test_full_size_form_step_sampled(precision):
    """The 256^3 periodic box in each form, one igr_advance step with a
    fixed dt (the call and launch configuration the throughput is measured
    with: FP32 runs two-sweep passes there, the 16-bit forms single sweeps),
    against the FP64 oracle's step of the form's stored initial state on a
    periodic window around sampled cells."""
    from gpu_common import window
    w = inputs.periodic_box(n=256, seed=0)
    banner(f"full-size {precision} step 256^3 sampled")
    s = igr.Solver.from_workload(w, precision=precision)
    U = s.state_from(w.U)
    S = s.new_field()
    U0 = to_host(s, U)                          # the stored (rounded) state, widened exactly
    dt = 0.8 * ref.compute_dt(problem_from(w), torch.from_numpy(U0), 0.5)
    s.advance(U, S, 1, dt_fixed=dt)
    s.check()
    Ug = to_host(s, U)
    Sg = to_host(s, S)
    R = 29                                      # three stages of the rhs dependency radius
    n = 2 * R + 1
    prob = ref.Problem(n, n, n, w.dx, w.dy, w.dz, alpha=w.alpha, faces=("periodic",) * 6, nsweeps=w.nsweeps)
    scale = np.abs(Ug).reshape(5, -1).max(axis=1)
    sscale = np.abs(Sg).max()
    rng = np.random.default_rng(5)
    for p in [tuple(rng.integers(0, 256, 3)) for _ in range(2)]:
        Uw, Sw = ref.rk3_step(prob, torch.from_numpy(window(U0, p, R)), torch.zeros((n, n, n), dtype=torch.float64), dt)
        k, j, i = p
        err = np.abs(Ug[:, k, j, i] - Uw[:, R, R, R].numpy()) / scale
        serr = abs(Sg[k, j, i] - float(Sw[R, R, R])) / sscale
        print(f"[gpu-case] {precision} sample {p}: rel err (rho, mx, my, mz, E) = {err}, Sigma {serr:.2e}", flush=True)
        assert (err <= STEP_BOUND[precision]).all(), (p, err)
        assert serr <= STEP_BOUND[precision], (p, serr)


def test_bf16_store_rounds_to_nearest_even():
    """BF16 stores round to nearest even.  Inside a sharp inflow disc
    (chi = 1) the stored ghost is the jet's conserved state converted to
    FP32 and then to BF16, with no other arithmetic in between; jet
    densities at BF16 ties (1 + 2^-8 rounds down to even, 1 + 3 * 2^-8 up
    to even) and just above a tie must give exactly the bits of torch's
    float32 -> bfloat16 conversion (round to nearest even)."""
    banner("bf16 rounding of the jet ghost at ties")
    n = 16
    dx = 1.0 / n
    rhos = [1.0 + 2.0 ** -8, 1.0 + 3.0 * 2.0 ** -8, 1.0 + 3.0 * 2.0 ** -8 + 2.0 ** -16]
    centres = [(0.25, 0.25), (0.75, 0.25), (0.5, 0.75)]
    jets = [inputs.Jet(yc=yc, zc=zc, r=1.5 * dx, rho=r, ux=1.0, uy=-1.0, uz=0.0, p=0.75)
            for (yc, zc), r in zip(centres, rhos)]
    w = inputs.Workload("ties", 8, n, n, dx, dx, dx, inputs.random_state(8, n, n, seed=1), alpha=0.0,
                        jets=jets, nsweeps=0)
    s = igr.Solver.from_workload(w, precision="bf16")
    U = s.state_from(w.U)
    S = s.new_field()
    s.sigma_solve(U, S, nsweeps=0)            # fills the state's ghosts
    torch.cuda.synchronize()
    G = igr.G
    checked = 0
    for q, jt in enumerate(jets):
        cons = torch.tensor([jt.rho, jt.rho * jt.ux, jt.rho * jt.uy, jt.rho * jt.uz,
                             jt.p / (w.gamma - 1.0) + 0.5 * jt.rho * (jt.ux ** 2 + jt.uy ** 2 + jt.uz ** 2)],
                            dtype=torch.float64)
        want = cons.float().bfloat16().view(torch.int16)
        for k in range(n):
            for j in range(n):
                y, z = (j + 0.5) * dx, (k + 0.5) * dx
                if (y - jt.yc) ** 2 + (z - jt.zc) ** 2 > jt.r ** 2:
                    continue
                got = U[:, k + G, j + G, :G].cpu().view(torch.int16)
                for layer in range(G):
                    assert torch.equal(got[:, layer], want), (q, j, k, layer, got[:, layer], want)
                checked += 1
    assert checked >= 3 * 4
    s.close()
