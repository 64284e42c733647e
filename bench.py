"""Throughput of the IGR hot path on one MI355X.

A step is one SSP-RK3 step of the whole path (three right-hand sides, each
with its ghost fill, Sigma source, Jacobi sweeps and fused reconstruction +
LLF flux + divergence + stage update, plus the FP64 CFL reduction; the
timed steps run through igr_advance with the CFL time step), with the state
resident in HBM.

Default workload: the largest single-GPU multi-jet box, 1024^3 cells, a
4 x 4 array of Mach-3 inflow discs of radius 10 cells on the x-min face
(rho = 0.5, p = 8, +-5 % seeded u_x), ambient (1, 0, 1), outflow elsewhere,
10 Jacobi sweeps per stage, alpha = 4 dx^2 (alpha = dx^2 loses positivity at
the Mach-3 jet edges under the unlimited fifth-order reconstruction).  The
FP64 form is `value`; FP32 and the 16-bit storage forms are timed the same
way under `forms`, each with its rate relative to FP64, the device bytes in
use and its per-field relative L1 error against the FP64 run after the same
number of fixed-dt steps.  The 256^3 periodic box (rms Mach 1.5,
alpha = dx^2, 5 sweeps) is timed under `extra`.

Prints one JSON line: cell-updates/s (cells x steps / time), the roofline
of the dominant kernel measured with HIP events on the solver's stream
during the timed region, and the oracle's rate on a bounded sample of the
same workload on the host cores.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2505_07392_amd", "csrc")


def sigma_schedule(nsweeps: int, sigma_block: int, smoother: str = "jacobi"):
    """Launches of one Sigma solve as the library runs them for the pass
    structure a context reports (Solver.sigma_block, default resolved):
    (passes that form the source, later two-sweep passes, later single
    sweeps).  With two-sweep passes an even count starts with a two-sweep
    pass that forms the source, an odd count with a single sweep.
    Red-black Gauss-Seidel runs one two-level pass per sweep with
    sigma_block 2 (each counted here as a two-sweep pass), else two in-place
    half-sweeps per sweep, each counted as a single sweep."""
    if nsweeps == 0:
        return 0, 0, 0
    if smoother == "rbgs":
        return (1, nsweeps - 1, 0) if sigma_block == 2 else (1, 0, 2 * nsweeps - 1)
    if sigma_block not in (1, 2):
        raise ValueError("the fused-source march passes are not modelled here")
    if sigma_block == 2 and nsweeps % 2 == 0:
        return 1, (nsweeps - 2) // 2, 0
    later = nsweeps - 1
    pairs = later // 2 if sigma_block == 2 else 0
    return 1, pairs, later - 2 * pairs


# bytes per stored value of each form: (state U^n, RK stage buffer, Sigma,
# arithmetic type of the source b and of a stored 1/rho)
FORM_BYTES = {"f64": (8, 8, 8, 8), "f32": (4, 4, 4, 4), "f16": (2, 2, 2, 4), "bf16": (2, 2, 2, 4),
              "bf16d": (4, 2, 2, 4)}


def algorithmic_bytes_per_cell(kernel: str, precision: str, nsweeps: int, sigma_block: int = 2,
                               smoother: str = "jacobi", viscous: bool = False) -> float:
    """Compulsory HBM bytes per interior cell for one launch of `kernel`
    (averaged over the launches of one RK step).  The split form (bf16d)
    reads a later stage state as U^n (FP32) plus its BF16 difference,
    writes the differences of stages 1 and 2 and U^(n+1) (FP32) in stage 3,
    and its first Sigma pass stores 1/rho (FP32), which the later passes
    read instead of rho.  With the viscous terms the first Sigma pass (a
    two-level pass or a single first sweep) also writes the six stress
    components."""
    eu, ed, es, c = FORM_BYTES[precision]
    split = precision == "bf16d"
    if kernel == "flux_rk":
        if split:
            # stage 1: U^n, Sigma -> delta1; 2: U^n + delta1, Sigma -> delta2;
            # 3: U^n + delta2, Sigma -> U^(n+1)
            return (5 * eu + es + 5 * ed + 5 * (eu + ed) + es + 5 * ed + 5 * (eu + ed) + es + 5 * eu) / 3.0
        # stage 1 reads U (5) + Sigma (1), writes 5; stages 2 and 3 also read Un (5)
        return eu * (11 + 16 + 16) / 3.0
    if kernel == "jacobi":
        # first pass (one or two sweeps): reads rho, m, Sigma; writes Sigma,
        # b.  Later passes, single or two sweeps: read Sigma, rho, b; write Sigma
        nf, npair, nsingle = sigma_schedule(nsweeps, sigma_block, smoother)
        if split:
            state = 4 * (eu + ed * 2.0 / 3.0)      # rho, m: stage 1 from U^n, stages 2, 3 from U^n + delta
            first = state + 2 * es + c + c          # + Sigma in/out, b and 1/rho written
            later = 2 * es + c + c                  # Sigma in/out, 1/rho and b read
        else:
            first = 5 * eu + eu + c
            later = 3 * eu + c
        if viscous and nsweeps > 0 and sigma_block in (1, 2):
            first += 6 * c
        return (nf * first + (npair + nsingle) * later) / (nf + npair + nsingle)
    if kernel == "source":
        return 4 * eu + c          # rho, m read; b written
    # rho, m of the stage input: the split form's later stages read U^n and
    # a difference
    state = 4 * (eu + ed * 2.0 / 3.0) if split else 4 * eu
    if kernel == "stress":
        return state + 6 * c       # rho, m read; the six stress components written
    if kernel == "viscous":
        # rho, m and the six stress components read; the stage's four momentum
        # and energy fields read and written (split form: the differences of
        # stages 1 and 2, U^(n+1) in stage 3)
        out = (2 * 8 * ed + 8 * eu) / 3.0 if split else 8 * eu
        return state + 6 * c + out
    if kernel == "dt":
        return 5 * eu
    raise KeyError(kernel)


def kernel_rooflines(kt, cells: int, precision: str, nsweeps: int, sigma_block: int, smoother: str = "jacobi",
                     viscous: bool = False):
    """Algorithmic GB/s and fraction of the 8 TB/s HBM peak of the flux and
    Sigma kernels (and, when they ran, the viscous stress and flux
    divergence) from their measured average launch time (sigma_block: the
    pass structure the context ran)."""
    out = {}
    for k in ("flux_rk", "jacobi", "stress", "viscous"):
        if k not in kt:
            continue
        ms, cnt = kt[k]
        if cnt:
            ab = algorithmic_bytes_per_cell(k, precision, nsweeps, sigma_block, smoother, viscous) * cells
            gbs = ab / (ms / cnt / 1e3) / 1e9
            out[k] = {"avg_ms": round(ms / cnt, 5), "launches": cnt, "achieved_GBs": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def strip_comments(src: str) -> str:
    """C++ source without its comments, each run of whitespace made one
    space: what the compiler sees (string and character literals are kept
    as written)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the kernel sources as compiled (comments and layout left
    out): a committed counter summary stays valid across comment edits and
    is dropped once any code changes."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), encoding="utf-8") as f:
            h.update(name.encode() + strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed PMC summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def _oracle_rate(prob, U, sig, steps_max: int, seconds_target: float, dt_fn):
    import torch  # noqa: F401

    from oracle import igr_ref as ref

    steps, t0 = 0, time.perf_counter()
    while True:
        U, sig = ref.rk3_step(prob, U, sig, dt_fn(U))
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds_target or steps >= steps_max:
            return steps, el


def cpu_baseline_box(w, seconds_target: float = 15.0):
    """The FP64 oracle on a 128^3 instance of the periodic-box recipe."""
    import torch

    from oracle import igr_ref as ref
    from paper_2505_07392_amd import inputs

    n = 128
    ws = inputs.periodic_box(n=n, seed=w.seed)
    prob = ref.Problem(n, n, n, ws.dx, ws.dy, ws.dz, alpha=ws.alpha, faces=("periodic",) * 6, nsweeps=ws.nsweeps)
    sig = torch.zeros((n, n, n), dtype=torch.float64)
    steps, el = _oracle_rate(prob, torch.from_numpy(ws.U), sig, 50, seconds_target,
                             lambda V: ref.compute_dt(prob, V, w.cfl))
    return {"value": n ** 3 * steps / el, "unit": "cell-updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{steps} RK3 steps of the FP64 oracle on the 128^3 periodic box (same recipe and seed), "
                      f"{el:.1f} s"}


def cpu_baseline_jets(w, seconds_target: float = 15.0):
    """The FP64 oracle on a 128^3 instance of the multi-jet recipe (the
    same 4 x 4 discs of radius 10 cells, Mach 3, seed, alpha = 4 dx^2 and
    10 sweeps), CFL time step, timed on the host cores."""
    import torch

    from oracle import igr_ref as ref
    from paper_2505_07392_amd import inputs

    n = 128
    ws = jet_workload(n, 0, build_state=True)
    patches = tuple(ref.Patch(j.yc, j.zc, j.r, j.rho, j.ux, j.uy, j.uz, j.p, j.width) for j in ws.jets)
    prob = ref.Problem(n, n, n, ws.dx, ws.dy, ws.dz, gamma=ws.gamma, alpha=ws.alpha, faces=tuple(ws.faces),
                       patches=patches, nsweeps=ws.nsweeps)
    U = torch.from_numpy(ws.U)
    sig = torch.zeros((n, n, n), dtype=torch.float64)
    steps, el = _oracle_rate(prob, U, sig, 50, seconds_target, lambda V: ref.compute_dt(prob, V, ws.cfl))
    out = {"value": n ** 3 * steps / el, "unit": "cell-updates/s", "cores": torch.get_num_threads(),
           "kind": "oracle",
           "sample": f"{steps} RK3 steps of the FP64 oracle on a 128^3 instance of the multi-jet recipe "
                     f"(4 x 4 Mach-3 discs of radius 10 cells, 10 sweeps, alpha = 4 dx^2), {el:.1f} s"}
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        U1 = torch.from_numpy(ws.U)
        sig1 = torch.zeros((n, n, n), dtype=torch.float64)
        s1, el1 = _oracle_rate(prob, U1, sig1, 1, 0.0, lambda V: ref.compute_dt(prob, V, ws.cfl))
    finally:
        torch.set_num_threads(nthreads)
    out["single_thread"] = {"value": n ** 3 * s1 / el1, "cores": 1,
                            "sample": f"1 RK3 step of the same 128^3 multi-jet box, {el1:.1f} s"}
    return out


def run_form(w, precision, steps, warmup, sigma_block=0, order=5, smoother="jacobi"):
    import torch

    from paper_2505_07392_amd import igr

    s = igr.Solver.from_workload(w, precision=precision, sigma_block=sigma_block, order=order, smoother=smoother)
    U = s.state_from(w.U)
    sig = s.new_field()
    s.advance(U, sig, warmup, cfl=w.cfl, sync=False)
    s.check()
    torch.cuda.synchronize()
    s.timing(True)
    t0 = time.perf_counter()
    s.advance(U, sig, steps, cfl=w.cfl, sync=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.timing(False)
    s.check()
    kt = {k: s.kernel_time(k) for k in igr.kernel_names()}
    sb = s.sigma_block
    s.close()
    return el, kt, sb


def jet_workload(n: int, nsteps: int, build_state: bool = False):
    from paper_2505_07392_amd import inputs

    w = inputs.multi_jet(n=n, jets_per_side=4, radius_cells=10.0, mach=3.0, seed=0, nsweeps=10, nsteps=nsteps,
                         build_state=build_state)
    w.alpha = 4.0 * w.dx * w.dx     # Mach-3 jets need alpha = 4 dx^2 (alpha = dx^2 loses positivity)
    return w


FIELD_NAMES = ["rho", "mx", "my", "mz", "E", "Sigma", "p"]


def _final_fields(s, U, S, gamma):
    """The six fields and the derived pressure as one FP64 device array,
    formed in place (at 1024^3 each FP64 field is 8.6 GB)."""
    import torch

    nz, ny, nx = (d - 6 for d in U.shape[1:])
    fin = torch.empty((7, nz, ny, nx), dtype=torch.float64, device=U.device)
    fin[:5].copy_(s.interior(U))
    fin[5].copy_(s.interior(S))
    pr = fin[6]
    torch.mul(fin[1], fin[1], out=pr)
    pr.addcmul_(fin[2], fin[2]).addcmul_(fin[3], fin[3]).div_(fin[0]).mul_(-0.5).add_(fin[4])
    pr.mul_(gamma - 1.0)
    return fin


def jets_forms(n: int, forms, steps: int, warmup: int, err_steps: int, log=None, mu: float = 0.0,
               zeta: float = 0.0, order: int = 5, sigma_block: int = 0, smoother: str = "jacobi"):
    """Multi-jet box in each precision form (FP64 first): the rate over
    `steps` CFL steps after `warmup` (igr_advance, HIP-event timing of every
    launch), the device memory in use, and the per-field rel L1 error of the
    six fields and the derived pressure against the FP64 run after
    `err_steps` steps from the initial state with one fixed dt (0.8 x the
    FP64 CFL step of the initial state).  mu, zeta: shear and bulk viscosity
    of eq. (5); order, sigma_block, smoother: the solver options (0: the
    library's default pass structure)."""
    import torch

    from paper_2505_07392_amd import igr, inputs

    w = jet_workload(n, err_steps)
    w.mu, w.zeta = mu, zeta
    say = log or (lambda m: print(m, file=sys.stderr, flush=True))
    out, ref, dt = {}, None, None
    for prec in forms:
        say(f"[bench] multi-jet {n}^3 {prec}: building the state")
        s = igr.Solver.from_workload(w, precision=prec, order=order, sigma_block=sigma_block, smoother=smoother)
        U = s.new_state()
        inputs.fill_multi_jet_state(w, s.interior(U))
        S = s.new_field()
        if dt is None:
            dt = 0.8 * s.compute_dt(U, w.cfl)
        say(f"[bench] multi-jet {n}^3 {prec}: {warmup} warm-up + {steps} timed steps")
        s.advance(U, S, warmup, cfl=w.cfl, sync=False)
        s.check()
        torch.cuda.synchronize()
        free, total = torch.cuda.mem_get_info()
        s.timing(True)
        t0 = time.perf_counter()
        s.advance(U, S, steps, cfl=w.cfl, sync=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.timing(False)
        s.check()
        kt = {k: s.kernel_time(k) for k in igr.kernel_names()}
        form = {"value": w.cells * steps / el, "ms_per_step": 1e3 * el / steps, "elapsed_s": el,
                "device_bytes_in_use": total - free, "frac_of_288GB": round((total - free) / 288e9, 4),
                "sigma_block": s.sigma_block, "kernel_times": kt}
        form.update(kernel_rooflines(kt, w.cells, prec, w.nsweeps, s.sigma_block, smoother, mu > 0 or zeta > 0))
        if err_steps > 0:
            say(f"[bench] multi-jet {n}^3 {prec}: {err_steps} fixed-dt steps for the error")
            inputs.fill_multi_jet_state(w, s.interior(U))
            S.zero_()
            try:
                s.advance(U, S, err_steps, dt_fixed=dt, sync=True)
            except igr.NonFiniteError as e:
                form["run_failed"] = f"non-physical state in the fixed-dt run: {e}"
            else:
                fin = _final_fields(s, U, S, w.gamma)
                if prec == "f64":
                    ref = fin
                elif ref is not None:
                    err = [float((fin[f] - ref[f]).abs().sum() / ref[f].abs().sum())
                           if float(ref[f].abs().sum()) > 0 else 0.0 for f in range(len(FIELD_NAMES))]
                    form["rel_l1_vs_f64"] = dict(zip(FIELD_NAMES, err))
                    del fin
        out[prec] = form
        del U, S
        s.close()
        torch.cuda.empty_cache()
    return w, out, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="multi_jet", choices=["multi_jet", "periodic_box"])
    ap.add_argument("--n", type=int, default=None, help="cells per side (default 1024 multi-jet, 256 box)")
    ap.add_argument("--precision", default="f64", choices=sorted(FORM_BYTES))
    ap.add_argument("--forms", default="f32,bf16d,f16,bf16", help="extra precision forms timed on the same workload")
    ap.add_argument("--err-steps", type=int, default=20,
                    help="fixed-dt steps of the multi-jet error run per form (0: none)")
    ap.add_argument("--no-extra", action="store_true", help="skip the 256^3 periodic box under `extra`")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sigma-block", type=int, default=0, choices=[0, 1, 2],
                    help="Sigma pass structure: 1 single sweeps, 2 two-sweep passes (0: library default)")
    ap.add_argument("--order", type=int, default=5, choices=[5, 3], help="reconstruction order")
    ap.add_argument("--smoother", default="jacobi", choices=["jacobi", "rbgs"], help="Sigma sweeps")
    ap.add_argument("--mu", type=float, default=0.0,
                    help="shear viscosity of eq. (5) (viscous terms)")
    ap.add_argument("--zeta", type=float, default=0.0, help="bulk viscosity of eq. (5)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path (the halo-exchange "
              "design is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    viscous = args.mu > 0.0 or args.zeta > 0.0

    import torch

    from paper_2505_07392_amd import igr, inputs

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = 1 << 27                        # 2^27 float64 = 1 GiB
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 3
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 4,
                          "seconds_per_copy": el, "GBs_read_plus_write": 2 * n * 8 / el / 1e9}))
        return
    forms_req = [x for x in args.forms.split(",") if x and x != args.precision]

    if args.workload == "multi_jet":
        n = args.n or 1024
        w, res, dt_err = jets_forms(n, [args.precision] + forms_req, args.steps, args.warmup, args.err_steps,
                                    mu=args.mu, zeta=args.zeta, order=args.order, sigma_block=args.sigma_block,
                                    smoother=args.smoother)
        main_form = res.pop(args.precision)
        cells, el, kt, sb = w.cells, main_form["elapsed_s"], main_form.pop("kernel_times"), main_form["sigma_block"]
        workload = f"multi_jet_{n}"
        desc = (f"{workload}: {n}^3 multi-jet box, 4 x 4 Mach-3 inflow discs of radius 10 cells on the x-min "
                f"face (rho 0.5, p 8, +-5 % seeded u_x), ambient (1, 0, 1), outflow elsewhere, "
                f"{w.nsweeps} Jacobi sweeps, alpha = 4 dx^2 (not dx^2: the Mach-3 jet edges lose positivity "
                f"at alpha = dx^2), CFL 0.5")
        if viscous:
            workload += "_viscous"
            desc += f", viscous terms of eq. (5) with mu = {args.mu:g}, zeta = {args.zeta:g}"
    else:
        n = args.n or 256
        print(f"[bench] generating the {n}^3 periodic box", file=sys.stderr, flush=True)
        w = inputs.periodic_box(n=n, seed=0)
        w.mu, w.zeta = args.mu, args.zeta
        cells = w.cells
        el, kt, sb = run_form(w, args.precision, args.steps, args.warmup, args.sigma_block, args.order,
                              args.smoother)
        workload = f"periodic_box_{n}"
        desc = (f"{workload}: periodic box {n}^3, rms Mach 1.5, alpha = dx^2, {w.nsweeps} Jacobi sweeps, "
                f"CFL 0.5")
        if viscous:
            workload += "_viscous"
            desc += f", viscous terms of eq. (5) with mu = {args.mu:g}, zeta = {args.zeta:g}"
        main_form = None

    value = cells * args.steps / el
    visc = args.mu > 0 or args.zeta > 0
    # dominant kernel by total time in the timed region
    dom = max((k for k in kt if kt[k][1] > 0), key=lambda k: kt[k][0])
    ms, count = kt[dom]
    avg_s = ms / count / 1e3
    try:
        abytes = algorithmic_bytes_per_cell(dom, args.precision, w.nsweeps, sb, args.smoother, visc) * cells
    except KeyError:
        abytes = None
    achieved = abytes / avg_s / 1e9 if abytes else None
    traffic = load_traffic(dom, f"{workload}_{args.precision}") if (args.order == 5 and not args.sigma_block
                                                                      and args.smoother == "jacobi") else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                "avg_launch_ms": ms / count, "launches": count,
                "algorithmic_bytes_per_launch": abytes}
    kernels = {k: {"ms_total": round(v[0], 4), "launches": v[1], "avg_ms": round(v[0] / v[1], 5)}
               for k, v in kt.items() if v[1] > 0}
    kernels.update({k + "_roofline": v for k, v in kernel_rooflines(kt, cells, args.precision, w.nsweeps,
                                                                    sb, args.smoother, visc).items()})

    forms = {}
    if args.workload == "multi_jet":
        for f, d in res.items():
            d.pop("kernel_times", None)
            d.pop("elapsed_s", None)
            d["vs_f64"] = round(d["value"] / value, 3) if args.precision == "f64" else None
            forms[f] = d
    else:
        for f in forms_req:
            print(f"[bench] timing {f}", file=sys.stderr, flush=True)
            e2, kt2, sb2 = run_form(w, f, args.steps, args.warmup, args.sigma_block, args.order, args.smoother)
            forms[f] = {"value": cells * args.steps / e2, "ms_per_step": 1e3 * e2 / args.steps,
                        "vs_f64": None, "sigma_block": sb2}
            forms[f].update(kernel_rooflines(kt2, cells, f, w.nsweeps, sb2, args.smoother, visc))
            if args.precision == "f64":
                forms[f]["vs_f64"] = round(forms[f]["value"] / value, 3)

    line = {
        "metric": "cell-updates/s per RK3 step (incl. Sigma Jacobi)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "grind_ns_per_cell_step": 1e9 / value,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": desc, "cells": cells, "sweeps": w.nsweeps, "alpha_over_dx2": w.alpha / w.dx ** 2,
                   "precision": args.precision, "order": args.order, "smoother": args.smoother,
                   "sigma_block": sb},
        "roofline": roofline,
        "kernels": kernels,
        "forms": forms,
    }
    if main_form is not None:
        line["device_bytes_in_use"] = main_form["device_bytes_in_use"]
        line["frac_of_288GB"] = main_form["frac_of_288GB"]
        line["error_run"] = {"steps": args.err_steps, "dt_fixed": dt_err,
                             "reference": "the FP64 GPU run of the same steps (parity-tested against the oracle)"}
    if args.workload == "multi_jet" and not args.no_extra:
        print("[bench] extra: generating the 256^3 periodic box", file=sys.stderr, flush=True)
        wb = inputs.periodic_box(n=256, seed=0)
        extra = {}
        for prec in ["f64"] + [f for f in forms_req if f != "f64"]:
            print(f"[bench] extra: periodic box 256^3 {prec}", file=sys.stderr, flush=True)
            eb, ktb, sbb = run_form(wb, prec, 20, 3)
            extra[prec] = {"value": wb.cells * 20 / eb, "ms_per_step": 1e3 * eb / 20, "sigma_block": sbb}
            extra[prec].update(kernel_rooflines(ktb, wb.cells, prec, wb.nsweeps, sbb))
        for prec in extra:
            extra[prec]["vs_f64"] = round(extra[prec]["value"] / extra["f64"]["value"], 3)
        line["extra"] = {"periodic_box_256": {"workload": "periodic box 256^3, rms Mach 1.5, alpha = dx^2, "
                                                          "5 Jacobi sweeps, CFL 0.5; 3 warm-up + 20 timed steps",
                                              "forms": extra}}
    if not args.no_cpu_baseline:
        print("[bench] oracle cpu baseline", file=sys.stderr, flush=True)
        if args.workload == "multi_jet":
            line["cpu_baseline"] = cpu_baseline_jets(w)
        else:
            line["cpu_baseline"] = cpu_baseline_box(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
