"""Plain FP64 reference of one IGR right-hand side and the SSP-RK3 step.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Everything is whole-array ``torch.float64`` on the CPU, written for a reader
holding the paper, with no blocking, fusion or reordering beyond what the
definitions state.  All operations are differentiable, so
``torch.autograd`` on these functions *is* the oracle's discrete adjoint.

Array convention
----------------
``U``      conserved state, shape ``[5, nz, ny, nx]`` (rho, rho*u, rho*v,
           rho*w, E), x fastest.  Interior cells only.
``sigma``  entropic pressure, shape ``[nz, ny, nx]``.
Padded arrays carry ``G = 3`` ghost layers on every side.  Axis ``d`` is
0 = x, 1 = y, 2 = z; it is tensor dimension ``-1 - d`` and momentum
component ``1 + d``.  Only face ghosts (one ghost index, the other two
interior) are ever read; edge and corner ghosts are filled but unused.

Method (paper section "Innovations Realized")
---------------------------------------------
* IGR-modified Euler system, eqs. (6)-(8) with tau = 0: p is replaced by
  p + Sigma in the momentum and energy fluxes.  With a nonzero shear or
  bulk viscosity the viscous stress of eq. (5) enters as in eqs. (2)-(3)
  and (7)-(8).
* Entropic pressure, eq. (9):
  alpha [tr((grad u)^2) + tr^2(grad u)] = Sigma/rho - alpha div(grad Sigma / rho).
* "Discretization" subsection: second-order central velocity gradients for
  the left side of eq. (9), a 7-point stencil for the operator on the right,
  a fixed number of Jacobi sweeps warm-started from the previous Sigma,
  fifth-order (or third-order) linear reconstruction, Lax-Friedrichs
  interface fluxes and a third-order SSP Runge-Kutta stepper (Gottlieb &
  Shu 1998).
* "The algorithm" subsection, Algorithm 1: dimension-by-dimension faces,
  reconstruction of the conserved variables and of Sigma on the stencil
  q = -2..3, conversion to primitives at the faces, inviscid flux.

Readings where the paper is silent:
* 7-point operator face coefficient: beta = (1/rho_c + 1/rho_nb) / 2.
* Jacobi: exactly ``nsweeps`` sweeps, Sigma ghosts refilled from the
  previous iterate before every sweep (zero-gradient or periodic).
  Red-black Gauss-Seidel (option): each sweep updates the cells with
  i + j + k even, then the others, each colour from the values at the
  start of its half-sweep.
* Local Lax-Friedrichs (Rusanov): lambda = max(|u_n| + c) over the two
  reconstructed states, thermodynamic p only; dissipation on the five
  conserved variables only (Sigma enters the central flux only).
* Boundary ghosts: periodic wrap, zero-gradient extrapolation (all three
  layers copy the first interior cell), and jet discs on the x-min face:
  each ghost column takes the nearest disc and blends its jet state with
  the extrapolated state by a tanh profile in the distance to the disc
  centre (a sharp disc when the width is zero).
* dt = CFL / max over cells of sum_d (|u_d| + c) / dx_d.
* Viscous terms: second-order central velocity gradients at cell centres
  (the paper: second-order derivatives of u suffice), ghost gradients by
  the rule of Sigma's ghosts, face gradients reconstructed with the weights
  of the conserved variables (Algorithm 1 reconstructs the gradients with
  the same coefficients), face velocities from the reconstructed conserved
  variables, and the mean of the two sides' viscous fluxes (no dissipation
  term); mu and zeta constant.

Parity pins (tests/test_oracle_*.py): reconstruction polynomial exactness
(degree <= 4 for the fifth-order, <= 2 for the third-order interpolant)
and mirror symmetry; source exactness for linear velocity fields; Jacobi
sweep against a brute-force dense assembly, symmetry of the assembled
operator, convergence to a dense solve, the 6/7 contraction factor;
flux consistency F(U, U) = F(U); uniform-state preservation; axis
permutation and mirror symmetry; alpha = 0 against an independently written
per-cell Lax-Friedrichs code; Sod against the exact Riemann solution;
periodic conservation; fifth- and third-order convergence on an entropy
wave; RK3 against its stability polynomial; the viscous stress and flux
against linear velocity fields (closed-form stress and heating, zero for a
rigid rotation), the Fourier symbol of the viscous operator on a shear
wave, and discrete conservation with viscosity.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Sequence

import torch

G = 3  # ghost layers needed by the five-point upwind reconstruction

PERIODIC = "periodic"
EXTRAP = "extrap"

# Fifth-order linear reconstruction from five cell averages (the optimal
# linear weights of WENO5).  Left state at face i+1/2 from cells i-2..i+2,
# right state at the same face from cells i-1..i+3 (mirror image).
RECON_LEFT = (2.0, -13.0, 47.0, 27.0, -3.0)
RECON_RIGHT = (-3.0, 27.0, 47.0, -13.0, 2.0)
RECON_DENOM = 60.0

# Third-order linear reconstruction from three cell averages (the paper's
# other order, "Discretization"; the optimal linear weights of WENO3).  Left
# state at face i+1/2 from cells i-1..i+1, right state from cells i..i+2.
RECON3_LEFT = (-1.0, 5.0, 2.0)
RECON3_RIGHT = (2.0, 5.0, -1.0)
RECON3_DENOM = 6.0


class NonPhysicalState(RuntimeError):
    """Raised when a face or cell state has rho <= 0, p <= 0 or is not finite."""


@dataclass
class Patch:
    """Dirichlet inflow disc on the x-min face (paper, "Example simulation
    result": engines are modelled by inflow boundary conditions).

    ``yc, zc, r, width`` are physical lengths; the primitive jet state may
    be floats or 0-dim float64 tensors (for differentiation).  The ghost
    state of a column at distance s from the disc centre is the blend
    chi U_jet + (1 - chi) U_extrap with chi = (1 - tanh((s - r)/width))/2,
    or the indicator s <= r when width is 0."""

    yc: float
    zc: float
    r: float
    rho: object
    ux: object
    uy: object
    uz: object
    p: object
    width: float = 0.0


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    gamma: float = 1.4
    alpha: float = 0.0
    faces: Sequence[str] = (EXTRAP,) * 6  # -x, +x, -y, +y, -z, +z
    patches: Sequence[Patch] = field(default_factory=tuple)
    nsweeps: int = 5
    order: int = 5          # reconstruction order: 5 or 3 ("Discretization")
    smoother: str = "jacobi"   # Sigma sweeps: "jacobi" or "rbgs" (red-black Gauss-Seidel)
    mu: float = 0.0         # shear viscosity, eq. (5) (0: the Euler system)
    zeta: float = 0.0       # bulk viscosity, eq. (5)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def n(self, d):
        return (self.nx, self.ny, self.nz)[d]

    def h(self, d):
        return (self.dx, self.dy, self.dz)[d]

    def axis_kind(self, d):
        lo, hi = self.faces[2 * d], self.faces[2 * d + 1]
        if (lo == PERIODIC) != (hi == PERIODIC):
            raise ValueError("periodic faces must come in pairs")
        return lo


# ---------------------------------------------------------------------------
# Boundary ghosts
# ---------------------------------------------------------------------------

def _source_index(n: int, g: int, periodic: bool) -> torch.Tensor:
    """Padded index p in [-g, n+g) -> interior index it copies."""
    p = torch.arange(-g, n + g)
    if periodic:
        return torch.remainder(p, n)
    return p.clamp(0, n - 1)


def patch_weights(prob: Problem):
    """Per x-min ghost column (k, j): the owning patch (nearest disc centre
    to the cell centre ((j+1/2) dy, (k+1/2) dz), lowest index on ties) and
    its blend weight chi.  Returns (owner [nz, ny] int64, chi [nz, ny])."""
    yc = (torch.arange(prob.ny, dtype=torch.float64) + 0.5) * prob.dy
    zc = (torch.arange(prob.nz, dtype=torch.float64) + 0.5) * prob.dz
    best = torch.full((prob.nz, prob.ny), float("inf"), dtype=torch.float64)
    owner = torch.full((prob.nz, prob.ny), -1, dtype=torch.int64)
    for q, pa in enumerate(prob.patches):
        d2 = (yc[None, :] - pa.yc) ** 2 + (zc[:, None] - pa.zc) ** 2
        closer = d2 < best
        best = torch.where(closer, d2, best)
        owner = torch.where(closer, torch.full_like(owner, q), owner)
    chi = torch.zeros((prob.nz, prob.ny), dtype=torch.float64)
    for q, pa in enumerate(prob.patches):
        mine = owner == q
        if pa.width > 0:
            w = 0.5 * (1.0 - torch.tanh((torch.sqrt(best) - pa.r) / pa.width))
        else:
            w = (best <= pa.r ** 2).to(torch.float64)
        chi = torch.where(mine, w, chi)
    return owner, chi


def jet_conserved(prob: Problem, pa: Patch) -> torch.Tensor:
    """Primitive jet state -> conserved 5-vector via the ideal-gas law, eq. (4)."""
    as_t = lambda v: v if torch.is_tensor(v) else torch.tensor(float(v), dtype=torch.float64)
    rho, ux, uy, uz, p = (as_t(v) for v in (pa.rho, pa.ux, pa.uy, pa.uz, pa.p))
    E = p / (prob.gamma - 1.0) + 0.5 * rho * (ux * ux + uy * uy + uz * uz)
    return torch.stack([rho, rho * ux, rho * uy, rho * uz, E])


def pad_state(prob: Problem, U: torch.Tensor, g: int = G) -> torch.Tensor:
    """Conserved state with g ghost layers: periodic wrap or zero-gradient
    copy per axis, then the jet discs on the x-min ghost columns."""
    V = U.index_select(-1, _source_index(prob.nx, g, prob.axis_kind(0) == PERIODIC))
    if prob.patches:
        if prob.axis_kind(0) == PERIODIC:
            raise ValueError("inflow patches need a non-periodic x-min face")
        owner, chi = patch_weights(prob)
        ghost = V[..., :g]
        blended = ghost
        for q in range(len(prob.patches)):
            jet = jet_conserved(prob, prob.patches[q]).reshape(5, 1, 1, 1)
            c = chi[None, :, :, None]
            mix = c * jet + (1.0 - c) * ghost
            blended = torch.where((owner == q)[None, :, :, None], mix, blended)
        V = torch.cat([blended, V[..., g:]], dim=-1)
    V = V.index_select(-2, _source_index(prob.ny, g, prob.axis_kind(1) == PERIODIC))
    V = V.index_select(-3, _source_index(prob.nz, g, prob.axis_kind(2) == PERIODIC))
    return V


def pad_sigma(prob: Problem, sigma: torch.Tensor, g: int) -> torch.Tensor:
    """Sigma with g ghost layers: periodic wrap, else zero gradient (every
    non-periodic face, jet discs included)."""
    V = sigma
    for d in range(3):
        V = V.index_select(-1 - d, _source_index(prob.n(d), g, prob.axis_kind(d) == PERIODIC))
    return V


def _interior(prob: Problem, a: torch.Tensor, g: int, d: int = -1, s: int = 0) -> torch.Tensor:
    """Interior block of a g-padded array, shifted by s cells along axis d."""
    sl = []
    for ax in (2, 1, 0):  # tensor dims z, y, x
        o = g + (s if ax == d else 0)
        sl.append(slice(o, o + prob.n(ax)))
    return a[(Ellipsis, *sl)]


# ---------------------------------------------------------------------------
# Entropic pressure: source and Jacobi sweeps (eq. 9, "Discretization")
# ---------------------------------------------------------------------------

def sigma_source(prob: Problem, Upad: torch.Tensor, g: int = G) -> torch.Tensor:
    """b = alpha [tr((grad u)^2) + tr^2(grad u)] with central differences.

    tr((grad u)^2) = sum_ij G_ij G_ji for G_ij = d u_i / d x_j."""
    u = Upad[1:4] / Upad[0]
    Gm = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            Gm[i][j] = (_interior(prob, u[i], g, j, +1) - _interior(prob, u[i], g, j, -1)) / (
                2.0 * prob.h(j))
    tr = Gm[0][0] + Gm[1][1] + Gm[2][2]
    tr_sq = sum(Gm[i][j] * Gm[j][i] for i in range(3) for j in range(3))
    return prob.alpha * (tr_sq + tr * tr)


def jacobi_sweep(prob: Problem, sigma: torch.Tensor, b: torch.Tensor,
                 rho_pad: torch.Tensor, g: int = G) -> torch.Tensor:
    """One Jacobi sweep for Sigma/rho - alpha div(beta grad Sigma) = b.

    Sigma_new = [b + alpha sum_d (beta+ S+ + beta- S-)/h_d^2]
              / [1/rho + alpha sum_d (beta+ + beta-)/h_d^2]
    with S+- the previous iterate at the axis neighbours (ghosts refilled
    from the previous iterate) and beta+- = (1/rho_c + 1/rho_nb)/2."""
    inv = 1.0 / rho_pad
    inv_c = _interior(prob, inv, g)
    sp = pad_sigma(prob, sigma, 1)
    num = b
    den = inv_c
    for d in range(3):
        h2 = prob.h(d) ** 2
        beta_p = 0.5 * (inv_c + _interior(prob, inv, g, d, +1))
        beta_m = 0.5 * (inv_c + _interior(prob, inv, g, d, -1))
        num = num + prob.alpha * (beta_p * _interior(prob, sp, 1, d, +1)
                                  + beta_m * _interior(prob, sp, 1, d, -1)) / h2
        den = den + prob.alpha * (beta_p + beta_m) / h2
    return num / den


def red_cells(prob: Problem) -> torch.Tensor:
    """Boolean mask of the 'red' cells, (i + j + k) even."""
    k, j, i = torch.meshgrid(torch.arange(prob.nz), torch.arange(prob.ny), torch.arange(prob.nx), indexing="ij")
    return (i + j + k) % 2 == 0


def rbgs_sweep(prob: Problem, sigma: torch.Tensor, b: torch.Tensor,
               rho_pad: torch.Tensor, g: int = G) -> torch.Tensor:
    """One red-black Gauss-Seidel sweep (the paper's alternative to Jacobi,
    "Discretization"): the Jacobi update applied to the red cells, then to
    the black cells with the new red values.  Within one colour every cell
    uses the values at the start of that half-sweep (ghosts refilled from
    them).  On a grid whose periodic extents are even a cell's axis
    neighbours all have the other colour, so this is the Gauss-Seidel
    iteration for the red-black ordering of the cells."""
    red = red_cells(prob)
    half = torch.where(red, jacobi_sweep(prob, sigma, b, rho_pad, g), sigma)
    return torch.where(red, half, jacobi_sweep(prob, half, b, rho_pad, g))


def sigma_solve(prob: Problem, U: torch.Tensor, sigma0: torch.Tensor,
                nsweeps: int | None = None, Upad: torch.Tensor | None = None):
    """Fill U ghosts, build b, run ``nsweeps`` sweeps of the problem's
    smoother (Jacobi, or red-black Gauss-Seidel) from sigma0.

    Returns (sigma, b)."""
    if Upad is None:
        Upad = pad_state(prob, U)
    S = prob.nsweeps if nsweeps is None else nsweeps
    b = sigma_source(prob, Upad)
    sweep = {"jacobi": jacobi_sweep, "rbgs": rbgs_sweep}[prob.smoother]
    sig = sigma0
    for _ in range(S):
        sig = sweep(prob, sig, b, Upad[0])
    return sig, b


def apply_sigma_operator(prob: Problem, U: torch.Tensor, sigma: torch.Tensor) -> torch.Tensor:
    """A Sigma = Sigma/rho - alpha div(beta grad Sigma) with the ghost rules
    of the sweep (zero-gradient faces contribute nothing)."""
    Upad = pad_state(prob, U)
    inv = 1.0 / Upad[0]
    inv_c = _interior(prob, inv, G)
    sp = pad_sigma(prob, sigma, 1)
    out = sigma * inv_c
    for d in range(3):
        h2 = prob.h(d) ** 2
        beta_p = 0.5 * (inv_c + _interior(prob, inv, G, d, +1))
        beta_m = 0.5 * (inv_c + _interior(prob, inv, G, d, -1))
        flux_p = beta_p * (_interior(prob, sp, 1, d, +1) - sigma)
        flux_m = beta_m * (sigma - _interior(prob, sp, 1, d, -1))
        out = out - prob.alpha * (flux_p - flux_m) / h2
    return out


def sigma_residual_l2(prob: Problem, U: torch.Tensor, sigma: torch.Tensor) -> float:
    """Plain l2 norm (no volume weight) of b - A Sigma over interior cells."""
    b = sigma_source(prob, pad_state(prob, U))
    r = b - apply_sigma_operator(prob, U, sigma)
    return float(torch.sqrt((r * r).sum()))


# ---------------------------------------------------------------------------
# Reconstruction and Lax-Friedrichs flux (Algorithm 1; "Discretization")
# ---------------------------------------------------------------------------

def reconstruct(prob: Problem, qpad: torch.Tensor, d: int, g: int = G):
    """Left/right states at the n_d + 1 faces along axis d (face f lies
    between cells f-1 and f), on the interior transverse range."""
    n = prob.n(d)
    dim = -1 - d

    def take(offset):
        t = qpad.narrow(dim, g + offset, n + 1)
        for ax in range(3):
            if ax != d:
                t = t.narrow(-1 - ax, g, prob.n(ax))
        return t

    # face f = i + 1/2 with i = f - 1 (take(o) is cell i + 1 + o)
    if prob.order == 5:       # left: cells i-2..i+2, right: i-1..i+3
        left = sum(c * take(o) for c, o in zip(RECON_LEFT, (-3, -2, -1, 0, 1))) / RECON_DENOM
        right = sum(c * take(o) for c, o in zip(RECON_RIGHT, (-2, -1, 0, 1, 2))) / RECON_DENOM
    elif prob.order == 3:     # left: cells i-1..i+1, right: i..i+2
        left = sum(c * take(o) for c, o in zip(RECON3_LEFT, (-2, -1, 0))) / RECON3_DENOM
        right = sum(c * take(o) for c, o in zip(RECON3_RIGHT, (-1, 0, 1))) / RECON3_DENOM
    else:
        raise ValueError("reconstruction order must be 3 or 5")
    return left, right


def pressure(prob: Problem, U: torch.Tensor) -> torch.Tensor:
    """Ideal-gas pressure, eq. (4): p = (gamma-1)(E - |m|^2 / (2 rho))."""
    m = U[1:4]
    return (prob.gamma - 1.0) * (U[4] - 0.5 * (m * m).sum(0) / U[0])


def _check_physical(rho, p, where):
    r, q = rho.detach(), p.detach()
    if not (torch.isfinite(r).all() and torch.isfinite(q).all()):
        raise NonPhysicalState(f"non-finite state at {where}")
    if (r <= 0).any() or (q <= 0).any():
        raise NonPhysicalState(f"rho <= 0 or p <= 0 at {where}")


def euler_flux(prob: Problem, U: torch.Tensor, sig: torch.Tensor, d: int):
    """Physical flux of eqs. (6)-(8) with tau = 0 along axis d, and the
    signal speed |u_d| + c.  Returns (F [5,...], speed)."""
    rho, m, E = U[0], U[1:4], U[4]
    p = pressure(prob, U)
    _check_physical(rho, p, f"faces along axis {d}")
    un = m[d] / rho
    c = torch.sqrt(prob.gamma * p / rho)
    F = [m[d]]
    for k in range(3):
        Fk = m[k] * un
        if k == d:
            Fk = Fk + (p + sig)
        F.append(Fk)
    F.append((E + p + sig) * un)
    return torch.stack(F), un.abs() + c


def llf_flux(prob: Problem, UL, UR, SL, SR, d: int) -> torch.Tensor:
    """Local Lax-Friedrichs numerical flux at faces along axis d."""
    FL, sL = euler_flux(prob, UL, SL, d)
    FR, sR = euler_flux(prob, UR, SR, d)
    lam = torch.maximum(sL, sR)
    return 0.5 * (FL + FR) - 0.5 * lam * (UR - UL)


def flux_divergence(prob: Problem, Upad: torch.Tensor, Spad: torch.Tensor) -> torch.Tensor:
    """L(U) = - sum_d (F_{i+1/2} - F_{i-1/2}) / h_d over interior cells."""
    L = torch.zeros((5,) + prob.shape, dtype=Upad.dtype)
    for d in range(3):
        UL, UR = reconstruct(prob, Upad, d)
        SL, SR = reconstruct(prob, Spad, d)
        F = llf_flux(prob, UL, UR, SL, SR, d)
        n = prob.n(d)
        dim = -1 - d
        L = L - (F.narrow(dim, 1, n) - F.narrow(dim, 0, n)) / prob.h(d)
    return L


# ---------------------------------------------------------------------------
# Viscous stress (eqs. (1)-(3) with eq. (5); "Discretization"; Algorithm 1's
# viscous flux)
# ---------------------------------------------------------------------------

def velocity_gradient(prob: Problem, Upad: torch.Tensor, g: int = G) -> torch.Tensor:
    """G[i][j] = d u_i / d x_j at interior cells by second-order central
    differences of u = m / rho.  Returns [3, 3, nz, ny, nx]."""
    u = Upad[1:4] / Upad[0]
    rows = []
    for i in range(3):
        rows.append(torch.stack([(_interior(prob, u[i], g, j, +1) - _interior(prob, u[i], g, j, -1)) /
                                 (2.0 * prob.h(j)) for j in range(3)]))
    return torch.stack(rows)


def pad_gradient(prob: Problem, Gm: torch.Tensor, g: int = G) -> torch.Tensor:
    """Gradient with g ghost layers, per component: periodic wrap, else a
    copy of the first interior cell (every non-periodic face, inflow discs
    included), the ghost rule of Sigma."""
    return torch.stack([torch.stack([pad_sigma(prob, Gm[i][j], g) for j in range(3)]) for i in range(3)])


def viscous_stress(prob: Problem, Gm):
    """Eq. (5): tau_ij = mu (G_ij + G_ji) + (zeta - 2 mu / 3) delta_ij div u,
    G_ij = d u_i / d x_j.  Returns a 3 x 3 nested list of tensors."""
    div = Gm[0][0] + Gm[1][1] + Gm[2][2]
    tau = [[prob.mu * (Gm[i][j] + Gm[j][i]) for j in range(3)] for i in range(3)]
    for i in range(3):
        tau[i][i] = tau[i][i] + (prob.zeta - 2.0 * prob.mu / 3.0) * div
    return tau


def viscous_flux_divergence(prob: Problem, Upad: torch.Tensor, Gpad: torch.Tensor) -> torch.Tensor:
    """Viscous part of L(U).  At every face along axis d: the velocity
    gradient on each side reconstructed from the cell-centre gradients with
    the weights of the conserved variables, the face velocity on each side
    from the reconstructed conserved variables, the stress of each side, and
    the mean of the two sides' viscous fluxes: -tau e_d for the momenta and
    -(u . tau) e_d for the energy (eqs. (2)-(3)); none for the mass.
    L_v = - sum_d (F_{i+1/2} - F_{i-1/2}) / h_d."""
    L = torch.zeros((5,) + prob.shape, dtype=Upad.dtype)
    for d in range(3):
        UL, UR = reconstruct(prob, Upad, d)
        GL = [[None] * 3 for _ in range(3)]
        GR = [[None] * 3 for _ in range(3)]
        for i in range(3):
            for j in range(3):
                GL[i][j], GR[i][j] = reconstruct(prob, Gpad[i][j], d)
        tL, tR = viscous_stress(prob, GL), viscous_stress(prob, GR)
        uL, uR = UL[1:4] / UL[0], UR[1:4] / UR[0]
        F = [torch.zeros_like(UL[0])]
        for k in range(3):
            F.append(-0.5 * (tL[k][d] + tR[k][d]))
        F.append(-0.5 * (sum(uL[k] * tL[k][d] for k in range(3)) + sum(uR[k] * tR[k][d] for k in range(3))))
        F = torch.stack(F)
        n = prob.n(d)
        dim = -1 - d
        L = L - (F.narrow(dim, 1, n) - F.narrow(dim, 0, n)) / prob.h(d)
    return L


def rhs(prob: Problem, U: torch.Tensor, sigma0: torch.Tensor):
    """One right-hand-side evaluation: ghosts, Sigma solve warm-started from
    sigma0, Sigma ghosts, reconstruction, LLF flux, divergence, and with a
    nonzero viscosity the viscous flux divergence.

    Returns (L(U), sigma)."""
    Upad = pad_state(prob, U)
    sig, _ = sigma_solve(prob, U, sigma0, Upad=Upad)
    L = flux_divergence(prob, Upad, pad_sigma(prob, sig, G))
    if prob.mu != 0.0 or prob.zeta != 0.0:
        L = L + viscous_flux_divergence(prob, Upad, pad_gradient(prob, velocity_gradient(prob, Upad)))
    return L, sig


# ---------------------------------------------------------------------------
# Time stepping, dt and diagnostics
# ---------------------------------------------------------------------------

def rk3_step(prob: Problem, U: torch.Tensor, sigma: torch.Tensor, dt,
             rhs_fn: Callable | None = None):
    """Third-order SSP Runge-Kutta (Gottlieb & Shu), one Sigma solve per
    stage, each warm-started from the previous stage.  Returns (U, sigma)."""
    f = rhs if rhs_fn is None else rhs_fn
    L0, s1 = f(prob, U, sigma)
    U1 = U + dt * L0
    L1, s2 = f(prob, U1, s1)
    U2 = 0.75 * U + 0.25 * (U1 + dt * L1)
    L2, s3 = f(prob, U2, s2)
    U3 = U / 3.0 + (2.0 / 3.0) * (U2 + dt * L2)
    return U3, s3


def compute_dt(prob: Problem, U: torch.Tensor, cfl: float) -> float:
    """dt = CFL / max_cells sum_d (|u_d| + c) / h_d (FP64)."""
    with torch.no_grad():
        rho = U[0]
        p = pressure(prob, U)
        _check_physical(rho, p, "cell centres")
        c = torch.sqrt(prob.gamma * p / rho)
        s = 0.0
        for d in range(3):
            s = s + ((U[1 + d] / rho).abs() + c) / prob.h(d)
        return float(cfl / s.max())


def conserved_sums(prob: Problem, U: torch.Tensor) -> torch.Tensor:
    """FP64 totals sum_cells U dV of the five conserved variables."""
    return U.sum(dim=(1, 2, 3)) * (prob.dx * prob.dy * prob.dz)


def run(prob: Problem, U: torch.Tensor, sigma: torch.Tensor, cfl: float,
        t_end: float, max_steps: int = 1_000_000):
    """Advance to t_end with the CFL rule, clipping the last step.
    Returns (U, sigma, t, steps)."""
    t, n = 0.0, 0
    while t < t_end and n < max_steps:
        dt = compute_dt(prob, U, cfl)
        if t + dt > t_end:
            dt = t_end - t
        U, sigma = rk3_step(prob, U, sigma, dt)
        t += dt
        n += 1
    return U, sigma, t, n


def to_tensor(a) -> torch.Tensor:
    return torch.as_tensor(a, dtype=torch.float64)

