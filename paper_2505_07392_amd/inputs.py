"""Seeded synthetic workloads for the IGR solver.

This module only *defines inputs*: grid, boundary description, inflow
discs, the seeded initial state and run lengths.  It holds none of the
solver's arithmetic and imports neither the HIP binding nor the oracle, so
both can be fed the same arrays.  Initial states are given as primitive
fields and turned into conserved variables with the ideal-gas law, which is
part of defining the input.

Workloads (all with gamma = 1.4 and alpha = 1 * dx^2):

``sod``            planar Sod tube along x, 128 x 16 x 16, extrapolation in x,
                   periodic in y and z, CFL 0.5 to t = 0.2, 5 sweeps; the
                   initial step is a tanh profile one cell wide.
``periodic_box``   256^3 periodic box: rho = 1 + 0.2 (G_4 * xi) with xi a
                   seeded standard normal per cell and G_4 a periodic
                   Gaussian of standard deviation 4 cells; solenoidal
                   velocity with random phases, shell spectrum E(k) ~ k^-2
                   for 1 <= |k| <= N/2 (k = 0 and Nyquist planes zeroed),
                   scaled to rms |u| = 1.5 sqrt(gamma) (rms Mach 1.5 at
                   p = rho = 1); p = 1; 5 sweeps; 100 steps.
``multi_jet``      n^3 box, ambient (rho, u, p) = (1, 0, 1); an m x m array of
                   circular inflow discs on the x-min face with centres at
                   ((a + 1/2) / m, (b + 1/2) / m) and radius r cells;
                   jet (rho, p) = (0.5, 8), u_x = Mach * sqrt(gamma p / rho)
                   times a seeded per-jet factor 1 + eps (2 xi - 1);
                   zero-gradient outflow on every other face.
``entropy_wave``   periodic density wave advected by a uniform velocity
                   (exact solution is a translation; Sigma stays zero).
``random_state``   iid bounded random fields for parity tests at small sizes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

PERIODIC = "periodic"
EXTRAP = "extrap"
GAMMA = 1.4


@dataclass
class Jet:
    """Inflow disc on the x-min face: centre (yc, zc), radius r (physical
    units) and the primitive jet state."""

    yc: float
    zc: float
    r: float
    rho: float
    ux: float
    uy: float
    uz: float
    p: float
    width: float = 0.0


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    U: np.ndarray                       # [5, nz, ny, nx] float64 conserved state
    gamma: float = GAMMA
    alpha: float = 0.0
    faces: Sequence[str] = (EXTRAP,) * 6  # -x, +x, -y, +y, -z, +z
    jets: List[Jet] = field(default_factory=list)
    nsweeps: int = 5
    cfl: float = 0.5
    t_end: Optional[float] = None
    nsteps: Optional[int] = None
    dt_fixed: Optional[float] = None
    seed: Optional[int] = None
    mu: float = 0.0                     # shear viscosity (0: the Euler system)
    zeta: float = 0.0                   # bulk viscosity

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def with_state(self, U: np.ndarray) -> "Workload":
        return replace(self, U=U)


def conserved(rho, ux, uy, uz, p, gamma=GAMMA) -> np.ndarray:
    """Stack primitive fields into the conserved state (ideal gas)."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    ux, uy, uz, p = (np.broadcast_to(np.asarray(a, dtype=np.float64), shape) for a in (ux, uy, uz, p))
    E = p / (gamma - 1.0) + 0.5 * rho * (ux * ux + uy * uy + uz * uz)
    return np.ascontiguousarray(np.stack([rho, rho * ux, rho * uy, rho * uz, E]))


def sod(nx: int = 128, ny: int = 16, nz: int = 16, nsweeps: int = 5,
        front_cells: float = 1.0) -> Workload:
    """Sod tube: (rho, u, p) = (1, 0, 1) left of x = 1/2, (0.125, 0, 0.1)
    right of it.  The step is a tanh profile of width ``front_cells`` cells
    (point values at cell centres): a sharp 10:1 energy jump would give
    negative face pressures under the unlimited fifth-order
    reconstruction before any regularisation acts."""
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    if front_cells > 0:
        chi = 0.5 * (1.0 - np.tanh((x - 0.5) / (front_cells * dx)))
    else:
        chi = (x < 0.5).astype(np.float64)
    shape = (nz, ny, nx)
    rho = np.broadcast_to(0.125 + 0.875 * chi, shape)
    p = np.broadcast_to(0.1 + 0.9 * chi, shape)
    U = conserved(rho, 0.0, 0.0, 0.0, p)
    return Workload("sod", nx, ny, nz, dx, dx, dx, U, alpha=dx * dx,
                    faces=(EXTRAP, EXTRAP, PERIODIC, PERIODIC, PERIODIC, PERIODIC),
                    nsweeps=nsweeps, cfl=0.5, t_end=0.2)


def _gaussian_smooth_periodic(xi: np.ndarray, sigma_cells: float) -> np.ndarray:
    """Periodic convolution with a unit-mass Gaussian of std sigma_cells."""
    n = xi.shape
    k = [np.fft.fftfreq(m) for m in n[:-1]] + [np.fft.rfftfreq(n[-1])]
    kz, ky, kx = np.meshgrid(*k, indexing="ij")
    filt = np.exp(-2.0 * math.pi ** 2 * sigma_cells ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    return np.fft.irfftn(np.fft.rfftn(xi) * filt, s=n, axes=(0, 1, 2))


def _solenoidal_velocity(n: int, rng: np.random.Generator, rms: float) -> np.ndarray:
    """Random solenoidal field, mode amplitude ~ |k|^-2 (shell spectrum
    ~ k^-2) for 1 <= |k| <= n/2, Nyquist planes and k = 0 removed."""
    kf = np.fft.fftfreq(n) * n
    kr = np.fft.rfftfreq(n) * n
    kz, ky, kx = np.meshgrid(kf, kf, kr, indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    shape = kk.shape
    amp = np.zeros(shape)
    band = (kk >= 1.0) & (kk <= n / 2)
    amp[band] = kk[band] ** -2.0
    nyq = (np.abs(kx) == n / 2) | (np.abs(ky) == n / 2) | (np.abs(kz) == n / 2)
    amp[nyq] = 0.0
    uh = [amp * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) for _ in range(3)]
    kvec = (kx, ky, kz)
    k2 = np.where(kk > 0, kk * kk, 1.0)
    kdotu = sum(kvec[i] * uh[i] for i in range(3))
    uh = [uh[i] - kvec[i] * kdotu / k2 for i in range(3)]
    u = np.stack([np.fft.irfftn(uh[i], s=(n, n, n), axes=(0, 1, 2)) for i in range(3)])
    scale = rms / math.sqrt(float(np.mean(np.sum(u * u, axis=0))))
    return u * scale


def periodic_box(n: int = 256, seed: int = 0, nsweeps: int = 5, nsteps: int = 100,
                 mach_rms: float = 1.5) -> Workload:
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((n, n, n))
    rho = 1.0 + 0.2 * _gaussian_smooth_periodic(xi, 4.0)
    u = _solenoidal_velocity(n, rng, mach_rms * math.sqrt(GAMMA))
    U = conserved(rho, u[0], u[1], u[2], 1.0)
    dx = 1.0 / n
    return Workload("periodic_box", n, n, n, dx, dx, dx, U, alpha=dx * dx,
                    faces=(PERIODIC,) * 6, nsweeps=nsweeps, nsteps=nsteps, seed=seed)


def _jet_blend(ny: int, nz: int, dx: float, jets: Sequence[Jet]):
    """Nearest-disc owner and tanh radial weight per (k, j) column."""
    yc = (np.arange(ny) + 0.5) * dx
    zc = (np.arange(nz) + 0.5) * dx
    best = np.full((nz, ny), np.inf)
    owner = np.full((nz, ny), -1)
    for q, j in enumerate(jets):
        d2 = (yc[None, :] - j.yc) ** 2 + (zc[:, None] - j.zc) ** 2
        closer = d2 < best
        best = np.where(closer, d2, best)
        owner = np.where(closer, q, owner)
    chi = np.zeros((nz, ny))
    for q, j in enumerate(jets):
        if j.width > 0:
            w = 0.5 * (1.0 - np.tanh((np.sqrt(best) - j.r) / j.width))
        else:
            w = (best <= j.r ** 2).astype(np.float64)
        chi = np.where(owner == q, w, chi)
    return owner, chi


def multi_jet(n: int = 512, jets_per_side: int = 4, radius_cells: float = 10.0,
              mach: float = 3.0, seed: int = 0, perturb: float = 0.05,
              nsweeps: int = 10, nsteps: int = 200, nx: Optional[int] = None,
              dt_fixed: Optional[float] = None, edge_cells: float = 2.0,
              plug_cells: float = 12.0, front_cells: Optional[float] = 6.0,
              name: str = "multi_jet", build_state: bool = True) -> Workload:
    """Array of supersonic inflow discs into a quiescent box (unit y/z extent).

    Each disc edge is a tanh profile of width ``edge_cells``; the initial
    state carries a plug of jet fluid in front of every disc (tanh front at
    ``plug_cells`` from the inlet, width ``front_cells``), so that neither
    the disc edge nor the inlet starts as a jump that the unlimited
    fifth-order reconstruction would turn into negative face pressures.
    With ``build_state=False`` the state is left out (``U is None``); fill a
    device array plane by plane with :func:`fill_multi_jet_state`."""
    ny = nz = n
    nx = n if nx is None else nx
    dx = 1.0 / n
    rng = np.random.default_rng(seed)
    rho_j, p_j = 0.5, 8.0
    u0 = mach * math.sqrt(GAMMA * p_j / rho_j)
    width = edge_cells * dx
    jets = []
    for b in range(jets_per_side):
        for a in range(jets_per_side):
            factor = 1.0 + perturb * (2.0 * rng.random() - 1.0) if perturb else 1.0
            jets.append(Jet(yc=(a + 0.5) / jets_per_side, zc=(b + 0.5) / jets_per_side,
                            r=radius_cells * dx, rho=rho_j, ux=u0 * factor, uy=0.0, uz=0.0,
                            p=p_j, width=width))
    w = Workload(name, nx, ny, nz, dx, dx, dx, None, alpha=dx * dx,
                 faces=(EXTRAP,) * 6, jets=jets, nsweeps=nsweeps, nsteps=nsteps,
                 dt_fixed=dt_fixed, seed=seed)
    w.plug = (plug_cells * dx, (edge_cells if front_cells is None else front_cells) * dx)
    if build_state:
        owner, chi_r = _jet_blend(ny, nz, dx, jets)
        chi_x = _plug_profile(nx, dx, *w.plug)
        chi = chi_r[:, :, None] * chi_x[None, None, :]
        amb = conserved(np.ones((nz, ny, nx)), 0.0, 0.0, 0.0, 1.0)
        jet_state = np.stack([conserved(j.rho, j.ux, j.uy, j.uz, j.p) for j in jets])  # [J, 5]
        Uj = np.moveaxis(jet_state[owner], -1, 0)[:, :, :, None]          # [5, nz, ny, 1]
        w.U = np.ascontiguousarray((1.0 - chi)[None] * amb + chi[None] * Uj)
    return w


def _plug_profile(nx: int, dx: float, plug: float, front: float) -> np.ndarray:
    x = (np.arange(nx) + 0.5) * dx
    if front > 0:
        return 0.5 * (1.0 - np.tanh((x - plug) / front))
    return (x <= plug).astype(np.float64)


def fill_multi_jet_state(w: Workload, out) -> None:
    """Write the multi-jet initial state (same definition as multi_jet's U)
    into ``out``, a torch tensor view [5, nz, ny, nx] on any device and of
    any dtype, one z plane at a time (for grids too large to build on the
    host)."""
    import torch

    owner, chi_r = _jet_blend(w.ny, w.nz, w.dx, w.jets)
    chi_x = torch.as_tensor(_plug_profile(w.nx, w.dx, *w.plug), device=out.device)
    amb = torch.as_tensor(conserved(1.0, 0.0, 0.0, 0.0, 1.0), device=out.device).reshape(5, 1, 1)
    jet_state = torch.as_tensor(np.stack([conserved(j.rho, j.ux, j.uy, j.uz, j.p) for j in w.jets]),
                                device=out.device)                                    # [J, 5]
    for k in range(w.nz):
        chi = torch.as_tensor(chi_r[k], device=out.device)[:, None] * chi_x[None, :]   # [ny, nx]
        Uj = jet_state[torch.as_tensor(owner[k], device=out.device)].T[:, :, None]    # [5, ny, 1]
        out[:, k].copy_(((1.0 - chi)[None] * amb + chi[None] * Uj).to(out.dtype))


def multi_jet_state_at(w: Workload, kk: Sequence[int], jj: Sequence[int], ii: Sequence[int]) -> np.ndarray:
    """The multi-jet initial state (same definition as multi_jet's U) at the
    cells kk x jj x ii (interior indices), as a float64 array
    [5, len(kk), len(jj), len(ii)]: a block of a grid too large to build
    whole on the host."""
    owner, chi_r = _jet_blend(w.ny, w.nz, w.dx, w.jets)
    kk, jj, ii = (np.asarray(a, dtype=np.int64) for a in (kk, jj, ii))
    chi_x = _plug_profile(w.nx, w.dx, *w.plug)[ii]
    chi = chi_r[kk[:, None], jj[None, :]][:, :, None] * chi_x[None, None, :]
    amb = conserved(1.0, 0.0, 0.0, 0.0, 1.0).reshape(5, 1, 1, 1)
    jet_state = np.stack([conserved(j.rho, j.ux, j.uy, j.uz, j.p) for j in w.jets])        # [J, 5]
    Uj = np.moveaxis(jet_state[owner[kk[:, None], jj[None, :]]], -1, 0)[:, :, :, None]   # [5, K, J, 1]
    return np.ascontiguousarray((1.0 - chi)[None] * amb + chi[None] * Uj)


def gradient_jets(n: int = 128) -> Workload:
    """2 x 2 Mach-2 discs of radius 6 cells, no perturbation, fixed dt from
    the inflow and ambient signal speeds at CFL 0.5 (sum rule)."""
    w = multi_jet(n=n, jets_per_side=2, radius_cells=6.0, mach=2.0, perturb=0.0,
                  nsweeps=5, nsteps=40, name="gradient_jets")
    j = w.jets[0]
    c_j = math.sqrt(GAMMA * j.p / j.rho)
    speed = (abs(j.ux) + c_j) / w.dx + 2.0 * c_j / w.dx
    w.dt_fixed = 0.5 / speed
    return w


def entropy_wave(n: int, amp: float = 0.2, u=(1.0, 0.0, 0.0), ny: int = 1, nz: int = 1) -> Workload:
    """rho = 1 + amp sin(2 pi x) as exact cell averages, uniform u and p = 1."""
    dx = 1.0 / n
    xc = (np.arange(n) + 0.5) * dx
    k = 2.0 * math.pi
    avg = np.sin(k * xc) * (math.sin(k * dx / 2) / (k * dx / 2))
    rho = np.broadcast_to(1.0 + amp * avg, (nz, ny, n)).copy()
    U = conserved(rho, u[0], u[1], u[2], 1.0)
    return Workload("entropy_wave", n, ny, nz, dx, dx, dx, U, alpha=dx * dx,
                    faces=(PERIODIC,) * 6)


def random_state(nx: int, ny: int, nz: int, seed: int, amp: float = 0.3,
                 umax: float = 0.5) -> np.ndarray:
    """iid bounded primitive fields (rho, p in [1-amp, 1+amp], |u_i| <= umax)."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = 1.0 + amp * (2.0 * rng.random(shape) - 1.0)
    p = 1.0 + amp * (2.0 * rng.random(shape) - 1.0)
    u = umax * (2.0 * rng.random((3,) + shape) - 1.0)
    return conserved(rho, u[0], u[1], u[2], p)
