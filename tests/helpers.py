"""Shared test helpers: turn a synthetic workload into the oracle's problem
description (the oracle never imports the product package)."""

import torch

from oracle import igr_ref as ref


def problem_from(w, nsweeps=None, alpha=None, order=5):
    patches = tuple(ref.Patch(j.yc, j.zc, j.r, j.rho, j.ux, j.uy, j.uz, j.p, j.width) for j in w.jets)
    return ref.Problem(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, gamma=w.gamma,
                       alpha=w.alpha if alpha is None else alpha, faces=tuple(w.faces),
                       patches=patches, nsweeps=w.nsweeps if nsweeps is None else nsweeps, order=order,
                       mu=getattr(w, "mu", 0.0), zeta=getattr(w, "zeta", 0.0))


def state_of(w):
    return torch.from_numpy(w.U.copy())
