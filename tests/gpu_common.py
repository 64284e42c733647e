"""Helpers for the GPU parity tests (HIP path through the C ABI vs the
FP64 oracle)."""

import numpy as np
import torch

from paper_2505_07392_amd import igr
from oracle import igr_ref as ref

TOL = 1e-12   # relative L-infinity per field, FP64


def rel_linf(got, want):
    """max|got - want| / max|want| per leading index (fields); a field that
    is identically zero in the oracle must be exactly zero."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if want.ndim == 3:
        got, want = got[None], want[None]
    out = []
    for g, w in zip(got, want):
        scale = np.abs(w).max()
        if scale == 0.0:
            out.append(0.0 if np.count_nonzero(g) == 0 else np.inf)
        else:
            out.append(float(np.abs(g - w).max() / scale))
    return np.array(out)


def to_host(solver, a):
    return solver.interior(a).double().cpu().numpy()


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)


def window(U, centre, R):
    """Periodic (2R+1)^3 window of an interior array [..., nz, ny, nx]."""
    k, j, i = centre
    nz, ny, nx = U.shape[-3:]
    iz = np.arange(k - R, k + R + 1) % nz
    iy = np.arange(j - R, j + R + 1) % ny
    ix = np.arange(i - R, i + R + 1) % nx
    return np.ascontiguousarray(U[..., iz[:, None, None], iy[None, :, None], ix[None, None, :]])
