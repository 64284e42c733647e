"""ctypes binding of libigr (C ABI in include/igr.h).

Argument marshalling only: every step of the solver runs in the HIP
library.  PyTorch provides device memory (padded tensors) and the stream
(``torch.cuda.current_stream()``); the library is loaded from this package
directory and a missing library raises immediately, there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import torch

G = 3
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigr.so")

IGR_OK, IGR_EINVAL, IGR_ENOMEM, IGR_EHIP, IGR_ENONFINITE, IGR_EUNSUPPORTED = range(6)
BC_KIND = {"periodic": 0, "extrap": 1}
PRECISION = {"f64": (0, torch.float64), "f32": (1, torch.float32), "bf16": (2, torch.bfloat16),
             "f16": (3, torch.float16), "bf16d": (4, torch.float32)}
# Sigma's element type where it differs from the state's: the split form
# (FP32 state, bfloat16 stage differences and Sigma)
SIGMA_DTYPE = {"bf16d": torch.bfloat16}
SMOOTHER = {"jacobi": 0, "rbgs": 1}


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class Patch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("yc", "zc", "r", "width", "rho", "ux", "uy", "uz", "p")]


class BC(ctypes.Structure):
    _fields_ = [("face", ctypes.c_int32 * 6), ("npatch", ctypes.c_int32), ("patch", ctypes.POINTER(Patch))]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("nsweeps", ctypes.c_int32), ("sigma_block", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("mu", ctypes.c_double), ("zeta", ctypes.c_double)]


class IGRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libigr error {code}: {msg}")
        self.code = code


class NonFiniteError(IGRError):
    pass


_lib = None

_SIGNATURES = {
    "igr_init": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.c_double, ctypes.c_double, ctypes.POINTER(BC),
                                ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_void_p)]),
    "igr_finalize": (ctypes.c_int, [ctypes.c_void_p]),
    "igr_last_error": (ctypes.c_char_p, []),
    "igr_field_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "igr_get_opts": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Opts)]),
    "igr_set_patch_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_void_p]),
    "igr_sigma_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_rhs": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "igr_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_rhs_adjoint": (ctypes.c_int, [ctypes.c_void_p] * 7 + [ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_step_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_compute_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_sums": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_compute_dt_noalloc": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "igr_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "igr_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "igr_kernel_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "igr_kernel_name": (ctypes.c_char_p, [ctypes.c_int32]),
}


def lib() -> ctypes.CDLL:
    """Load libigr.so from the package directory (raises if not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_07392_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != IGR_OK:
        msg = lib().igr_last_error().decode()
        raise (NonFiniteError if rc == IGR_ENONFINITE else IGRError)(rc, msg)


def kernel_names() -> list:
    out, i = [], 0
    while True:
        n = lib().igr_kernel_name(i)
        if not n:
            return out
        out.append(n.decode())
        i += 1


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One libigr context: grid, boundary description, precision, sweeps."""

    def __init__(self, nx: int, ny: int, nz: int, dx: float, dy: float, dz: float, *, gamma: float = 1.4,
                 alpha: float = 0.0, faces: Sequence[str] = ("extrap",) * 6, jets: Iterable = (),
                 nsweeps: int = 5, precision: str = "f64", sigma_block: int = 0, order: int = 5,
                 smoother: str = "jacobi", mu: float = 0.0, zeta: float = 0.0, device=None):
        if precision not in PRECISION:
            raise ValueError(f"precision must be one of {list(PRECISION)}")
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dx, self.dy, self.dz = dx, dy, dz
        self.gamma, self.alpha, self.nsweeps = gamma, alpha, nsweeps
        self.precision = precision
        self.dtype = PRECISION[precision][1]
        self.sigma_dtype = SIGMA_DTYPE.get(precision, self.dtype)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.shape = (nz + 2 * G, ny + 2 * G, nx + 2 * G)
        jets = list(jets)
        self.npatch = len(jets)
        self.jets = [[j.rho, j.ux, j.uy, j.uz, j.p] for j in jets]
        self._patches = (Patch * max(1, len(jets)))()
        for i, j in enumerate(jets):
            self._patches[i] = Patch(j.yc, j.zc, j.r, getattr(j, "width", 0.0), j.rho, j.ux, j.uy, j.uz, j.p)
        bc = BC((ctypes.c_int32 * 6)(*[BC_KIND[f] for f in faces]), len(jets), self._patches)
        if smoother not in SMOOTHER:
            raise ValueError(f"smoother must be one of {list(SMOOTHER)}")
        self.order, self.smoother = order, smoother
        self.mu, self.zeta = mu, zeta
        opts = Opts(PRECISION[precision][0], order, nsweeps, sigma_block, SMOOTHER[smoother], mu, zeta)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().igr_init(ctypes.byref(Grid(nx, ny, nz, dx, dy, dz)), gamma, alpha, ctypes.byref(bc),
                                  ctypes.byref(opts), ctypes.byref(handle)))
        self._ctx = handle
        eff = Opts()
        _check(lib().igr_get_opts(self._ctx, ctypes.byref(eff)))
        self.sigma_block = eff.sigma_block   # the pass structure the library runs (default resolved)

    @classmethod
    def from_workload(cls, w, precision: str = "f64", nsweeps: Optional[int] = None, sigma_block: int = 0,
                      order: int = 5, smoother: str = "jacobi", device=None) -> "Solver":
        return cls(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, gamma=w.gamma, alpha=w.alpha, faces=tuple(w.faces),
                   jets=w.jets, nsweeps=w.nsweeps if nsweeps is None else nsweeps, precision=precision,
                   sigma_block=sigma_block, order=order, smoother=smoother, mu=getattr(w, "mu", 0.0),
                   zeta=getattr(w, "zeta", 0.0), device=device)

    # -- memory ------------------------------------------------------------
    def new_state(self) -> torch.Tensor:
        return torch.zeros((5,) + self.shape, dtype=self.dtype, device=self.device)

    def new_field(self) -> torch.Tensor:
        """A padded Sigma field (Sigma's element type)."""
        return torch.zeros(self.shape, dtype=self.sigma_dtype, device=self.device)

    @staticmethod
    def interior(a: torch.Tensor) -> torch.Tensor:
        return a[..., G:-G, G:-G, G:-G]

    def state_from(self, U) -> torch.Tensor:
        """Padded device state from an interior array [5, nz, ny, nx]."""
        out = self.new_state()
        self.interior(out).copy_(torch.as_tensor(U).to(dtype=torch.float64).to(self.dtype))
        return out

    def field_from(self, S) -> torch.Tensor:
        out = self.new_field()
        self.interior(out).copy_(torch.as_tensor(S).to(dtype=torch.float64).to(self.sigma_dtype))
        return out

    def _validate(self, t: torch.Tensor, nfields: int, name: str):
        shape = ((nfields,) if nfields > 1 else ()) + self.shape
        dtype = self.dtype if nfields > 1 else self.sigma_dtype
        if tuple(t.shape) != shape or t.dtype != dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous {dtype} tensor of shape {shape} on {self.device}, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # -- solver calls --------------------------------------------------------
    def sigma_solve(self, U: torch.Tensor, sigma: torch.Tensor, nsweeps: Optional[int] = None,
                    residual: bool = False) -> Optional[float]:
        self._validate(U, 5, "U")
        self._validate(sigma, 1, "sigma")
        r = ctypes.c_double(0.0)
        _check(lib().igr_sigma_solve(self._ctx, _ptr(U), _ptr(sigma),
                                     self.nsweeps if nsweeps is None else nsweeps,
                                     ctypes.byref(r) if residual else None, self._stream()))
        return r.value if residual else None

    def rhs(self, U: torch.Tensor, sigma: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._validate(U, 5, "U")
        self._validate(sigma, 1, "sigma")
        out = self.new_state() if out is None else out
        self._validate(out, 5, "rhs")
        _check(lib().igr_rhs(self._ctx, _ptr(U), _ptr(sigma), _ptr(out), self._stream()))
        return out

    def step(self, U: torch.Tensor, sigma: torch.Tensor, cfl: float = 0.5, dt_fixed: float = 0.0,
             sync: bool = True) -> Optional[float]:
        """One SSP-RK3 step in place; returns dt (and checks the non-finite
        flag) when sync is True."""
        self._validate(U, 5, "U")
        self._validate(sigma, 1, "sigma")
        dt = ctypes.c_double(0.0)
        _check(lib().igr_step(self._ctx, _ptr(U), _ptr(sigma), cfl, dt_fixed,
                              ctypes.byref(dt) if sync else None, self._stream()))
        return dt.value if sync else None

    def advance(self, U: torch.Tensor, sigma: torch.Tensor, nsteps: int, cfl: float = 0.5, dt_fixed: float = 0.0,
                sync: bool = True) -> Optional[float]:
        """nsteps SSP-RK3 steps in place (each later step's CFL maximum is
        fused into the previous step's last stage); returns the last dt (and
        checks the non-finite flag) when sync is True."""
        self._validate(U, 5, "U")
        self._validate(sigma, 1, "sigma")
        dt = ctypes.c_double(0.0)
        _check(lib().igr_advance(self._ctx, _ptr(U), _ptr(sigma), int(nsteps), cfl, dt_fixed,
                                 ctypes.byref(dt) if sync else None, self._stream()))
        return dt.value if sync else None

    def rhs_adjoint(self, U, sigma_prev, rhs_bar, sigma_bar):
        """Cotangents (U_bar, sigma_prev_bar, patch_bar [npatch, 5]) of one
        right-hand side given (rhs_bar, sigma_bar)."""
        for t, n, name in ((U, 5, "U"), (sigma_prev, 1, "sigma_prev"), (rhs_bar, 5, "rhs_bar"),
                           (sigma_bar, 1, "sigma_bar")):
            self._validate(t, n, name)
        Ub, Sb = self.new_state(), self.new_field()
        npatch = max(1, self.npatch)
        pb = (ctypes.c_double * (5 * npatch))()
        _check(lib().igr_rhs_adjoint(self._ctx, _ptr(U), _ptr(sigma_prev), _ptr(rhs_bar), _ptr(sigma_bar),
                                     _ptr(Ub), _ptr(Sb), pb, self._stream()))
        return Ub, Sb, torch.tensor(list(pb), dtype=torch.float64).reshape(npatch, 5)[: self.npatch]

    def step_adjoint(self, U_n, sigma_n, dt: float, U_bar, sigma_bar):
        """Cotangents (U_bar_n, sigma_bar_n, patch_bar [npatch, 5]) of one
        fixed-dt step given the cotangents of its output."""
        for t, n, name in ((U_n, 5, "U_n"), (sigma_n, 1, "sigma_n"), (U_bar, 5, "U_bar"), (sigma_bar, 1, "sigma_bar")):
            self._validate(t, n, name)
        Ub, Sb = self.new_state(), self.new_field()
        npatch = max(1, self.npatch)
        pb = (ctypes.c_double * (5 * npatch))()
        _check(lib().igr_step_adjoint(self._ctx, _ptr(U_n), _ptr(sigma_n), dt, _ptr(U_bar), _ptr(sigma_bar),
                                      _ptr(Ub), _ptr(Sb), pb, self._stream()))
        return Ub, Sb, torch.tensor(list(pb), dtype=torch.float64).reshape(npatch, 5)[: self.npatch]

    def compute_dt(self, U: torch.Tensor, cfl: float) -> float:
        self._validate(U, 5, "U")
        dt = ctypes.c_double(0.0)
        _check(lib().igr_compute_dt(self._ctx, _ptr(U), cfl, ctypes.byref(dt), self._stream()))
        return dt.value

    def sums(self, U: torch.Tensor) -> list:
        self._validate(U, 5, "U")
        out = (ctypes.c_double * 5)()
        _check(lib().igr_sums(self._ctx, _ptr(U), out, self._stream()))
        return list(out)

    def check(self):
        _check(lib().igr_check(self._ctx, self._stream()))

    def set_jet_state(self, index: int, rho: float, ux: float, uy: float, uz: float, p: float):
        prim = (ctypes.c_double * 5)(rho, ux, uy, uz, p)
        _check(lib().igr_set_patch_state(self._ctx, index, prim, self._stream()))
        self.jets[index] = [rho, ux, uy, uz, p]

    def timing(self, enable: bool):
        _check(lib().igr_timing(self._ctx, 1 if enable else 0))

    def kernel_time(self, name: str):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib().igr_kernel_time(self._ctx, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def run(self, U, sigma, cfl: float, t_end: float, max_steps: int = 10 ** 7):
        """Advance to t_end with the CFL rule, clipping the last step.
        Returns (t, steps)."""
        t, n = 0.0, 0
        while t < t_end and n < max_steps:
            dt = self.compute_dt(U, cfl)          # the one synchronising call per step
            if t + dt > t_end:
                dt = t_end - t
            self.step(U, sigma, dt_fixed=dt, sync=False)
            t += dt
            n += 1
        self.check()
        return t, n

    def close(self):
        if getattr(self, "_ctx", None):
            lib().igr_finalize(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
