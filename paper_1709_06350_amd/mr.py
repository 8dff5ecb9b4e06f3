"""Thin ctypes binding of libmr.so (include/mr.h). Argument marshalling only.

Every computation runs in the HIP library; this module converts torch CUDA tensors (float64,
contiguous, on the current device) to raw device pointers and passes the current torch stream.
It never falls back to another implementation: if libmr.so is missing or a call fails, it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmr.so")

MR_OK = 0
MR_NOT_CONVERGED = 1
MR_EINVAL = -1
MR_EDOMAIN = -2
MR_EDIVERGED = -3
MR_EHIP = -4
MR_ENOMEM = -5
MR_FLAG_EAGER = 1
MR_FLAG_TWO_PASS = 2
MR_FLAG_ADJ_ROWS = 4
MR_FLAG_ADJ_TILED = 8
MR_FLAG_ORDER4 = 16
MR_FLAG_ANDERSON = 32
MR_FLAG_PLAIN_INNER = 64
MR_FLAG_DEPOSIT_SCATTER = 128
PREC_FP64 = 0
PREC_MIXED = 1
MR_SCHED_TILED = 0
MR_SCHED_PIPELINED = 1
MR_SCHED_FUSED = 2
MR_STREAM_COPY = 0
MR_STREAM_READ = 1
MR_STREAM_TRIAD = 2
MR_DEPOSIT_NGP = 0
MR_DEPOSIT_CIC = 1
MR_DEPOSIT_TSC = 2
DEPOSIT_SCHEMES = {"ngp": MR_DEPOSIT_NGP, "cic": MR_DEPOSIT_CIC, "tsc": MR_DEPOSIT_TSC}

EXPORTED = [
    "mr_default_opts", "mr_create", "mr_destroy", "mr_set_opts", "mr_size", "mr_levels",
    "mr_get_schedule", "mr_set_schedule", "mr_schedule_candidates", "mr_get_lin_schedule",
    "mr_deposit", "mr_deposit_cic", "mr_lagrangian", "mr_residual", "mr_solve", "mr_solve_anderson", "mr_adjoint_solve", "mr_adjoint_solve_anderson", "mr_solve_batched",
    "mr_batch_create", "mr_batch_solve", "mr_batch_destroy",
    "mr_tune_lin_tiles",
    "mr_sweep", "mr_defect_restrict", "mr_tau_rhs", "mr_prolong_correct", "mr_restrict",
    "mr_lin_residual", "mr_lin_defect_restrict", "mr_lin_vcycles", "mr_lin_sweep", "mr_lin_prolong_add",
    "mr_timing_enable", "mr_timing_read", "mr_hbm_stream", "mr_residual_noalloc",
    "mr_tuning_file", "mr_tuning_file_path", "mr_tuning_store", "mr_tuning_lookup", "mr_last_error",
]


class mr_opts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_cycles", ctypes.c_int),
        ("npre", ctypes.c_int),
        ("npost", ctypes.c_int),
        ("ncoarse", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("warm_start", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]


class mr_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("cycles", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("r0_norm", ctypes.c_double),
        ("m_shift", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("history", ctypes.c_double * 128),
        ("inner_cycles", ctypes.c_int),
    ]


class mr_timing(ctypes.Structure):
    _fields_ = [
        ("sweep64_ms", ctypes.c_double),
        ("sweep64_launches", ctypes.c_int64),
        ("sweep32_ms", ctypes.c_double),
        ("sweep32_launches", ctypes.c_int64),
        ("finest_cells", ctypes.c_int64),
    ]


class MRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmr error {code}: {msg}")
        self.code = code


_lib = None


def load(path: Optional[str] = None):
    """Load libmr.so (built by paper_1709_06350_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python -m paper_1709_06350_amd.build` "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    lib = ctypes.CDLL(p)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.mr_default_opts.argtypes = [ctypes.POINTER(mr_opts)]
    lib.mr_default_opts.restype = None
    lib.mr_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(mr_opts), vp]
    lib.mr_destroy.argtypes = [vp]
    lib.mr_destroy.restype = None
    lib.mr_set_opts.argtypes = [vp, ctypes.POINTER(mr_opts)]
    lib.mr_size.argtypes = [vp]
    lib.mr_levels.argtypes = [vp]
    lib.mr_lagrangian.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp]
    lib.mr_get_schedule.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.mr_set_schedule.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.mr_schedule_candidates.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int), ip]
    lib.mr_deposit_cic.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, vp]
    lib.mr_deposit.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int, vp]
    lib.mr_residual.argtypes = [vp, vp, vp, vp, dp, dp]
    lib.mr_solve.argtypes = [vp, vp, vp, ctypes.POINTER(mr_info)]
    lib.mr_solve_anderson.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(mr_info)]
    lib.mr_adjoint_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(mr_info)]
    lib.mr_adjoint_solve_anderson.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(mr_info)]
    lib.mr_solve_batched.argtypes = [ip, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), ctypes.POINTER(mr_opts),
                                     ctypes.POINTER(mr_info), vp]
    lib.mr_batch_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(mr_opts), vp]
    lib.mr_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(mr_info)]
    lib.mr_batch_destroy.argtypes = [vp]
    lib.mr_tune_lin_tiles.argtypes = [ip, vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
    lib.mr_sweep.argtypes = [vp, ip, ctypes.c_double, vp, vp, ctypes.c_double, vp, vp, dp]
    lib.mr_defect_restrict.argtypes = [vp, ip, ctypes.c_double, vp, vp, ctypes.c_double, vp, vp, vp]
    lib.mr_tau_rhs.argtypes = [vp, ip, ctypes.c_double, vp, vp, vp, vp, dp]
    lib.mr_prolong_correct.argtypes = [vp, ip, vp, vp, vp]
    lib.mr_restrict.argtypes = [vp, ip, vp, vp]
    lib.mr_lin_residual.argtypes = [vp, ip, ctypes.c_double, vp, vp, vp, vp, ctypes.c_double, vp]
    lib.mr_lin_defect_restrict.argtypes = [vp, ip, ctypes.c_double, vp, vp, vp, vp, ctypes.c_double, vp]
    lib.mr_lin_vcycles.argtypes = [vp, vp, vp, vp, ip, vp]
    lib.mr_lin_sweep.argtypes = [vp, ip, ctypes.c_double, vp, vp, vp, vp, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_int), vp]
    lib.mr_lin_prolong_add.argtypes = [vp, ip, vp, vp, vp]
    lib.mr_timing_enable.argtypes = [vp, ip]
    lib.mr_timing_read.argtypes = [vp, ctypes.POINTER(mr_timing)]
    lib.mr_hbm_stream.argtypes = [ip, ip, vp, vp, vp, ctypes.c_size_t, ip, vp, ctypes.POINTER(ctypes.c_float)]
    lib.mr_residual_noalloc.argtypes = [ip, vp, vp, vp, dp, dp, vp]
    lib.mr_get_lin_schedule.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.mr_tuning_file.argtypes = [ctypes.c_char_p]
    lib.mr_tuning_file_path.argtypes = []
    lib.mr_tuning_file_path.restype = ctypes.c_char_p
    cp = ctypes.c_char_p
    lib.mr_tuning_store.argtypes = [cp, cp, cp, ip, ip, ctypes.POINTER(ctypes.c_int), ip]
    lib.mr_tuning_lookup.argtypes = [cp, cp, cp, ip, ip, ctypes.POINTER(ctypes.c_int), ip,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.mr_last_error.argtypes = []
    lib.mr_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("mr_default_opts", "mr_destroy", "mr_last_error", "mr_tuning_file_path"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code: int, allow=(MR_OK,)):
    if code not in allow:
        raise MRError(code, load().mr_last_error().decode())
    return code


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _need(t: Optional[torch.Tensor], count: int, what: str):
    """Host-side size check: the kernels index the buffers by the mesh and particle counts."""
    if t is not None and t.numel() != count:
        raise ValueError(f"{what}: expected {count} values, got {t.numel()}")


def _particles(pos: torch.Tensor) -> int:
    if pos.numel() % 3 != 0:
        raise ValueError("pos: expected np x 3 coordinates")
    return pos.numel() // 3


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw) -> mr_opts:
    o = mr_opts()
    load().mr_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class Info:
    status: int
    cycles: int
    rel_residual: float
    r0_norm: float
    m_shift: float
    seconds: float
    history: List[float] = field(default_factory=list)
    inner_cycles: int = 0

    @staticmethod
    def from_c(i: mr_info) -> "Info":
        return Info(i.status, i.cycles, i.rel_residual, i.r0_norm, i.m_shift, i.seconds,
                    list(i.history[: min(i.cycles, 127) + 1]), i.inner_cycles)


class Context:
    """An mr_ctx for n^3 meshes bound to the current torch stream."""

    def __init__(self, n: int, **opts):
        self.lib = load()
        self.n = n
        self.opts = default_opts(**opts)
        h = ctypes.c_void_p()
        _check(self.lib.mr_create(ctypes.byref(h), n, ctypes.byref(self.opts), _stream()))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.mr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def levels(self) -> int:
        return self.lib.mr_levels(self.h)

    def get_schedule(self, level: int = 0):
        """FP64 relaxation schedule of a level (mr_get_schedule): (kind, tm, tj, nchunks)."""
        a = (ctypes.c_int * 4)()
        _check(self.lib.mr_get_schedule(self.h, level, a))
        return tuple(a)

    def set_schedule(self, level: int, sched):
        """Pin a level's FP64 relaxation schedule (mr_set_schedule); sched = (kind, tm, tj, nchunks)."""
        a = (ctypes.c_int * 4)(*sched)
        _check(self.lib.mr_set_schedule(self.h, level, a))

    def get_lin_schedule(self, level: int = 0):
        """FP32 sweep schedule of the mixed form on a level (mr_get_lin_schedule): (kind, tm, tj, nchunks)."""
        a = (ctypes.c_int * 4)()
        _check(self.lib.mr_get_lin_schedule(self.h, level, a))
        return tuple(a)

    def schedule_candidates(self, level: int = 0):
        """Every schedule the tuner times for a level (mr_schedule_candidates), as (kind, tm, tj, nchunks)."""
        count = self.lib.mr_schedule_candidates(self.h, level, None, 0)
        _check(min(count, 0))
        a = (ctypes.c_int * (4 * max(count, 1)))()
        _check(min(self.lib.mr_schedule_candidates(self.h, level, a, count), 0))
        return [tuple(a[4 * i:4 * i + 4]) for i in range(count)]

    def _empty(self, n=None):
        n = self.n if n is None else n
        return torch.empty((n, n, n), dtype=torch.float64, device="cuda")

    # -- the four calls of the path ----------------------------------------------------------
    def deposit(self, pos: torch.Tensor, mass: float = 1.0, scheme: str = "cic",
                out: Optional[torch.Tensor] = None):
        """Density assignment (mr_deposit) with scheme "ngp", "cic" or "tsc"; returns delta."""
        if scheme not in DEPOSIT_SCHEMES:
            raise ValueError(f"unknown scheme {scheme!r}")
        out = self._empty() if out is None else out
        npart = _particles(pos)
        _need(out, self.n ** 3, "out")
        _check(self.lib.mr_deposit(self.h, _ptr(pos), npart, mass, DEPOSIT_SCHEMES[scheme], _ptr(out)))
        return out

    def deposit_cic(self, pos: torch.Tensor, mass: float = 1.0, out: Optional[torch.Tensor] = None):
        out = self._empty() if out is None else out
        npart = _particles(pos)
        _need(out, self.n ** 3, "out")
        _check(self.lib.mr_deposit_cic(self.h, _ptr(pos), npart, mass, _ptr(out)))
        return out

    def lagrangian(self, theta: torch.Tensor, pos: torch.Tensor, want_psi: bool = False, out=None):
        """Lagrangian mapping (mr_lagrangian): per-particle displacement psi(x_p) (np x 3, so that
        q = pos + disp) and, if want_psi, the mesh field psi (n x n x n x 3)."""
        npart = _particles(pos)
        _need(theta, self.n ** 3, "theta")
        disp = torch.empty((npart, 3), dtype=torch.float64, device="cuda") if out is None else out
        _need(disp, 3 * npart, "out")
        psi = torch.empty((self.n, self.n, self.n, 3), dtype=torch.float64, device="cuda") if want_psi else None
        _check(self.lib.mr_lagrangian(self.h, _ptr(theta), _ptr(pos), npart, _ptr(disp), _ptr(psi)))
        return disp, psi

    def residual(self, delta: torch.Tensor, theta: torch.Tensor, want_r: bool = True):
        r = self._empty() if want_r else None
        _need(delta, self.n ** 3, "delta")
        _need(theta, self.n ** 3, "theta")
        rel = ctypes.c_double()
        ms = ctypes.c_double()
        _check(self.lib.mr_residual(self.h, _ptr(delta), _ptr(theta), _ptr(r), ctypes.byref(rel),
                                    ctypes.byref(ms)))
        return r, rel.value, ms.value

    def solve(self, delta: torch.Tensor, theta: Optional[torch.Tensor] = None, check: bool = True):
        theta = torch.zeros_like(delta) if theta is None else theta
        _need(delta, self.n ** 3, "delta")
        _need(theta, self.n ** 3, "theta")
        info = mr_info()
        code = self.lib.mr_solve(self.h, _ptr(delta), _ptr(theta), ctypes.byref(info))
        if check:
            _check(code)
        return theta, Info.from_c(info)

    def solve_anderson(self, delta: torch.Tensor, theta: Optional[torch.Tensor] = None, depth: int = 6,
                       check: bool = True):
        """FP64 solve with Anderson-accelerated V-cycles (mr_solve_anderson)."""
        theta = torch.zeros_like(delta) if theta is None else theta
        _need(delta, self.n ** 3, "delta")
        _need(theta, self.n ** 3, "theta")
        info = mr_info()
        code = self.lib.mr_solve_anderson(self.h, _ptr(delta), _ptr(theta), depth, ctypes.byref(info))
        if check:
            _check(code)
        return theta, Info.from_c(info)

    def set_opts(self, **kw):
        """Change solver options of this context (mr_set_opts); keywords are mr_opts fields."""
        for k, v in kw.items():
            if not hasattr(self.opts, k):
                raise KeyError(k)
            setattr(self.opts, k, v)
        _check(self.lib.mr_set_opts(self.h, ctypes.byref(self.opts)))

    def adjoint_solve(self, delta, theta_star, g, out=None, check: bool = True, anderson_depth: int = 0):
        """dL/ddelta (mr_adjoint_solve, or mr_adjoint_solve_anderson when anderson_depth > 0)."""
        out = self._empty() if out is None else out
        for t, what in ((delta, "delta"), (theta_star, "theta_star"), (g, "g"), (out, "out")):
            _need(t, self.n ** 3, what)
        info = mr_info()
        if anderson_depth > 0:
            code = self.lib.mr_adjoint_solve_anderson(self.h, _ptr(delta), _ptr(theta_star), _ptr(g), _ptr(out),
                                                      anderson_depth, ctypes.byref(info))
        else:
            code = self.lib.mr_adjoint_solve(self.h, _ptr(delta), _ptr(theta_star), _ptr(g), _ptr(out),
                                             ctypes.byref(info))
        if check:
            _check(code)
        return out, Info.from_c(info)

    def timing_enable(self, on: bool = True):
        _check(self.lib.mr_timing_enable(self.h, 1 if on else 0))

    def timing_read(self) -> dict:
        t = mr_timing()
        _check(self.lib.mr_timing_read(self.h, ctypes.byref(t)))
        return dict(sweep64_ms=t.sweep64_ms, sweep64_launches=t.sweep64_launches,
                    sweep32_ms=t.sweep32_ms, sweep32_launches=t.sweep32_launches,
                    finest_cells=t.finest_cells)

    # -- building blocks ---------------------------------------------------------------------
    def sweep(self, delta, theta_in, h=1.0, f=None, cshift=0.0, out=None):
        nl = theta_in.shape[0]
        out = self._empty(nl) if out is None else out
        for t, what in ((delta, "delta"), (f, "f"), (theta_in, "theta_in"), (out, "out")):
            _need(t, nl ** 3, what)
        s = ctypes.c_double()
        _check(self.lib.mr_sweep(self.h, nl, h, _ptr(delta), _ptr(f), cshift, _ptr(theta_in), _ptr(out),
                                 ctypes.byref(s)))
        return out, s.value

    def defect_restrict(self, delta, theta, h=1.0, f=None, cshift=0.0):
        nl = theta.shape[0]
        for t, what in ((delta, "delta"), (f, "f"), (theta, "theta")):
            _need(t, nl ** 3, what)
        tc = self._empty(nl // 2)
        dr = self._empty(nl // 2)
        _check(self.lib.mr_defect_restrict(self.h, nl, h, _ptr(delta), _ptr(f), cshift, _ptr(theta),
                                           _ptr(tc), _ptr(dr)))
        return tc, dr

    def lin_residual(self, delta, theta_base, e, h=1.0, rhs=None, cshift=0.0):
        """mr_lin_residual: rhs + dSigma(e) - lap(e) - cshift of the FP32 inner operator at theta_base."""
        nl = e.shape[0]
        for t, what in ((delta, "delta"), (theta_base, "theta_base"), (e, "e"), (rhs, "rhs")):
            _need(t, nl ** 3, what)
        out = self._empty(nl)
        _check(self.lib.mr_lin_residual(self.h, nl, h, _ptr(delta), _ptr(theta_base), _ptr(e), _ptr(rhs),
                                        cshift, _ptr(out)))
        return out

    def lin_defect_restrict(self, delta, theta_base, e, h=1.0, rhs=None, cshift=0.0):
        """mr_lin_defect_restrict: R(rhs + dSigma(e) - lap(e) - cshift) on the (nl/2)^3 mesh."""
        nl = e.shape[0]
        for t, what in ((delta, "delta"), (theta_base, "theta_base"), (e, "e"), (rhs, "rhs")):
            _need(t, nl ** 3, what)
        out = self._empty(nl // 2)
        _check(self.lib.mr_lin_defect_restrict(self.h, nl, h, _ptr(delta), _ptr(theta_base), _ptr(e), _ptr(rhs),
                                               cshift, _ptr(out)))
        return out

    def lin_prolong_add(self, ec, e_in):
        """mr_lin_prolong_add: e_in + P ec (FP32 inner-solve prolongation) on the nl^3 mesh."""
        nl = e_in.shape[0]
        _need(e_in, nl ** 3, "e_in")
        _need(ec, (nl // 2) ** 3, "ec")
        out = self._empty(nl)
        _check(self.lib.mr_lin_prolong_add(self.h, nl, _ptr(ec), _ptr(e_in), _ptr(out)))
        return out

    def lin_sweep(self, delta, theta_base, e_in, h=1.0, rhs=None, cshift=0.0, sched=None):
        """mr_lin_sweep: one red-black sweep of the FP32 inner smoother; sched = (kind, tm, tj, nchunks)."""
        nl = e_in.shape[0]
        for t, what in ((delta, "delta"), (theta_base, "theta_base"), (e_in, "e_in"), (rhs, "rhs")):
            _need(t, nl ** 3, what)
        out = self._empty(nl)
        sp = None if sched is None else (ctypes.c_int * 4)(*sched)
        _check(self.lib.mr_lin_sweep(self.h, nl, h, _ptr(delta), _ptr(theta_base), _ptr(e_in), _ptr(rhs), cshift,
                                     sp, _ptr(out)))
        return out

    def lin_vcycles(self, delta, theta_base, rhs, ncycles=1):
        """mr_lin_vcycles: ncycles inner FP32 V-cycles for J_p(theta_base) e = rhs from e = 0."""
        for t, what in ((delta, "delta"), (theta_base, "theta_base"), (rhs, "rhs")):
            _need(t, self.n ** 3, what)
        out = self._empty()
        _check(self.lib.mr_lin_vcycles(self.h, _ptr(delta), _ptr(theta_base), _ptr(rhs), ncycles, _ptr(out)))
        return out

    def tau_rhs(self, delta, theta_hat, rd, h):
        nl = theta_hat.shape[0]
        for t, what in ((delta, "delta"), (theta_hat, "theta_hat"), (rd, "rd")):
            _need(t, nl ** 3, what)
        f = self._empty(nl)
        s = ctypes.c_double()
        _check(self.lib.mr_tau_rhs(self.h, nl, h, _ptr(delta), _ptr(theta_hat), _ptr(rd), _ptr(f),
                                   ctypes.byref(s)))
        return f, s.value

    def prolong_correct(self, theta_c, theta_hat_c, theta):
        nl = theta.shape[0]
        _need(theta, nl ** 3, "theta")
        _need(theta_c, (nl // 2) ** 3, "theta_c")
        _need(theta_hat_c, (nl // 2) ** 3, "theta_hat_c")
        _check(self.lib.mr_prolong_correct(self.h, nl, _ptr(theta_c), _ptr(theta_hat_c), _ptr(theta)))
        return theta

    def restrict(self, fine):
        nl = fine.shape[0]
        _need(fine, nl ** 3, "fine")
        out = self._empty(nl // 2)
        _check(self.lib.mr_restrict(self.h, nl, _ptr(fine), _ptr(out)))
        return out


def solve_batched(deltas: Sequence[torch.Tensor], thetas: Optional[Sequence[torch.Tensor]] = None,
                  check: bool = True, eager: bool = False, anderson: bool = False, **opts):
    """Solve independent periodic boxes of possibly different sizes in one batched call
    (mr_solve_batched: mixed precision, one launch per phase and box size, graph replay).

    deltas: contiguous float64 CUDA tensors of shapes (n_b, n_b, n_b). thetas: output tensors of
    the same shapes (allocated when None). eager: launch every pass directly instead of replaying
    the captured graph. anderson: mix each box's outer iterations (MR_FLAG_ANDERSON). Remaining
    keywords set mr_opts fields (tol, max_cycles, npre, ...). Returns (thetas, infos)."""
    lib = load()
    nbox = len(deltas)
    thetas = [torch.zeros_like(d) for d in deltas] if thetas is None else list(thetas)
    o = default_opts(**opts)
    if eager:
        o.flags |= MR_FLAG_EAGER
    if anderson:
        o.flags |= MR_FLAG_ANDERSON
    for t in list(deltas) + thetas:
        _ptr(t)
    ns = (ctypes.c_int * nbox)(*[d.shape[0] for d in deltas])
    dp = (ctypes.c_void_p * nbox)(*[d.data_ptr() for d in deltas])
    tp = (ctypes.c_void_p * nbox)(*[t.data_ptr() for t in thetas])
    infos = (mr_info * nbox)()
    code = lib.mr_solve_batched(nbox, ns, dp, tp, ctypes.byref(o), infos, _stream())
    if check:
        _check(code)
    return thetas, [Info.from_c(i) for i in infos]


class Batch:
    """A reusable batch (mr_batch_create / mr_batch_solve / mr_batch_destroy): the working set of
    boxes of sizes `ns` is allocated and one outer iteration captured once; each solve() then runs
    the batched mixed-precision solve on new inputs without device allocation."""

    def __init__(self, ns: Sequence[int], eager: bool = False, anderson: bool = False, **opts):
        self.lib = load()
        self.ns = [int(x) for x in ns]
        o = default_opts(**opts)
        if eager:
            o.flags |= MR_FLAG_EAGER
        if anderson:
            o.flags |= MR_FLAG_ANDERSON
        h = ctypes.c_void_p()
        arr = (ctypes.c_int * len(self.ns))(*self.ns)
        _check(self.lib.mr_batch_create(ctypes.byref(h), len(self.ns), arr, ctypes.byref(o), _stream()))
        self.h = h

    def solve(self, deltas: Sequence[torch.Tensor], thetas: Optional[Sequence[torch.Tensor]] = None,
              check: bool = True):
        """Solve the boxes (shapes (n_b,)*3 in the batch's order); returns (thetas, infos)."""
        if len(deltas) != len(self.ns):
            raise ValueError(f"expected {len(self.ns)} boxes, got {len(deltas)}")
        thetas = [torch.zeros_like(d) for d in deltas] if thetas is None else list(thetas)
        for d, t, n in zip(deltas, thetas, self.ns):
            _need(d, n ** 3, "delta")
            _need(t, n ** 3, "theta")
            _ptr(d)
            _ptr(t)
        nbox = len(self.ns)
        dp = (ctypes.c_void_p * nbox)(*[d.data_ptr() for d in deltas])
        tp = (ctypes.c_void_p * nbox)(*[t.data_ptr() for t in thetas])
        infos = (mr_info * nbox)()
        code = self.lib.mr_batch_solve(self.h, dp, tp, infos)
        if check:
            _check(code)
        return thetas, [Info.from_c(i) for i in infos]

    def close(self):
        if getattr(self, "h", None):
            self.lib.mr_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_lin_tiles(n: int):
    """Tile tuner of the batched FP32 sweep (mr_tune_lin_tiles) on the current device:
    returns (tm, tj, ci, ms) for an n^3 box; the choice is cached per device and n."""
    lib = load()
    tm, tj, ci = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ms = ctypes.c_float()
    _check(lib.mr_tune_lin_tiles(n, _stream(), ctypes.byref(tm), ctypes.byref(tj), ctypes.byref(ci), ctypes.byref(ms)))
    return tm.value, tj.value, ci.value, ms.value


def hbm_stream(kind: int, a: torch.Tensor, c: torch.Tensor, b: Optional[torch.Tensor] = None,
               nontemporal: bool = False, blocks_per_cu: int = 8) -> float:
    """One launch of the HBM streaming probe (mr_hbm_stream); returns its duration in ms."""
    lib = load()
    ms = ctypes.c_float()
    _check(lib.mr_hbm_stream(kind, int(nontemporal), _ptr(a), _ptr(b), _ptr(c), a.numel(), blocks_per_cu,
                             _stream(), ctypes.byref(ms)))
    return ms.value


def residual_noalloc(delta: torch.Tensor, theta: torch.Tensor, r_out: Optional[torch.Tensor] = None):
    """mr_residual_noalloc: (r_out or None, rel, <Sigma>) without a context or device allocation."""
    n = round(delta.numel() ** (1.0 / 3.0))
    for t, what in ((delta, "delta"), (theta, "theta"), (r_out, "r_out")):
        _need(t, n ** 3, what)
    rel, ms = ctypes.c_double(), ctypes.c_double()
    _check(load().mr_residual_noalloc(n, _ptr(delta), _ptr(theta), _ptr(r_out), ctypes.byref(rel), ctypes.byref(ms),
                                      _stream()))
    return r_out, rel.value, ms.value


def tuning_file(path: Optional[str]):
    """mr_tuning_file: record tuner choices in `path` from now on (None: the default location,
    "": no file)."""
    _check(load().mr_tuning_file(None if path is None else path.encode()))


def tuning_file_path() -> str:
    """mr_tuning_file_path: the file of recorded tuner choices in use ("" if none)."""
    return load().mr_tuning_file_path().decode()


def tuning_store(kind: str, arch: str, device: str, cus: int, n: int, values):
    """mr_tuning_store: record integer values under (kind, arch, device, cus, n)."""
    vals = (ctypes.c_int * len(values))(*values)
    _check(load().mr_tuning_store(kind.encode(), arch.encode(), device.encode(), cus, n, vals, len(values)))


def tuning_lookup(kind: str, arch: str, device: str, cus: int, n: int, max_count: int = 64):
    """mr_tuning_lookup: the values recorded under the key, or None."""
    vals = (ctypes.c_int * max_count)()
    cnt = ctypes.c_int()
    _check(load().mr_tuning_lookup(kind.encode(), arch.encode(), device.encode(), cus, n, vals, max_count,
                                   ctypes.byref(cnt)))
    return list(vals[: cnt.value]) if cnt.value else None
