"""ctypes binding of the C ABI declared in include/dd_dlra.h.

Argument marshalling only: every step of the method runs in the HIP library.
Device memory may come from PyTorch (``workspace='torch'``) and the stream
from ``torch.cuda.current_stream()``; otherwise the library allocates its
own arena and stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

DD_OK, DD_EINVAL, DD_ENOMEM, DD_EHIP, DD_ERANK, DD_ENUMERIC, DD_ESTATE = 0, -1, -2, -3, -4, -5, -6
DD_PREC_FP64, DD_PREC_MIXED_FP32, DD_PREC_MIXED_BF16 = 0, 1, 2
DD_RANK_FIXED, DD_RANK_ADAPTIVE = 0, 1
DD_EXEC_PER_SUBDOMAIN, DD_EXEC_BATCHED, DD_EXEC_BATCHED_GRAPH = 0, 1, 2
DD_INT_EULER, DD_INT_RK4 = 0, 1
DD_BC_VACUUM, DD_BC_INFLOW_LOWRANK = 0, 1
DD_PROBE_VHAT, DD_PROBE_K1, DD_PROBE_U1, DD_PROBE_S2, DD_PROBE_L1 = 1, 2, 3, 4, 5

EXPORTS = (
    "dd_dlra_workspace_size", "dd_dlra_create", "dd_dlra_step", "dd_dlra_stage", "dd_dlra_get_ranks",
    "dd_dlra_get_factors", "dd_dlra_moments", "dd_dlra_moments_noalloc", "dd_dlra_probe", "dd_dlra_set_factors", "dd_dlra_force_ranks", "dd_dlra_autotune",
    "dd_dlra_set_tiling",
    "dd_dlra_profile", "dd_dlra_kernel_stats", "dd_dlra_kernel_name",
    "dd_dlra_sync", "dd_dlra_destroy", "dd_dlra_last_error",
)

_HERE = os.path.dirname(os.path.abspath(__file__))
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("px", ctypes.c_int32), ("py", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("n_dir", ctypes.c_int32),
        ("omega_x", _DP), ("omega_y", _DP), ("w", _DP),
        ("c_adv", ctypes.c_double),
        ("sigma_s", _DP), ("sigma_a", _DP), ("Q", _DP),
        ("dt", ctypes.c_double),
        ("rank_mode", ctypes.c_int32), ("r_fixed", ctypes.c_int32), ("r_min", ctypes.c_int32),
        ("r_max", ctypes.c_int32), ("r_int_max", ctypes.c_int32),
        ("tol", ctypes.c_double), ("tol_aug_rel", ctypes.c_double),
        ("precision", ctypes.c_int32), ("exec_mode", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
        ("strict_caps", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("bc_rank", ctypes.c_int32 * 4), ("bc_a", _DP * 4), ("bc_b", _DP * 4),
    ]


class DDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dd_dlra status {status}: {msg}")
        self.status = status


def library_path() -> str:
    return os.environ.get("DD_DLRA_LIB", os.path.join(_HERE, "libdd_dlra.so"))


_lib = None


def load_library():
    """Load libdd_dlra.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing; build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.dd_dlra_workspace_size.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]
    lib.dd_dlra_create.argtypes = [ctypes.POINTER(Config), _IP, ctypes.POINTER(_DP), ctypes.POINTER(_DP),
                                   ctypes.POINTER(_DP), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.dd_dlra_step.argtypes = [vp, ctypes.c_int32]
    lib.dd_dlra_stage.argtypes = [vp, ctypes.c_int32]
    lib.dd_dlra_get_ranks.argtypes = [vp, _IP, _IP, ctypes.POINTER(ctypes.c_int64)]
    lib.dd_dlra_get_factors.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _IP, _DP, _DP, _DP]
    lib.dd_dlra_moments.argtypes = [vp, _DP, _DP, _DP, ctypes.c_int32]
    lib.dd_dlra_moments_noalloc.argtypes = [vp, _DP, _DP, _DP]
    lib.dd_dlra_probe.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _DP, _IP, _IP]
    lib.dd_dlra_autotune.argtypes = [vp, ctypes.c_int32, _IP, _DP]
    lib.dd_dlra_set_tiling.argtypes = [vp, ctypes.c_int32]
    lib.dd_dlra_set_factors.argtypes = [vp, _IP, ctypes.POINTER(_DP), ctypes.POINTER(_DP), ctypes.POINTER(_DP)]
    lib.dd_dlra_force_ranks.argtypes = [vp, _IP, _IP]
    lib.dd_dlra_profile.argtypes = [vp, ctypes.c_int32]
    lib.dd_dlra_kernel_stats.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double), _IP]
    lib.dd_dlra_kernel_name.argtypes = [ctypes.c_int32]
    lib.dd_dlra_kernel_name.restype = ctypes.c_char_p
    lib.dd_dlra_sync.argtypes = [vp]
    lib.dd_dlra_destroy.argtypes = [vp]
    lib.dd_dlra_last_error.argtypes = [vp]
    lib.dd_dlra_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("dd_dlra_last_error", "dd_dlra_kernel_name"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


class _ConfigHolder:
    """Keeps the numpy arrays a Config points to alive."""

    def __init__(self, wl, precision: int, exec_mode: int, strict: int):
        integ = str(getattr(wl, "integrator", "euler"))
        if integ not in ("euler", "rk4"):
            raise ValueError(f"integrator {integ!r}: the engine takes 'euler' or 'rk4'")
        self.ox = _f64(wl.omega_x)
        self.oy = _f64(wl.omega_y)
        self.w = _f64(wl.w)
        self.ss = _f64(wl.sigma_s)
        self.sa = _f64(wl.sigma_a)
        self.q = _f64(wl.Q)
        c = Config()
        c.nx, c.ny, c.px, c.py = int(wl.nx), int(wl.ny), int(wl.px), int(wl.py)
        c.x0, c.x1, c.y0, c.y1 = float(wl.x0), float(wl.x1), float(wl.y0), float(wl.y1)
        c.n_dir = int(self.w.shape[0])
        c.omega_x, c.omega_y, c.w = _dp(self.ox), _dp(self.oy), _dp(self.w)
        c.c_adv = float(wl.c_adv)
        c.sigma_s, c.sigma_a, c.Q = _dp(self.ss), _dp(self.sa), _dp(self.q)
        c.dt = float(wl.dt)
        c.rank_mode = int(wl.rank_mode)
        c.r_fixed, c.r_min, c.r_max = int(wl.r_fixed), int(wl.r_min), int(wl.r_max)
        c.r_int_max = int(wl.r_int_max)
        c.tol, c.tol_aug_rel = float(wl.tol), float(wl.tol_aug_rel)
        c.precision, c.exec_mode = int(precision), int(exec_mode)
        c.bc[:] = [0, 0, 0, 0]
        self.bc_arrays = []
        for f, spec in enumerate(getattr(wl, "inflow", None) or [None] * 4):
            if spec is None:
                continue
            A = np.asarray(spec[0], float)
            B = np.asarray(spec[1], float)
            if A.ndim == 1:
                A = A[:, None]
            if B.ndim == 1:
                B = B[:, None]
            a = np.ascontiguousarray(A.T)   # [rb][face cells]
            b = np.ascontiguousarray(B.T)   # [rb][M]
            self.bc_arrays += [a, b]
            c.bc[f] = DD_BC_INFLOW_LOWRANK
            c.bc_rank[f] = int(A.shape[1])
            c.bc_a[f] = _dp(a)
            c.bc_b[f] = _dp(b)
        c.strict_caps = int(strict)
        c.integrator = DD_INT_RK4 if integ == "rk4" else DD_INT_EULER
        self.cfg = c


def workspace_size(wl, precision=DD_PREC_FP64, exec_mode=DD_EXEC_BATCHED_GRAPH) -> int:
    lib = load_library()
    h = _ConfigHolder(wl, precision, exec_mode, 0)
    n = ctypes.c_size_t(0)
    st = lib.dd_dlra_workspace_size(ctypes.byref(h.cfg), ctypes.byref(n))
    if st != DD_OK:
        raise DDError(st, lib.dd_dlra_last_error(None).decode())
    return int(n.value)


def _factor_ptrs(U, S, V):
    Us = [np.asfortranarray(np.asarray(u, np.float64)) for u in U]
    Ss = [np.asfortranarray(np.asarray(s, np.float64)) for s in S]
    Vs = [np.asfortranarray(np.asarray(v, np.float64)) for v in V]
    n = len(Us)
    pu = (_DP * n)(*[u.ctypes.data_as(_DP) for u in Us])
    ps = (_DP * n)(*[s.ctypes.data_as(_DP) for s in Ss])
    pv = (_DP * n)(*[v.ctypes.data_as(_DP) for v in Vs])
    ranks = np.ascontiguousarray([s.shape[0] for s in Ss], dtype=np.int32)
    return (Us, Ss, Vs, ranks), pu, ps, pv


class DDDLRA:
    """One DD-DLRA engine instance on the current GPU.

    wl: a problem description with the attributes of ``workloads.Workload``
    (grid, directions, fields, rank settings and the initial factors U0, S0,
    V0 per subdomain, column-major N x r, r x r, M x r)."""

    def __init__(self, wl, precision: int = DD_PREC_FP64, exec_mode: int = DD_EXEC_BATCHED_GRAPH,
                 strict_caps: int = 0, workspace: Optional[str] = None, stream=None):
        self.lib = load_library()
        self.wl = wl
        self.nsub = int(wl.px * wl.py)
        self.N = int((wl.nx // wl.px) * (wl.ny // wl.py))
        self.M = int(np.asarray(wl.w).shape[0])
        self.nx, self.ny = int(wl.nx), int(wl.ny)
        self._cfg = _ConfigHolder(wl, precision, exec_mode, strict_caps)
        keep, pu, ps, pv = _factor_ptrs(wl.U0, wl.S0, wl.V0)
        self._ws_tensor = None
        ws_ptr, ws_bytes = None, 0
        stream_ptr = None
        if workspace == "torch":
            import torch
            nbytes = workspace_size(wl, precision, exec_mode)
            self._ws_tensor = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ws_ptr, ws_bytes = self._ws_tensor.data_ptr(), nbytes
        if stream is not None:
            stream_ptr = int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)
        h = ctypes.c_void_p()
        st = self.lib.dd_dlra_create(ctypes.byref(self._cfg.cfg), keep[3].ctypes.data_as(_IP), pu, ps, pv,
                                     ws_ptr, ws_bytes, stream_ptr, ctypes.byref(h))
        if st != DD_OK:
            raise DDError(st, self.lib.dd_dlra_last_error(None).decode())
        self.h = h

    # ------------------------------------------------------------------ helpers
    def _check(self, st):
        if st != DD_OK:
            raise DDError(st, self.lib.dd_dlra_last_error(self.h).decode())

    def step(self, n: int = 1):
        self._check(self.lib.dd_dlra_step(self.h, int(n)))

    def stage(self, which: int):
        """Run one stage: 0 = x-advection, 1 = y-advection, 2 = collision."""
        self._check(self.lib.dd_dlra_stage(self.h, int(which)))

    def sync(self):
        self._check(self.lib.dd_dlra_sync(self.h))

    def ranks(self) -> Tuple[np.ndarray, np.ndarray, int]:
        r = np.zeros(self.nsub, np.int32)
        t = np.zeros(self.nsub, np.int32)
        c = ctypes.c_int64(0)
        self._check(self.lib.dd_dlra_get_ranks(self.h, r.ctypes.data_as(_IP), t.ctypes.data_as(_IP),
                                                ctypes.byref(c)))
        return r, t, int(c.value)

    def factors(self, sd: int):
        cap = int(self.wl.r_int_max)
        r = ctypes.c_int32(0)
        U = np.zeros(self.N * cap)
        S = np.zeros(cap * cap)
        V = np.zeros(self.M * cap)
        self._check(self.lib.dd_dlra_get_factors(self.h, int(sd), cap, ctypes.byref(r), _dp(U), _dp(S), _dp(V)))
        k = r.value
        return (U[: self.N * k].reshape(k, self.N).T.copy(), S[: k * k].reshape(k, k).T.copy(),
                V[: self.M * k].reshape(k, self.M).T.copy())

    def state(self) -> List[tuple]:
        return [self.factors(s) for s in range(self.nsub)]

    def moments(self, out=None):
        """Scalar flux on the global grid; out may be a CUDA torch tensor."""
        if out is not None:
            self._check(self.lib.dd_dlra_moments(self.h, ctypes.cast(out.data_ptr(), _DP), None, None, 1))
            return out
        rho = np.zeros(self.nx * self.ny)
        self._check(self.lib.dd_dlra_moments(self.h, _dp(rho), None, None, 0))
        return rho

    def moments_noalloc(self, rho, jx=None, jy=None):
        """Moments into device buffers (CUDA tensors of nx*ny doubles) without
        any device allocation (the library's static scratch).  Asynchronous on
        the engine's stream."""
        p = lambda t: None if t is None else ctypes.cast(t.data_ptr(), _DP)
        self._check(self.lib.dd_dlra_moments_noalloc(self.h, p(rho), p(jx), p(jy)))
        return rho

    def probe(self, stage: int, upto: int, sd: int) -> np.ndarray:
        """One working array of subdomain sd after advection stage `stage` ran
        up to phase `upto` (DD_PROBE_*); the state is left as it was."""
        cap = max(self.N, self.M) * int(self.wl.r_int_max)
        buf = np.zeros(cap)
        r = ctypes.c_int32(0)
        c = ctypes.c_int32(0)
        self._check(self.lib.dd_dlra_probe(self.h, int(stage), int(upto), int(sd), cap, _dp(buf), ctypes.byref(r),
                                           ctypes.byref(c)))
        return buf[: r.value * c.value].reshape(c.value, r.value).T.copy()

    def autotune(self, steps: int = 2) -> Tuple[int, float]:
        """Pick the workgroups per subdomain of the tall-skinny kernels by
        timing the live problem (state unchanged); returns (choice, ms/step)."""
        wg = ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        self._check(self.lib.dd_dlra_autotune(self.h, int(steps), ctypes.byref(wg), ctypes.byref(ms)))
        return int(wg.value), float(ms.value)

    def set_tiling(self, wg_per_subdomain: int):
        """Workgroups per subdomain of the tall-skinny kernels."""
        self._check(self.lib.dd_dlra_set_tiling(self.h, int(wg_per_subdomain)))

    def currents(self):
        """(rho, jx, jy): scalar flux and current density on the global grid."""
        rho, jx, jy = (np.zeros(self.nx * self.ny) for _ in range(3))
        self._check(self.lib.dd_dlra_moments(self.h, _dp(rho), _dp(jx), _dp(jy), 0))
        return rho, jx, jy

    def set_factors(self, U: Sequence, S: Sequence, V: Sequence):
        keep, pu, ps, pv = _factor_ptrs(U, S, V)
        self._check(self.lib.dd_dlra_set_factors(self.h, keep[3].ctypes.data_as(_IP), pu, ps, pv))

    def force_ranks(self, t: Optional[Sequence[int]], r_out: Optional[Sequence[int]]):
        ta = None if t is None else np.ascontiguousarray(t, np.int32)
        ra = None if r_out is None else np.ascontiguousarray(r_out, np.int32)
        self._check(self.lib.dd_dlra_force_ranks(self.h, None if ta is None else ta.ctypes.data_as(_IP),
                                                  None if ra is None else ra.ctypes.data_as(_IP)))

    def profile(self, enable=True):
        """Bracket later non-graph phase launches with hipEvents.  An integer
        k > 1 also launches each repeatable tall-skinny phase k times inside
        its event pair."""
        level = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        self._check(self.lib.dd_dlra_profile(self.h, level))

    def kernel_stats(self) -> dict:
        """{kernel name: (launches, total milliseconds)} of the profiled launches."""
        n = ctypes.c_int32(0)
        self._check(self.lib.dd_dlra_kernel_stats(self.h, 0, None, None, ctypes.byref(n)))
        k = n.value
        cnt = np.zeros(k, np.int64)
        ms = np.zeros(k)
        self._check(self.lib.dd_dlra_kernel_stats(self.h, k, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                  _dp(ms), ctypes.byref(n)))
        return {self.lib.dd_dlra_kernel_name(i).decode(): (int(cnt[i]), float(ms[i])) for i in range(k)}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.dd_dlra_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
