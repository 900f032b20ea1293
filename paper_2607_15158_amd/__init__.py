"""MI355X SI-CTMRG: Python binding of libsictm.so (include/ctm.h).

The binding only marshals arguments: every step of a CTMRG move runs in the
library's HIP kernels.  PyTorch supplies device memory (the workspace and the
input tensors) and the stream.  Importing this package fails loudly when the
library has not been built (``python paper_2607_15158_amd/build_lib.py``).
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsictm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2607_15158_amd/build_lib.py` "
        "(the HIP library is required; there is no CPU fallback)")

# torch is imported first so that its HIP runtime is the one in the process:
# the library's libamdhip64.so.7 / libhsa-runtime64.so.1 dependencies then
# bind to the copies torch already loaded (same sonames).  Loading the
# library first would bring in a second HIP/HSA runtime, which cannot share
# the device, the streams or the allocations with torch.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

CTM_OK, CTM_E_ARG, CTM_E_SHAPE, CTM_E_NOMEM, CTM_E_DEVICE, CTM_E_NUMERIC, \
    CTM_E_NOT_CONVERGED, CTM_E_STATE = range(8)
PROJ = {"svd": 0, "fullsvd": 0, "si": 1}
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
SVD_DRIVER = {"gesvd": 0, "gesdd": 1, "gesvdx": 2}
GROWTH = {"svd": 0, "si": 1}
SYM = {"none": 0, "c4v": 1}
OBS_NORM, OBS_ONESITE, OBS_BOND_H, OBS_BOND_V, OBS_BOND_D, OBS_BOND_AD, OBS_XI_H, OBS_XI_V = range(8)


class ctm_config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("D", ctypes.c_int), ("chi", ctypes.c_int),
                ("p", ctypes.c_int), ("n_si", ctypes.c_int), ("proj", ctypes.c_int),
                ("prec", ctypes.c_int), ("stabilized", ctypes.c_int),
                ("pinv_rtol", ctypes.c_double), ("svd_driver", ctypes.c_int), ("sym", ctypes.c_int),
                ("recycle_sin2", ctypes.c_double), ("min_si_moves", ctypes.c_int),
                ("growth", ctypes.c_int)]


class ctm_move_info(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("mode", ctypes.c_int), ("chi_env", ctypes.c_int),
                ("gap", ctypes.c_double), ("n_si", ctypes.c_int), ("sin2", ctypes.c_double)]


class ctm_result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("moves", ctypes.c_int), ("converged", ctypes.c_int),
                ("delta", ctypes.c_double), ("kappa", ctypes.c_double), ("bond_h", ctypes.c_double),
                ("bond_v", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("bytes", ctypes.c_size_t)]


class ctm_prof_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class ctm_cell_config(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("d", ctypes.c_int),
                ("D", ctypes.c_int), ("chi", ctypes.c_int), ("p", ctypes.c_int),
                ("n_si", ctypes.c_int), ("stabilized", ctypes.c_int),
                ("pinv_rtol", ctypes.c_double)]


CELL_RSVD, CELL_SI, CELL_SVD, CELL_GROW = range(4)
CELL_MODE = {"rsvd": CELL_RSVD, "si": CELL_SI, "svd": CELL_SVD}

_vp, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_sigs = {
    "ctm_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ctm_last_error": (ctypes.c_char_p, [_vp]),
    "ctm_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ctm_config), ctypes.POINTER(ctypes.c_size_t)]),
    "ctm_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(ctm_config), _vp, _vp, _vp,
                                ctypes.c_size_t, _vp]),
    "ctm_destroy": (None, [_vp]),
    "ctm_set_isometries": (ctypes.c_int, [_vp, _vp, _vp]),
    "ctm_move": (ctypes.c_int, [_vp, ctypes.POINTER(ctm_move_info)]),
    "ctm_move_async": (ctypes.c_int, [_vp]),
    "ctm_use_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ctm_move_poll": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctm_move_info)]),
    "ctm_move_batch": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctm_move_info)]),
    "ctm_move_batch_async": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "ctm_server_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_size_t, ctypes.c_int]),
    "ctm_server_destroy": (None, [_vp]),
    "ctm_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(ctm_config), _dp, _dp, _dp, _dp, _dp,
                                         ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "ctm_server_pump": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ctm_server_batching": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ctm_server_result": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctm_result)]),
    "ctm_server_error": (ctypes.c_char_p, [_vp, ctypes.c_int]),
    "ctm_server_clock": (ctypes.c_double, [_vp]),
    "ctm_converge": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), _dp]),
    "ctm_observable": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "ctm_state_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ctm_get_state": (ctypes.c_int, [_vp, _dp, ctypes.c_size_t]),
    "ctm_get_state_device": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "ctm_set_state": (ctypes.c_int, [_vp, _dp, ctypes.c_size_t]),
    "ctm_profile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ctm_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctm_prof_entry), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "ctm_gemm_f64": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                    ctypes.c_double, ctypes.c_int, _vp]),
    "ctm_gemm_f64_split_scratch_bytes": (ctypes.c_size_t, []),
    "ctm_gemm_f64_split": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                          ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_long,
                                          ctypes.c_long, ctypes.c_long, ctypes.c_double, ctypes.c_int,
                                          _vp, ctypes.c_size_t, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int), _vp]),
    "ctm_qr_f64": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp]),
    "ctm_qr_f64_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int,
                                          ctypes.c_int, _vp]),
    "ctm_qr_f64_noalloc_max_bytes": (ctypes.c_size_t, []),
    "ctm_vjp_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ctm_config), ctypes.POINTER(ctypes.c_size_t)]),
    "ctm_move_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t]),
    "ctm_energy_vjp": (ctypes.c_int, [_vp, _vp, _dp, _dp, _vp, _vp, _vp, ctypes.c_size_t]),
    "ctm_bond_energy_vjp": (ctypes.c_int, [_vp, _vp, _dp, ctypes.c_int, _dp, _vp, _vp, _vp,
                                           ctypes.c_size_t]),
    "ctm_fixed_point_vjp": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _vp, _vp,
                                           _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int),
                                           _dp]),
    "ctm_svd_f64": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                   ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "ctm_cell_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ctm_cell_config),
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "ctm_cell_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(ctm_cell_config), _vp,
                                       _vp]),
    "ctm_cell_destroy": (None, [_vp]),
    "ctm_cell_last_error": (ctypes.c_char_p, [_vp]),
    "ctm_cell_set_blocks": (ctypes.c_int, [_vp, _vp, _vp]),
    "ctm_cell_iterate": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "ctm_cell_run": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    _ip, _dp, _ip]),
    "ctm_cell_env_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ctm_cell_get_env": (ctypes.c_int, [_vp, _dp, ctypes.c_size_t, _ip]),
    "ctm_cell_set_env": (ctypes.c_int, [_vp, _dp, ctypes.c_size_t, _ip]),
    "ctm_cell_get_blocks": (ctypes.c_int, [_vp, _dp, _dp]),
    "ctm_cell_state_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ctm_cell_get_state_device": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "ctm_cell_set_state_device": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "ctm_cell_move_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "ctm_cell_energy_vjp": (ctypes.c_int, [_vp, _vp, _dp, ctypes.c_int, _dp, _vp, _vp]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class CtmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.ctm_status_str(status).decode()}: {msg}")
        self.status = status


def _check(status: int, ctx=None):
    if status != CTM_OK:
        raise CtmError(status, _lib.ctm_last_error(ctx).decode())
    return status


def _ptr(t) -> int:
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclass
class Config:
    d: int
    D: int
    chi: int
    p: int = 8
    n_si: int = 2
    proj: str = "si"
    prec: str = "f64"
    stabilized: int = 1
    pinv_rtol: float = 1e-12
    svd_driver: str = "gesvd"
    sym: str = "none"
    recycle_sin2: float = 0.0
    min_si_moves: int = 3
    growth: str = "svd"

    def c(self) -> ctm_config:
        return ctm_config(self.d, self.D, self.chi, self.p, self.n_si, PROJ[self.proj],
                          PREC[self.prec], self.stabilized, self.pinv_rtol,
                          SVD_DRIVER[self.svd_driver], SYM[self.sym], self.recycle_sin2,
                          self.min_si_moves, GROWTH[self.growth])

    @property
    def Dl(self) -> int:
        return self.D * self.D if self.d > 0 else self.D

    @property
    def N(self) -> int:
        return self.chi * self.Dl

    @property
    def k(self) -> int:
        return min(self.chi + self.p, self.N)


def workspace_bytes(cfg: Config) -> int:
    n = ctypes.c_size_t(0)
    c = cfg.c()
    _check(_lib.ctm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)))
    return n.value


class Ctm:
    """One environment solve on the GPU (owns a torch workspace tensor)."""

    def __init__(self, cfg: Config, site, boundary=None, stream=None, workspace=None):
        import torch
        self.cfg = cfg
        self._c = cfg.c()
        dev = torch.device("cuda", torch.cuda.current_device())
        self._site = site.to(dev, torch.float64).contiguous()
        self._bnd = None if boundary is None else boundary.to(dev, torch.float64).contiguous()
        nbytes = workspace_bytes(cfg)
        self.workspace = (torch.empty(nbytes, dtype=torch.uint8, device=dev)
                          if workspace is None else workspace)
        self.stream = stream
        self._vjp_ws = None
        h = ctypes.c_void_p()
        _check(_lib.ctm_init(ctypes.byref(h), ctypes.byref(self._c), _ptr(self._site),
                             None if self._bnd is None else _ptr(self._bnd),
                             _ptr(self.workspace), nbytes, _stream(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.ctm_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter exit the HIP runtime (and a profiler's tool library)
        # may already be torn down: a context still open then is left to the
        # process teardown instead of calling into the runtime (the check is
        # bound at definition time, since module globals may be gone by then).
        if _finalizing():
            return
        self.close()

    def set_isometries(self, X, Yt):
        """X, Yt: device float64 tensors of shape (4, N, k)."""
        X = X.contiguous()
        Yt = Yt.contiguous()
        _check(_lib.ctm_set_isometries(self._h, _ptr(X), _ptr(Yt)), self._h)
        self._keep = (X, Yt)

    def move(self) -> dict:
        info = ctm_move_info()
        _check(_lib.ctm_move(self._h, ctypes.byref(info)), self._h)
        return {"delta": info.delta, "mode": info.mode, "chi_env": info.chi_env, "gap": info.gap,
                "n_si": info.n_si, "sin2": info.sin2}

    def use_graphs(self, enable: bool = True) -> None:
        _check(_lib.ctm_use_graphs(self._h, int(enable)), self._h)

    def move_async(self) -> None:
        _check(_lib.ctm_move_async(self._h), self._h)

    def move_poll(self) -> Optional[dict]:
        """None while the move in flight runs, else its info."""
        done = ctypes.c_int(0)
        info = ctm_move_info()
        _check(_lib.ctm_move_poll(self._h, ctypes.byref(done), ctypes.byref(info)), self._h)
        if not done.value:
            return None
        return {"delta": info.delta, "mode": info.mode, "chi_env": info.chi_env, "gap": info.gap,
                "n_si": info.n_si, "sin2": info.sin2}

    def converge(self, tol: float, max_moves: int, raise_on_budget: bool = False):
        n = ctypes.c_int(0)
        dl = ctypes.c_double(0.0)
        st = _lib.ctm_converge(self._h, tol, max_moves, ctypes.byref(n), ctypes.byref(dl))
        if st not in (CTM_OK, CTM_E_NOT_CONVERGED) or (raise_on_budget and st != CTM_OK):
            _check(st, self._h)
        return {"converged": st == CTM_OK, "moves": n.value, "delta": dl.value}

    def observable(self, kind: int, op: Optional[np.ndarray] = None) -> np.ndarray:
        out = np.zeros(8)
        opa = None if op is None else np.ascontiguousarray(op, dtype=np.float64)
        _check(_lib.ctm_observable(self._h, kind,
                                   None if opa is None else opa.ctypes.data_as(_dp),
                                   out.ctypes.data_as(_dp)), self._h)
        return out

    def kappa(self) -> float:
        return float(self.observable(OBS_NORM)[0])

    def correlation_length(self, direction: str = "h", iters: int = 100):
        """(xi, |l2/l1|) of the column (``h``) or row (``v``) transfer matrix."""
        out = self.observable(OBS_XI_H if direction == "h" else OBS_XI_V,
                              np.array([float(iters)]))
        return float(out[0]), float(out[1])

    def state_size(self) -> int:
        n = ctypes.c_size_t(0)
        _check(_lib.ctm_state_size(self._h, ctypes.byref(n)), self._h)
        return n.value

    def get_state(self) -> np.ndarray:
        n = self.state_size()
        buf = np.zeros(n)
        _check(_lib.ctm_get_state(self._h, buf.ctypes.data_as(_dp), n), self._h)
        return buf

    def get_state_device(self):
        """The state vector as a float64 device tensor (a device-to-device copy)."""
        import torch
        n = self.state_size()
        out = torch.empty(n, dtype=torch.float64, device=self._site.device)
        _check(_lib.ctm_get_state_device(self._h, out.data_ptr(), n), self._h)
        return out

    def set_state(self, state: np.ndarray):
        buf = np.ascontiguousarray(state, dtype=np.float64)
        _check(_lib.ctm_set_state(self._h, buf.ctypes.data_as(_dp), buf.size), self._h)

    # adjoint -----------------------------------------------------------------
    def move_vjp(self, state_in, out_bar, want_out: bool = True, site_bar=None):
        """Vector-Jacobian product of one SI move from ``state_in`` (a float64
        device tensor in the state layout): returns the cotangent of the input
        state, the move's output state (or None) and ``site_bar`` (the site
        tensor's cotangent, accumulated into the given tensor or a new one)."""
        import torch
        self._ensure_vjp_ws()
        dev = self._site.device
        sin = state_in.to(dev, torch.float64).contiguous()
        sbar = out_bar.to(dev, torch.float64).contiguous()
        in_bar = torch.empty_like(sin)
        out = torch.empty_like(sin) if want_out else None
        if site_bar is None:
            site_bar = torch.zeros_like(self._site)
        _check(_lib.ctm_move_vjp(self._h, sin.data_ptr(), sbar.data_ptr(), in_bar.data_ptr(),
                                 None if out is None else out.data_ptr(), site_bar.data_ptr(),
                                 self._vjp_ws.data_ptr(), self._vjp_ws.numel()), self._h)
        return in_bar, out, site_bar

    def _ensure_vjp_ws(self):
        import torch
        if self._vjp_ws is None:
            n = ctypes.c_size_t(0)
            _check(_lib.ctm_vjp_workspace_bytes(ctypes.byref(self._c), ctypes.byref(n)))
            self._vjp_ws = torch.empty(n.value, dtype=torch.uint8, device=self._site.device)
        return self._vjp_ws

    def fixed_point_vjp(self, state_star, g_bar, tol: float = 1e-10, max_iter: int = 200,
                        site_bar=None):
        """Fixed-point gradient (eq. implicit) at the converged ``state_star``
        for the state cotangent ``g_bar``: returns (x_bar, site_bar, passes,
        relative norm of the last term); raises if the series did not reach
        ``tol`` within ``max_iter`` passes."""
        import torch
        ws = self._ensure_vjp_ws()
        dev = self._site.device
        x = state_star.to(dev, torch.float64).contiguous()
        g = g_bar.to(dev, torch.float64).contiguous()
        x_bar = torch.empty_like(x)
        if site_bar is None:
            site_bar = torch.zeros_like(self._site)
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        _check(_lib.ctm_fixed_point_vjp(self._h, x.data_ptr(), g.data_ptr(), float(tol),
                                        int(max_iter), x_bar.data_ptr(), site_bar.data_ptr(),
                                        ws.data_ptr(), ws.numel(), ctypes.byref(it),
                                        ctypes.byref(rel)), self._h)
        return x_bar, site_bar, it.value, rel.value

    def energy_vjp(self, state, op, site_bar=None, bonds: str = "hv"):
        """e = sum of <op> over ``bonds`` (``h``, ``v``, ``d`` diagonal, ``a``
        anti-diagonal), or with ``op`` a dict {bond letter: operator} the sum
        of each bond's own operator, at the environment of ``state`` (device
        tensor, state layout) and its gradient: returns (e, state_bar,
        site_bar).  One library call evaluates every bond."""
        import torch
        ws = self._ensure_vjp_ws()
        dev = self._site.device
        st = state.to(dev, torch.float64).contiguous()
        if isinstance(op, dict):
            bonds = "".join(sorted(op, key="hvda".index))
        mask = bond_mask(bonds)
        # one operator per bond of the mask, in the order H, V, D, AD
        order = [b for b in "hvda" if mask & BOND_BITS[b]]
        ops = np.ascontiguousarray(np.stack([np.asarray(op[b] if isinstance(op, dict) else op,
                                                        dtype=np.float64) for b in order]))
        e = ctypes.c_double(0.0)
        bar = torch.empty_like(st)
        if site_bar is None:
            site_bar = torch.zeros_like(self._site)
        _check(_lib.ctm_bond_energy_vjp(self._h, st.data_ptr(), ops.ctypes.data_as(_dp), mask,
                                        ctypes.byref(e), bar.data_ptr(), site_bar.data_ptr(),
                                        ws.data_ptr(), ws.numel()), self._h)
        return e.value, bar, site_bar

    def energy_gradient(self, op, tol: float = 1e-12, max_iter: int = 400, bonds: str = "hv"):
        """Gradient of the converged energy e (the sum of <op> over ``bonds``,
        as in :meth:`energy_vjp`; or, with ``op`` a dict {bond letter:
        operator}, the sum of each bond's own operator) with respect to the
        site tensor at the context's current (converged) environment: the
        direct term plus the fixed-point term (eq. implicit).  Returns
        (e, dE/dA as a device tensor, passes of the fixed-point series)."""
        import torch
        star = torch.from_numpy(self.get_state()).to(self._site.device)
        e, g, site_bar = self.energy_vjp(star, op, bonds=bonds)
        _, site_bar, passes, _ = self.fixed_point_vjp(star, g, tol, max_iter, site_bar)
        return e, site_bar, passes

    def unpack_state(self, state: np.ndarray) -> dict:
        """Splits a state vector into C, T (cut to chi_env), X, Yt, chi_env."""
        chi, Dl, N, k = self.cfg.chi, self.cfg.Dl, self.cfg.N, self.cfg.k
        o = 0
        C = [state[o + i * chi * chi: o + (i + 1) * chi * chi] for i in range(4)]
        o += 4 * chi * chi
        T = [state[o + i * chi * Dl * chi: o + (i + 1) * chi * Dl * chi] for i in range(4)]
        o += 4 * chi * Dl * chi
        X = state[o: o + 4 * N * k].reshape(4, N, k)
        o += 4 * N * k
        Yt = state[o: o + 4 * N * k].reshape(4, N, k)
        o += 4 * N * k
        x = int(state[o])
        C = [c[: x * x].reshape(x, x) for c in C]
        T = [t[: x * Dl * x].reshape(x, Dl, x) for t in T]
        return {"C": C, "T": T, "X": X, "Yt": Yt, "chi_env": x, "si_moves": int(state[o + 1]),
                "recycling": bool(state[o + 2]), "si_updates": int(state[o + 3])}

    def pack_state(self, C, T, X, Yt, si_moves: int = 0, recycling: bool = False,
                   si_updates: int = 0) -> np.ndarray:
        chi, Dl, N, k = self.cfg.chi, self.cfg.Dl, self.cfg.N, self.cfg.k
        x = C[0].shape[0]
        out = np.zeros(self.state_size())
        o = 0
        for c in C:
            out[o: o + x * x] = np.asarray(c).ravel()
            o += chi * chi
        for t in T:
            out[o: o + x * Dl * x] = np.asarray(t).ravel()
            o += chi * Dl * chi
        out[o: o + 4 * N * k] = np.asarray(X).ravel()
        o += 4 * N * k
        out[o: o + 4 * N * k] = np.asarray(Yt).ravel()
        o += 4 * N * k
        out[o] = x
        out[o + 1] = si_moves
        out[o + 2] = 1.0 if recycling else 0.0
        out[o + 3] = si_updates
        return out

    # profiling ---------------------------------------------------------------
    def profile(self, enable: bool):
        _check(_lib.ctm_profile(self._h, int(enable)), self._h)

    def profile_read(self) -> list:
        arr = (ctm_prof_entry * 16)()
        n = ctypes.c_int(0)
        _check(_lib.ctm_profile_read(self._h, arr, 16, ctypes.byref(n)), self._h)
        return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "ms": arr[i].ms,
                 "flops": arr[i].flops, "bytes": arr[i].bytes} for i in range(n.value)]


def converged_energy(A, cfg: Config, op, X0, Yt0, tol: float = 1e-12, max_moves: int = 400,
                     fp_tol: float = 1e-12, fp_max_iter: int = 400, bonds: str = "hv"):
    """Energy (the sum of <op> over ``bonds``; ``hvd`` for the triangular
    lattice) of the converged environment of the site tensor
    ``A`` (a float64 device tensor with ``requires_grad``), differentiable:
    the backward pass is the energy's gradient plus the fixed-point term of
    eq. implicit, computed by the library (ctm_energy_vjp,
    ctm_fixed_point_vjp) together with the value in the forward call.
    ``X0, Yt0`` are the start blocks of the SI moves (4 x N x k each)."""
    import torch

    class _ConvergedEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, site):
            c = Ctm(cfg, site.detach())
            c.set_isometries(torch.as_tensor(X0).to(site.device), torch.as_tensor(Yt0).to(site.device))
            r = c.converge(tol, max_moves)
            if not r["converged"]:
                raise CtmError(CTM_E_NOT_CONVERGED, f"no convergence in {max_moves} moves "
                                                    f"(delta {r['delta']:.2e})")
            e, grad, _ = c.energy_gradient(op, fp_tol, fp_max_iter, bonds)
            ctx.save_for_backward(grad)
            c.close()
            return torch.tensor(e, dtype=torch.float64, device=site.device)

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return g * grad

    return _ConvergedEnergy.apply(A)


def unrolled_energy(A, cfg: Config, op, state0, moves: int, bonds: str = "hv"):
    """Energy (the sum of <op> over ``bonds``, or with ``op`` a dict {bond
    letter: operator} the sum of each bond's own operator) after ``moves`` SI
    moves from ``state0`` (a
    float64 device tensor in the state layout, chi_env == chi), differentiable
    with respect to the site tensor ``A`` by unrolling: the forward pass keeps
    the state at every move boundary on the device (checkpoints), the
    backward pass runs the library's energy gradient and then ctm_move_vjp
    from each checkpoint in reverse order, recomputing each move from its
    checkpoint."""
    import torch

    class _UnrolledEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, site):
            c = Ctm(cfg, site.detach())
            c.set_state(state0.detach().cpu().numpy())
            states = [c.get_state_device()]
            for _ in range(moves):
                c.move()
                states.append(c.get_state_device())
            e, bar, site_bar = c.energy_vjp(states[-1], op, bonds=bonds)
            for st in reversed(states[:-1]):
                bar, _, site_bar = c.move_vjp(st, bar, want_out=False, site_bar=site_bar)
            ctx.save_for_backward(site_bar)
            c.close()
            return torch.tensor(e, dtype=torch.float64, device=site.device)

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return g * grad

    return _UnrolledEnergy.apply(A)


def chi_ramp(A, D: int, chis, op=None, bonds: str = "hvd", p_frac: float = 0.15, n_si: int = 2,
             tol: float = 1e-10, max_moves: int = 300, growth: str = "si", xi_iters: int = 60,
             seed: int = 0) -> list:
    """Environment dimension ramp (iPEPS benchmark section): converge the
    environment of the site tensor ``A`` (float64 device tensor, d x D^4) at
    each chi of the increasing sequence ``chis``, with the oversampling p the
    fraction ``p_frac`` of chi (rounded up), each run starting from the
    previous converged environment (its growth moves enlarge it, randomized
    when ``growth`` is ``si``).  At every chi: moves, convergence, kappa, the
    bond values of ``op`` over ``bonds`` and their sum (when ``op`` is given)
    and the correlation lengths of both transfer matrices."""
    import torch
    chis = [int(c) for c in chis]
    if any(b <= a for a, b in zip(chis, chis[1:])):
        raise ValueError("chis must increase")
    kinds = {"h": OBS_BOND_H, "v": OBS_BOND_V, "d": OBS_BOND_D, "a": OBS_BOND_AD}
    d = int(A.shape[0])
    rng = np.random.default_rng(seed)
    prev, out = None, []
    for chi in chis:
        p = max(1, int(np.ceil(p_frac * chi)))
        cfg = Config(d=d, D=D, chi=chi, p=p, n_si=n_si, growth=growth)
        c = Ctm(cfg, A)
        X = rng.standard_normal((4, cfg.N, cfg.k))
        Y = rng.standard_normal((4, cfg.N, cfg.k))
        if prev is None:
            c.set_isometries(torch.from_numpy(X).to(A.device), torch.from_numpy(Y).to(A.device))
        else:
            c.set_state(c.pack_state(prev[0], prev[1], X, Y))
        r = c.converge(tol, max_moves)
        rec = {"chi": chi, "p": p, "moves": r["moves"], "converged": r["converged"],
               "delta": r["delta"], "kappa": c.kappa()}
        if op is not None:
            for bd in bonds:
                rec["e_" + bd] = float(c.observable(kinds[bd], op)[0])
            rec["energy"] = sum(rec["e_" + bd] for bd in bonds)
        for direction in "hv":
            rec["xi_" + direction], rec["l2_" + direction] = c.correlation_length(direction, xi_iters)
        st = c.unpack_state(c.get_state())
        prev = (st["C"], st["T"])
        out.append(rec)
        c.close()
    return out


def spiral_bond_operators(h, angles) -> dict:
    """Bond operators of a single-site ansatz for a spiral state of spin 1/2:
    the site at lattice vector n carries the rotation exp(-i theta.n S^y), so
    that a translation-invariant tensor describes the spiral; every bond b
    then sees h_b = (1 x U_b) h (1 x U_b)^T with U_b the (real) rotation by
    the angle of its bond vector.  ``angles``: {bond letter: angle}; the 120
    degree order of the triangular lattice drawn on the square one with the
    diagonal bond d uses {"h": 2 pi/3, "v": 2 pi/3, "d": 4 pi/3}."""
    h = np.asarray(h, dtype=np.float64)
    out = {}
    for bd, th in angles.items():
        U = np.array([[np.cos(th / 2), -np.sin(th / 2)], [np.sin(th / 2), np.cos(th / 2)]])
        K = np.kron(np.eye(2), U)
        out[bd] = K @ h @ K.T
    return out


def optimize_lbfgs(A0, cfg: Config, bond_ops: dict, iterations: int = 10, tol: float = 1e-10,
                   max_moves: int = 300, fp_tol: float = 1e-10, fp_max_iter: int = 400,
                   history_size: int = 10, X0=None, Yt0=None) -> tuple:
    """Variational optimisation of a single-site tensor (the optimisation
    loop of the paper: L-BFGS over the site tensor, the energy of the
    converged environment and its gradient from the fixed-point adjoint,
    eq. implicit).  Each evaluation starts its CTMRG from the previous
    converged environment and SI blocks (recycling); the first from ``X0,
    Yt0`` (4 x N x k) or the library's start blocks.  ``bond_ops``: {bond
    letter: operator}, e.g. from :func:`spiral_bond_operators`.  Returns the
    optimised tensor (device) and the history of (energy, gradient norm,
    CTMRG moves, the evaluated site tensor as a host array) per evaluation."""
    import torch
    A = A0.detach().clone().to(torch.float64).requires_grad_(True)
    opt = torch.optim.LBFGS([A], lr=1.0, max_iter=iterations, history_size=history_size,
                            line_search_fn="strong_wolfe", tolerance_grad=1e-12,
                            tolerance_change=1e-14)
    prev = {"state": None}
    history = []

    def closure():
        opt.zero_grad()
        c = Ctm(cfg, A.detach())
        if prev["state"] is not None:
            c.set_state(prev["state"])
        elif X0 is not None:
            c.set_isometries(torch.as_tensor(X0).to(A.device), torch.as_tensor(Yt0).to(A.device))
        r = c.converge(tol, max_moves)
        e, grad, _ = c.energy_gradient(bond_ops, fp_tol, fp_max_iter)
        prev["state"] = c.get_state()
        c.close()
        A.grad = grad.detach().clone()
        history.append((e, float(grad.norm()), r["moves"], A.detach().cpu().numpy().copy()))
        return torch.tensor(e, dtype=torch.float64)

    opt.step(closure)
    return A.detach(), history


BOND_BITS = {"h": 1, "v": 2, "d": 4, "a": 8}


def bond_mask(bonds: str) -> int:
    """Mask of the bonds named by the letters h, v, d (diagonal), a (anti-diagonal)."""
    if not bonds or any(c not in BOND_BITS for c in bonds):
        raise ValueError(f"bonds must be letters of 'hvda', got {bonds!r}")
    m = 0
    for c in bonds:
        m |= BOND_BITS[c]
    return m


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


class Server:
    """Continuous batching of environment solves (see ctm_server_* in include/ctm.h)."""

    STATES = ("queued", "running", "done", "failed")

    def __init__(self, arena_bytes: int, max_slots: int, batch_max_n: int = 0):
        self._h = _vp()
        st = _lib.ctm_server_create(ctypes.byref(self._h), int(arena_bytes), int(max_slots))
        if st != CTM_OK:
            raise CtmError(st, "ctm_server_create failed")
        if batch_max_n:
            _check(_lib.ctm_server_batching(self._h, int(batch_max_n)))

    def submit(self, cfg: Config, site, boundary=None, X0=None, Yt0=None, op=None,
               tol: float = 1e-10, max_moves: int = 100) -> int:
        c = cfg.c()
        keep = [_dptr(site), _dptr(boundary), _dptr(X0), _dptr(Yt0), _dptr(op)]
        rid = ctypes.c_int(-1)
        st = _lib.ctm_server_submit(self._h, ctypes.byref(c), *[p for _, p in keep], float(tol),
                                    int(max_moves), ctypes.byref(rid))
        if st != CTM_OK:
            raise CtmError(st, "ctm_server_submit rejected the request")
        return rid.value

    def pump(self):
        run, queued = ctypes.c_int(0), ctypes.c_int(0)
        _check(_lib.ctm_server_pump(self._h, ctypes.byref(run), ctypes.byref(queued)))
        return run.value, queued.value

    def result(self, rid: int) -> dict:
        r = ctm_result()
        _check(_lib.ctm_server_result(self._h, int(rid), ctypes.byref(r)))
        out = {f: getattr(r, f) for f, _ in ctm_result._fields_}
        out["state"] = self.STATES[r.state]
        if r.state == 3:
            out["error"] = _lib.ctm_server_error(self._h, int(rid)).decode()
        return out

    def clock(self) -> float:
        return _lib.ctm_server_clock(self._h)

    def close(self):
        if self._h:
            _lib.ctm_server_destroy(self._h)
            self._h = _vp()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        self.close()


def move_batch(ctxs: Sequence["Ctm"]) -> list:
    """One move of every context, SI moves of float64 contexts batched into
    grouped launches (ctm_move_batch); returns each move's info."""
    n = len(ctxs)
    hs = (_vp * n)(*[c._h for c in ctxs])
    infos = (ctm_move_info * n)()
    st = _lib.ctm_move_batch(hs, n, infos)
    if st != CTM_OK:
        raise CtmError(st, _lib.ctm_last_error(None).decode())
    return [{"delta": i.delta, "mode": i.mode, "chi_env": i.chi_env, "gap": i.gap,
             "n_si": i.n_si, "sin2": i.sin2} for i in infos]


def gemm_f64(A: Sequence, B: Sequence, C: Sequence, M, N, K, trans_a=0, lda=None, ldb=None,
             ldc=None, alpha=1.0, accumulate=0, stream=None):
    lda = (M if trans_a else K) if lda is None else lda
    ldb = N if ldb is None else ldb
    ldc = N if ldc is None else ldc
    _check(_lib.ctm_gemm_f64(len(A), _ptr_array(A), _ptr_array(B), _ptr_array(C), M, N, K,
                             trans_a, lda, ldb, ldc, alpha, accumulate, _stream(stream)))


def gemm_f64_split_scratch_bytes() -> int:
    return int(_lib.ctm_gemm_f64_split_scratch_bytes())


def gemm_f64_split(A: Sequence, B: Sequence, C: Sequence, M, N, K, trans_a: Sequence, scratch,
                   ncu=256, lda=None, ldb=None, ldc=None, alpha=1.0, accumulate=0,
                   stream=None) -> bool:
    """The SI product split evenly over ncu CUs; returns whether the split
    ran (else the plain tile kernel did)."""
    tr = (ctypes.c_int * len(A))(*[int(t) for t in trans_a])
    if lda is None:
        if len(set(int(t) for t in trans_a)) > 1 and M != K:
            raise ValueError("mixed trans_a with M != K needs an explicit lda")
        lda = M if trans_a[0] else K
    ldb = N if ldb is None else ldb
    ldc = N if ldc is None else ldc
    used = ctypes.c_int(0)
    sp = None if scratch is None else ctypes.c_void_p(scratch.data_ptr())
    sb = 0 if scratch is None else scratch.numel() * scratch.element_size()
    _check(_lib.ctm_gemm_f64_split(len(A), _ptr_array(A), _ptr_array(B), _ptr_array(C), M, N, K,
                                   tr, lda, ldb, ldc, alpha, accumulate, sp, sb, ncu,
                                   ctypes.byref(used), _stream(stream)))
    return bool(used.value)


def qr_f64(W: Sequence, stream=None):
    """In-place thin Householder QR (R_ii >= 0) of N x k device matrices."""
    N, k = W[0].shape
    _check(_lib.ctm_qr_f64(len(W), _ptr_array(W), N, k, _stream(stream)))


def qr_f64_noalloc(W: Sequence, stream=None):
    """As :func:`qr_f64`, with the library's static scratch (no allocation,
    no synchronisation)."""
    N, k = W[0].shape
    _check(_lib.ctm_qr_f64_noalloc(len(W), _ptr_array(W), N, k, _stream(stream)))


def svd_f64(rho: Sequence, u: Sequence, s: Sequence, v: Sequence, stream=None):
    n = rho[0].shape[0]
    _check(_lib.ctm_svd_f64(len(rho), _ptr_array(rho), None if u is None else _ptr_array(u),
                            _ptr_array(s), None if v is None else _ptr_array(v), n,
                            _stream(stream)))


# ---------------------------------------------------------------------------
# unit cells (ctm_cell_* of include/ctm.h)
# ---------------------------------------------------------------------------
def _check_cell(status: int, h=None):
    if status != CTM_OK:
        raise CtmError(status, _lib.ctm_cell_last_error(h).decode())
    return status


@dataclass
class CellConfig:
    Lx: int
    Ly: int
    d: int
    D: int
    chi: int
    p: int = 8
    n_si: int = 2
    stabilized: int = 1
    pinv_rtol: float = 1e-12

    @property
    def Dl(self) -> int:
        return self.D * self.D if self.d > 0 else self.D

    @property
    def N(self) -> int:
        return self.chi * self.Dl

    @property
    def k(self) -> int:
        return min(self.chi + self.p, self.N)

    @property
    def ns(self) -> int:
        return self.Lx * self.Ly

    def c(self) -> ctm_cell_config:
        return ctm_cell_config(self.Lx, self.Ly, self.d, self.D, self.chi, self.p, self.n_si,
                               self.stabilized, self.pinv_rtol)


def cell_workspace_bytes(cfg: CellConfig) -> int:
    n = ctypes.c_size_t(0)
    _check_cell(_lib.ctm_cell_workspace_bytes(ctypes.byref(cfg.c()), ctypes.byref(n)))
    return int(n.value)


class Cell:
    """CTMRG of an Lx x Ly unit cell on the GPU.

    ``sites``: a float64 device tensor of the Lx*Ly site tensors, site
    (x, y) at index y*Lx + x (A[s, u, l, d, r], or a[u, l, d, r] when
    d == 0); ``boundary``: None or a device tensor [Lx*Ly, 4, Dl] of the
    vectors that close legs u, l, d, r of each site in its neighbours'
    initial environments."""

    def __init__(self, cfg: CellConfig, sites, boundary=None):
        self.cfg = cfg
        self._h = _vp()
        self._keep = (sites.contiguous(), None if boundary is None else boundary.contiguous())
        torch.cuda.synchronize()   # the cell copies the inputs on its own stream
        _check_cell(_lib.ctm_cell_create(ctypes.byref(self._h), ctypes.byref(cfg.c()),
                                         self._keep[0].data_ptr(),
                                         None if boundary is None else self._keep[1].data_ptr()))

    def close(self):
        if self._h:
            _lib.ctm_cell_destroy(self._h)
            self._h = _vp()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        self.close()

    def set_blocks(self, X, Yt):
        """Start blocks [4, Lx*Ly, N, k] (device tensors) of every cut."""
        X, Yt = X.contiguous(), Yt.contiguous()
        torch.cuda.synchronize()
        _check_cell(_lib.ctm_cell_set_blocks(self._h, X.data_ptr(), Yt.data_ptr()), self._h)

    def iterate(self, mode: str = "si") -> float:
        delta = ctypes.c_double(0.0)
        _check_cell(_lib.ctm_cell_iterate(self._h, CELL_MODE[mode], ctypes.byref(delta)), self._h)
        return float(delta.value)

    def run(self, warmup: int, tol: float, max_iter: int, warm_mode: str = "rsvd") -> dict:
        iters = ctypes.c_int(0)
        deltas = (ctypes.c_double * max(1, max_iter))()
        kinds = (ctypes.c_int * max(1, max_iter))()
        st = _lib.ctm_cell_run(self._h, warmup, CELL_MODE[warm_mode], tol, max_iter,
                               ctypes.byref(iters), deltas, kinds)
        if st not in (CTM_OK, CTM_E_NOT_CONVERGED):
            _check_cell(st, self._h)
        n = iters.value
        names = {CELL_RSVD: "rsvd", CELL_SI: "si", CELL_SVD: "svd"}
        return {"iters": n, "converged": st == CTM_OK, "deltas": list(deltas[:n]),
                "kinds": [names[k] for k in kinds[:n]]}

    def _env_size(self) -> int:
        n = ctypes.c_size_t(0)
        _check_cell(_lib.ctm_cell_env_size(self._h, ctypes.byref(n)), self._h)
        return int(n.value)

    def get_env(self) -> dict:
        """{(x, y): (C1..C4, T1..T4)} as numpy arrays of their own shapes."""
        cfg = self.cfg
        n = self._env_size()
        buf = np.zeros(n)
        dims = (ctypes.c_int * (16 * cfg.ns))()
        _check_cell(_lib.ctm_cell_get_env(self._h, buf.ctypes.data_as(_dp), n, dims), self._h)
        chi, Dl = cfg.chi, cfg.Dl
        out, off = {}, 0
        for s in range(cfg.ns):
            C, T = [], []
            for i in range(4):
                r, c = dims[16 * s + 2 * i], dims[16 * s + 2 * i + 1]
                C.append(buf[off:off + r * c].reshape(r, c).copy())
                off += chi * chi
            for i in range(4):
                a, b = dims[16 * s + 8 + 2 * i], dims[16 * s + 9 + 2 * i]
                T.append(buf[off:off + a * Dl * b].reshape(a, Dl, b).copy())
                off += chi * Dl * chi
            out[(s % cfg.Lx, s // cfg.Lx)] = (C, T)
        return out

    def set_env(self, env: dict):
        cfg = self.cfg
        chi, Dl = cfg.chi, cfg.Dl
        buf = np.zeros(self._env_size())
        dims = (ctypes.c_int * (16 * cfg.ns))()
        off = 0
        for s in range(cfg.ns):
            C, T = env[(s % cfg.Lx, s // cfg.Lx)]
            for i in range(4):
                r, c = C[i].shape
                buf[off:off + r * c] = np.ascontiguousarray(C[i]).ravel()
                dims[16 * s + 2 * i], dims[16 * s + 2 * i + 1] = r, c
                off += chi * chi
            for i in range(4):
                a, _, b = T[i].shape
                buf[off:off + a * Dl * b] = np.ascontiguousarray(T[i]).ravel()
                dims[16 * s + 8 + 2 * i], dims[16 * s + 9 + 2 * i] = a, b
                off += chi * Dl * chi
        _check_cell(_lib.ctm_cell_set_env(self._h, buf.ctypes.data_as(_dp), buf.size, dims),
                    self._h)

    # --- state vector and adjoint ------------------------------------------
    def state_size(self) -> int:
        n = ctypes.c_size_t(0)
        _check_cell(_lib.ctm_cell_state_size(self._h, ctypes.byref(n)), self._h)
        return int(n.value)

    def get_state_device(self):
        """The state vector (environment of dimension chi and the blocks the
        next SI iteration starts from) as a float64 device tensor."""
        out = torch.empty(self.state_size(), dtype=torch.float64, device=self._keep[0].device)
        torch.cuda.synchronize()
        _check_cell(_lib.ctm_cell_get_state_device(self._h, out.data_ptr(), out.numel()), self._h)
        return out

    def set_state_device(self, state):
        state = state.contiguous()
        torch.cuda.synchronize()
        _check_cell(_lib.ctm_cell_set_state_device(self._h, state.data_ptr(), state.numel()),
                    self._h)

    def site_size(self) -> int:
        cfg = self.cfg
        return cfg.ns * (cfg.d * cfg.D ** 4 if cfg.d > 0 else cfg.Dl ** 4)

    def move_vjp(self, state, bar=None, site_bar=None, want_out=True):
        """One SI iteration from ``state`` (device tensor): returns
        (state_out or None, state_bar or None, site_bar); with ``bar`` the
        cotangent of the output state, ``site_bar`` (created when None)
        accumulates the site tensors' cotangent."""
        state = state.contiguous()
        dev = state.device
        out = torch.empty_like(state) if want_out else None
        sbar = None
        if bar is not None:
            bar = bar.contiguous()
            sbar = torch.empty_like(state)
            if site_bar is None:
                site_bar = torch.zeros(self.site_size(), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        _check_cell(_lib.ctm_cell_move_vjp(
            self._h, state.data_ptr(), None if bar is None else bar.data_ptr(),
            None if sbar is None else sbar.data_ptr(),
            None if site_bar is None else site_bar.data_ptr(),
            None if out is None else out.data_ptr()), self._h)
        return out, sbar, site_bar

    def energy_vjp(self, state, ops: dict, grad: bool = True, site_bar=None):
        """Energy per site sum over the bonds in ``ops`` ({'h'|'v'|'d':
        operator d^2 x d^2}); with ``grad`` also (state_bar, site_bar)."""
        d = self.cfg.d
        mask, buf = 0, np.zeros((3, d * d, d * d))
        for b, name in enumerate("hvd"):
            if name in ops:
                mask |= 1 << b
                buf[b] = np.asarray(ops[name], dtype=np.float64)
        state = state.contiguous()
        e = ctypes.c_double(0.0)
        sbar = torch.empty_like(state) if grad else None
        if grad and site_bar is None:
            site_bar = torch.zeros(self.site_size(), dtype=torch.float64, device=state.device)
        torch.cuda.synchronize()
        _check_cell(_lib.ctm_cell_energy_vjp(
            self._h, state.data_ptr(), buf.ctypes.data_as(_dp), mask, ctypes.byref(e),
            None if sbar is None else sbar.data_ptr(),
            None if not grad else site_bar.data_ptr()), self._h)
        return (float(e.value), sbar, site_bar) if grad else float(e.value)

    def get_blocks(self):
        cfg = self.cfg
        X = np.zeros((4, cfg.ns, cfg.N, cfg.k))
        Y = np.zeros_like(X)
        _check_cell(_lib.ctm_cell_get_blocks(self._h, X.ctypes.data_as(_dp), Y.ctypes.data_as(_dp)),
                    self._h)
        return X, Y


def unrolled_cell_energy(sites, cfg: CellConfig, ops: dict, state0, moves: int):
    """Energy per site of the cell (bonds and operators in ``ops``) after
    ``moves`` SI iterations from ``state0`` (a float64 device state vector of
    a cell environment of dimension chi), differentiable with respect to the
    stacked site tensors ``sites`` ([Lx*Ly, d, D, D, D, D], site (x, y) at
    y*Lx + x) by unrolling: the forward pass keeps the state at every
    iteration boundary on the device (checkpoints), the backward pass takes
    the energy's gradient and then the adjoint of every iteration from its
    checkpoint in reverse order, recomputing each iteration there."""

    class _Unrolled(torch.autograd.Function):
        @staticmethod
        def forward(ctx, site):
            c = Cell(cfg, site.detach())
            c.set_state_device(state0.detach())
            states = [state0.detach().clone()]
            for _ in range(moves):
                c.iterate("si")
                states.append(c.get_state_device())
            e, bar, site_bar = c.energy_vjp(states[-1], ops)
            for st in reversed(states[:-1]):
                _, bar, site_bar = c.move_vjp(st, bar, site_bar, want_out=False)
            ctx.save_for_backward(site_bar.reshape(site.shape))
            c.close()
            return torch.tensor(e, dtype=torch.float64, device=site.device)

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return g * grad

    return _Unrolled.apply(sites)
