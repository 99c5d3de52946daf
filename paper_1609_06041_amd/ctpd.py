"""Python binding of libctpd (the C ABI declared in include/ctpd.h).

Argument marshalling only: tensors are checked for dtype, device, shape and
contiguity, and their device pointers go straight to the library; every step
of the computation runs in the HIP kernels.  The library is required -- if
``libctpd.so`` is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_void_p

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctpd.so")

CTPD_OK, CTPD_EINVAL, CTPD_EDOMAIN, CTPD_EHIP, CTPD_ENOMEM = 0, -1, -2, -3, -4
MAX_BINS = 4096

# Every symbol the header declares, with its ctypes signature.
_SIGNATURES = {
    "ctpd_op_create": (c_int, [c_void_p, c_void_p, POINTER(c_void_p)]),
    "ctpd_op_destroy": (None, [c_void_p]),
    "ctpd_project": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ctpd_backproject": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ctpd_ramp_filter": (c_int, [c_void_p, c_double, c_double, c_void_p, c_void_p]),
    "ctpd_ramp_filter_f64": (c_int, [c_void_p, c_double, c_double, c_void_p, c_void_p]),
    "ctpd_filter_taps": (c_int, [c_void_p, c_double, c_double, POINTER(c_double)]),
    "ctpd_tv_prox": (c_int, [c_void_p, c_void_p, c_double, c_int32, c_double, c_void_p, c_void_p]),
    "ctpd_pd_lowdose_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p,
                                      c_void_p]),
    "ctpd_pd_fewview_solve": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "ctpd_pd_fewview_eps_solve": (c_int, [c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p, c_void_p]),
    "ctpd_app_identity_lowdose_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p,
                                                c_void_p, c_void_p]),
    "ctpd_gist_lowdose_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p,
                                        c_void_p]),
    "ctpd_cp_fewview_solve": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "ctpd_batch_create": (c_int, [c_void_p, c_int32, c_void_p, POINTER(c_void_p)]),
    "ctpd_batch_destroy": (None, [c_void_p]),
    "ctpd_batch_lowdose_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                         c_void_p]),
    "ctpd_unrolled_ckpt_floats": (c_int, [c_void_p, c_int32, POINTER(ctypes.c_size_t)]),
    "ctpd_unrolled_lowdose_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_double, c_int32,
                                              c_void_p, c_void_p, c_void_p]),
    "ctpd_unrolled_lowdose_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_double, c_int32,
                                               c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "ctpd_unrolled_lowdose_forward_many": (c_int, [c_int32, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                                   POINTER(c_double), POINTER(c_double), c_int32, c_void_p, c_void_p,
                                                   c_void_p]),
    "ctpd_unrolled_lowdose_backward_many": (c_int, [c_int32, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                                    POINTER(c_double), POINTER(c_double), c_int32, c_void_p,
                                                    c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    "ctpd_batch_set_tiles": (c_int, [c_void_p, c_void_p]),
    "ctpd_batch_get_tiles": (c_int, [c_void_p, c_void_p]),
    "ctpd_batch_time_loop": (c_int, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_double)]),
    "ctpd_strerror": (ctypes.c_char_p, [c_int]),
}


class CtpdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ctpd error {code}: {msg}")
        self.code = code


class Geometry(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_views", c_int32), ("n_bins", c_int32), ("reserved", c_int32),
                ("angles", POINTER(c_double))]


def _geometry(n, m, nb, angles):
    """(Geometry, keep-alive) for the C call; angles: None or m view angles in radians."""
    if angles is None:
        return Geometry(n, m, nb, 0, None), None
    a = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).reshape(-1))
    if a.shape != (m,):
        raise ValueError(f"need {m} view angles, got {a.shape}")
    return Geometry(n, m, nb, 0, a.ctypes.data_as(POINTER(c_double))), a


class Params(ctypes.Structure):
    _fields_ = [("tau", c_double), ("sigma", c_double), ("tv_step", c_double), ("safety", c_double),
                ("tv_iters", c_int32), ("norm_steps", c_int32), ("record_cost", c_int32), ("reserved", c_int32),
                ("state", c_void_p)]


class State(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("mu", c_void_p), ("mu_prev", c_void_p), ("p", c_void_p), ("y", c_void_p),
                ("k", c_int32), ("reserved", c_int32), ("tau", c_double), ("sigma", c_double)]


class Checkpoint:
    """The iterate state (x^k, mu^k, mu^{k-1}, p^k[, y^k]) of an APP solve in
    device tensors.  Passed as ``state=`` to ``lowdose_solve``, ``fewview_solve``
    or ``fewview_eps_solve``, the solve starts from it (the zero start while
    ``k == 0``) and writes its end state back, so K1 iterations followed by K2
    more equal K1 + K2 iterations of one solve bit for bit."""

    def __init__(self, op: "Operator", with_y: bool = False):
        z = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=op.device)
        self.shape = (op.n, op.m, op.nb)
        self.x = z(op.n, op.n)
        self.mu = z(op.m, op.nb)
        self.mu_prev = z(op.m, op.nb)
        self.p = z(2, op.n, op.n)
        self.y = z(op.m, op.nb) if with_y else None
        self.k, self.tau, self.sigma = 0, 0.0, 0.0

    def _struct(self, op: "Operator") -> State:
        if self.shape != (op.n, op.m, op.nb):
            raise ValueError(f"checkpoint of shape {self.shape} for an operator of {(op.n, op.m, op.nb)}")
        ptr = lambda t: None if t is None else c_void_p(t.data_ptr())
        return State(x=ptr(self.x), mu=ptr(self.mu), mu_prev=ptr(self.mu_prev), p=ptr(self.p), y=ptr(self.y),
                     k=int(self.k), reserved=0, tau=float(self.tau), sigma=float(self.sigma))

    def _absorb(self, st: State) -> None:
        self.k, self.tau, self.sigma = int(st.k), float(st.tau), float(st.sigma)


class BatchTiles(ctypes.Structure):
    _fields_ = [("placement", c_int32), ("tv_threads", c_int32), ("fwd_form", c_int32), ("reserved", c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("tau", c_double), ("sigma", c_double), ("kappa", c_double), ("lambda_a", c_double),
                ("lambda_h", c_double), ("norm_steps_a", c_int32), ("norm_steps_h", c_int32),
                ("iters_done", c_int32), ("reserved", c_int32), ("setup_ms", c_double), ("loop_ms", c_double),
                ("cost", POINTER(c_double)), ("mu_out", c_void_p), ("p_out", c_void_p),
                ("gap", POINTER(c_double)), ("resid", POINTER(c_double)), ("rmse", POINTER(c_double)),
                ("x_ref", c_void_p)]


MONITORS = ("gap", "resid", "rmse")


_lib = None


def load() -> ctypes.CDLL:
    """Load libctpd.so (raises CtpdError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CtpdError(CTPD_EHIP, f"{LIB_PATH} is not built; run `python -m paper_1609_06041_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(code: int) -> None:
    if code != CTPD_OK:
        msg = load().ctpd_strerror(code)
        raise CtpdError(code, msg.decode() if msg else "?")


def _ptr(t: torch.Tensor, shape, name: str) -> c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return c_void_p(t.data_ptr())


def _ptr64(t: torch.Tensor, shape, name: str) -> c_void_p:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 torch.Tensor")
    if t.device.type != "cuda" or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous GPU tensor of shape {tuple(shape)}")
    return c_void_p(t.data_ptr())


def _params(tau, sigma, tv_iters, tv_step, safety, norm_steps, record_cost) -> Params:
    return Params(tau=float(tau or 0.0), sigma=float(sigma or 0.0), tv_step=float(tv_step or 0.0),
                  safety=float(safety or 0.0), tv_iters=int(tv_iters or 0), norm_steps=int(norm_steps or 0),
                  record_cost=1 if record_cost else 0, reserved=0, state=None)


class Operator:
    """A scan geometry (n x n image, n_views x n_bins sinogram) bound to a stream."""

    def __init__(self, n: int, n_views: int, n_bins: int, stream: torch.cuda.Stream | None = None,
                 angles=None):
        """angles: None (theta_v = v pi / n_views) or n_views view angles in radians."""
        self.n, self.m, self.nb = int(n), int(n_views), int(n_bins)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        geo, keep = _geometry(self.n, self.m, self.nb, angles)
        self.angles = None if keep is None else keep.copy()
        h = c_void_p()
        with torch.cuda.device(self.device):
            _check(load().ctpd_op_create(byref(geo), c_void_p(self.stream.cuda_stream), byref(h)))
        self._h = h

    # -- lifetime --------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ctpd_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers ---------------------------------------------------------
    def _img(self):
        return torch.empty((self.n, self.n), dtype=torch.float32, device=self.device)

    def _sino(self):
        return torch.empty((self.m, self.nb), dtype=torch.float32, device=self.device)

    # -- single operators --------------------------------------------------
    def project(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._sino() if out is None else out
        _check(load().ctpd_project(self._h, _ptr(x, (self.n, self.n), "x"), _ptr(out, (self.m, self.nb), "out")))
        return out

    def backproject(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._img() if out is None else out
        _check(load().ctpd_backproject(self._h, _ptr(y, (self.m, self.nb), "y"), _ptr(out, (self.n, self.n), "out")))
        return out

    def ramp_filter(self, s: torch.Tensor, tau: float, kappa: float = 0.0,
                    out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._sino() if out is None else out
        _check(load().ctpd_ramp_filter(self._h, float(tau), float(kappa), _ptr(s, (self.m, self.nb), "s"),
                                       _ptr(out, (self.m, self.nb), "out")))
        return out

    def ramp_filter_f64(self, s: torch.Tensor, tau: float, kappa: float = 0.0,
                        out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty((self.m, self.nb), dtype=torch.float64, device=self.device) if out is None else out
        _check(load().ctpd_ramp_filter_f64(self._h, float(tau), float(kappa), _ptr64(s, (self.m, self.nb), "s"),
                                           _ptr64(out, (self.m, self.nb), "out")))
        return out

    def filter_taps(self, tau: float, kappa: float = 0.0) -> np.ndarray:
        taps = np.zeros(2 * self.nb - 1, dtype=np.float64)
        _check(load().ctpd_filter_taps(self._h, float(tau), float(kappa),
                                       taps.ctypes.data_as(POINTER(c_double))))
        return taps

    def tv_prox(self, z: torch.Tensor, lam: float, p: torch.Tensor | None = None, n_iter: int = 10,
                tv_step: float = 0.125, out: torch.Tensor | None = None):
        """Returns (x, p); p (shape [2, n, n]) is updated in place when given."""
        if p is None:
            p = torch.zeros((2, self.n, self.n), dtype=torch.float32, device=self.device)
        out = self._img() if out is None else out
        _check(load().ctpd_tv_prox(self._h, _ptr(z, (self.n, self.n), "z"), float(lam), int(n_iter),
                                   float(tv_step), _ptr(p, (2, self.n, self.n), "p"),
                                   _ptr(out, (self.n, self.n), "out")))
        return out, p

    # -- solvers -------------------------------------------------------------
    def _report(self, iters, record_cost, return_state, monitors=(), x_ref=None):
        """monitors: names from MONITORS to record per iteration; x_ref: the
        reference image of the rmse monitor."""
        rep = Report()
        cost = None
        if record_cost and iters > 0:
            cost = np.zeros(iters, dtype=np.float64)
            rep.cost = cost.ctypes.data_as(POINTER(c_double))
        state = {}
        for name in monitors:
            if name not in MONITORS:
                raise ValueError(f"unknown monitor {name!r}; choose from {MONITORS}")
            arr = np.zeros(max(iters, 1), dtype=np.float64)
            setattr(rep, name, arr.ctypes.data_as(POINTER(c_double)))
            state[name] = arr
        if x_ref is not None:
            rep.x_ref = _ptr(x_ref, (self.n, self.n), "x_ref")
            state["_x_ref"] = x_ref   # keeps the tensor alive for the call
        if return_state:
            state["mu"] = self._sino()
            state["p"] = torch.empty((2, self.n, self.n), dtype=torch.float32, device=self.device)
            rep.mu_out = c_void_p(state["mu"].data_ptr())
            rep.p_out = c_void_p(state["p"].data_ptr())
        return rep, cost, state

    def checkpoint(self, with_y: bool = False) -> Checkpoint:
        """A zero-start checkpoint for this geometry (with_y: for fewview_eps_solve)."""
        return Checkpoint(self, with_y)

    def _attach(self, prm: Params, state: "Checkpoint | None"):
        if state is None:
            return None
        cst = state._struct(self)
        prm.state = ctypes.cast(ctypes.pointer(cst), c_void_p)
        return cst

    @staticmethod
    def _info(rep: Report, cost, state) -> dict:
        info = {k: getattr(rep, k) for k in ("tau", "sigma", "kappa", "lambda_a", "lambda_h", "norm_steps_a",
                                            "norm_steps_h", "iters_done", "setup_ms", "loop_ms")}
        if cost is not None:
            info["cost"] = cost
        info.update({k: v for k, v in state.items() if not k.startswith("_")})
        return info

    def lowdose_solve(self, b: torch.Tensor, w: torch.Tensor, beta: float, iters: int, *, tau=None, sigma=None,
                      tv_iters=10, tv_step=0.125, safety=0.95, norm_steps=100, record_cost=False,
                      return_state=False, monitors=(), x_ref=None,
                      state: Checkpoint | None = None, out: torch.Tensor | None = None):
        """Algorithm 1 (beta > 0) / 1' (beta = 0).  Returns (x, info)."""
        out = self._img() if out is None else out
        prm = _params(tau, sigma, tv_iters, tv_step, safety, norm_steps, record_cost)
        rep, cost, extra = self._report(iters, record_cost, return_state, monitors, x_ref)
        cst = self._attach(prm, state)
        _check(load().ctpd_pd_lowdose_solve(self._h, _ptr(b, (self.m, self.nb), "b"),
                                            _ptr(w, (self.m, self.nb), "w"), float(beta), int(iters),
                                            byref(prm), _ptr(out, (self.n, self.n), "out"), byref(rep)))
        if state is not None:
            state._absorb(cst)
        return out, self._info(rep, cost, extra)

    def app_identity_lowdose_solve(self, b: torch.Tensor, w: torch.Tensor, beta: float, iters: int, *, tau=None,
                                   sigma=None, tv_iters=10, tv_step=0.125, safety=0.95, norm_steps=100,
                                   record_cost=False, return_state=False, monitors=(), x_ref=None,
                                   out: torch.Tensor | None = None):
        """Algorithm 1 with D = I (the unpreconditioned ablation).  Returns (x, info)."""
        out = self._img() if out is None else out
        prm = _params(tau, sigma, tv_iters, tv_step, safety, norm_steps, record_cost)
        rep, cost, state = self._report(iters, record_cost, return_state, monitors, x_ref)
        _check(load().ctpd_app_identity_lowdose_solve(self._h, _ptr(b, (self.m, self.nb), "b"),
                                                      _ptr(w, (self.m, self.nb), "w"), float(beta), int(iters),
                                                      byref(prm), _ptr(out, (self.n, self.n), "out"), byref(rep)))
        return out, self._info(rep, cost, state)

    def fewview_solve(self, b: torch.Tensor, iters: int, *, tau=None, sigma=None, tv_iters=10, tv_step=0.125,
                      safety=0.95, norm_steps=100, record_cost=False, return_state=False,
                      monitors=(), x_ref=None,
                      state: Checkpoint | None = None, out: torch.Tensor | None = None):
        """Algorithm 2.  Returns (x, info)."""
        out = self._img() if out is None else out
        prm = _params(tau, sigma, tv_iters, tv_step, safety, norm_steps, record_cost)
        rep, cost, extra = self._report(iters, record_cost, return_state, monitors, x_ref)
        cst = self._attach(prm, state)
        _check(load().ctpd_pd_fewview_solve(self._h, _ptr(b, (self.m, self.nb), "b"), int(iters), byref(prm),
                                            _ptr(out, (self.n, self.n), "out"), byref(rep)))
        if state is not None:
            state._absorb(cst)
        return out, self._info(rep, cost, extra)

    def fewview_eps_solve(self, b: torch.Tensor, eps: float, iters: int, *, tau=None, sigma=None, tv_iters=10,
                          tv_step=0.125, safety=0.95, norm_steps=100, record_cost=False, return_state=False,
                          monitors=(), x_ref=None, state: Checkpoint | None = None, out: torch.Tensor | None = None):
        """Error-tolerant few-view solve: min psi(x) s.t. ||Ax - b|| <= eps, x >= 0.  Returns (x, info)."""
        out = self._img() if out is None else out
        prm = _params(tau, sigma, tv_iters, tv_step, safety, norm_steps, record_cost)
        rep, cost, extra = self._report(iters, record_cost, return_state, monitors, x_ref)
        cst = self._attach(prm, state)
        _check(load().ctpd_pd_fewview_eps_solve(self._h, _ptr(b, (self.m, self.nb), "b"), float(eps), int(iters),
                                                byref(prm), _ptr(out, (self.n, self.n), "out"), byref(rep)))
        if state is not None:
            state._absorb(cst)
        return out, self._info(rep, cost, extra)

    def gist_lowdose_solve(self, b: torch.Tensor, w: torch.Tensor, beta: float, iters: int, *, gamma=None,
                           lam=None, safety=0.95, norm_steps=100, record_cost=False, return_state=False,
                           monitors=(), x_ref=None,
                           out: torch.Tensor | None = None):
        """GIST comparator for Eq. 1 (no preconditioner).  Returns (x, info); info['tau'] is gamma."""
        out = self._img() if out is None else out
        prm = _params(gamma, lam, 0, 0, safety, norm_steps, record_cost)
        rep, cost, state = self._report(iters, record_cost, return_state, monitors, x_ref)
        _check(load().ctpd_gist_lowdose_solve(self._h, _ptr(b, (self.m, self.nb), "b"),
                                              _ptr(w, (self.m, self.nb), "w"), float(beta), int(iters),
                                              byref(prm), _ptr(out, (self.n, self.n), "out"), byref(rep)))
        return out, self._info(rep, cost, state)

    def cp_fewview_solve(self, b: torch.Tensor, iters: int, *, t=None, s=None, safety=0.95, norm_steps=100,
                         record_cost=False, return_state=False, monitors=(), x_ref=None,
                         out: torch.Tensor | None = None):
        """Chambolle-Pock comparator for the few-view problem.  Returns (x, info)."""
        out = self._img() if out is None else out
        prm = _params(t, s, 0, 0, safety, norm_steps, record_cost)
        rep, cost, state = self._report(iters, record_cost, return_state, monitors, x_ref)
        _check(load().ctpd_cp_fewview_solve(self._h, _ptr(b, (self.m, self.nb), "b"), int(iters), byref(prm),
                                            _ptr(out, (self.n, self.n), "out"), byref(rep)))
        return out, self._info(rep, cost, state)


    # -- unrolled Algorithm 1 (forward with checkpoints, reverse pass) -------------
    def ckpt_floats(self, iters: int) -> int:
        cnt = ctypes.c_size_t()
        _check(load().ctpd_unrolled_ckpt_floats(self._h, int(iters), byref(cnt)))
        return int(cnt.value)

    def unrolled_forward(self, b, w, beta, tau, sigma, iters, ckpt, *, tv_iters=10, tv_step=0.125, out=None):
        out = self._img() if out is None else out
        prm = _params(None, None, tv_iters, tv_step, None, None, False)
        if ckpt.dtype != torch.float32 or ckpt.numel() < self.ckpt_floats(iters) or not ckpt.is_contiguous():
            raise ValueError("checkpoint buffer too small or not contiguous float32")
        _check(load().ctpd_unrolled_lowdose_forward(self._h, _ptr(b, (self.m, self.nb), "b"),
                                                    _ptr(w, (self.m, self.nb), "w"), float(beta), float(tau),
                                                    float(sigma), int(iters), byref(prm), c_void_p(ckpt.data_ptr()),
                                                    _ptr(out, (self.n, self.n), "out")))
        return out

    def unrolled_backward(self, b, w, beta, tau, sigma, iters, ckpt, x_grad, *, tv_iters=10, tv_step=0.125,
                          b_grad=None):
        b_grad = self._sino() if b_grad is None else b_grad
        prm = _params(None, None, tv_iters, tv_step, None, None, False)
        g = (c_double * 3)()
        _check(load().ctpd_unrolled_lowdose_backward(self._h, _ptr(b, (self.m, self.nb), "b"),
                                                     _ptr(w, (self.m, self.nb), "w"), float(beta), float(tau),
                                                     float(sigma), int(iters), byref(prm),
                                                     c_void_p(ckpt.data_ptr()),
                                                     _ptr(x_grad, (self.n, self.n), "x_grad"),
                                                     _ptr(b_grad, (self.m, self.nb), "b_grad"), g))
        return b_grad, (g[0], g[1], g[2])


def _ptr_array(ptrs):
    return (c_void_p * len(ptrs))(*[p.value for p in ptrs])


def _f64_array(vals):
    return (c_double * len(vals))(*[float(v) for v in vals])


def _check_ckpt(op: "Operator", ckpt: torch.Tensor, iters: int) -> c_void_p:
    if ckpt.dtype != torch.float32 or ckpt.numel() < op.ckpt_floats(iters) or not ckpt.is_contiguous():
        raise ValueError("checkpoint buffer too small or not contiguous float32")
    return c_void_p(ckpt.data_ptr())


def unrolled_forward_many(ops, bs, ws, betas, taus, sigmas, iters, ckpts, *, tv_iters=10, tv_step=0.125,
                          outs=None):
    """The unrolled forward pass of several independent problems in one call,
    each on its operator's stream (the library synchronises once for all the
    kappa reductions, then queues every loop).  Returns the list of x."""
    P = len(ops)
    if not (len(bs) == len(ws) == len(betas) == len(taus) == len(sigmas) == len(ckpts) == P) or P == 0:
        raise ValueError("one b, w, beta, tau, sigma and checkpoint buffer per operator")
    outs = [op._img() for op in ops] if outs is None else outs
    prm = _params(None, None, tv_iters, tv_step, None, None, False)
    _check(load().ctpd_unrolled_lowdose_forward_many(
        P, _ptr_array([op._h for op in ops]),
        _ptr_array([_ptr(b, (op.m, op.nb), "b") for op, b in zip(ops, bs)]),
        _ptr_array([_ptr(w, (op.m, op.nb), "w") for op, w in zip(ops, ws)]),
        _f64_array(betas), _f64_array(taus), _f64_array(sigmas), int(iters), byref(prm),
        _ptr_array([_check_ckpt(op, c, iters) for op, c in zip(ops, ckpts)]),
        _ptr_array([_ptr(x, (op.n, op.n), "out") for op, x in zip(ops, outs)])))
    return outs


def unrolled_backward_many(ops, bs, ws, betas, taus, sigmas, iters, ckpts, x_grads, *, tv_iters=10,
                           tv_step=0.125, b_grads=None):
    """The reverse passes of several independent problems in one call (one
    host synchronisation at the end for all the scalar gradients).  Returns
    (list of dL/db, list of (dL/dbeta, dL/dtau, dL/dsigma))."""
    P = len(ops)
    if not (len(bs) == len(ws) == len(betas) == len(taus) == len(sigmas) == len(ckpts) == len(x_grads) == P) \
            or P == 0:
        raise ValueError("one b, w, beta, tau, sigma, checkpoint buffer and x gradient per operator")
    b_grads = [op._sino() for op in ops] if b_grads is None else b_grads
    prm = _params(None, None, tv_iters, tv_step, None, None, False)
    g = (c_double * (3 * P))()
    _check(load().ctpd_unrolled_lowdose_backward_many(
        P, _ptr_array([op._h for op in ops]),
        _ptr_array([_ptr(b, (op.m, op.nb), "b") for op, b in zip(ops, bs)]),
        _ptr_array([_ptr(w, (op.m, op.nb), "w") for op, w in zip(ops, ws)]),
        _f64_array(betas), _f64_array(taus), _f64_array(sigmas), int(iters), byref(prm),
        _ptr_array([_check_ckpt(op, c, iters) for op, c in zip(ops, ckpts)]),
        _ptr_array([_ptr(x, (op.n, op.n), "x_grad") for op, x in zip(ops, x_grads)]),
        _ptr_array([_ptr(x, (op.m, op.nb), "b_grad") for op, x in zip(ops, b_grads)]), g))
    return b_grads, [(g[3 * i], g[3 * i + 1], g[3 * i + 2]) for i in range(P)]


class Batch:
    """Independent low-dose problems of uneven sizes, solved together (Algorithm 1 on each)."""

    def __init__(self, geoms, stream: torch.cuda.Stream | None = None):
        """geoms: (n, n_views, n_bins) or (n, n_views, n_bins, angles) per problem."""
        self.geoms = [(int(g[0]), int(g[1]), int(g[2])) for g in geoms]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        built = [_geometry(*gg, g[3] if len(g) > 3 else None) for gg, g in zip(self.geoms, geoms)]
        arr = (Geometry * len(self.geoms))(*[b[0] for b in built])
        h = c_void_p()
        with torch.cuda.device(self.device):
            _check(load().ctpd_batch_create(arr, len(self.geoms), c_void_p(self.stream.cuda_stream), byref(h)))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ctpd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def lowdose_solve(self, bs, ws, betas, iters: int, *, tau=None, sigma=None, tv_iters=10, tv_step=0.125,
                      safety=0.95, norm_steps=100, outs=None):
        """Returns (list of x, list of info dicts)."""
        P = len(self.geoms)
        if not (len(bs) == len(ws) == len(betas) == P):
            raise ValueError(f"need {P} sinograms, weights and betas")
        if outs is None:
            outs = [torch.empty((n, n), dtype=torch.float32, device=self.device) for n, _, _ in self.geoms]
        pb = (c_void_p * P)(*[_ptr(b, (m, nb), "b") for b, (_, m, nb) in zip(bs, self.geoms)])
        pw = (c_void_p * P)(*[_ptr(w, (m, nb), "w") for w, (_, m, nb) in zip(ws, self.geoms)])
        px = (c_void_p * P)(*[_ptr(x, (n, n), "out") for x, (n, _, _) in zip(outs, self.geoms)])
        pbeta = (c_double * P)(*[float(v) for v in betas])
        prm = _params(tau, sigma, tv_iters, tv_step, safety, norm_steps, False)
        reps = (Report * P)()
        _check(load().ctpd_batch_lowdose_solve(self._h, pb, pw, pbeta, int(iters), byref(prm), px, reps))
        return outs, [Operator._info(r, None, {}) for r in reps]

    def set_tiles(self, placement: int, tv_threads: int, fwd_form: int) -> None:
        _check(load().ctpd_batch_set_tiles(self._h, byref(BatchTiles(placement, tv_threads, fwd_form, 0))))

    def get_tiles(self) -> dict:
        t = BatchTiles()
        _check(load().ctpd_batch_get_tiles(self._h, byref(t)))
        return {"placement": t.placement, "tv_threads": t.tv_threads, "fwd_form": t.fwd_form}

    def time_loop(self, iters: int, tv_iters: int = 10, reps: int = 3) -> float:
        """Median device ms of one replay of the loop graph (needs a previous solve)."""
        ms = c_double()
        _check(load().ctpd_batch_time_loop(self._h, int(iters), int(tv_iters), int(reps), byref(ms)))
        return ms.value


# ---- forward projection without device allocation ---------------------------------
_SIGNATURES["ctpd_project_noalloc"] = (c_int, [c_void_p, c_void_p, c_void_p, c_void_p])


def project_noalloc(x: torch.Tensor, n_views: int, n_bins: int, stream: torch.cuda.Stream | None = None,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x for uniform angles v pi / n_views through ctpd_project_noalloc,
    which allocates nothing (its scratch is a static device array shared by
    every call on the GPU: calls must not overlap).  n <= 1024, n_views <= 4096."""
    n = int(x.shape[0]) if isinstance(x, torch.Tensor) and x.dim() == 2 else -1
    stream = stream if stream is not None else torch.cuda.current_stream()
    out = torch.empty((int(n_views), int(n_bins)), dtype=torch.float32, device=stream.device) if out is None else out
    geo = Geometry(n, int(n_views), int(n_bins), 0, None)
    with torch.cuda.device(stream.device):
        _check(load().ctpd_project_noalloc(byref(geo), c_void_p(stream.cuda_stream), _ptr(x, (n, n), "x"),
                                           _ptr(out, (int(n_views), int(n_bins)), "out")))
    return out
