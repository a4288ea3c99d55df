"""PyTorch binding of the C ABI (include/nfft.h).

Device memory and streams come from PyTorch; every step of the transform runs
in the HIP library. Function names mirror the C entry points; :class:`Plan`
wraps them for convenience.

    plan = Plan(nodes, M=256, sigma=2.0, m=6, precision="f32")
    plan.set_weights(w)            # complex128, caller's node order
    fhat = plan.adjoint(f)         # fhat ~ D^* F^* B^* W f   (eq. (3.7))
    f2   = plan.forward(fhat)      # f ~ B F D fhat           (Algorithm 2.1)
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import NFFT_F32, NFFT_F64, NfftError, check  # noqa: F401

_PREC = {"f64": NFFT_F64, "f32": NFFT_F32, NFFT_F64: NFFT_F64, NFFT_F32: NFFT_F32}
_CDTYPE = {NFFT_F64: torch.complex128, NFFT_F32: torch.complex64}


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_f64_nodes(nodes) -> torch.Tensor:
    if isinstance(nodes, np.ndarray):
        nodes = torch.from_numpy(np.ascontiguousarray(nodes, dtype=np.float64))
    t = nodes.to(torch.float64).contiguous()
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    return t


def check_out(out: torch.Tensor, dtype: torch.dtype, device: torch.device, numel: int) -> None:
    """Reject a caller-supplied output buffer that the library would write
    out of bounds or misread: wrong dtype or device, not contiguous, or fewer
    than `numel` elements."""
    if not isinstance(out, torch.Tensor):
        raise ValueError(f"out must be a torch.Tensor, got {type(out).__name__}")
    if out.dtype != dtype:
        raise ValueError(f"out has dtype {out.dtype}, the plan writes {dtype}")
    dev = torch.device(device)
    if out.device.type != dev.type or (dev.index is not None and out.device.index != dev.index):
        raise ValueError(f"out is on {out.device}, the plan's device is {dev}")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    if out.numel() < numel:
        raise ValueError(f"out holds {out.numel()} elements, the call writes {numel}")


def oversampled_size(M: int, sigma: float) -> int:
    """M_sigma = 2 ceil(ceil(sigma M)/2) (host-side shape arithmetic)."""
    import math
    return 2 * math.ceil(math.ceil(sigma * M) / 2)


# ------------------------------------------------------------ C-ABI mirrors
def nfft_plan(d: int, M: int, sigma: float, m: int, nodes: torch.Tensor, precision=NFFT_F64,
              max_rhs: int = 1, stream=None) -> ctypes.c_void_p:
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.nfft_plan(ctypes.byref(h), d, M, float(sigma), m, nodes.shape[0],
                       ctypes.c_void_p(nodes.data_ptr()), _PREC[precision], max_rhs,
                       _stream_ptr(stream))
    check(st, None)
    return h


TUNING_KEYS = ("tile_edge", "item_nodes", "spread_threads", "rhs_per_group", "fft_min_wg",
               "spread_planes", "spread_mode")


def _tuning_array(tuning) -> Optional[ctypes.Array]:
    """dict (keys of TUNING_KEYS) or sequence -> int32 array; None = defaults."""
    if tuning is None:
        return None
    if isinstance(tuning, dict):
        unknown = set(tuning) - set(TUNING_KEYS)
        if unknown:
            raise ValueError(f"unknown tuning keys {sorted(unknown)}")
        vals = [int(tuning.get(k, 0) or 0) for k in TUNING_KEYS]
    else:
        vals = [int(v) for v in tuning]
    return (ctypes.c_int32 * len(vals))(*vals)


def nfft_plan_tuned(d: int, M: int, sigma: float, m: int, nodes: torch.Tensor, precision=NFFT_F64,
                    max_rhs: int = 1, tuning=None, stream=None) -> ctypes.c_void_p:
    lib = _lib.load()
    h = ctypes.c_void_p()
    arr = _tuning_array(tuning)
    st = lib.nfft_plan_tuned(ctypes.byref(h), d, M, float(sigma), m, nodes.shape[0],
                             ctypes.c_void_p(nodes.data_ptr()), _PREC[precision], max_rhs,
                             arr, len(arr) if arr is not None else 0, _stream_ptr(stream))
    check(st, None)
    return h


def nfft_plan_autotune(d: int, M: int, sigma: float, m: int, nodes: torch.Tensor, precision=NFFT_F64,
                       max_rhs: int = 1, nrhs: int = 1, stream=None):
    """-> (handle, milliseconds per adjoint of the winner)."""
    lib = _lib.load()
    h = ctypes.c_void_p()
    best = ctypes.c_double(0.0)
    st = lib.nfft_plan_autotune(ctypes.byref(h), d, M, float(sigma), m, nodes.shape[0],
                                ctypes.c_void_p(nodes.data_ptr()), _PREC[precision], max_rhs, nrhs,
                                ctypes.byref(best), _stream_ptr(stream))
    check(st, None)
    return h, best.value


def nfft_get_tuning(plan) -> dict:
    out = (ctypes.c_int32 * _lib.NFFT_TUNE_COUNT)()
    check(_lib.load().nfft_get_tuning(plan, out, _lib.NFFT_TUNE_COUNT), plan)
    return dict(zip(TUNING_KEYS, (int(v) for v in out)))


def nfft_set_tuning(plan, knob, value: int) -> None:
    k = TUNING_KEYS.index(knob) if isinstance(knob, str) else int(knob)
    check(_lib.load().nfft_set_tuning(plan, k, int(value)), plan)


def nfft_plan_clone(plan, max_rhs: int, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(_lib.load().nfft_plan_clone(plan, max_rhs, ctypes.byref(h), _stream_ptr(stream)), plan)
    return h


def nfft_set_weights(plan, w: torch.Tensor, stream=None) -> None:
    check(_lib.load().nfft_set_weights(plan, ctypes.c_void_p(w.data_ptr()), _stream_ptr(stream)), plan)


def nfft_adjoint(plan, f: torch.Tensor, fhat: torch.Tensor, nrhs: int, stream=None) -> None:
    check(_lib.load().nfft_adjoint(plan, ctypes.c_void_p(f.data_ptr()),
                                   ctypes.c_void_p(fhat.data_ptr()), nrhs, _stream_ptr(stream)), plan)


def nfft_adjoint_scratch(plan, f: torch.Tensor, fhat: torch.Tensor, nrhs: int, stream=None) -> None:
    check(_lib.load().nfft_adjoint_scratch(plan, ctypes.c_void_p(f.data_ptr()),
                                           ctypes.c_void_p(fhat.data_ptr()), nrhs,
                                           _stream_ptr(stream)), plan)


def nfft_forward(plan, fhat: torch.Tensor, f: torch.Tensor, nrhs: int, stream=None) -> None:
    check(_lib.load().nfft_forward(plan, ctypes.c_void_p(fhat.data_ptr()),
                                   ctypes.c_void_p(f.data_ptr()), nrhs, _stream_ptr(stream)), plan)


def nfft_refine(plan, f: torch.Tensor, fhat: torch.Tensor, nrhs: int, iters: int,
                residuals: bool = False, stream=None) -> Optional[np.ndarray]:
    """fhat_iters of the weighted iterative refinement (nfft_refine); with
    residuals, the relative residuals ||f - A fhat_k|| / ||f||, k = 0..iters."""
    res = (ctypes.c_double * (iters + 1))() if residuals and iters >= 0 else None
    check(_lib.load().nfft_refine(plan, ctypes.c_void_p(f.data_ptr()),
                                  ctypes.c_void_p(fhat.data_ptr()), nrhs, int(iters), res,
                                  _stream_ptr(stream)), plan)
    return np.array(res[:], dtype=np.float64) if res is not None else None


def nfft_weights(d: int, M: int, sigma: float, m: int, nodes: torch.Tensor, tol: float,
                 maxit: int, w: torch.Tensor, stream=None) -> dict:
    """Algorithm 3.6 on the device (float64); w: complex128 device tensor of N."""
    info = (ctypes.c_double * 4)()
    check(_lib.load().nfft_weights(d, M, float(sigma), m, nodes.shape[0],
                                   ctypes.c_void_p(nodes.data_ptr()), float(tol), int(maxit),
                                   ctypes.c_void_p(w.data_ptr()), info, _stream_ptr(stream)), None)
    return {"iterations": int(info[0]), "rel_residual": float(info[1]),
            "branch": "3.15" if int(info[2]) == 15 else "3.16", "epsilon": float(info[3])}


WEIGHT_SCHEMES = {"alg3.6": 0, "relaxed": 1, "pcf": 2}
_BRANCH = {15: "3.15", 16: "3.16", 62: "3.62", 63: "3.63"}


def nfft_weights_ex(d: int, M: int, sigma: float, m: int, nodes: torch.Tensor, scheme, tol: float,
                    maxit: int, w: torch.Tensor, stream=None) -> dict:
    info = (ctypes.c_double * 4)()
    sch = WEIGHT_SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    check(_lib.load().nfft_weights_ex(d, M, float(sigma), m, nodes.shape[0],
                                      ctypes.c_void_p(nodes.data_ptr()), sch, float(tol), int(maxit),
                                      ctypes.c_void_p(w.data_ptr()), info, _stream_ptr(stream)), None)
    return {"iterations": int(info[0]), "rel_residual": float(info[1]),
            "branch": _BRANCH.get(int(info[2]), str(int(info[2]))), "epsilon": float(info[3])}


def compute_weights(nodes, M: int, sigma: float = 2.0, m: int = 8, tol: float = 1e-13,
                    maxit: int = 1000, device=None, stream=None, scheme: str = "alg3.6"):
    """Density-compensation weights for a node set, computed on the GPU in
    float64: Algorithm 3.6 (scheme "alg3.6", the default), the relaxed
    conditions A A^* w = 1 of (3.63) ("relaxed") or the PCF weights (3.62)
    ("pcf"). Returns (w, info): w complex128 on the device in the caller's
    node order, info with iterations, relative residual, branch and epsilon
    (for "relaxed": max |A A^* w - 1|)."""
    dev = torch.device(device or "cuda")
    x = _as_f64_nodes(nodes).to(dev)
    N, d = x.shape
    w = torch.empty(N, dtype=torch.complex128, device=dev)
    with torch.cuda.device(dev):
        info = nfft_weights_ex(d, M, sigma, m, x, scheme, tol, maxit, w, stream)
    return w, info


def nfft_bopt_build(plan, nodes: torch.Tensor, stream=None) -> dict:
    info = (ctypes.c_double * 3)()
    check(_lib.load().nfft_bopt_build(plan, ctypes.c_void_p(nodes.data_ptr()), info,
                                      _stream_ptr(stream)), plan)
    return {"max_column": int(info[0]), "nnz": int(info[1]), "singular_columns": int(info[2])}


def nfft_bopt_adjoint(plan, f: torch.Tensor, fhat: torch.Tensor, nrhs: int, stream=None) -> None:
    check(_lib.load().nfft_bopt_adjoint(plan, ctypes.c_void_p(f.data_ptr()),
                                        ctypes.c_void_p(fhat.data_ptr()), nrhs,
                                        _stream_ptr(stream)), plan)


def nfft_bopt_inverse_adjoint(plan, h: torch.Tensor, f: torch.Tensor, nrhs: int, stream=None) -> None:
    check(_lib.load().nfft_bopt_inverse_adjoint(plan, ctypes.c_void_p(h.data_ptr()),
                                                ctypes.c_void_p(f.data_ptr()), nrhs,
                                                _stream_ptr(stream)), plan)


def nfft_bopt_get(plan, ncols: int):
    """-> (col_ptr int64[ncols+1], nodes int32[nnz], vals float64[nnz]) on the host."""
    lib = _lib.load()
    nnz = ctypes.c_int64(0)
    check(lib.nfft_bopt_get(plan, ctypes.byref(nnz), None, None, None), plan)
    ptr = np.empty(ncols + 1, dtype=np.int64)
    nodes = np.empty(max(1, nnz.value), dtype=np.int32)
    vals = np.empty(max(1, nnz.value), dtype=np.float64)
    check(lib.nfft_bopt_get(plan, None, ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), plan)
    return ptr, nodes[:nnz.value], vals[:nnz.value]


def nfft_destroy(plan) -> None:
    check(_lib.load().nfft_destroy(plan), None)


def nfft_footprint(d: int, M: int, sigma: float, m: int, N: int, precision=NFFT_F64,
                   max_rhs: int = 1) -> int:
    return int(_lib.load().nfft_footprint(d, M, float(sigma), m, N, _PREC[precision], max_rhs))


def nfft_strerror(status: int) -> str:
    return _lib.load().nfft_strerror(status).decode()


def nfft_last_error(plan=None) -> str:
    return _lib.load().nfft_last_error(plan).decode(errors="replace")


def nfft_plan_info(plan) -> dict:
    out = (ctypes.c_int64 * 13)()
    check(_lib.load().nfft_plan_info(plan, out, 13), plan)
    keys = ("d", "M", "Ms", "m", "N", "precision", "max_rhs", "tile", "tiles", "items",
            "max_tile_nodes", "bytes", "workspace_bytes")
    return dict(zip(keys, (int(v) for v in out)))


def nfft_permutation(plan, N: int) -> np.ndarray:
    out = np.empty(N, dtype=np.int32)
    check(_lib.load().nfft_permutation(plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), plan)
    return out


def nfft_set_profiling(plan, enable: bool) -> None:
    check(_lib.load().nfft_set_profiling(plan, int(bool(enable))), plan)


STAGE_NAMES = ("spread", "split_tile_reduce", "fft_merge", "fft_rest_deconv", "fwd_fft_deconv",
               "fwd_sums", "bopt_apply", "bopt_fft")


def nfft_stage_times(plan, reset: bool = False) -> dict:
    n = 2 * _lib.NFFT_STAGES
    out = (ctypes.c_double * n)()
    check(_lib.load().nfft_stage_times(plan, out, n, int(bool(reset))), plan)
    return {name: (out[2 * i], int(out[2 * i + 1])) for i, name in enumerate(STAGE_NAMES)}


# ------------------------------------------------------------------- Plan
class Plan:
    """One node set on one device (nodes wrapped onto [-1/2, 1/2)^d)."""

    def __init__(self, nodes, M: int, sigma: float = 2.0, m: int = 6, precision="f64",
                 max_rhs: int = 1, device: Optional[torch.device] = None, stream=None,
                 tuning=None):
        """tuning: None (defaults), a dict of TUNING_KEYS, or "auto" (the
        library times candidate tunings for max_rhs right-hand sides and keeps
        the fastest; see nfft_plan_autotune)."""
        self.device = torch.device(device or "cuda")
        x = _as_f64_nodes(nodes).to(self.device)
        self.N, self.d = x.shape
        self.M, self.sigma, self.m = M, float(sigma), m
        self.prec = _PREC[precision]
        self.cdtype = _CDTYPE[self.prec]
        self.max_rhs = max_rhs
        self.Ms = oversampled_size(M, sigma)
        self._h = None
        with torch.cuda.device(self.device):
            self.tuned_ms = None
            if isinstance(tuning, str):
                if tuning != "auto":
                    raise ValueError(f"tuning={tuning!r}: expected None, a dict or 'auto'")
                self._h, self.tuned_ms = nfft_plan_autotune(self.d, M, sigma, m, x, self.prec,
                                                            max_rhs, max_rhs, stream)
            else:
                self._h = nfft_plan_tuned(self.d, M, sigma, m, x, self.prec, max_rhs, tuning,
                                          stream)

    @property
    def handle(self):
        return self._h

    def clone(self, max_rhs: int, stream=None) -> "Plan":
        """A handle on the same node set and weights with its own workspace."""
        c = Plan.__new__(Plan)
        c.__dict__.update({k: v for k, v in self.__dict__.items() if k != "_h"})
        c.max_rhs = max_rhs
        c._h = None
        with torch.cuda.device(self.device):
            c._h = nfft_plan_clone(self._h, max_rhs, stream)
        return c

    def set_weights(self, w, stream=None) -> None:
        if isinstance(w, np.ndarray):
            w = torch.from_numpy(np.ascontiguousarray(w, dtype=np.complex128))
        w = w.to(torch.complex128).reshape(-1).contiguous().to(self.device)
        if w.numel() != self.N:
            raise ValueError(f"expected {self.N} weights, got {w.numel()}")
        nfft_set_weights(self._h, w, stream)

    def _coerce(self, t, n):
        if isinstance(t, np.ndarray):
            t = torch.from_numpy(t)
        t = t.to(device=self.device, dtype=self.cdtype).contiguous()
        if t.numel() % n:
            raise ValueError(f"size {t.numel()} is not a multiple of {n}")
        return t

    def adjoint(self, f, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """fhat = D^* F^* B^* W f; f is (N,) or (nrhs, N)."""
        single = f.dim() == 1 if isinstance(f, torch.Tensor) else np.ndim(f) == 1
        f = self._coerce(f, self.N)
        nrhs = f.numel() // self.N
        K = self.M ** self.d
        if out is None:
            out = torch.empty((nrhs, K), dtype=self.cdtype, device=self.device)
        check_out(out, self.cdtype, self.device, nrhs * K)
        nfft_adjoint(self._h, f, out, nrhs, stream)
        return out.reshape(K) if single else out

    def adjoint_scratch(self, f, out: torch.Tensor, stream=None) -> torch.Tensor:
        """self.adjoint with the library's scratch array in place of the plan's
        workspace (nfft_adjoint_scratch: no device allocation by the library;
        calls overlapping on one GPU race). out is required, so that nothing
        is allocated here either."""
        f = self._coerce(f, self.N)
        nrhs = f.numel() // self.N
        check_out(out, self.cdtype, self.device, nrhs * self.M ** self.d)
        nfft_adjoint_scratch(self._h, f, out, nrhs, stream)
        return out

    def forward(self, fhat, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """f = B F D fhat; fhat is (M^d,) or (nrhs, M^d)."""
        K = self.M ** self.d
        single = fhat.dim() == 1 if isinstance(fhat, torch.Tensor) else np.ndim(fhat) == 1
        fhat = self._coerce(fhat, K)
        nrhs = fhat.numel() // K
        if out is None:
            out = torch.empty((nrhs, self.N), dtype=self.cdtype, device=self.device)
        check_out(out, self.cdtype, self.device, nrhs * self.N)
        nfft_forward(self._h, fhat, out, nrhs, stream)
        return out.reshape(self.N) if single else out

    def refine(self, f, iters: int, out: Optional[torch.Tensor] = None, residuals: bool = False,
               stream=None):
        """The adjoint reconstruction improved by `iters` steps of
        fhat <- fhat + A^* W (f - A fhat) (nfft_refine); f is (N,) or
        (nrhs, N). Returns fhat, or (fhat, relative residuals k = 0..iters)
        with residuals=True (the call then waits for the stream)."""
        single = f.dim() == 1 if isinstance(f, torch.Tensor) else np.ndim(f) == 1
        f = self._coerce(f, self.N)
        nrhs = f.numel() // self.N
        K = self.M ** self.d
        if out is None:
            out = torch.empty((nrhs, K), dtype=self.cdtype, device=self.device)
        check_out(out, self.cdtype, self.device, nrhs * K)
        res = nfft_refine(self._h, f, out, nrhs, iters, residuals, stream)
        out = out.reshape(K) if single else out
        return (out, res) if residuals else out

    def _graph(self, fn, src: torch.Tensor, out: torch.Tensor):
        """Capture fn(src, out=out) (every kernel of one transform) into a HIP
        graph on a side stream; replaying it reruns the transform on whatever
        src holds then. The transform allocates nothing and clears nothing
        with memset, so the captured launches are exactly the eager ones."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            fn(src, out=out)  # warm-up outside the capture
        torch.cuda.current_stream(self.device).wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            fn(src, out=out)
        return g

    def graph_adjoint(self, f: torch.Tensor, out: torch.Tensor):
        """HIP graph of self.adjoint(f, out=out); f and out stay bound to it."""
        return self._graph(self.adjoint, f, out)

    def graph_forward(self, fhat: torch.Tensor, out: torch.Tensor):
        """HIP graph of self.forward(fhat, out=out)."""
        return self._graph(self.forward, fhat, out)

    def build_bopt(self, nodes, stream=None) -> dict:
        """Algorithm 4.3 on the device for this node set (pass the same nodes
        again, float64); afterwards bopt_adjoint is available."""
        x = _as_f64_nodes(nodes).to(self.device)
        with torch.cuda.device(self.device):
            return nfft_bopt_build(self._h, x, stream)

    def bopt_adjoint(self, f, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """h_opt = D^* F^* B_opt^* f (Algorithm 4.4); f is (N,) or (nrhs, N)."""
        single = f.dim() == 1 if isinstance(f, torch.Tensor) else np.ndim(f) == 1
        f = self._coerce(f, self.N)
        nrhs = f.numel() // self.N
        K = self.M ** self.d
        if out is None:
            out = torch.empty((nrhs, K), dtype=self.cdtype, device=self.device)
        check_out(out, self.cdtype, self.device, nrhs * K)
        nfft_bopt_adjoint(self._h, f, out, nrhs, stream)
        return out.reshape(K) if single else out

    def bopt_inverse_adjoint(self, h, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """f = B_opt F D h, an approximate solution of A^* f = h (Remark 4.6);
        h is (M^d,) or (nrhs, M^d)."""
        K = self.M ** self.d
        single = h.dim() == 1 if isinstance(h, torch.Tensor) else np.ndim(h) == 1
        h = self._coerce(h, K)
        nrhs = h.numel() // K
        if out is None:
            out = torch.empty((nrhs, self.N), dtype=self.cdtype, device=self.device)
        check_out(out, self.cdtype, self.device, nrhs * self.N)
        nfft_bopt_inverse_adjoint(self._h, h, out, nrhs, stream)
        return out.reshape(self.N) if single else out

    def bopt_matrix(self):
        """B_opt on the host: (col_ptr, nodes, vals) by grid columns."""
        return nfft_bopt_get(self._h, self.Ms ** self.d)

    def info(self) -> dict:
        return nfft_plan_info(self._h)

    def tuning(self) -> dict:
        return nfft_get_tuning(self._h)

    def set_tuning(self, knob, value: int) -> None:
        """Change a launch-time knob (spread_threads, rhs_per_group, fft_min_wg, spread_planes,
        spread_mode)."""
        nfft_set_tuning(self._h, knob, value)

    def permutation(self) -> np.ndarray:
        return nfft_permutation(self._h, self.N)

    def set_profiling(self, on: bool) -> None:
        nfft_set_profiling(self._h, on)

    def stage_times(self, reset: bool = False) -> dict:
        return nfft_stage_times(self._h, reset)

    def close(self) -> None:
        if self._h is not None:
            nfft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
