"""Torch-facing wrappers of the C ABI (device memory and streams only).

    ctx = Context(0)
    out = estep(Y, W, pi, sigma, Hprime=12, gamma=4)           # BSC, FP32
    acc = new_acc("bsc", D, H); estep(..., acc=acc)             # accumulate statistics
    W1, theta = mstep(acc, W, model="bsc")                      # FP64 M-step on device
    estep(Y, W, sigma=s, Hprime=8, gamma=3, model="dsc",        # discrete values phi_v
          phi=(0, 1, -1, 2), pv=(0.7, 0.1, 0.1, 0.1))

All tensors live on the GPU; every step of the computation runs in
libprosper.so.  Outputs are valid once the current stream is synchronised.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import torch

from . import _lib

__all__ = ["Context", "context", "estep", "mstep", "mstep_et", "new_acc", "zero_acc", "state_count",
           "state_table", "dsc_state_count", "dsc_state_table", "ProsperError"]

ProsperError = _lib.ProsperError
state_count = _lib.state_count
state_table = _lib.state_table
dsc_state_count = _lib.dsc_state_count
dsc_state_table = _lib.dsc_state_table


class Context:
    """A libprosper context bound to one HIP device (owns workspace and the
    cached state tables)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        lib = _lib.load()
        h = C.c_void_p()
        _lib.check(lib.prosper_ctx_create(int(device), int(workspace_bytes), C.byref(h)))
        self.handle = h
        self.device = int(device)

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().prosper_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return _lib.last_error(self.handle)


_contexts: Dict[int, Context] = {}


def context(device: Optional[int] = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _dev_f32(name: str, t: torch.Tensor) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    return t


def new_acc(model: str, D: int, H: int, device=None, nvalues: int = 0) -> Dict[str, torch.Tensor]:
    """Zeroed M-step accumulators (A: D x H, B: H x H, or D x H for MCA/MMCA, scal: 5 doubles;
    DSC also vcount: `nvalues` doubles)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    Bshape = (D, H) if model in ("mca", "mmca") else (H, H)
    acc = {"A": torch.zeros((D, H), dtype=torch.float32, device=dev),
           "B": torch.zeros(Bshape, dtype=torch.float32, device=dev),
           "scal": torch.zeros(5, dtype=torch.float64, device=dev)}
    if model == "dsc":
        if nvalues < 2:
            raise ValueError("DSC accumulators need nvalues >= 2")
        acc["vcount"] = torch.zeros(nvalues, dtype=torch.float64, device=dev)
    return acc


def _acc_struct(acc: Dict[str, torch.Tensor]):
    return _lib.Acc(_ptr(acc["A"]), _ptr(acc["B"]), _ptr(acc["scal"]), _ptr(acc.get("vcount")))


def zero_acc(acc: Dict[str, torch.Tensor]):
    for t in acc.values():
        t.zero_()


def estep(Y: torch.Tensor, W: torch.Tensor, pi: float = 0.5, sigma: float = 1.0, *,
          Hprime: int, gamma: int, model: str = "bsc", precision: str = "fp32",
          topk: int = 0, acc: Optional[Dict[str, torch.Tensor]] = None,
          theta: Optional[torch.Tensor] = None,
          want: Sequence[str] = ("sel", "s_mean", "logL", "flagged"),
          out: Optional[Dict[str, torch.Tensor]] = None,
          ctx: Optional[Context] = None, stream: Optional[torch.cuda.Stream] = None,
          factor_b: bool = False, static: bool = False,
          beta: float = 1.0, phi: Optional[Sequence[float]] = None,
          pv: Optional[Sequence[float]] = None, zero_acc: bool = False) -> Dict[str, torch.Tensor]:
    """Truncated E-step over the rows of Y (N x D) for dictionary W (D x H).

    Returns the requested per-point outputs: sel (N x H' int32), s_mean
    (N x H'), logL (N), flagged (N uint8), top_mask / top_q (N x topk), and
    for BSC/TSC k_mean and res (N each: <#non-zero> and <||y - W s||^2>, the
    inputs of `mstep_et`).
    `theta` (2 doubles on the device: pi, sigma) overrides pi and sigma.
    `out` may supply preallocated output tensors (same keys).
    `factor_b` (with `acc`, BSC/TSC): this call completes the accumulation;
    B is factored for the next `mstep` with the same acc, overlapped with the
    A statistics (PROSPER_FLAG_FACTOR_B).
    `static` calls prosper_estep_static, which allocates nothing (its
    intermediates live in the library's fixed device array); no context.
    `beta` is the posterior temperature of deterministic annealing (q
    proportional to p(y, s)^beta; logL untempered).
    `zero_acc` (with `acc`): overwrite the accumulators instead of adding into
    them (PROSPER_FLAG_ZERO_ACC; no separate clearing needed).
    DSC (model="dsc"): `phi` is the value set (phi[0] = 0) and `pv` its prior
    (ignored when `theta` = (pi, sigma, pv_0 .. pv_{V-1}) is given); top_mask
    is N x topk x 4 (active mask, three bit planes of the value codes).
    """
    _dev_f32("Y", Y)
    _dev_f32("W", W)
    N, D = Y.shape
    D2, H = W.shape
    if D2 != D:
        raise ValueError("Y is N x D and W must be D x H")
    if not static:
        ctx = ctx or context(Y.device.index)
    dev = Y.device
    res: Dict[str, torch.Tensor] = {}
    out = dict(out or {})

    def get(key, shape, dtype):
        if key in out:
            t = out[key]
            if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous():
                raise ValueError(f"out[{key!r}] must be {dtype} {tuple(shape)} contiguous")
            return t
        return torch.empty(shape, dtype=dtype, device=dev)

    if "sel" in want or "sel" in out:
        res["sel"] = get("sel", (N, Hprime), torch.int32)
    if "s_mean" in want or "s_mean" in out:
        res["s_mean"] = get("s_mean", (N, Hprime), torch.float32)
    if "logL" in want or "logL" in out:
        res["logL"] = get("logL", (N,), torch.float32)
    if "flagged" in want or "flagged" in out:
        res["flagged"] = get("flagged", (N,), torch.uint8)
    for key in ("k_mean", "res"):   # BSC/TSC: per-point inputs of mstep_et
        if key in want or key in out:
            res[key] = get(key, (N,), torch.float32)
    if topk:
        mshape = {"tsc": (N, topk, 2), "dsc": (N, topk, 4)}.get(model, (N, topk))
        res["top_mask"] = get("top_mask", mshape, torch.int32)
        res["top_q"] = get("top_q", (N, topk), torch.float32)
    po = _lib.PointOut(_ptr(res.get("sel")), _ptr(res.get("s_mean")), _ptr(res.get("logL")),
                       _ptr(res.get("top_mask")), _ptr(res.get("top_q")), _ptr(res.get("flagged")),
                       _ptr(res.get("k_mean")), _ptr(res.get("res")))
    accs = None
    if acc is not None:
        accs = _acc_struct(acc)
    if model == "dsc" and phi is None:
        raise ValueError("DSC needs the value set phi")
    flags = (_lib.FLAG_FACTOR_B if factor_b else 0) | (_lib.FLAG_ZERO_ACC if zero_acc else 0)
    args = _lib.make_args(model, precision, N, D, H, Hprime, gamma, pi, sigma,
                          _ptr(theta), topk, 1 if acc is not None else 0, flags, beta,
                          phi if model == "dsc" else None, pv if model == "dsc" else None)
    st = (stream or torch.cuda.current_stream(dev)).cuda_stream
    lib = _lib.load()
    if static:
        with torch.cuda.device(dev):
            _lib.check(lib.prosper_estep_static(C.byref(args), _ptr(Y), _ptr(W), C.byref(po),
                                                C.byref(accs) if accs is not None else None,
                                                C.c_void_p(st)))
        return res
    _lib.check(lib.prosper_estep(ctx.handle, C.byref(args), _ptr(Y), _ptr(W), C.byref(po),
                                 C.byref(accs) if accs is not None else None, C.c_void_p(st)),
               ctx.handle)
    return res


def mstep(acc: Dict[str, torch.Tensor], W_old: torch.Tensor, *, model: str = "bsc",
          W_new: Optional[torch.Tensor] = None, theta_new: Optional[torch.Tensor] = None,
          ctx: Optional[Context] = None, stream: Optional[torch.cuda.Stream] = None):
    """FP64 M-step on the device.  Returns (W_new, theta_new) where theta_new
    holds (pi, sigma) as two doubles on the device; DSC: (pi, sigma, pv_0 ..
    pv_{V-1}), V the length of acc["vcount"]."""
    _dev_f32("W_old", W_old)
    D, H = W_old.shape
    ctx = ctx or context(W_old.device.index)
    nv = int(acc["vcount"].numel()) if model == "dsc" else 0
    if W_new is None:
        W_new = torch.empty_like(W_old)
    if theta_new is None:
        theta_new = torch.empty(2 + nv, dtype=torch.float64, device=W_old.device)
    args = _lib.make_args(model, "fp32", 0, D, H, 1, 0)
    args.nvalues = nv
    accs = _acc_struct(acc)
    st = (stream or torch.cuda.current_stream(W_old.device)).cuda_stream
    _lib.check(_lib.load().prosper_mstep(ctx.handle, C.byref(args), C.byref(accs), _ptr(W_old),
                                         _ptr(W_new), _ptr(theta_new), C.c_void_p(st)),
               ctx.handle)
    return W_new, theta_new


def mstep_et(acc: Dict[str, torch.Tensor], W_old: torch.Tensor, points: Dict[str, torch.Tensor],
             *, gamma: int, model: str = "bsc", pi: float = 0.5,
             theta: Optional[torch.Tensor] = None, W_new: Optional[torch.Tensor] = None,
             theta_new: Optional[torch.Tensor] = None, ctx: Optional[Context] = None,
             stream: Optional[torch.cuda.Stream] = None):
    """The selected-points M-step (prosper_mstep_et): W_new from all points as
    `mstep`; pi and sigma from the points with the largest logL (their count
    from the prior's share of draws with at most `gamma` causes).  `points`
    holds the E-step's logL, k_mean and res; the E-step's pi is `theta[0]`
    when given, else `pi`.  Returns (W_new, theta_new)."""
    _dev_f32("W_old", W_old)
    D, H = W_old.shape
    N = int(points["logL"].numel())
    ctx = ctx or context(W_old.device.index)
    if W_new is None:
        W_new = torch.empty_like(W_old)
    if theta_new is None:
        theta_new = torch.empty(2, dtype=torch.float64, device=W_old.device)
    args = _lib.make_args(model, "fp32", N, D, H, 1, gamma, pi=pi, theta_dev=_ptr(theta))
    st = (stream or torch.cuda.current_stream(W_old.device)).cuda_stream
    _lib.check(_lib.load().prosper_mstep_et(ctx.handle, C.byref(args), C.byref(_acc_struct(acc)),
                                            _ptr(points["logL"]), _ptr(points["k_mean"]),
                                            _ptr(points["res"]), _ptr(W_old), _ptr(W_new),
                                            _ptr(theta_new), C.c_void_p(st)), ctx.handle)
    return W_new, theta_new
