"""Python handle of the C serving runtime (prosper_serve*): E-step-only
posterior inference with continuous batching on one GPU.

    srv = Server(W, pi=6/512, sigma=0.5, precision="bf16")
    rid, out = srv.submit(Y, Hprime=10, gamma=4, topk=3)     # non-blocking
    latency_ms = srv.wait(rid)                                # out[...] now filled
    srv.stop()

Requests carry host (NumPy) buffers; the runtime copies them to the device,
runs the kernels on one of its streams and copies the results back.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Tuple

import numpy as np

from . import _lib


class Server:
    def __init__(self, W, pi: float, sigma: float, *, model: str = "bsc",
                 precision: str = "bf16", mem_budget_bytes: int = 512 << 20,
                 max_inflight: int = 16, n_streams: int = 4, queue_capacity: int = 4096,
                 ctx=None):
        from . import api
        import torch
        self.ctx = ctx or api.context()
        if isinstance(W, torch.Tensor):
            Wt = W.detach().to(torch.float32).contiguous()
            on_dev = 1 if Wt.is_cuda else 0
            ptr = Wt.data_ptr()
            self._W_keep = Wt
        else:
            Wn = np.ascontiguousarray(W, dtype=np.float32)
            on_dev, ptr = 0, Wn.ctypes.data
            self._W_keep = Wn
        self.D, self.H = int(self._W_keep.shape[0]), int(self._W_keep.shape[1])
        self.model = model
        h = C.c_void_p()
        lib = _lib.load()
        st = lib.prosper_serve(self.ctx.handle, C.c_void_p(ptr), on_dev, _lib.MODELS[model],
                               self.D, self.H, float(pi), float(sigma),
                               _lib.PRECISIONS[precision], int(mem_budget_bytes),
                               int(max_inflight), int(n_streams), int(queue_capacity),
                               C.byref(h))
        _lib.check(st, self.ctx.handle)
        self.handle = h
        self._live: Dict[int, tuple] = {}

    def submit(self, Y: np.ndarray, Hprime: int, gamma: int, topk: int = 0,
               outputs=("sel", "s_mean", "logL")) -> Tuple[int, Dict[str, np.ndarray]]:
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        n = Y.shape[0]
        out: Dict[str, np.ndarray] = {}
        if "sel" in outputs:
            out["sel"] = np.empty((n, Hprime), dtype=np.int32)
        if "s_mean" in outputs:
            out["s_mean"] = np.empty((n, Hprime), dtype=np.float32)
        if "logL" in outputs:
            out["logL"] = np.empty(n, dtype=np.float32)
        if "flagged" in outputs:
            out["flagged"] = np.empty(n, dtype=np.uint8)
        if topk:
            out["top_mask"] = np.empty((n, topk, 2) if self.model == "tsc" else (n, topk),
                                       dtype=np.uint32)
            out["top_q"] = np.empty((n, topk), dtype=np.float32)

        def p(k):
            return out[k].ctypes.data if k in out else None
        po = _lib.PointOut(p("sel"), p("s_mean"), p("logL"), p("top_mask"), p("top_q"),
                           p("flagged"))
        rid = C.c_uint64(0)
        st = _lib.load().prosper_serve_submit(self.handle, C.c_void_p(Y.ctypes.data), n,
                                              Hprime, gamma, topk, C.byref(po), C.byref(rid))
        if st != 0:
            raise _lib.ProsperError(st, "serve_submit rejected the request")
        self._live[rid.value] = (Y, out, po)
        return rid.value, out

    def wait(self, rid: int, timeout_us: int = -1) -> float:
        lat = C.c_double(0.0)
        st = _lib.load().prosper_serve_wait(self.handle, C.c_uint64(rid), int(timeout_us),
                                            C.byref(lat))
        if st == -6:
            raise TimeoutError(f"request {rid} still running")
        self._live.pop(rid, None)
        if st != 0:
            raise _lib.ProsperError(st, f"request {rid} failed")
        return lat.value

    STAGES = ("queue", "launch", "device_span", "gpu", "delivery", "total")

    def wait_stages(self, rid: int, timeout_us: int = -1) -> dict:
        """Like wait, returning the request's time split into stages (ms):
        queue wait, the batch's launch calls, launch-to-completion-seen (of
        which `gpu` is the batch's GPU time), delivery, total."""
        st6 = (C.c_double * 6)()
        st = _lib.load().prosper_serve_wait_stages(self.handle, C.c_uint64(rid),
                                                   int(timeout_us), st6)
        if st == -6:
            raise TimeoutError(f"request {rid} still running")
        self._live.pop(rid, None)
        if st != 0:
            raise _lib.ProsperError(st, f"request {rid} failed")
        return dict(zip(self.STAGES, list(st6)))

    def stop(self):
        if getattr(self, "handle", None):
            _lib.load().prosper_serve_stop(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
