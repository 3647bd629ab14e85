"""Model, annealing and EM objects of the library's user interface (section
"ProSper's user interface"): a model is instantiated with its sizes and
approximation parameters, parameters are initialised from the data with
`standard_init`, an annealing schedule fixes the number of iterations, the
parameter noise and the posterior temperature, `EM(model, anneal).run()`
learns, and `model.inference(anneal, params, Y)` returns the most likely
latent states and their approximate posterior probabilities.

    model = BSC_ET(D, H, Hprime, gamma)
    anneal = LinearAnnealing(150)
    params = model.standard_init({"y": Y})
    em = EM(model=model, anneal=anneal, data={"y": Y}, lparams=params)
    em.run()
    res = model.inference(anneal, em.lparams, Y)    # res["s"], res["p"]

These are drivers: every E-step and M-step runs in libprosper.so through
`api.estep` / `api.mstep` (truncated E-step with the statistics, FP64
M-step on the device); parameters stay in device memory between
iterations.  Parameter noise and the expansion of the top states into
H-dimensional vectors are plain tensor operations on the device.
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np
import torch

from . import api

__all__ = ["Model", "BSC_ET", "TSC_ET", "MCA_ET", "MMCA_ET", "DSC_ET", "Annealing",
           "LinearAnnealing", "EM"]


def _device_tensor(x, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device=device)


class Model:
    """A truncated-EM sparse coding model (Eq. 1: prior, Eq. 2: noisy
    superposition; Table 1) with its truncation parameters H' and gamma."""

    kind = "bsc"

    def __init__(self, D: int, H: int, Hprime: int, gamma: int, precision: str = "bf16",
                 device: Optional[int] = None):
        if not (1 <= Hprime <= min(H, 32)) or not (0 <= gamma <= Hprime):
            raise ValueError("need 1 <= Hprime <= min(H, 32) and 0 <= gamma <= Hprime")
        self.D, self.H, self.Hprime, self.gamma = int(D), int(H), int(Hprime), int(gamma)
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else device)

    # ------------------------------------------------------------ parameters
    def standard_init(self, data: Dict, seed: int = 0) -> Dict:
        """Random initial parameters from the data: W with N(0, 1/D) entries
        (|.| for MCA, whose components are nonnegative), pi = 1/H, sigma the
        standard deviation of all of y."""
        Y = _device_tensor(data["y"], self.device)
        if Y.shape[1] != self.D:
            raise ValueError(f"data has {Y.shape[1]} columns, the model D = {self.D}")
        g = torch.Generator(device=self.device)
        g.manual_seed(int(seed))
        W = torch.randn((self.D, self.H), generator=g, device=self.device) / float(np.sqrt(self.D))
        if self.kind == "mca":
            W = W.abs()
        sigma = float(torch.std(Y.double(), correction=0))
        return {"W": W.contiguous(), "pi": 1.0 / self.H, "sigma": sigma}

    # the DSC subclass adds its value set and prior; these are the hooks
    def _phi(self):
        return None

    def _pv(self, params: Dict):
        return None

    def _nvalues(self) -> int:
        return 0

    def _theta(self, params: Dict) -> List[float]:
        return [float(params["pi"]), float(params["sigma"])]

    def _params_from_theta(self, W, th) -> Dict:
        return {"W": W, "pi": float(th[0]), "sigma": float(th[1])}

    def _state_count(self) -> int:
        return api.state_count(self.kind, self.Hprime, self.gamma)

    # ------------------------------------------------------------- inference
    def inference(self, anneal: "Annealing", params: Dict, Y, topk: int = 5,
                  beta: Optional[float] = None) -> Dict:
        """Approximate posterior information per data point: res["s"]
        (N x topk x H latent states, most likely first), res["p"] (N x topk
        truncated-posterior probabilities), plus the preselection ("sel"),
        the posterior means on it ("s_mean"), logL and the near-tie flag.
        The temperature is the schedule's last one unless `beta` is given."""
        Yd = _device_tensor(Y, self.device)
        W = _device_tensor(params["W"], self.device)
        b = anneal.beta(anneal.iterations - 1) if beta is None else float(beta)
        k = min(int(topk), self._state_count())
        out = api.estep(Yd, W, float(params.get("pi", 0.5)), float(params["sigma"]),
                        Hprime=self.Hprime, gamma=self.gamma, model=self.kind,
                        precision=self.precision, topk=k, beta=b, phi=self._phi(),
                        pv=self._pv(params))
        sel = out["sel"].long()
        N = sel.shape[0]
        slots = torch.arange(self.Hprime, device=sel.device)
        if self.kind == "dsc":
            # value codes from the three bit planes, then the values themselves
            act = out["top_mask"][..., 0].long()
            code = sum(((out["top_mask"][..., 1 + p].long()[..., None] >> slots) & 1) << p
                       for p in range(3))
            phi = torch.tensor(self._phi(), dtype=torch.float32, device=sel.device)
            vals = phi[code] * ((act[..., None] >> slots) & 1)
            s = torch.zeros((N, k, self.H), dtype=torch.float32, device=sel.device)
            s.scatter_(2, sel[:, None, :].expand(N, k, self.Hprime), vals)
            return {"s": s, "p": out["top_q"], "sel": out["sel"], "s_mean": out["s_mean"],
                    "logL": out["logL"], "flagged": out["flagged"]}
        if self.kind == "tsc":
            act = out["top_mask"][..., 0].long()
            neg = out["top_mask"][..., 1].long()
            on = (act[..., None] >> slots) & 1
            sign = 1 - 2 * ((neg[..., None] >> slots) & 1)
            vals = (on * sign).to(torch.int8)
        else:
            act = out["top_mask"].long()
            vals = ((act[..., None] >> slots) & 1).to(torch.int8)
        s = torch.zeros((N, k, self.H), dtype=torch.int8, device=sel.device)
        s.scatter_(2, sel[:, None, :].expand(N, k, self.Hprime), vals)
        return {"s": s, "p": out["top_q"], "sel": out["sel"], "s_mean": out["s_mean"],
                "logL": out["logL"], "flagged": out["flagged"]}


class BSC_ET(Model):
    """Binary sparse coding: Bernoulli prior, linear superposition."""
    kind = "bsc"


class TSC_ET(Model):
    """Ternary sparse coding: latents in {-1, 0, 1}, linear superposition."""
    kind = "tsc"


class MCA_ET(Model):
    """Maximal causes analysis: Bernoulli prior, max superposition of
    nonnegative components."""
    kind = "mca"


class MMCA_ET(Model):
    """Max-magnitude superposition: the active component of largest
    magnitude at each pixel."""
    kind = "mmca"


class DSC_ET(Model):
    """Discrete sparse coding: each latent takes one of the values phi
    (phi[0] = 0) with a learned categorical prior pv; linear superposition.
    The parameters carry "pv" beside W and sigma ("pi" = 1 - pv[0])."""
    kind = "dsc"

    def __init__(self, D: int, H: int, Hprime: int, gamma: int, phi, precision: str = "bf16",
                 device: Optional[int] = None):
        super().__init__(D, H, Hprime, gamma, precision, device)
        self.phi = tuple(float(x) for x in phi)
        if len(self.phi) < 2 or self.phi[0] != 0.0:
            raise ValueError("phi holds at least two values and phi[0] = 0")

    def standard_init(self, data: Dict, seed: int = 0) -> Dict:
        """As the other models, with pv_0 = 1 - 1/H and the rest of the
        prior spread evenly over the non-zero values."""
        p = super().standard_init(data, seed)
        V = len(self.phi)
        p["pv"] = (1.0 - 1.0 / self.H,) + (1.0 / (self.H * (V - 1)),) * (V - 1)
        return p

    def _phi(self):
        return self.phi

    def _pv(self, params: Dict):
        return tuple(float(x) for x in params["pv"])

    def _nvalues(self) -> int:
        return len(self.phi)

    def _theta(self, params: Dict) -> List[float]:
        pv = self._pv(params)
        return [1.0 - pv[0], float(params["sigma"]), *pv]

    def _params_from_theta(self, W, th) -> Dict:
        return {"W": W, "pi": float(th[0]), "sigma": float(th[1]),
                "pv": tuple(float(x) for x in th[2:])}

    def _state_count(self) -> int:
        return api.dsc_state_count(len(self.phi), self.Hprime, self.gamma)


class Annealing:
    """Schedule of an EM run: number of iterations, posterior temperature
    beta(it) in (0, 1] (deterministic annealing: q proportional to
    p(y, s)^beta), and the standard deviation of the noise added to W after
    the M-step of iteration it."""

    iterations: int = 0

    def beta(self, it: int) -> float:
        return 1.0

    def noise(self, it: int) -> float:
        return 0.0


class LinearAnnealing(Annealing):
    """Linear schedules over the first `anneal_steps` iterations (all of them
    by default): beta from beta_start to 1, parameter noise from
    noise_start to 0; constant afterwards."""

    def __init__(self, iterations: int, beta_start: float = 1.0, noise_start: float = 0.0,
                 anneal_steps: Optional[int] = None):
        if iterations < 1:
            raise ValueError("at least one iteration")
        if not (0.0 < beta_start <= 1.0):
            raise ValueError("beta_start must lie in (0, 1]")
        if noise_start < 0.0:
            raise ValueError("noise_start must be >= 0")
        self.iterations = int(iterations)
        self.beta_start = float(beta_start)
        self.noise_start = float(noise_start)
        self.anneal_steps = int(iterations if anneal_steps is None else anneal_steps)

    def _frac(self, it: int) -> float:
        if self.anneal_steps <= 1:
            return 1.0
        return min(1.0, max(0.0, it / (self.anneal_steps - 1)))

    def beta(self, it: int) -> float:
        return self.beta_start + (1.0 - self.beta_start) * self._frac(it)

    def noise(self, it: int) -> float:
        return self.noise_start * (1.0 - self._frac(it))


class EM:
    """Truncated EM: per iteration one E-step over all data with the
    statistics (at the schedule's temperature) and the FP64 M-step, both on
    the device; W, pi and sigma stay in device memory.  `lparams` holds the
    learned parameters, `logL` the per-iteration sum of the data
    log-likelihood bound (read back only when `track_logL`).
    `selected_points` (BSC/TSC) takes pi and sigma from the points best
    explained by at most gamma causes (`api.mstep_et`); W from all points."""

    def __init__(self, model: Model, anneal: Annealing, data: Optional[Dict] = None,
                 lparams: Optional[Dict] = None, track_logL: bool = True, seed: int = 0,
                 selected_points: bool = False):
        if selected_points and model.kind not in ("bsc", "tsc"):
            raise ValueError("the selected-points M-step is defined for BSC and TSC")
        self.selected_points = bool(selected_points)
        self.model = model
        self.anneal = anneal
        self.data = data
        self.lparams = lparams
        self.track_logL = track_logL
        self.logL: List[float] = []
        self._gen = torch.Generator(device=model.device)
        self._gen.manual_seed(int(seed))

    def run(self, data: Optional[Dict] = None, callback=None) -> Dict:
        """Runs the schedule; `callback(it, W, theta)` (device tensors, W the
        new dictionary, theta = (pi, sigma), DSC: (pi, sigma, pv_0, ..)) is called
        after every M-step."""
        m = self.model
        data = data if data is not None else self.data
        if data is None:
            raise ValueError("EM.run needs data ({'y': Y})")
        Y = _device_tensor(data["y"], m.device)
        if self.lparams is None:
            self.lparams = m.standard_init({"y": Y})
        W = _device_tensor(self.lparams["W"], m.device).clone()
        theta = torch.tensor(m._theta(self.lparams), dtype=torch.float64, device=m.device)
        ctx = api.context(m.device.index)
        acc = api.new_acc(m.kind, m.D, m.H, device=m.device.index, nvalues=m._nvalues())
        W_next = torch.empty_like(W)
        factor_b = m.kind in ("bsc", "tsc", "dsc")
        for it in range(self.anneal.iterations):
            beta = self.anneal.beta(it)
            want = ("logL", "k_mean", "res") if self.selected_points else ()
            pts = api.estep(Y, W, Hprime=m.Hprime, gamma=m.gamma, model=m.kind,
                            precision=m.precision, theta=theta, acc=acc, want=want, ctx=ctx,
                            factor_b=factor_b, beta=beta, phi=m._phi(), zero_acc=True)
            if self.selected_points:
                api.mstep_et(acc, W, pts, gamma=m.gamma, model=m.kind, theta=theta,
                             W_new=W_next, theta_new=theta, ctx=ctx)
            else:
                api.mstep(acc, W, model=m.kind, W_new=W_next, theta_new=theta, ctx=ctx)
            W, W_next = W_next, W
            eps = self.anneal.noise(it)
            if eps > 0.0:
                W.add_(torch.randn(W.shape, generator=self._gen, device=W.device), alpha=eps)
                if m.kind == "mca":
                    W.clamp_(min=0.0)
            if self.track_logL:
                self.logL.append(float(acc["scal"][1]))
            if callback is not None:
                callback(it, W, theta)
        self.lparams = m._params_from_theta(W, theta.cpu().numpy())
        return self.lparams
