"""Seeded synthetic workloads for the truncated-EM sparse-coding models.

This module only *samples* data from the generative process of the paper
(Section "Learning Algorithm and Data Models", Eq. 1-2 with the per-model
priors and superpositions of Table 1).  It holds none of the inference
arithmetic: no posterior, no state set, no log-joint, no parameter update.
Both the FP64 oracle (test infrastructure) and the GPU library consume the
float32 arrays produced here; they share data, never computation.

Every generator takes an explicit seed and uses NumPy's PCG64 bit generator,
draws in float64 and returns float32 arrays (the precision of the GPU input).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "rng", "bars_dictionary", "unit_norm_gaussian_dictionary",
    "abs_gaussian_dictionary", "sample_binary", "sample_ternary", "sample_discrete",
    "linear_observations", "max_observations", "Workload", "WORKLOADS",
    "make_workload", "initial_params", "initial_dsc_prior", "serving_requests",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# dictionaries (ground-truth W, D x H, column h is component h)
# --------------------------------------------------------------------------
def bars_dictionary(side: int = 5, amplitude: float = 10.0) -> np.ndarray:
    """Bars dictionary on a side x side image flattened row-major (d = side*r + c).

    Component h < side is horizontal bar (row h); component h >= side is the
    vertical bar (column h - side).  Amplitude 10 per active pixel.
    """
    D, H = side * side, 2 * side
    W = np.zeros((D, H), dtype=np.float64)
    for h in range(side):
        for c in range(side):
            W[side * h + c, h] = amplitude
    for h in range(side):
        for r in range(side):
            W[side * r + h, side + h] = amplitude
    return W


def unit_norm_gaussian_dictionary(g: np.random.Generator, D: int, H: int) -> np.ndarray:
    W = g.standard_normal((D, H))
    W /= np.sqrt((W * W).sum(axis=0, keepdims=True))
    return W


def abs_gaussian_dictionary(g: np.random.Generator, D: int, H: int) -> np.ndarray:
    return np.abs(g.standard_normal((D, H)))


# --------------------------------------------------------------------------
# latents and observations (Eq. 1: prior draw; Eq. 2: noisy superposition)
# --------------------------------------------------------------------------
def sample_binary(g: np.random.Generator, N: int, H: int, pi: float) -> np.ndarray:
    """s_h ~ Bernoulli(pi), independently (BSC / MCA prior)."""
    return (g.random((N, H)) < pi).astype(np.float64)


def sample_ternary(g: np.random.Generator, N: int, H: int, pi: float) -> np.ndarray:
    """s_h in {-1, 0, +1} with P(+1) = P(-1) = pi/2 (zero-mean TSC prior)."""
    u = g.random((N, H))
    s = np.zeros((N, H))
    s[u < pi / 2] = -1.0
    s[(u >= pi / 2) & (u < pi)] = 1.0
    return s


def sample_discrete(g: np.random.Generator, N: int, H: int, phi, pv) -> np.ndarray:
    """s_h = phi_v with probability pv_v, independently (DSC categorical prior)."""
    codes = g.choice(len(phi), size=(N, H), p=np.asarray(pv, dtype=np.float64))
    return np.asarray(phi, dtype=np.float64)[codes]


def linear_observations(g: np.random.Generator, W: np.ndarray, S: np.ndarray,
                        sigma: float) -> np.ndarray:
    """y = W s + sigma * eps, eps ~ N(0, I)  (linear superposition)."""
    return S @ W.T + sigma * g.standard_normal((S.shape[0], W.shape[0]))


def max_observations(g: np.random.Generator, W: np.ndarray, S: np.ndarray,
                     sigma: float, chunk: int = 4096) -> np.ndarray:
    """y_d = max_h s_h W_dh + sigma * eps_d  (max superposition)."""
    N, D = S.shape[0], W.shape[0]
    Y = np.empty((N, D))
    for a in range(0, N, chunk):
        Sc = S[a:a + chunk]
        Y[a:a + chunk] = (Sc[:, None, :] * W[None, :, :]).max(axis=2)
    return Y + sigma * g.standard_normal((N, D))


# --------------------------------------------------------------------------
# the five workloads (sizes, priors, noise, truncation parameters)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    model: str            # "bsc" | "tsc" | "mca"
    D: int
    H: int
    N: int
    pi: float
    sigma: float
    Hprime: int
    gamma: int
    data_seed: int
    init_seed: int
    iters: int = 1
    note: str = ""
    phi: Tuple[float, ...] = ()   # DSC value set (phi_0 = 0)
    pv: Tuple[float, ...] = ()    # DSC prior over the values


WORKLOADS = {
    "bars": Workload("bars", "bsc", 25, 10, 1000, 2.0 / 10, 2.0, 10, 10, 0, 100, 10,
                     "5x5 bars, amplitude 10, exact posterior (H'=H=gamma)"),
    "bsc256": Workload("bsc256", "bsc", 256, 256, 200000, 5.0 / 256, 0.5, 12, 4, 1, 101, 20,
                       "Gaussian unit-norm dictionary, D=H=256"),
    "mca": Workload("mca", "mca", 100, 200, 100000, 3.0 / 200, 0.3, 10, 3, 2, 102, 1,
                    "10x10 patches, |N(0,1)| dictionary, max superposition"),
    "tsc": Workload("tsc", "tsc", 144, 100, 100000, 4.0 / 100, 1.0, 8, 3, 3, 103, 1,
                    "ternary latents, Gaussian unit-norm dictionary"),
    "serve": Workload("serve", "bsc", 256, 512, 0, 6.0 / 512, 0.5, 12, 5, 4, 104, 0,
                      "resident dictionary for E-step-only serving"),
    "dsc": Workload("dsc", "dsc", 144, 100, 100000, 0.04, 1.0, 8, 3, 5, 105, 1,
                    "discrete latents in {0, 1, -1, 2, -2}, Gaussian unit-norm dictionary",
                    phi=(0.0, 1.0, -1.0, 2.0, -2.0), pv=(0.96, 0.015, 0.015, 0.005, 0.005)),
}


def make_workload(name: str, N: Optional[int] = None, seed: Optional[int] = None
                  ) -> Tuple[np.ndarray, np.ndarray, np.ndarray, Workload]:
    """Return (Y float32 N x D, W_gt float32 D x H, S float64 N x H, workload).

    N and seed override the workload's defaults (smaller parity cases use the
    same recipe at fewer points).
    """
    wl = WORKLOADS[name]
    N = wl.N if N is None else N
    g = rng(wl.data_seed if seed is None else seed)
    if name == "bars":
        W = bars_dictionary()
    elif wl.model == "mca":
        W = abs_gaussian_dictionary(g, wl.D, wl.H)
    else:
        W = unit_norm_gaussian_dictionary(g, wl.D, wl.H)
    if wl.model == "tsc":
        S = sample_ternary(g, N, wl.H, wl.pi)
    elif wl.model == "dsc":
        S = sample_discrete(g, N, wl.H, wl.phi, wl.pv)
    else:
        S = sample_binary(g, N, wl.H, wl.pi)
    if wl.model == "mca":
        Y = max_observations(g, W, S, wl.sigma)
    else:
        Y = linear_observations(g, W, S, wl.sigma)
    return Y.astype(np.float32), W.astype(np.float32), S, wl


def initial_params(wl: Workload, Y: np.ndarray, seed: Optional[int] = None):
    """Learning-run initialisation: W0, pi0 = 1/H, sigma0 = std of all of Y.

    Bars: W0 ~ N(0, 1).  Other workloads: W0 ~ N(0, 1/D); MCA takes |.| so the
    initial components are nonnegative like the generating ones.  DSC starts
    its prior at pv_0 = 1 - 1/H with the rest spread evenly (see
    initial_dsc_prior).
    """
    g = rng(wl.init_seed if seed is None else seed)
    if wl.name == "bars":
        W0 = g.standard_normal((wl.D, wl.H))
    else:
        W0 = g.standard_normal((wl.D, wl.H)) / np.sqrt(wl.D)
        if wl.model == "mca":
            W0 = np.abs(W0)
    pi0 = 1.0 / wl.H
    sigma0 = float(np.asarray(Y, dtype=np.float64).std())
    return W0.astype(np.float32), pi0, sigma0


def initial_dsc_prior(wl: Workload) -> Tuple[float, ...]:
    """pv_0 = 1 - 1/H, the other V - 1 values 1/(H (V - 1)) each."""
    V = len(wl.phi)
    return (1.0 - 1.0 / wl.H,) + (1.0 / (wl.H * (V - 1)),) * (V - 1)


def serving_requests(n_requests: int, seed: int = 4, max_patches: int = 4096,
                     mix=((8, 3), (10, 4), (12, 5))):
    """Request sizes and truncation parameters for the serving workload.

    Patch counts are log-uniform on [1, max_patches]: floor(exp(U[0, ln(max+1)))).
    (H', gamma) is uniform over `mix`.
    """
    g = rng(seed)
    u = g.random(n_requests) * np.log(max_patches + 1)
    sizes = np.minimum(np.floor(np.exp(u)).astype(np.int64), max_patches)
    sizes = np.maximum(sizes, 1)
    choice = g.integers(0, len(mix), n_requests)
    return sizes, [mix[c] for c in choice]
