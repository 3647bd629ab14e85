"""Shared helpers of the GPU parity tests: running the HIP path through the C
ABI, cached oracle results and the parity metrics.

Metrics (per point, over points that the oracle does not flag):
  sel      bit-exact (also required of the BF16 path)
  <s>      ||d<s>||_inf / max(||<s>_ref||_inf, 1e-3)
  logL     |d logL| / max(|logL_ref|, 1)
Tolerances: FP32 1e-5 on both; BF16 (the head/tail split and the single
product with the FP32 fix-up of the candidates) 2e-3 on <s>, 1e-4 on logL.
"""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import prosper_oracle as O

TOL = {"fp32": (1e-5, 1e-5), "bf16": (2e-3, 1e-4), "bf16x1": (2e-3, 1e-4)}


def workload_params(name, theta, Y, N=None):
    """(W, pi, sigma) at the generating parameters ("gt") or at the learning
    initialisation ("init")."""
    wl = synth.WORKLOADS[name]
    if theta == "gt":
        _, W, _, _ = synth.make_workload(name, N=1)
        return W, wl.pi, wl.sigma
    W0, pi0, s0 = synth.initial_params(wl, Y)
    return W0, pi0, s0


@functools.lru_cache(maxsize=None)
def problem(name, N, theta, seed=None):
    Y, Wgt, S, wl = synth.make_workload(name, N=N, seed=seed)
    W, pi, sigma = workload_params(name, theta, Y)
    return Y, np.ascontiguousarray(W, dtype=np.float32), float(pi), float(sigma), wl


@functools.lru_cache(maxsize=None)
def oracle_run(name, N, theta, Hp, gamma, topk=0, seed=None):
    Y, W, pi, sigma, wl = problem(name, N, theta, seed)
    return O.estep(wl.model, Y, W, pi, sigma, Hp, gamma, topk=topk)


def gpu_estep(model, prec, Y, W, pi, sigma, Hp, gamma, topk=0, accumulate=False, beta=1.0):
    import torch
    from paper_1908_06843_amd import api
    dev = torch.device("cuda", 0)
    Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(dev)
    Wd = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32)).to(dev)
    acc = api.new_acc(model, W.shape[0], W.shape[1]) if accumulate else None
    out = api.estep(Yd, Wd, pi, sigma, Hprime=Hp, gamma=gamma, model=model, precision=prec,
                    topk=topk, acc=acc, beta=beta)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if acc is not None:
        res.update({"A": acc["A"].cpu().numpy(), "B": acc["B"].cpu().numpy(),
                    "scal": acc["scal"].cpu().numpy()})
    return res


def parity_stats(g, r, idx=None):
    """Compare GPU outputs g with oracle outputs r (optionally r is for the
    subset idx of g's points)."""
    gs, gsm, gl = g["sel"], g["s_mean"], g["logL"]
    if idx is not None:
        gs, gsm, gl = gs[idx], gsm[idx], gl[idx]
    flagged = np.asarray(r["flagged"], dtype=bool)
    same = np.all(gs == r["sel"], axis=1)
    bad = (~same) & (~flagged)
    use = same & ~flagged
    es = (np.abs(gsm[use] - r["s_mean"][use]).max(axis=1)
          / np.maximum(np.abs(r["s_mean"][use]).max(axis=1), 1e-3))
    el = np.abs(gl[use].astype(np.float64) - r["logL"][use]) / np.maximum(np.abs(r["logL"][use]), 1.0)
    return dict(n=len(same), flagged=int(flagged.sum()), sel_mismatch=int(bad.sum()),
                s_max=float(es.max(initial=0.0)), s_p999=float(np.quantile(es, 0.999)) if len(es) else 0.0,
                s_mean=float(es.mean()) if len(es) else 0.0,
                l_max=float(el.max(initial=0.0)), l_mean=float(el.mean()) if len(el) else 0.0)


def assert_parity(g, r, prec, label, idx=None):
    st = parity_stats(g, r, idx)
    ts, tl = TOL[prec]
    print(f"[parity] {label} {prec}: {st}", flush=True)
    assert st["sel_mismatch"] == 0, f"{label}: unflagged selection mismatch {st}"
    assert st["s_max"] <= ts, f"{label}: <s> error {st['s_max']:.3g} > {ts}"
    assert st["l_max"] <= tl, f"{label}: logL error {st['l_max']:.3g} > {tl}"
    return st
