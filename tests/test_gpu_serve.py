"""Serving runtime (prosper_serve*) on the GPU: E-step-only inference with
continuous batching.  Results of a request are the same alone and in a mix
of concurrent requests of other sizes and (H', gamma); they match the
direct E-step entry point and the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import prosper_oracle as O
from tests._common import TOL

pytestmark = pytest.mark.gpu


def _dictionary():
    wl = synth.WORKLOADS["serve"]
    g = synth.rng(wl.data_seed)
    W = synth.unit_norm_gaussian_dictionary(g, wl.D, wl.H).astype(np.float32)
    return wl, g, W


def _patches(g, W, wl, n):
    S = synth.sample_binary(g, n, wl.H, wl.pi)
    return synth.linear_observations(g, W.astype(np.float64), S, wl.sigma).astype(np.float32)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_same_alone_and_in_the_mix(prec):
    from paper_1908_06843_amd.serve import Server
    wl, g, W = _dictionary()
    probe = _patches(g, W, wl, 300)
    srv = Server(W, wl.pi, wl.sigma, precision=prec, mem_budget_bytes=64 << 20,
                 max_inflight=8, n_streams=4)
    try:
        alone = {}
        for hp, gm in ((8, 3), (10, 4), (12, 5)):
            rid, out = srv.submit(probe, hp, gm, topk=3,
                                  outputs=("sel", "s_mean", "logL", "flagged"))
            srv.wait(rid)
            alone[(hp, gm)] = out
        # the same requests inside a burst of others of mixed sizes and shapes
        sizes, mix = synth.serving_requests(60, seed=9)
        pending = []
        for i, (n, (hp, gm)) in enumerate(zip(sizes, mix)):
            pending.append(srv.submit(_patches(g, W, wl, int(min(n, 1500))), hp, gm)[0])
            if i in (5, 25, 45):
                for hp2, gm2 in ((8, 3), (10, 4), (12, 5)):
                    rid, out = srv.submit(probe, hp2, gm2, topk=3,
                                          outputs=("sel", "s_mean", "logL", "flagged"))
                    pending.append(rid)
                    alone.setdefault(("mix", hp2, gm2), []).append((rid, out))
        for rid in pending:
            srv.wait(rid)
        for hp, gm in ((8, 3), (10, 4), (12, 5)):
            ref = alone[(hp, gm)]
            for _, out in alone[("mix", hp, gm)]:
                for k in ("sel", "s_mean", "logL", "flagged", "top_mask", "top_q"):
                    np.testing.assert_array_equal(out[k], ref[k], err_msg=f"{k} H'={hp}")
    finally:
        srv.stop()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_serving_matches_oracle(prec):
    from paper_1908_06843_amd.serve import Server
    wl, g, W = _dictionary()
    Y = _patches(g, W, wl, 97)
    srv = Server(W, wl.pi, wl.sigma, precision=prec, mem_budget_bytes=32 << 20)
    try:
        for hp, gm in ((8, 3), (10, 4), (12, 5)):
            rid, out = srv.submit(Y, hp, gm, outputs=("sel", "s_mean", "logL", "flagged"))
            lat = srv.wait(rid)
            assert lat > 0
            r = O.estep("bsc", Y, W, wl.pi, wl.sigma, hp, gm)
            ok = (~r["flagged"].astype(bool)) & np.all(out["sel"] == r["sel"], axis=1)
            fl = r["flagged"].astype(bool)
            assert np.all(np.all(out["sel"] == r["sel"], axis=1) | fl)
            ts, tl = TOL[prec]
            es = (np.abs(out["s_mean"][ok] - r["s_mean"][ok]).max(1)
                  / np.maximum(np.abs(r["s_mean"][ok]).max(1), 1e-3))
            el = (np.abs(out["logL"][ok].astype(np.float64) - r["logL"][ok])
                  / np.maximum(np.abs(r["logL"][ok]), 1.0))
            assert es.max() <= ts and el.max() <= tl, (hp, gm, es.max(), el.max())
    finally:
        srv.stop()


def test_serving_equals_direct_estep():
    import torch
    from paper_1908_06843_amd import api
    from paper_1908_06843_amd.serve import Server
    wl, g, W = _dictionary()
    Y = _patches(g, W, wl, 513)
    srv = Server(W, wl.pi, wl.sigma, precision="bf16", mem_budget_bytes=32 << 20)
    try:
        rid, out = srv.submit(Y, 10, 4, topk=2, outputs=("sel", "s_mean", "logL", "flagged"))
        srv.wait(rid)
    finally:
        srv.stop()
    dev = torch.device("cuda", 0)
    d = api.estep(torch.tensor(Y, device=dev), torch.tensor(W, device=dev), wl.pi, wl.sigma,
                  Hprime=10, gamma=4, precision="bf16", topk=2)
    torch.cuda.synchronize()
    for k in ("sel", "s_mean", "logL", "flagged", "top_q"):
        np.testing.assert_array_equal(out[k], d[k].cpu().numpy(), err_msg=k)
    np.testing.assert_array_equal(out["top_mask"].view(np.int32), d["top_mask"].cpu().numpy())


def test_admission_by_memory_and_errors():
    from paper_1908_06843_amd import _lib
    from paper_1908_06843_amd.serve import Server
    wl, g, W = _dictionary()
    # a budget that holds about two 1000-patch requests at once
    srv = Server(W, wl.pi, wl.sigma, precision="bf16", mem_budget_bytes=3 << 20,
                 max_inflight=16)
    try:
        with pytest.raises(_lib.ProsperError):
            srv.submit(_patches(g, W, wl, 4000), 8, 3)      # larger than the whole budget
        with pytest.raises(_lib.ProsperError):
            srv.submit(_patches(g, W, wl, 10), 40, 3)       # H' out of range
        ids = [srv.submit(_patches(g, W, wl, 1000), 8, 3)[0] for _ in range(12)]
        lats = [srv.wait(r) for r in ids]
        assert all(x > 0 for x in lats)
        with pytest.raises(_lib.ProsperError):
            srv.wait(ids[0])                                # already collected
    finally:
        srv.stop()


def _mmca_problem(N, seed=7):
    """MMCA data: signed N(0,1) dictionary D=100, H=200, pi=3/H, sigma=0.3."""
    g = synth.rng(seed)
    W = g.standard_normal((100, 200))
    S = synth.sample_binary(g, N, 200, 3.0 / 200)
    Y = O.superposition(O.MMCA, W, S) + 0.3 * g.standard_normal((N, 100))
    return Y.astype(np.float32), W.astype(np.float32), 3.0 / 200, 0.3


@pytest.mark.parametrize("model,name,Hp,gamma", [("tsc", "tsc", 8, 3), ("mca", "mca", 10, 3),
                                                 ("mmca", None, 10, 3)])
def test_serving_other_models_match_oracle(model, name, Hp, gamma):
    """TSC, MCA and MMCA dictionaries served: per-point outputs and the top
    states against the oracle."""
    from paper_1908_06843_amd.serve import Server
    if model == "mmca":
        Y, W, pi, sigma = _mmca_problem(90)
    else:
        Y, W, _, wl = synth.make_workload(name, N=90)
        pi, sigma = wl.pi, wl.sigma
        W = W.astype(np.float32)
    srv = Server(W, pi, sigma, model=model, precision="fp32", mem_budget_bytes=32 << 20)
    try:
        rid, out = srv.submit(Y, Hp, gamma, topk=3,
                              outputs=("sel", "s_mean", "logL", "flagged", "top_mask", "top_q"))
        srv.wait(rid)
    finally:
        srv.stop()
    r = O.estep(model, Y, W, pi, sigma, Hp, gamma, topk=3)
    fl = r["flagged"].astype(bool)
    same = np.all(out["sel"] == r["sel"], axis=1)
    assert np.all(same | fl)
    ok = same & ~fl
    ts, tl = TOL["fp32"]
    es = (np.abs(out["s_mean"][ok] - r["s_mean"][ok]).max(1)
          / np.maximum(np.abs(r["s_mean"][ok]).max(1), 1e-3))
    el = (np.abs(out["logL"][ok].astype(np.float64) - r["logL"][ok])
          / np.maximum(np.abs(r["logL"][ok]), 1.0))
    assert es.max() <= ts and el.max() <= tl, (es.max(), el.max())
    # single-state probabilities: the FP32 rounding of one log-joint, about
    # 15 roundings of |lj|; |lj| reaches ~100-200 log2 units for MCA and,
    # relative to the zero state, lam ||y||^2 ~ 800 for MMCA
    rq = {"mca": 1e-4, "mmca": 5e-4}.get(model, 3e-5)
    np.testing.assert_allclose(out["top_q"][ok], r["top_q"][ok], rtol=rq, atol=1e-7)


def test_wait_stages_add_up():
    """The stage split of prosper_serve_wait_stages: all stages >= 0, the
    host stages add up to the total, the batch's GPU time fits in the span
    from the start of its launch calls (its first event is recorded before
    the rest of the launch is issued, so the GPU may start meanwhile) to the
    completion seen."""
    from paper_1908_06843_amd.serve import Server
    wl, g, W = _dictionary()
    srv = Server(W, wl.pi, wl.sigma, precision="bf16", mem_budget_bytes=32 << 20)
    try:
        ids = [srv.submit(_patches(g, W, wl, n), 10, 4)[0] for n in (5, 300, 17, 2000, 1)]
        for rid in ids:
            st = srv.wait_stages(rid)
            print(f"[stages] {st}", flush=True)
            assert all(v >= 0.0 for v in st.values())
            host = st["queue"] + st["launch"] + st["device_span"] + st["delivery"]
            assert abs(host - st["total"]) <= 1e-3 + 1e-6 * st["total"]
            assert 0.0 < st["gpu"] <= st["launch"] + st["device_span"] + 0.05
    finally:
        srv.stop()
