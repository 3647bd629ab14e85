"""GPU parity of the selected-points M-step (prosper_mstep_et) and of the
per-point E-step outputs it takes (<k>_n and <||y_n - W s||^2>_n), against
the FP64 oracle.

The kept set is the N_cut points of largest logL.  The GPU ranks its own
FP32 logL, so near the cut its set may differ from the oracle's by points
whose logL agree to rounding; the checks allow exactly that and otherwise
compare the update on the GPU's set.  A planted-tie case drives the
selection kernel directly (equal logL with distinct <k> and res, across
many 1024-point chunks) to check the lower-index rule."""
import numpy as np
import pytest

import synth
from oracle import prosper_oracle as O
from tests._common import problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def oracle_point_res(Y, W, est, H):
    out = np.zeros(Y.shape[0])
    for n, (c, q) in enumerate(est["posterior"]):
        S = np.zeros((len(est["table"]), H))
        for i, (slots, vals) in enumerate(est["table"]):
            for j, v in zip(slots, vals):
                S[i, c[j]] = v
        R = Y[n][None, :] - S @ W.T
        out[n] = float(q @ (R * R).sum(1))
    return out


def kept(logL, n_cut):
    return np.sort(np.lexsort((np.arange(len(logL)), -np.asarray(logL, np.float64)))[:n_cut])


@pytest.mark.parametrize("name,model,N,Hp,gamma", [("bsc256", "bsc", 1500, 12, 4),
                                                   ("tsc", "tsc", 1200, 8, 3),
                                                   ("serve", "bsc", 900, 10, 2)])
def test_selected_points_mstep_matches_oracle(name, model, N, Hp, gamma):
    import torch
    from paper_1908_06843_amd import api
    Y, W, pi, sigma, wl = problem(name, N, "init")
    dev = torch.device("cuda", 0)
    acc = api.new_acc(model, W.shape[0], W.shape[1])
    Wd = torch.tensor(W, device=dev)
    out = api.estep(torch.tensor(Y, device=dev), Wd, pi, sigma, Hprime=Hp, gamma=gamma,
                    model=model, acc=acc, want=("sel", "logL", "k_mean", "res", "flagged"))
    W1, th = api.mstep_et(acc, Wd, out, gamma=gamma, model=model, pi=pi)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    r = O.estep(model, Y, W, pi, sigma, Hp, gamma, keep_posterior=True)
    ok = ~r["flagged"] & np.all(g["sel"] == r["sel"], axis=1)
    res_o = oracle_point_res(Y.astype(np.float64), W.astype(np.float64), r, W.shape[1])
    ek = np.abs(g["k_mean"][ok] - r["k_mean"][ok]).max() / max(np.abs(r["k_mean"]).max(), 1e-3)
    er = np.abs(g["res"][ok] - res_o[ok]) / np.maximum(res_o[ok], 1.0)
    print(f"[points] {name}: k {ek:.2e} res {er.max():.2e}", flush=True)
    assert ek < 1e-5 and er.max() < 1e-5
    # the kept sets agree but for points at the cut within rounding
    H = W.shape[1]
    A, B = O.truncated_prior_moments(H, gamma, pi)
    n_cut = min(N, max(1, int(round(N * A))))
    Mg, Mo = kept(g["logL"], n_cut), kept(r["logL"], n_cut)
    T = np.sort(r["logL"])[::-1][n_cut - 1]
    diff = np.setxor1d(Mg, Mo)
    assert np.all(np.abs(r["logL"][diff] - T) <= 1e-5 * max(1.0, abs(T))), diff
    # the update on the GPU's set, in FP64 from the oracle's per-point values
    pi_ref = pi * float(np.mean(r["k_mean"][Mg])) * A / B
    s_ref = np.sqrt(float(res_o[Mg].sum()) / (n_cut * Y.shape[1]))
    th = th.cpu().numpy()
    Wr, _, _ = O.mstep(model, Y, W, r)
    print(f"[mstep_et] {name}: n_cut {n_cut}/{N} set diff {len(diff)} W {rel(W1.cpu().numpy(), Wr):.2e} "
          f"pi {th[0]} vs {pi_ref} sigma {th[1]} vs {s_ref}", flush=True)
    assert th[0] == pytest.approx(pi_ref, rel=2e-5)
    assert th[1] == pytest.approx(s_ref, rel=2e-5)
    assert rel(W1.cpu().numpy(), Wr) < 1e-4
    # and against the oracle's own variant when the sets agree
    if len(diff) == 0:
        _, pn, sn, _ = O.mstep_et(model, Y, W, r, pi, gamma)
        assert th[0] == pytest.approx(pn, rel=2e-5) and th[1] == pytest.approx(sn, rel=2e-5)


@pytest.mark.parametrize("N", [5000, 300007])
def test_selection_kernel_takes_lower_indices_on_ties(N):
    """Synthetic logL with a large block of equal values across the cut and
    distinct <k> and res: the kept points at the cut are the lowest indices
    of the block, over many 1024-point chunks."""
    import torch
    from paper_1908_06843_amd import api
    g = np.random.default_rng(4)
    H, D, gamma, pi = 64, 32, 3, 0.03
    A, B = O.truncated_prior_moments(H, gamma, pi)
    n_cut = min(N, max(1, int(round(N * A))))
    logL = g.standard_normal(N).astype(np.float32)
    order = np.argsort(-logL.astype(np.float64), kind="stable")
    T = logL[order[n_cut - 1]]
    tie = order[n_cut - 40:n_cut + 400]      # 440 points straddling the cut
    logL[tie] = T
    k_mean = g.random(N).astype(np.float32) * 3
    res = (g.random(N) * 50 + 10).astype(np.float32)
    M = kept(logL, n_cut)
    above = int((logL > T).sum())
    eq = np.sort(np.nonzero(logL == T)[0])
    assert np.array_equal(np.intersect1d(M, eq), eq[:n_cut - above])
    pi_ref = pi * float(np.mean(k_mean[M].astype(np.float64))) * A / B
    s_ref = np.sqrt(float(res[M].astype(np.float64).sum()) / (n_cut * D))
    dev = torch.device("cuda", 0)
    acc = api.new_acc("bsc", D, H)
    acc["B"].copy_(torch.eye(H, device=dev))
    W = torch.zeros((D, H), device=dev)
    pts = {"logL": torch.tensor(logL, device=dev), "k_mean": torch.tensor(k_mean, device=dev),
           "res": torch.tensor(res, device=dev)}
    acc["scal"][4] = N
    _, th = api.mstep_et(acc, W, pts, gamma=gamma, pi=pi)
    th = th.cpu().numpy()
    print(f"[ties] N={N} n_cut={n_cut} at the cut {n_cut - above}/{len(eq)}: pi {th[0]} vs {pi_ref}"
          f" sigma {th[1]} vs {s_ref}", flush=True)
    assert th[0] == pytest.approx(pi_ref, rel=1e-9)
    assert th[1] == pytest.approx(s_ref, rel=1e-9)


def test_per_point_outputs_rejected_for_max_models():
    import torch
    from paper_1908_06843_amd import api
    dev = torch.device("cuda", 0)
    Y = torch.rand((10, 16), device=dev)
    W = torch.rand((16, 8), device=dev)
    with pytest.raises(api.ProsperError):
        api.estep(Y, W, 0.1, 0.5, Hprime=4, gamma=2, model="mca", want=("k_mean",))


def test_em_driver_selected_points_iteration():
    """EM(..., selected_points=True): one iteration against the oracle's
    E-step and selected-points M-step from the same parameters."""
    import torch
    from paper_1908_06843_amd import em
    Y, _, _, wl = synth.make_workload("tsc", N=600)
    model = em.TSC_ET(wl.D, wl.H, 8, 3, precision="fp32", device=0)
    params = model.standard_init({"y": Y}, seed=2)
    W0 = params["W"].cpu().numpy().astype(np.float64)
    run = em.EM(model, em.LinearAnnealing(1), data={"y": Y}, lparams=params,
                selected_points=True)
    out = run.run()
    r = O.estep("tsc", Y, W0, params["pi"], params["sigma"], 8, 3, keep_posterior=True)
    Wr, pr, sr, _ = O.mstep_et("tsc", Y, W0, r, params["pi"], 3)
    print(f"[em-et] W {rel(out['W'].cpu().numpy(), Wr):.2e} pi {out['pi']} vs {pr} "
          f"sigma {out['sigma']} vs {sr}", flush=True)
    assert rel(out["W"].cpu().numpy(), Wr) < 1e-4
    assert out["pi"] == pytest.approx(pr, rel=1e-3)     # the kept set may move at the cut
    assert out["sigma"] == pytest.approx(sr, rel=1e-3)
