"""GPU parity of the DSC path (discrete latents with a categorical prior,
linear superposition; Table 1) against the FP64 oracle: preselection with
the DSC score, the table-driven walk over value codes, the top states, the
statistics (A, B, scal and the value counts), the tempered posterior, the
allocation-free entry point and the M-step with its prior update.

Tolerances are those of the other linear models (FP32: 1e-5 relative on
<s> and logL; BF16: 2e-3 and 1e-4), with the DSC terms kept at TSC's scale
(unit-norm components, values up to 2 in magnitude, sigma = 1).
"""
import numpy as np
import pytest

import synth
from oracle import prosper_oracle as O
from tests._common import assert_parity, parity_stats

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["dsc"]


def dsc_problem(N, theta, seed=None):
    Y, Wgt, _, wl = synth.make_workload("dsc", N=N, seed=seed)
    if theta == "gt":
        return Y, Wgt, wl.phi, wl.pv, wl.sigma
    W0, _, s0 = synth.initial_params(wl, Y)
    return Y, W0, wl.phi, synth.initial_dsc_prior(wl), s0


def run_gpu(Y, W, phi, pv, sigma, Hp, gamma, prec="fp32", topk=0, accumulate=False, beta=1.0,
            static=False):
    import torch
    from paper_1908_06843_amd import api
    dev = torch.device("cuda", 0)
    Yd = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(dev)
    Wd = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32)).to(dev)
    acc = api.new_acc("dsc", W.shape[0], W.shape[1], nvalues=len(phi)) if accumulate else None
    out = api.estep(Yd, Wd, sigma=sigma, Hprime=Hp, gamma=gamma, model="dsc", precision=prec,
                    topk=topk, acc=acc, beta=beta, phi=phi, pv=pv, static=static)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if acc is not None:
        res.update({k: v.cpu().numpy() for k, v in acc.items()})
    return res


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def decode_top(mask, sel_row, H):
    """GPU top state (4 words) -> (slots, codes) of the oracle's table."""
    act = int(mask[0])
    slots, codes = [], []
    j, m = 0, act
    while m:
        if m & 1:
            c = ((int(mask[1]) >> j) & 1) | (((int(mask[2]) >> j) & 1) << 1) \
                | (((int(mask[3]) >> j) & 1) << 2)
            slots.append(j)
            codes.append(c)
        m >>= 1
        j += 1
    return tuple(slots), tuple(codes)


@pytest.mark.parametrize("theta", ["gt", "init"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_dsc_point_parity(prec, theta):
    N = 301   # 75 full groups of four points and a ragged one
    Y, W, phi, pv, sigma = dsc_problem(N, theta)
    print(f"[case] dsc {prec} {theta} N={N}", flush=True)
    g = run_gpu(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, prec)
    r = O.dsc_estep(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma)
    assert_parity(g, r, prec, f"dsc {theta}")


def test_dsc_top_states():
    N, topk = 120, 5
    Y, W, phi, pv, sigma = dsc_problem(N, "gt", seed=17)
    g = run_gpu(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, topk=topk)
    r = O.dsc_estep(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, topk=topk)
    ok = ~np.asarray(r["flagged"], dtype=bool) & np.all(g["sel"] == r["sel"], axis=1)
    np.testing.assert_allclose(g["top_q"][ok], r["top_q"][ok], rtol=3e-5, atol=1e-7)
    tab = r["table"]
    checked = 0
    for n in np.nonzero(ok)[0]:
        q = r["top_q"][n]
        for t in range(topk):
            # order is decided where the oracle's probabilities are apart
            apart = (t == 0 or q[t - 1] - q[t] > 1e-4 * q[t]) and \
                    (t == topk - 1 or q[t] - q[t + 1] > 1e-4 * q[t])
            if apart:
                assert decode_top(g["top_mask"][n, t], g["sel"][n], W.shape[1]) == \
                    tab[r["top_index"][n, t]], (n, t)
                checked += 1
    assert checked > N


@pytest.mark.parametrize("phi,pv,Hp,gamma", [
    ((0.0, 1.0), (0.97, 0.03), 10, 4),                       # V = 2: BSC's states
    ((0.0, 1.0, -1.0), (0.96, 0.02, 0.02), 8, 3),             # V = 3: TSC's states
    ((0.0, 0.5, -0.5, 1.0, -1.0, 2.0, -2.0, 3.0),             # V = 8: full 3-bit codes
     (0.93, 0.02, 0.02, 0.01, 0.01, 0.005, 0.004, 0.001), 5, 3),
])
def test_dsc_value_sets_with_statistics(phi, pv, Hp, gamma):
    N, D, H = 180, 64, 40
    gen = synth.rng(23)
    W = synth.unit_norm_gaussian_dictionary(gen, D, H)
    S = synth.sample_discrete(gen, N, H, phi, pv)
    Y = (S @ W.T + 0.8 * gen.standard_normal((N, D))).astype(np.float32)
    W = W.astype(np.float32)
    print(f"[case] dsc V={len(phi)} ({Hp},{gamma})", flush=True)
    g = run_gpu(Y, W, phi, pv, 0.8, Hp, gamma, accumulate=True)
    r = O.dsc_estep(Y, W, phi, pv, 0.8, Hp, gamma)
    assert_parity(g, r, "fp32", f"dsc V={len(phi)}")
    flagged = np.asarray(r["flagged"], dtype=bool)
    if flagged.any():   # sums on the GPU's (equally valid) candidate sets
        r = O.dsc_estep(Y, W, phi, pv, 0.8, Hp, gamma, sel=g["sel"])
    Bg = np.triu(g["B"]) + np.triu(g["B"], 1).T
    ea, eb = rel(g["A"], r["A"]), rel(Bg, r["B"])
    ev = rel(g["vcount"][1:], r["vcount"][1:])
    print(f"[stats] A {ea:.2e} B {eb:.2e} vcount {ev:.2e}", flush=True)
    assert ea < 2e-5 and eb < 2e-5 and ev < 1e-5
    assert g["scal"][0] == pytest.approx(r["scal"][0], rel=1e-5)
    assert g["scal"][1] == pytest.approx(r["scal"][1], rel=1e-5)
    assert g["scal"][2] == pytest.approx(r["scal"][2], rel=1e-6)
    assert g["scal"][4] == N


def test_dsc_tempered_posterior():
    N = 100
    Y, W, phi, pv, sigma = dsc_problem(N, "init", seed=31)
    g = run_gpu(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, topk=3, beta=0.6)
    r = O.dsc_estep(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, topk=3, beta=0.6)
    assert_parity(g, r, "fp32", "dsc beta=0.6")
    ok = ~np.asarray(r["flagged"], dtype=bool)
    np.testing.assert_allclose(g["top_q"][ok], r["top_q"][ok], rtol=3e-5, atol=1e-7)


def test_dsc_static_entry_matches_context_entry():
    N = 257
    Y, W, phi, pv, sigma = dsc_problem(N, "gt", seed=41)
    a = run_gpu(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, topk=2, accumulate=True)
    b = run_gpu(Y, W, phi, pv, sigma, WL.Hprime, WL.gamma, topk=2, accumulate=True, static=True)
    for k in ("sel", "s_mean", "logL", "flagged", "top_mask", "top_q"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for k in ("A", "B", "vcount"):
        assert rel(b[k], a[k]) < 1e-5, k


def test_dsc_mstep_matches_oracle():
    """E-step statistics and M-step on the device vs the oracle's E-step and
    M-step (W = A B^-1, sigma from the direct sweep, pv from the value
    counts), every latent in every point's candidate set."""
    import torch
    from paper_1908_06843_amd import api
    phi, pv = (0.0, 1.0, -1.0, 2.0), (0.7, 0.12, 0.12, 0.06)
    N, D, H, Hp, gamma = 400, 16, 8, 8, 3
    gen = synth.rng(51)
    Wt = synth.unit_norm_gaussian_dictionary(gen, D, H)
    S = synth.sample_discrete(gen, N, H, phi, pv)
    Y = (S @ Wt.T + 0.4 * gen.standard_normal((N, D))).astype(np.float32)
    W0 = (Wt + 0.2 * gen.standard_normal((D, H))).astype(np.float32)
    pv0 = (0.6, 0.15, 0.15, 0.1)
    dev = torch.device("cuda", 0)
    acc = api.new_acc("dsc", D, H, nvalues=4)
    Wd = torch.tensor(W0, device=dev)
    api.estep(torch.tensor(Y, device=dev), Wd, sigma=0.5, Hprime=Hp, gamma=gamma, model="dsc",
              phi=phi, pv=pv0, acc=acc, want=())
    W1, th = api.mstep(acc, Wd, model="dsc")
    torch.cuda.synchronize()
    r = O.dsc_estep(Y, W0, phi, pv0, 0.5, Hp, gamma, keep_posterior=True)
    Wr, pvr, sr = O.dsc_mstep(Y, W0, r)
    th = th.cpu().numpy()
    eW = rel(W1.cpu().numpy(), Wr)
    print(f"[mstep] W {eW:.2e} pv {th[2:]} vs {pvr} sigma {th[1]} vs {sr}", flush=True)
    assert eW < 1e-4
    np.testing.assert_allclose(th[2:], pvr, rtol=1e-5)
    assert th[0] == pytest.approx(1.0 - pvr[0], rel=1e-5)
    assert th[1] == pytest.approx(sr, rel=1e-4)


def test_dsc_device_theta_and_em_iterations():
    """Three EM iterations with theta = (pi, sigma, pv) kept on the device,
    each compared with the oracle's iteration from the same parameters."""
    import torch
    from paper_1908_06843_amd import api
    phi, pv = (0.0, 1.0, -1.0, 2.0, -2.0), (0.9, 0.03, 0.03, 0.02, 0.02)
    N, D, H, Hp, gamma = 300, 36, 12, 6, 3
    gen = synth.rng(61)
    Wt = synth.unit_norm_gaussian_dictionary(gen, D, H)
    S = synth.sample_discrete(gen, N, H, phi, pv)
    Y = (S @ Wt.T + 0.5 * gen.standard_normal((N, D))).astype(np.float32)
    W = (Wt + 0.3 * gen.standard_normal((D, H))).astype(np.float32)
    dev = torch.device("cuda", 0)
    Yd = torch.tensor(Y, device=dev)
    Wd = torch.tensor(W, device=dev)
    prior = np.array([0.8, 0.05, 0.05, 0.05, 0.05])
    theta = torch.tensor([0.2, 0.7, *prior], dtype=torch.float64, device=dev)
    acc = api.new_acc("dsc", D, H, nvalues=5)
    W2 = torch.empty_like(Wd)
    for it in range(3):
        Wc = Wd.cpu().numpy()
        th = theta.cpu().numpy()
        api.zero_acc(acc)
        api.estep(Yd, Wd, Hprime=Hp, gamma=gamma, model="dsc", phi=phi, theta=theta, acc=acc,
                  want=())
        api.mstep(acc, Wd, model="dsc", W_new=W2, theta_new=theta)
        Wd, W2 = W2, Wd
        torch.cuda.synchronize()
        r = O.dsc_estep(Y, Wc, phi, th[2:], th[1], Hp, gamma, keep_posterior=True)
        Wr, pvr, sr = O.dsc_mstep(Y, Wc, r)
        got = theta.cpu().numpy()
        eW = rel(Wd.cpu().numpy(), Wr)
        print(f"[em] it {it}: W {eW:.2e} sigma {got[1]:.6f}/{sr:.6f}", flush=True)
        assert eW < 2e-4
        np.testing.assert_allclose(got[2:], pvr, rtol=2e-5)
        assert got[1] == pytest.approx(sr, rel=2e-4)


def test_dsc_edge_cases():
    import torch
    from paper_1908_06843_amd import api
    phi, pv = (0.0, 1.0, -1.0), (0.8, 0.1, 0.1)
    gen = synth.rng(71)
    W = synth.unit_norm_gaussian_dictionary(gen, 20, 6).astype(np.float32)
    Y = gen.standard_normal((5, 20)).astype(np.float32)
    # H' = H (no selection), gamma = H', and a single point
    for Y2, Hp, gamma in ((Y, 6, 6), (Y[:1], 6, 2), (Y, 3, 0)):
        g = run_gpu(Y2, W, phi, pv, 0.9, Hp, gamma)
        r = O.dsc_estep(Y2, W, phi, pv, 0.9, Hp, gamma)
        assert_parity(g, r, "fp32", f"dsc edge ({Hp},{gamma}) N={len(Y2)}")
    # N = 0 is a no-op; bad value sets are refused before any launch
    dev = torch.device("cuda", 0)
    out = api.estep(torch.empty((0, 20), device=dev), torch.tensor(W, device=dev), sigma=1.0,
                    Hprime=3, gamma=2, model="dsc", phi=phi, pv=pv)
    assert out["sel"].shape == (0, 3)
    with pytest.raises(api.ProsperError):
        api.estep(torch.tensor(Y, device=dev), torch.tensor(W, device=dev), sigma=1.0,
                  Hprime=3, gamma=2, model="dsc", phi=(0.0, 1.0, 1.0), pv=(0.8, 0.1, 0.1))


def test_dsc_full_workload_sampled():
    """The full DSC workload (N = 100000) in the benchmark's form (BF16
    projection, statistics accumulated, walk over the whole grid-stride
    range): 256 sampled points against the oracle one by one, and the sums
    against what holds at any size (value counts add up to sum <k>, which
    lies within [0, gamma N]; B's diagonal is sum <s_h^2>)."""
    import torch
    from paper_1908_06843_amd import api
    Y, W, phi, pv, sigma = dsc_problem(WL.N, "init")
    dev = torch.device("cuda", 0)
    acc = api.new_acc("dsc", WL.D, WL.H, nvalues=len(phi))
    out = api.estep(torch.tensor(Y, device=dev), torch.tensor(W, device=dev), sigma=sigma,
                    Hprime=WL.Hprime, gamma=WL.gamma, model="dsc", precision="bf16", phi=phi,
                    pv=pv, acc=acc, factor_b=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    idx = np.sort(synth.rng(3).choice(WL.N, 256, replace=False))
    r = O.dsc_estep(Y[idx], W, phi, pv, sigma, WL.Hprime, WL.gamma)
    assert_parity(g, r, "bf16", "dsc full workload (sample)", idx=idx)
    vc = acc["vcount"].cpu().numpy()
    sc = acc["scal"].cpu().numpy()
    assert sc[4] == WL.N
    assert vc[1:].sum() == pytest.approx(sc[0], rel=1e-6)
    assert 0.0 <= sc[0] <= WL.gamma * WL.N
    B = acc["B"].cpu().numpy()
    assert np.all(np.diag(B) >= 0.0)
    assert float(np.diag(B).sum()) <= (max(abs(p) for p in phi) ** 2) * sc[0] * (1 + 1e-5)


def test_dsc_compiled_walk_hands_off_overflowing_points():
    """(H', gamma) = (8, 3) runs the compiled walk; its pivot is the best
    state with at most two actives, so points whose best state has three
    actives far above it (here: three components at phi = +-2, little
    noise) would overflow its weights and go to the table-driven kernel.
    Every point, handed off or not, matches the oracle, and so do the sums."""
    phi, pv = WL.phi, WL.pv
    N, D, H = 150, 64, 30
    gen = synth.rng(81)
    W = synth.unit_norm_gaussian_dictionary(gen, D, H)
    S = np.zeros((N, H))
    for n in range(N):
        if n % 3:   # two in three points: three strong actives
            S[n, gen.choice(H, 3, replace=False)] = gen.choice([2.0, -2.0], 3)
        else:
            S[n, gen.choice(H, 1)] = 1.0
    Y = (S @ W.T + 0.05 * gen.standard_normal((N, D))).astype(np.float32)
    W = W.astype(np.float32)
    # the oracle's log-joints show that points do cross the hand-off line:
    # best state above the best with <= 2 actives by more than 64 log2 units
    crossing = 0
    for n in range(0, N, 10):
        pt = O.dsc_estep_point(Y[n], W, phi, pv, 0.05, 8, 3)
        k = np.array([len(sl) for sl, _ in O.dsc_state_table(len(phi), 8, 3)])
        gap = (pt["lj"].max() - pt["lj"][k <= 2].max()) / np.log(2.0)
        crossing += int(gap > 64.0)
    assert crossing >= 5
    g = run_gpu(Y, W, phi, pv, 0.05, 8, 3, accumulate=True)
    r = O.dsc_estep(Y, W, phi, pv, 0.05, 8, 3)
    st = parity_stats(g, r)
    print(f"[parity] dsc hand-off: {st}", flush=True)
    assert st["sel_mismatch"] == 0 and st["s_max"] <= 1e-5
    # logL is a small difference of terms of size lam ||y||^2 (~2400 here):
    # FP32 rounding is relative to those terms, not to logL
    scale = np.maximum(np.abs(r["logL"]), (Y.astype(np.float64) ** 2).sum(1) / (2 * 0.05 ** 2))
    assert np.all(np.abs(g["logL"] - r["logL"]) <= 1e-5 * scale)
    if np.asarray(r["flagged"], dtype=bool).any():
        r = O.dsc_estep(Y, W, phi, pv, 0.05, 8, 3, sel=g["sel"])
    Bg = np.triu(g["B"]) + np.triu(g["B"], 1).T
    assert rel(g["A"], r["A"]) < 2e-5 and rel(Bg, r["B"]) < 2e-5
    assert rel(g["vcount"][1:], r["vcount"][1:]) < 1e-5
    assert g["scal"][1] == pytest.approx(r["scal"][1], rel=1e-5)
