"""Pins of the FP64 oracle's DSC functions (discrete latents with a
categorical prior, linear superposition, Gaussian noise; Table 1) against
things other than themselves: brute force over all V^H states with scipy's
multivariate normal, the special cases that are BSC (V = 2) and TSC (V = 3,
values 0, 1, -1, equal probabilities of the two signs), the closed count of
the truncated state set, the closed-form posterior at H = 1, the stationarity
of the M-step's objective, and the EM monotonicity theorem.  CPU only."""
import itertools
import math

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import multivariate_normal

from oracle import prosper_oracle as O
import synth


def dsc_problem(D, H, phi, pv, sigma, N, seed):
    g = synth.rng(seed)
    W = g.standard_normal((D, H))
    C = g.choice(len(phi), size=(N, H), p=pv)
    Y = np.asarray(phi)[C] @ W.T + sigma * g.standard_normal((N, D))
    return Y, W


def brute(y, W, phi, pv, sigma):
    """Every one of the V^H states, joint by scipy: log p(y), posterior
    mean of s and of s s^T, expected number of latents at each value."""
    D, H = W.shape
    lj, S, C = [], [], []
    for codes in itertools.product(range(len(phi)), repeat=H):
        s = np.array([phi[c] for c in codes])
        lj.append(sum(math.log(pv[c]) for c in codes)
                  + multivariate_normal.logpdf(y, mean=W @ s, cov=sigma * sigma * np.eye(D)))
        S.append(s)
        C.append(codes)
    lj = np.array(lj)
    q = np.exp(lj - logsumexp(lj))
    S, C = np.array(S), np.array(C)
    vm = np.array([q @ (C == v).sum(axis=1) for v in range(len(phi))])
    return logsumexp(lj), q @ S, (S * q[:, None]).T @ S, vm


PHI4 = (0.0, 1.0, -0.5, 2.0)
PV4 = (0.55, 0.2, 0.15, 0.1)


def test_state_count_closed_form():
    for V in (2, 3, 4, 5):
        for Hp in (1, 4, 7):
            for gamma in range(0, Hp + 1):
                tab = O.dsc_state_table(V, Hp, gamma)
                want = sum(math.comb(Hp, k) * (V - 1) ** k for k in range(gamma + 1))
                assert len(tab) == want == O.dsc_state_count(V, Hp, gamma)
                # every state once, codes in 1..V-1, support of size <= gamma
                keys = {(sl, cd) for sl, cd in tab}
                assert len(keys) == len(tab)
                assert all(len(sl) == len(cd) <= gamma and all(1 <= c < V for c in cd)
                           for sl, cd in tab)
            # untruncated: all V^H' states
            assert len(O.dsc_state_table(V, Hp, Hp)) == V ** Hp


def test_untruncated_matches_brute_force():
    """H' = gamma = H: the truncated posterior is the exact posterior."""
    D, H = 5, 4
    Y, W = dsc_problem(D, H, PHI4, PV4, 0.6, 3, seed=21)
    for y in Y:
        p = O.dsc_estep_point(y, W, PHI4, PV4, 0.6, H, H)
        logL, m, mm, vm = brute(y, W, PHI4, PV4, 0.6)
        assert p["logL"] == pytest.approx(logL, rel=1e-12, abs=1e-10)
        sel = p["sel"]
        np.testing.assert_allclose(p["s_mean"], m[sel], rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(p["ss_mean"], mm[np.ix_(sel, sel)], rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(p["v_mean"][1:], vm[1:], rtol=1e-10, atol=1e-12)


def test_truncated_is_brute_force_restricted():
    """H' < H: logL is the log-sum over exactly the states with support in
    the preselected set and at most gamma actives, all values allowed."""
    D, H, Hp, gamma = 4, 5, 3, 2
    Y, W = dsc_problem(D, H, PHI4, PV4, 0.5, 2, seed=4)
    for y in Y:
        p = O.dsc_estep_point(y, W, PHI4, PV4, 0.5, Hp, gamma)
        sel = set(p["sel"].tolist())
        lj = []
        for codes in itertools.product(range(4), repeat=H):
            act = {h for h in range(H) if codes[h]}
            if act <= sel and len(act) <= gamma:
                s = np.array([PHI4[c] for c in codes])
                lj.append(sum(math.log(PV4[c]) for c in codes)
                          + multivariate_normal.logpdf(y, mean=W @ s, cov=0.25 * np.eye(D)))
        assert len(lj) == O.dsc_state_count(4, Hp, gamma)
        assert p["logL"] == pytest.approx(logsumexp(lj), rel=1e-12)


def test_selection_is_best_singleton():
    """The selection score ranks latents by their best singleton
    log-joint: brute force over (h, v) with every other latent at phi_0."""
    D, H = 6, 9
    Y, W = dsc_problem(D, H, PHI4, PV4, 0.8, 3, seed=8)
    for y in Y:
        r = O.dsc_selection_scores(y, W, np.array(PHI4), np.array(PV4), 0.8)
        best = []
        for h in range(H):
            vals = []
            for v in range(1, 4):
                s = np.zeros(H)
                s[h] = PHI4[v]
                vals.append(math.log(PV4[v]) + (H - 1) * math.log(PV4[0])
                            + multivariate_normal.logpdf(y, mean=W @ s, cov=0.64 * np.eye(D)))
            best.append(max(vals))
        best = np.array(best)
        # same order and, after the factor sigma^2 and an h-independent
        # shift, the same values
        assert list(np.argsort(-r, kind="stable")) == list(np.argsort(-best, kind="stable"))
        np.testing.assert_allclose(r - r.max(), 0.64 * (best - best.max()), atol=1e-10)


def test_v2_is_bsc():
    D, H, Hp, gamma, pi, sigma = 7, 12, 5, 3, 0.2, 0.5
    g = synth.rng(3)
    W = g.standard_normal((D, H))
    Y = synth.sample_binary(g, 10, H, pi) @ W.T + sigma * g.standard_normal((10, D))
    d = O.dsc_estep(Y, W, (0.0, 1.0), (1 - pi, pi), sigma, Hp, gamma, topk=4)
    b = O.estep(O.BSC, Y, W, pi, sigma, Hp, gamma, topk=4)
    np.testing.assert_array_equal(d["sel"], b["sel"])
    np.testing.assert_allclose(d["logL"], b["logL"], rtol=1e-13)
    np.testing.assert_allclose(d["s_mean"], b["s_mean"], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(d["A"], b["A"], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(d["B"], b["B"], rtol=1e-11, atol=1e-12)
    np.testing.assert_array_equal(d["top_index"], b["top_index"])
    assert d["vcount"][1] == pytest.approx(b["scal"][0], rel=1e-12)


def test_v3_sign_pair_is_tsc():
    """phi = (0, 1, -1) and pv = (1 - pi, pi/2, pi/2) is TSC, state for state
    (the code order puts -1 after +1 at each digit, as TSC's sign order)."""
    D, H, Hp, gamma, pi, sigma = 6, 10, 5, 3, 0.25, 0.6
    g = synth.rng(9)
    W = g.standard_normal((D, H))
    S = synth.sample_binary(g, 8, H, pi) * (1 - 2 * synth.sample_binary(g, 8, H, 0.5))
    Y = S @ W.T + sigma * g.standard_normal((8, D))
    d = O.dsc_estep(Y, W, (0.0, 1.0, -1.0), (1 - pi, pi / 2, pi / 2), sigma, Hp, gamma, topk=6)
    t = O.estep(O.TSC, Y, W, pi, sigma, Hp, gamma, topk=6)
    np.testing.assert_array_equal(d["sel"], t["sel"])
    np.testing.assert_allclose(d["logL"], t["logL"], rtol=1e-13)
    np.testing.assert_allclose(d["s_mean"], t["s_mean"], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(d["B"], t["B"], rtol=1e-11, atol=1e-12)
    np.testing.assert_array_equal(d["top_index"], t["top_index"])
    np.testing.assert_allclose(d["top_q"], t["top_q"], rtol=1e-12)
    assert d["vcount"][1] + d["vcount"][2] == pytest.approx(t["scal"][0], rel=1e-12)


def test_h1_closed_form():
    """H = 1: p(s = phi_v | y) is proportional to pv_v N(y; phi_v w, sigma^2 I)."""
    phi, pv, sigma = np.array(PHI4), np.array(PV4), 0.7
    w = np.array([0.3, -1.2, 0.8])
    y = np.array([0.5, -2.0, 1.1])
    logits = np.log(pv) - ((y[None, :] - phi[:, None] * w[None, :]) ** 2).sum(1) / (2 * sigma ** 2)
    post = np.exp(logits - logits.max())
    post /= post.sum()
    p = O.dsc_estep_point(y, w[:, None], phi, pv, sigma, 1, 1)
    np.testing.assert_allclose(p["v_mean"], post, rtol=1e-12)
    assert p["s_mean"][0] == pytest.approx(float(post @ phi), rel=1e-12)
    assert p["ss_mean"][0, 0] == pytest.approx(float(post @ phi ** 2), rel=1e-12)
    const = -1.5 * math.log(2 * math.pi * sigma ** 2)
    assert p["logL"] == pytest.approx(const + logsumexp(logits), rel=1e-12)


def test_value_counts_are_a_distribution():
    D, H, Hp, gamma = 5, 8, 4, 2
    Y, W = dsc_problem(D, H, PHI4, PV4, 0.5, 6, seed=12)
    est = O.dsc_estep(Y, W, PHI4, PV4, 0.5, Hp, gamma)
    assert est["vcount"].sum() == pytest.approx(6 * H, rel=1e-13)
    assert np.all(est["vcount"] >= 0)
    assert est["vcount"][1:].sum() == pytest.approx(est["scal"][0], rel=1e-12)


def test_mstep_is_stationary():
    """The new parameters maximise the expected complete-data log-likelihood
    under the truncated posteriors: its gradient in W vanishes, pv is the
    maximiser on the simplex (no feasible direction raises it), and sigma
    maximises it for W_new."""
    D, H, Hp, gamma = 5, 6, 4, 2
    Y, W = dsc_problem(D, H, PHI4, PV4, 0.6, 20, seed=5)
    est = O.dsc_estep(Y, W, PHI4, PV4, 0.6, Hp, gamma, keep_posterior=True)
    W1, pv1, s1 = O.dsc_mstep(Y, W, est)
    phi = np.array(PHI4)

    def Q(Wq, pvq, sq):
        tot = 0.0
        for n, (c, q) in enumerate(est["posterior"]):
            S = np.zeros((len(est["table"]), H))
            Cd = np.zeros((len(est["table"]), H), dtype=int)
            for i, (slots, codes) in enumerate(est["table"]):
                for j, cc in zip(slots, codes):
                    S[i, c[j]] = phi[cc]
                    Cd[i, c[j]] = cc
            lp = np.log(pvq)[Cd].sum(1)
            R = Y[n][None, :] - S @ Wq.T
            ll = -0.5 * D * math.log(2 * math.pi * sq * sq) - (R * R).sum(1) / (2 * sq * sq)
            tot += float(q @ (lp + ll))
        return tot

    q0 = Q(W1, pv1, s1)
    g = synth.rng(0)
    for _ in range(4):
        dW = g.standard_normal(W1.shape) * 1e-4
        assert Q(W1 + dW, pv1, s1) <= q0 + 1e-12
        dv = g.standard_normal(4) * 1e-4
        dv -= dv.mean()
        assert Q(W1, pv1 + dv, s1) <= q0 + 1e-12
    for f in (0.999, 1.001):
        assert Q(W1, pv1, s1 * f) <= q0 + 1e-12


def test_em_is_monotone_untruncated():
    """With H' = gamma = H the truncated posterior is exact and EM cannot
    lower the log-likelihood."""
    D, H = 4, 3
    Y, W = dsc_problem(D, H, PHI4, PV4, 0.5, 15, seed=30)
    g = synth.rng(31)
    W = g.standard_normal((D, H))
    pv, sigma = np.array([0.4, 0.2, 0.2, 0.2]), 1.0
    prev = -np.inf
    for _ in range(6):
        est = O.dsc_estep(Y, W, PHI4, pv, sigma, H, H, keep_posterior=True)
        L = float(est["scal"][1])
        assert L >= prev - 1e-9
        prev = L
        W, pv, sigma = O.dsc_mstep(Y, W, est)


def test_rejects_bad_value_sets():
    W = np.eye(3)
    y = np.ones(3)
    with pytest.raises(ValueError):
        O.dsc_estep_point(y, W, (1.0, 2.0), (0.5, 0.5), 1.0, 2, 1)      # phi_0 != 0
    with pytest.raises(ValueError):
        O.dsc_estep_point(y, W, (0.0, 1.0, 1.0), (0.5, 0.25, 0.25), 1.0, 2, 1)
    with pytest.raises(ValueError):
        O.dsc_estep_point(y, W, (0.0, 1.0), (0.6, 0.6), 1.0, 2, 1)
