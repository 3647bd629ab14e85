"""Pins of the oracle outputs that feed the noise update and the inference
call: the expected squared residual of the max-superposition models and the
ordering of the most probable states.

Expected residual (section "Learning Algorithm and Data Models", Eq. 2 with
Table 1's max and largest-magnitude superpositions): res_mean is
E_q ||y - f(s)||^2 under the truncated posterior, which the noise update of
MCA/MMCA divides by N D.  It is checked against explicit loops over every
state, with the posterior weights taken from scipy's Gaussian log-density
and Bernoulli log-pmf, untruncated (H' = H = gamma) and restricted to a
truncated set built here by brute force.

Most probable states (the API section's inference call: configurations
res["s"] and their probabilities res["p"]): top_index / top_q must be the
states of largest posterior probability in descending order, equal
probabilities ordered by the lower canonical table index.  Checked against a
brute-force sort of the brute-force posterior, including exact ties built
from repeated dictionary columns.
CPU only.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import bernoulli, multivariate_normal

from oracle import prosper_oracle as O


def loop_superposition(model, W, s):
    D, H = W.shape
    out = np.zeros(D)
    for d in range(D):
        terms = [s[h] * W[d, h] for h in range(H)]
        if model == "mca":
            out[d] = max(terms)
        elif model == "mmca":
            best = terms[0]
            for t in terms[1:]:
                if abs(t) > abs(best):
                    best = t
            out[d] = best
        else:
            out[d] = sum(terms)
    return out


def loop_log_joint(model, y, W, pi, sigma, s):
    D = y.shape[0]
    mu = loop_superposition(model, W, s)
    return (float(bernoulli.logpmf(s.astype(int), pi).sum())
            + float(multivariate_normal.logpdf(y, mean=mu, cov=sigma * sigma * np.eye(D))))


def loop_residual(model, y, W, s):
    mu = loop_superposition(model, W, s)
    return float(sum((y[d] - mu[d]) ** 2 for d in range(y.shape[0])))


def signed_problem(D, H, seed, neg_row=True):
    g = np.random.default_rng(seed)
    W = g.standard_normal((D, H))
    if neg_row:
        W[1, :] = -np.abs(W[1, :]) - 0.1     # a pixel whose whole row is negative
    s = (g.random(H) < 0.4).astype(float)
    y = loop_superposition("mca", W, s) + 0.5 * g.standard_normal(D)
    return y, W


@pytest.mark.parametrize("model", ["mca", "mmca"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_expected_residual_untruncated(model, seed):
    D, H, pi, sigma = 5, 4, 0.3, 0.8
    y, W = signed_problem(D, H, seed)
    states = [np.array(v, dtype=float) for v in itertools.product((0, 1), repeat=H)]
    lj = np.array([loop_log_joint(model, y, W, pi, sigma, s) for s in states])
    q = np.exp(lj - logsumexp(lj))
    ref = sum(qk * loop_residual(model, y, W, s) for qk, s in zip(q, states))
    p = O.estep_point(model, y, W, pi, sigma, H, H)
    assert p["res_mean"] == pytest.approx(ref, rel=1e-12)
    assert p["logL"] == pytest.approx(logsumexp(lj), rel=1e-12)


@pytest.mark.parametrize("model", ["mca", "mmca"])
def test_expected_residual_truncated(model):
    """Truncated set built by brute force: support inside the H' latents of
    largest singleton log-joint, at most gamma active."""
    D, H, Hp, gamma, pi, sigma = 6, 6, 4, 2, 0.25, 0.7
    for seed in range(4):
        y, W = signed_problem(D, H, 10 + seed, neg_row=False)
        if model == "mca":
            W = np.abs(W)
        single = [loop_log_joint(model, y, W, pi, sigma, np.eye(H)[h]) for h in range(H)]
        order = sorted(range(H), key=lambda h: (-single[h], h))
        keep = set(order[:Hp])
        states = [np.array(v, dtype=float) for v in itertools.product((0, 1), repeat=H)
                  if sum(v) <= gamma and all(h in keep for h in range(H) if v[h])]
        lj = np.array([loop_log_joint(model, y, W, pi, sigma, s) for s in states])
        q = np.exp(lj - logsumexp(lj))
        ref = sum(qk * loop_residual(model, y, W, s) for qk, s in zip(q, states))
        p = O.estep_point(model, y, W, pi, sigma, Hp, gamma)
        assert sorted(p["sel"].tolist()) == sorted(keep)
        assert p["res_mean"] == pytest.approx(ref, rel=1e-12)


def test_mca_all_active_state_takes_the_negative_row_max():
    """With H' = H = gamma the state with every latent active has no zero
    term in its max: a pixel whose whole row of W is negative gets a negative
    mean.  The oracle's log-joint of that state equals the loop value."""
    D, H, pi, sigma = 4, 3, 0.3, 0.6
    y, W = signed_problem(D, H, 5)
    assert (W[1] < 0).all()
    s = np.ones(H)
    mu = loop_superposition("mca", W, s)
    assert mu[1] < 0
    p = O.estep_point("mca", y, W, pi, sigma, H, H)
    tab = O.state_table("mca", H, H)
    k_all = [i for i, (slots, _) in enumerate(tab) if len(slots) == H][0]
    assert p["lj"][k_all] == pytest.approx(loop_log_joint("mca", y, W, pi, sigma, s), rel=1e-12)


def brute_top(q, topk):
    """Descending probability, equal probabilities by lower table index."""
    idx = sorted(range(len(q)), key=lambda i: (-q[i], i))[:topk]
    return np.array(idx), q[idx]


@pytest.mark.parametrize("model", ["bsc", "tsc", "mca"])
def test_top_states_brute_force_sort(model):
    g = np.random.default_rng(3)
    D, H, Hp, gamma, pi, sigma = 5, 5, 5, 3, 0.3, 0.9
    W = g.standard_normal((D, H))
    if model == "mca":
        W = np.abs(W)
    tab = O.state_table(model, Hp, gamma)
    for n in range(4):
        y = g.standard_normal(D) * 1.5
        p = O.estep_point(model, y, W, pi, sigma, Hp, gamma, topk=6)
        # brute force posterior over the same table (all latents selected)
        lj = []
        for slots, vals in tab:
            s = np.zeros(H)
            for j, v in zip(slots, vals):
                s[p["sel"][j]] = v
            if model == "tsc":
                prior = sum(np.log(pi / 2) if s[h] != 0 else np.log1p(-pi) for h in range(H))
                mu = loop_superposition("bsc", W, s)
                lj.append(prior + float(multivariate_normal.logpdf(
                    y, mean=mu, cov=sigma * sigma * np.eye(D))))
            else:
                lj.append(loop_log_joint(model, y, W, pi, sigma, s))
        lj = np.array(lj)
        q = np.exp(lj - logsumexp(lj))
        bi, bq = brute_top(q, 6)
        assert np.array_equal(p["top_index"], bi)
        np.testing.assert_allclose(p["top_q"], bq, rtol=1e-10)
        assert np.all(np.diff(p["top_q"]) <= 0)


def test_top_states_exact_tie_goes_to_lower_table_index():
    """Two identical dictionary columns make the states {0} and {1} (and any
    pair of states that swap them) exactly equally probable; the lower table
    index must come first."""
    g = np.random.default_rng(8)
    D, H, pi, sigma = 4, 3, 0.3, 0.8
    W = g.standard_normal((D, H))
    W[:, 1] = W[:, 0]
    y = W[:, 0] + 0.05 * g.standard_normal(D)
    p = O.estep_point("bsc", y, W, pi, sigma, H, H, topk=8)
    tab = O.state_table("bsc", H, H)
    q = p["q"]
    i0 = tab.index(((0,), (1,)))
    i1 = tab.index(((1,), (1,)))
    assert q[i0] == q[i1]                     # an exact tie in FP64
    order = list(p["top_index"])
    assert order.index(i0) < order.index(i1)
    bi, _ = brute_top(q, 8)
    assert np.array_equal(p["top_index"], bi)


def test_forced_candidate_set_is_the_restricted_posterior():
    """estep_point(sel=...) gives the exact posterior renormalised on the
    states supported inside the given set (brute force over all states)."""
    g = np.random.default_rng(21)
    D, H, Hp, gamma, pi, sigma = 5, 6, 3, 2, 0.3, 0.9
    W = g.standard_normal((D, H))
    y = g.standard_normal(D)
    forced = [4, 0, 2]
    states = [np.array(v, dtype=float) for v in itertools.product((0, 1), repeat=H)
              if sum(v) <= gamma and all(h in forced for h in range(H) if v[h])]
    lj = np.array([loop_log_joint("bsc", y, W, pi, sigma, s) for s in states])
    q = np.exp(lj - logsumexp(lj))
    mean = q @ np.array(states)
    p = O.estep_point("bsc", y, W, pi, sigma, Hp, gamma, sel=forced)
    assert p["sel"].tolist() == [0, 2, 4]
    assert p["logL"] == pytest.approx(logsumexp(lj), rel=1e-12)
    np.testing.assert_allclose(p["s_mean"], mean[[0, 2, 4]], rtol=1e-10, atol=1e-14)
    with pytest.raises(ValueError):
        O.estep_point("bsc", y, W, pi, sigma, Hp, gamma, sel=[1, 1, 2])


# ---------------------------------------------------------------- annealing
def tempered_params(model, pi, sigma, beta):
    """p(y, s)^beta is, up to a constant, the joint of the same model with the
    prior probabilities raised to beta and renormalised and the noise
    variance divided by beta."""
    if model == "tsc":
        a, z = (pi / 2) ** beta, (1 - pi) ** beta
        return 2 * a / (2 * a + z), sigma / np.sqrt(beta)
    a, z = pi ** beta, (1 - pi) ** beta
    return a / (a + z), sigma / np.sqrt(beta)


@pytest.mark.parametrize("model", ["bsc", "tsc", "mca", "mmca"])
@pytest.mark.parametrize("beta", [0.5, 0.2])
def test_tempered_posterior_is_the_posterior_of_a_rescaled_model(model, beta):
    g = np.random.default_rng(41)
    D, H, Hp, gamma = 6, 7, 5, 3
    W = g.standard_normal((D, H))
    if model == "mca":
        W = np.abs(W)
    pi, sigma = 0.2, 0.8
    pt, st = tempered_params(model, pi, sigma, beta)
    for n in range(3):
        y = g.standard_normal(D) * 1.3
        a = O.estep_point(model, y, W, pi, sigma, Hp, gamma, beta=beta,
                          sel=O.estep_point(model, y, W, pi, sigma, Hp, gamma)["sel"])
        b = O.estep_point(model, y, W, pt, st, Hp, gamma, sel=a["sel"])
        np.testing.assert_allclose(a["q"], b["q"], rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(a["s_mean"], b["s_mean"], rtol=1e-10, atol=1e-15)
        # logL stays the untempered one
        c = O.estep_point(model, y, W, pi, sigma, Hp, gamma, sel=a["sel"])
        assert a["logL"] == pytest.approx(c["logL"], rel=1e-14)


def test_tempered_posterior_brute_force_and_the_flat_limit():
    g = np.random.default_rng(43)
    D, H, pi, sigma, beta = 5, 4, 0.3, 0.7, 0.35
    W = g.standard_normal((D, H))
    y = g.standard_normal(D)
    states = [np.array(v, dtype=float) for v in itertools.product((0, 1), repeat=H)]
    lj = np.array([loop_log_joint("bsc", y, W, pi, sigma, s) for s in states])
    q = np.exp(beta * lj - logsumexp(beta * lj))
    p = O.estep_point("bsc", y, W, pi, sigma, H, H, beta=beta)
    np.testing.assert_allclose(p["s_mean"], q @ np.array(states), rtol=1e-10)
    # beta -> 0: uniform over K, so <s_j> = #{states with slot j} / |K|
    Hp, gamma = 6, 3
    W = g.standard_normal((8, 9))
    y = g.standard_normal(8)
    p = O.estep_point("bsc", y, W, pi, sigma, Hp, gamma, beta=1e-12)
    K = sum(math.comb(Hp, k) for k in range(gamma + 1))
    per = sum(math.comb(Hp - 1, k - 1) for k in range(1, gamma + 1))
    np.testing.assert_allclose(p["s_mean"], per / K, rtol=1e-9)
