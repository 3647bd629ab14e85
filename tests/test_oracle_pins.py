"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against the mathematics the paper fixes (Eq. 1-2,
Table 1, truncated posteriors, EM) through an independent route: brute force
over all states with scipy's multivariate normal, closed forms at H = 1,
special cases where max superposition reduces to linear, posterior
invariants, textbook least squares, the EM monotonicity theorem.
CPU only.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import bernoulli, multivariate_normal

from oracle import prosper_oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers
def brute_states(model, H):
    vals = (-1, 0, 1) if model == O.TSC else (0, 1)
    return [np.array(v, dtype=float) for v in itertools.product(vals, repeat=H)]


def brute_mean(model, W, s):
    """f(Theta, s) with explicit loops (Table 1 superposition)."""
    D, H = W.shape
    if model == O.MCA:
        return np.array([max(s[h] * W[d, h] for h in range(H)) for d in range(D)])
    return np.array([sum(W[d, h] * s[h] for h in range(H)) for d in range(D)])


def brute_logprior(model, s, pi):
    if model == O.TSC:
        # categorical over {-1, 0, +1} with probabilities (pi/2, 1-pi, pi/2)
        p = {-1.0: pi / 2, 0.0: 1 - pi, 1.0: pi / 2}
        return sum(math.log(p[float(v)]) for v in s)
    return float(bernoulli.logpmf(s.astype(int), pi).sum())


def brute_posterior(model, y, W, pi, sigma):
    D, H = W.shape
    S = brute_states(model, H)
    lj = np.array([brute_logprior(model, s, pi)
                   + multivariate_normal.logpdf(y, mean=brute_mean(model, W, s),
                                                cov=sigma * sigma * np.eye(D))
                   for s in S])
    logL = logsumexp(lj)
    q = np.exp(lj - logL)
    Sm = np.array(S)
    return logL, q @ Sm, (Sm * q[:, None]).T @ Sm, S, q


def rand_problem(model, D, H, seed, sigma=0.7, pi=0.3, scale=1.0):
    g = np.random.default_rng(seed)
    W = g.standard_normal((D, H)) * scale
    if model == O.MCA:
        W = np.abs(W)
    s = (g.random(H) < pi).astype(float)
    if model == O.TSC:
        s *= np.where(g.random(H) < 0.5, -1.0, 1.0)
    y = brute_mean(model, W, s) + sigma * g.standard_normal(D)
    return y, W, pi, sigma


# ---------------------------------------------------------------- state set
def closed_form_count(model, Hp, gamma):
    V = 3 if model == O.TSC else 2
    return sum(math.comb(Hp, k) * (V - 1) ** k for k in range(gamma + 1))


def test_golden_state_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "state_counts.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for model, hp, g, cnt in rows:
        hp, g, cnt = int(hp), int(g), int(cnt)
        assert closed_form_count(model, hp, g) == cnt
        assert len(O.state_table(model, hp, g)) == cnt


@pytest.mark.parametrize("model,Hp,gamma", [("bsc", 6, 3), ("bsc", 5, 5), ("bsc", 7, 0),
                                            ("tsc", 5, 2), ("tsc", 4, 4), ("mca", 6, 2)])
def test_state_table_brute_force(model, Hp, gamma):
    tab = O.state_table(model, Hp, gamma)
    vals = (-1, 0, 1) if model == "tsc" else (0, 1)
    brute = {v for v in itertools.product(vals, repeat=Hp) if sum(x != 0 for x in v) <= gamma}
    mine = []
    for slots, sv in tab:
        v = [0] * Hp
        for j, x in zip(slots, sv):
            v[j] = x
        mine.append(tuple(v))
    assert len(mine) == len(set(mine)) == len(brute) == closed_form_count(model, Hp, gamma)
    assert set(mine) == brute
    # canonical order: (k, slot tuple) non-decreasing, sign codes counting up
    keys = [(len(sl), sl) for sl, _ in tab]
    assert keys == sorted(keys)
    act, sgn = O.state_masks(model, Hp, gamma)
    for (slots, sv), a, s in zip(tab, act, sgn):
        assert bin(int(a)).count("1") == len(slots) <= gamma
        assert int(a) == sum(1 << j for j in slots)
        assert int(s) == sum(1 << j for j, x in zip(slots, sv) if x < 0)
    if model == "tsc":
        i = 0
        while i < len(tab):
            sl = tab[i][0]
            for code in range(1 << len(sl)):
                assert tab[i + code][0] == sl
                assert tab[i + code][1] == tuple(-1 if (code >> b) & 1 else 1 for b in range(len(sl)))
            i += 1 << len(sl)


# ---------------------------------------------------------------- exact posterior
@pytest.mark.parametrize("model,D,H,seed", [("bsc", 6, 4, 0), ("bsc", 9, 5, 1), ("tsc", 5, 3, 2),
                                            ("tsc", 7, 4, 3), ("mca", 6, 4, 4), ("mca", 8, 5, 5)])
def test_truncated_equals_brute_force_when_untruncated(model, D, H, seed):
    y, W, pi, sigma = rand_problem(model, D, H, seed)
    logL, sm, ssm, _, _ = brute_posterior(model, y, W, pi, sigma)
    p = O.estep_point(model, y, W, pi, sigma, Hp=H, gamma=H)
    assert np.array_equal(p["sel"], np.arange(H))
    assert p["logL"] == pytest.approx(logL, rel=1e-12, abs=1e-10)
    np.testing.assert_allclose(p["s_mean"], sm, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(p["ss_mean"], ssm, rtol=1e-10, atol=1e-12)


def test_truncated_equals_brute_force_restricted():
    """Truncation (H' < H, gamma < H') equals brute force restricted to K_n."""
    model, D, H, Hp, gamma = "bsc", 8, 6, 4, 2
    y, W, pi, sigma = rand_problem(model, D, H, 11)
    p = O.estep_point(model, y, W, pi, sigma, Hp, gamma)
    sel = set(p["sel"].tolist())
    _, _, _, S, _ = brute_posterior(model, y, W, pi, sigma)
    keep = [s for s in S if set(np.nonzero(s)[0]) <= sel and np.count_nonzero(s) <= gamma]
    lj = np.array([brute_logprior(model, s, pi) + multivariate_normal.logpdf(
        y, mean=brute_mean(model, W, s), cov=sigma ** 2 * np.eye(D)) for s in keep])
    assert len(keep) == closed_form_count(model, Hp, gamma)
    assert p["logL"] == pytest.approx(logsumexp(lj), rel=1e-12)
    q = np.exp(lj - logsumexp(lj))
    sm = q @ np.array(keep)
    np.testing.assert_allclose(p["s_mean"], sm[p["sel"]], rtol=1e-10, atol=1e-13)


# ---------------------------------------------------------------- closed forms at H = 1
def _gauss_logpdf(y, mu, sigma):
    return multivariate_normal.logpdf(y, mean=mu, cov=sigma ** 2 * np.eye(len(y)))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bsc_single_latent_closed_form(seed):
    g = np.random.default_rng(seed)
    D = 7
    W = g.standard_normal((D, 1))
    y = g.standard_normal(D) + W[:, 0] * (seed % 2)
    pi, sigma = 0.15 + 0.2 * seed, 0.5 + 0.3 * seed
    p = O.estep_point("bsc", y, W, pi, sigma, 1, 1)
    w = W[:, 0]
    q1 = 1 / (1 + np.exp(-(np.log(pi / (1 - pi)) + (w @ y - 0.5 * w @ w) / sigma ** 2)))
    logL = np.logaddexp(np.log(1 - pi) + _gauss_logpdf(y, 0 * w, sigma),
                        np.log(pi) + _gauss_logpdf(y, w, sigma))
    assert p["s_mean"][0] == pytest.approx(q1, rel=1e-12)
    assert p["logL"] == pytest.approx(logL, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_tsc_single_latent_closed_form(seed):
    g = np.random.default_rng(10 + seed)
    D = 5
    W = g.standard_normal((D, 1))
    y = g.standard_normal(D) - W[:, 0]
    pi, sigma = 0.3, 0.9
    w = W[:, 0]
    comps = np.array([np.log(pi / 2) + _gauss_logpdf(y, -w, sigma),
                      np.log(1 - pi) + _gauss_logpdf(y, 0 * w, sigma),
                      np.log(pi / 2) + _gauss_logpdf(y, w, sigma)])
    logL = logsumexp(comps)
    r = np.exp(comps - logL)
    p = O.estep_point("tsc", y, W, pi, sigma, 1, 1)
    assert p["logL"] == pytest.approx(logL, rel=1e-12)
    assert p["s_mean"][0] == pytest.approx(r[2] - r[0], rel=1e-10, abs=1e-14)
    assert p["ss_mean"][0, 0] == pytest.approx(r[2] + r[0], rel=1e-10)


def test_mca_single_latent_closed_form():
    """With one latent the max superposition of s=1 is W itself (even where
    W < 0): a two-component mixture with means 0 and W."""
    g = np.random.default_rng(3)
    W = g.standard_normal((6, 1))
    y = W[:, 0] + 0.4 * g.standard_normal(6)
    pi, sigma = 0.25, 0.6
    logL = np.logaddexp(np.log(1 - pi) + _gauss_logpdf(y, 0 * y, sigma),
                        np.log(pi) + _gauss_logpdf(y, W[:, 0], sigma))
    p = O.estep_point("mca", y, W, pi, sigma, 1, 1)
    assert p["logL"] == pytest.approx(logL, rel=1e-12)


# ---------------------------------------------------------------- MCA special cases
def test_mca_equals_bsc_for_disjoint_nonnegative_components():
    g = np.random.default_rng(7)
    D, H = 12, 4
    W = np.zeros((D, H))
    for h in range(H):   # disjoint supports: max == sum
        W[3 * h:3 * h + 3, h] = np.abs(g.standard_normal(3)) + 0.1
    for n in range(4):
        y = W @ (g.random(H) < 0.5) + 0.3 * g.standard_normal(D)
        for Hp, gamma in [(4, 4), (3, 2), (2, 1)]:
            a = O.estep_point("mca", y, W, 0.3, 0.5, Hp, gamma)
            b = O.estep_point("bsc", y, W, 0.3, 0.5, Hp, gamma)
            assert np.array_equal(a["sel"], b["sel"])
            assert a["logL"] == pytest.approx(b["logL"], rel=1e-12)
            np.testing.assert_allclose(a["s_mean"], b["s_mean"], rtol=1e-10, atol=1e-14)


def test_mca_equals_bsc_when_one_cause():
    g = np.random.default_rng(8)
    D, H = 9, 6
    W = np.abs(g.standard_normal((D, H)))
    y = W[:, 2] + 0.2 * g.standard_normal(D)
    a = O.estep_point("mca", y, W, 0.2, 0.4, 4, 1)
    b = O.estep_point("bsc", y, W, 0.2, 0.4, 4, 1)
    assert np.array_equal(a["sel"], b["sel"])
    assert a["logL"] == pytest.approx(b["logL"], rel=1e-12)


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("model", ["bsc", "tsc", "mca"])
def test_posterior_invariants(model):
    y, W, pi, sigma = rand_problem(model, 10, 8, 21, sigma=1.0, pi=0.25)
    p = O.estep_point(model, y, W, pi, sigma, 6, 3)
    assert p["q"].sum() == pytest.approx(1.0, abs=1e-13)
    lo = -1 if model == "tsc" else 0
    assert np.all(p["s_mean"] >= lo - 1e-15) and np.all(p["s_mean"] <= 1 + 1e-15)
    d = np.diag(p["ss_mean"])
    if model != "tsc":
        np.testing.assert_allclose(d, p["s_mean"], rtol=1e-12)
    assert d.sum() == pytest.approx(p["k_mean"], rel=1e-12)
    assert np.linalg.eigvalsh(p["ss_mean"]).min() > -1e-12


def test_tsc_sign_symmetry():
    y, W, pi, sigma = rand_problem("tsc", 9, 7, 31)
    a = O.estep_point("tsc", y, W, pi, sigma, 5, 3)
    b = O.estep_point("tsc", -y, W, pi, sigma, 5, 3)
    assert np.array_equal(a["sel"], b["sel"])
    assert a["logL"] == pytest.approx(b["logL"], rel=1e-12)
    np.testing.assert_allclose(a["s_mean"], -b["s_mean"], atol=1e-12)


@pytest.mark.parametrize("model", ["bsc", "tsc", "mca"])
def test_column_permutation_equivariance(model):
    y, W, pi, sigma = rand_problem(model, 10, 7, 41)
    perm = np.random.default_rng(5).permutation(7)
    a = O.estep_point(model, y, W, pi, sigma, 5, 3)
    b = O.estep_point(model, y, W[:, perm], pi, sigma, 5, 3)
    full_a = np.zeros(7)
    full_a[a["sel"]] = a["s_mean"]
    full_b = np.zeros(7)
    full_b[b["sel"]] = b["s_mean"]
    np.testing.assert_allclose(full_b, full_a[perm], rtol=1e-10, atol=1e-14)
    assert a["logL"] == pytest.approx(b["logL"], rel=1e-12)


# ---------------------------------------------------------------- selection
@pytest.mark.parametrize("model", ["bsc", "tsc", "mca"])
def test_selection_ranks_by_singleton_log_joint(model):
    """The score orders latents like log p(y, e_h) (scipy logpdf), TSC taking
    the better sign."""
    y, W, pi, sigma = rand_problem(model, 8, 9, 51)
    H = W.shape[1]
    lj = []
    for h in range(H):
        cands = [1.0, -1.0] if model == "tsc" else [1.0]
        best = -np.inf
        for v in cands:
            s = np.zeros(H)
            s[h] = v
            best = max(best, _gauss_logpdf(y, brute_mean(model, W, s), sigma))
        lj.append(best)
    r = O.selection_scores(model, y, W)
    assert list(np.argsort(-np.array(lj), kind="stable")) == list(np.argsort(-r, kind="stable"))
    np.testing.assert_allclose(np.array(lj) - np.array(lj)[0], (r - r[0]) / sigma ** 2, atol=1e-9)


def test_selection_ties_go_to_lower_index_and_flag():
    g = np.random.default_rng(6)
    D, H = 6, 5
    W = g.standard_normal((D, H))
    W[:, 3] = W[:, 1]                 # exact duplicate columns: tied scores
    y = W[:, 1] * 2 + 0.01 * g.standard_normal(D)
    r = O.selection_scores("bsc", y, W)
    assert r[1] == r[3]
    order = sorted(range(H), key=lambda h: (-r[h], h))
    k = order.index(1)
    sel, flagged = O.preselect(r, k + 1)
    assert 1 in sel and 3 not in sel and flagged
    sel2, flagged2 = O.preselect(r, k + 2)
    assert 1 in sel2 and 3 in sel2
    sel3, f3 = O.preselect(r, H)
    assert list(sel3) == list(range(H)) and not f3


# ---------------------------------------------------------------- M-step
@pytest.mark.parametrize("model", ["bsc", "tsc"])
def test_mstep_point_mass_is_least_squares(model):
    """With posteriors concentrated on one state per point, W = A B^-1 is the
    ordinary least-squares fit of Y on S."""
    g = np.random.default_rng(61)
    N, D, H = 40, 6, 4
    S = (g.random((N, H)) < 0.5).astype(float)
    if model == "tsc":
        S *= np.where(g.random((N, H)) < 0.5, -1, 1)
    Y = g.standard_normal((N, D))
    est = dict(A=Y.T @ S, B=S.T @ S, scal=np.array([np.count_nonzero(S), 0, 0, 0, N]),
               table=O.state_table(model, H, H),
               posterior=[])
    # point masses: q = 1 on the state equal to S[n]
    tab = est["table"]
    for n in range(N):
        q = np.zeros(len(tab))
        for i, (slots, vals) in enumerate(tab):
            v = np.zeros(H)
            v[list(slots)] = vals
            if np.array_equal(v, S[n]):
                q[i] = 1.0
        assert q.sum() == 1.0
        est["posterior"].append((np.arange(H), q))
    Wn, pin, sgn = O.mstep(model, Y, np.zeros((D, H)), est)
    Wls = np.linalg.lstsq(S, Y, rcond=None)[0].T
    np.testing.assert_allclose(Wn, Wls, rtol=1e-10, atol=1e-12)
    assert pin == pytest.approx(np.count_nonzero(S) / (N * H))
    resid = Y - S @ Wls.T
    assert sgn == pytest.approx(np.sqrt((resid ** 2).sum() / (N * D)), rel=1e-12)


def test_mstep_sigma_sweep_equals_closed_form():
    wl = synth.WORKLOADS["bsc256"]
    Y, Wgt, _, _ = synth.make_workload("bars", N=60)
    W0, pi0, s0 = synth.initial_params(synth.WORKLOADS["bars"], Y)
    est = O.estep("bsc", Y, W0, pi0, s0, 6, 3, keep_posterior=True)
    Wn, _, sig = O.mstep("bsc", Y, W0, est)
    A, B, scal = est["A"], est["B"], est["scal"]
    N, D = Y.shape
    closed = (scal[2] - 2 * np.trace(Wn.T @ A) + np.trace(Wn.T @ Wn @ B)) / (N * D)
    assert sig ** 2 == pytest.approx(closed, rel=1e-10)
    assert wl.D == 256


def test_mstep_inactive_latent_keeps_column():
    g = np.random.default_rng(3)
    Y = g.standard_normal((30, 5)).astype(np.float32)
    W = g.standard_normal((5, 6))
    W[:, 4] = 50.0   # far from every point: never preselected at H'=2
    est = O.estep("bsc", Y, W, 0.2, 1.0, 2, 2, keep_posterior=True)
    assert np.all(est["sel"] != 4)
    Wn, _, _ = O.mstep("bsc", Y, W, est)
    np.testing.assert_array_equal(Wn[:, 4], W[:, 4])


def test_mca_mstep_responsibilities_sum():
    """Responsibilities of a pixel sum to the posterior mass of states whose
    max over active components is positive (here: every non-zero state)."""
    g = np.random.default_rng(9)
    D, H = 7, 5
    W = np.abs(g.standard_normal((D, H))) + 0.05
    y = W[:, 0] + 0.3 * g.standard_normal(D)
    p = O.estep_point("mca", y, W, 0.2, 0.5, 4, 2)
    q0 = p["q"][0]   # zero state comes first in the table
    np.testing.assert_allclose(p["R"].sum(axis=1), 1 - q0, rtol=1e-12)


def test_mca_mstep_single_cause_is_cluster_mean():
    """With one cause per point (gamma = 1) and posteriors concentrated on the
    generating cause (small sigma, well separated non-negative columns), the
    MCA responsibilities are hard assignments and the W update is the mean
    of the points assigned to each component (a k-means centroid step)."""
    g = np.random.default_rng(17)
    D, H, N = 9, 4, 80
    W = np.abs(g.standard_normal((D, H))) * 3.0 + 0.5
    lab = g.integers(0, H, N)
    Y = W[:, lab].T + 0.05 * g.standard_normal((N, D))
    est = O.estep("mca", Y, W, 0.3, 0.05, H, 1)
    Wn, _, _ = O.mstep("mca", Y, W, est)
    for h in range(H):
        np.testing.assert_allclose(Wn[:, h], Y[lab == h].mean(axis=0), rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- EM
def test_exact_em_free_energy_monotone_on_bars():
    Y, _, _, wl = synth.make_workload("bars", N=300)
    W0, pi0, s0 = synth.initial_params(wl, Y)
    F, W, pi, sigma = O.em_run("bsc", Y, W0, pi0, s0, 10, 10, 10)
    assert all(b >= a - 1e-7 * abs(a) for a, b in zip(F, F[1:])), F
    assert F[-1] > F[0]


def _bars_match(W):
    from scipy.optimize import linear_sum_assignment
    G = synth.bars_dictionary()
    Wn = W / np.linalg.norm(W, axis=0, keepdims=True)
    Gn = G / np.linalg.norm(G, axis=0, keepdims=True)
    C = Gn.T @ Wn
    r, c = linear_sum_assignment(-C)
    return C[r, c]


def test_bars_recovered():
    """Exact EM from W0 ~ N(0,1) recovers the ten generating bars and the
    generating prior and noise (pi = 0.2, sigma = 2)."""
    Y, _, _, wl = synth.make_workload("bars", N=300)
    for seed in (100, 101):
        W0, pi0, s0 = synth.initial_params(wl, Y, seed=seed)
        F, W, pi, sigma = O.em_run("bsc", Y, W0, pi0, s0, 10, 10, 15)
        assert _bars_match(W).min() >= 0.95
        assert abs(pi - 0.2) < 0.03 and abs(sigma - 2.0) < 0.1
