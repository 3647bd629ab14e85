"""Pins of the oracle's MMCA model (Table 1: maximal-magnitude superposition).

f_d(s) is the s_h W_dh of largest magnitude; with binary s the inactive
latents contribute 0.  The pins reach the oracle through routes of their own:
hand-worked values, brute force over all 2^H states with explicit loops and
scipy's multivariate normal, and the reductions to MCA (non-negative or
non-positive dictionaries) and to BSC (a single latent).  CPU only.
"""
import itertools

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import bernoulli, multivariate_normal

from oracle import prosper_oracle as O


def loop_mean(W, s):
    """Largest-magnitude term per pixel, first one kept on a tie."""
    D, H = W.shape
    out = np.zeros(D)
    for d in range(D):
        best = 0.0
        for h in range(H):
            v = s[h] * W[d, h]
            if abs(v) > abs(best):
                best = v
        out[d] = best
    return out


def brute_posterior(y, W, pi, sigma):
    D, H = W.shape
    S = [np.array(v, dtype=float) for v in itertools.product((0, 1), repeat=H)]
    lj = np.array([bernoulli.logpmf(s.astype(int), pi).sum()
                   + multivariate_normal.logpdf(y, mean=loop_mean(W, s),
                                                cov=sigma * sigma * np.eye(D))
                   for s in S])
    logL = logsumexp(lj)
    q = np.exp(lj - logL)
    return logL, q @ np.array(S)


def problem(D, H, seed, sign=None, sigma=0.6, pi=0.3):
    g = np.random.default_rng(seed)
    W = g.standard_normal((D, H))
    if sign == "+":
        W = np.abs(W)
    elif sign == "-":
        W = -np.abs(W)
    s = (g.random(H) < pi).astype(float)
    Y = np.stack([loop_mean(W, (g.random(H) < pi).astype(float)) + sigma * g.standard_normal(D)
                  for _ in range(12)])
    return Y, W, pi, sigma


def test_hand_worked_superposition():
    W = np.array([[1.0, -2.0], [-1.0, 0.5], [3.0, -3.0]])
    S = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=float)
    f = O.superposition(O.MMCA, W, S)
    np.testing.assert_array_equal(f[0], [0.0, 0.0, 0.0])
    np.testing.assert_array_equal(f[1], [1.0, -1.0, 3.0])
    np.testing.assert_array_equal(f[2], [-2.0, 0.5, -3.0])
    # pixel 0: |-2| beats |1|; pixel 1: |-1| beats |0.5|; pixel 2: tie, lower h
    np.testing.assert_array_equal(f[3], [-2.0, -1.0, 3.0])


@pytest.mark.parametrize("D,H,seed", [(5, 3, 0), (4, 4, 1), (6, 2, 2)])
def test_untruncated_equals_brute_force(D, H, seed):
    Y, W, pi, sigma = problem(D, H, seed)
    for y in Y[:4]:
        p = O.estep_point(O.MMCA, y, W, pi, sigma, H, H)
        logL, s_mean = brute_posterior(y, W, pi, sigma)
        assert p["logL"] == pytest.approx(logL, rel=1e-12, abs=1e-12)
        np.testing.assert_allclose(p["s_mean"], s_mean[p["sel"]], rtol=1e-10, atol=1e-12)


def _same_estep(a, b, negate_A=False):
    np.testing.assert_array_equal(a["sel"], b["sel"])
    np.testing.assert_allclose(a["logL"], b["logL"], rtol=1e-12)
    np.testing.assert_allclose(a["s_mean"], b["s_mean"], rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(a["A"], -b["A"] if negate_A else b["A"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(a["B"], b["B"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(a["scal"], b["scal"], rtol=1e-10)


def test_equals_mca_for_nonnegative_dictionary():
    Y, W, pi, sigma = problem(8, 6, 3, sign="+")
    a = O.estep(O.MMCA, Y, W, pi, sigma, 4, 3)
    b = O.estep(O.MCA, Y, W, pi, sigma, 4, 3)
    _same_estep(a, b)
    Wa, pa, sa = O.mstep(O.MMCA, Y, W, a)
    Wb, pb, sb = O.mstep(O.MCA, Y, W, b)
    np.testing.assert_allclose(Wa, Wb, rtol=1e-12)
    assert (pa, sa) == pytest.approx((pb, sb), rel=1e-12)


def test_nonpositive_dictionary_mirrors_mca():
    # f_MMCA(W) = -f_MCA(-W) when W <= 0, so the point (y, W) behaves as
    # (-y, -W) does under MCA; the responsibilities are the same and the
    # numerator changes sign with y.
    Y, W, pi, sigma = problem(8, 6, 4, sign="-")
    a = O.estep(O.MMCA, Y, W, pi, sigma, 4, 3)
    b = O.estep(O.MCA, -Y, -W, pi, sigma, 4, 3)
    _same_estep(a, b, negate_A=True)
    Wa, _, sa = O.mstep(O.MMCA, Y, W, a)
    Wb, _, sb = O.mstep(O.MCA, -Y, -W, b)
    np.testing.assert_allclose(Wa, -Wb, rtol=1e-12)
    assert sa == pytest.approx(sb, rel=1e-12)


def test_single_latent_equals_bsc():
    g = np.random.default_rng(5)
    W = g.standard_normal((7, 1))
    Y = np.outer(g.random(10) < 0.5, W[:, 0]) + 0.5 * g.standard_normal((10, 7))
    a = O.estep(O.MMCA, Y, W, 0.4, 0.5, 1, 1)
    b = O.estep(O.BSC, Y, W, 0.4, 0.5, 1, 1, keep_posterior=True)
    np.testing.assert_allclose(a["logL"], b["logL"], rtol=1e-12)
    np.testing.assert_allclose(a["s_mean"], b["s_mean"], rtol=1e-12)
    # every pixel of the one latent is non-zero, so R = <s> and W = sum<s>y / sum<s>
    Wa, pa, _ = O.mstep(O.MMCA, Y, W, a)
    Wb, pb, _ = O.mstep(O.BSC, Y, W, b)
    np.testing.assert_allclose(Wa, Wb, rtol=1e-10)
    assert pa == pytest.approx(pb, rel=1e-12)
