"""Pins of the oracle's selected-points M-step (pi and sigma from the points
best explained by at most gamma causes; W from all points).  The variant is
a reading -- the paper names M-step variants but gives no formula -- so its
form is parity unpinned; its arithmetic is pinned here: the truncated-prior
moments against brute force over every binary vector, the reduction to the
plain M-step when gamma = H, the selection as a sort with ties to the lower
index, and the sigma sum against an explicit loop over the posterior."""
import itertools
import math

import numpy as np
import pytest

from oracle import prosper_oracle as O
import synth


@pytest.mark.parametrize("H,gamma,pi", [(6, 2, 0.2), (5, 0, 0.3), (7, 7, 0.1), (9, 3, 0.45)])
def test_truncated_prior_moments_brute_force(H, gamma, pi):
    A = B = 0.0
    for s in itertools.product((0, 1), repeat=H):
        k = sum(s)
        p = math.prod(pi if v else 1.0 - pi for v in s)
        if k <= gamma:
            A += p
            B += k * p
    a, b = O.truncated_prior_moments(H, gamma, pi)
    assert a == pytest.approx(A, rel=1e-12) and b == pytest.approx(B, rel=1e-12, abs=1e-15)


def problem(model, N=40, D=8, H=6, seed=2):
    g = synth.rng(seed)
    W = g.standard_normal((D, H))
    if model == O.TSC:
        S = synth.sample_ternary(g, N, H, 0.3)
    else:
        S = synth.sample_binary(g, N, H, 0.3)
    Y = S @ W.T + 0.5 * g.standard_normal((N, D))
    return Y, W


@pytest.mark.parametrize("model", [O.BSC, O.TSC])
def test_gamma_h_is_the_plain_mstep(model):
    """gamma = H: A = 1, B = H pi, every point selected; pi_new is the plain
    update and sigma the direct sweep with the E-step's W."""
    Y, W = problem(model)
    H = W.shape[1]
    est = O.estep(model, Y, W, 0.3, 0.6, H, H, keep_posterior=True)
    Wn, pn, sn, M = O.mstep_et(model, Y, W, est, 0.3, H)
    Wp, pp, _ = O.mstep(model, Y, W, est)
    np.testing.assert_allclose(Wn, Wp, rtol=1e-12)
    assert pn == pytest.approx(pp, rel=1e-12)
    assert len(M) == Y.shape[0]
    # sigma: explicit loop over every state of every point
    tot = 0.0
    for n, (c, q) in enumerate(est["posterior"]):
        for i, (slots, vals) in enumerate(est["table"]):
            s = np.zeros(H)
            for j, v in zip(slots, vals):
                s[c[j]] = v
            r = Y[n] - W @ s
            tot += q[i] * float(r @ r)
    assert sn == pytest.approx(math.sqrt(tot / (Y.shape[0] * Y.shape[1])), rel=1e-12)


def test_selection_is_the_top_logl_with_lower_index_ties():
    Y, W = problem(O.BSC, N=30)
    est = O.estep(O.BSC, Y, W, 0.3, 0.6, 4, 2, keep_posterior=True)
    A, _ = O.truncated_prior_moments(6, 2, 0.3)
    n_cut = int(round(30 * A))
    order = np.argsort(-est["logL"], kind="stable")
    _, pn, _, M = O.mstep_et(O.BSC, Y, W, est, 0.3, 2)
    np.testing.assert_array_equal(M, np.sort(order[:n_cut]))
    assert 0 < pn < 1
    # a planted four-way tie straddling the cut: exactly the lowest indices
    # of the tie fill the places left above it
    T = np.sort(est["logL"])[::-1][n_cut - 1]
    lg = est["logL"].copy()
    lg[order[[n_cut, n_cut + 2, n_cut + 4]]] = T   # three points from below the cut
    above = int((lg > T).sum())
    tie = np.sort(np.nonzero(lg == T)[0])
    assert len(tie) >= 4 and above < n_cut < above + len(tie)
    _, _, _, M2 = O.mstep_et(O.BSC, Y, W, dict(est, logL=lg), 0.3, 2)
    np.testing.assert_array_equal(np.intersect1d(M2, tie), tie[:n_cut - above])
    assert set(np.nonzero(lg > T)[0]) <= set(M2.tolist())


def test_pi_correction_fixed_point():
    """When the selected points' mean number of causes equals B/A at pi,
    pi is a fixed point of the update."""
    Y, W = problem(O.BSC)
    est = O.estep(O.BSC, Y, W, 0.25, 0.6, 6, 2, keep_posterior=True)
    A, B = O.truncated_prior_moments(6, 2, 0.25)
    est["k_mean"] = np.full(Y.shape[0], B / A)
    _, pn, _, _ = O.mstep_et(O.BSC, Y, W, est, 0.25, 2)
    assert pn == pytest.approx(0.25, rel=1e-12)


def test_rejects_max_models():
    Y, W = problem(O.BSC)
    est = O.estep(O.MCA, Y, np.abs(W), 0.3, 0.6, 4, 2)
    with pytest.raises(ValueError):
        O.mstep_et(O.MCA, Y, np.abs(W), est, 0.3, 2)
