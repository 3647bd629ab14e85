"""Plain FP64 reference of the truncated-EM sparse-coding learners.

TEST INFRASTRUCTURE.  This file is the oracle that the GPU library is checked
against.  Only the test-suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product path never does, and the two share
no code.  Everything here is written for obviousness, not speed: every
log-joint is evaluated from its definition with the *direct* residual
||y - f(s)||^2 and library routines (matrix product, logsumexp, linear solve)
are the only building blocks.

What is computed (ProSper, "Learning Algorithm and Data Models", Eq. 1-2,
Table 1; truncated posteriors per the same section and the introduction):

* generative model  p(s | Theta) p(y | s, Theta) with Gaussian noise of
  standard deviation sigma and mean f(Theta, s):
    - BSC: s in {0,1}^H, Bernoulli(pi) prior, f = W s
    - TSC: s in {-1,0,1}^H, P(+-1) = pi/2, P(0) = 1 - pi, f = W s
    - MCA: s in {0,1}^H, Bernoulli(pi) prior, f_d = max_h s_h W_dh
    - MMCA: s in {0,1}^H, Bernoulli(pi) prior, f_d = the s_h W_dh of
      largest magnitude (ties to the lower h)
* E-step with truncated posteriors: per data point a set I_n of H' latents is
  preselected ("Hprime" of the API section), the state set K_n holds every
  state whose support lies in I_n with at most gamma non-zero entries
  ("gamma" of the API section), and q_n(s) is the exact posterior
  renormalised on K_n.
* M-step: the joint maximiser of sum_n sum_s q_n(s) log p(y_n, s | Theta).

Annealing: an optional posterior temperature beta (q proportional to
p(y, s)^beta on K_n), the deterministic annealing of the approximate
posterior named for the schedule object of the user-interface section;
logL is reported untempered.

Readings where the paper is silent (each listed in the design notes):
  selection score = singleton log-joint, ties to the lower index, points
  flagged when the H'-th and (H'+1)-th scores lie within 1e-6 relative;
  canonical state order = (number of active slots, lexicographic slot
  tuple, TSC sign pattern in binary counting order);
  MCA M-step = hard-max responsibilities (limit of the smooth max), sigma
  from the old W in the same sweep; MMCA takes the same M-step with the
  responsibility given to the active latent of largest |W_dh|.

DSC (discrete sparse coding, Table 1: linear superposition, Gaussian noise,
discrete latents with a categorical prior): s_h takes one of V values
phi_0 = 0, phi_1, ..., phi_{V-1} with probabilities pv_0 .. pv_{V-1} (the
value set is given, the probabilities are learned).  Its functions are the
dsc_* ones below, written out separately; with V = 2, phi = (0, 1) it is
BSC and with V = 3, phi = (0, 1, -1), pv = (1 - pi, pi/2, pi/2) it is TSC.
Readings: K_n as for TSC with the V - 1 non-zero values per active slot
(|K| = sum_k C(H', k) (V - 1)^k), value codes of one support in mixed-radix
counting order with the first active slot's digit least significant; the
selection score of latent h is its best singleton log-joint over the
non-zero values, in the units of the other scores (times sigma^2, up to
h-independent terms); the M-step sets pv_v (v >= 1) to the expected share
of latents taking phi_v.

Parity pins: see tests/test_oracle_*.py (brute force over all states with
scipy's multivariate normal, closed forms at H = 1, MCA == BSC special cases,
posterior invariants, textbook least squares, the MCA update as a cluster
mean for single-cause posteriors, the EM monotonicity theorem, bars
recovery).

Parity unpinned: the MCA noise update's use of the old W (mstep, MCA
branch) is a reading with nothing outside this file to check it against;
its W update and everything else here is pinned.
"""
from __future__ import annotations

import math
from itertools import combinations
from typing import Dict, List, Sequence, Tuple

import numpy as np
from scipy.special import logsumexp

__all__ = [
    "BSC", "TSC", "MCA", "MMCA", "MODELS", "MAX_MODELS", "TIE_REL",
    "state_table", "state_masks", "log_prior", "superposition", "log_joint",
    "selection_scores", "preselect", "estep_point", "estep", "mstep",
    "em_run", "free_energy", "truncated_prior_moments", "mstep_et", "DSC", "dsc_state_table", "dsc_state_count",
    "dsc_log_joint", "dsc_selection_scores", "dsc_estep_point", "dsc_estep", "dsc_mstep",
]

BSC, TSC, MCA, MMCA = "bsc", "tsc", "mca", "mmca"
MODELS = (BSC, TSC, MCA, MMCA)
MAX_MODELS = (MCA, MMCA)  # non-linear superposition, responsibility M-step
TIE_REL = 1e-6  # selection boundary flag band (relative, floor 1)


# --------------------------------------------------------------------------
# truncated state set K (API section: Hprime, gamma)
# --------------------------------------------------------------------------
def state_table(model: str, Hp: int, gamma: int) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """All states with support inside the H' slots and at most gamma actives.

    A state is (slots, values): ascending slot indices j in [0, H') and the
    value of each active slot (+1 for BSC/MCA; +-1 for TSC).
    Canonical order: k ascending; slot tuples lexicographically; for TSC the
    sign patterns of one support in binary counting order, bit i of the
    counter giving the sign of the i-th active slot (0 -> +1, 1 -> -1).
    """
    out = []
    for k in range(0, min(gamma, Hp) + 1):
        for slots in combinations(range(Hp), k):
            if model == TSC:
                for code in range(1 << k):
                    vals = tuple(-1 if (code >> i) & 1 else 1 for i in range(k))
                    out.append((slots, vals))
            else:
                out.append((slots, (1,) * k))
    return out


def state_masks(model: str, Hp: int, gamma: int) -> Tuple[np.ndarray, np.ndarray]:
    """Bit masks of the canonical table: active[k] has bit j set iff slot j is
    active; sign[k] has bit j set iff slot j holds -1."""
    tab = state_table(model, Hp, gamma)
    act = np.zeros(len(tab), dtype=np.uint32)
    sgn = np.zeros(len(tab), dtype=np.uint32)
    for i, (slots, vals) in enumerate(tab):
        for j, v in zip(slots, vals):
            act[i] |= np.uint32(1 << j)
            if v < 0:
                sgn[i] |= np.uint32(1 << j)
    return act, sgn


def _embed(tab, sel: Sequence[int], H: int) -> np.ndarray:
    """States of the table as full H-vectors (rows), slots mapped through sel."""
    S = np.zeros((len(tab), H))
    for i, (slots, vals) in enumerate(tab):
        for j, v in zip(slots, vals):
            S[i, sel[j]] = v
    return S


# --------------------------------------------------------------------------
# the generative model (Eq. 1 prior, Eq. 2 Gaussian noise around f(Theta, s))
# --------------------------------------------------------------------------
def log_prior(model: str, S: np.ndarray, pi: float) -> np.ndarray:
    """log p(s | Theta) for every row of S (sum over latents of log p(s_h))."""
    nz = (S != 0)
    if model == TSC:
        per = np.where(nz, np.log(pi / 2.0), np.log1p(-pi))
    else:
        per = np.where(nz, np.log(pi), np.log1p(-pi))
    return per.sum(axis=-1)


def superposition(model: str, W: np.ndarray, S: np.ndarray) -> np.ndarray:
    """f(Theta, s) for every row of S: W s (linear), max_h s_h W_dh (MCA) or
    the s_h W_dh of largest magnitude, ties to the lower h (MMCA)."""
    if model == MCA:
        return (S[:, None, :] * W[None, :, :]).max(axis=2)
    if model == MMCA:
        SW = S[:, None, :] * W[None, :, :]                 # |K| x D x H
        win = np.abs(SW).argmax(axis=2)                     # first maximum
        return np.take_along_axis(SW, win[:, :, None], axis=2)[:, :, 0]
    return S @ W.T


def log_joint(model: str, y: np.ndarray, W: np.ndarray, pi: float, sigma: float,
              S: np.ndarray) -> np.ndarray:
    """log p(y, s | Theta) for every row s of S, with the direct residual."""
    D = y.shape[0]
    R = y[None, :] - superposition(model, W, S)
    sq = (R * R).sum(axis=1)
    return (log_prior(model, S, pi)
            - 0.5 * D * np.log(2.0 * np.pi * sigma * sigma)
            - sq / (2.0 * sigma * sigma))


# --------------------------------------------------------------------------
# preselection of H' latents
# --------------------------------------------------------------------------
def selection_scores(model: str, y: np.ndarray, W: np.ndarray) -> np.ndarray:
    """r_h = 1/2||y||^2 - 1/2||y - f(e_h)||^2 (the singleton log-joint up to
    h-independent terms and the positive factor 1/sigma^2); for TSC the better
    of the two signs."""
    H = W.shape[1]
    E = np.eye(H)
    yy = 0.5 * float(y @ y)
    R = y[None, :] - superposition(model, W, E)
    r = yy - 0.5 * (R * R).sum(axis=1)
    if model == TSC:
        Rm = y[None, :] - superposition(model, W, -E)
        r = np.maximum(r, yy - 0.5 * (Rm * Rm).sum(axis=1))
    return r


def preselect(r: np.ndarray, Hp: int, tie_rel: float = TIE_REL) -> Tuple[np.ndarray, bool]:
    """The H' largest scores, ties to the lower index, returned ascending.
    Flagged when the H'-th and (H'+1)-th largest scores are within tie_rel
    (relative to max(1, |r_(H')|))."""
    H = r.shape[0]
    order = sorted(range(H), key=lambda h: (-r[h], h))
    sel = np.array(sorted(order[:Hp]), dtype=np.int64)
    flagged = False
    if Hp < H:
        a, b = r[order[Hp - 1]], r[order[Hp]]
        flagged = bool(abs(a - b) <= tie_rel * max(1.0, abs(a)))
    return sel, flagged


# --------------------------------------------------------------------------
# E-step
# --------------------------------------------------------------------------
def estep_point(model: str, y: np.ndarray, W: np.ndarray, pi: float, sigma: float,
                Hp: int, gamma: int, topk: int = 0, tab=None, sel=None,
                beta: float = 1.0) -> Dict:
    """Truncated posterior of one data point (all float64).

    `sel` (optional, H' distinct latents) replaces the preselected set I_n;
    it is meant for near-tie points, where more than one candidate set is a
    correct preselection and the posterior on another valid one is wanted.
    The scores and the near-tie flag are still those of the data point.

    `beta` in (0, 1] is the posterior temperature of deterministic annealing
    (the schedule object of the user-interface section anneals the
    approximate posterior): q(s) is proportional to p(y, s | Theta)^beta on
    K_n, and every moment and statistic is taken under that q.  logL stays
    the untempered log sum_{s in K_n} p(y, s | Theta)."""
    y = np.asarray(y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    H = W.shape[1]
    r = selection_scores(model, y, W)
    auto, flagged = preselect(r, Hp)
    if sel is None:
        sel = auto
    else:
        sel = np.sort(np.asarray(sel, dtype=np.int64))
        if sel.shape != (Hp,) or len(set(sel.tolist())) != Hp or sel[0] < 0 or sel[-1] >= H:
            raise ValueError("sel must hold H' distinct latent indices")
    if tab is None:
        tab = state_table(model, Hp, gamma)
    S = _embed(tab, sel, H)                      # |K| x H
    lj = log_joint(model, y, W, pi, sigma, S)    # |K|
    logL = float(logsumexp(lj))
    q = np.exp(beta * lj - logsumexp(beta * lj))
    Ss = S[:, sel]                               # |K| x H' (values per slot)
    s_mean = q @ Ss
    ss_mean = (Ss * q[:, None]).T @ Ss
    k = (Ss != 0).sum(axis=1)
    out = dict(sel=sel, flagged=flagged, scores=r, lj=lj, q=q, logL=logL,
               s_mean=s_mean, ss_mean=ss_mean, k_mean=float(q @ k))
    if topk:
        idx = np.arange(len(tab))
        order = np.lexsort((idx, -q))[:topk]
        out["top_index"] = order
        out["top_q"] = q[order]
    if model in MAX_MODELS:
        # responsibilities: R[d, j] = sum_s q(s) [slot j is the lowest-index
        # active slot attaining the max of W_d (MCA) or of |W_d| (MMCA) over
        # the active set, and that max is > 0]
        Wc = W[:, sel]
        R = np.zeros((W.shape[0], Hp))
        res = y[None, :] - superposition(model, W, S)
        for i, (slots, _vals) in enumerate(tab):
            if not slots:
                continue
            sub = Wc[:, list(slots)]
            if model == MMCA:
                sub = np.abs(sub)
            am = np.argmax(sub, axis=1)
            mx = sub[np.arange(sub.shape[0]), am]
            pos = mx > 0
            R[np.nonzero(pos)[0], np.array(slots)[am[pos]]] += q[i]
        out["R"] = R
        out["res_mean"] = float(q @ (res * res).sum(axis=1))
    return out


def estep(model: str, Y: np.ndarray, W: np.ndarray, pi: float, sigma: float,
          Hp: int, gamma: int, topk: int = 0, keep_posterior: bool = False,
          sel: np.ndarray = None, beta: float = 1.0) -> Dict:
    """Truncated E-step over all points, plus the M-step accumulators.
    `sel` (optional, N x H') replaces the preselection point by point, and
    `beta` is the posterior temperature (see estep_point).

    Returns per-point arrays (sel, flagged, logL, s_mean, ss_mean, k_mean,
    top_index, top_q) and the sums
      BSC/TSC: A = sum y <s>^T (D x H), B = sum <ss^T> (H x H)
      MCA/MMCA: A = sum R * y (D x H),  B = sum R (D x H)
      scal = [sum <k>, sum logL, sum ||y||^2, sum <||y - f(s)||^2> (MCA/MMCA), N]
    """
    Y = np.asarray(Y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    N, D = Y.shape
    H = W.shape[1]
    forced = sel
    tab = state_table(model, Hp, gamma)
    sel = np.zeros((N, Hp), dtype=np.int64)
    flagged = np.zeros(N, dtype=bool)
    logL = np.zeros(N)
    s_mean = np.zeros((N, Hp))
    ss_mean = np.zeros((N, Hp, Hp))
    k_mean = np.zeros(N)
    top_index = np.zeros((N, topk), dtype=np.int64)
    top_q = np.zeros((N, topk))
    A = np.zeros((D, H))
    B = np.zeros((H, H)) if model not in MAX_MODELS else np.zeros((D, H))
    res_sum = 0.0
    post = []
    for n in range(N):
        p = estep_point(model, Y[n], W, pi, sigma, Hp, gamma, topk, tab,
                        None if forced is None else forced[n], beta)
        sel[n], flagged[n], logL[n] = p["sel"], p["flagged"], p["logL"]
        s_mean[n], ss_mean[n], k_mean[n] = p["s_mean"], p["ss_mean"], p["k_mean"]
        if topk:
            top_index[n], top_q[n] = p["top_index"], p["top_q"]
        c = p["sel"]
        if model in MAX_MODELS:
            A[:, c] += p["R"] * Y[n][:, None]
            B[:, c] += p["R"]
            res_sum += p["res_mean"]
        else:
            A[:, c] += np.outer(Y[n], p["s_mean"])
            B[np.ix_(c, c)] += p["ss_mean"]
        if keep_posterior:
            post.append((c, p["q"]))
    scal = np.array([k_mean.sum(), logL.sum(), float((Y * Y).sum()), res_sum, float(N)])
    out = dict(sel=sel, flagged=flagged, logL=logL, s_mean=s_mean, ss_mean=ss_mean,
               k_mean=k_mean, top_index=top_index, top_q=top_q, A=A, B=B, scal=scal,
               table=tab)
    if keep_posterior:
        out["posterior"] = post
    return out


def free_energy(est: Dict) -> float:
    """Truncated free energy sum_n log sum_{s in K_n} p(y_n, s | Theta)."""
    return float(est["scal"][1])


# --------------------------------------------------------------------------
# M-step: joint maximiser of sum_n sum_s q_n(s) log p(y_n, s | Theta)
# --------------------------------------------------------------------------
def mstep(model: str, Y: np.ndarray, W_old: np.ndarray, est: Dict,
          Hp: int = None, gamma: int = None):
    """New (W, pi, sigma) from one E-step's statistics.

    BSC/TSC: W = A B^-1 on the latents with B_hh > 0 (others keep their old
    column); pi = sum<k>/(N H); sigma^2 = sum_n sum_s q ||y - W_new s||^2/(N D)
    as a direct second sweep over each K_n (needs keep_posterior=True).
    MCA/MMCA: W_dh = sum R y / sum R (zero denominator keeps the old value);
    pi as BSC; sigma^2 = sum_n sum_s q ||y - f_{W_old}(s)||^2 / (N D).
    """
    Y = np.asarray(Y, dtype=np.float64)
    W_old = np.asarray(W_old, dtype=np.float64)
    N, D = Y.shape
    H = W_old.shape[1]
    A, B, scal = est["A"], est["B"], est["scal"]
    pi_new = scal[0] / (N * H)
    W_new = W_old.copy()
    if model in MAX_MODELS:
        pos = B > 0
        W_new[pos] = A[pos] / B[pos]
        sigma2 = scal[3] / (N * D)
    else:
        act = np.diag(B) > 0
        if act.any():
            Bact = B[np.ix_(act, act)]
            W_new[:, act] = np.linalg.solve(Bact, A[:, act].T).T
        tab = est["table"]
        tot = 0.0
        for n, (c, q) in enumerate(est["posterior"]):
            S = _embed(tab, c, H)
            R = Y[n][None, :] - S @ W_new.T
            tot += float(q @ (R * R).sum(axis=1))
        sigma2 = tot / (N * D)
    return W_new, float(pi_new), float(np.sqrt(sigma2))


# --------------------------------------------------------------------------
# M-step variant: pi and sigma from the points best explained by <= gamma
# causes (deterministic-annealing section's "M-step variants"; a reading,
# the paper gives no formula)
# --------------------------------------------------------------------------
def truncated_prior_moments(H: int, gamma: int, pi: float) -> Tuple[float, float]:
    """A = P(#non-zero latents <= gamma) and B = E[#non-zero; #non-zero <= gamma]
    under the prior of Eq. 1 with H independent latents, each non-zero with
    probability pi (BSC, and TSC's two signs together)."""
    A = B = 0.0
    for k in range(0, min(gamma, H) + 1):
        p = math.comb(H, k) * pi ** k * (1.0 - pi) ** (H - k)
        A += p
        B += k * p
    return A, B


def mstep_et(model: str, Y: np.ndarray, W_old: np.ndarray, est: Dict, pi: float,
             gamma: int):
    """BSC/TSC M-step with pi and sigma taken from the selected points:
    W_new as `mstep` (all points); M = the N_cut = clamp(round(N A(pi)), 1, N)
    points with the largest logL_n (ties to the lower index) -- the share of
    prior draws with at most gamma causes;
      pi_new = pi * mean_{n in M} <k>_n * A(pi) / B(pi)   (pi if B = 0),
    which maps the mean number of causes among truncated explanations
    (B/A at the generating pi) back to pi; and
      sigma_new^2 = sum_{n in M} sum_s q_n(s) ||y_n - W_old s||^2 / (N_cut D)
    with the W of the E-step.  Needs keep_posterior.  Returns
    (W_new, pi_new, sigma_new, M)."""
    if model not in (BSC, TSC):
        raise ValueError("the selected-points M-step is defined for BSC and TSC")
    Y = np.asarray(Y, dtype=np.float64)
    W_old = np.asarray(W_old, dtype=np.float64)
    N, D = Y.shape
    H = W_old.shape[1]
    W_new, _, _ = mstep(model, Y, W_old, est)
    A, B = truncated_prior_moments(H, gamma, pi)
    n_cut = min(N, max(1, int(round(N * A))))
    logL = est["logL"]
    M = sorted(range(N), key=lambda n: (-logL[n], n))[:n_cut]
    kbar = float(np.mean(est["k_mean"][M]))
    pi_new = pi * kbar * A / B if B > 0.0 else pi
    tot = 0.0
    for n in M:
        c, q = est["posterior"][n]
        S = _embed(est["table"], c, H)
        R = Y[n][None, :] - S @ W_old.T
        tot += float(q @ (R * R).sum(axis=1))
    return W_new, float(pi_new), float(np.sqrt(tot / (n_cut * D))), np.array(sorted(M))


def em_run(model: str, Y: np.ndarray, W0: np.ndarray, pi0: float, sigma0: float,
           Hp: int, gamma: int, iters: int, callback=None):
    """Plain EM loop: E-step at Theta_t, M-step to Theta_{t+1}.

    Returns the list of free energies F(Theta_t) (t = 0..iters-1) and the
    final parameters.
    """
    W, pi, sigma = np.asarray(W0, dtype=np.float64), float(pi0), float(sigma0)
    F = []
    for it in range(iters):
        est = estep(model, Y, W, pi, sigma, Hp, gamma, keep_posterior=(model not in MAX_MODELS))
        F.append(free_energy(est))
        W, pi, sigma = mstep(model, Y, W, est)
        if callback is not None:
            callback(it, W, pi, sigma, est)
    return F, W, pi, sigma


# --------------------------------------------------------------------------
# DSC: discrete latents phi_0 = 0, phi_1, ..., phi_{V-1}, categorical prior pv
# --------------------------------------------------------------------------
DSC = "dsc"


def _check_dsc(phi, pv):
    phi = np.asarray(phi, dtype=np.float64)
    pv = np.asarray(pv, dtype=np.float64)
    if phi.ndim != 1 or phi.shape != pv.shape or phi.shape[0] < 2 or phi[0] != 0.0:
        raise ValueError("phi and pv hold V >= 2 entries and phi[0] = 0")
    if np.any(phi[1:] == 0.0) or len(set(phi.tolist())) != len(phi):
        raise ValueError("the non-zero values phi_1.. must be distinct and non-zero")
    if np.any(pv <= 0.0) or abs(pv.sum() - 1.0) > 1e-12:
        raise ValueError("pv must be positive and sum to 1")
    return phi, pv


def dsc_state_table(V: int, Hp: int, gamma: int) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
    """All states with support inside the H' slots and at most gamma actives,
    as (slots, codes): ascending slot indices and the value code (1..V-1,
    index into phi) of each active slot.  Order: k ascending; slot tuples
    lexicographically; the codes of one support in mixed-radix counting
    order, the digit of the first active slot least significant."""
    out = []
    for k in range(0, min(gamma, Hp) + 1):
        for slots in combinations(range(Hp), k):
            for count in range((V - 1) ** k):
                codes, c = [], count
                for _ in range(k):
                    codes.append(1 + c % (V - 1))
                    c //= V - 1
                out.append((slots, tuple(codes)))
    return out


def dsc_state_count(V: int, Hp: int, gamma: int) -> int:
    return sum(math.comb(Hp, k) * (V - 1) ** k for k in range(0, min(gamma, Hp) + 1))


def _dsc_embed(tab, sel, H, phi):
    """States of the table as H-vectors of values and of value codes."""
    S = np.zeros((len(tab), H))
    C = np.zeros((len(tab), H), dtype=np.int64)
    for i, (slots, codes) in enumerate(tab):
        for j, c in zip(slots, codes):
            S[i, sel[j]] = phi[c]
            C[i, sel[j]] = c
    return S, C


def dsc_log_joint(y, W, phi, pv, sigma, S, C) -> np.ndarray:
    """log p(y, s | Theta) for every row (values S, codes C): the categorical
    prior sum_h log pv[c_h] and the Gaussian noise with the direct residual."""
    D = y.shape[0]
    logp = np.log(pv)[C].sum(axis=1)
    R = y[None, :] - S @ W.T
    return logp - 0.5 * D * np.log(2.0 * np.pi * sigma * sigma) - (R * R).sum(axis=1) / (2.0 * sigma * sigma)


def dsc_selection_scores(y, W, phi, pv, sigma) -> np.ndarray:
    """r_h = max over v >= 1 of sigma^2 log(pv_v / pv_0) + 1/2||y||^2
    - 1/2||y - phi_v W_h||^2: sigma^2 times the singleton log-joint of
    (h, phi_v) up to h-independent terms."""
    H = W.shape[1]
    yy = 0.5 * float(y @ y)
    best = np.full(H, -np.inf)
    for v in range(1, len(phi)):
        R = y[None, :] - phi[v] * W.T
        r = sigma * sigma * np.log(pv[v] / pv[0]) + yy - 0.5 * (R * R).sum(axis=1)
        best = np.maximum(best, r)
    return best


def dsc_estep_point(y, W, phi, pv, sigma, Hp, gamma, topk=0, tab=None, beta=1.0,
                    sel=None) -> Dict:
    """Truncated posterior of one point for DSC (all float64); outputs as
    estep_point plus v_mean[v] = expected number of latents taking phi_v.
    `sel` (optional) replaces the preselected set, as in estep_point."""
    phi, pv = _check_dsc(phi, pv)
    y = np.asarray(y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    H = W.shape[1]
    V = len(phi)
    r = dsc_selection_scores(y, W, phi, pv, sigma)
    if sel is None:
        sel, flagged = preselect(r, Hp)
    else:
        flagged = preselect(r, Hp)[1]
        sel = np.sort(np.asarray(sel, dtype=np.int64))
    if tab is None:
        tab = dsc_state_table(V, Hp, gamma)
    S, C = _dsc_embed(tab, sel, H, phi)
    lj = dsc_log_joint(y, W, phi, pv, sigma, S, C)
    logL = float(logsumexp(lj))
    q = np.exp(beta * lj - logsumexp(beta * lj))
    Ss, Cs = S[:, sel], C[:, sel]
    v_mean = np.array([float(q @ (Cs == v).sum(axis=1)) for v in range(V)])
    out = dict(sel=sel, flagged=flagged, scores=r, lj=lj, q=q, logL=logL,
               s_mean=q @ Ss, ss_mean=(Ss * q[:, None]).T @ Ss,
               k_mean=float(q @ (Cs != 0).sum(axis=1)), v_mean=v_mean)
    if topk:
        idx = np.arange(len(tab))
        order = np.lexsort((idx, -q))[:topk]
        out["top_index"] = order
        out["top_q"] = q[order]
    return out


def dsc_estep(Y, W, phi, pv, sigma, Hp, gamma, topk=0, keep_posterior=False, beta=1.0,
              sel=None) -> Dict:
    """DSC E-step over all points with the M-step sums: A = sum y <s>^T,
    B = sum <s s^T>, vcount[v] = sum_n <#latents at phi_v> (v = 0..V-1),
    scal = [sum <k>, sum logL, sum ||y||^2, 0, N].  `sel` (optional, N x H')
    replaces the preselection point by point."""
    forced = sel
    phi, pv = _check_dsc(phi, pv)
    Y = np.asarray(Y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    N, D = Y.shape
    H = W.shape[1]
    V = len(phi)
    tab = dsc_state_table(V, Hp, gamma)
    sel = np.zeros((N, Hp), dtype=np.int64)
    flagged = np.zeros(N, dtype=bool)
    logL = np.zeros(N)
    s_mean = np.zeros((N, Hp))
    k_mean = np.zeros(N)
    top_index = np.zeros((N, topk), dtype=np.int64)
    top_q = np.zeros((N, topk))
    A = np.zeros((D, H))
    B = np.zeros((H, H))
    vcount = np.zeros(V)
    post = []
    for n in range(N):
        p = dsc_estep_point(Y[n], W, phi, pv, sigma, Hp, gamma, topk, tab, beta,
                            None if forced is None else forced[n])
        sel[n], flagged[n], logL[n] = p["sel"], p["flagged"], p["logL"]
        s_mean[n], k_mean[n] = p["s_mean"], p["k_mean"]
        if topk:
            top_index[n], top_q[n] = p["top_index"], p["top_q"]
        c = p["sel"]
        A[:, c] += np.outer(Y[n], p["s_mean"])
        B[np.ix_(c, c)] += p["ss_mean"]
        vcount += p["v_mean"]
        if keep_posterior:
            post.append((c, p["q"]))
    vcount[0] = N * H - vcount[1:].sum()  # latents outside K's support are at phi_0
    scal = np.array([k_mean.sum(), logL.sum(), float((Y * Y).sum()), 0.0, float(N)])
    out = dict(sel=sel, flagged=flagged, logL=logL, s_mean=s_mean, k_mean=k_mean,
               top_index=top_index, top_q=top_q, A=A, B=B, scal=scal, vcount=vcount,
               table=tab, phi=phi)
    if keep_posterior:
        out["posterior"] = post
    return out


def dsc_mstep(Y, W_old, est):
    """New (W, pv, sigma): W = A B^-1 on the latents with B_hh > 0 (others
    keep their column); pv_v = vcount_v / (N H); sigma^2 = sum_n sum_s q
    ||y - W_new s||^2 / (N D) as a direct sweep (needs keep_posterior)."""
    Y = np.asarray(Y, dtype=np.float64)
    W_old = np.asarray(W_old, dtype=np.float64)
    N, D = Y.shape
    H = W_old.shape[1]
    A, B = est["A"], est["B"]
    W_new = W_old.copy()
    act = np.diag(B) > 0
    if act.any():
        W_new[:, act] = np.linalg.solve(B[np.ix_(act, act)], A[:, act].T).T
    pv_new = est["vcount"] / (N * H)
    tot = 0.0
    for n, (c, q) in enumerate(est["posterior"]):
        S, _ = _dsc_embed(est["table"], c, H, est["phi"])
        R = Y[n][None, :] - S @ W_new.T
        tot += float(q @ (R * R).sum(axis=1))
    return W_new, pv_new, float(np.sqrt(tot / (N * D)))
