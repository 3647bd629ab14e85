"""GPU parity at the sizes and launch shapes the benchmark uses.

At N = 150000 (BSC at scale) the persistent state walk with statistics makes
more than one pass over its points (it runs on at most one workgroup per CU
with 512 points per pass), the MFMA statistics kernel loops over many point
tiles per workgroup, and the deferred exact-selection kernel sees thousands
of points.  The max-superposition walk caps its grid at 8192 workgroups, so
N = 20000 runs its grid-stride loop.  Every point is compared with the FP64
oracle (run in a process pool), and so are the M-step sums A, B and scal.

Near-tie flag (the 1e-6 rule of the selection): the GPU flags a point when
its refined H'-th and (H'+1)-th scores are within 1e-6 max(1, |r|).  The
refined scores carry a few 1e-7 of rounding, so the checks leave that much
room: every GPU-flagged point has an oracle gap within 2e-6 max(1, |r|),
and every point whose oracle gap is within 0.4e-6 max(1, |r|) is flagged.
Points flagged by the oracle may carry another (equally valid) selection;
their share of the sums is then recomputed by the oracle on the GPU's
candidate set.
"""
import numpy as np
import pytest

import synth
from tests._common import TOL, assert_parity, gpu_estep, workload_params
from tests._pool import oracle_pool

pytestmark = pytest.mark.gpu

_ORACLE = {}


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def full_problem(name, N, theta, seed=None):
    Y, _, _, wl = synth.make_workload(name, N=N, seed=seed)
    W, pi, sigma = workload_params(name, theta, Y)
    return Y, np.ascontiguousarray(W, dtype=np.float32), float(pi), float(sigma), wl


def oracle_full(key, model, Y, W, pi, sigma, Hp, gamma):
    if key not in _ORACLE:
        print(f"[oracle] {key}: {Y.shape[0]} points in a process pool", flush=True)
        _ORACLE[key] = oracle_pool(model, Y, W, pi, sigma, Hp, gamma)
    return _ORACLE[key]


def reconciled_sums(model, Y, W, pi, sigma, Hp, gamma, g, r):
    """Oracle sums with every near-tie point whose GPU selection differs
    taken on the GPU's candidate set."""
    same = np.all(g["sel"] == r["sel"], axis=1)
    mism = np.nonzero(~same)[0]
    assert r["flagged"][mism].all(), "selection differs on a point the oracle does not flag"
    A, B, scal = r["A"].copy(), r["B"].copy(), r["scal"].copy()
    if len(mism):
        a = oracle_pool(model, Y[mism], W, pi, sigma, Hp, gamma, workers=1)
        b = oracle_pool(model, Y[mism], W, pi, sigma, Hp, gamma, sel=g["sel"][mism], workers=1)
        A += b["A"] - a["A"]
        B += b["B"] - a["B"]
        scal += b["scal"] - a["scal"]
    return A, B, scal, len(mism)


def check_flags(g, r, label):
    gf = np.asarray(g["flagged"], dtype=bool)
    scale = np.maximum(1.0, np.abs(r["rH"]))
    near = r["gap"] <= 0.4e-6 * scale
    print(f"[flags] {label}: gpu {int(gf.sum())} oracle {int(r['flagged'].sum())} "
          f"clear near-ties {int(near.sum())}", flush=True)
    assert np.all(r["gap"][gf] <= 2e-6 * scale[gf]), "GPU flagged a point that is no near-tie"
    assert np.all(gf[near]), "a clear near-tie is not flagged"


def check_sums(model, g, A, B, scal, N, tol):
    Bg = g["B"]
    if model in ("bsc", "tsc"):       # the GPU accumulates the upper triangle of B
        Bg = np.triu(Bg) + np.triu(Bg, 1).T
    ea, eb = rel(g["A"], A), rel(Bg, B)
    es = np.abs(g["scal"] - scal) / np.maximum(np.abs(scal), 1.0)
    print(f"[sums] A {ea:.2e} B {eb:.2e} scal {es}", flush=True)
    assert ea < tol and eb < tol
    assert es[0] < tol and es[1] < 1e-5 and es[2] < 1e-9
    if model in ("mca", "mmca"):
        assert es[3] < 1e-5
    assert g["scal"][4] == N


@pytest.mark.parametrize("prec", ["bf16", "fp32", "bf16x1"])
def test_bsc256_statistics_full_size(prec):
    name, N = "bsc256", 150000
    Y, W, pi, sigma, wl = full_problem(name, N, "init")
    print(f"[case] {name} N={N} init {prec} with statistics", flush=True)
    g = gpu_estep("bsc", prec, Y, W, pi, sigma, wl.Hprime, wl.gamma, accumulate=True)
    r = oracle_full((name, N, "init"), "bsc", Y, W, pi, sigma, wl.Hprime, wl.gamma)
    assert_parity(g, r, prec, f"full {name} N={N}")
    check_flags(g, r, f"{name} {prec}")
    A, B, scal, nm = reconciled_sums("bsc", Y, W, pi, sigma, wl.Hprime, wl.gamma, g, r)
    print(f"[sums] near-tie points on another selection: {nm}", flush=True)
    check_sums("bsc", g, A, B, scal, N, 3e-5 if prec == "fp32" else 1e-4)


@pytest.mark.parametrize("model", ["mca", "mmca"])
def test_max_models_grid_stride_with_statistics(model):
    """N = 20000 > 8192 workgroups: every max-superposition walk workgroup
    takes several points.  MMCA runs on a signed dictionary."""
    N = 20000
    Y, W, pi, sigma, wl = full_problem("mca", N, "init")
    if model == "mmca":
        W = np.ascontiguousarray(
            W * np.where(np.random.default_rng(5).random(W.shape) < 0.5, -1.0, 1.0), np.float32)
    print(f"[case] {model} N={N} init fp32 with statistics", flush=True)
    g = gpu_estep(model, "fp32", Y, W, pi, sigma, wl.Hprime, wl.gamma, accumulate=True)
    r = oracle_full((model, N, "init"), model, Y, W, pi, sigma, wl.Hprime, wl.gamma)
    assert_parity(g, r, "fp32", f"{model} N={N}")
    check_flags(g, r, model)
    A, B, scal, _ = reconciled_sums(model, Y, W, pi, sigma, wl.Hprime, wl.gamma, g, r)
    check_sums(model, g, A, B, scal, N, 3e-5)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tsc_full_size_with_statistics(prec):
    name = "tsc"
    Y, W, pi, sigma, wl = full_problem(name, None, "init")
    N = Y.shape[0]
    print(f"[case] {name} N={N} init {prec} with statistics", flush=True)
    g = gpu_estep("tsc", prec, Y, W, pi, sigma, wl.Hprime, wl.gamma, accumulate=True)
    r = oracle_full((name, N, "init"), "tsc", Y, W, pi, sigma, wl.Hprime, wl.gamma)
    assert_parity(g, r, prec, f"full {name}")
    check_flags(g, r, f"{name} {prec}")
    A, B, scal, _ = reconciled_sums("tsc", Y, W, pi, sigma, wl.Hprime, wl.gamma, g, r)
    check_sums("tsc", g, A, B, scal, N, 1e-4 if prec == "bf16" else 3e-5)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x1"])
def test_planted_exact_tie_is_flagged_and_takes_the_lower_index(prec):
    """Latents 5 and 9 have identical columns and sit exactly at the H'-th and
    (H'+1)-th place: the oracle flags the point and selects 5; so must the GPU."""
    g = np.random.default_rng(17)
    D, H, Hp = 64, 32, 4
    W = g.standard_normal((D, H))
    W /= np.linalg.norm(W, axis=0)
    W[:, 9] = W[:, 5]
    Y = []
    for n in range(40):
        y = 3.0 * (W[:, 0] + W[:, 1] + W[:, 2]) + 1.2 * W[:, 5] + 0.01 * g.standard_normal(D)
        Y.append(y)
    Y = np.array(Y, dtype=np.float32)
    W = W.astype(np.float32)
    from oracle import prosper_oracle as O
    r = O.estep("bsc", Y, W, 0.1, 0.5, Hp, 2)
    assert r["flagged"].all() and np.all(r["sel"] == [0, 1, 2, 5])
    out = gpu_estep("bsc", prec, Y, W, 0.1, 0.5, Hp, 2)
    assert np.all(out["flagged"] == 1)
    assert np.all(out["sel"] == [0, 1, 2, 5])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mca_all_active_state_with_negative_row(prec):
    """H' = H = gamma: the state with every latent active takes max_h W_dh of
    the unclamped dictionary, negative on a pixel whose row is all negative."""
    from oracle import prosper_oracle as O
    g = np.random.default_rng(23)
    D, H, N = 16, 6, 300
    W = np.abs(g.standard_normal((D, H)))
    W[3, :] = -np.abs(W[3, :]) - 0.2
    W[7, :] = -0.5
    S = (g.random((N, H)) < 0.5).astype(float)
    S[: N // 3] = 1.0
    mu = (S[:, None, :] * W[None, :, :]).max(axis=2)
    Y = (mu + 0.3 * g.standard_normal((N, D))).astype(np.float32)
    W = W.astype(np.float32)
    r = O.estep("mca", Y, W, 0.4, 0.3, H, H)
    out = gpu_estep("mca", prec, Y, W, 0.4, 0.3, H, H, accumulate=True)
    assert_parity(out, r, prec, "mca all-active")
    assert rel(out["A"], r["A"]) < 3e-5 and rel(out["B"], r["B"]) < 3e-5
    assert out["scal"][3] == pytest.approx(r["scal"][3], rel=2e-5)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_every_point_a_near_tie_overflows_the_deferral_list(prec):
    """8000 points, all with an exact tie at the selection boundary: more
    than the deferral list holds, so the rest take the exact selection inside
    the projection workgroups."""
    from oracle import prosper_oracle as O
    g = np.random.default_rng(31)
    D, H, Hp, N = 64, 32, 4, 8000
    W = g.standard_normal((D, H))
    W /= np.linalg.norm(W, axis=0)
    W[:, 9] = W[:, 5]
    Y = (3.0 * (W[:, 0] + W[:, 1] + W[:, 2]) + 1.2 * W[:, 5])[None, :] \
        + 0.01 * g.standard_normal((N, D))
    Y, W = Y.astype(np.float32), W.astype(np.float32)
    out = gpu_estep("bsc", prec, Y, W, 0.1, 0.5, Hp, 2)
    idx = np.sort(g.choice(N, 300, replace=False))
    r = O.estep("bsc", Y[idx], W, 0.1, 0.5, Hp, 2)
    assert r["flagged"].all()
    assert np.all(out["flagged"] == 1)
    assert np.all(out["sel"] == [0, 1, 2, 5])
    np.testing.assert_array_equal(out["sel"][idx], r["sel"])
    tol = TOL[prec]
    es = np.abs(out["s_mean"][idx] - r["s_mean"]).max()
    el = (np.abs(out["logL"][idx] - r["logL"]) / np.maximum(np.abs(r["logL"]), 1)).max()
    assert es <= tol[0] and el <= tol[1]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_wide_exact_tie_at_the_selection_boundary(prec):
    """54 identical columns tie at the selection boundary: the exact
    selection must keep the lowest tied indices and flag every point."""
    from oracle import prosper_oracle as O
    g = np.random.default_rng(37)
    D, H, Hp, N = 48, 64, 12, 700
    W = g.standard_normal((D, H))
    W /= np.linalg.norm(W, axis=0)
    W[:, 10:] = W[:, 10:11]
    Y = (3.0 * (W[:, 0] + W[:, 1] + W[:, 2]) + 1.0 * W[:, 10])[None, :] \
        + 0.01 * g.standard_normal((N, D))
    Y, W = Y.astype(np.float32), W.astype(np.float32)
    out = gpu_estep("bsc", prec, Y, W, 0.05, 0.5, Hp, 3)
    r = O.estep("bsc", Y[:60], W, 0.05, 0.5, Hp, 3)
    assert np.all(r["sel"] == [0, 1, 2] + list(range(10, 19)))
    assert np.all(out["sel"] == [0, 1, 2] + list(range(10, 19)))
    assert np.all(out["flagged"] == 1)
    tol = TOL[prec]
    es = np.abs(out["s_mean"][:60] - r["s_mean"]).max()
    el = (np.abs(out["logL"][:60] - r["logL"]) / np.maximum(np.abs(r["logL"]), 1)).max()
    assert es <= tol[0] and el <= tol[1]
