"""GPU parity of the truncated E-step (HIP path through the C ABI) against
the FP64 oracle, on seeded synthetic data shaped like the five workloads.

Sizes span several workgroup tiles and a ragged tail; each case runs at the
generating parameters (peaked posteriors) and at the learning
initialisation (diffuse posteriors)."""
import numpy as np
import pytest

import synth
from oracle import prosper_oracle as O
from tests._common import assert_parity, gpu_estep, oracle_run, problem

pytestmark = pytest.mark.gpu

CASES = [
    # name, N, H', gamma  (bars: exact posterior, 1024 states; generic kernel)
    ("bars", 517, 10, 10),
    ("bsc256", 1037, 12, 4),      # unrolled (12, 4) walk
    ("tsc", 517, 8, 3),           # unrolled TSC (8, 3) walk
    ("mca", 203, 10, 3),          # max-superposition kernel
    ("serve", 131, 8, 3),
    ("serve", 131, 10, 4),
    ("serve", 131, 12, 5),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x1"])
@pytest.mark.parametrize("theta", ["gt", "init"])
@pytest.mark.parametrize("name,N,Hp,gamma", CASES)
def test_estep_parity(name, N, Hp, gamma, theta, prec):
    Y, W, pi, sigma, wl = problem(name, N, theta)
    print(f"[case] {name} N={N} H'={Hp} gamma={gamma} theta={theta} {prec}", flush=True)
    g = gpu_estep(wl.model, prec, Y, W, pi, sigma, Hp, gamma)
    r = oracle_run(name, N, theta, Hp, gamma)
    assert_parity(g, r, prec, f"{name}/{theta}/H'={Hp},g={gamma}")
    # selection is returned ascending and distinct
    assert np.all(np.diff(g["sel"], axis=1) > 0)
    # the GPU flags only near-ties; it must flag every point the oracle flags
    # whose gap it also sees inside its band (here: agreement on unflagged)
    assert np.all(g["s_mean"] >= (-1 if wl.model == "tsc" else 0) - 1e-6)
    assert np.all(g["s_mean"] <= 1 + 1e-6)


def test_generic_kernel_shapes():
    """Shapes without a compile-time walk go through the table kernel."""
    Y, W, pi, sigma, wl = problem("bsc256", 300, "init")
    for Hp, gamma in [(6, 2), (12, 3), (16, 2), (5, 5)]:
        g = gpu_estep("bsc", "fp32", Y, W, pi, sigma, Hp, gamma)
        r = O.estep("bsc", Y, W, pi, sigma, Hp, gamma)
        assert_parity(g, r, "fp32", f"generic H'={Hp} g={gamma}")


@pytest.mark.parametrize("model", ["bsc", "tsc"])
def test_deep_ragged_dictionary(model):
    """D = 300 (two depth chunks of the W^T W kernel, the second partial) and
    H = 37 (a partial 16 x 16 tile) with the generic walk."""
    g = synth.rng(31)
    D, H, N, pi, sigma = 300, 37, 401, 0.08, 0.6
    W = synth.unit_norm_gaussian_dictionary(g, D, H) * 2.0
    S = (synth.sample_binary if model == "bsc" else synth.sample_ternary)(g, N, H, pi)
    Y = np.ascontiguousarray(synth.linear_observations(g, W, S, sigma), dtype=np.float32)
    W = np.ascontiguousarray(W, dtype=np.float32)
    for prec in ("fp32", "bf16"):
        gout = gpu_estep(model, prec, Y, W, pi, sigma, 7, 3)
        r = O.estep(model, Y, W, pi, sigma, 7, 3)
        assert_parity(gout, r, prec, f"{model} D={D} H={H} {prec}")


def test_gamma_zero_and_one():
    Y, W, pi, sigma, wl = problem("bsc256", 200, "gt")
    for Hp, gamma in [(4, 0), (6, 1)]:
        g = gpu_estep("bsc", "fp32", Y, W, pi, sigma, Hp, gamma)
        r = O.estep("bsc", Y, W, pi, sigma, Hp, gamma)
        assert_parity(g, r, "fp32", f"H'={Hp} g={gamma}")
        if gamma == 0:
            assert np.all(g["s_mean"] == 0)


def test_single_point_and_all_latents():
    """N = 1, and H' = H (no preselection) with a non-multiple-of-4 D."""
    Y, W, pi, sigma, wl = problem("bars", 1, "gt")
    g = gpu_estep("bsc", "fp32", Y, W, pi, sigma, 10, 3)
    r = O.estep("bsc", Y, W, pi, sigma, 10, 3)
    assert_parity(g, r, "fp32", "N=1")
    assert list(g["sel"][0]) == list(range(10))


def test_empty_input_is_a_no_op():
    import torch
    from paper_1908_06843_amd import api
    Y = torch.zeros((0, 16), dtype=torch.float32, device="cuda")
    W = torch.randn((16, 8), dtype=torch.float32, device="cuda")
    out = api.estep(Y, W, 0.1, 1.0, Hprime=4, gamma=2)
    assert out["sel"].shape == (0, 4)


def test_invalid_arguments_raise():
    import torch
    from paper_1908_06843_amd import api
    Y = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    W = torch.randn((16, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(api.ProsperError):
        api.estep(Y, W, 0.1, 1.0, Hprime=9, gamma=2)
    with pytest.raises(api.ProsperError):
        api.estep(Y, W, 1.5, 1.0, Hprime=4, gamma=2)


@pytest.mark.parametrize("model,name,N,Hp,gamma", [("bsc", "bsc256", 300, 12, 4),
                                                   ("tsc", "tsc", 200, 8, 3),
                                                   ("mca", "mca", 100, 10, 3),
                                                   ("bsc", "bars", 200, 10, 10)])
def test_topk_matches_oracle(model, name, N, Hp, gamma):
    topk = 5
    Y, W, pi, sigma, wl = problem(name, N, "init")
    g = gpu_estep(model, "fp32", Y, W, pi, sigma, Hp, gamma, topk=topk)
    act, sgn = O.state_masks(model, Hp, gamma)
    r = O.estep(model, Y, W, pi, sigma, Hp, gamma, topk=topk)
    # a single state's q inherits the FP32 rounding of its log-joint
    # (|lj| 2^-24 ~ 1e-5 at |lj| ~ 200 log2 units): 3e-5 relative.  The
    # max-superposition walk sums its residual directly over the D pixels
    # (per lane, then across 16 lanes): up to ~15 roundings of |lj|, 1e-4.
    rq = 1e-4 if model == "mca" else 3e-5
    checked = 0
    for n in range(N):
        if r["flagged"][n] or not np.array_equal(g["sel"][n], r["sel"][n]):
            continue
        p = O.estep_point(model, Y[n], W, pi, sigma, Hp, gamma)
        qmap = {}
        for i in range(len(act)):
            key = (int(act[i]), int(sgn[i])) if model == "tsc" else int(act[i])
            qmap[key] = p["q"][i]
        for t in range(topk):
            q_ref = r["top_q"][n, t]
            assert abs(g["top_q"][n, t] - q_ref) <= rq * max(q_ref, 1e-3) + 1e-7
            key = ((int(g["top_mask"][n, t, 0]) & 0xffffffff, int(g["top_mask"][n, t, 1]) & 0xffffffff)
                   if model == "tsc" else int(g["top_mask"][n, t]) & 0xffffffff)
            # the GPU's t-th state has the oracle probability of rank t (ties allowed)
            assert abs(qmap[key] - q_ref) <= rq * max(q_ref, 1e-3) + 1e-7
        checked += 1
    assert checked > 0.9 * N


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x1"])
def test_full_size_bsc256_sampled(prec):
    """The benchmark configuration (N = 200000) on the GPU, checked against the
    oracle on a seeded sample of points (every output is per point), plus
    invariants over all points."""
    name = "bsc256"
    Y, Wgt, _, wl = synth.make_workload(name)
    W0, pi0, s0 = synth.initial_params(wl, Y)
    for W, pi, sigma, label in [(Wgt, wl.pi, wl.sigma, "gt"), (W0, pi0, s0, "init")]:
        print(f"[case] full-size {name} {label} {prec}", flush=True)
        g = gpu_estep("bsc", prec, Y, W, pi, sigma, wl.Hprime, wl.gamma)
        idx = np.sort(np.random.default_rng(7).choice(Y.shape[0], 150, replace=False))
        r = O.estep("bsc", Y[idx], W, pi, sigma, wl.Hprime, wl.gamma)
        assert_parity(g, r, prec, f"full {name}/{label}", idx=idx)
        assert np.all(np.isfinite(g["logL"]))
        assert np.all(np.diff(g["sel"], axis=1) > 0)
        assert g["s_mean"].min() >= 0 and g["s_mean"].max() <= 1 + 1e-6


@pytest.mark.parametrize("beta", [0.5, 0.1])
@pytest.mark.parametrize("model,name,N,Hp,gamma", [("bsc", "bsc256", 300, 12, 4),
                                                   ("tsc", "tsc", 300, 8, 3),
                                                   ("mca", "mca", 120, 10, 3),
                                                   ("bsc", "bars", 200, 10, 10)])
def test_annealed_posterior_matches_oracle(model, name, N, Hp, gamma, beta):
    """Posterior temperature (deterministic annealing): moments, top-k and
    statistics under q proportional to p(y, s)^beta, logL untempered."""
    Y, W, pi, sigma, wl = problem(name, N, "init")
    print(f"[case] annealed {name} beta={beta}", flush=True)
    g = gpu_estep(model, "fp32", Y, W, pi, sigma, Hp, gamma, topk=3, accumulate=True, beta=beta)
    r = O.estep(model, Y, W, pi, sigma, Hp, gamma, topk=3, beta=beta)
    assert_parity(g, r, "fp32", f"annealed {name} beta={beta}")
    ok = ~np.asarray(r["flagged"], dtype=bool)
    # single-state q: the FP32 rounding of its log-joint (see the top-k test)
    rq = 1e-4 if model == "mca" else 3e-5
    np.testing.assert_allclose(g["top_q"][ok], r["top_q"][ok], rtol=rq, atol=1e-7)
    B = g["B"]
    if model != "mca":
        B = np.triu(B) + np.triu(B, 1).T
    ea = np.abs(g["A"] - r["A"]).max() / np.abs(r["A"]).max()
    eb = np.abs(B - r["B"]).max() / np.abs(r["B"]).max()
    assert ea < 2e-5 and eb < 2e-5
    assert g["scal"][0] == pytest.approx(r["scal"][0], rel=1e-5)
    assert g["scal"][1] == pytest.approx(r["scal"][1], rel=1e-5)


def test_invalid_temperature_is_rejected():
    import torch
    from paper_1908_06843_amd import api
    Y = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    W = torch.randn((16, 8), dtype=torch.float32, device="cuda")
    for beta in (1.5, -0.5, float("nan")):
        with pytest.raises(api.ProsperError):
            api.estep(Y, W, 0.1, 1.0, Hprime=4, gamma=2, beta=beta)
