"""GPU parity of the max-superposition walks (MCA, MMCA) against the FP64
oracle, over the shapes that select each of them: the compile-time walk for
(H', gamma) = (10, 3) at 4, 7 and 8 pixels per lane (D = 60, 100, 128), the
table-driven walk for other (H', gamma) and for D beyond 128.  N = 120 leaves
a ragged last group of 16 points.  Each case checks the per-point outputs
and the accumulated statistics (responsibility numerator and denominator,
the FP64 sums), at parameters near the generating ones (peaked posteriors,
where the responsibility walk skips most states) and at a diffuse start."""
import numpy as np
import pytest

import synth
from oracle import prosper_oracle as O
from tests._common import assert_parity, gpu_estep

pytestmark = pytest.mark.gpu

H = 200


def max_problem(model, D, N, theta, seed=11):
    g = synth.rng(seed)
    if model == "mca":
        W = synth.abs_gaussian_dictionary(g, D, H)
    else:
        W = g.standard_normal((D, H))
    pi, sigma = 3.0 / H, 0.3
    S = synth.sample_binary(g, N, H, pi)
    mdl = O.MCA if model == "mca" else O.MMCA
    Y = (O.superposition(mdl, W, S) + sigma * g.standard_normal((N, D))).astype(np.float32)
    if theta == "gt":
        return Y, W.astype(np.float32), pi, sigma
    W0 = g.standard_normal((D, H)) / np.sqrt(D)
    if model == "mca":
        W0 = np.abs(W0)
    return Y, W0.astype(np.float32), 1.0 / H, float(Y.astype(np.float64).std())


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def check_statistics(g, r, N, label):
    ea, eb = rel(g["A"], r["A"]), rel(g["B"], r["B"])
    print(f"[stats] {label}: A {ea:.2e} B {eb:.2e}", flush=True)
    assert ea < 2e-5 and eb < 2e-5, label
    s = r["scal"]
    assert g["scal"][0] == pytest.approx(s[0], rel=1e-5)
    assert g["scal"][1] == pytest.approx(s[1], rel=1e-5)
    assert g["scal"][3] == pytest.approx(s[3], rel=1e-5)
    assert g["scal"][4] == N


@pytest.mark.parametrize("theta", ["gt", "init"])
@pytest.mark.parametrize("D", [60, 100, 128])
@pytest.mark.parametrize("model", ["mca", "mmca"])
def test_compiled_walk_parity(model, D, theta):
    N = 120
    Y, W, pi, sigma = max_problem(model, D, N, theta)
    print(f"[case] {model} D={D} N={N} (10,3) {theta}", flush=True)
    g = gpu_estep(model, "fp32", Y, W, pi, sigma, 10, 3, topk=4, accumulate=True)
    r = O.estep(model, Y, W, pi, sigma, 10, 3, topk=4)
    assert_parity(g, r, "fp32", f"{model} D={D} {theta}")
    ok = ~np.asarray(r["flagged"], dtype=bool)
    # one state's q carries the FP32 rounding of its own log-joint: |lj| up
    # to ~100 log2 units here, its residual summed over D <= 128 pixels in
    # about 12 rounding steps (8 per lane, 4 across the lanes), each at most
    # 2^-24 |lj|: ~7e-5 log2 units, i.e. ~5e-5 relative in q
    np.testing.assert_allclose(g["top_q"][ok], r["top_q"][ok], rtol=1e-4, atol=1e-7)
    check_statistics(g, r, N, f"{model} D={D} {theta}")


@pytest.mark.parametrize("Hp,gamma,D", [(8, 3, 100), (10, 2, 100), (10, 3, 150)])
@pytest.mark.parametrize("model", ["mca", "mmca"])
def test_table_walk_parity(model, Hp, gamma, D):
    N = 90
    Y, W, pi, sigma = max_problem(model, D, N, "init", seed=5)
    print(f"[case] table walk {model} D={D} ({Hp},{gamma})", flush=True)
    g = gpu_estep(model, "fp32", Y, W, pi, sigma, Hp, gamma, accumulate=True)
    r = O.estep(model, Y, W, pi, sigma, Hp, gamma)
    assert_parity(g, r, "fp32", f"table {model} D={D} ({Hp},{gamma})")
    check_statistics(g, r, N, f"table {model}")


@pytest.mark.parametrize("model", ["mca", "mmca"])
def test_compiled_walk_accumulates_across_calls(model):
    """Two accumulating calls add into the same accumulators (the walk's
    transposed partials are cleared per call)."""
    Y, W, pi, sigma = max_problem(model, 100, 140, "init", seed=3)
    import torch
    from paper_1908_06843_amd import api
    dev = torch.device("cuda", 0)
    acc = api.new_acc(model, 100, H)
    Wd = torch.tensor(W, device=dev)
    for part in (Y[:70], Y[70:]):
        api.estep(torch.tensor(part, device=dev), Wd, pi, sigma, Hprime=10, gamma=3, model=model,
                  acc=acc, want=())
    torch.cuda.synchronize()
    r = O.estep(model, Y, W, pi, sigma, 10, 3)
    g = {k: v.cpu().numpy() for k, v in acc.items()}
    check_statistics(g, r, 140, f"{model} two calls")
