"""GPU parity of MMCA (largest-magnitude superposition) through the C ABI
against the FP64 oracle: E-step outputs, the responsibility statistics and the
M-step.  Signed N(0,1) dictionary, D=100, H=200, pi=3/H, sigma=0.3 (the MCA
patch workload with both signs), at the generating parameters and at a
diffuse initialisation; N spans several workgroups."""
import numpy as np
import pytest

import synth
from oracle import prosper_oracle as O
from tests._common import assert_parity, gpu_estep

pytestmark = pytest.mark.gpu

D, H, PI, SIGMA, HP, GAMMA = 100, 200, 3.0 / 200, 0.3, 10, 3


def mmca_problem(N, theta, seed=7):
    g = synth.rng(seed)
    W = g.standard_normal((D, H))
    S = synth.sample_binary(g, N, H, PI)
    Y = O.superposition(O.MMCA, W, S) + SIGMA * g.standard_normal((N, D))
    Y = Y.astype(np.float32)
    if theta == "gt":
        return Y, W.astype(np.float32), PI, SIGMA
    W0 = (g.standard_normal((D, H)) / np.sqrt(D)).astype(np.float32)
    return Y, W0, 1.0 / H, float(Y.astype(np.float64).std())


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("theta", ["gt", "init"])
def test_mmca_estep_parity(theta, prec):
    Y, W, pi, sigma = mmca_problem(203, theta)
    print(f"[case] mmca N=203 theta={theta} {prec}", flush=True)
    g = gpu_estep("mmca", prec, Y, W, pi, sigma, HP, GAMMA)
    r = O.estep(O.MMCA, Y, W, pi, sigma, HP, GAMMA)
    assert_parity(g, r, prec, f"mmca/{theta}")


def test_mmca_accumulators_and_mstep():
    import torch
    from paper_1908_06843_amd import api
    Y, W, pi, sigma = mmca_problem(203, "init")
    print("[case] mmca accumulators N=203", flush=True)
    g = gpu_estep("mmca", "fp32", Y, W, pi, sigma, HP, GAMMA, accumulate=True)
    r = O.estep(O.MMCA, Y, W, pi, sigma, HP, GAMMA)
    assert rel(g["A"], r["A"]) < 2e-5
    assert rel(g["B"], r["B"]) < 2e-5
    s = r["scal"]
    assert g["scal"][0] == pytest.approx(s[0], rel=1e-5)
    assert g["scal"][1] == pytest.approx(s[1], rel=1e-5)
    assert g["scal"][3] == pytest.approx(s[3], rel=1e-5)
    assert g["scal"][4] == 203
    # device M-step on the oracle's statistics
    Wr, pir, sr = O.mstep(O.MMCA, Y, W, r)
    dev = torch.device("cuda", 0)
    acc = {"A": torch.tensor(r["A"], dtype=torch.float32, device=dev),
           "B": torch.tensor(r["B"], dtype=torch.float32, device=dev),
           "scal": torch.tensor(r["scal"], dtype=torch.float64, device=dev)}
    Wn, th = api.mstep(acc, torch.tensor(W, device=dev), model="mmca")
    torch.cuda.synchronize()
    Wn, th = Wn.cpu().numpy(), th.cpu().numpy()
    assert rel(Wn, Wr) < 1e-4
    assert th[0] == pytest.approx(pir, rel=1e-9)
    assert th[1] == pytest.approx(sr, rel=1e-5)
